// Particle kernels of the PSWF fast Ewald pipeline for one precision and one range of window
// supports: spreading (Alg. 2 step 1) as a matrix product on the matrix cores, by register
// columns or by LDS atomics, and interpolation of potentials and gradients with the energy
// reduction (Alg. 2 step 5, eq. force). The build
// compiles this file once per (precision, P range), so the many template instances of these
// kernels compile in parallel; PSWFE_PREC (0 float, 1 double), PSWFE_PLO and PSWFE_PHI select
// the instance.
#include "device_common.hpp"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#ifndef PSWFE_PREC
#error "PSWFE_PREC must be defined (0 float, 1 double)"
#endif
#if !defined(PSWFE_PLO) || !defined(PSWFE_PHI)
#error "PSWFE_PLO / PSWFE_PHI must be defined"
#endif

#define PSWFE_CAT(a, b, c, d) a##_##b##_##c##_##d
#define PSWFE_XCAT(a, b, c, d) PSWFE_CAT(a, b, c, d)
#define PSWFE_PARTICLE_FN(name) PSWFE_XCAT(particles, name, PSWFE_PREC, PSWFE_PLO)

namespace pswfe {
namespace {

// ------------------------------------------------------------------------------------
// Particle kernels, one launch per (window support P, degree bucket D) over the tiles of the
// systems in that group. A workgroup (4 waves) owns one tile of B^3 cells of one system and an
// LDS copy of the S^3 grid points its particles' supports touch (S = B + P - 1, rounded up to odd).
// Each wave works on 4 particles at a time, 16 lanes per particle:
//  * lane j evaluates window piece j for the three coordinates at once (3 independent Horner
//    chains, 6 with derivatives; pieces j and j + 16 when P > 16), the coefficients of piece j
//    read from an LDS copy into registers, and writes the values to a per-slot LDS record;
//  * the 16 lanes then share the P^2 (y, z) lines of the support, each lane running the
//    x-direction of its lines. Lanes of a particle touch distinct lines (stride S), so their
//    LDS accesses do not conflict, and no workgroup barrier is needed between particles.
// Window values, products and sums are float64 in both precisions: on MI355X a float64 FMA
// issues at the non-packed float32 rate, and float32 window values and products lose ~1e-6
// relative on systems of neutral molecules, where the grid values are small sums of larger
// terms of both signs.
// ------------------------------------------------------------------------------------
constexpr int kLanesPerParticle = 16;

// Workgroups of the particle kernels have 256, 512 or 1024 threads (4 particle slots per
// wave); 1024 only where the kernel fits in 128 VGPRs (P <= 13), so that 16 waves can share
// one compute unit's LDS tile.
template <int P>
constexpr int particle_max_threads() { return P <= 13 ? 1024 : 512; }

// Per-wave ordering of LDS accesses between lanes (the record written by one lane is read by
// other lanes of the same wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup id in tile order. Workgroups are dispatched to the 8 XCDs (each with its own L2)
// in turn; with `xcd` set, the ids are mapped so that each XCD takes a contiguous range of
// tiles, whose halos overlap, instead of every eighth tile. Set when the whole grid is resident
// at once (measured: water-box interpolation 40.9 -> 38.3 us in float32; 52.3 -> 53.7 us in
// float64, where the grid runs in two rounds).
__device__ __forceinline__ int tile_order_block(int xcd) {
  const int b = static_cast<int>(blockIdx.x), n = static_cast<int>(gridDim.x);
  const int full = n - n % 8;
  if (xcd && b < full) return (b % 8) * (full / 8) + b / 8;
  return b;
}

// Particles [p0, p1) of part `part` of `parts` equal slices of tile gtile's bin: a dense tile
// is shared by several workgroups (each spreading into its own partial block, or interpolating
// its own particles), so that small grids with many particles per tile still fill the GPU.
__device__ __forceinline__ void tile_slice(const int* __restrict__ tile_start, int gtile, int sub_log2, int part,
                                           int parts, int& p0, int& p1) {
  const int a = tile_start[gtile << sub_log2], b = tile_start[(gtile + 1) << sub_log2];
  const int64_t nt = b - a;
  p0 = a + static_cast<int>(nt * part / parts);
  p1 = a + static_cast<int>(nt * (part + 1) / parts);
}

// Copies the window coefficients (P pieces of deg + 1 powers, float64) into LDS rows of
// coef_stride(D) doubles, zero above deg.
template <int P, int D>
__device__ __forceinline__ void stage_coefficients(const double* __restrict__ coef, int deg, double* lcoef) {
  constexpr int CS = coef_stride(D);
  const global_ptr<double> gcoef = as_global(coef);
  for (int i = threadIdx.x; i < P * CS; i += blockDim.x) {
    const int j = i / CS, k = i - j * CS;
    lcoef[i] = k <= deg ? gcoef[j * (deg + 1) + k] : 0.0;
  }
}

// The same in two halves, so that other loads can be issued in between: coef_load reads this
// thread's entries (at most kCoefPerThread; P * coef_stride(D) <= kCoefPerThread * blockDim.x)
// into registers, coef_store writes them to LDS.
constexpr int kCoefPerThread = 3;
template <int P, int D>
__device__ __forceinline__ void coef_load(const double* __restrict__ coef, int deg, double (&v)[kCoefPerThread]) {
  constexpr int CS = coef_stride(D);
  const global_ptr<double> gcoef = as_global(coef);
#pragma unroll
  for (int u = 0; u < kCoefPerThread; ++u) {
    const int i = threadIdx.x + u * blockDim.x;
    const int j = i / CS, k = i - j * CS;
    v[u] = (i < P * CS && k <= deg) ? gcoef[j * (deg + 1) + k] : 0.0;
  }
}
template <int P, int D>
__device__ __forceinline__ void coef_store(double* lcoef, const double (&v)[kCoefPerThread]) {
  constexpr int CS = coef_stride(D);
#pragma unroll
  for (int u = 0; u < kCoefPerThread; ++u) {
    const int i = threadIdx.x + u * blockDim.x;
    if (i < P * CS) lcoef[i] = v[u];
  }
}

// Spreading (Alg. 2 step 1): the tile accumulates q w_x w_y w_z over the supports with LDS
// float64 atomic adds (on gfx950 about 20x the throughput of float32 LDS atomics), then adds
// the tile into its system's float64 HBM grid with atomics (a point lies in the halos of up
// to ceil(S/B)^3 tiles; their partial sums are larger than the total on systems of neutral
// molecules, so they are added in float64 and rounded once, by the first FFT pass).
// A lane reads the weights of up to kLineChunk lines and the x-window into registers before
// issuing their atomics: LDS operations complete in order, so an LDS read between atomics
// would wait for all of them.
constexpr int kLineChunk = 12;

template <class T, int P, int D>
__global__ __launch_bounds__(particle_max_threads<P>()) void k_spread(const typename Vec4<T>::type* __restrict__ sorted,
                                                const int* __restrict__ cells, const int* __restrict__ tile_start,
                                                int sub_log2, int nsys, const SysDesc* __restrict__ sys,
                                                const int* __restrict__ tile_prefix, const int* __restrict__ tile_sys,
                                                int tile_offset, int parts, int xcd) {
  constexpr int REC = 3 * P;  // window values of one particle: x, y, z
  constexpr int CS = coef_stride(D);
  constexpr int NL = (P * P + kLanesPerParticle - 1) / kLanesPerParticle;  // lines per lane
  extern __shared__ unsigned char smem_raw[];
  const int wgid = tile_order_block(xcd);
  const int gtile = tile_offset + wgid / parts;
  int p0, p1;
  tile_slice(tile_start, gtile, sub_log2, wgid % parts, parts, p0, p1);
  if (p0 == p1) return;
  const SysDesc& sd = sys[nsys == 1 ? 0 : tile_sys[find_sys(tile_prefix, nsys, gtile)]];
  const int m = sd.m, B = sd.B, Tn = sd.Tn, S = sd.S;
  double* __restrict__ grid = sd.grid_a;
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int S3 = S * S * S;
  const int nslots = blockDim.x / kLanesPerParticle;
  double* recs = acc + S3;                           // nslots * REC
  double* lcoef = recs + nslots * REC;               // P * CS
  const int tile = gtile - sd.tile_base;
  const int tx = tile % Tn, ty = (tile / Tn) % sd.Tny, tz = tile / (Tn * sd.Tny);
  const int T0x = tx * B, T0y = ty * B, T0z = tz * B;
  stage_coefficients<P, D>(sd.coef, sd.deg, lcoef);
  for (int i = threadIdx.x; i < S3; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int slot = threadIdx.x >> 4;
  const int li = lane & (kLanesPerParticle - 1);
  double* rec = recs + slot * REC;
  const int nt = p1 - p0;
  // the record of the next round is loaded while this round's particle is spread
  auto r_next = sorted[min(p0 + slot, p1 - 1)];
  int c_next = cells[min(p0 + slot, p1 - 1)];
  for (int base = 0; base < nt; base += nslots) {
    const int pi = p0 + base + slot;
    const bool active = pi < p1;
    const auto r = r_next;
    const int cp = c_next;
    r_next = sorted[min(pi + nslots, p1 - 1)];
    c_next = cells[min(pi + nslots, p1 - 1)];
    int o[3];
    double g[3];
    g[0] = static_cast<double>(r.x);
    o[0] = cell_x(cp) - T0x;
    g[1] = static_cast<double>(r.y);
    o[1] = cell_y(cp) - T0y;
    g[2] = static_cast<double>(r.z);
    o[2] = cell_z(cp) - T0z;
#pragma unroll
    for (int jj = 0; jj < (P + kLanesPerParticle - 1) / kLanesPerParticle; ++jj) {
      const int j = li + kLanesPerParticle * jj;
      if (j >= P) break;
      double c[D + 1];
#pragma unroll
      for (int k = 0; k <= D; ++k) c[k] = lcoef[j * CS + k];
      double vx = c[D], vy = c[D], vz = c[D];
#pragma unroll
      for (int k = D - 1; k >= 0; --k) {
        vx = fma(vx, g[0], c[k]);
        vy = fma(vy, g[1], c[k]);
        vz = fma(vz, g[2], c[k]);
      }
      rec[j] = vx;
      rec[P + j] = vy;
      rec[2 * P + j] = vz;
    }
    wave_lds_sync();
    if (active) {
      const double q = static_cast<double>(r.w);
      double wx[P];
#pragma unroll
      for (int j = 0; j < P; ++j) wx[j] = rec[j];
#pragma unroll
      for (int t0 = 0; t0 < NL; t0 += kLineChunk) {
        double wl[kLineChunk];
        int off[kLineChunk];
#pragma unroll
        for (int t = 0; t < kLineChunk; ++t) {
          const int e = li + kLanesPerParticle * (t0 + t);
          const int jz = e / P, jy = e - jz * P;
          const bool ok = t0 + t < NL && e < P * P;
          wl[t] = ok ? q * rec[P + jy] * rec[2 * P + jz] : 0.0;
          off[t] = ok ? ((o[2] + jz) * S + (o[1] + jy)) * S + o[0] : -1;
        }
#pragma unroll
        for (int t = 0; t < kLineChunk; ++t) {
          if (off[t] >= 0) {
            double* row = acc + off[t];
#pragma unroll
            for (int jx = 0; jx < P; ++jx) atomicAdd(row + jx, wl[t] * wx[jx]);
          }
        }
      }
    }
    wave_lds_sync();
  }
  __syncthreads();
  const int half = (P + 1) / 2;
  const int Ox = T0x + 1 - half, Oy = T0y + 1 - half, Oz = T0z + 1 - half;
  double v[8];
  walk_tile<8>(
      S, m, sd.my, sd.mz, Ox, Oy, Oz, [&](int k, int li_, int64_t) { v[k] = acc[li_]; },
      [&](int k, int, int64_t gi) {
        if (v[k] != 0.0) atomic_add_global(grid + gi, v[k]);
      });
}

// Spreading by columns, for tiles of edge B = 4, 6 or 8 (Alg. 2 step 1, same sums as k_spread).
// Thread (ix, iz) of the S x S face of the tile's block owns the S points of its y-column in
// registers. Particles are taken kColBatch at a time: their window values are written to LDS
// as S-long arrays per dimension, zero outside the support (Horner runs once per value), and
// every thread adds q w_x[ix] w_z[iz] w_y[iy] to its S points, skipping particles whose support
// misses its column. The P^3 products of a particle become register FMAs instead of LDS
// atomics (on gfx950 a float64 FMA costs far less issue time than a float64 LDS atomic);
// the block then adds its S^3 points into the float64 grid with global atomics, lanes of
// consecutive ix writing consecutive addresses.
constexpr int kColBatch = 32;
template <int P, int B>
constexpr int col_edge() { return B + P - 1; }
template <int P, int B>
constexpr int col_threads() { return (col_edge<P, B>() * col_edge<P, B>() + 63) / 64 * 64; }

template <class T, int P, int D, int B>
__global__ __launch_bounds__((col_threads<P, B>())) void k_spread_cols(
    const typename Vec4<T>::type* __restrict__ sorted, const int* __restrict__ cells,
    const int* __restrict__ tile_start, int sub_log2, int nsys, const SysDesc* __restrict__ sys,
    const int* __restrict__ tile_prefix, const int* __restrict__ tile_sys, int tile_offset, int parts, int xcd) {
  constexpr int S = col_edge<P, B>();
  constexpr int CS = coef_stride(D);
  constexpr int RS = 3 * S;  // a particle's padded window values: x, y, z
  extern __shared__ unsigned char smem_raw[];
  const int wgid = tile_order_block(xcd);
  const int gtile = tile_offset + wgid / parts;
  int p0, p1;
  tile_slice(tile_start, gtile, sub_log2, wgid % parts, parts, p0, p1);
  if (p0 == p1) return;
  const SysDesc& sd = sys[nsys == 1 ? 0 : tile_sys[find_sys(tile_prefix, nsys, gtile)]];
  const int m = sd.m, Tn = sd.Tn;
  double* __restrict__ grid = sd.grid_a;
  double* lcoef = reinterpret_cast<double*>(smem_raw);  // P * CS
  double* recs = lcoef + P * CS;                        // kColBatch * RS
  double* pg = recs + kColBatch * RS;                   // kColBatch * 4: g_x, g_y, g_z, q
  int* po = reinterpret_cast<int*>(pg + kColBatch * 4); // kColBatch * 4: o_x, o_y, o_z
  const int tile = gtile - sd.tile_base;
  const int tx = tile % Tn, ty = (tile / Tn) % sd.Tny, tz = tile / (Tn * sd.Tny);
  const int T0x = tx * B, T0y = ty * B, T0z = tz * B;
  stage_coefficients<P, D>(sd.coef, sd.deg, lcoef);
  const int t = threadIdx.x;
  const bool owner = t < S * S;
  const int iz = t / S, ix = t - (t / S) * S;
  double acc[S];
#pragma unroll
  for (int k = 0; k < S; ++k) acc[k] = 0.0;
  // the records of the next batch are loaded while this batch is accumulated
  auto r_next = sorted[min(p0 + t, p1 - 1)];
  int c_next = cells[min(p0 + t, p1 - 1)];
  for (int b0 = p0; b0 < p1; b0 += kColBatch) {
    const int nb = min(kColBatch, p1 - b0);
    const auto r = r_next;
    const int cp = c_next;
    if (t < kColBatch) {
      r_next = sorted[min(b0 + kColBatch + t, p1 - 1)];
      c_next = cells[min(b0 + kColBatch + t, p1 - 1)];
    }
    if (t < nb) {
      int o0, o1, o2;
      pg[4 * t + 0] = static_cast<double>(r.x);
      o0 = cell_x(cp) - T0x;
      pg[4 * t + 1] = static_cast<double>(r.y);
      o1 = cell_y(cp) - T0y;
      pg[4 * t + 2] = static_cast<double>(r.z);
      o2 = cell_z(cp) - T0z;
      pg[4 * t + 3] = static_cast<double>(r.w);
      po[4 * t + 0] = o0;
      po[4 * t + 1] = o1;
      po[4 * t + 2] = o2;
    }
    __syncthreads();
    for (int e = t; e < nb * RS; e += blockDim.x) {
      const int k = e / RS, rr = e - k * RS, d = rr / S, i = rr - d * S;
      const int j = i - po[4 * k + d];
      double v = 0.0;
      if (j >= 0 && j < P) {
        const double g = pg[4 * k + d];
        const double* c = lcoef + j * CS;
        v = c[D];
#pragma unroll
        for (int kk = D - 1; kk >= 0; --kk) v = fma(v, g, c[kk]);
      }
      recs[e] = v;
    }
    __syncthreads();
    if (owner) {
      for (int k = 0; k < nb; ++k) {
        const double* R = recs + k * RS;
        const double tq = pg[4 * k + 3] * R[ix] * R[2 * S + iz];
        if (tq != 0.0) {
#pragma unroll
          for (int iy = 0; iy < S; ++iy) acc[iy] = fma(tq, R[S + iy], acc[iy]);
        }
      }
    }
    __syncthreads();
  }
  if (owner) {
    constexpr int half = (P + 1) / 2;
    const int my = sd.my;
    const int gx = fold_index(T0x + 1 - half + ix, m);
    const int64_t gz = fold_index(T0z + 1 - half + iz, sd.mz);
#pragma unroll
    for (int iy = 0; iy < S; ++iy) {
      if (acc[iy] != 0.0) {
        const int gy = fold_index(T0y + 1 - half + iy, my);
        atomic_add_global(grid + (gz * my + gy) * m + gx, acc[iy]);
      }
    }
  }
}

// Spreading as a matrix product on the matrix cores, for tile edges 4, 6 and 8 (Alg. 2 step 1,
// same sums as k_spread). Over a tile's particles the S^3 block is
//   C[(z, y), x] = sum_p U[(z, y), p] V[p, x],  U = q_p w_z,p[z] w_y,p[y],  V = w_x,p[x],
// a product of an S^2 x K and a K x S matrix (K = the tile's particles). The block is cut into
// 16 x 16 pieces of C held in the accumulators of v_mfma_f64_16x16x4f64 (or, with A = float, of
// v_mfma_f32_16x16x4f32), kMfmaPieces row pieces per wave; each instruction takes 4 particles.
// Particles are taken kColBatch at a time: their window values are written to LDS as S-long arrays
// per dimension (zero outside the support, the z-values multiplied by the charge).
// Column slices: when S exceeds 16 but a particle's x-support (P points from o_x in [0, B)) fits
// one 16-column piece starting at column 0 (o_x <= 16 - P) or at column S - 16 (o_x >= S - 16),
// every particle is assigned to one of these two slices, each batch is ordered by slice (each
// slice padded to whole groups of 4 with zero records), and a group's instructions use only its
// slice's 16 columns: one column piece per row piece instead of two, half the matrix work (tile
// edge 8 with P = 10-13). The two slices' accumulators are added in LDS at the end.
// The block is then written to LDS and added to the grid with lanes of consecutive x on
// consecutive addresses.
// Accumulator layouts (checked on the GPU): float64, item r of lane l at row l / 16 + 4 r,
// column l % 16; float32, item r of lane l at row 4 (l / 16) + r, column l % 16. Operand a of lane
// l is A[l % 16][l / 16], operand b is B[l / 16][l % 16].
// A = float keeps window values, products and the tile's sums in float32 on the matrix cores
// (the float32 arithmetic path of float32 plans); the block is flushed into the float64 grid,
// or (grid32, A = float only) into the same buffer read as a float32 grid.
template <class A>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MfmaAcc<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// One value of a tile's block added to the grid: float64, or float32 where the plan
// accumulates its float32-arithmetic spread in a float32 grid (grid32).
template <class A>
__device__ __forceinline__ void flush_add(double* grid, int64_t gi, double v, int grid32) {
  if constexpr (sizeof(A) == sizeof(float)) {
    if (grid32) {
      atomic_add_global(reinterpret_cast<float*>(grid) + gi, static_cast<float>(v));
      return;
    }
  }
  atomic_add_global(grid + gi, v);
}

constexpr int kMfmaPieces = 4;
template <int P, int B>
constexpr int mfma_row_pieces() { return (col_edge<P, B>() * col_edge<P, B>() + 15) / 16; }
template <int P, int B>
constexpr int mfma_col_pieces() { return (col_edge<P, B>() + 15) / 16; }
template <int P, int B>
constexpr int mfma_threads() { return 64 * ((mfma_row_pieces<P, B>() + kMfmaPieces - 1) / kMfmaPieces); }
template <int P, int B>
constexpr bool mfma_sliced() { return mfma_sliced_host(P, B); }
// Particles per batch of the matrix-core spread: 64 (fewer barrier-separated rounds: water box
// 44.6 -> 43.8 us, n = 1e6 float32 417 -> 391 us against 32), 32 by columns of tiles (float64
// n = 1e6: 2.19 against 2.33 ms with 64). Record slots: a batch plus the padding of two slices.
template <bool ROLL>
constexpr int mfma_batch() { return ROLL ? kMfmaRollBatchHost : kMfmaBatchHost; }

template <class T, int P, int D, int B, class A, bool ROLL>
__global__ __launch_bounds__((mfma_threads<P, B>())) void k_spread_mfma(
    const typename Vec4<T>::type* __restrict__ sorted, const int* __restrict__ cells,
    const int* __restrict__ tile_start, int sub_log2, int nsys, const SysDesc* __restrict__ sys,
    const int* __restrict__ tile_prefix, const int* __restrict__ tile_sys, int tile_offset, int parts, int xcd,
    int seg_len, int nseg, int grid32) {
  constexpr int S = col_edge<P, B>();
  constexpr int MR = mfma_row_pieces<P, B>();
  constexpr bool SL = mfma_sliced<P, B>();
  constexpr int NC = SL ? 2 : mfma_col_pieces<P, B>();  // column pieces, or the two slices
  constexpr int X1 = S - 16;                              // first column of slice 1
  constexpr int CS = coef_stride(D);
  constexpr int RS = 3 * S;
  constexpr int CB = mfma_batch<ROLL>(), NREC = CB + 8;
  static_assert(CB <= 64 && NREC <= 128, "wave 0 holds a batch and marks its slots");
  using M = MfmaAcc<A>;
  typedef typename M::v4 acc_t;
  // dynamic LDS only: a static array beside a large dynamic allocation measured 2.8x slower
  // (P = 18, 125 KB of LDS per workgroup)
  extern __shared__ unsigned char smem_raw[];
  // ROLL: the workgroup takes tiles z0..z1-1 of column (tx, ty) of a single system in turn,
  // keeping their S^3 blocks in LDS as a ring of z-planes (plane z of tile z0 + k in slot
  // (k B + z) mod S) ahead of the records; after each tile only the B planes that no later tile
  // of the column reaches are added to the grid, the others carry over. Otherwise: one tile (or
  // one slice of a tile's particles) per workgroup, its block over the records' LDS.
  const int wgid = ROLL ? static_cast<int>(blockIdx.x) : tile_order_block(xcd);
  int p0 = 0, p1 = 0, gtile = 0;
  if constexpr (!ROLL) {
    gtile = tile_offset + wgid / parts;
    tile_slice(tile_start, gtile, sub_log2, wgid % parts, parts, p0, p1);
    if (p0 == p1) return;
  }
  const SysDesc& sd = sys[(ROLL || nsys == 1) ? 0 : tile_sys[find_sys(tile_prefix, nsys, gtile)]];
  const int m = sd.m, Tn = sd.Tn;
  double* __restrict__ grid = sd.grid_a;
  double* ring = reinterpret_cast<double*>(smem_raw);      // ROLL: S^3
  double* lcoef = ring + (ROLL ? S * S * S : 0);           // P * CS
  double* pg = lcoef + P * CS;                             // NREC * 4: g_x, g_y, g_z, q
  int* po = reinterpret_cast<int*>(pg + NREC * 4);         // NREC * 4: o_x, o_y, o_z, valid
  A* recs = reinterpret_cast<A*>(po + NREC * 4);           // NREC * RS
  // groups of 4: slice 0 in [0, s_split[0]), slice 1 up to s_split[1]
  int* s_split = reinterpret_cast<int*>(recs + NREC * RS);
  int tx, ty, tz, z1 = 0;
  if constexpr (ROLL) {
    const int col = wgid / nseg, seg = wgid - col * nseg;
    tx = col % Tn;
    ty = col / Tn;
    tz = seg * seg_len;
    z1 = min(sd.Tnz, tz + seg_len);
    if (tz >= z1) return;
    const int gt = sd.tile_base + (tz * sd.Tny + ty) * Tn + tx;
    p0 = tile_start[gt << sub_log2];
    p1 = tile_start[(gt + 1) << sub_log2];
  } else {
    const int tile = gtile - sd.tile_base;
    tx = tile % Tn;
    ty = (tile / Tn) % sd.Tny;
    tz = tile / (Tn * sd.Tny);
  }
  const int T0x = tx * B, T0y = ty * B;
  int T0z = tz * B;
  const int t = threadIdx.x;
  // the first batch's records are loaded before the coefficients are staged: the two round
  // trips to memory overlap
  auto r_next = sorted[min(p0 + t, max(p1 - 1, 0))];
  int c_next = cells[min(p0 + t, max(p1 - 1, 0))];
  stage_coefficients<P, D>(sd.coef, sd.deg, lcoef);
  if constexpr (ROLL) {
    for (int i = t; i < S * S * S; i += blockDim.x) ring[i] = 0.0;
  }
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  // waves whose row pieces are all inside the block run the group loop without per-piece checks
  const bool full_wave = (wave + 1) * kMfmaPieces <= MR;
  // this lane's rows of U (one per row piece) and columns of V (one per column piece or slice)
  int zo[kMfmaPieces], yo[kMfmaPieces];
  A rmask[kMfmaPieces];
#pragma unroll
  for (int u = 0; u < kMfmaPieces; ++u) {
    const int row = (wave * kMfmaPieces + u) * 16 + lr;
    const bool ok = row < S * S;
    zo[u] = 2 * S + (ok ? row / S : 0);
    yo[u] = S + (ok ? row % S : 0);
    rmask[u] = ok ? A(1) : A(0);
  }
  int xo[NC];
  A cmask[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int x = SL ? (c == 0 ? lr : X1 + lr) : c * 16 + lr;
    xo[c] = x < S ? x : 0;
    cmask[c] = x < S ? A(1) : A(0);
  }
  acc_t acc[kMfmaPieces][NC];
  constexpr int half = (P + 1) / 2;
  for (int k = 0;; ++k) {
#pragma unroll
  for (int u = 0; u < kMfmaPieces; ++u)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[u][c] = acc_t{0, 0, 0, 0};
  if constexpr (ROLL) __syncthreads();  // the ring's zeros, or the previous tile's flush
  for (int b0 = p0; b0 < p1; b0 += CB) {
    const int nb = min(CB, p1 - b0);
    const auto r = r_next;
    const int cp = c_next;
    if (t < CB) {
      r_next = sorted[min(b0 + CB + t, p1 - 1)];
      c_next = cells[min(b0 + CB + t, p1 - 1)];
    }
    if (t < 64) {  // wave 0 holds the batch (CB <= 64): record slots, ordered by slice
      const bool act = t < nb;
      const int ox = cell_x(cp) - T0x;
      int pos = t, ng0 = (nb + 3) >> 2, ng = ng0;
      if constexpr (SL) {
        const bool s1 = act && ox > 16 - P;
        const uint64_t m1 = __ballot(s1), m0 = __ballot(act && !s1);
        const uint64_t below = (uint64_t(1) << t) - 1;
        const int n0 = __popcll(m0), n0p = (n0 + 3) & ~3, n1 = __popcll(m1);
        pos = s1 ? n0p + __popcll(m1 & below) : __popcll(m0 & below);
        ng0 = n0p >> 2;
        ng = ng0 + ((n1 + 3) >> 2);
        // slots of the padding: [n0, n0p) and [n0p + n1, 4 ng)
        // (lane t marks slots t and t + 64: a batch of more than 58 particles has slots beyond
        // the wave's lanes)
        if (t < 4 * ng && !((t < n0) || (t >= n0p && t < n0p + n1))) po[4 * t + 3] = 0;
        if constexpr (NREC > 64) {
          const int t2 = t + 64;
          if (t2 < 4 * ng && !((t2 < n0) || (t2 >= n0p && t2 < n0p + n1))) po[4 * t2 + 3] = 0;
        }
      } else {
        if (t >= nb && t < 4 * ng) po[4 * t + 3] = 0;
        if constexpr (NREC > 64) {
          if (t + 64 < 4 * ng) po[4 * (t + 64) + 3] = 0;  // t + 64 >= nb
        }
      }
      if (act) {
        pg[4 * pos + 0] = static_cast<double>(r.x);
        pg[4 * pos + 1] = static_cast<double>(r.y);
        pg[4 * pos + 2] = static_cast<double>(r.z);
        pg[4 * pos + 3] = static_cast<double>(r.w);
        po[4 * pos + 0] = ox;
        po[4 * pos + 1] = cell_y(cp) - T0y;
        po[4 * pos + 2] = cell_z(cp) - T0z;
        po[4 * pos + 3] = 1;
      }
      if (t == 0) {
        s_split[0] = 4 * ng0;
        s_split[1] = 4 * ng;
      }
    }
    __syncthreads();
    const int nrec = s_split[1];
    // the P window values of each particle and dimension (Horner), then the S - P zeros around
    // them, so that no lane runs Horner for a zero; padding slots are all zero
    for (int e = t; e < nrec * 3 * P; e += blockDim.x) {
      const int k = e / (3 * P), rr = e - k * (3 * P), d = rr / P, j = rr - d * P;
      const bool ok = po[4 * k + 3] != 0;
      double v = 0.0;
      if (ok) {
        const double g = pg[4 * k + d];
        const double* c = lcoef + j * CS;
        v = c[D];
#pragma unroll
        for (int kk = D - 1; kk >= 0; --kk) v = fma(v, g, c[kk]);
        if (d == 2) v *= pg[4 * k + 3];
      }
      recs[k * RS + d * S + (ok ? po[4 * k + d] : 0) + j] = static_cast<A>(v);
    }
    for (int e = t; e < nrec * 3 * (S - P); e += blockDim.x) {
      const int k = e / (3 * (S - P)), rr = e - k * (3 * (S - P)), d = rr / (S - P), jj = rr - d * (S - P);
      const int o = po[4 * k + 3] != 0 ? po[4 * k + d] : 0;
      recs[k * RS + d * S + (jj < o ? jj : jj + P)] = A(0);
    }
    __syncthreads();
    // every piece takes every group of its slice: skipping the pieces outside a group's z-range
    // (the particles are ordered by z) measured slower, as the branches break up the chain of
    // matrix instructions
    auto groups = [&](int k_begin, int k_end, auto slice, auto full) {
      constexpr int s = decltype(slice)::value;
      constexpr bool all_pieces = decltype(full)::value;
      for (int k4 = k_begin; k4 < k_end; k4 += 4) {
        const A* R = recs + (k4 + lk) * RS;
        A bv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (!SL || c == s) bv[c] = R[xo[c]] * cmask[c];
        if constexpr (sizeof(A) == sizeof(float)) {
          // float32: the row operands of all pieces are read first (registers allow it)
          A av[kMfmaPieces];
#pragma unroll
          for (int u = 0; u < kMfmaPieces; ++u) av[u] = R[zo[u]] * R[yo[u]] * rmask[u];
#pragma unroll
          for (int u = 0; u < kMfmaPieces; ++u) {
            if (all_pieces || wave * kMfmaPieces + u < MR) {
#pragma unroll
              for (int c = 0; c < NC; ++c)
                if (!SL || c == s) acc[u][c] = M::mfma(av[u], bv[c], acc[u][c]);
            }
          }
        } else {
          // float64: one piece's operand at a time, which keeps the kernel within 128 VGPRs
          // (reading all four first took 160 and lost a workgroup per compute unit)
#pragma unroll
          for (int u = 0; u < kMfmaPieces; ++u) {
            if (all_pieces || wave * kMfmaPieces + u < MR) {
              const A av = R[zo[u]] * R[yo[u]] * rmask[u];
#pragma unroll
              for (int c = 0; c < NC; ++c)
                if (!SL || c == s) acc[u][c] = M::mfma(av, bv[c], acc[u][c]);
            }
          }
        }
      }
    };
    auto slices = [&](auto full) {
      if constexpr (SL) {
        groups(0, s_split[0], std::integral_constant<int, 0>(), full);
        groups(s_split[0], nrec, std::integral_constant<int, 1>(), full);
      } else {
        groups(0, nrec, std::integral_constant<int, 0>(), full);
      }
    };
    if constexpr (sizeof(A) == sizeof(float)) {
      if (full_wave)
        slices(std::true_type());
      else
        slices(std::false_type());
    } else {
      slices(std::false_type());  // one copy of the loop: a second one took 150+ VGPRs
    }
    __syncthreads();
  }
  if constexpr (ROLL) {
    // the tile's sums into the ring (slot of plane z: (k B + z) mod S); every row belongs to one
    // wave, so the two slices' additions (one lane after another) need no barrier between them
#pragma unroll
    for (int u = 0; u < kMfmaPieces; ++u) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = SL ? (c == 0 ? lr : X1 + lr) : c * 16 + lr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = (wave * kMfmaPieces + u) * 16 + M::row(lk, q);
          if (row < S * S && x < S) {
            const int z = row / S, y = row - z * S;
            int zs = (k * B) % S + z;
            zs -= zs >= S ? S : 0;
            ring[(zs * S + y) * S + x] += static_cast<double>(acc[u][c][q]);
          }
        }
      }
    }
    __syncthreads();
    // the planes no later tile of the column reaches (all S after the last tile) into the grid,
    // their slots cleared for the planes the next tile adds
    const bool last = tz + 1 >= z1;
    const int nplanes = last ? S : B;
    const int Ox = T0x + 1 - half, Oy = T0y + 1 - half, Oz = T0z + 1 - half;
    const int S2 = S * S, items = nplanes * S2, nt = static_cast<int>(blockDim.x);
    for (int base = t; base < items; base += 8 * nt) {
      double v[8];
      int li[8];
      int64_t gi[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = base + j * nt;
        li[j] = -1;
        if (e < items) {
          const int z = e / S2, rem = e - z * S2, y = rem / S, x = rem - y * S;
          int zs = (k * B) % S + z;
          zs -= zs >= S ? S : 0;
          li[j] = (zs * S + y) * S + x;
          gi[j] = (static_cast<int64_t>(fold_index(Oz + z, sd.mz)) * sd.my + fold_index(Oy + y, sd.my)) * m +
                  fold_index(Ox + x, m);
          v[j] = ring[li[j]];
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (li[j] < 0) continue;
        if (v[j] != 0.0) flush_add<A>(grid, gi[j], v[j], grid32);
        ring[li[j]] = 0.0;
      }
    }
    if (last) break;
    // the next tile of the column
    ++tz;
    T0z = tz * B;
    const int gt = sd.tile_base + (tz * sd.Tny + ty) * Tn + tx;
    p0 = tile_start[gt << sub_log2];
    p1 = tile_start[(gt + 1) << sub_log2];
    r_next = sorted[min(p0 + t, max(p1 - 1, 0))];
    c_next = cells[min(p0 + t, max(p1 - 1, 0))];
  } else {
  double* blk = reinterpret_cast<double*>(smem_raw);  // S^3, over the coefficients and records
  // column piece c (or slice 0) first; with slices, the columns only slice 1 reaches are zeroed
  // and slice 1 is added after a barrier
#pragma unroll
  for (int u = 0; u < kMfmaPieces; ++u) {
#pragma unroll
    for (int c = 0; c < (SL ? 1 : NC); ++c) {
      const int x = c * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = (wave * kMfmaPieces + u) * 16 + M::row(lk, q);
        if (row < S * S && x < S) blk[row * S + x] = static_cast<double>(acc[u][c][q]);
      }
    }
  }
  if constexpr (SL) {
    for (int i = t; i < S * S * (S - 16); i += blockDim.x) {
      const int row = i / (S - 16);
      blk[row * S + 16 + (i - row * (S - 16))] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMfmaPieces; ++u) {
      const int x = X1 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = (wave * kMfmaPieces + u) * 16 + M::row(lk, q);
        if (row < S * S) blk[row * S + x] += static_cast<double>(acc[u][1][q]);
      }
    }
  }
  __syncthreads();
  double v[8];
  walk_tile<8>(
      S, m, sd.my, sd.mz, T0x + 1 - half, T0y + 1 - half, T0z + 1 - half,
      [&](int k, int li_, int64_t) { v[k] = blk[li_]; },
      [&](int k, int, int64_t gi) {
        if (v[k] != 0.0) flush_add<A>(grid, gi, v[k], grid32);
      });
  break;
  }
  }
}

// Interpolation (Alg. 2 step 5 and eq. force): phi = sum b w_x w_y w_z and its gradient as
// nested sums: each lane runs the x-sums of its lines for the value and the x-derivative,
// weights them with the y/z windows and derivatives, and the 16 lanes of a particle reduce.
// grid_override (single system) replaces the system's grid_b; energy holds one double per
// system. G is the arithmetic of the window values and sums: float64, or float32 for the float32
// arithmetic path (the potential, self term and energy are then still formed in float64).
//
// The particles [p0, p1) of one tile against its S^3 block in LDS (tb, x fastest). The first
// records (at p0 + slot) are passed in, loaded by the caller.
template <class T, int P, int D, class G>
struct GatherOut {
  T* phi;
  T* vec;
  int vec_mode, add_self;
  const double* phi_add;
  const double* vec_add;
};

template <class T, int P, int D, class G>
__device__ __forceinline__ void gather_tile(const typename Vec4<T>::type* __restrict__ sorted,
                                            const int* __restrict__ cells, const int* __restrict__ perm, int p0,
                                            int p1, int T0x, int T0y, int T0z, int S, const T* tb, G* recs,
                                            const double* lcoef, const SysDesc& sd,
                                            const GatherOut<T, P, D, G>& out, typename Vec4<T>::type r_next,
                                            int c_next, int i_next, double& esum) {
  constexpr int REC = 6 * P;  // values x, y, z then derivatives x, y, z (d/dg)
  constexpr int CS = coef_stride(D);
  const int nslots = blockDim.x / kLanesPerParticle;
  const int lane = threadIdx.x & 63;
  const int slot = threadIdx.x >> 4;
  const int li = lane & (kLanesPerParticle - 1);
  G* rec = recs + slot * REC;
  const int nt = p1 - p0;
  for (int base = 0; base < nt; base += nslots) {
    const int pi = p0 + base + slot;
    const bool active = pi < p1;
    const auto r = r_next;
    const int cp = c_next;
    const int idx = i_next;
    r_next = sorted[min(pi + nslots, p1 - 1)];
    c_next = cells[min(pi + nslots, p1 - 1)];
    i_next = perm[min(pi + nslots, p1 - 1)];
    int o[3];
    double g[3];
    g[0] = static_cast<double>(r.x);
    o[0] = cell_x(cp) - T0x;
    g[1] = static_cast<double>(r.y);
    o[1] = cell_y(cp) - T0y;
    g[2] = static_cast<double>(r.z);
    o[2] = cell_z(cp) - T0z;
#pragma unroll
    for (int jj = 0; jj < (P + kLanesPerParticle - 1) / kLanesPerParticle; ++jj) {
      const int j = li + kLanesPerParticle * jj;
      if (j >= P) break;
      double c[D + 1];
#pragma unroll
      for (int k = 0; k <= D; ++k) c[k] = lcoef[j * CS + k];
      double v0 = c[D], v1 = c[D], v2 = c[D], d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
      for (int k = D - 1; k >= 0; --k) {
        d0 = fma(d0, g[0], v0);
        d1 = fma(d1, g[1], v1);
        d2 = fma(d2, g[2], v2);
        v0 = fma(v0, g[0], c[k]);
        v1 = fma(v1, g[1], c[k]);
        v2 = fma(v2, g[2], c[k]);
      }
      rec[j] = static_cast<G>(v0);
      rec[P + j] = static_cast<G>(v1);
      rec[2 * P + j] = static_cast<G>(v2);
      rec[3 * P + j] = static_cast<G>(d0);
      rec[4 * P + j] = static_cast<G>(d1);
      rec[5 * P + j] = static_cast<G>(d2);
    }
    wave_lds_sync();
    G ph = 0, gx = 0, gy = 0, gz = 0;
    if (active) {
      G wx[P], dx[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        wx[j] = rec[j];
        dx[j] = rec[3 * P + j];
      }
      auto load_row = [&](int roff, T (&bl)[P]) {
        const T* row = tb + roff;
#pragma unroll
        for (int jx = 0; jx < P; ++jx) bl[jx] = row[jx];
      };
      auto sum_row = [&](int jy, int jz, const T (&bl)[P]) {
        G sx0 = 0, sx1 = 0, sd0 = 0, sd1 = 0;
#pragma unroll
        for (int jx = 0; jx + 1 < P; jx += 2) {
          const G b0 = static_cast<G>(bl[jx]), b1 = static_cast<G>(bl[jx + 1]);
          sx0 = fma(b0, wx[jx], sx0);
          sd0 = fma(b0, dx[jx], sd0);
          sx1 = fma(b1, wx[jx + 1], sx1);
          sd1 = fma(b1, dx[jx + 1], sd1);
        }
        if constexpr (P % 2 == 1) {
          const G b = static_cast<G>(bl[P - 1]);
          sx0 = fma(b, wx[P - 1], sx0);
          sd0 = fma(b, dx[P - 1], sd0);
        }
        const G sx = sx0 + sx1, sdx = sd0 + sd1;
        const G wy = rec[P + jy], dy = rec[4 * P + jy], wz = rec[2 * P + jz], dz = rec[5 * P + jz];
        const G wyz = wy * wz;
        ph = fma(sx, wyz, ph);
        gx = fma(sdx, wyz, gx);
        gy = fma(sx, dy * wz, gy);
        gz = fma(sx, wy * dz, gz);
      };
      constexpr int L = kLanesPerParticle;
      {
        // one row at a time, its values loaded together before they are summed (two row
        // buffers, the next row's loads in flight during the sums, measured slower). Row e =
        // (jy, jz) = (e mod P, e / P) of the lane's rows e = li, li + L, ... and its offset in
        // the block advance by constant steps (one more z-line when jy passes P), without a
        // division per row.
        constexpr int DY = L % P, DZ = L / P;
        int jz = li / P, jy = li - jz * P;
        int roff = ((o[2] + jz) * S + (o[1] + jy)) * S + o[0];
        const int step = (DZ * S + DY) * S, wrap = (S - P) * S;
#pragma unroll 2
        for (int e = li; e < P * P; e += L) {
          T bl[P];
          load_row(roff, bl);
          sum_row(jy, jz, bl);
          jy += DY;
          jz += DZ;
          roff += step;
          if (jy >= P) {
            jy -= P;
            jz += 1;
            roff += wrap;
          }
        }
      }
    }
#pragma unroll
    for (int off = kLanesPerParticle / 2; off > 0; off >>= 1) {
      ph += __shfl_xor(ph, off, kLanesPerParticle);
      gx += __shfl_xor(gx, off, kLanesPerParticle);
      gy += __shfl_xor(gy, off, kLanesPerParticle);
      gz += __shfl_xor(gz, off, kLanesPerParticle);
    }
    if (active && li == 0) {
      const double qd = static_cast<double>(r.w);
      if (qd != qd) ph = gx = gy = gz = static_cast<G>(qd);  // binning marks a non-finite position with a NaN charge
      double phd = static_cast<double>(ph);
      if (out.add_self) phd -= sd.self_coef * qd;
      if (out.phi_add) phd += out.phi_add[idx];  // the real-space residual, computed alongside (float64)
      if (out.phi) out.phi[idx] = static_cast<T>(phd);
      if (out.vec) {
        const double sc = out.vec_mode == 0 ? -qd : 1.0;  // d/dx_d = (1 / h_d) d/dg_d
        double v0 = sc * sd.inv_h * static_cast<double>(gx), v1 = sc * sd.inv_hy * static_cast<double>(gy),
               v2 = sc * sd.inv_hz * static_cast<double>(gz);
        if (out.vec_add) {
          v0 += out.vec_add[3 * idx + 0];
          v1 += out.vec_add[3 * idx + 1];
          v2 += out.vec_add[3 * idx + 2];
        }
        out.vec[3 * idx + 0] = static_cast<T>(v0);
        out.vec[3 * idx + 1] = static_cast<T>(v1);
        out.vec[3 * idx + 2] = static_cast<T>(v2);
      }
      esum += qd * phd;
    }
    wave_lds_sync();
  }
}

// The workgroup's energy sum into energy[s] (one atomic per workgroup).
__device__ __forceinline__ void gather_energy(double esum, double* s_red, double* energy) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) esum += __shfl_xor(esum, off, 64);
  if (lane == 0) s_red[threadIdx.x >> 6] = esum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) tot += s_red[w];
    safeAtomicAdd(energy, 0.5 * tot);  // caller's memory: the CAS form
  }
}

template <class T, int P, int D, class G>
__global__ __launch_bounds__(particle_max_threads<P>()) void k_gather(const typename Vec4<T>::type* __restrict__ sorted,
                                                const int* __restrict__ cells, const int* __restrict__ perm,
                                                const int* __restrict__ tile_start, int sub_log2, int nsys,
                                                const SysDesc* __restrict__ sys, const int* __restrict__ tile_prefix,
                                                const int* __restrict__ tile_sys, int tile_offset, int parts, int xcd,
                                                const T* __restrict__ grid_override, T* __restrict__ phi,
                                                T* __restrict__ vec, int vec_mode, int add_self,
                                                double* __restrict__ energy, const double* __restrict__ phi_add,
                                                const double* __restrict__ vec_add) {
  constexpr int CS = coef_stride(D);
  // dynamic LDS only (see k_spread_mfma)
  extern __shared__ unsigned char smem_raw[];
  const int wgid = tile_order_block(xcd);
  const int gtile = tile_offset + wgid / parts;
  int p0, p1;
  tile_slice(tile_start, gtile, sub_log2, wgid % parts, parts, p0, p1);
  if (p0 == p1) return;
  const int s = nsys == 1 ? 0 : tile_sys[find_sys(tile_prefix, nsys, gtile)];
  const SysDesc& sd = sys[s];
  const int m = sd.m, B = sd.B, Tn = sd.Tn, S = sd.S;
  const global_ptr<T> grid = as_global(grid_override ? grid_override : static_cast<const T*>(sd.grid_b));
  // the S^3 block first, at LDS address 0, so that a row's offsets from its first value fit
  // the immediate offsets of the LDS loads; then the energy's per-wave sums (16), the
  // coefficients (P * CS) and one window record per particle slot
  T* tb = reinterpret_cast<T*>(smem_raw);
  double* s_red = reinterpret_cast<double*>(smem_raw + gather_block_bytes(S, sizeof(T)));
  double* lcoef = s_red + 16;
  G* recs = reinterpret_cast<G*>(lcoef + P * CS);
  const int tile = gtile - sd.tile_base;
  const int tx = tile % Tn, ty = (tile / Tn) % sd.Tny, tz = tile / (Tn * sd.Tny);
  const int T0x = tx * B, T0y = ty * B, T0z = tz * B;
  const int half = (P + 1) / 2;
  const int Ox = T0x + 1 - half, Oy = T0y + 1 - half, Oz = T0z + 1 - half;
  const int slot = threadIdx.x >> 4;
  // the first particles' records are loaded before the grid block is staged: the two round
  // trips to memory overlap
  const auto r0 = sorted[min(p0 + slot, p1 - 1)];
  const int c0 = cells[min(p0 + slot, p1 - 1)];
  const int i0 = perm[min(p0 + slot, p1 - 1)];
  static_assert(P * coef_stride(D) <= kCoefPerThread * 256, "coefficients per thread");
  double cv[kCoefPerThread];
  coef_load<P, D>(sd.coef, sd.deg, cv);
  // the S^3 block: by aligned 16-byte loads of whole row segments where no row wraps around the
  // grid in x (and rows start on 16 bytes), else point by point
  constexpr int VW = 16 / static_cast<int>(sizeof(T));  // values per 16-byte load
  const T* gsrc = grid_override ? grid_override : static_cast<const T*>(sd.grid_b);
  // the chunks of a row end at or before the row's end: x + S <= m and m is a multiple of VW
  if (Ox >= 0 && Ox + S <= m && m % VW == 0 && (reinterpret_cast<uintptr_t>(gsrc) & 15) == 0) {
    using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const int a0 = Ox & ~(VW - 1);                         // first aligned x of every row
    const int nch = (Ox + S - a0 + VW - 1) / VW;           // 16-byte chunks per row
    const int items = S * S * nch;
    const int nt = static_cast<int>(blockDim.x);
    constexpr int K = 4;
    for (int base = threadIdx.x; base < items; base += nt * K) {
      V16 v[K];
      int row[K], ch[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int it = base + k * nt;
        row[k] = it / nch;
        ch[k] = it - row[k] * nch;
        if (it < items) {
          const int z = row[k] / S, y = row[k] - z * S;
          const int64_t g0 = (static_cast<int64_t>(fold_index(Oz + z, sd.mz)) * sd.my + fold_index(Oy + y, sd.my)) * m + a0;
          v[k] = *reinterpret_cast<const V16*>(gsrc + g0 + ch[k] * VW);
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (base + k * nt >= items) continue;
        const T* e = reinterpret_cast<const T*>(&v[k]);
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          const int x = a0 + ch[k] * VW + j - Ox;
          if (x >= 0 && x < S) tb[row[k] * S + x] = e[j];
        }
      }
    }
  } else {
    T v[8];
    walk_tile<8>(
        S, m, sd.my, sd.mz, Ox, Oy, Oz, [&](int k, int, int64_t gi) { v[k] = grid[gi]; },
        [&](int k, int li_, int64_t) { tb[li_] = v[k]; });
  }
  coef_store<P, D>(lcoef, cv);
  __syncthreads();
  double esum = 0.0;
  const GatherOut<T, P, D, G> out{phi, vec, vec_mode, add_self, phi_add, vec_add};
  gather_tile<T, P, D, G>(sorted, cells, perm, p0, p1, T0x, T0y, T0z, S, tb, recs, lcoef, sd, out, r0, c0, i0, esum);
  if (energy) gather_energy(esum, s_red, energy + s);
}

// Interpolation of one system by a fixed grid of workgroups that each take a sequence of tiles
// (float64 plans on large grids, where one 125 KB block per compute unit leaves no second
// workgroup to hide the block's loading). While a tile's particles are interpolated from its
// block in LDS, the first half of the next tile's block is loaded into registers as aligned
// 16-byte row segments and written to LDS once the tile is done, with the rest (at most
// kStreamChunks segments per thread in all); a tile whose rows wrap around the grid in x, or whose
// block has more segments, is loaded after the tile instead.
// Workgroup w runs on XCD w mod 8 (the dispatch order): the XCD's workgroups take consecutive
// tiles of one eighth of the tile range, so neighbouring tiles' overlapping blocks are read
// through the same L2.
constexpr int kStreamChunks = 16;
// segments per thread loaded ahead, during the previous tile (registers held across its
// interpolation: 16 took 256 VGPRs and spilled)
constexpr int kStreamAhead = 4;

template <class T>
struct StreamBlock {
  int Ox, Oy, Oz, a0, nch, items;
  bool vec;  // loaded as 16-byte segments
};

template <class T, int P, int D, class G>
__global__ __launch_bounds__(particle_max_threads<P>()) void k_gather_stream(
    const typename Vec4<T>::type* __restrict__ sorted, const int* __restrict__ cells, const int* __restrict__ perm,
    const int* __restrict__ tile_start, int sub_log2, const SysDesc* __restrict__ sys, int tile_offset, int ntiles,
    const T* __restrict__ grid_override, T* __restrict__ phi, T* __restrict__ vec, int vec_mode, int add_self,
    double* __restrict__ energy, const double* __restrict__ phi_add, const double* __restrict__ vec_add) {
  constexpr int CS = coef_stride(D);
  constexpr int VW = 16 / static_cast<int>(sizeof(T));
  using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[0];
  const int m = sd.m, B = sd.B, Tn = sd.Tn, S = sd.S;
  T* tb = reinterpret_cast<T*>(smem_raw);
  double* s_red = reinterpret_cast<double*>(smem_raw + gather_block_bytes(S, sizeof(T)));
  double* lcoef = s_red + 16;
  G* recs = reinterpret_cast<G*>(lcoef + P * CS);
  const T* gsrc = grid_override ? grid_override : static_cast<const T*>(sd.grid_b);
  const bool aligned = m % VW == 0 && (reinterpret_cast<uintptr_t>(gsrc) & 15) == 0;
  const int nt = static_cast<int>(blockDim.x), t = static_cast<int>(threadIdx.x);
  const int half = (P + 1) / 2;
  // tile sequence: XCD x = w mod 8 takes tiles [x per, (x + 1) per), its workgroups in turn
  const int w = static_cast<int>(blockIdx.x), G8 = static_cast<int>(gridDim.x) / 8;
  const int xcd = w % 8, per = (ntiles + 7) / 8;
  const int first = xcd * per, last = min(ntiles, first + per);
  auto block_of = [&](int u) {
    const int tile = tile_offset + u - sd.tile_base;
    const int tx = tile % Tn, ty = (tile / Tn) % sd.Tny, tz = tile / (Tn * sd.Tny);
    StreamBlock<T> b;
    b.Ox = tx * B + 1 - half;
    b.Oy = ty * B + 1 - half;
    b.Oz = tz * B + 1 - half;
    b.a0 = b.Ox & ~(VW - 1);
    b.nch = (b.Ox + S - b.a0 + VW - 1) / VW;
    b.items = S * S * b.nch;
    b.vec = aligned && b.Ox >= 0 && b.Ox + S <= m && b.items <= kStreamChunks * nt;
    return b;
  };
  auto seg_addr = [&](const StreamBlock<T>& b, int it, int& row, int& ch) {
    row = it / b.nch;
    ch = it - row * b.nch;
    const int z = row / S, y = row - z * S;
    return (static_cast<int64_t>(fold_index(b.Oz + z, sd.mz)) * sd.my + fold_index(b.Oy + y, sd.my)) * m + b.a0 +
           ch * VW;
  };
  auto seg_store = [&](const StreamBlock<T>& b, int row, int ch, const V16& v) {
    const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
    for (int j = 0; j < VW; ++j) {
      const int x = b.a0 + ch * VW + j - b.Ox;
      if (x >= 0 && x < S) tb[row * S + x] = e[j];
    }
  };
  auto stage_now = [&](const StreamBlock<T>& b) {  // the block loaded and stored in one pass
    if (b.vec) {
      V16 v[kStreamChunks];
#pragma unroll
      for (int k = 0; k < kStreamChunks; ++k) {
        const int it = t + k * nt;
        int row, ch;
        if (it < b.items) v[k] = *reinterpret_cast<const V16*>(gsrc + seg_addr(b, it, row, ch));
      }
#pragma unroll
      for (int k = 0; k < kStreamChunks; ++k) {
        const int it = t + k * nt;
        int row, ch;
        if (it < b.items) {
          (void)seg_addr(b, it, row, ch);
          seg_store(b, row, ch, v[k]);
        }
      }
    } else {
      const global_ptr<T> grid = as_global(gsrc);
      T v[8];
      walk_tile<8>(
          S, m, sd.my, sd.mz, b.Ox, b.Oy, b.Oz, [&](int k, int, int64_t gi) { v[k] = grid[gi]; },
          [&](int k, int li_, int64_t) { tb[li_] = v[k]; });
    }
  };
  int u = first + w / 8;
  if (G8 == 0 || u >= last) return;
  double cv[kCoefPerThread];
  coef_load<P, D>(sd.coef, sd.deg, cv);
  StreamBlock<T> cur = block_of(u);
  stage_now(cur);
  coef_store<P, D>(lcoef, cv);
  __syncthreads();
  double esum = 0.0;
  const GatherOut<T, P, D, G> out{phi, vec, vec_mode, add_self, phi_add, vec_add};
  const int slot = t >> 4;
  for (;;) {
    const int un = u + G8;
    const bool more = un < last;
    StreamBlock<T> nxt{};
    V16 pre[kStreamAhead];
    if (more) {
      nxt = block_of(un);
      if (nxt.vec) {
#pragma unroll
        for (int k = 0; k < kStreamAhead; ++k) {
          const int it = t + k * nt;
          int row, ch;
          if (it < nxt.items) pre[k] = *reinterpret_cast<const V16*>(gsrc + seg_addr(nxt, it, row, ch));
        }
      }
    }
    const int gtile = tile_offset + u;
    const int p0 = tile_start[gtile << sub_log2], p1 = tile_start[(gtile + 1) << sub_log2];
    if (p1 > p0) {
      const int tile = gtile - sd.tile_base;
      const int tx = tile % Tn, ty = (tile / Tn) % sd.Tny, tz = tile / (Tn * sd.Tny);
      const auto r0 = sorted[min(p0 + slot, p1 - 1)];
      const int c0 = cells[min(p0 + slot, p1 - 1)];
      const int i0 = perm[min(p0 + slot, p1 - 1)];
      gather_tile<T, P, D, G>(sorted, cells, perm, p0, p1, tx * B, ty * B, tz * B, S, tb, recs, lcoef, sd, out, r0,
                              c0, i0, esum);
    }
    __syncthreads();  // every read of this tile's block is done
    if (!more) break;
    if (nxt.vec) {
      // the segments not loaded ahead, their loads issued before the stores of those that were
      V16 rest[kStreamChunks - kStreamAhead];
#pragma unroll
      for (int k = kStreamAhead; k < kStreamChunks; ++k) {
        const int it = t + k * nt;
        int row, ch;
        if (it < nxt.items) rest[k - kStreamAhead] = *reinterpret_cast<const V16*>(gsrc + seg_addr(nxt, it, row, ch));
      }
#pragma unroll
      for (int k = 0; k < kStreamChunks; ++k) {
        const int it = t + k * nt;
        int row, ch;
        if (it < nxt.items) {
          (void)seg_addr(nxt, it, row, ch);
          seg_store(nxt, row, ch, k < kStreamAhead ? pre[k] : rest[k - kStreamAhead]);
        }
      }
    } else {
      stage_now(nxt);
    }
    __syncthreads();
    u = un;
    cur = nxt;
  }
  if (energy) gather_energy(esum, s_red, energy);
}

template <class T, int P, int D>
hipError_t spread_impl(const DevPlan& d, const PGroup& g, hipStream_t st) {
  auto cols = [&](auto kern, int threads) {
    hipLaunchKernelGGL(kern, dim3((g.tile_end - g.tile_begin) * g.parts), dim3(threads), g.lds_spread, st,
                       static_cast<const typename Vec4<T>::type*>(d.sorted), d.cells, d.tile_start, d.sub_log2, d.nsys,
                       d.sys_dev, d.tile_prefix, d.tile_sys, g.tile_begin, g.parts, g.xcd_spread);
  };
  if (g.mfma) {
    auto launch = [&](auto kern, int threads) {
      const bool roll = g.roll_len > 0;
      hipLaunchKernelGGL(kern, dim3(roll ? g.roll_cols * g.roll_nseg : (g.tile_end - g.tile_begin) * g.parts),
                         dim3(threads), g.lds_spread, st, static_cast<const typename Vec4<T>::type*>(d.sorted),
                         d.cells, d.tile_start, d.sub_log2, d.nsys, d.sys_dev, d.tile_prefix, d.tile_sys,
                         g.tile_begin, g.parts, g.xcd_spread, g.roll_len, g.roll_nseg, d.grid32);
    };
    auto mf = [&](auto acc) {
      using A = decltype(acc);
      const bool roll = g.roll_len > 0;
      if (g.col_tile == 4)
        roll ? launch(k_spread_mfma<T, P, D, 4, A, true>, mfma_threads<P, 4>())
             : launch(k_spread_mfma<T, P, D, 4, A, false>, mfma_threads<P, 4>());
      else if (g.col_tile == 6)
        roll ? launch(k_spread_mfma<T, P, D, 6, A, true>, mfma_threads<P, 6>())
             : launch(k_spread_mfma<T, P, D, 6, A, false>, mfma_threads<P, 6>());
      else
        roll ? launch(k_spread_mfma<T, P, D, 8, A, true>, mfma_threads<P, 8>())
             : launch(k_spread_mfma<T, P, D, 8, A, false>, mfma_threads<P, 8>());
    };
    if constexpr (std::is_same_v<T, float>) {
      if (g.acc32) {
        mf(float());
        return hipGetLastError();
      }
    }
    mf(double());
  } else if (g.col_tile == 4)
    cols(k_spread_cols<T, P, D, 4>, col_threads<P, 4>());
  else if (g.col_tile == 6)
    cols(k_spread_cols<T, P, D, 6>, col_threads<P, 6>());
  else if (g.col_tile == 8)
    cols(k_spread_cols<T, P, D, 8>, col_threads<P, 8>());
  else
    hipLaunchKernelGGL((k_spread<T, P, D>), dim3((g.tile_end - g.tile_begin) * g.parts), dim3(g.spread_threads),
                       g.lds_spread, st, static_cast<const typename Vec4<T>::type*>(d.sorted), d.cells, d.tile_start,
                       d.sub_log2, d.nsys, d.sys_dev, d.tile_prefix, d.tile_sys, g.tile_begin, g.parts,
                       g.xcd_spread);
  return hipGetLastError();
}

template <class T, int P, int D>
hipError_t gather_impl(const DevPlan& d, const PGroup& g, const void* grid, void* phi, void* vec, int vec_mode,
                       bool add_self, double* energy, const double* phi_add, const double* vec_add,
                       hipStream_t st) {
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((g.tile_end - g.tile_begin) * g.parts), dim3(g.gather_threads), g.lds_gather, st,
                       static_cast<const typename Vec4<T>::type*>(d.sorted), d.cells, d.perm, d.tile_start, d.sub_log2,
                       d.nsys, d.sys_dev, d.tile_prefix, d.tile_sys, g.tile_begin, g.parts, g.xcd_gather,
                       static_cast<const T*>(grid), static_cast<T*>(phi), static_cast<T*>(vec), vec_mode,
                       add_self ? 1 : 0, energy, phi_add, vec_add);
  };
  if constexpr (std::is_same_v<T, float>) {
    if (g.acc32) {
      launch(k_gather<T, P, D, float>);
      return hipGetLastError();
    }
  } else {
    if (g.gather_stream > 0) {
      hipLaunchKernelGGL((k_gather_stream<T, P, D, double>), dim3(g.gather_stream), dim3(g.gather_threads),
                         g.lds_gather, st, static_cast<const typename Vec4<T>::type*>(d.sorted), d.cells, d.perm,
                         d.tile_start, d.sub_log2, d.sys_dev, g.tile_begin, g.tile_end - g.tile_begin,
                         static_cast<const T*>(grid), static_cast<T*>(phi), static_cast<T*>(vec), vec_mode,
                         add_self ? 1 : 0, energy, phi_add, vec_add);
      return hipGetLastError();
    }
  }
  launch(k_gather<T, P, D, double>);
  return hipGetLastError();
}

// Raises the dynamic-LDS limit of the particle kernels of one group where needed, and turns on
// the XCD-aware tile order for a kernel whose whole grid is resident at once.
template <class T, int P, int D>
const void* mfma_fn(const PGroup& g) {
  auto pick = [&](auto acc) -> const void* {
    using A = decltype(acc);
    if (g.roll_len > 0)
      return g.col_tile == 4   ? reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 4, A, true>)
             : g.col_tile == 6 ? reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 6, A, true>)
                               : reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 8, A, true>);
    return g.col_tile == 4   ? reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 4, A, false>)
           : g.col_tile == 6 ? reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 6, A, false>)
                             : reinterpret_cast<const void*>(&k_spread_mfma<T, P, D, 8, A, false>);
  };
  if constexpr (std::is_same_v<T, float>) {
    if (g.acc32) return pick(float());
  }
  return pick(double());
}

template <class T, int P, int D>
hipError_t prepare_impl(PGroup& g) {
  const void* spread_fn =
      g.mfma                      ? mfma_fn<T, P, D>(g)
      : g.col_tile == 4           ? reinterpret_cast<const void*>(&k_spread_cols<T, P, D, 4>)
      : g.col_tile == 6           ? reinterpret_cast<const void*>(&k_spread_cols<T, P, D, 6>)
      : g.col_tile == 8           ? reinterpret_cast<const void*>(&k_spread_cols<T, P, D, 8>)
                                  : reinterpret_cast<const void*>(&k_spread<T, P, D>);
  const void* gather_fn = reinterpret_cast<const void*>(&k_gather<T, P, D, double>);
  if constexpr (std::is_same_v<T, float>) {
    if (g.acc32) gather_fn = reinterpret_cast<const void*>(&k_gather<T, P, D, float>);
  }
  if (g.lds_spread > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute(spread_fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(g.lds_spread));
    if (e != hipSuccess) return e;
  }
  if (g.lds_gather > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(gather_fn,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(g.lds_gather));
    if (e != hipSuccess) return e;
  }
  bool xcd_ok = true;
  if (const char* env = std::getenv("PSWFE_XCD_ORDER")) xcd_ok = std::atoi(env) != 0;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t grid = static_cast<int64_t>(g.tile_end - g.tile_begin) * g.parts;
  auto resident = [&](const void* fn, int threads, size_t lds, int* out) -> hipError_t {
    int per_cu = 0;
    const hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    *out = r == hipSuccess && xcd_ok && grid >= 8 && grid <= static_cast<int64_t>(per_cu) * cus ? 1 : 0;
    return r;
  };
  e = resident(spread_fn, g.spread_threads, g.lds_spread, &g.xcd_spread);
  if (e == hipSuccess) e = resident(gather_fn, g.gather_threads, g.lds_gather, &g.xcd_gather);
  // the tile-sequence interpolation (float64; asked for by the plan with gather_stream = -1): as
  // many workgroups as are resident at once, a multiple of the 8 XCDs
  if (e == hipSuccess && g.gather_stream < 0) {
    g.gather_stream = 0;
    if constexpr (std::is_same_v<T, double>) {
      const void* fn = reinterpret_cast<const void*>(&k_gather_stream<T, P, D, double>);
      if (g.lds_gather > 64 * 1024)
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(g.lds_gather));
      int per_cu = 0;
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, g.gather_threads, g.lds_gather);
      const int64_t resident_wg = static_cast<int64_t>(per_cu) * cus / 8 * 8;
      if (e == hipSuccess && resident_wg >= 8 && resident_wg < grid) g.gather_stream = static_cast<int>(resident_wg);
    }
  }
  return e;
}

// Calls f.template operator()<P, D>() for the group's (P, D), P in [PSWFE_PLO, PSWFE_PHI];
// hipErrorInvalidValue if none.
template <int P, class F>
hipError_t with_group(const PGroup& g, F&& f) {
  if (g.P == P) {
    if (g.D == 11) return f.template operator()<P, 11>();
    if (g.D == 17) return f.template operator()<P, 17>();
    if (g.D == kMaxDeg) return f.template operator()<P, kMaxDeg>();
    return hipErrorInvalidValue;
  }
  if constexpr (P < PSWFE_PHI) return with_group<P + 1>(g, f);
  return hipErrorInvalidValue;
}

#if PSWFE_PREC == 0
using Real = float;
#else
using Real = double;
#endif

}  // namespace

hipError_t PSWFE_PARTICLE_FN(prepare)(PGroup& g) {
  return with_group<PSWFE_PLO>(g, [&]<int P, int D>() { return prepare_impl<Real, P, D>(g); });
}

hipError_t PSWFE_PARTICLE_FN(spread)(const DevPlan& d, const PGroup& g, hipStream_t st) {
  return with_group<PSWFE_PLO>(g, [&]<int P, int D>() { return spread_impl<Real, P, D>(d, g, st); });
}

hipError_t PSWFE_PARTICLE_FN(gather)(const DevPlan& d, const PGroup& g, const void* grid, void* phi, void* vec,
                                     int vec_mode, bool add_self, double* energy, const double* phi_add,
                                     const double* vec_add, hipStream_t st) {
  return with_group<PSWFE_PLO>(g, [&]<int P, int D>() {
    return gather_impl<Real, P, D>(d, g, grid, phi, vec, vec_mode, add_self, energy, phi_add, vec_add, st);
  });
}

}  // namespace pswfe
