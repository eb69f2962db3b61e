// HIP kernels for gfx950: binning, spreading (Alg. 2 step 1), smooth-size FFTs with the
// k-space scaling fused between the forward and inverse z passes (steps 2-4), and
// interpolation of potentials and gradients with the energy reduction (step 5, eq. force).
// Each kernel covers every system of a batch in one launch: a workgroup (or, in binning, a
// thread) looks up its system in a prefix table of the global index space it runs over.
#include "device_common.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <utility>

namespace pswfe {
namespace {
// ------------------------------------------------------------------------------------
// Binning: a counting sort of the particles by bucket (the tile of B^3 grid cells that holds
// the particle's support anchor, split into z sub-buckets; packed particle i belongs to the
// system whose range [part_prefix[s], part_prefix[s+1]) holds it). Two levels, so that no step
// issues one global atomic per particle or scatters lone records across memory:
//   k_bin_count   each workgroup takes per_thread particles per thread, stores their buckets and
//                 counts the coarse buckets (bucket >> shift, at most kCoarse of them) in LDS, then
//                 adds each nonzero count to the global coarse counts with one atomic;
//   k_bin_coarse  moves the particles into coarse-bucket order: a workgroup ranks its particles
//                 per coarse bucket in LDS and reserves its range in each coarse bucket with one
//                 atomic, so its particles of one coarse bucket land next to each other;
//   k_bin_fine    one workgroup per coarse bucket counts its particles per bucket in LDS, writes
//                 the bucket starts, and writes each particle's record, cell and original index in
//                 bucket order.
// The coarse counters are zero between calls: k_bin_fine clears them after their last use.
// ------------------------------------------------------------------------------------
constexpr int kBinThreads = 256;
constexpr int kFineThreads = 1024;
constexpr int kFineStage = 128 * 1024;     // LDS staging of the fine pass's records
constexpr size_t kFineLdsMax = 160 * 1024; // LDS per workgroup on gfx950

// Tile bucket of a particle at (x, y, z) (the anchor's tile, and within it the sub-bucket of the
// z-cell: a tile's particles come out ordered by z, so the slices of a tile shared by several
// workgroups cover narrow z-ranges and their partial blocks flush fewer nonzero points); the
// packed anchor and the centred offsets g go to `cell` and `g`.
template <class T>
__device__ __forceinline__ int bin_bucket(const SysDesc& sd, int sub_log2, T x, T y, T z, int& cell, T g[3]) {
  T f[3];
  const int c0 = grid_coord(x, T(sd.ih_hi), T(sd.ih_lo), T(sd.L), sd.m, f[0]);
  const int c1 = grid_coord(y, T(sd.ihy_hi), T(sd.ihy_lo), T(sd.Ly), sd.my, f[1]);
  const int c2 = grid_coord(z, T(sd.ihz_hi), T(sd.ihz_lo), T(sd.Lz), sd.mz, f[2]);
  const int cx = support_anchor(c0, f[0], sd.P, sd.m, g[0]);
  const int cy = support_anchor(c1, f[1], sd.P, sd.my, g[1]);
  const int cz = support_anchor(c2, f[2], sd.P, sd.mz, g[2]);
  const int B = sd.B;
  cell = pack_cell(cx, cy, cz);
  const int tile = sd.tile_base + ((cz / B) * sd.Tny + cy / B) * sd.Tn + cx / B;
  return (tile << sub_log2) | (((cz % B) << sub_log2) / B);
}

// Exclusive prefix sum of a[0, count) in LDS, in place, by the whole workgroup; returns the total.
// Each thread sums a run of consecutive entries, the run sums are scanned across lanes and waves
// (s_wave: one int per wave), then each thread rewrites its run. Ends with a barrier.
__device__ __forceinline__ int block_scan_lds(int* a, int count, int* s_wave) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int per = (count + static_cast<int>(blockDim.x) - 1) / static_cast<int>(blockDim.x);
  const int b0 = min(tid * per, count), b1 = min(b0 + per, count);
  int sum = 0;
  for (int i = b0; i < b1; ++i) sum += a[i];
  int x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wid] = x;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    const int v = s_wave[w];
    before += w < wid ? v : 0;
    total += v;
  }
  int run = before + x - sum;
  for (int i = b0; i < b1; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

template <class T>
__global__ __launch_bounds__(kBinThreads) void k_bin_count(int64_t n, int nsys, const SysDesc* __restrict__ sys,
                                                        const int64_t* __restrict__ part_prefix,
                                                        const T* __restrict__ pos, int sub_log2, int per_thread,
                                                        int shift, int ncoarse, int* __restrict__ coarse_count,
                                                        int* __restrict__ key, double* __restrict__ energy) {
  __shared__ int hist[kCoarse];
  const int tid = threadIdx.x;
  {
    const int64_t e = blockIdx.x * static_cast<int64_t>(kBinThreads) + tid;
    if (energy && e < nsys) energy[e] = 0.0;
  }
  for (int c = tid; c < kCoarse; c += kBinThreads) hist[c] = 0;
  __syncthreads();
  if (n > 0) {
    const int64_t i0 = blockIdx.x * static_cast<int64_t>(kBinThreads) * per_thread + tid;
    // the systems of the workgroup's particles (one, unless the chunk spans a boundary)
    const int64_t c0 = min(blockIdx.x * static_cast<int64_t>(kBinThreads) * per_thread, n - 1);
    const int64_t c1 = min(c0 + static_cast<int64_t>(kBinThreads) * per_thread, n) - 1;
    const int s_lo = nsys == 1 ? 0 : find_sys(part_prefix, nsys, c0);
    const int s_hi = nsys == 1 ? 0 : find_sys(part_prefix, nsys, c1);
    // every load is issued (at clamped, valid indices) before any position is used
    T x[kBinMaxPerThread][3];
#pragma unroll
    for (int k = 0; k < kBinMaxPerThread; ++k) {
      const int64_t i = min(i0 + static_cast<int64_t>(min(k, per_thread - 1)) * kBinThreads, n - 1);
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) x[k][dd] = pos[3 * i + dd];
    }
#pragma unroll
    for (int k = 0; k < kBinMaxPerThread; ++k) {
      const int64_t i = i0 + static_cast<int64_t>(k) * kBinThreads;
      if (k < per_thread && i < n) {
        const SysDesc& sd = sys[s_lo == s_hi ? s_lo : find_sys_in(part_prefix, s_lo, s_hi, i)];
        int cell;
        T g[3];
        const int b = bin_bucket(sd, sub_log2, x[k][0], x[k][1], x[k][2], cell, g);
        key[i] = b;
        atomicAdd(&hist[b >> shift], 1);
      }
    }
  }
  __syncthreads();
  int* __restrict__ mine = coarse_count + (blockIdx.x % kCoarseCopies) * kCoarse;
  for (int c = tid; c < ncoarse; c += kBinThreads)
    if (hist[c] > 0) atomicAdd(&mine[c], hist[c]);
}

// LDS of the coarse pass: coarse starts, counts, local starts, wave sums, then the workgroup's
// records and (index, bucket) pairs in coarse-bucket order.
template <class T>
constexpr size_t coarse_lds_bytes() {
  return sizeof(int) * (3 * kCoarse + 16) + (sizeof(typename Vec4<T>::type) + sizeof(int2)) * kBinThreads * kBinMaxPerThread;
}

template <class T>
__global__ __launch_bounds__(kBinThreads) void k_bin_coarse(int64_t n, const T* __restrict__ pos,
                                                         const T* __restrict__ q, int per_thread, int shift,
                                                         int ncoarse, const int* __restrict__ coarse_count,
                                                         int* __restrict__ coarse_cursor,
                                                         int* __restrict__ coarse_start, const int* __restrict__ key,
                                                         typename Vec4<T>::type* __restrict__ tmp_rec,
                                                         int2* __restrict__ tmp_ib) {
  using V = typename Vec4<T>::type;
  extern __shared__ int smem_int[];
  int* s_start = smem_int;                 // kCoarse
  int* hist = s_start + kCoarse;           // kCoarse: counts, then the global slot of each run
  int* s_lp = hist + kCoarse;              // kCoarse: start of each coarse bucket's run in the stage
  int* s_wave = s_lp + kCoarse;            // 16
  V* st_rec = reinterpret_cast<V*>(s_wave + 16);
  int2* st_ib = reinterpret_cast<int2*>(st_rec + kBinThreads * kBinMaxPerThread);
  const int tid = threadIdx.x;
  const int copy = blockIdx.x % kCoarseCopies;
  const int64_t i0 = blockIdx.x * static_cast<int64_t>(kBinThreads) * per_thread + tid;
  // this thread's particles: bucket, position and charge, all loads issued at once
  int kb[kBinMaxPerThread], lr[kBinMaxPerThread];
  V r[kBinMaxPerThread];
#pragma unroll
  for (int k = 0; k < kBinMaxPerThread; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * kBinThreads;
    const int64_t ic = min(i0 + static_cast<int64_t>(min(k, per_thread - 1)) * kBinThreads, n - 1);
    kb[k] = key[ic];
    if (!(k < per_thread && i < n)) kb[k] = -1;
    r[k].x = pos[3 * ic + 0];
    r[k].y = pos[3 * ic + 1];
    r[k].z = pos[3 * ic + 2];
    r[k].w = q ? q[ic] : T(0);
  }
  // coarse starts (the scan over all copies) and this copy's offset within each coarse bucket
  int own = 0;
  if (tid < kCoarse) {
    int tot = 0;
    if (tid < ncoarse) {
#pragma unroll
      for (int k = 0; k < kCoarseCopies; ++k) {
        const int v = coarse_count[k * kCoarse + tid];
        own += k < copy ? v : 0;
        tot += v;
      }
    }
    s_start[tid] = tot;
    hist[tid] = 0;
  }
  __syncthreads();
  const int total = block_scan_lds(s_start, ncoarse, s_wave);
  if (blockIdx.x == 0) {
    for (int c = tid; c < ncoarse; c += kBinThreads) coarse_start[c] = s_start[c];
    if (tid == 0) coarse_start[ncoarse] = total;
  }
#pragma unroll
  for (int k = 0; k < kBinMaxPerThread; ++k)
    if (kb[k] >= 0) lr[k] = atomicAdd(&hist[kb[k] >> shift], 1);
  __syncthreads();
  if (tid < kCoarse) s_lp[tid] = tid < ncoarse ? hist[tid] : 0;
  __syncthreads();
  const int cnt = block_scan_lds(s_lp, ncoarse, s_wave);
  // each nonzero count becomes the workgroup's first slot in that coarse bucket
  if (tid < ncoarse && hist[tid] > 0)
    hist[tid] = s_start[tid] + own + atomicAdd(&coarse_cursor[copy * kCoarse + tid], hist[tid]);
  // the workgroup's particles in coarse-bucket order in LDS
#pragma unroll
  for (int k = 0; k < kBinMaxPerThread; ++k) {
    if (kb[k] < 0) continue;
    const int sp = s_lp[kb[k] >> shift] + lr[k];
    st_rec[sp] = r[k];
    st_ib[sp] = int2{static_cast<int>(i0 + static_cast<int64_t>(k) * kBinThreads), kb[k]};
  }
  __syncthreads();
  // then stored run by run: consecutive lanes on consecutive slots of one coarse bucket
  for (int p = tid; p < cnt; p += kBinThreads) {
    const int2 iv = st_ib[p];
    const int cb = iv.y >> shift;
    const int dst = hist[cb] + (p - s_lp[cb]);
    if (dst >= n) continue;  // only if the coarse counters were not zero at the start
    tmp_rec[dst] = st_rec[p];
    tmp_ib[dst] = iv;
  }
}

// Sorted record: (g_x, g_y, g_z, q), the centred offsets from the support anchors, and the
// packed anchor of the particle in its system. A coarse bucket of up to kFineRes items per thread
// is held in registers from one round of loads; when `staged`, its records are then put in bucket
// order in LDS (kFineStage bytes at a time) and stored with consecutive lanes on consecutive
// addresses, instead of one scattered store per lane. Larger coarse buckets are read twice and
// stored directly.
constexpr int kFineRes = 8;
template <class T>
__global__ __launch_bounds__(kFineThreads) void k_bin_fine(int64_t n, int nsys, const SysDesc* __restrict__ sys,
                                                        const int* __restrict__ tile_prefix,
                                                        const int* __restrict__ tile_sys, int sub_log2, int shift,
                                                        int ncoarse, int nbuckets, const int* __restrict__ coarse_start,
                                                        int* __restrict__ coarse_count, int* __restrict__ coarse_cursor,
                                                        const typename Vec4<T>::type* __restrict__ tmp_rec,
                                                        const int2* __restrict__ tmp_ib, int* __restrict__ tile_start,
                                                        typename Vec4<T>::type* __restrict__ sorted,
                                                        int* __restrict__ cells, int* __restrict__ perm, int staged) {
  using V = typename Vec4<T>::type;
  extern __shared__ int smem_int[];
  const int nf = 1 << shift;
  int* fine = smem_int;             // nf: counts, then cursors
  int* s_wave = smem_int + nf;      // kFineThreads / 64
  // staging area, 16-byte aligned, after the counters
  unsigned char* stage = reinterpret_cast<unsigned char*>(smem_int + ((nf + kFineThreads / 64 + 3) & ~3));
  const int tid = threadIdx.x, c = blockIdx.x;
  // clamped to [0, n]: the ranges are inside the particle arrays whatever the counters held
  const int s1 = static_cast<int>(min<int64_t>(max(coarse_start[c + 1], 0), n));
  const int s0 = min(max(coarse_start[c], 0), s1);
  const bool resident = s1 - s0 <= kFineRes * kFineThreads;
  // the (group-ordered) systems whose tiles this coarse bucket covers: an item's system follows
  // from its bucket's tile, searched within that range
  const int k_lo = nsys == 1 ? 0 : find_sys(tile_prefix, nsys, (c << shift) >> sub_log2);
  const int k_hi = nsys == 1 ? 0 : find_sys(tile_prefix, nsys, (min(nbuckets, (c + 1) << shift) - 1) >> sub_log2);
  V r[kFineRes];
  int2 ib[kFineRes];
  if (resident) {
#pragma unroll
    for (int u = 0; u < kFineRes; ++u) {
      const int j = min(s0 + tid + u * kFineThreads, s1 - 1);
      if (s1 > s0) {
        r[u] = tmp_rec[j];
        ib[u] = tmp_ib[j];
      }
    }
  }
  for (int f = tid; f < nf; f += kFineThreads) fine[f] = 0;
  __syncthreads();
  if (resident) {
#pragma unroll
    for (int u = 0; u < kFineRes; ++u)
      if (s0 + tid + u * kFineThreads < s1) atomicAdd(&fine[ib[u].y & (nf - 1)], 1);
  } else {
    for (int j = s0 + tid; j < s1; j += kFineThreads) atomicAdd(&fine[tmp_ib[j].y & (nf - 1)], 1);
  }
  __syncthreads();
  block_scan_lds(fine, nf, s_wave);
  const int b0 = c << shift;
  for (int f = tid; f < nf; f += kFineThreads) {
    const int st = fine[f] + s0;
    fine[f] = st;
    if (b0 + f < nbuckets) tile_start[b0 + f] = st;
  }
  if (c == ncoarse - 1 && tid == 0) tile_start[nbuckets] = s1;
  for (int k = tid; k < kCoarseCopies; k += kFineThreads) {
    coarse_count[k * kCoarse + c] = 0;
    coarse_cursor[k * kCoarse + c] = 0;
  }
  __syncthreads();
  // the final record of one item, and its slot (or -1 when the counters were inconsistent)
  auto finish = [&](const V rv, int2 iv, V& rec, int& cell) {  // rv by value: rec may be its source
    const int dst = atomicAdd(&fine[iv.y & (nf - 1)], 1);
    const SysDesc& sd =
        sys[nsys == 1 ? 0 : tile_sys[k_lo == k_hi ? k_lo : find_sys_in(tile_prefix, k_lo, k_hi, iv.y >> sub_log2)]];
    T g[3];
    bin_bucket(sd, 0, rv.x, rv.y, rv.z, cell, g);
    rec.x = g[0];
    rec.y = g[1];
    rec.z = g[2];
    rec.w = rv.w;
    // a non-finite position is moved to cell 0 by grid_coord; its NaN charge poisons the outputs
    // instead (spreading adds NaN into the grid, interpolation returns NaN for it)
    if (!(isfinite(rv.x) && isfinite(rv.y) && isfinite(rv.z))) rec.w = std::numeric_limits<T>::quiet_NaN();
    return dst < s1 ? dst : -1;
  };
  if (!resident) {
    for (int j = s0 + tid; j < s1; j += kFineThreads) {
      const int2 iv = tmp_ib[j];
      V rec;
      int cell;
      const int dst = finish(tmp_rec[j], iv, rec, cell);
      if (dst < 0) continue;
      sorted[dst] = rec;
      cells[dst] = cell;
      perm[dst] = iv.x;
    }
    return;
  }
  int slot[kFineRes], cl[kFineRes];
#pragma unroll
  for (int u = 0; u < kFineRes; ++u) {
    slot[u] = -1;
    if (s0 + tid + u * kFineThreads < s1) {
      const int dst = finish(r[u], ib[u], r[u], cl[u]);
      slot[u] = dst < 0 ? -1 : dst - s0;
    }
  }
  if (!staged) {
#pragma unroll
    for (int u = 0; u < kFineRes; ++u) {
      if (slot[u] < 0) continue;
      sorted[s0 + slot[u]] = r[u];
      cells[s0 + slot[u]] = cl[u];
      perm[s0 + slot[u]] = ib[u].x;
    }
    return;
  }
  const int cnt = s1 - s0;
  {
    V* sv = reinterpret_cast<V*>(stage);
    constexpr int cap = kFineStage / static_cast<int>(sizeof(V));
    for (int w0 = 0; w0 < cnt; w0 += cap) {
#pragma unroll
      for (int u = 0; u < kFineRes; ++u)
        if (slot[u] >= w0 && slot[u] < w0 + cap) sv[slot[u] - w0] = r[u];
      __syncthreads();
      for (int p = tid; p < min(cap, cnt - w0); p += kFineThreads) sorted[s0 + w0 + p] = sv[p];
      __syncthreads();
    }
  }
  {
    int2* sv = reinterpret_cast<int2*>(stage);
    constexpr int cap = kFineStage / static_cast<int>(sizeof(int2));
    for (int w0 = 0; w0 < cnt; w0 += cap) {
#pragma unroll
      for (int u = 0; u < kFineRes; ++u)
        if (slot[u] >= w0 && slot[u] < w0 + cap) sv[slot[u] - w0] = int2{cl[u], ib[u].x};
      __syncthreads();
      for (int p = tid; p < min(cap, cnt - w0); p += kFineThreads) {
        const int2 v = sv[p];
        cells[s0 + w0 + p] = v.x;
        perm[s0 + w0 + p] = v.y;
      }
      __syncthreads();
    }
  }
}

// System of particle i (i < n) for kernels with one particle per thread: the systems of the
// workgroup's first and last particles are found once (the same for every thread), and only a
// workgroup that spans a boundary searches between them per particle.
__device__ __forceinline__ int block_sys(const int64_t* __restrict__ part_prefix, int nsys, int64_t n, int64_t i) {
  if (nsys == 1) return 0;
  const int64_t b0 = blockIdx.x * static_cast<int64_t>(blockDim.x);
  const int lo = find_sys(part_prefix, nsys, b0);
  const int hi = find_sys(part_prefix, nsys, min(b0 + static_cast<int64_t>(blockDim.x), n) - 1);
  return lo == hi ? lo : find_sys_in(part_prefix, lo, hi, i);
}

// One-level counting sort, for small systems (three short launches with no chain of dependent
// passes): a returning atomic per particle gives its rank within its bucket, one workgroup scans
// the bucket counts (k_scan), and the scatter writes each particle at its bucket's start plus
// its rank.
template <class T>
__global__ __launch_bounds__(kBinThreads) void k_bin_count1(int64_t n, int nsys, const SysDesc* __restrict__ sys,
                                                         const int64_t* __restrict__ part_prefix,
                                                         const T* __restrict__ pos, int sub_log2,
                                                         int* __restrict__ tile_count, int* __restrict__ key,
                                                         int* __restrict__ rank, double* __restrict__ energy) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kBinThreads) + threadIdx.x;
  if (energy && i < nsys) energy[i] = 0.0;
  if (i >= n) return;
  const SysDesc& sd = sys[block_sys(part_prefix, nsys, n, i)];
  int cell;
  T g[3];
  const int b = bin_bucket(sd, sub_log2, pos[3 * i + 0], pos[3 * i + 1], pos[3 * i + 2], cell, g);
  key[i] = b;
  rank[i] = atomicAdd(&tile_count[b], 1);
}

template <class T>
__global__ __launch_bounds__(kBinThreads) void k_bin_scatter1(
    int64_t n, int nsys, const SysDesc* __restrict__ sys, const int64_t* __restrict__ part_prefix,
    const T* __restrict__ pos, const T* __restrict__ q, const int* __restrict__ key, const int* __restrict__ rank,
    const int* __restrict__ tile_start, typename Vec4<T>::type* __restrict__ sorted, int* __restrict__ cells,
    int* __restrict__ perm) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kBinThreads) + threadIdx.x;
  if (i >= n) return;
  const SysDesc& sd = sys[block_sys(part_prefix, nsys, n, i)];
  const int dst = tile_start[key[i]] + rank[i];
  const T x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
  typename Vec4<T>::type rec;
  int cell;
  T g[3];
  bin_bucket(sd, 0, x, y, z, cell, g);
  rec.x = g[0];
  rec.y = g[1];
  rec.z = g[2];
  rec.w = q ? q[i] : T(0);
  // a non-finite position is moved to cell 0 by grid_coord; its NaN charge poisons the outputs
  // instead (spreading adds NaN into the grid, interpolation returns NaN for it)
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) rec.w = std::numeric_limits<T>::quiet_NaN();
  sorted[dst] = rec;
  cells[dst] = cell;
  perm[dst] = static_cast<int>(i);
}

// Exclusive scan of the counts (one workgroup of 1,024 threads, 16 consecutive counts per thread
// per pass, held in registers from one round of loads); resets the counts to zero.
constexpr int kScanK = 16;
__global__ __launch_bounds__(1024) void k_scan(int ntiles, int* __restrict__ count, int* __restrict__ start) {
  __shared__ int s_part[16];
  __shared__ int s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += 1024 * kScanK) {
    const int i0 = base + kScanK * tid;
    int v[kScanK];
    if (i0 + kScanK <= ntiles) {
      // the count and start buffers are 256-byte aligned and i0 is a multiple of 16
      const int4* c4 = reinterpret_cast<const int4*>(count + i0);
#pragma unroll
      for (int k = 0; k < kScanK / 4; ++k) {
        const int4 w = c4[k];
        v[4 * k] = w.x;
        v[4 * k + 1] = w.y;
        v[4 * k + 2] = w.z;
        v[4 * k + 3] = w.w;
      }
      int4* z4 = reinterpret_cast<int4*>(count + i0);
#pragma unroll
      for (int k = 0; k < kScanK / 4; ++k) z4[k] = int4{0, 0, 0, 0};
    } else {
#pragma unroll
      for (int k = 0; k < kScanK; ++k) {
        v[k] = i0 + k < ntiles ? count[i0 + k] : 0;
        if (i0 + k < ntiles) count[i0 + k] = 0;
      }
    }
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanK; ++k) sum += v[k];
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_part[wid] = x;
    __syncthreads();
    if (wid == 0) {
      int p = lane < 16 ? s_part[lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const int y = __shfl_up(p, o, 64);
        if (lane >= o) p += y;
      }
      if (lane < 16) s_part[lane] = p;
    }
    __syncthreads();
    int excl = x - sum + (wid > 0 ? s_part[wid - 1] : 0) + s_carry;
    int e[kScanK];
#pragma unroll
    for (int k = 0; k < kScanK; ++k) {
      e[k] = excl;
      excl += v[k];
    }
    if (i0 + kScanK <= ntiles) {
      int4* s4 = reinterpret_cast<int4*>(start + i0);
#pragma unroll
      for (int k = 0; k < kScanK / 4; ++k) s4[k] = int4{e[4 * k], e[4 * k + 1], e[4 * k + 2], e[4 * k + 3]};
    } else {
#pragma unroll
      for (int k = 0; k < kScanK; ++k)
        if (i0 + k < ntiles) start[i0 + k] = e[k];
    }
    __syncthreads();
    if (tid == 1023) s_carry = excl;
    __syncthreads();
  }
  if (tid == 0) start[ntiles] = s_carry;
}

// Input check (PSWFE_CHECK_INPUT): per system s, out[3 s] = sum q, out[3 s + 1] = sum |q| (float64)
// and out[3 s + 2] = the number of particles with a non-finite position or charge; out is
// zeroed by k_zero first. A wave whose particles all belong to one system adds its reduced sums
// with one atomic each; a wave spanning systems adds per particle.
__global__ void k_zero(double* __restrict__ out, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = 0.0;
}

// Zeroes `words` 32-bit words (a fill kernel rather than a memset node, so the call can sit in a
// captured graph).
__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t words) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

template <class T>
__global__ __launch_bounds__(256) void k_check_input(int64_t n, int nsys, const int64_t* __restrict__ part_prefix,
                                                     const T* __restrict__ pos, const T* __restrict__ q,
                                                     double* __restrict__ out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const bool valid = i < n;
  const int64_t ic = valid ? i : n - 1;
  const int s = nsys == 1 ? 0 : find_sys(part_prefix, nsys, ic);
  double v = 0.0, a = 0.0, bad = 0.0;
  if (valid) {
    const T qi = q[i];
    const bool finite = isfinite(pos[3 * i + 0]) && isfinite(pos[3 * i + 1]) && isfinite(pos[3 * i + 2]) && isfinite(qi);
    v = finite ? static_cast<double>(qi) : 0.0;
    a = finite ? fabs(static_cast<double>(qi)) : 0.0;
    bad = finite ? 0.0 : 1.0;
  }
  const int s0 = __shfl(s, 0, 64);
  if (__all(s == s0)) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v += __shfl_xor(v, off, 64);
      a += __shfl_xor(a, off, 64);
      bad += __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(out + 3 * s0, v);
      atomicAdd(out + 3 * s0 + 1, a);
      atomicAdd(out + 3 * s0 + 2, bad);
    }
  } else if (valid) {
    atomicAdd(out + 3 * s, v);
    atomicAdd(out + 3 * s + 1, a);
    atomicAdd(out + 3 * s + 2, bad);
  }
}

// ------------------------------------------------------------------------------------
// Real-space residual (Sec. 3.1.1, eq. R): phi_local,i = sum'_j q_j R(|x_i - x_j|) over the
// pairs closer than r_c (minimum image, r_c < L/2), with R(r) = 1/r - K G(r^2/r_c^2 - 1/2), and
// its gradient sum'_j q_j R'(r)/r (x_i - x_j). Particles are sorted by cells of edge L/nc >= r_c,
// so a particle's pairs lie in its 27 neighbour cells (every pair of the system when nc < 3).
// Positions are wrapped and differenced in float64, and all sums are float64.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double wrap_pos(double x, double L) {
  const double xr = x - L * floor(x / L);
  return (xr >= 0.0 && xr < L) ? xr : 0.0;  // rounding up to L, or a non-finite input
}

__device__ __forceinline__ int cell_of_pos(double xr, double scale, int nc) {
  const int c = static_cast<int>(xr * scale);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

template <class T>
__global__ void k_cell_count(int64_t n, int nsys, const SysDesc* __restrict__ sys,
                             const int64_t* __restrict__ part_prefix, const T* __restrict__ pos,
                             int* __restrict__ cell_count, int* __restrict__ cell_of, int* __restrict__ cell_rank,
                             double* __restrict__ energy) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (energy && i < nsys) energy[i] = 0.0;
  if (i >= n) return;
  const SysDesc& sd = sys[nsys == 1 ? 0 : find_sys(part_prefix, nsys, i)];
  const int cx = cell_of_pos(wrap_pos(static_cast<double>(pos[3 * i + 0]), sd.L), sd.nc / sd.L, sd.nc);
  const int cy = cell_of_pos(wrap_pos(static_cast<double>(pos[3 * i + 1]), sd.Ly), sd.ncy / sd.Ly, sd.ncy);
  const int cz = cell_of_pos(wrap_pos(static_cast<double>(pos[3 * i + 2]), sd.Lz), sd.ncz / sd.Lz, sd.ncz);
  const int cell = sd.cell_base + (cz * sd.ncy + cy) * sd.nc + cx;
  cell_of[i] = cell;
  cell_rank[i] = atomicAdd(&cell_count[cell], 1);
}

template <class T>
__global__ void k_cell_scatter(int64_t n, int nsys, const SysDesc* __restrict__ sys,
                               const int64_t* __restrict__ part_prefix, const T* __restrict__ pos,
                               const T* __restrict__ q, const int* __restrict__ cell_of,
                               const int* __restrict__ cell_rank, const int* __restrict__ cell_start,
                               double4* __restrict__ lsorted, int* __restrict__ lperm) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const SysDesc& sd = sys[nsys == 1 ? 0 : find_sys(part_prefix, nsys, i)];
  const int dst = cell_start[cell_of[i]] + cell_rank[i];
  const bool finite = isfinite(pos[3 * i + 0]) && isfinite(pos[3 * i + 1]) && isfinite(pos[3 * i + 2]);
  lsorted[dst] = make_double4(wrap_pos(static_cast<double>(pos[3 * i + 0]), sd.L),
                              wrap_pos(static_cast<double>(pos[3 * i + 1]), sd.Ly),
                              wrap_pos(static_cast<double>(pos[3 * i + 2]), sd.Lz),
                              finite ? static_cast<double>(q[i]) : std::numeric_limits<double>::quiet_NaN());
  lperm[dst] = static_cast<int>(i);
}

// One workgroup per cell: the particles of the 27 neighbour cells (of the whole system when
// nc < 3) are staged in LDS, kLocalChunk at a time, and each target particle of the cell is
// handled by L lanes that split the sources and reduce with shuffles, L = NT / (the cell's
// target count rounded up to a power of 2), between kLocalLanes and 64: the lanes a small cell
// would leave idle shorten its targets' source loops instead. The residual's polynomial
// coefficients are held in registers, and no division or memory access other than LDS reads
// sits in the pair loop.
// Workgroups of NT = 512 threads (128 and 256 on request): the kernel is latency-bound, and
// measured on MI355X more waves per cell pay (with 8 lanes per target: 112 / 84 / 80 us for
// NT = 128 / 256 / 512 on the water box, and 3.4 / 2.6 / 2.4 ms at n = 1e6).
constexpr int kLocalLanes = 8;
constexpr int kLocalChunk = 1024;
// DEG: the residual polynomial G, zero-padded to this degree (an instance per 12, 16, 20, 24)
template <class T, int DEG, int NT>
__global__ __launch_bounds__(NT) void k_local(int nsys, const SysDesc* __restrict__ sys,
                                                         const int* __restrict__ cell_prefix,
                                                         const double4* __restrict__ lsorted,
                                                         const int* __restrict__ lperm,
                                                         const int* __restrict__ cell_start, T* __restrict__ phi,
                                                         T* __restrict__ vec, int vec_mode, int accumulate,
                                                         double* __restrict__ energy, double* __restrict__ phi_d,
                                                         double* __restrict__ vec_d) {
  __shared__ double4 src[kLocalChunk];
  __shared__ int src_id[kLocalChunk];
  __shared__ int nb_begin[27], nb_off[28];
  __shared__ double s_red[NT / 64];
  const int gcell = blockIdx.x;
  const int t0 = cell_start[gcell], t1 = cell_start[gcell + 1];
  if (t0 == t1) return;
  const int s = find_sys(cell_prefix, nsys, gcell);
  const SysDesc& sd = sys[s];
  const int nc = sd.nc, ncy = sd.ncy, ncz = sd.ncz;
  const double Lx = sd.L, Ly = sd.Ly, Lz = sd.Lz, inv_Lx = 1.0 / Lx, inv_Ly = 1.0 / Ly, inv_Lz = 1.0 / Lz;
  const double rc2 = sd.rc * sd.rc, inv_rc2 = 1.0 / rc2, K = sd.lK;
  double cr[DEG + 1];
  const global_ptr<double> lcoef = as_global(sd.lcoef);
#pragma unroll
  for (int k = 0; k <= DEG; ++k) cr[k] = k <= sd.ldeg ? lcoef[k] : 0.0;
  const int tid = threadIdx.x;
  // source ranges: the 27 neighbour cells (distinct, as every nc >= 3), or the system's one cell
  if (tid < 27) {
    int b = 0, e = 0;
    if (nc >= 3) {
      const int lc = gcell - sd.cell_base;
      const int cx = lc % nc, cy = (lc / nc) % ncy, cz = lc / (nc * ncy);
      const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = tid / 9 - 1;
      const int x = (cx + dx + nc) % nc, y = (cy + dy + ncy) % ncy, z = (cz + dz + ncz) % ncz;
      const int cell = sd.cell_base + (z * ncy + y) * nc + x;
      b = cell_start[cell];
      e = cell_start[cell + 1];
    } else if (tid == 0) {
      b = t0;
      e = t1;
    }
    nb_begin[tid] = b;
    nb_off[tid + 1] = e - b;
  }
  __syncthreads();
  if (tid == 0) {
    nb_off[0] = 0;
    for (int k = 0; k < 27; ++k) nb_off[k + 1] += nb_off[k];
  }
  __syncthreads();
  const int ns = nb_off[27];
  int lanes = NT;  // lanes per target (a power of 2, 8..64), the same for the whole workgroup
  for (int pw = 1; pw < t1 - t0 && lanes > kLocalLanes; pw <<= 1) lanes >>= 1;
  lanes = min(lanes, 64);
  const int grp = tid / lanes, lane = tid % lanes;
  const int targets_per_pass = NT / lanes;
  double esum = 0.0;
  for (int tb = t0; tb < t1; tb += targets_per_pass) {
    const int ti = tb + grp;
    const bool tvalid = ti < t1;
    const double4 xi = lsorted[tvalid ? ti : t0];
    double ph = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int c0 = 0; c0 < ns; c0 += kLocalChunk) {
      const int nchunk = min(kLocalChunk, ns - c0);
      __syncthreads();
      for (int k = tid; k < nchunk; k += NT) {
        const int gk = c0 + k;
        int lo = 0, hi = 26;  // the neighbour cell holding source gk: largest cc with nb_off[cc] <= gk
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (nb_off[mid] <= gk)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int j = nb_begin[lo] + (gk - nb_off[lo]);
        src[k] = lsorted[j];
        src_id[k] = j;
      }
      __syncthreads();
      if (tvalid) {
        for (int k = lane; k < nchunk; k += lanes) {
          if (src_id[k] == ti) continue;
          const double4 xj = src[k];
          double dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
          dx -= Lx * rint(dx * inv_Lx);  // minimum image (pairs near L/2 lie beyond r_c)
          dy -= Ly * rint(dy * inv_Ly);
          dz -= Lz * rint(dz * inv_Lz);
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (!(r2 < rc2) || r2 == 0.0) continue;  // beyond the cutoff, or coincident positions
          const double rinv = rsqrt(r2);
          const double g = r2 * inv_rc2 - 0.5;
          double G = cr[DEG], dG = 0.0;
#pragma unroll
          for (int kk = DEG - 1; kk >= 0; --kk) {
            dG = fma(dG, g, G);
            G = fma(G, g, cr[kk]);
          }
          const double R = rinv - K * G;                                  // eq. R
          const double dRr = -rinv * rinv * rinv - 2.0 * K * inv_rc2 * dG;  // R'(r) / r
          ph = fma(xj.w, R, ph);
          const double f = xj.w * dRr;
          g0 = fma(f, dx, g0);
          g1 = fma(f, dy, g1);
          g2 = fma(f, dz, g2);
        }
      }
    }
    for (int off = lanes / 2; off > 0; off >>= 1) {  // within the aligned group of `lanes` lanes
      ph += __shfl_xor(ph, off);
      g0 += __shfl_xor(g0, off);
      g1 += __shfl_xor(g1, off);
      g2 += __shfl_xor(g2, off);
    }
    if (tvalid && lane == 0) {
      const int idx = lperm[ti];
      const double qi = xi.w;
      const double sc = vec_mode == 0 ? -qi : 1.0;
      const double v[3] = {sc * g0, sc * g1, sc * g2};
      if (phi_d) {  // float64 terms for the interpolation to add
        phi_d[idx] = ph;
        if (vec_d) {
#pragma unroll
          for (int d = 0; d < 3; ++d) vec_d[3 * idx + d] = v[d];
        }
      } else {
        if (phi) phi[idx] = static_cast<T>(accumulate ? static_cast<double>(phi[idx]) + ph : ph);
        if (vec) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
            vec[3 * idx + d] = static_cast<T>(accumulate ? static_cast<double>(vec[3 * idx + d]) + v[d] : v[d]);
        }
      }
      esum += 0.5 * qi * ph;
    }
  }
  if (energy) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) esum += __shfl_xor(esum, off, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = esum;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int w = 0; w < NT / 64; ++w) tot += s_red[w];
      safeAtomicAdd(energy + s, tot);  // caller's memory: the CAS form
    }
  }
}

// ------------------------------------------------------------------------------------
// FFT: Stockham autosort passes in LDS over a batch of sequences. Stage with radix R and
// current sub-length Ls: butterfly b (k = b mod Ls, j = b / Ls) reads x[b + t N/R],
// multiplies by w_{R Ls}^{t k}, takes an R-point DFT, and writes y_u to j R Ls + u Ls + k.
// The table `tw` holds exp(sign 2 pi i e / N), e = 0..N-1.
// ------------------------------------------------------------------------------------
template <class C, int R>
__device__ __forceinline__ void butterfly(const C* __restrict__ in, int NR, C* __restrict__ out, int Ls, int k,
                                          int twstep, const C* __restrict__ tw, int N) {
  C a[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    C x = in[t * NR];
    if (t > 0) x = cmul(x, tw[t * k * twstep]);
    a[t] = x;
  }
  if constexpr (R == 2) {
    out[0] = cadd(a[0], a[1]);
    out[Ls] = csub(a[0], a[1]);
  } else if constexpr (R == 4) {
    const C w = tw[N / 4];  // (0, +-1)
    const C s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const C s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    const C wd13 = cmul(w, d13);
    out[0] = cadd(s02, s13);
    out[Ls] = cadd(d02, wd13);
    out[2 * Ls] = csub(s02, s13);
    out[3 * Ls] = csub(d02, wd13);
  } else if constexpr (R == 8) {
    // y_u = sum_t a_t w^{t u}, w = tw[N/8]: split t into t and t + 4 (w^4 = -1), then two
    // 4-point DFTs with w^2 = tw[N/4] = +-i: even u from a_t + a_{t+4}, odd u from
    // (a_t - a_{t+4}) w^t.
    const C w8 = tw[N / 8], w4 = tw[N / 4];
    const C w83 = cmul(w8, w4);
    const C b0 = cadd(a[0], a[4]), b1 = cadd(a[1], a[5]), b2 = cadd(a[2], a[6]), b3 = cadd(a[3], a[7]);
    const C c0 = csub(a[0], a[4]), c1 = cmul(csub(a[1], a[5]), w8), c2 = cmul(csub(a[2], a[6]), w4),
            c3 = cmul(csub(a[3], a[7]), w83);
    {
      const C s02 = cadd(b0, b2), d02 = csub(b0, b2), s13 = cadd(b1, b3), d13 = cmul(csub(b1, b3), w4);
      out[0] = cadd(s02, s13);
      out[4 * Ls] = csub(s02, s13);
      out[2 * Ls] = cadd(d02, d13);
      out[6 * Ls] = csub(d02, d13);
    }
    {
      const C s02 = cadd(c0, c2), d02 = csub(c0, c2), s13 = cadd(c1, c3), d13 = cmul(csub(c1, c3), w4);
      out[Ls] = cadd(s02, s13);
      out[5 * Ls] = csub(s02, s13);
      out[3 * Ls] = cadd(d02, d13);
      out[7 * Ls] = csub(d02, d13);
    }
  } else {
    C wr[R];
#pragma unroll
    for (int v = 0; v < R; ++v) wr[v] = tw[v * (N / R)];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      C y = a[0];
#pragma unroll
      for (int t = 1; t < R; ++t) {
        const C p = cmul(a[t], wr[(t * u) % R]);
        y.x += p.x;
        y.y += p.y;
      }
      out[u * Ls] = y;
    }
  }
}

// Runs all stages; returns the buffer that holds the result (A or Bf).
template <class C>
__device__ __forceinline__ C* fft_lds(C* A, C* Bf, int nseq, int ss, const FftPlan& pl, const C* __restrict__ tw) {
  const int N = pl.N;
  int Ls = 1;
  C* src = A;
  C* dst = Bf;
  for (int st = 0; st < pl.nst; ++st) {
    const int R = pl.radix[st];
    const int NR = N / R;
    const int twstep = N / (R * Ls);
    for (int b = threadIdx.x; b < nseq * NR; b += blockDim.x) {
      const int s = b / NR, bb = b - s * NR;
      const int k = bb % Ls, j = bb / Ls;
      const C* in = src + s * ss + bb;
      C* out = dst + s * ss + j * R * Ls + k;
      switch (R) {
        case 2: butterfly<C, 2>(in, NR, out, Ls, k, twstep, tw, N); break;
        case 3: butterfly<C, 3>(in, NR, out, Ls, k, twstep, tw, N); break;
        case 4: butterfly<C, 4>(in, NR, out, Ls, k, twstep, tw, N); break;
        case 5: butterfly<C, 5>(in, NR, out, Ls, k, twstep, tw, N); break;
        case 7: butterfly<C, 7>(in, NR, out, Ls, k, twstep, tw, N); break;
        default: butterfly<C, 8>(in, NR, out, Ls, k, twstep, tw, N); break;
      }
    }
    __syncthreads();
    C* tmp = src;
    src = dst;
    dst = tmp;
    Ls *= R;
  }
  return src;
}

// Copies count items from global memory into LDS with up to K loads per thread in flight:
// v = load(i) for K indices, then store(i, v) for the same indices (the loads do not wait on
// the stores, which go to another address space).
template <int K, class Load, class Store>
__device__ __forceinline__ void staged_copy(int count, Load&& load, Store&& store) {
  using V = decltype(load(0));
  const int nt = blockDim.x;
  for (int base = threadIdx.x; base < count; base += nt * K) {
    V v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (base + k * nt < count) v[k] = load(base + k * nt);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (base + k * nt < count) store(base + k * nt, v[k]);
  }
}

// Twiddle tables copied into LDS: the loads (up to 4 per thread, count <= 4 * blockDim.x) are
// issued first and written to LDS only after the caller has issued its data loads, so that the
// two round trips to memory overlap instead of following each other.
template <class C, class Get>
__device__ __forceinline__ void table_load(int count, Get&& get, C (&v)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    if (e < count) v[k] = get(e);
  }
}
template <class C, class Put>
__device__ __forceinline__ void table_store(int count, Put&& put, const C (&v)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    if (e < count) put(e, v[k]);
  }
}

// x-direction real-to-complex FFT (sign +) of the m^2 rows of m reals of each system, via an
// m/2-point complex FFT of (a_2j + i a_2j+1); writes X_k, k = 0..m/2, to the system's spectrum.
// The input is the float64 grid_a (zeroed after it is read when zero_input is set) or, for a
// single system, in_override.
template <class T, class TI>
__global__ __launch_bounds__(256) void k_fft_x_r2c(int nsys, const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ xblk_prefix, const TI* in_override,
                                                   int zero_input) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(xblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int m = sd.m, N = m / 2, nrows = sd.my * sd.mz, rpb = sd.rows_per_block;
  const C* __restrict__ tw_half = static_cast<const C*>(sd.twhp);
  const C* __restrict__ tw_full = static_cast<const C*>(sd.twfp);
  C* A = reinterpret_cast<C*>(smem_raw);
  C* Bf = A + rpb * N;
  C* tw_h = Bf + rpb * N;          // N twiddles of the half-length FFT, then N + 1 of length m
  C* tw_f = tw_h + N;
  const int row0 = (static_cast<int>(blockIdx.x) - sd.xblk_base) * rpb;
  const int nr = min(rpb, nrows - row0);
  C twv[4];
  table_load(2 * N + 1, [&](int e) { return e < N ? gload(tw_half + e) : gload(tw_full + (e - N)); }, twv);
  using CI = typename Cplx<TI>::type;  // a pair (a_2j, a_2j+1) of the input row, one vector load
  const TI* grid = in_override ? in_override : reinterpret_cast<const TI*>(sd.grid_a);
  const CI* src = reinterpret_cast<const CI*>(grid + static_cast<int64_t>(row0) * m);
  staged_copy<8>(
      nr * N, [&](int e) { return gload(src + e); },
      [&](int e, CI v) { A[e] = C{static_cast<T>(v.x), static_cast<T>(v.y)}; });
  table_store(2 * N + 1, [&](int e, C v) { (e < N ? tw_h[e] : tw_f[e - N]) = v; }, twv);
  if (zero_input) {
    CI* zsrc = const_cast<CI*>(src);
    for (int e = threadIdx.x; e < nr * N; e += blockDim.x) gstore(zsrc + e, CI{TI(0), TI(0)});
  }
  __syncthreads();
  const C* Z = fft_lds(A, Bf, nr, N, sd.fh, tw_h);
  const int sp = sd.spec_pitch;
  C* out = static_cast<C*>(sd.spec) + static_cast<int64_t>(row0) * sp;
  for (int e = threadIdx.x; e < nr * (N + 1); e += blockDim.x) {
    const int r = e / (N + 1), k = e - r * (N + 1);
    const C zk = Z[r * N + (k == N ? 0 : k)];
    const C zn = cconj(Z[r * N + (k == 0 ? 0 : N - k)]);
    const C ev = C{T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y + zn.y)};
    const C dd = csub(zk, zn);
    const C od = C{T(0.5) * dd.y, T(-0.5) * dd.x};  // (zk - zn) / (2i)
    const C w = tw_f[k];
    gstore(out + r * sp + k, cadd(ev, cmul(w, od)));
  }
}

// x-direction complex-to-real inverse FFT (sign -): from X_k, k = 0..m/2 (Hermitian), forms
// Z_k = (X_k + conj X_{N-k}) + i w^{-k} (X_k - conj X_{N-k}), an m/2-point inverse FFT, and writes
// a_2j = Re z_j, a_2j+1 = Im z_j to the system's grid_b (or, single system, out_override).
template <class T>
__global__ __launch_bounds__(256) void k_fft_x_c2r(int nsys, const SysDesc* __restrict__ sys,
                                                   const int* __restrict__ xblk_prefix, T* out_override) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(xblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int m = sd.m, N = m / 2, nrows = sd.my * sd.mz, rpb = sd.rows_per_block;
  const C* __restrict__ tw_half = static_cast<const C*>(sd.twhm);
  const C* __restrict__ tw_full = static_cast<const C*>(sd.twfm);
  C* A = reinterpret_cast<C*>(smem_raw);   // rpb * (N + 1)
  C* Bf = A + rpb * (N + 1);               // rpb * N
  C* tw_h = Bf + rpb * N;                  // N twiddles of the half-length FFT, then N of length m
  C* tw_f = tw_h + N;
  const int row0 = (static_cast<int>(blockIdx.x) - sd.xblk_base) * rpb;
  const int nr = min(rpb, nrows - row0);
  C twv[4];
  table_load(2 * N, [&](int e) { return e < N ? gload(tw_half + e) : gload(tw_full + (e - N)); }, twv);
  const int sp = sd.spec_pitch;
  const C* in = static_cast<const C*>(sd.spec) + static_cast<int64_t>(row0) * sp;
  staged_copy<8>(
      nr * (N + 1),
      [&](int e) {
        const int r = e / (N + 1), k = e - r * (N + 1);
        return gload(in + r * sp + k);
      },
      [&](int e, C v) { A[e] = v; });
  table_store(2 * N, [&](int e, C v) { (e < N ? tw_h[e] : tw_f[e - N]) = v; }, twv);
  __syncthreads();
  for (int e = threadIdx.x; e < nr * N; e += blockDim.x) {
    const int r = e / N, k = e - r * N;
    const C xk = A[r * (N + 1) + k];
    const C xn = cconj(A[r * (N + 1) + N - k]);
    const C s = cadd(xk, xn);
    const C d = cmul(tw_f[k], csub(xk, xn));
    Bf[e] = C{s.x - d.y, s.y + d.x};  // s + i d
  }
  __syncthreads();
  const C* Z = fft_lds(Bf, A, nr, N, sd.fh, tw_h);
  T* grid = out_override ? out_override : static_cast<T*>(sd.grid_b);
  C* dst = reinterpret_cast<C*>(grid + static_cast<int64_t>(row0) * m);
  for (int e = threadIdx.x; e < nr * N; e += blockDim.x) gstore(dst + e, Z[e]);
}

// Forward x and y FFTs of one z-plane per workgroup (used when a plane fits in LDS): the m
// rows' real-to-complex FFTs as in k_fft_x_r2c, their half spectra written transposed into LDS
// (column kx of length m, padded stride m + 1), the y FFT of those m/2 + 1 columns, and the
// result stored to the spectrum in the layout k_fft_cols reads. One launch instead of two, and
// the plane does not travel through HBM in between.
template <class T, class TI>
__global__ __launch_bounds__(256) void k_fft_plane_fwd(int nsys, const SysDesc* __restrict__ sys,
                                                       const int* __restrict__ pblk_prefix, const TI* in_override,
                                                       int zero_input) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(pblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int m = sd.m, N = m / 2, nx1 = N + 1, ss = m + 1;
  const int z = static_cast<int>(blockIdx.x) - sd.pblk_base;
  C* U = reinterpret_cast<C*>(smem_raw);  // nx1 * ss each
  C* V = U + nx1 * ss;
  C* tw_h = V + nx1 * ss;  // N twiddles of the half-length FFT, then m of length m (sign +)
  C* tw_f = tw_h + N;
  {
    const C* __restrict__ tw_half = static_cast<const C*>(sd.twhp);
    const C* __restrict__ tw_full = static_cast<const C*>(sd.twfp);
    for (int e = threadIdx.x; e < N + m; e += blockDim.x) {
      if (e < N)
        tw_h[e] = gload(tw_half + e);
      else
        tw_f[e - N] = gload(tw_full + (e - N));
    }
  }
  using CI = typename Cplx<TI>::type;
  const TI* grid = in_override ? in_override : reinterpret_cast<const TI*>(sd.grid_a);
  const CI* src = reinterpret_cast<const CI*>(grid + static_cast<int64_t>(z) * m * m);
  staged_copy<8>(
      m * N, [&](int e) { return gload(src + e); },
      [&](int e, CI v) { U[e] = C{static_cast<T>(v.x), static_cast<T>(v.y)}; });
  if (zero_input) {
    CI* zsrc = const_cast<CI*>(src);
    for (int e = threadIdx.x; e < m * N; e += blockDim.x) gstore(zsrc + e, CI{TI(0), TI(0)});
  }
  __syncthreads();
  const C* Z = fft_lds(U, V, m, N, sd.fh, tw_h);  // rows y = 0..m-1, N points each
  C* Tc = (Z == U) ? V : U;
  for (int e = threadIdx.x; e < m * nx1; e += blockDim.x) {
    const int y = e / nx1, k = e - y * nx1;
    const C zk = Z[y * N + (k == N ? 0 : k)];
    const C zn = cconj(Z[y * N + (k == 0 ? 0 : N - k)]);
    const C ev = C{T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y + zn.y)};
    const C dd = csub(zk, zn);
    const C od = C{T(0.5) * dd.y, T(-0.5) * dd.x};
    Tc[k * ss + y] = cadd(ev, cmul(tw_f[k], od));
  }
  __syncthreads();
  C* other = (Tc == U) ? V : U;
  const C* R = fft_lds(Tc, other, nx1, ss, sd.ff, tw_f);
  const int sp = sd.spec_pitch;
  C* out = static_cast<C*>(sd.spec) + static_cast<int64_t>(z) * m * sp;
  for (int e = threadIdx.x; e < m * nx1; e += blockDim.x) {
    const int y = e / nx1, k = e - y * nx1;
    gstore(out + y * sp + k, R[k * ss + y]);
  }
}

// Inverse y and x FFTs of one z-plane per workgroup, the mirror of k_fft_plane_fwd: the plane's
// half spectrum loaded transposed, the inverse y FFT of its m/2 + 1 columns, then the
// complex-to-real inverse x FFT of its m rows as in k_fft_x_c2r, written to grid_b (or, single
// system, out_override).
template <class T>
__global__ __launch_bounds__(256) void k_fft_plane_inv(int nsys, const SysDesc* __restrict__ sys,
                                                       const int* __restrict__ pblk_prefix, T* out_override) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(pblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int m = sd.m, N = m / 2, nx1 = N + 1, ss = m + 1;
  const int z = static_cast<int>(blockIdx.x) - sd.pblk_base;
  C* U = reinterpret_cast<C*>(smem_raw);
  C* V = U + nx1 * ss;
  C* tw_h = V + nx1 * ss;  // N twiddles of the half-length FFT, then m of length m (sign -)
  C* tw_f = tw_h + N;
  {
    const C* __restrict__ tw_half = static_cast<const C*>(sd.twhm);
    const C* __restrict__ tw_full = static_cast<const C*>(sd.twfm);
    for (int e = threadIdx.x; e < N + m; e += blockDim.x) {
      if (e < N)
        tw_h[e] = gload(tw_half + e);
      else
        tw_f[e - N] = gload(tw_full + (e - N));
    }
  }
  const int sp = sd.spec_pitch;
  const C* in = static_cast<const C*>(sd.spec) + static_cast<int64_t>(z) * m * sp;
  staged_copy<8>(
      m * nx1,
      [&](int e) {
        const int y = e / nx1, k = e - y * nx1;
        return gload(in + y * sp + k);
      },
      [&](int e, C v) {
        const int y = e / nx1, k = e - y * nx1;
        U[k * ss + y] = v;
      });
  __syncthreads();
  const C* R = fft_lds(U, V, nx1, ss, sd.ff, tw_f);  // inverse y of each column kx
  C* W = (R == U) ? V : U;
  for (int e = threadIdx.x; e < m * N; e += blockDim.x) {
    const int y = e / N, k = e - y * N;
    const C xk = R[k * ss + y];
    const C xn = cconj(R[(N - k) * ss + y]);
    const C s = cadd(xk, xn);
    const C d = cmul(tw_f[k], csub(xk, xn));
    W[e] = C{s.x - d.y, s.y + d.x};  // s + i d
  }
  __syncthreads();
  C* other = (W == U) ? V : U;
  const C* Z = fft_lds(W, other, m, N, sd.fh, tw_h);
  T* grid = out_override ? out_override : static_cast<T*>(sd.grid_b);
  C* dst = reinterpret_cast<C*>(grid + static_cast<int64_t>(z) * m * m);
  for (int e = threadIdx.x; e < m * N; e += blockDim.x) gstore(dst + e, Z[e]);
}

// Radial factor of the scaling at |w|^2 = w2 for systems without a T_M table (cuboids):
// 4 pi prod_d h_d^2 / V * gammahat(|w|) / |w|^2 inside the band, 0 outside and at w = 0.
// PSWF split: gammahat = psi_0^{c_s}(r_c |w| / c_s) / psi_0^{c_s}(0), a polynomial in
// u = (r_c |w| / c_s)^2 - 1/2; Gaussian split: exp(-sigma^2 |w|^2 / 4).
__device__ __forceinline__ double radial_factor(const SysDesc& sd, double w2) {
  if (!(w2 > 0.0) || w2 > sd.rband2) return 0.0;
  double g;
  if (sd.radial == 2) {
    g = exp(-sd.rsig2 * w2);
  } else {
    const global_ptr<double> c = as_global(sd.rleg);
    const double u = sd.rscale * w2 - 0.5;
    g = c[sd.rleg_n];
    for (int k = sd.rleg_n - 1; k >= 0; --k) g = fma(g, u, c[k]);
  }
  return sd.rpref * g / w2;
}

// FFT along y or z of each system's half spectrum (mz planes of my rows of m/2 + 1 complex
// values). A system's blocks are (outer, column block) pairs; sequence c of a block is the
// column kx0 + c, whose element e sits at spec[outer * ostride + e * estride + kx0 + c].
//   mode 0: forward y (outer = z plane; length my);  mode 2: inverse y;
//   mode 1: forward z (outer = y row; length mz), multiply by
//           s_k = T_M(|k|) W[|kx|] Wy[|ky|] Wz[|kz|], inverse z (Alg. 2 steps 2-4 for this column).
template <class T>
__global__ __launch_bounds__(256) void k_fft_cols(int nsys, const SysDesc* __restrict__ sys,
                                                  const int* __restrict__ cblk_prefix, int mode) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(cblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int m = sd.m, my = sd.my, mz = sd.mz, nx1 = m / 2 + 1, cpb = sd.cols_per_block;
  const int len = mode == 1 ? mz : my;
  const int nxb = (nx1 + cpb - 1) / cpb;
  const int lb = static_cast<int>(blockIdx.x) - (mode == 1 ? sd.zblk_base : sd.cblk_base);
  const int outer = lb / nxb;
  const int kx0 = (lb - outer * nxb) * cpb;
  const int nc = min(cpb, nx1 - kx0);
  const int64_t plane = static_cast<int64_t>(my) * sd.spec_pitch;
  const int64_t ostride = mode == 1 ? int64_t(sd.spec_pitch) : plane;
  const int64_t estride = mode == 1 ? plane : int64_t(sd.spec_pitch);
  const int ss = len + 1;  // padded sequence stride in LDS
  const FftPlan& pl = mode == 1 ? sd.ffz : sd.ffy;
  C* A = reinterpret_cast<C*>(smem_raw);
  C* Bf = A + cpb * ss;
  C* tw_p = Bf + cpb * ss;  // twiddles of length len: sign + then sign -
  C* tw_m = tw_p + len;
  C twv[4];
  {
    const C* __restrict__ gp = static_cast<const C*>(mode == 1 ? sd.twzp : sd.twyp);
    const C* __restrict__ gm = static_cast<const C*>(mode == 1 ? sd.twzm : sd.twym);
    table_load(2 * len, [&](int e) { return e < len ? gload(gp + e) : gload(gm + (e - len)); }, twv);
  }
  const C* tw = mode == 2 ? tw_m : tw_p;
  C* base = static_cast<C*>(sd.spec) + outer * ostride + kx0;
  staged_copy<8>(
      nc * len,
      [&](int i) {
        const int e = i / nc, c = i - e * nc;
        return gload(base + e * estride + c);
      },
      [&](int i, C v) {
        const int e = i / nc, c = i - e * nc;
        A[c * ss + e] = v;
      });
  table_store(2 * len, [&](int e, C v) { (e < len ? tw_p[e] : tw_m[e - len]) = v; }, twv);
  __syncthreads();
  C* R1 = fft_lds(A, Bf, nc, ss, pl, tw);
  if (mode == 1) {
    const auto wk = as_global(static_cast<const T*>(sd.wk));
    const auto wky = as_global(static_cast<const T*>(sd.wky));
    const auto wkz = as_global(static_cast<const T*>(sd.wkz));
    const int ky = outer <= (my - 1) / 2 ? outer : my - outer;
    for (int i = threadIdx.x; i < nc * mz; i += blockDim.x) {
      const int c = i / mz, e = i - c * mz;
      const int kx = kx0 + c;
      const int kz = e <= (mz - 1) / 2 ? e : mz - e;
      T rad;
      if (sd.radial == 0) {
        rad = as_global(static_cast<const T*>(sd.tm))[kx * kx + ky * ky + kz * kz];
      } else {
        rad = static_cast<T>(radial_factor(sd, sd.w2x * kx * kx + sd.w2y * ky * ky + sd.w2z * kz * kz));
      }
      const T sc = rad * wk[kx] * wky[ky] * wkz[kz];
      C v = R1[c * ss + e];
      v.x *= sc;
      v.y *= sc;
      R1[c * ss + e] = v;
    }
    __syncthreads();
    C* other = (R1 == A) ? Bf : A;
    R1 = fft_lds(R1, other, nc, ss, pl, tw_m);
  }
  for (int i = threadIdx.x; i < nc * len; i += blockDim.x) {
    const int e = i / nc, c = i - e * nc;
    gstore(base + e * estride + c, R1[c * ss + e]);
  }
}

// The y and z passes of one column kx of a system's half spectrum in one workgroup: forward y,
// forward z, the scaling s_k, inverse z and inverse y (Alg. 2 steps 2-4 along y and z) with the
// column's (y, z) plane of my x mz complex values kept in LDS between them, for grids whose plane
// fits; one launch and one read and write of the spectrum instead of three. Block b of system s
// is column kx = b - yzblk_base.
template <class T>
__global__ __launch_bounds__(512) void k_fft_yz(int nsys, const SysDesc* __restrict__ sys,
                                                const int* __restrict__ yzblk_prefix) {
  using C = typename Cplx<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const SysDesc& sd = sys[find_sys(yzblk_prefix, nsys, static_cast<int>(blockIdx.x))];
  const int my = sd.my, mz = sd.mz;
  const int kx = static_cast<int>(blockIdx.x) - sd.yzblk_base;
  const int ssy = my + 1, ssz = mz + 1;  // padded sequence strides: y sequences, then z sequences
  const int cap = max(mz * ssy, my * ssz);
  C* A = reinterpret_cast<C*>(smem_raw);
  C* Bf = A + cap;
  C* twy_p = Bf + cap;  // twiddles of length my (sign +, then -), then of length mz
  C* twy_m = twy_p + my;
  C* twz_p = twy_m + my;
  C* twz_m = twz_p + mz;
  const int ntw = 2 * (my + mz);
  C twv[4];
  {
    const C* __restrict__ yp = static_cast<const C*>(sd.twyp);
    const C* __restrict__ ym = static_cast<const C*>(sd.twym);
    const C* __restrict__ zp = static_cast<const C*>(sd.twzp);
    const C* __restrict__ zm = static_cast<const C*>(sd.twzm);
    table_load(ntw, [&](int e) {
      if (e < my) return gload(yp + e);
      if (e < 2 * my) return gload(ym + (e - my));
      if (e < 2 * my + mz) return gload(zp + (e - 2 * my));
      return gload(zm + (e - 2 * my - mz));
    }, twv);
  }
  const int64_t sp = sd.spec_pitch, plane = static_cast<int64_t>(my) * sp;
  C* base = static_cast<C*>(sd.spec) + kx;
  // sequence z of the y pass: A[z * ssy + y]
  staged_copy<8>(
      my * mz,
      [&](int i) {
        const int z = i / my, y = i - z * my;
        return gload(base + z * plane + y * sp);
      },
      [&](int i, C v) {
        const int z = i / my, y = i - z * my;
        A[z * ssy + y] = v;
      });
  table_store(ntw, [&](int e, C v) { twy_p[e] = v; }, twv);
  __syncthreads();
  C* R = fft_lds(A, Bf, mz, ssy, sd.ffy, twy_p);  // forward y
  C* W = (R == A) ? Bf : A;
  for (int i = threadIdx.x; i < my * mz; i += blockDim.x) {  // sequence y of the z pass: W[y * ssz + z]
    const int y = i / mz, z = i - y * mz;
    W[y * ssz + z] = R[z * ssy + y];
  }
  __syncthreads();
  R = fft_lds(W, R, my, ssz, sd.ffz, twz_p);  // forward z
  {
    const auto wk = as_global(static_cast<const T*>(sd.wk));
    const auto wky = as_global(static_cast<const T*>(sd.wky));
    const auto wkz = as_global(static_cast<const T*>(sd.wkz));
    const T wx = wk[kx];
    // K factors per thread computed (their table loads in flight together) before they are applied
    constexpr int K = 8;
    const int nt = static_cast<int>(blockDim.x), count = my * mz;
    for (int i0 = threadIdx.x; i0 < count; i0 += K * nt) {
      T sc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = i0 + k * nt;
        if (i >= count) break;
        const int y = i / mz, z = i - y * mz;
        const int ky = y <= (my - 1) / 2 ? y : my - y;
        const int kz = z <= (mz - 1) / 2 ? z : mz - z;
        T rad;
        if (sd.radial == 0) {
          rad = as_global(static_cast<const T*>(sd.tm))[kx * kx + ky * ky + kz * kz];
        } else {
          rad = static_cast<T>(radial_factor(sd, sd.w2x * kx * kx + sd.w2y * ky * ky + sd.w2z * kz * kz));
        }
        sc[k] = rad * wx * wky[ky] * wkz[kz];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = i0 + k * nt;
        if (i >= count) break;
        const int y = i / mz, z = i - y * mz;
        C v = R[y * ssz + z];
        v.x *= sc[k];
        v.y *= sc[k];
        R[y * ssz + z] = v;
      }
    }
  }
  __syncthreads();
  C* other = (R == A) ? Bf : A;
  R = fft_lds(R, other, my, ssz, sd.ffz, twz_m);  // inverse z
  W = (R == A) ? Bf : A;
  for (int i = threadIdx.x; i < my * mz; i += blockDim.x) {  // back to sequences along y
    const int z = i / my, y = i - z * my;
    W[z * ssy + y] = R[y * ssz + z];
  }
  __syncthreads();
  R = fft_lds(W, R, mz, ssy, sd.ffy, twy_m);  // inverse y
  for (int i = threadIdx.x; i < my * mz; i += blockDim.x) {
    const int z = i / my, y = i - z * my;
    gstore(base + z * plane + y * sp, R[z * ssy + y]);
  }
}

// Copies the accumulation grid (float64, or float32 where the plan accumulates in float32) into
// a grid of the plan's precision and zeroes it.
template <class TA, class T>
__global__ void k_drain(TA* __restrict__ acc, T* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    out[i] = static_cast<T>(acc[i]);
    acc[i] = TA(0);
  }
}

// ------------------------------------------------------------------------------------
// Launch helpers
// ------------------------------------------------------------------------------------
inline unsigned blocks_for(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

template <class T>
hipError_t bin_impl(const DevPlan& d, int64_t n, const void* pos, const void* q, double* energy, hipStream_t st) {
  stage_begin(d, kStageBin, st);
  if (d.bin_levels == 1) {
    const int64_t nthreads = std::max<int64_t>(n, energy ? d.nsys : 0);
    if (nthreads > 0)
      hipLaunchKernelGGL(k_bin_count1<T>, dim3(blocks_for(nthreads, kBinThreads)), dim3(kBinThreads), 0, st, n,
                         d.nsys, d.sys_dev, d.part_prefix, static_cast<const T*>(pos), d.sub_log2, d.tile_count,
                         d.tile_of, d.bin_rank, energy);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d.total_tiles << d.sub_log2, d.tile_count, d.tile_start);
    if (n > 0)
      hipLaunchKernelGGL(k_bin_scatter1<T>, dim3(blocks_for(n, kBinThreads)), dim3(kBinThreads), 0, st, n, d.nsys,
                         d.sys_dev, d.part_prefix, static_cast<const T*>(pos), static_cast<const T*>(q), d.tile_of,
                         d.bin_rank, d.tile_start, static_cast<typename Vec4<T>::type*>(d.sorted), d.cells, d.perm);
    stage_end(d, kStageBin, st);
    return hipGetLastError();
  }
  // counting: per_thread particles per thread, and at least one thread per system for the energy
  // reset; then the coarse pass and one workgroup per coarse bucket
  const int64_t chunk = static_cast<int64_t>(kBinThreads) * d.bin_per_thread;
  const int64_t blocks = std::max<int64_t>(blocks_for(n, static_cast<int>(chunk)), energy ? blocks_for(d.nsys, kBinThreads) : 0);
  if (blocks > 0)
    hipLaunchKernelGGL(k_bin_count<T>, dim3(static_cast<unsigned>(blocks)), dim3(kBinThreads), 0, st, n, d.nsys,
                       d.sys_dev, d.part_prefix, static_cast<const T*>(pos), d.sub_log2, d.bin_per_thread, d.bin_shift,
                       d.bin_ncoarse, d.coarse_count, d.tile_of, energy);
  if (n > 0)
    hipLaunchKernelGGL(k_bin_coarse<T>, dim3(blocks_for(n, static_cast<int>(chunk))), dim3(kBinThreads),
                       coarse_lds_bytes<T>(), st, n,
                       static_cast<const T*>(pos), static_cast<const T*>(q), d.bin_per_thread, d.bin_shift,
                       d.bin_ncoarse, d.coarse_count, d.coarse_cursor, d.coarse_start, d.tile_of,
                       static_cast<typename Vec4<T>::type*>(d.bin_tmp), d.bin_tmp_ib);
  else
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(d.coarse_start),
                       static_cast<int64_t>(kCoarse + 1));
  // counters, then the staging area (when it fits beside them)
  const size_t counters = sizeof(int) * (((size_t(1) << d.bin_shift) + kFineThreads / 64 + 3) & ~size_t(3));
  const bool staged = counters + kFineStage <= kFineLdsMax;
  hipLaunchKernelGGL(k_bin_fine<T>, dim3(d.bin_ncoarse), dim3(kFineThreads), counters + (staged ? kFineStage : 0), st,
                     n, d.nsys, d.sys_dev, d.tile_prefix, d.tile_sys, d.sub_log2, d.bin_shift, d.bin_ncoarse,
                     d.total_tiles << d.sub_log2,
                     d.coarse_start, d.coarse_count, d.coarse_cursor,
                     static_cast<const typename Vec4<T>::type*>(d.bin_tmp), d.bin_tmp_ib, d.tile_start,
                     static_cast<typename Vec4<T>::type*>(d.sorted), d.cells, d.perm, staged ? 1 : 0);
  stage_end(d, kStageBin, st);
  return hipGetLastError();
}

template <class T>
hipError_t transform_impl(const DevPlan& d, const void* in_override, void* out_override, hipStream_t st) {
  if (d.plane_fft) {
    stage_begin(d, kStageFftX, st);
    if (in_override)
      hipLaunchKernelGGL((k_fft_plane_fwd<T, T>), dim3(d.total_pblk), dim3(256), d.lds_p, st, d.nsys, d.sys_dev,
                         d.pblk_prefix, static_cast<const T*>(in_override), 0);
    else
      hipLaunchKernelGGL((k_fft_plane_fwd<T, double>), dim3(d.total_pblk), dim3(256), d.lds_p, st, d.nsys,
                         d.sys_dev, d.pblk_prefix, static_cast<const double*>(nullptr), 1);
    stage_end(d, kStageFftX, st);
    stage_begin(d, kStageFftY, st);  // fused into the x stage: recorded as an empty stage
    stage_end(d, kStageFftY, st);
    stage_begin(d, kStageFftZScale, st);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(d.total_zblk), dim3(256), d.lds_c, st, d.nsys, d.sys_dev, d.zblk_prefix,
                       1);
    stage_end(d, kStageFftZScale, st);
    stage_begin(d, kStageIfftY, st);  // fused into the inverse x stage
    stage_end(d, kStageIfftY, st);
    stage_begin(d, kStageIfftX, st);
    hipLaunchKernelGGL(k_fft_plane_inv<T>, dim3(d.total_pblk), dim3(256), d.lds_p, st, d.nsys, d.sys_dev,
                       d.pblk_prefix, static_cast<T*>(out_override));
    stage_end(d, kStageIfftX, st);
    return hipGetLastError();
  }
  stage_begin(d, kStageFftX, st);
  if (in_override)
    hipLaunchKernelGGL((k_fft_x_r2c<T, T>), dim3(d.total_xblk), dim3(256), d.lds_x, st, d.nsys, d.sys_dev,
                       d.xblk_prefix, static_cast<const T*>(in_override), 0);
  else if (std::is_same_v<T, float> && d.grid32)
    hipLaunchKernelGGL((k_fft_x_r2c<T, float>), dim3(d.total_xblk), dim3(256), d.lds_x, st, d.nsys, d.sys_dev,
                       d.xblk_prefix, static_cast<const float*>(nullptr), 1);
  else
    hipLaunchKernelGGL((k_fft_x_r2c<T, double>), dim3(d.total_xblk), dim3(256), d.lds_x, st, d.nsys, d.sys_dev,
                       d.xblk_prefix, static_cast<const double*>(nullptr), 1);
  stage_end(d, kStageFftX, st);
  if (d.yz_fft) {
    stage_begin(d, kStageFftY, st);  // fused into the z stage: recorded as an empty stage
    stage_end(d, kStageFftY, st);
    stage_begin(d, kStageFftZScale, st);
    hipLaunchKernelGGL(k_fft_yz<T>, dim3(d.total_yzblk), dim3(512), d.lds_yz, st, d.nsys, d.sys_dev,
                       d.yzblk_prefix);
    stage_end(d, kStageFftZScale, st);
    stage_begin(d, kStageIfftY, st);  // fused into the z stage
    stage_end(d, kStageIfftY, st);
  } else {
    stage_begin(d, kStageFftY, st);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(d.total_cblk), dim3(256), d.lds_c, st, d.nsys, d.sys_dev, d.cblk_prefix,
                       0);
    stage_end(d, kStageFftY, st);
    stage_begin(d, kStageFftZScale, st);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(d.total_zblk), dim3(256), d.lds_c, st, d.nsys, d.sys_dev, d.zblk_prefix,
                       1);
    stage_end(d, kStageFftZScale, st);
    stage_begin(d, kStageIfftY, st);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(d.total_cblk), dim3(256), d.lds_c, st, d.nsys, d.sys_dev, d.cblk_prefix,
                       2);
    stage_end(d, kStageIfftY, st);
  }
  stage_begin(d, kStageIfftX, st);
  hipLaunchKernelGGL(k_fft_x_c2r<T>, dim3(d.total_xblk), dim3(256), d.lds_x, st, d.nsys, d.sys_dev, d.xblk_prefix,
                     static_cast<T*>(out_override));
  stage_end(d, kStageIfftX, st);
  return hipGetLastError();
}

// Particle-kernel instance covering (precision, P).
struct ParticleFns {
  int prec, lo, hi;
  hipError_t (*prepare)(PGroup&);
  hipError_t (*spread)(const DevPlan&, const PGroup&, hipStream_t);
  hipError_t (*gather)(const DevPlan&, const PGroup&, const void*, void*, void*, int, bool, double*, const double*,
                       const double*, hipStream_t);
};

#define PSWFE_PARTICLE_ENTRY(prec, lo, hi) \
  {prec, lo, hi, particles_prepare_##prec##_##lo, particles_spread_##prec##_##lo, particles_gather_##prec##_##lo},
constexpr ParticleFns kParticleFns[] = {PSWFE_PARTICLE_INSTANCES(PSWFE_PARTICLE_ENTRY)};
#undef PSWFE_PARTICLE_ENTRY

const ParticleFns* particle_fns(int prec, int P) {
  for (const ParticleFns& f : kParticleFns)
    if (f.prec == prec && f.lo <= P && P <= f.hi) return &f;
  return nullptr;
}

}  // namespace

template <class T>
hipError_t raise_fft_lds(const DevPlan& d) {
  auto set = [](const void* f, size_t bytes) {
    return bytes > 64 * 1024
               ? hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes))
               : hipSuccess;
  };
  hipError_t e = set(reinterpret_cast<const void*>(&k_fft_x_r2c<T, T>), d.lds_x);
  if (e == hipSuccess) e = set(reinterpret_cast<const void*>(&k_fft_x_r2c<T, double>), d.lds_x);
  if (e == hipSuccess) e = set(reinterpret_cast<const void*>(&k_fft_x_c2r<T>), d.lds_x);
  if (e == hipSuccess) e = set(reinterpret_cast<const void*>(&k_fft_cols<T>), d.lds_c);
  if (e == hipSuccess && d.yz_fft) e = set(reinterpret_cast<const void*>(&k_fft_yz<T>), d.lds_yz);
  // the binning fine pass stages its records in up to kFineLdsMax bytes
  if (e == hipSuccess && d.bin_levels == 2) e = set(reinterpret_cast<const void*>(&k_bin_fine<T>), kFineLdsMax);
  if (e == hipSuccess && d.bin_levels == 2) e = set(reinterpret_cast<const void*>(&k_bin_coarse<T>), coarse_lds_bytes<T>());
  return e;
}

hipError_t prepare_kernels(DevPlan& d) {
  {
    const hipError_t e = d.prec == 0 ? raise_fft_lds<float>(d) : raise_fft_lds<double>(d);
    if (e != hipSuccess) return e;
  }
  if (d.plane_fft && d.lds_p > 64 * 1024) {
    hipError_t e;
    if (d.prec == 0)
      e = [&] {
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_fwd<float, float>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(d.lds_p));
        if (r == hipSuccess)
          r = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_fwd<float, double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(d.lds_p));
        if (r == hipSuccess)
          r = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_inv<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(d.lds_p));
        return r;
      }();
    else
      e = [&] {
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_fwd<double, double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(d.lds_p));
        if (r == hipSuccess)
          r = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_inv<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(d.lds_p));
        return r;
      }();
    if (e != hipSuccess) return e;
  }
  for (PGroup& g : d.groups) {
    const ParticleFns* f = particle_fns(d.prec, g.P);
    const hipError_t e = f ? f->prepare(g) : hipErrorInvalidValue;
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>(bytes / 4);
  if (words > 0)
    hipLaunchKernelGGL(k_zero_words, dim3(std::max(1u, std::min(blocks_for(words, 256), 2048u))), dim3(256), 0, st,
                       static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

hipError_t launch_check(const DevPlan& d, int64_t n_total, const void* pos, const void* q, double* out,
                        hipStream_t st) {
  const int count = 3 * d.nsys;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(count, 256)), dim3(256), 0, st, out, count);
  if (n_total > 0) {
    if (d.prec == 0)
      hipLaunchKernelGGL(k_check_input<float>, dim3(blocks_for(n_total, 256)), dim3(256), 0, st, n_total, d.nsys,
                         d.part_prefix, static_cast<const float*>(pos), static_cast<const float*>(q), out);
    else
      hipLaunchKernelGGL(k_check_input<double>, dim3(blocks_for(n_total, 256)), dim3(256), 0, st, n_total, d.nsys,
                         d.part_prefix, static_cast<const double*>(pos), static_cast<const double*>(q), out);
  }
  return hipGetLastError();
}

hipError_t launch_bin(const DevPlan& d, int64_t n_total, const void* pos, const void* q, double* energy,
                      hipStream_t st) {
  return d.prec == 0 ? bin_impl<float>(d, n_total, pos, q, energy, st)
                     : bin_impl<double>(d, n_total, pos, q, energy, st);
}

hipError_t launch_spread(const DevPlan& d, hipStream_t st) {
  hipError_t e = hipSuccess;
  stage_begin(d, kStageSpread, st);
  for (const PGroup& g : d.groups) {
    const ParticleFns* f = particle_fns(d.prec, g.P);
    e = f ? f->spread(d, g, st) : hipErrorInvalidValue;
    if (e != hipSuccess) break;
  }
  stage_end(d, kStageSpread, st);
  return e;
}

hipError_t launch_drain(const DevPlan& d, void* out, hipStream_t st) {
  const SysDesc& s0 = d.sys[0];
  const int64_t count = static_cast<int64_t>(s0.m) * s0.my * s0.mz;
  const unsigned nb = std::max(1u, std::min<unsigned>(blocks_for(count, 256), 4096u));
  if (d.prec == 0 && d.grid32)
    hipLaunchKernelGGL((k_drain<float, float>), dim3(nb), dim3(256), 0, st, reinterpret_cast<float*>(s0.grid_a),
                       static_cast<float*>(out), count);
  else if (d.prec == 0)
    hipLaunchKernelGGL((k_drain<double, float>), dim3(nb), dim3(256), 0, st, s0.grid_a, static_cast<float*>(out),
                       count);
  else
    hipLaunchKernelGGL((k_drain<double, double>), dim3(nb), dim3(256), 0, st, s0.grid_a, static_cast<double*>(out),
                       count);
  return hipGetLastError();
}

template <class T>
hipError_t local_impl(const DevPlan& d, int64_t n, const void* pos, const void* q, void* phi, void* vec, int vec_mode,
                      double* energy, bool accumulate, hipStream_t st, double* phi_d, double* vec_d) {
  stage_begin(d, kStageLocal, st);
  const int64_t nthreads = std::max<int64_t>(n, (energy && !accumulate) ? d.nsys : 0);
  if (nthreads > 0)
    hipLaunchKernelGGL(k_cell_count<T>, dim3(blocks_for(nthreads, 256)), dim3(256), 0, st, n, d.nsys, d.sys_dev,
                       d.part_prefix, static_cast<const T*>(pos), d.cell_count, d.cell_of, d.cell_rank,
                       accumulate ? nullptr : energy);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d.total_cells, d.cell_count, d.cell_start);
  if (n > 0) {
    hipLaunchKernelGGL(k_cell_scatter<T>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, d.nsys, d.sys_dev,
                       d.part_prefix, static_cast<const T*>(pos), static_cast<const T*>(q), d.cell_of, d.cell_rank,
                       d.cell_start, reinterpret_cast<double4*>(d.lsorted), d.lperm);
    const auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(d.total_cells), dim3(d.local_threads), 0, st, d.nsys, d.sys_dev, d.cell_prefix,
                         reinterpret_cast<const double4*>(d.lsorted), d.lperm, d.cell_start, static_cast<T*>(phi),
                         static_cast<T*>(vec), vec_mode, accumulate ? 1 : 0, energy, phi_d, vec_d);
    };
    const auto by_threads = [&]<int DEG>() {
      if (d.local_threads == 128)
        launch(k_local<T, DEG, 128>);
      else if (d.local_threads == 256)
        launch(k_local<T, DEG, 256>);
      else
        launch(k_local<T, DEG, 512>);
    };
    if (d.local_deg <= 12)
      by_threads.template operator()<12>();
    else if (d.local_deg <= 16)
      by_threads.template operator()<16>();
    else if (d.local_deg <= 20)
      by_threads.template operator()<20>();
    else
      by_threads.template operator()<24>();
  }
  stage_end(d, kStageLocal, st);
  return hipGetLastError();
}

hipError_t launch_local(const DevPlan& d, int64_t n_total, const void* pos, const void* q, void* phi, void* vec,
                        int vec_mode, double* energy, bool accumulate, hipStream_t st, double* phi_d, double* vec_d) {
  return d.prec == 0 ? local_impl<float>(d, n_total, pos, q, phi, vec, vec_mode, energy, accumulate, st, phi_d, vec_d)
                     : local_impl<double>(d, n_total, pos, q, phi, vec, vec_mode, energy, accumulate, st, phi_d, vec_d);
}

hipError_t launch_transform(const DevPlan& d, const void* in_override, void* out_override, hipStream_t st) {
  return d.prec == 0 ? transform_impl<float>(d, in_override, out_override, st)
                     : transform_impl<double>(d, in_override, out_override, st);
}

hipError_t launch_gather(const DevPlan& d, const void* grid_override, void* phi, void* vec, int vec_mode,
                         bool add_self, double* energy, hipStream_t st, const double* phi_add, const double* vec_add) {
  hipError_t e = hipSuccess;
  stage_begin(d, kStageGather, st);
  for (const PGroup& g : d.groups) {
    const ParticleFns* f = particle_fns(d.prec, g.P);
    e = f ? f->gather(d, g, grid_override, phi, vec, vec_mode, add_self, energy, phi_add, vec_add, st)
          : hipErrorInvalidValue;
    if (e != hipSuccess) break;
  }
  stage_end(d, kStageGather, st);
  return e;
}

}  // namespace pswfe
