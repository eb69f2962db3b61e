// Device kernels of the PSWF fast Ewald pipeline (Alg. 2) and their launch helpers.
//
// Every launch covers a batch of independent systems (a single-system plan is a batch of one):
// each system has a descriptor (grid size, tile geometry, tables, buffers) and owns a
// contiguous range of the global tile, block and packed-particle index spaces; a workgroup
// finds its system by binary search in a small prefix table.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

namespace pswfe {

constexpr int kMaxStages = 16;
constexpr int kPmin = 3;
constexpr int kPmax = 24;

// Radix plan of one 1-D FFT length.
struct FftPlan {
  int N = 0;
  int nst = 0;
  int radix[kMaxStages] = {};
};

// Pipeline stages, for event-based timing of one stage at a time.
enum Stage {
  kStageBin = 0, kStageSpread = 1, kStageFftX = 2, kStageFftY = 3, kStageFftZScale = 4, kStageIfftY = 5,
  kStageIfftX = 6, kStageGather = 7, kStageAll = 8, kStageLocal = 9, kNumStages = 10
};

// HIP events recorded around one stage of successive calls (owned by the plan).
struct StageTimer {
  int stage = -1;
  int cap = 0;
  int count = 0;
  hipEvent_t* ev = nullptr;  // 2 * cap events: start, stop per call
};

// One system of a batch. Pointers are device pointers; real arrays are in the plan precision
// unless stated.
// Boxes are cuboids [0, L) x [0, Ly) x [0, Lz) with m x my x mz grid points (a cube has equal
// sizes; the cuboid remark of Sec. 6.1); x fields keep the unsuffixed names.
struct SysDesc {
  int m = 0, P = 0, deg = 0;  // m: grid points along x
  int my = 0, mz = 0;         // grid points along y and z
  int B = 0;                  // tile edge in grid cells
  int Tn = 0;                 // tiles along x
  int Tny = 0, Tnz = 0;       // tiles along y and z
  int S = 0;                  // LDS tile edge = (B + P - 1) rounded up to odd
  int tile_base = 0;          // first global tile of this system
  int rows_per_block = 1;     // x-direction FFT batching
  int cols_per_block = 1;     // y/z-direction FFT batching (a multiple of spec_align where nx1 allows)
  int spec_pitch = 0;         // complex values per spectrum row: nx1 = m/2 + 1 rounded up to 128 bytes
  int xblk_base = 0;          // first block of this system in the x-direction FFT launches
  int pblk_base = 0;          // first block (z-plane) of this system in the plane FFT launches
  int cblk_base = 0;          // first block in the y-direction FFT launches
  int zblk_base = 0;          // first block in the z-direction FFT launch
  int yzblk_base = 0;         // first block (spectrum column kx) in the fused y/z FFT launch
  int64_t part_base = 0;      // first packed particle of this system
  double L = 0, inv_h = 0, ih_hi = 0, ih_lo = 0, self_coef = 0;  // x: box side, 1/h (split in two)
  double Ly = 0, inv_hy = 0, ihy_hi = 0, ihy_lo = 0;
  double Lz = 0, inv_hz = 0, ihz_hi = 0, ihz_lo = 0;
  double* grid_a = nullptr;   // mz * my * m float64 spread target; kept all-zero between calls
  void* grid_b = nullptr;     // mz * my * m transformed grid
  void* spec = nullptr;       // mz * my * (m/2 + 1) complex half spectrum
  const double* coef = nullptr;  // P * (deg + 1) window polynomial coefficients (float64)
  // radial scaling: radial == 0, a table T_M[|k|^2] over 3 (m/2)^2 + 1 entries (cubes); else the
  // factor is evaluated per mode from |w|^2 = w2x kx^2 + w2y ky^2 + w2z kz^2 (radial == 1: PSWF
  // split, Legendre series of psi_0^{c_s}; radial == 2: Gaussian split)
  const void* tm = nullptr;
  int radial = 0, rleg_n = 0;
  const double* rleg = nullptr;  // Legendre coefficients of P_0, P_2, ... of psi_0^{c_s}
  double w2x = 0, w2y = 0, w2z = 0, rscale = 0, rpref = 0, rband2 = 0, rsig2 = 0;
  const void* wk = nullptr;   // m/2 + 1 window factors (x), then my/2 + 1 (y), mz/2 + 1 (z)
  const void* wky = nullptr;
  const void* wkz = nullptr;
  const void* twhp = nullptr; // exp(+2 pi i e / (m/2)), e < m/2
  const void* twhm = nullptr; // exp(-2 pi i e / (m/2))
  const void* twfp = nullptr; // exp(+2 pi i e / m), e < m
  const void* twfm = nullptr; // exp(-2 pi i e / m)
  const void* twyp = nullptr; // the same for lengths my and mz
  const void* twym = nullptr;
  const void* twzp = nullptr;
  const void* twzm = nullptr;
  FftPlan fh, ff;             // radix plans for lengths m/2 and m
  FftPlan ffy, ffz;           // lengths my and mz
  // real-space residual (Sec. 3.1.1): cells of edge L / nc >= r_c (nc >= 3), or one cell
  // holding the whole system when nc < 3
  int nc = 1;                 // cells along x
  int ncy = 1, ncz = 1;       // along y and z
  int cell_base = 0;          // first global cell of this system
  int ldeg = 0;               // degree of the residual polynomial G
  double rc = 0, lK = 0;      // cutoff and K of R(r) = 1/r - K G(r^2/r_c^2 - 1/2)
  const double* lcoef = nullptr;  // ldeg + 1 coefficients of G (float64)
};

// Horner degree buckets of the particle kernels: a window polynomial of degree deg is
// evaluated as one of degree D = degree_bucket(deg) >= deg whose extra leading coefficients are
// zero (exact: the first Horner steps then produce zeros). Coefficient rows are staged in LDS
// with an odd stride in doubles, so the 16 lanes of a particle read 16 rows without conflicts.
inline int degree_bucket(int deg) { return deg <= 11 ? 11 : (deg <= 17 ? 17 : 28); }
constexpr int coef_stride(int D) { return (D + 1) % 2 ? D + 1 : D + 2; }
constexpr int kMaxDeg = 28;
// Bytes of the interpolation's S^3 grid block at the start of its LDS, rounded up to 16 so that
// the float64 arrays after it stay aligned.
__host__ __device__ constexpr size_t gather_block_bytes(int S, size_t elem) {
  return (elem * static_cast<size_t>(S) * S * S + 15) & ~static_cast<size_t>(15);
}

// Systems sharing one window support P and degree bucket D: their tiles form the contiguous
// global range [tile_begin, tile_end), covered by one launch of each particle kernel
// (templated on P and D).
struct PGroup {
  int P = 0, D = 0;
  int tile_begin = 0, tile_end = 0;
  int spread_threads = 256, gather_threads = 256;  // workgroup sizes (multiples of 64, <= 1024)
  int col_tile = 0;  // spreading in registers when the group's tiles all have this edge (4, 6, 8)
  int mfma = 0;      // ... as a matrix product on the matrix cores (k_spread_mfma) rather than by y-columns
  int acc32 = 0;     // ... with float32 window values, products and tile sums (float32 plans only)
  int parts = 1;     // workgroups per tile, each taking an equal slice of the tile's particles
  int xcd_spread = 0, xcd_gather = 0;  // XCD-aware tile order (set at plan creation)
  // matrix-core spreading by columns of tiles with a ring of z-planes in LDS (single systems):
  // roll_len tiles per workgroup, roll_nseg segments per column, roll_cols columns (0: off)
  int roll_len = 0, roll_nseg = 0, roll_cols = 0;
  // interpolation by a fixed grid of workgroups that each take a sequence of tiles, loading the
  // next tile's block while interpolating the current one: its workgroup count (0: off; the plan
  // sets -1 to ask for it, and preparing the kernels resolves it)
  int gather_stream = 0;
  size_t lds_spread = 0, lds_gather = 0;  // maxima over the group's systems
};

// Largest workgroup of the particle kernels for window support P (their launch bound).
inline int particle_max_threads_host(int P) { return P <= 13 ? 1024 : 512; }

// Spreading by columns: tile edges served, particles per batch, block edge S, workgroup size
// and LDS.
inline bool col_tile_ok(int B) { return B == 4 || B == 6 || B == 8; }
constexpr int kColBatchHost = 32;
inline int col_edge_host(int P, int B) { return B + P - 1; }
inline int col_threads_host(int P, int B) { return (col_edge_host(P, B) * col_edge_host(P, B) + 63) / 64 * 64; }
inline int mfma_threads_host(int P, int B) {
  const int S = col_edge_host(P, B), pieces = (S * S + 15) / 16;
  return 64 * ((pieces + 3) / 4);
}
// Matrix-core spreading by two column slices: the block is wider than one 16-column piece
// (S > 16), and every particle's x-support fits the columns [0, 16) (o_x <= 16 - P) or
// [S - 16, S) (o_x >= S - 16), o_x in [0, B): B + 2 P <= 34.
constexpr bool mfma_sliced_host(int P, int B) { return B + P - 1 > 16 && B + 2 * P <= 34; }
// particles per batch of the matrix-core spread: one tile per workgroup, and by columns of tiles
constexpr int kMfmaBatchHost = 64, kMfmaRollBatchHost = 32;
// LDS of a batch's records: coefficients, offsets, window values, and slots for a batch plus the
// padding of two slices
inline size_t mfma_batch_lds_bytes(int P, int D, int B, size_t acc_bytes, int batch) {
  const size_t S = static_cast<size_t>(col_edge_host(P, B)), nrec = static_cast<size_t>(batch) + 8;
  return sizeof(double) * (static_cast<size_t>(P) * coef_stride(D) + nrec * 4) + sizeof(int) * nrec * 4 +
         acc_bytes * nrec * 3 * S + 16;
}
inline size_t mfma_lds_bytes(int P, int D, int B, size_t acc_bytes) {
  const size_t S = static_cast<size_t>(col_edge_host(P, B));
  const size_t batch = mfma_batch_lds_bytes(P, D, B, acc_bytes, kMfmaBatchHost);
  return std::max(batch, sizeof(double) * S * S * S);  // the records, then the block
}
// The same with the ring of a column of tiles (S^3 float64) ahead of the records.
inline size_t mfma_roll_lds_bytes(int P, int D, int B, size_t acc_bytes) {
  const size_t S = static_cast<size_t>(col_edge_host(P, B));
  return sizeof(double) * S * S * S + mfma_batch_lds_bytes(P, D, B, acc_bytes, kMfmaRollBatchHost);
}
inline size_t col_lds_bytes(int P, int D, int B) {
  const int S = col_edge_host(P, B);
  return sizeof(double) * (static_cast<size_t>(P) * coef_stride(D) + kColBatchHost * (3 * S + 4)) +
         sizeof(int) * kColBatchHost * 4;
}

// binning: at most kCoarse coarse buckets, counted in kCoarseCopies copies (workgroup w adds
// into copy w % kCoarseCopies, so fewer atomics queue on one address), and at most
// kBinMaxPerThread particles per thread
constexpr int kCoarse = 256;
constexpr int kCoarseCopies = 16;
constexpr int kBinMaxPerThread = 8;
constexpr int kBinMaxFine = 16384;  // buckets per coarse bucket (LDS counters of the fine pass)

struct DevPlan {
  int prec = 0;               // 0 float, 1 double
  int nsys = 0;
  int64_t n_max = 0;          // packed particles accepted (batch: exactly this many)
  std::vector<SysDesc> sys;   // host copies of the descriptors
  std::vector<PGroup> groups; // by increasing (P, D)
  SysDesc* sys_dev = nullptr;
  int* tile_prefix = nullptr;      // nsys + 1: tile ranges in global tile order (grouped by P, D)
  int* tile_sys = nullptr;         // nsys: system owning the k-th tile range
  int* xblk_prefix = nullptr;      // nsys + 1, in system order
  int* zblk_prefix = nullptr;      // nsys + 1: blocks of the z-direction pass
  int total_zblk = 0;
  // y and z passes fused per spectrum column (k_fft_yz) when every system's (y, z) plane fits in LDS
  int yz_fft = 0;
  // float32-arithmetic plans whose spread accumulates into grid_a read as a float32 grid
  int grid32 = 0;
  int* yzblk_prefix = nullptr;     // nsys + 1: blocks (columns) of the fused pass
  int total_yzblk = 0;
  size_t lds_yz = 0;
  int* pblk_prefix = nullptr;      // nsys + 1: z-planes, for the plane FFT kernels
  int plane_fft = 0;               // x and y FFTs fused per z-plane (every system's plane fits in LDS)
  int total_pblk = 0;
  size_t lds_p = 0;                // LDS of the plane FFT kernels
  int* cblk_prefix = nullptr;      // nsys + 1, in system order
  int64_t* part_prefix = nullptr;  // nsys + 1 (batches; a single system takes n per call)
  int total_tiles = 0, total_xblk = 0, total_cblk = 0;
  size_t lds_x = 0, lds_c = 0;     // maxima over the systems
  // binning, over all systems. Each tile is split into 2^sub_log2 buckets by the particle's
  // z-cell within the tile, so a tile's particles come out ordered by z; a tile's particles stay
  // contiguous: tile t owns [tile_start[t << sub_log2], tile_start[(t+1) << sub_log2]). The sort
  // runs in two levels: coarse buckets (bucket >> bin_shift, bin_ncoarse <= kCoarse of them), then
  // the buckets within each coarse bucket.
  int sub_log2 = 0;
  int bin_levels = 2;          // 1: one-level sort (small systems), 2: two-level sort
  int* tile_count = nullptr;   // one-level: total_tiles << sub_log2, kept all-zero between calls
  int* bin_rank = nullptr;     // one-level: n_max ranks within the bucket (over bin_tmp_ib)
  int bin_shift = 0;
  int bin_ncoarse = 1;
  int bin_per_thread = 1;      // particles per thread in the counting and coarse passes
  int* coarse_count = nullptr; // kCoarseCopies x kCoarse, kept all-zero between calls
  int* coarse_cursor = nullptr;// kCoarseCopies x kCoarse, kept all-zero between calls
  int* coarse_start = nullptr; // kCoarse + 1
  void* bin_tmp = nullptr;     // n_max x 4: (x, y, z, q) in coarse-bucket order
  int2* bin_tmp_ib = nullptr;  // n_max: (input index, bucket) in coarse-bucket order
  int* tile_start = nullptr;   // (total_tiles << sub_log2) + 1
  int* tile_of = nullptr;      // n_max: bucket of each particle
  int* perm = nullptr;         // n_max: sorted slot -> packed input index
  int* cells = nullptr;        // n_max: packed cell cx + m (cy + m cz) of each sorted particle
  void* sorted = nullptr;      // n_max x 4: (f_x, f_y, f_z, q), fractional cell offsets in [0, 1]
  // real-space cell list, over all systems
  int total_cells = 0;
  int* cell_prefix = nullptr;  // nsys + 1: first global cell of each system
  int* cell_count = nullptr;   // total_cells, kept all-zero between calls
  int* cell_start = nullptr;   // total_cells + 1
  int* cell_of = nullptr;      // n_max
  int* cell_rank = nullptr;    // n_max
  double* lsorted = nullptr;   // n_max x 4: wrapped position (float64) and charge, by cell
  int* lperm = nullptr;        // n_max: cell-sorted slot -> packed input index
  int local_deg = 0;           // highest residual polynomial degree over the systems
  int local_threads = 512;     // residual workgroup size (128, 256, 512)
  StageTimer* timer = nullptr; // optional instrumentation
  double* check = nullptr;     // 3 nsys doubles: results of the input check
};

inline void stage_begin(const DevPlan& d, int stage, hipStream_t st) {
  StageTimer* t = d.timer;
  if (t && t->stage == stage && t->count < t->cap) (void)hipEventRecord(t->ev[2 * t->count], st);
}
inline void stage_end(const DevPlan& d, int stage, hipStream_t st) {
  StageTimer* t = d.timer;
  if (t && t->stage == stage && t->count < t->cap) {
    (void)hipEventRecord(t->ev[2 * t->count + 1], st);
    ++t->count;
  }
}

// The particle kernels (spreading, interpolation) are compiled from one source once per
// precision (0 float, 1 double) and range [lo, hi] of window supports P, so that their many
// template instances build in parallel. Each instance defines the three functions below with
// the suffix _<prec>_<lo>; the ranges cover [kPmin, kPmax] without overlap.
#define PSWFE_PARTICLE_INSTANCES(X) \
  X(0, 3, 8) X(0, 9, 12) X(0, 13, 16) X(0, 17, 20) X(0, 21, 24) \
  X(1, 3, 8) X(1, 9, 12) X(1, 13, 16) X(1, 17, 20) X(1, 21, 24)

#define PSWFE_PARTICLE_DECLARE(prec, lo, hi)                                                              \
  hipError_t particles_prepare_##prec##_##lo(PGroup& g);                                                  \
  hipError_t particles_spread_##prec##_##lo(const DevPlan& d, const PGroup& g, hipStream_t st);           \
  hipError_t particles_gather_##prec##_##lo(const DevPlan& d, const PGroup& g, const void* grid, void* phi, \
                                            void* vec, int vec_mode, bool add_self, double* energy,       \
                                            const double* phi_add, const double* vec_add, hipStream_t st);
PSWFE_PARTICLE_INSTANCES(PSWFE_PARTICLE_DECLARE)
#undef PSWFE_PARTICLE_DECLARE

// One-time kernel attributes (dynamic LDS above 64 KiB) and launch choices that depend on
// occupancy; call at plan creation.
hipError_t prepare_kernels(DevPlan& d);

// Pipeline pieces; all enqueue on `stream` and return hipSuccess or the launch error.
// n_total: packed particles (a single system: its n). energy: nsys doubles zeroed here, or NULL.
hipError_t launch_bin(const DevPlan& d, int64_t n_total, const void* pos, const void* q, double* energy,
                      hipStream_t stream);
// Zeroes `bytes` (a multiple of 4) at device address p with a fill kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);
// Input check: per system s, out[3 s .. 3 s + 2] = (sum q, sum |q|, number of particles with a
// non-finite position or charge), float64; out holds 3 nsys doubles (zeroed here).
hipError_t launch_check(const DevPlan& d, int64_t n_total, const void* pos, const void* q, double* out,
                        hipStream_t stream);
// Spreads the binned particles into each system's float64 grid_a.
hipError_t launch_spread(const DevPlan& d, hipStream_t stream);
// Copies grid_a of system 0 into `out` (plan precision) and zeroes it.
hipError_t launch_drain(const DevPlan& d, void* out, hipStream_t stream);
// Steps 2-4 for every system, grid_a -> grid_b (grid_a zeroed after it is read). With
// in_override / out_override (single system only) the input is the plan-precision grid
// in_override (not modified) and the output goes to out_override.
hipError_t launch_transform(const DevPlan& d, const void* in_override, void* out_override, hipStream_t stream);
// vec_mode: 0 writes force -q grad(phi), 1 writes grad(phi). add_self adds -self_coef q to phi.
// grid_override (single system only) replaces grid_b. energy: nsys doubles, accumulated.
// phi_add / vec_add (nullable, float64, n and n x 3 in input order) are added to each particle's
// potential and vec term before they are rounded and before the energy sum.
hipError_t launch_gather(const DevPlan& d, const void* grid_override, void* phi, void* vec, int vec_mode,
                         bool add_self, double* energy, hipStream_t stream, const double* phi_add = nullptr,
                         const double* vec_add = nullptr);
// Real-space residual of every system: cell binning, then phi_local, its gradient term and
// energy, added to phi / vec / energy when accumulate is set, else written (energy zeroed
// first). vec_mode as in launch_gather. With phi_d set, phi_local and the vec term (if vec_d)
// are written to these float64 arrays instead, and phi, vec, energy are not touched.
hipError_t launch_local(const DevPlan& d, int64_t n_total, const void* pos, const void* q, void* phi, void* vec,
                        int vec_mode, double* energy, bool accumulate, hipStream_t stream, double* phi_d = nullptr,
                        double* vec_d = nullptr);

}  // namespace pswfe
