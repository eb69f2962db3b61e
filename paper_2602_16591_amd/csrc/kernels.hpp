// Device kernels of the PSWF fast Ewald pipeline (Alg. 2) and their launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
  kStageIfftX = 6, kStageGather = 7, kStageAll = 8, kNumStages = 9
};

// HIP events recorded around one stage of successive calls (owned by the plan).
struct StageTimer {
  int stage = -1;
  int cap = 0;
  int count = 0;
  hipEvent_t* ev = nullptr;  // 2 * cap events: start, stop per call
};

// Everything a launch needs about a plan, in device terms. Pointers are device pointers in
// the plan's precision T (real) or 2T (complex interleaved) unless stated.
struct DevPlan {
  int prec = 0;        // 0 float, 1 double
  int m = 0, P = 0, deg = 0;
  int B = 0;           // tile edge in grid cells (binning and spread/gather tiles)
  int Tn = 0;          // tiles per dimension
  int ntiles = 0;
  int S = 0;           // LDS tile edge = B + 2 ceil(P/2) - 1
  double L = 0, h = 0, inv_h = 0, self_coef = 0;
  double inv_h_hi = 0, inv_h_lo = 0;  // m/L split into a working-precision word and its remainder
  int64_t n_max = 0;
  // binning
  int* tile_count = nullptr;   // ntiles, kept all-zero between calls
  int* tile_start = nullptr;   // ntiles + 1
  int* tile_of = nullptr;      // n_max
  int* rank = nullptr;         // n_max
  int* perm = nullptr;         // n_max: sorted slot -> input index
  void* sorted = nullptr;      // n_max x 4 T: (f_x, f_y, f_z, q), fractional cell offsets in [0, 1]
  int* cells = nullptr;        // n_max: packed cell cx + m (cy + m cz) of each sorted particle
  // grids
  void* grid_a = nullptr;      // m^3 float64 spread target (both precisions); kept all-zero between calls
  void* grid_b = nullptr;      // m^3 T, transformed grid
  void* spec = nullptr;        // m * m * (m/2 + 1) complex T
  // tables (plan precision)
  void* coef = nullptr;        // P * (deg + 1) window polynomial coefficients
  void* tm = nullptr;          // 3 (m/2)^2 + 1
  void* wk = nullptr;          // m/2 + 1
  void* tw_half_p = nullptr;   // N = m/2, exp(+2 pi i e / N)
  void* tw_half_m = nullptr;   // N = m/2, exp(-2 pi i e / N)
  void* tw_full_p = nullptr;   // N = m,   exp(+2 pi i e / N)
  void* tw_full_m = nullptr;   // N = m,   exp(-2 pi i e / N)
  FftPlan fft_half, fft_full;
  StageTimer* timer = nullptr; // optional instrumentation
  int rows_per_block = 1;      // x-direction R2C / C2R batching
  int cols_per_block = 1;      // y/z-direction batching
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

// Pipeline pieces (all enqueue on `stream`, return hipSuccess or the launch error).
hipError_t launch_bin(const DevPlan& d, int64_t n, const void* pos, const void* q, double* energy_zero,
                      hipStream_t stream);
// Spreads the binned particles into the float64 grid d.grid_a.
hipError_t launch_spread(const DevPlan& d, void* grid, hipStream_t stream);
// Copies d.grid_a into `out` (plan precision) and zeroes d.grid_a.
hipError_t launch_drain(const DevPlan& d, void* out, hipStream_t stream);
hipError_t launch_zero(const DevPlan& d, void* buf, int64_t count, hipStream_t stream);
// grid_in is float64 when in_f64 (always for float64 plans), else the plan precision.
hipError_t launch_transform(const DevPlan& d, const void* grid_in, bool in_f64, void* grid_out, bool zero_input,
                            hipStream_t stream);
// vec_mode: 0 writes force -q grad(phi), 1 writes grad(phi). add_self adds -self_coef q to phi.
hipError_t launch_gather(const DevPlan& d, int64_t n, const void* grid, void* phi, void* vec, int vec_mode,
                         bool add_self, double* energy, hipStream_t stream);

}  // namespace pswfe
