// C-ABI of the library (declared in include/pswfe.h): parameter choice, plans, compute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pswfe.h"
#include "host.hpp"
#include "kernels.hpp"

struct pswfe_plan {
  pswfe::Params p;
  pswfe::Tables tab;
  pswfe::DevPlan d;
  pswfe::StageTimer timer;
  int device = 0;
};

namespace {

pswfe_status from_hip(hipError_t e) { return e == hipSuccess ? PSWFE_OK : PSWFE_E_HIP; }

void to_c(const pswfe::Params& p, pswfe_params* o) {
  o->L = p.L;
  o->eps = p.eps;
  o->rc = p.rc;
  o->cs = p.cs;
  o->cw = p.cw;
  o->alpha = p.alpha;
  o->h = p.h;
  o->lambda0_s = p.lambda0_s;
  o->cs_alg = p.cs_alg;
  o->cw_alg = p.cw_alg;
  o->alpha_alg = p.alpha_alg;
  o->m = p.m;
  o->P = p.P;
  o->tol_mode = p.tol_mode;
  o->reserved = 0;
}

pswfe::FftPlan make_fft_plan(int N) {
  pswfe::FftPlan pl;
  pl.N = N;
  int r = N;
  auto push = [&](int R) { pl.radix[pl.nst++] = R; r /= R; };
  while (r % 8 == 0 && pl.nst < pswfe::kMaxStages) push(8);
  while (r % 4 == 0 && pl.nst < pswfe::kMaxStages) push(4);
  while (r % 2 == 0 && pl.nst < pswfe::kMaxStages) push(2);
  for (int R : {3, 5, 7})
    while (r % R == 0 && pl.nst < pswfe::kMaxStages) push(R);
  if (r != 1) pl.nst = -1;
  return pl;
}

// Tile edge B (cells) for binning, spreading and interpolation. The spreading tile holds
// S^3 float64 accumulators (S = B + 2 ceil(P/2) - 1), at most 150 KiB; the interpolation tile
// S^3 values of the plan precision plus the window records of 16 particles, at most 156 KiB.
// Default: B = 8 (measured best on gfx950 for 64^3 and 128^3 grids with P = 12-18), reduced to
// fit the LDS limits and to give at least 64 tiles on small grids.
size_t gather_lds_bytes(int S, int P, int elem) {
  return static_cast<size_t>(elem) * S * S * S + sizeof(double) * 16 * 6 * P;
}

bool tile_fits(int B, int P, int elem) {
  const int S = B + 2 * ((P + 1) / 2) - 1;
  return 8.0 * (static_cast<double>(S) * S * S + 16 * 3 * P) <= 150.0 * 1024 &&
         gather_lds_bytes(S, P, elem) <= 156 * 1024;
}

int choose_tile(int m, int P, int requested, int elem) {
  int B = requested;
  if (B <= 0) {
    if (const char* env = std::getenv("PSWFE_TILE")) B = std::atoi(env);
  }
  if (B <= 0) {
    B = 8;
    while (B > 2 && (m + B - 1) / B < 4) --B;
  }
  B = std::max(2, std::min(B, m));
  while (B > 2 && !tile_fits(B, P, elem)) --B;
  return B;
}

template <class T>
pswfe_status upload(const std::vector<double>& src, void** dst) {
  std::vector<T> tmp(src.begin(), src.end());
  if (hipMalloc(dst, sizeof(T) * std::max<size_t>(tmp.size(), 1)) != hipSuccess) return PSWFE_E_ALLOC;
  if (!tmp.empty() && hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice) != hipSuccess)
    return PSWFE_E_HIP;
  return PSWFE_OK;
}

void free_timer(pswfe::StageTimer& t) {
  if (t.ev) {
    for (int i = 0; i < 2 * t.cap; ++i)
      if (t.ev[i]) (void)hipEventDestroy(t.ev[i]);
    delete[] t.ev;
  }
  t = pswfe::StageTimer();
}

void free_plan_buffers(pswfe::DevPlan& d) {
  void* bufs[] = {d.tile_count, d.tile_start, d.tile_of, d.rank, d.perm, d.cells, d.sorted, d.grid_a, d.grid_b, d.spec,
                  d.coef, d.tm, d.wk, d.tw_half_p, d.tw_half_m, d.tw_full_p, d.tw_full_m};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

}  // namespace

extern "C" {

const char* pswfe_status_str(pswfe_status s) {
  switch (s) {
    case PSWFE_OK: return "ok";
    case PSWFE_E_ARG: return "invalid argument";
    case PSWFE_E_EPS_RANGE: return "tolerance outside the supported range";
    case PSWFE_E_GRID: return "unsupported grid size or window support";
    case PSWFE_E_ALLOC: return "device allocation failed";
    case PSWFE_E_HIP: return "HIP runtime error";
    case PSWFE_E_CAPACITY: return "more particles than the plan's n_max";
    case PSWFE_E_PREC: return "unknown precision";
  }
  return "unknown status";
}

const char* pswfe_version(void) { return "pswfe 0.1 gfx950"; }

pswfe_status pswfe_choose_params(double eps, double L, double rc, int32_t m, int64_t n, double q_l2,
                                 int32_t tol_mode, pswfe_params* out) {
  if (!out) return PSWFE_E_ARG;
  pswfe::Params p{};
  const int rcode = pswfe::choose_params(eps, L, rc, m, n, q_l2, tol_mode, &p);
  if (rcode != 0) return static_cast<pswfe_status>(rcode);
  to_c(p, out);
  return PSWFE_OK;
}

pswfe_status pswfe_host_pswf(double c, double x, double* psi, double* dpsi, double* lambda0, double* chi0) {
  if (!(c > 0.0) || c > 60.0 || !(x >= -1.0 && x <= 1.0)) return PSWFE_E_ARG;
  const pswfe::Pswf f(c);
  if (psi) *psi = f.psi(x);
  if (dpsi) *dpsi = f.dpsi(x);
  if (lambda0) *lambda0 = f.lambda0;
  if (chi0) *chi0 = f.chi0;
  return PSWFE_OK;
}

namespace {
pswfe_status params_from_c(const pswfe_params* pp, pswfe::Params* p) {
  const int m = pp->m, P = pp->P;
  if (!pswfe::is_smooth_even(m) || m < 8 || m > 512 || P < pswfe::kPmin || P > pswfe::kPmax || P > m)
    return PSWFE_E_GRID;
  if (!(pp->L > 0) || !(pp->rc > 0) || !(pp->cs > 0) || !(pp->cw > 0) || !(pp->alpha > 0) || !(pp->eps > 0))
    return PSWFE_E_ARG;
  if (pp->cs > 40.0 || pp->cw > 40.0) return PSWFE_E_EPS_RANGE;
  p->L = pp->L;
  p->eps = pp->eps;
  p->rc = pp->rc;
  p->cs = pp->cs;
  p->cw = pp->cw;
  p->alpha = pp->alpha;
  p->h = pp->L / m;
  p->cs_alg = pp->cs_alg;
  p->cw_alg = pp->cw_alg;
  p->alpha_alg = pp->alpha_alg;
  p->m = m;
  p->P = P;
  p->tol_mode = pp->tol_mode;
  p->lambda0_s = pswfe::Pswf(p->cs).lambda0;
  return PSWFE_OK;
}

double fit_tolerance(double eps, int prec) { return std::max(0.01 * eps, prec == PSWFE_FP32 ? 5e-9 : 1e-15); }
}  // namespace

pswfe_status pswfe_host_tables(const pswfe_params* pp, int32_t prec, double* tm, int64_t tm_len, double* w,
                               int64_t w_len, double* coef, int64_t coef_len, double* info) {
  if (!pp) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64) return PSWFE_E_PREC;
  pswfe::Params p{};
  const pswfe_status st = params_from_c(pp, &p);
  if (st != PSWFE_OK) return st;
  pswfe::Tables t;
  pswfe::build_tables(p, 0, fit_tolerance(p.eps, prec), &t);
  if ((tm && tm_len < static_cast<int64_t>(t.tm.size())) || (w && w_len < static_cast<int64_t>(t.w.size())) ||
      (coef && coef_len < static_cast<int64_t>(t.coef.size())))
    return PSWFE_E_ARG;
  if (tm) std::copy(t.tm.begin(), t.tm.end(), tm);
  if (w) std::copy(t.w.begin(), t.w.end(), w);
  if (coef) std::copy(t.coef.begin(), t.coef.end(), coef);
  if (info) {
    info[0] = t.deg;
    info[1] = t.fit_err;
    info[2] = t.fit_err_deriv;
    info[3] = t.self_coef;
  }
  return PSWFE_OK;
}

pswfe_status pswfe_plan_params(const pswfe_plan* plan, pswfe_params* out) {
  if (!plan || !out) return PSWFE_E_ARG;
  to_c(plan->p, out);
  return PSWFE_OK;
}

int32_t pswfe_plan_tile(const pswfe_plan* plan) { return plan ? plan->d.B : 0; }

pswfe_status pswfe_plan_create(const pswfe_params* pp, int32_t prec, int64_t n_max, pswfe_plan** out) {
  return pswfe_plan_create_tiled(pp, prec, n_max, 0, out);
}

pswfe_status pswfe_plan_create_tiled(const pswfe_params* pp, int32_t prec, int64_t n_max, int32_t tile,
                                     pswfe_plan** out) {
  if (!out) return PSWFE_E_ARG;
  *out = nullptr;
  if (!pp || n_max < 0 || n_max > (int64_t(1) << 31) - 1) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64) return PSWFE_E_PREC;
  pswfe::Params pcheck{};
  const pswfe_status pst = params_from_c(pp, &pcheck);
  if (pst != PSWFE_OK) return pst;
  const int m = pp->m, P = pp->P;
  pswfe_plan* plan = new (std::nothrow) pswfe_plan();
  if (!plan) return PSWFE_E_ALLOC;
  pswfe::Params& p = plan->p;
  p = pcheck;
  pswfe::build_tables(p, 0, fit_tolerance(p.eps, prec), &plan->tab);
  (void)hipGetDevice(&plan->device);

  pswfe::DevPlan& d = plan->d;
  const int elem = prec == PSWFE_FP32 ? 4 : 8;
  d.prec = prec;
  d.m = m;
  d.P = P;
  d.deg = plan->tab.deg;
  if (tile < 0 || tile > m) {
    delete plan;
    return PSWFE_E_ARG;
  }
  d.B = choose_tile(m, P, tile, elem);
  d.Tn = (m + d.B - 1) / d.B;
  d.ntiles = d.Tn * d.Tn * d.Tn;
  d.S = d.B + 2 * ((P + 1) / 2) - 1;
  d.L = p.L;
  d.h = p.h;
  d.inv_h = m / p.L;
  {
    const long double ih = static_cast<long double>(m) / static_cast<long double>(p.L);
    if (prec == PSWFE_FP32) {
      const float hi = static_cast<float>(ih);
      d.inv_h_hi = hi;
      d.inv_h_lo = static_cast<float>(ih - static_cast<long double>(hi));
    } else {
      const double hi = static_cast<double>(ih);
      d.inv_h_hi = hi;
      d.inv_h_lo = static_cast<double>(ih - static_cast<long double>(hi));
    }
  }
  d.self_coef = plan->tab.self_coef;
  d.n_max = n_max;
  d.fft_half = make_fft_plan(m / 2);
  d.fft_full = make_fft_plan(m);
  if (d.fft_half.nst < 0 || d.fft_full.nst < 0) {
    delete plan;
    return PSWFE_E_GRID;
  }
  const int N = m / 2;
  d.rows_per_block = std::max(1, std::min(64, 2048 / (N + 1)));
  while (d.rows_per_block > 1 && size_t(2) * d.rows_per_block * (N + 1) * 2 * elem > 64 * 1024) --d.rows_per_block;
  int cmax = std::max(1, std::min(64, 2048 / (m + 1)));
  while (cmax > 1 && size_t(2) * cmax * (m + 1) * 2 * elem > 64 * 1024) --cmax;
  const int nblk = (N + 1 + cmax - 1) / cmax;
  d.cols_per_block = (N + 1 + nblk - 1) / nblk;

  const size_t m3 = size_t(m) * m * m;
  const size_t nspec = size_t(m) * m * (N + 1);
  const size_t nm = std::max<int64_t>(n_max, 1);
  pswfe_status st = PSWFE_OK;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (st == PSWFE_OK && hipMalloc(ptr, std::max<size_t>(bytes, 16)) != hipSuccess) st = PSWFE_E_ALLOC;
  };
  alloc(reinterpret_cast<void**>(&d.tile_count), sizeof(int) * d.ntiles);
  alloc(reinterpret_cast<void**>(&d.tile_start), sizeof(int) * (d.ntiles + 1));
  alloc(reinterpret_cast<void**>(&d.tile_of), sizeof(int) * nm);
  alloc(reinterpret_cast<void**>(&d.rank), sizeof(int) * nm);
  alloc(reinterpret_cast<void**>(&d.perm), sizeof(int) * nm);
  alloc(reinterpret_cast<void**>(&d.cells), sizeof(int) * nm);
  alloc(&d.sorted, size_t(4) * elem * nm);
  alloc(&d.grid_a, sizeof(double) * m3);
  alloc(&d.grid_b, elem * m3);
  alloc(&d.spec, size_t(2) * elem * nspec);
  if (st == PSWFE_OK) {
    std::vector<double> twhp, twhm, twfp, twfm;
    pswfe::twiddles(N, +1, &twhp);
    pswfe::twiddles(N, -1, &twhm);
    pswfe::twiddles(m, +1, &twfp);
    pswfe::twiddles(m, -1, &twfm);
    auto up = [&](const std::vector<double>& v, void** dst) {
      if (st == PSWFE_OK) st = prec == PSWFE_FP32 ? upload<float>(v, dst) : upload<double>(v, dst);
    };
    if (st == PSWFE_OK) st = upload<double>(plan->tab.coef, &d.coef);  // window polynomials: float64
    up(plan->tab.tm, &d.tm);
    up(plan->tab.w, &d.wk);
    up(twhp, &d.tw_half_p);
    up(twhm, &d.tw_half_m);
    up(twfp, &d.tw_full_p);
    up(twfm, &d.tw_full_m);
  }
  if (st == PSWFE_OK && (hipMemset(d.tile_count, 0, sizeof(int) * d.ntiles) != hipSuccess ||
                         hipMemset(d.grid_a, 0, sizeof(double) * m3) != hipSuccess ||
                         hipDeviceSynchronize() != hipSuccess))
    st = PSWFE_E_HIP;
  if (st != PSWFE_OK) {
    free_plan_buffers(d);
    delete plan;
    return st;
  }
  *out = plan;
  return PSWFE_OK;
}

pswfe_status pswfe_plan_destroy(pswfe_plan* plan) {
  if (!plan) return PSWFE_OK;
  (void)hipDeviceSynchronize();
  free_timer(plan->timer);
  free_plan_buffers(plan->d);
  delete plan;
  return PSWFE_OK;
}

pswfe_status pswfe_timing_enable(pswfe_plan* plan, int32_t stage, int32_t max_calls) {
  if (!plan || stage < -1 || stage >= pswfe::kNumStages || (stage >= 0 && (max_calls < 1 || max_calls > 1 << 20)))
    return PSWFE_E_ARG;
  (void)hipDeviceSynchronize();
  free_timer(plan->timer);
  plan->d.timer = nullptr;
  if (stage < 0) return PSWFE_OK;
  pswfe::StageTimer& t = plan->timer;
  t.ev = new (std::nothrow) hipEvent_t[2 * static_cast<size_t>(max_calls)]();
  if (!t.ev) return PSWFE_E_ALLOC;
  t.cap = max_calls;
  for (int i = 0; i < 2 * max_calls; ++i)
    if (hipEventCreate(&t.ev[i]) != hipSuccess) {
      free_timer(t);
      return PSWFE_E_HIP;
    }
  t.stage = stage;
  t.count = 0;
  plan->d.timer = &t;
  return PSWFE_OK;
}

pswfe_status pswfe_timing_read(pswfe_plan* plan, double* total_ms, int64_t* calls) {
  if (!plan || !total_ms || !calls) return PSWFE_E_ARG;
  pswfe::StageTimer& t = plan->timer;
  double sum = 0.0;
  if (t.count > 0 && hipEventSynchronize(t.ev[2 * t.count - 1]) != hipSuccess) return PSWFE_E_HIP;
  for (int i = 0; i < t.count; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) != hipSuccess) return PSWFE_E_HIP;
    sum += ms;
  }
  *total_ms = sum;
  *calls = t.count;
  t.count = 0;
  return PSWFE_OK;
}

namespace {
pswfe_status compute_impl(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                          int vec_mode, double* energy, void* stream) {
  if (!plan || n < 0) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const pswfe::DevPlan& d = plan->d;
  pswfe::stage_begin(d, pswfe::kStageAll, s);
  hipError_t e = pswfe::launch_bin(d, n, pos, q, energy, s);
  if (e == hipSuccess) e = pswfe::launch_spread(d, d.grid_a, s);
  if (e == hipSuccess) e = pswfe::launch_transform(d, d.grid_a, true, d.grid_b, true, s);
  if (e == hipSuccess && n > 0) e = pswfe::launch_gather(d, n, d.grid_b, phi, vec, vec_mode, true, energy, s);
  pswfe::stage_end(d, pswfe::kStageAll, s);
  return from_hip(e);
}
}  // namespace

pswfe_status pswfe_compute(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* force,
                           double* energy, void* stream) {
  return compute_impl(plan, n, pos, q, phi, force, 0, energy, stream);
}

pswfe_status pswfe_compute_grad(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* grad,
                                double* energy, void* stream) {
  return compute_impl(plan, n, pos, q, phi, grad, 1, energy, stream);
}

pswfe_status pswfe_spread(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* grid, void* stream) {
  if (!plan || n < 0 || !grid) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const pswfe::DevPlan& d = plan->d;
  hipError_t e = pswfe::launch_bin(d, n, pos, q, nullptr, s);
  if (e == hipSuccess) e = pswfe::launch_spread(d, d.grid_a, s);
  if (e == hipSuccess) e = pswfe::launch_drain(d, grid, s);
  return from_hip(e);
}

pswfe_status pswfe_transform(pswfe_plan* plan, const void* grid_in, void* grid_out, void* stream) {
  if (!plan || !grid_in || !grid_out) return PSWFE_E_ARG;
  return from_hip(pswfe::launch_transform(plan->d, grid_in, plan->d.prec == 1, grid_out, false,
                                          static_cast<hipStream_t>(stream)));
}

pswfe_status pswfe_interpolate(pswfe_plan* plan, int64_t n, const void* pos, const void* grid, void* phi, void* grad,
                               void* stream) {
  if (!plan || n < 0 || !grid) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && !pos) return PSWFE_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const pswfe::DevPlan& d = plan->d;
  hipError_t e = pswfe::launch_bin(d, n, pos, nullptr, nullptr, s);
  if (e == hipSuccess && n > 0) e = pswfe::launch_gather(d, n, grid, phi, grad, 1, false, nullptr, s);
  return from_hip(e);
}

}  // extern "C"
