// C-ABI of the library (declared in include/pswfe.h): parameter choice, plans, compute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/pswfe.h"
#include "host.hpp"
#include "kernels.hpp"

// Device memory of pswfe_compute_noalloc: every buffer of its pipeline (tables, descriptors,
// grids, spectrum, particle bins) is laid out in this array, one copy per GPU, held until the
// process ends. In host code the name stands for a host-side shadow, not a device address: the
// device address is taken once per device with hipGetSymbolAddress and used everywhere instead.
static constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct pswfe_plan {
  std::vector<pswfe::Params> p;   // effective parameters of each system
  std::vector<pswfe::Tables> tab; // host tables of each system
  std::vector<pswfe::LocalTable> ltab;  // real-space residual tables
  bool local_ok = true;           // every system has r_c < L/2 (minimum image)
  std::vector<int64_t> count;     // batch plans: particles of each system
  bool batch = false;             // created by pswfe_batch_plan_create
  pswfe::DevPlan d;
  pswfe::StageTimer timer;
  int device = 0;
  std::vector<void*> allocs;      // device allocations owned by the plan
  // The real-space residual of PSWFE_TOTAL calls runs on a stream of its own, forked from and
  // joined back to the caller's stream with events, while binning, spreading and the FFT run on
  // the caller's; interpolation then adds its float64 results (phi_d, vec_d).
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* phi_d = nullptr;        // n_max
  double* vec_d = nullptr;        // n_max x 3
  bool overlap = true;            // PSWFE_LOCAL_OVERLAP=0: residual after the long-range part, same stream
  // device arena holding every buffer (owned, or caller-provided memory), its size, the byte
  // ranges that must start at zero, and (caller-provided memory only) the host image of its
  // constant part, uploaded at compute time
  unsigned char* base = nullptr;
  size_t arena_bytes = 0;
  std::vector<std::pair<size_t, size_t>> zero;
  std::vector<unsigned char> img;
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
  o->split = p.split;
  o->window = p.window;
  o->reserved = 0;
  o->cg = p.cg;
  o->Ly = p.side(1);
  o->Lz = p.side(2);
  o->my = p.grid(1);
  o->mz = p.grid(2);
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
// S^3 float64 accumulators (S = lds_edge(B, P)), at most 150 KiB; the interpolation tile
// S^3 values of the plan precision plus the window records of 16 particles, at most 156 KiB.
// Both also hold the P coefficient rows of the window polynomials (coef_stride(D) doubles each)
// and one window record per particle slot (16 lanes each).
size_t coef_lds_bytes(int P, int D) { return sizeof(double) * P * pswfe::coef_stride(D); }
size_t spread_lds_bytes(int S, int P, int D, int threads) {
  return sizeof(double) * (static_cast<size_t>(S) * S * S + (threads / 16) * 3 * P) + coef_lds_bytes(P, D);
}
size_t gather_lds_bytes(int S, int P, int D, int elem, int threads, size_t gbytes = sizeof(double)) {
  return pswfe::gather_block_bytes(S, elem) + sizeof(double) * 16 + gbytes * (threads / 16) * 6 * P +
         coef_lds_bytes(P, D);
}
// LDS tile edge of interpolation and LDS-atomic spreading: the halo block B + P - 1 (supports
// start at o in [0, B-1]), made odd so that the 16 lanes of a particle, reading or adding lines
// at stride S, hit distinct banks (an even S = 20 took the water-box interpolation from 39 to
// 42 us in float32 and from 50 to 76 us in float64). The register kernels use B + P - 1.
int lds_edge(int B, int P) { return (B + P - 1) | 1; }
constexpr size_t kLdsLimit = 160 * 1024;
// largest LDS of the fused y/z FFT workgroup
constexpr size_t kYzLdsMax = kLdsLimit;
// fewest workgroups (spectrum columns over all systems) for which the fused y/z pass is chosen
constexpr int kYzMinBlocks = 256;
// fewest grid points over all systems for which a float32-arithmetic plan accumulates in float32
constexpr int64_t kGrid32MinPoints = int64_t(1) << 20;

bool tile_fits(int B, int P, int elem) {
  const int S = lds_edge(B, P);
  const int D = pswfe::kMaxDeg;  // whatever the degree, the tile fits with 256-thread workgroups
  return spread_lds_bytes(S, P, D, 256) <= kLdsLimit && gather_lds_bytes(S, P, D, elem, 256) <= kLdsLimit;
}

// Workgroup size of a particle kernel: the most resident waves per compute unit (LDS and the
// 16-wave budget of kernels near 128 VGPRs). On ties, spreading takes the larger workgroup
// (more particle slots share one LDS tile), interpolation the smaller (two workgroups per
// compute unit overlap one's grid staging with the other's sums: 40 against 44 us on the
// water box), and at most `cap` threads. PSWFE_PARTICLE_THREADS overrides it (if that fits).
int particle_threads(int P, const std::function<size_t(int)>& lds_of, bool larger_on_ties, int cap = 1024) {
  int best = 256, best_waves = 0;
  const int tmax = std::min(cap, pswfe::particle_max_threads_host(P));
  for (int t = 256; t <= tmax; t *= 2) {
    const size_t lds = lds_of(t);
    if (lds > kLdsLimit) break;
    const int blocks = static_cast<int>(kLdsLimit / std::max<size_t>(lds, 1));
    const int waves = std::min(blocks * (t / 64), 16);
    if (waves > best_waves || (waves == best_waves && larger_on_ties)) {
      best = t;
      best_waves = waves;
    }
  }
  if (const char* env = std::getenv("PSWFE_PARTICLE_THREADS")) {
    const int t = std::atoi(env);
    if ((t == 256 || t == 512 || t == 1024) && t <= tmax && lds_of(t) <= kLdsLimit) best = t;
  }
  return best;
}

// Single systems: B = 8 (measured best on gfx950 for 64^3 and 128^3 grids with P = 12-18;
// spreading then runs on the matrix cores), reduced to give at least 4 tiles per dimension on
// small grids. Batches: B = 8 (measured best on a 256-system ensemble of 16^3-50^3 grids;
// many small systems fill the chip together). Both are then reduced until the LDS limits
// hold.
int choose_tile(int m, int P, int requested, int elem, int64_t n_batch) {
  int B = requested;
  if (B <= 0 && n_batch < 0) {
    if (const char* env = std::getenv("PSWFE_TILE")) B = std::atoi(env);
  }
  if (B <= 0) {
    if (n_batch < 0) {
      B = 8;
      while (B > 2 && (m + B - 1) / B < 4) --B;
    } else {
      B = 8;
    }
  }
  B = std::max(2, std::min(B, m));
  while (B > 2 && !tile_fits(B, P, elem)) --B;
  return B;
}

double fit_tolerance(double eps, int prec) { return std::max(0.01 * eps, prec == PSWFE_FP32 ? 5e-9 : 1e-15); }

// Relative accuracy of the residual polynomial G. The residual is exact up to rounding (it does
// not depend on eps), so this is set by the output precision: 1e-10 lies far below float32's
// unit roundoff of 6e-8 and lets float32 plans run about half the Horner steps.
double local_fit_tolerance(int prec) { return prec == PSWFE_FP32 ? 1e-10 : 1e-15; }

void free_timer(pswfe::StageTimer& t) {
  if (t.ev) {
    for (int i = 0; i < 2 * t.cap; ++i)
      if (t.ev[i]) (void)hipEventDestroy(t.ev[i]);
    delete[] t.ev;
  }
  t = pswfe::StageTimer();
}

void free_plan(pswfe_plan* plan) {
  if (plan->side) (void)hipStreamDestroy(plan->side);
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
  for (void* b : plan->allocs)
    if (b) (void)hipFree(b);
  plan->allocs.clear();
  delete plan;
}

pswfe_status params_from_c(const pswfe_params* pp, pswfe::Params* p) {
  const int m = pp->m, P = pp->P;
  const int my = pp->my > 0 ? pp->my : m, mz = pp->mz > 0 ? pp->mz : m;
  for (int md : {m, my, mz})
    if (!pswfe::is_smooth_even(md) || md < 8 || md > 512 || P > md) return PSWFE_E_GRID;
  if (pp->my < 0 || pp->mz < 0 || P < pswfe::kPmin || P > pswfe::kPmax) return PSWFE_E_GRID;
  if (pp->Ly < 0 || pp->Lz < 0 || !std::isfinite(pp->Ly) || !std::isfinite(pp->Lz)) return PSWFE_E_ARG;
  if (!(pp->L > 0) || !(pp->rc > 0) || !(pp->cs > 0) || !(pp->cw > 0) || !(pp->alpha > 0) || !(pp->eps > 0))
    return PSWFE_E_ARG;
  if (pp->split != PSWFE_SPLIT_PSWF && pp->split != PSWFE_SPLIT_GAUSS) return PSWFE_E_ARG;
  if (pp->window != PSWFE_WINDOW_PSWF && pp->window != PSWFE_WINDOW_GAUSS && pp->window != PSWFE_WINDOW_BSPLINE)
    return PSWFE_E_ARG;
  if (pp->window == PSWFE_WINDOW_GAUSS && !(pp->cg > 0)) return PSWFE_E_ARG;
  if (pp->cs > 40.0 || (pp->window == PSWFE_WINDOW_PSWF && pp->cw > 40.0)) return PSWFE_E_EPS_RANGE;
  // the window transform of Table 2 holds inside the window's band: alpha w <= c_w on the grid
  if (pp->window == PSWFE_WINDOW_PSWF && pp->cw < 0.5 * 3.14159265358979323846 * P * (1.0 - 1e-12))
    return PSWFE_E_ARG;
  p->split = pp->split;
  p->window = pp->window;
  p->cg = pp->cg;
  p->Ly = pp->Ly > 0 ? pp->Ly : pp->L;
  p->Lz = pp->Lz > 0 ? pp->Lz : pp->L;
  p->my = my;
  p->mz = mz;
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

// Byte layout of one arena: sub-buffers at 256-byte aligned offsets.
struct Arena {
  size_t size = 0;
  size_t take(size_t bytes) {
    const size_t off = size;
    size += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    return off;
  }
};

template <class T>
void put(std::vector<unsigned char>& img, size_t off, const std::vector<double>& v) {
  for (size_t i = 0; i < v.size(); ++i) {
    const T x = static_cast<T>(v[i]);
    std::memcpy(img.data() + off + i * sizeof(T), &x, sizeof(T));
  }
}

// Where a plan's device arena lives: allocated by the plan (base == nullptr) or at `base`, device
// memory of `capacity` bytes that the caller provides and keeps (no real-space residual buffers
// then; the constant part is uploaded by the caller of build_plan at compute time).
// With `external` and base == nullptr, build_plan only checks that the arena fits `capacity`
// (PSWFE_OK with *out = nullptr, or PSWFE_E_CAPACITY) and touches no device.
struct Placement {
  bool external = false;
  unsigned char* base = nullptr;
  size_t capacity = 0;
};

// Builds a plan over `ps.size()` systems. counts == NULL: single system taking up to n_max
// particles per call; otherwise a batch with counts[s] particles in system s.
pswfe_status build_plan(std::vector<pswfe::Params> ps, int prec, int64_t n_max, const int64_t* counts,
                        const int32_t* tiles, pswfe_plan** out, Placement place = Placement()) {
  // float32 arithmetic path: float32 storage, as PSWFE_FP32, with float32 particle arithmetic
  const bool arith32 = prec == PSWFE_FP32_ARITH;
  if (arith32) prec = PSWFE_FP32;
  const int nsys = static_cast<int>(ps.size());
  const int elem = prec == PSWFE_FP32 ? 4 : 8;
  const size_t celem = 2 * static_cast<size_t>(elem);
  pswfe_plan* plan = new (std::nothrow) pswfe_plan();
  if (!plan) return PSWFE_E_ALLOC;
  plan->batch = counts != nullptr;
  plan->p = ps;
  plan->tab.resize(nsys);
  plan->ltab.resize(nsys);
  (void)hipGetDevice(&plan->device);
  pswfe::DevPlan& d = plan->d;
  d.prec = prec;
  d.nsys = nsys;
  d.sys.resize(nsys);
  std::vector<int> xblk_prefix(nsys + 1, 0), cblk_prefix(nsys + 1, 0), pblk_prefix(nsys + 1, 0);
  std::vector<int> zblk_prefix(nsys + 1, 0), yzblk_prefix(nsys + 1, 0);
  // y and z passes fused per spectrum column (k_fft_yz) when every system's (y, z) plane, two
  // padded copies plus twiddles, fits in LDS and the columns of all systems give at least one
  // workgroup per compute unit (batches of small grids: 256 systems of 16^3-50^3, 206 -> 153 us;
  // a single 64^3 grid has 33 columns, and the three separate passes over 192 workgroups each
  // took 30 against 31 us). PSWFE_YZ_FFT=0 turns it off, =1 on wherever it fits.
  int yz_env = -1;
  if (const char* env = std::getenv("PSWFE_YZ_FFT")) yz_env = std::atoi(env) != 0 ? 1 : 0;
  bool yz_ok = yz_env != 0;
  // x and y FFTs fused per z-plane (PSWFE_PLANE_FFT=1) when every system's plane (two padded
  // copies of its half spectrum plus twiddles) fits in LDS. Off by default: measured on MI355X,
  // one workgroup per plane (64-128 of them) costs as much as the two separate passes it saves a
  // launch over (water box 64^3: 135.5 against 136.0 us per step in float32, 153.9 against 152.7
  // in float64; 128^3 float32: 3.6 us slower).
  bool plane_ok = false;
  if (const char* env = std::getenv("PSWFE_PLANE_FFT")) plane_ok = std::atoi(env) != 0;
  std::vector<int64_t> part_prefix(nsys + 1, 0);
  // complex values per FFT workgroup (measured on gfx950: 1024 on grids up to 96^3, 2048 above)
  int fft_env = 0;
  if (const char* env = std::getenv("PSWFE_FFT_ELEMS")) fft_env = std::max(64, std::min(8192, std::atoi(env)));
  // LDS per FFT workgroup (PSWFE_FFT_LDS_KIB overrides, up to 160). Larger blocks measured slower
  // on MI355X: 160 KiB with 4096 complex values per workgroup took the 216^3 float64 z pass from
  // 139 to 179 us and the water-box step from 138 to 150 us.
  size_t fft_lds_cap = 64 * 1024;
  if (const char* env = std::getenv("PSWFE_FFT_LDS_KIB"))
    fft_lds_cap = static_cast<size_t>(std::max(16, std::min(160, std::atoi(env)))) * 1024;
  Arena work, tabs;
  struct TabOff { size_t coef, tm, wk, wky, wkz, twhp, twhm, twfp, twfm, twyp, twym, twzp, twzm, lcoef, rpoly; };
  int cell_prefix = 0;
  std::vector<int> cell_prefix_v(nsys + 1, 0);
  struct WorkOff { size_t a, b, spec; };
  std::vector<TabOff> toff(nsys);
  std::vector<WorkOff> woff(nsys);
  for (int s = 0; s < nsys; ++s) {
    const pswfe::Params& p = ps[s];
    pswfe::Tables& t = plan->tab[s];
    pswfe::build_tables(p, 0, fit_tolerance(p.eps, prec), &t);
    if (p.split == pswfe::kSplitPswf) {
      pswfe::build_local_table(p, local_fit_tolerance(prec), &plan->ltab[s]);
      d.local_deg = std::max(d.local_deg, plan->ltab[s].deg);
    } else {
      plan->ltab[s].coef.assign(1, 0.0);  // no residual for the Gaussian split (never launched)
      plan->local_ok = false;
    }
    pswfe::SysDesc& sd = d.sys[s];
    const int m = p.m, N = m / 2, nx1 = N + 1, my = p.grid(1), mz = p.grid(2);
    const int mmin = std::min(m, std::min(my, mz)), mlen = std::max(my, mz);
    if (counts) {
      if (counts[s] < 0) {
        free_plan(plan);
        return PSWFE_E_ARG;
      }
      part_prefix[s + 1] = part_prefix[s] + counts[s];
      plan->count.push_back(counts[s]);
    }
    const int req = tiles ? tiles[s] : 0;
    if (req < 0 || req > mmin) {
      free_plan(plan);
      return PSWFE_E_ARG;
    }
    const int P = p.P;
    sd.m = m;
    sd.my = my;
    sd.mz = mz;
    sd.P = P;
    sd.deg = t.deg;
    sd.B = choose_tile(mmin, P, req, elem, counts ? counts[s] : -1);
    sd.Tn = (m + sd.B - 1) / sd.B;
    sd.Tny = (my + sd.B - 1) / sd.B;
    sd.Tnz = (mz + sd.B - 1) / sd.B;
    sd.S = lds_edge(sd.B, P);
    sd.L = p.side(0);
    sd.Ly = p.side(1);
    sd.Lz = p.side(2);
    // 1/h_d split into a high and a low word of the plan precision (exact product error)
    auto inv_spacing = [&](int md, double Ld, double* inv, double* hi_out, double* lo_out) {
      *inv = md / Ld;
      const long double ih = static_cast<long double>(md) / static_cast<long double>(Ld);
      if (prec == PSWFE_FP32) {
        const float hi = static_cast<float>(ih);
        *hi_out = hi;
        *lo_out = static_cast<float>(ih - static_cast<long double>(hi));
      } else {
        const double hi = static_cast<double>(ih);
        *hi_out = hi;
        *lo_out = static_cast<double>(ih - static_cast<long double>(hi));
      }
    };
    inv_spacing(m, sd.L, &sd.inv_h, &sd.ih_hi, &sd.ih_lo);
    inv_spacing(my, sd.Ly, &sd.inv_hy, &sd.ihy_hi, &sd.ihy_lo);
    inv_spacing(mz, sd.Lz, &sd.inv_hz, &sd.ihz_hi, &sd.ihz_lo);
    sd.self_coef = t.self_coef;
    sd.radial = t.radial;
    sd.rleg_n = t.radial == 1 ? static_cast<int>(t.rpoly.size()) - 1 : 0;
    sd.w2x = (2.0 * M_PI / sd.L) * (2.0 * M_PI / sd.L);
    sd.w2y = (2.0 * M_PI / sd.Ly) * (2.0 * M_PI / sd.Ly);
    sd.w2z = (2.0 * M_PI / sd.Lz) * (2.0 * M_PI / sd.Lz);
    sd.rscale = t.rscale;
    sd.rpref = t.rpref;
    sd.rband2 = t.rband2;
    sd.rsig2 = t.rsig2;
    sd.fh = make_fft_plan(N);
    sd.ff = make_fft_plan(m);
    sd.ffy = make_fft_plan(my);
    sd.ffz = make_fft_plan(mz);
    if (sd.fh.nst < 0 || sd.ff.nst < 0 || sd.ffy.nst < 0 || sd.ffz.nst < 0) {
      free_plan(plan);
      return PSWFE_E_GRID;
    }
    // FFT batching: about fft_elems complex values per workgroup, at most 64 KiB of LDS with
    // the twiddle tables.
    const int fft_elems = fft_env > 0 ? fft_env : (m <= 96 ? 1024 : 2048);
    int rpb = std::max(1, std::min(64, fft_elems / nx1));
    while (rpb > 1 && (2 * static_cast<size_t>(rpb) * nx1 + 2 * N + 1) * celem > fft_lds_cap) --rpb;
    int cmax = std::max(1, std::min(64, fft_elems / (mlen + 1)));
    while (cmax > 1 && (2 * static_cast<size_t>(cmax) * (mlen + 1) + 2 * mlen) * celem > fft_lds_cap) --cmax;
    // Spectrum rows padded to 128 bytes, and column blocks of whole 128-byte segments (16
    // float32 or 8 float64 complex values), so that a column pass reads each line once: blocks
    // of other widths start inside lines and read about twice the bytes (measured at 128^3).
    const int spec_align = static_cast<int>(128 / celem);
    sd.spec_pitch = (nx1 + spec_align - 1) / spec_align * spec_align;
    int cpb = cmax >= spec_align ? cmax / spec_align * spec_align : spec_align;
    while (cpb > 1 && (2 * static_cast<size_t>(cpb) * (mlen + 1) + 2 * mlen) * celem > fft_lds_cap)
      cpb = cpb > spec_align ? cpb - spec_align : cpb - 1;
    sd.rows_per_block = rpb;
    sd.cols_per_block = cpb;
    sd.xblk_base = xblk_prefix[s];
    sd.pblk_base = pblk_prefix[s];
    pblk_prefix[s + 1] = pblk_prefix[s] + m;
    {
      const size_t lds_plane = (2 * static_cast<size_t>(nx1) * (m + 1) + N + m) * celem;
      d.lds_p = std::max(d.lds_p, lds_plane);
      if (lds_plane > kLdsLimit || !p.cubic()) plane_ok = false;
    }
    sd.cblk_base = cblk_prefix[s];
    sd.zblk_base = zblk_prefix[s];
    sd.yzblk_base = yzblk_prefix[s];
    yzblk_prefix[s + 1] = yzblk_prefix[s] + nx1;
    {
      const size_t cap = std::max(static_cast<size_t>(mz) * (my + 1), static_cast<size_t>(my) * (mz + 1));
      const size_t lds_yz = (2 * cap + 2 * static_cast<size_t>(my + mz)) * celem;
      d.lds_yz = std::max(d.lds_yz, lds_yz);
      if (lds_yz > kYzLdsMax) yz_ok = false;
    }
    sd.part_base = part_prefix[s];
    const int ncb = (nx1 + sd.cols_per_block - 1) / sd.cols_per_block;
    xblk_prefix[s + 1] = xblk_prefix[s] + (my * mz + rpb - 1) / rpb;
    cblk_prefix[s + 1] = cblk_prefix[s] + ncb * mz;  // y passes: one row of blocks per z plane
    zblk_prefix[s + 1] = zblk_prefix[s] + ncb * my;  // z pass: one per y row
    // data buffers plus the twiddle tables the kernels copy into LDS
    d.lds_x = std::max(d.lds_x, (2 * static_cast<size_t>(rpb) * nx1 + 2 * N + 1) * celem);
    d.lds_c = std::max(d.lds_c, (2 * static_cast<size_t>(sd.cols_per_block) * (mlen + 1) + 2 * mlen) * celem);
    const size_t m3 = static_cast<size_t>(m) * my * mz;
    woff[s] = {work.take(sizeof(double) * m3), work.take(elem * m3),
               work.take(celem * static_cast<size_t>(mz) * my * sd.spec_pitch)};
    // real-space cells of edge L_d / nc_d >= r_c (at most 128 per dimension); one cell holding
    // the whole system when any dimension has fewer than 3
    sd.rc = p.rc;
    sd.lK = plan->ltab[s].K;
    sd.ldeg = plan->ltab[s].deg;
    sd.nc = std::max(1, std::min(128, static_cast<int>(std::floor(sd.L / p.rc))));
    sd.ncy = std::max(1, std::min(128, static_cast<int>(std::floor(sd.Ly / p.rc))));
    sd.ncz = std::max(1, std::min(128, static_cast<int>(std::floor(sd.Lz / p.rc))));
    if (sd.nc < 3 || sd.ncy < 3 || sd.ncz < 3) sd.nc = sd.ncy = sd.ncz = 1;
    sd.cell_base = cell_prefix;
    cell_prefix += sd.nc * sd.ncy * sd.ncz;
    cell_prefix_v[s + 1] = cell_prefix;
    if (!(p.rc < 0.5 * std::min(sd.L, std::min(sd.Ly, sd.Lz)))) plan->local_ok = false;
    toff[s] = {tabs.take(sizeof(double) * t.coef.size()), tabs.take(elem * t.tm.size()),
               tabs.take(elem * t.w.size()), tabs.take(elem * t.wy.size()), tabs.take(elem * t.wz.size()),
               tabs.take(celem * N), tabs.take(celem * N), tabs.take(celem * m), tabs.take(celem * m),
               tabs.take(celem * my), tabs.take(celem * my), tabs.take(celem * mz), tabs.take(celem * mz),
               tabs.take(sizeof(double) * plan->ltab[s].coef.size()),
               tabs.take(sizeof(double) * std::max<size_t>(1, t.rpoly.size()))};
  }
  // Global tile order: systems grouped by P (stable), so each P's tiles are one contiguous
  // range covered by one launch of the particle kernels.
  std::vector<int> order(nsys), tile_prefix(nsys + 1, 0);
  for (int s = 0; s < nsys; ++s) order[s] = s;
  // spreading in registers (matrix cores or y-columns) where the tile edge allows it
  // (PSWFE_SPREAD_COLUMNS=0 turns it off: LDS atomics for every edge)
  bool columns_ok = true;
  if (const char* env = std::getenv("PSWFE_SPREAD_COLUMNS")) columns_ok = std::atoi(env) != 0;
  auto cols = [&](int s) { return columns_ok && pswfe::col_tile_ok(d.sys[s].B) ? d.sys[s].B : 0; };
  auto key = [&](int s) { return std::make_tuple(d.sys[s].P, pswfe::degree_bucket(d.sys[s].deg), cols(s)); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
  std::vector<int64_t> group_particles;
  for (int k = 0; k < nsys; ++k) {
    pswfe::SysDesc& sd = d.sys[order[k]];
    const int D = pswfe::degree_bucket(sd.deg);
    sd.tile_base = tile_prefix[k];
    tile_prefix[k + 1] = tile_prefix[k] + sd.Tn * sd.Tny * sd.Tnz;
    if (d.groups.empty() || d.groups.back().P != sd.P || d.groups.back().D != D ||
        d.groups.back().col_tile != cols(order[k])) {
      pswfe::PGroup g;
      g.P = sd.P;
      g.D = D;
      g.col_tile = cols(order[k]);
      g.tile_begin = tile_prefix[k];
      d.groups.push_back(g);
      group_particles.push_back(0);
    }
    pswfe::PGroup& g = d.groups.back();
    g.tile_end = tile_prefix[k + 1];
    group_particles.back() += counts ? counts[order[k]] : n_max;
    g.lds_spread = std::max<size_t>(g.lds_spread, lds_edge(sd.B, sd.P));  // largest S of the group, for now
  }
  // Dense tiles are shared by several workgroups, each taking a slice of the tile's particles,
  // when a group has too few tiles to fill the GPU: up to about 1024 workgroups per launch, with
  // at least 32 particles (on average) per workgroup and at most 16 workgroups per tile.
  // PSWFE_TILE_PARTS overrides it.
  int parts_env = 0;
  if (const char* env = std::getenv("PSWFE_TILE_PARTS")) parts_env = std::max(1, std::min(16, std::atoi(env)));
  for (size_t gi = 0; gi < d.groups.size(); ++gi) {
    pswfe::PGroup& g = d.groups[gi];
    const int64_t tiles = g.tile_end - g.tile_begin;
    const int64_t per_tile = group_particles[gi] / std::max<int64_t>(tiles, 1);
    int64_t parts = 1;
    if (tiles < 1024) parts = std::min<int64_t>((1024 + tiles - 1) / tiles, std::max<int64_t>(1, per_tile / 32));
    g.parts = parts_env ? parts_env : static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(16, parts)));
  }
  // the matrix-core form rather than y-columns for the tile edges 4, 6, 8 (PSWFE_SPREAD_MFMA=0
  // turns it off)
  bool mfma_ok = true;
  if (const char* env = std::getenv("PSWFE_SPREAD_MFMA")) mfma_ok = std::atoi(env) != 0;
  for (pswfe::PGroup& g : d.groups) {
    const int S = static_cast<int>(g.lds_spread), P = g.P, D = g.D;
    g.mfma = g.col_tile && mfma_ok ? 1 : 0;
    // float32 window values, products and sums in spreading (matrix cores) and interpolation
    g.acc32 = arith32 ? 1 : 0;
    g.spread_threads = g.mfma       ? pswfe::mfma_threads_host(P, g.col_tile)
                       : g.col_tile ? pswfe::col_threads_host(P, g.col_tile)
                                    : particle_threads(P, [&](int t) { return spread_lds_bytes(S, P, D, t); }, true);
    const size_t gbytes = g.acc32 ? sizeof(float) : sizeof(double);
    // interpolation: at most 512 threads (1,024 measured slower on every workload: water box
    // float64 55.2 against 52.9 us, n = 1e6 float32 468 against 366 us)
    g.gather_threads =
        particle_threads(P, [&](int t) { return gather_lds_bytes(S, P, D, elem, t, gbytes); }, false, 512);
    g.lds_spread = g.mfma       ? pswfe::mfma_lds_bytes(P, D, g.col_tile, g.acc32 ? sizeof(float) : sizeof(double))
                   : g.col_tile ? pswfe::col_lds_bytes(P, D, g.col_tile)
                                : spread_lds_bytes(S, P, D, g.spread_threads);
    g.lds_gather = gather_lds_bytes(S, P, D, elem, g.gather_threads, gbytes);
  }
  // Matrix-core spreading by columns of tiles (float64 single systems with at least 2,048 tiles,
  // so that the columns still fill the GPU): each tile then adds B S^2 points to the grid instead
  // of S^3 (n = 1e6 float64: 2.30 -> 2.20 ms; float32 plans, whose flush is a small share,
  // measured slower: 410 -> 640 us). Segments per column: about 1,024 workgroups.
  // PSWFE_SPREAD_ROLL=0 turns it off, =1 turns it on wherever it applies (whole columns), =2 turns
  // it on with the automatic segments for any precision and tile count.
  {
    int roll_env = -1;
    if (const char* env = std::getenv("PSWFE_SPREAD_ROLL")) roll_env = std::max(0, std::min(2, std::atoi(env)));
    if (nsys == 1 && d.groups.size() == 1 && d.groups[0].mfma && d.groups[0].parts == 1 && roll_env != 0) {
      pswfe::PGroup& g = d.groups[0];
      const pswfe::SysDesc& sd = d.sys[0];
      const int cols = sd.Tn * sd.Tny, tiles = cols * sd.Tnz;
      const size_t lds = pswfe::mfma_roll_lds_bytes(g.P, g.D, g.col_tile, g.acc32 ? sizeof(float) : sizeof(double));
      if ((roll_env >= 1 || (tiles >= 2048 && prec == PSWFE_FP64)) && sd.Tnz >= 2 && lds <= kLdsLimit) {
        const int nseg0 = roll_env == 1 ? 1 : std::max(1, std::min(sd.Tnz, (1024 + cols - 1) / cols));
        const int len = (sd.Tnz + nseg0 - 1) / nseg0;
        if (len >= 2) {
          g.roll_cols = cols;
          g.roll_len = len;
          g.roll_nseg = (sd.Tnz + len - 1) / len;
          g.lds_spread = lds;
        }
      }
    }
  }
  d.total_tiles = tile_prefix[nsys];
  d.total_xblk = xblk_prefix[nsys];
  d.total_pblk = pblk_prefix[nsys];
  d.total_zblk = zblk_prefix[nsys];
  d.plane_fft = plane_ok ? 1 : 0;
  d.yz_fft = yz_ok && !plane_ok && (yz_env == 1 || yzblk_prefix[nsys] >= kYzMinBlocks) ? 1 : 0;
  // Interpolation by tile sequences (k_gather_stream) for float64 single systems with at least
  // 2,048 tiles (n = 1e6: 216^3 2.55 -> 2.50 ms, 128^3 1.88 -> 1.80 ms): PSWFE_GATHER_STREAM=0
  // turns it off, =1 on for any float64 single system.
  {
    int env = -1;
    if (const char* e = std::getenv("PSWFE_GATHER_STREAM")) env = std::atoi(e) != 0 ? 1 : 0;
    const int tiles = d.sys[0].Tn * d.sys[0].Tny * d.sys[0].Tnz;
    if (nsys == 1 && d.groups.size() == 1 && d.groups[0].parts == 1 && prec == PSWFE_FP64 &&
        (env == 1 || (env != 0 && tiles >= 2048)))
      d.groups[0].gather_stream = -1;
  }
  // Float32-arithmetic plans spread into a float32 grid (grid_a's bytes read as float32, summed
  // with float32 atomics) when every group spreads on the matrix cores and the grids hold at
  // least kGrid32MinPoints points in all: 256-system ensemble 1.16 -> 0.95 ms, n = 1e6 on 128^3
  // 430 -> 417 us; a single 64^3 grid (the water box) measured slower, 44 -> 47 us, its float32
  // atomics meeting twice as often in one cache line. PSWFE_GRID32=0 turns it off, =1 on
  // wherever it applies.
  {
    int env = -1;
    if (const char* e = std::getenv("PSWFE_GRID32")) env = std::atoi(e) != 0 ? 1 : 0;
    bool ok = arith32 && !plane_ok && env != 0;
    for (const pswfe::PGroup& g : d.groups) ok = ok && g.mfma && g.acc32;
    int64_t points = 0;
    for (const pswfe::SysDesc& sd : d.sys) points += static_cast<int64_t>(sd.m) * sd.my * sd.mz;
    d.grid32 = ok && (env == 1 || points >= kGrid32MinPoints) ? 1 : 0;
  }
  d.total_yzblk = yzblk_prefix[nsys];
  d.total_cblk = cblk_prefix[nsys];
  d.n_max = counts ? part_prefix[nsys] : n_max;
  if (d.n_max > (int64_t(1) << 31) - 1) {
    free_plan(plan);
    return PSWFE_E_ARG;
  }
  if (!counts) part_prefix[1] = 0;  // unused: one system takes every particle of a call

  // sub-buckets per tile: at least 8 particles each on average, at most 16 per tile and
  // 32768 buckets in all
  {
    const double per_tile = static_cast<double>(d.n_max) / std::max(d.total_tiles, 1);
    while (d.sub_log2 < 4 && 8.0 * (1 << d.sub_log2) <= per_tile &&
           (static_cast<int64_t>(d.total_tiles) << (d.sub_log2 + 1)) <= 32768)
      ++d.sub_log2;
  }
  const int64_t nbuckets = static_cast<int64_t>(d.total_tiles) << d.sub_log2;
  // two-level sort: the fewest buckets per coarse bucket (a power of two) that leave at most
  // kCoarse coarse buckets; particles per thread so that about 512 workgroups share the passes
  while (((nbuckets + (int64_t(1) << d.bin_shift) - 1) >> d.bin_shift) > pswfe::kCoarse) ++d.bin_shift;
  d.bin_ncoarse = static_cast<int>((nbuckets + (int64_t(1) << d.bin_shift) - 1) >> d.bin_shift);
  if ((1 << d.bin_shift) > pswfe::kBinMaxFine) {
    free_plan(plan);
    return PSWFE_E_GRID;
  }
  // the one-level sort below 200,000 particles (PSWFE_BIN_LEVELS=1 or 2 overrides)
  d.bin_levels = d.n_max < 200000 ? 1 : 2;
  if (const char* env = std::getenv("PSWFE_BIN_LEVELS")) {
    const int v = std::atoi(env);
    if (v == 1 || v == 2) d.bin_levels = v;
  }
  d.bin_per_thread = static_cast<int>(std::min<int64_t>(
      pswfe::kBinMaxPerThread, std::max<int64_t>(1, (d.n_max + 256 * 512 - 1) / (256 * 512))));
  const size_t nm = static_cast<size_t>(std::max<int64_t>(d.n_max, 1));
  d.total_cells = cell_prefix;
  // residual workgroup size: 512 threads (PSWFE_LOCAL_THREADS=128 or 256 overrides)
  d.local_threads = 512;
  if (const char* env = std::getenv("PSWFE_LOCAL_THREADS")) {
    const int v = std::atoi(env);
    if (v == 128 || v == 256) d.local_threads = v;
  }
  const bool with_local = !place.external;  // the residual's buffers: plans that own memory only
  if (with_local && plan->local_ok) {
    if (const char* env = std::getenv("PSWFE_LOCAL_OVERLAP")) plan->overlap = std::atoi(env) != 0;
  } else {
    plan->overlap = false;
  }
  if (!with_local) plan->local_ok = false;

  // Every device buffer of the plan lives in one arena: first the constant part (tables,
  // descriptors, prefix tables), uploaded from a host image; then the work grids and the
  // particle bins. grid_a and the counters must start at zero (kept zero between calls).
  Arena dev;
  const size_t o_tab = dev.take(tabs.size);
  const size_t o_sys = dev.take(sizeof(pswfe::SysDesc) * nsys);
  const size_t o_tile_prefix = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_tile_sys = dev.take(sizeof(int) * nsys);
  const size_t o_cell_prefix = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_xblk = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_pblk = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_zblk = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_yzblk = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_cblk = dev.take(sizeof(int) * (nsys + 1));
  const size_t o_part = dev.take(sizeof(int64_t) * (nsys + 1));
  const size_t const_end = dev.size;
  const size_t o_work = dev.take(work.size);
  // coarse counts and cursors (kCoarseCopies copies each), then the coarse starts
  const size_t o_coarse = dev.take(sizeof(int) * (2 * pswfe::kCoarseCopies * pswfe::kCoarse + pswfe::kCoarse + 1));
  const size_t o_tile_count = dev.take(sizeof(int) * nbuckets);
  const size_t o_tile_start = dev.take(sizeof(int) * (nbuckets + 1));
  const size_t o_tile_of = dev.take(sizeof(int) * nm);
  // the two-level sort's staging copy of the records (one-level plans use none)
  const size_t o_bin_tmp = d.bin_levels == 2 ? dev.take(4 * static_cast<size_t>(elem) * nm) : 0;
  const size_t o_bin_tmp_ib = dev.take(sizeof(int2) * nm);
  const size_t o_perm = dev.take(sizeof(int) * nm);
  const size_t o_cells = dev.take(sizeof(int) * nm);
  const size_t o_sorted = dev.take(4 * static_cast<size_t>(elem) * nm);
  const size_t o_check = dev.take(sizeof(double) * 3 * nsys);
  size_t o_cell_count = 0, o_cell_start = 0, o_cell_of = 0, o_cell_rank = 0, o_lsorted = 0, o_lperm = 0;
  size_t o_phi_d = 0, o_vec_d = 0;
  if (with_local) {
    o_cell_count = dev.take(sizeof(int) * d.total_cells);
    o_cell_start = dev.take(sizeof(int) * (d.total_cells + 1));
    o_cell_of = dev.take(sizeof(int) * nm);
    o_cell_rank = dev.take(sizeof(int) * nm);
    o_lsorted = dev.take(sizeof(double) * 4 * nm);
    o_lperm = dev.take(sizeof(int) * nm);
    if (plan->overlap) {
      o_phi_d = dev.take(sizeof(double) * nm);
      o_vec_d = dev.take(sizeof(double) * 3 * nm);
    }
  }
  plan->arena_bytes = dev.size;
  unsigned char* base = place.base;
  if (place.external) {
    const bool fits = dev.size <= place.capacity;
    if (!fits || !base) {
      free_plan(plan);
      return fits ? PSWFE_OK : PSWFE_E_CAPACITY;
    }
  } else {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, dev.size) != hipSuccess) {
      free_plan(plan);
      return PSWFE_E_ALLOC;
    }
    plan->allocs.push_back(ptr);
    base = static_cast<unsigned char*>(ptr);
  }
  unsigned char* work_dev = base + o_work;
  unsigned char* tab_dev = base + o_tab;
  d.sys_dev = reinterpret_cast<pswfe::SysDesc*>(base + o_sys);
  d.tile_prefix = reinterpret_cast<int*>(base + o_tile_prefix);
  d.tile_sys = reinterpret_cast<int*>(base + o_tile_sys);
  d.cell_prefix = reinterpret_cast<int*>(base + o_cell_prefix);
  d.xblk_prefix = reinterpret_cast<int*>(base + o_xblk);
  d.pblk_prefix = reinterpret_cast<int*>(base + o_pblk);
  d.zblk_prefix = reinterpret_cast<int*>(base + o_zblk);
  d.yzblk_prefix = reinterpret_cast<int*>(base + o_yzblk);
  d.cblk_prefix = reinterpret_cast<int*>(base + o_cblk);
  d.part_prefix = reinterpret_cast<int64_t*>(base + o_part);
  d.coarse_count = reinterpret_cast<int*>(base + o_coarse);
  d.coarse_cursor = d.coarse_count + pswfe::kCoarseCopies * pswfe::kCoarse;
  d.coarse_start = d.coarse_cursor + pswfe::kCoarseCopies * pswfe::kCoarse;
  d.tile_start = reinterpret_cast<int*>(base + o_tile_start);
  d.tile_of = reinterpret_cast<int*>(base + o_tile_of);
  d.bin_tmp = d.bin_levels == 2 ? base + o_bin_tmp : nullptr;
  d.bin_tmp_ib = reinterpret_cast<int2*>(base + o_bin_tmp_ib);
  d.bin_rank = reinterpret_cast<int*>(base + o_bin_tmp_ib);
  d.tile_count = reinterpret_cast<int*>(base + o_tile_count);
  d.perm = reinterpret_cast<int*>(base + o_perm);
  d.cells = reinterpret_cast<int*>(base + o_cells);
  d.sorted = base + o_sorted;
  d.check = reinterpret_cast<double*>(base + o_check);
  if (with_local) {
    d.cell_count = reinterpret_cast<int*>(base + o_cell_count);
    d.cell_start = reinterpret_cast<int*>(base + o_cell_start);
    d.cell_of = reinterpret_cast<int*>(base + o_cell_of);
    d.cell_rank = reinterpret_cast<int*>(base + o_cell_rank);
    d.lsorted = reinterpret_cast<double*>(base + o_lsorted);
    d.lperm = reinterpret_cast<int*>(base + o_lperm);
    if (plan->overlap) {
      plan->phi_d = reinterpret_cast<double*>(base + o_phi_d);
      plan->vec_d = reinterpret_cast<double*>(base + o_vec_d);
    }
  }
  // host image of the constant part: tables, then descriptors (with the arena's device
  // addresses) and prefix tables
  std::vector<unsigned char> img(const_end, 0);
  for (int s = 0; s < nsys; ++s) {
    pswfe::SysDesc& sd = d.sys[s];
    const pswfe::Tables& t = plan->tab[s];
    const int m = sd.m, N = m / 2;
    sd.grid_a = reinterpret_cast<double*>(work_dev + woff[s].a);
    sd.grid_b = work_dev + woff[s].b;
    sd.spec = work_dev + woff[s].spec;
    sd.coef = reinterpret_cast<const double*>(tab_dev + toff[s].coef);
    sd.tm = tab_dev + toff[s].tm;
    sd.wk = tab_dev + toff[s].wk;
    sd.wky = tab_dev + toff[s].wky;
    sd.wkz = tab_dev + toff[s].wkz;
    sd.twhp = tab_dev + toff[s].twhp;
    sd.twhm = tab_dev + toff[s].twhm;
    sd.twfp = tab_dev + toff[s].twfp;
    sd.twfm = tab_dev + toff[s].twfm;
    sd.twyp = tab_dev + toff[s].twyp;
    sd.twym = tab_dev + toff[s].twym;
    sd.twzp = tab_dev + toff[s].twzp;
    sd.twzm = tab_dev + toff[s].twzm;
    sd.lcoef = reinterpret_cast<const double*>(tab_dev + toff[s].lcoef);
    sd.rleg = reinterpret_cast<const double*>(tab_dev + toff[s].rpoly);
    const size_t T0 = o_tab;
    put<double>(img, T0 + toff[s].lcoef, plan->ltab[s].coef);
    put<double>(img, T0 + toff[s].rpoly, t.rpoly.empty() ? std::vector<double>(1, 0.0) : t.rpoly);
    std::vector<double> twhp, twhm, twfp, twfm, twyp, twym, twzp, twzm;
    pswfe::twiddles(N, +1, &twhp);
    pswfe::twiddles(N, -1, &twhm);
    pswfe::twiddles(m, +1, &twfp);
    pswfe::twiddles(m, -1, &twfm);
    pswfe::twiddles(sd.my, +1, &twyp);
    pswfe::twiddles(sd.my, -1, &twym);
    pswfe::twiddles(sd.mz, +1, &twzp);
    pswfe::twiddles(sd.mz, -1, &twzm);
    put<double>(img, T0 + toff[s].coef, t.coef);  // window polynomials: float64 in both precisions
    auto put_real = [&](size_t off, const std::vector<double>& v) {
      if (prec == PSWFE_FP32)
        put<float>(img, T0 + off, v);
      else
        put<double>(img, T0 + off, v);
    };
    put_real(toff[s].tm, t.tm);
    put_real(toff[s].wk, t.w);
    put_real(toff[s].wky, t.wy);
    put_real(toff[s].wkz, t.wz);
    put_real(toff[s].twhp, twhp);
    put_real(toff[s].twhm, twhm);
    put_real(toff[s].twfp, twfp);
    put_real(toff[s].twfm, twfm);
    put_real(toff[s].twyp, twyp);
    put_real(toff[s].twym, twym);
    put_real(toff[s].twzp, twzp);
    put_real(toff[s].twzm, twzm);
  }
  auto put_bytes = [&](size_t off, const void* src, size_t bytes) { std::memcpy(img.data() + off, src, bytes); };
  put_bytes(o_sys, d.sys.data(), sizeof(pswfe::SysDesc) * nsys);
  put_bytes(o_tile_prefix, tile_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_tile_sys, order.data(), sizeof(int) * nsys);
  put_bytes(o_cell_prefix, cell_prefix_v.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_xblk, xblk_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_pblk, pblk_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_zblk, zblk_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_yzblk, yzblk_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_cblk, cblk_prefix.data(), sizeof(int) * (nsys + 1));
  put_bytes(o_part, part_prefix.data(), sizeof(int64_t) * (nsys + 1));
  // ranges that must start at zero: each system's grid_a and the bin counters
  for (int s = 0; s < nsys; ++s)
    plan->zero.push_back({o_work + woff[s].a, sizeof(double) * static_cast<size_t>(d.sys[s].m) * d.sys[s].my *
                                                  d.sys[s].mz});
  plan->zero.push_back({o_coarse, sizeof(int) * 2 * static_cast<size_t>(pswfe::kCoarseCopies * pswfe::kCoarse)});
  plan->zero.push_back({o_tile_count, sizeof(int) * static_cast<size_t>(nbuckets)});
  if (with_local) plan->zero.push_back({o_cell_count, sizeof(int) * static_cast<size_t>(d.total_cells)});
  plan->base = base;
  if (place.external) {
    // a plan in caller-provided memory keeps its image for uploads at compute time
    plan->img = std::move(img);
    if (pswfe::prepare_kernels(d) != hipSuccess) {
      free_plan(plan);
      return PSWFE_E_HIP;
    }
    *out = plan;
    return PSWFE_OK;
  }
  bool ok = hipMemcpy(base, img.data(), img.size(), hipMemcpyHostToDevice) == hipSuccess;
  for (const auto& z : plan->zero) ok = ok && hipMemset(base + z.first, 0, z.second) == hipSuccess;
  ok = ok && pswfe::prepare_kernels(d) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (ok && plan->overlap) {
    // default priority (a stream of another priority is never used here)
    ok = hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&plan->ev_join, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    free_plan(plan);
    return PSWFE_E_HIP;
  }
  *out = plan;
  return PSWFE_OK;
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
    case PSWFE_E_NONNEUTRAL: return "charges do not sum to zero";
    case PSWFE_E_NONFINITE: return "a position or charge is not finite";
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

pswfe_status pswfe_choose_params_box(double eps, double Lx, double Ly, double Lz, double rc, int32_t m, int64_t n,
                                     double q_l2, int32_t tol_mode, pswfe_params* out) {
  if (!out) return PSWFE_E_ARG;
  pswfe::Params p{};
  const int rcode = pswfe::choose_params_box(eps, Lx, Ly, Lz, rc, m, n, q_l2, tol_mode, &p);
  if (rcode != 0) return static_cast<pswfe_status>(rcode);
  to_c(p, out);
  return PSWFE_OK;
}

pswfe_status pswfe_oversample_params(const pswfe_params* base, double sigma, pswfe_params* out) {
  if (!base || !out) return PSWFE_E_ARG;
  pswfe::Params b{};
  const pswfe_status st = params_from_c(base, &b);
  if (st != PSWFE_OK) return st;
  pswfe::Params p{};
  const int rcode = pswfe::oversample_params(b, sigma, &p);
  if (rcode == 3) return PSWFE_E_GRID;
  if (rcode != 0) return PSWFE_E_ARG;
  if (p.cw > 40.0) return PSWFE_E_EPS_RANGE;
  to_c(p, out);
  return PSWFE_OK;
}

pswfe_status pswfe_variant_params(int32_t split, int32_t window, double L, double rc, double cs, int32_t m,
                                  int32_t P, double cg, double eps, pswfe_params* out) {
  if (!out) return PSWFE_E_ARG;
  if (split != PSWFE_SPLIT_PSWF && split != PSWFE_SPLIT_GAUSS) return PSWFE_E_ARG;
  if (window != PSWFE_WINDOW_PSWF && window != PSWFE_WINDOW_GAUSS && window != PSWFE_WINDOW_BSPLINE)
    return PSWFE_E_ARG;
  if (!(L > 0) || !std::isfinite(L) || !(rc > 0) || !(rc < 0.5 * L) || !(cs > 0)) return PSWFE_E_ARG;
  if (!pswfe::is_smooth_even(m) || m < 8 || m > 512 || P < pswfe::kPmin || P > pswfe::kPmax || P > m)
    return PSWFE_E_GRID;
  if (cs > 40.0 || !(eps >= 1e-14 && eps <= 0.1)) return PSWFE_E_EPS_RANGE;
  pswfe::Params p{};
  p.L = L;
  p.eps = eps;
  p.rc = rc;
  p.cs = cs;
  p.m = m;
  p.P = P;
  p.h = L / m;
  p.alpha = 0.5 * P * p.h;
  p.cw = 0.5 * 3.14159265358979323846 * P;
  p.cs_alg = p.cs;
  p.cw_alg = p.cw;
  p.alpha_alg = p.alpha;
  p.tol_mode = PSWFE_TOL_REL;
  p.lambda0_s = pswfe::Pswf(cs).lambda0;
  p.split = split;
  p.window = window;
  p.cg = window == PSWFE_WINDOW_GAUSS ? (cg > 0 ? cg : pswfe::default_gauss_shape(P)) : 0.0;
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

pswfe_status pswfe_host_tables(const pswfe_params* pp, int32_t prec, double* tm, int64_t tm_len, double* w,
                               int64_t w_len, double* coef, int64_t coef_len, double* info) {
  if (!pp) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64 && prec != PSWFE_FP32_ARITH) return PSWFE_E_PREC;
  pswfe::Params p{};
  const pswfe_status st = params_from_c(pp, &p);
  if (st != PSWFE_OK) return st;
  pswfe::Tables t;
  pswfe::build_tables(p, 0, fit_tolerance(p.eps, prec == PSWFE_FP32_ARITH ? PSWFE_FP32 : prec), &t);
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
  to_c(plan->p[0], out);
  return PSWFE_OK;
}

int32_t pswfe_plan_tile(const pswfe_plan* plan) { return plan ? plan->d.sys[0].B : 0; }

int32_t pswfe_plan_num_systems(const pswfe_plan* plan) { return plan ? plan->d.nsys : 0; }

pswfe_status pswfe_plan_system(const pswfe_plan* plan, int32_t s, pswfe_params* params, int64_t* offset,
                               int64_t* count, int32_t* tile) {
  if (!plan || s < 0 || s >= plan->d.nsys) return PSWFE_E_ARG;
  if (params) to_c(plan->p[s], params);
  if (offset) *offset = plan->batch ? plan->d.sys[s].part_base : 0;
  if (count) *count = plan->batch ? plan->count[s] : plan->d.n_max;
  if (tile) *tile = plan->d.sys[s].B;
  return PSWFE_OK;
}

pswfe_status pswfe_plan_create(const pswfe_params* pp, int32_t prec, int64_t n_max, pswfe_plan** out) {
  return pswfe_plan_create_tiled(pp, prec, n_max, 0, out);
}

pswfe_status pswfe_plan_create_tiled(const pswfe_params* pp, int32_t prec, int64_t n_max, int32_t tile,
                                     pswfe_plan** out) {
  if (!out) return PSWFE_E_ARG;
  *out = nullptr;
  if (!pp || n_max < 0 || n_max > (int64_t(1) << 31) - 1) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64 && prec != PSWFE_FP32_ARITH) return PSWFE_E_PREC;
  std::vector<pswfe::Params> ps(1);
  const pswfe_status st = params_from_c(pp, &ps[0]);
  if (st != PSWFE_OK) return st;
  return build_plan(ps, prec, n_max, nullptr, &tile, out);
}

pswfe_status pswfe_batch_plan_create(int32_t nsys, const pswfe_params* params, const int64_t* counts, int32_t prec,
                                     const int32_t* tiles, pswfe_plan** out) {
  if (!out) return PSWFE_E_ARG;
  *out = nullptr;
  if (nsys < 1 || nsys > (1 << 20) || !params || !counts) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64 && prec != PSWFE_FP32_ARITH) return PSWFE_E_PREC;
  std::vector<pswfe::Params> ps(nsys);
  int64_t total = 0;
  for (int s = 0; s < nsys; ++s) {
    const pswfe_status st = params_from_c(&params[s], &ps[s]);
    if (st != PSWFE_OK) return st;
    if (counts[s] < 0 || (tiles && (tiles[s] < 0 || tiles[s] > ps[s].m))) return PSWFE_E_ARG;
    total += counts[s];
    if (total > (int64_t(1) << 31) - 1) return PSWFE_E_ARG;
  }
  return build_plan(ps, prec, 0, counts, tiles, out);
}

pswfe_status pswfe_plan_destroy(pswfe_plan* plan) {
  if (!plan) return PSWFE_OK;
  (void)hipDeviceSynchronize();
  free_timer(plan->timer);
  free_plan(plan);
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
// Bin, spread, transform and gather over every system of the plan; n particles in all; with
// `total`, the real-space residual is added: computed on the plan's side stream while the
// long-range part runs, and added by the interpolation (or, without the side stream, computed
// after it and accumulated).
hipError_t run_pipeline(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                        int vec_mode, double* energy, bool total, hipStream_t s) {
  const pswfe::DevPlan& d = plan->d;
  const bool fork = total && n > 0 && plan->side;
  pswfe::stage_begin(d, pswfe::kStageAll, s);
  hipError_t e = hipSuccess;
  bool forked = false;  // the side stream waits on the caller's: it must be joined back, whatever fails
  if (fork) {
    e = hipEventRecord(plan->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->side, plan->ev_fork, 0);
    forked = e == hipSuccess;
    if (e == hipSuccess)
      e = pswfe::launch_local(d, n, pos, q, nullptr, nullptr, vec_mode, nullptr, false, plan->side, plan->phi_d,
                              vec ? plan->vec_d : nullptr);
  }
  if (e == hipSuccess) e = pswfe::launch_bin(d, n, pos, q, energy, s);
  if (e == hipSuccess) e = pswfe::launch_spread(d, s);
  if (e == hipSuccess) e = pswfe::launch_transform(d, nullptr, nullptr, s);
  if (forked) {
    // join before returning, also after a failed launch, keeping the first error: the residual
    // reads the caller's inputs and writes plan scratch, and a capture must not end unjoined
    hipError_t j = hipEventRecord(plan->ev_join, plan->side);
    if (j == hipSuccess) j = hipStreamWaitEvent(s, plan->ev_join, 0);
    if (e == hipSuccess) e = j;
  }
  if (e == hipSuccess && n > 0)
    e = pswfe::launch_gather(d, nullptr, phi, vec, vec_mode, true, energy, s, fork ? plan->phi_d : nullptr,
                             fork && vec ? plan->vec_d : nullptr);
  if (e == hipSuccess && total && !fork) e = pswfe::launch_local(d, n, pos, q, phi, vec, vec_mode, energy, true, s);
  pswfe::stage_end(d, pswfe::kStageAll, s);
  return e;
}

constexpr int32_t kKnownFlags = PSWFE_VEC_GRAD | PSWFE_TOTAL | PSWFE_CHECK_INPUT;

// Relative charge imbalance above which PSWFE_CHECK_INPUT reports a system as non-neutral.
constexpr double kNeutralTol = 1e-6;

// PSWFE_CHECK_INPUT: per-system charge sums and non-finite counts on the device, read back with
// a synchronisation of `s` (refused while `s` is being captured).
pswfe_status check_input(pswfe_plan* plan, int64_t n, const void* pos, const void* q, hipStream_t s) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return PSWFE_E_HIP;
  if (cap != hipStreamCaptureStatusNone) return PSWFE_E_ARG;
  const pswfe::DevPlan& d = plan->d;
  std::vector<double> h(3 * static_cast<size_t>(d.nsys), 0.0);
  hipError_t e = pswfe::launch_check(d, n, pos, q, d.check, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d.check, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PSWFE_E_HIP;
  for (int k = 0; k < d.nsys; ++k)
    if (h[3 * k + 2] > 0.0) return PSWFE_E_NONFINITE;
  for (int k = 0; k < d.nsys; ++k)
    if (std::fabs(h[3 * k]) > kNeutralTol * h[3 * k + 1]) return PSWFE_E_NONNEUTRAL;
  return PSWFE_OK;
}

pswfe_status compute_impl(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                          int32_t flags, double* energy, void* stream) {
  if (!plan || plan->batch || n < 0 || (flags & ~kKnownFlags)) return PSWFE_E_ARG;
  if ((flags & PSWFE_TOTAL) && !plan->local_ok) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  if (flags & PSWFE_CHECK_INPUT) {
    const pswfe_status c = check_input(plan, n, pos, q, static_cast<hipStream_t>(stream));
    if (c != PSWFE_OK) return c;
  }
  return from_hip(run_pipeline(plan, n, pos, q, phi, vec, (flags & PSWFE_VEC_GRAD) ? 1 : 0, energy,
                               (flags & PSWFE_TOTAL) != 0, static_cast<hipStream_t>(stream)));
}

pswfe_status batch_impl(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* vec, int32_t flags,
                        double* energy, void* stream) {
  if (!plan || !plan->batch || (flags & ~kKnownFlags)) return PSWFE_E_ARG;
  if ((flags & PSWFE_TOTAL) && !plan->local_ok) return PSWFE_E_ARG;
  const int64_t n = plan->d.n_max;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  if (flags & PSWFE_CHECK_INPUT) {
    const pswfe_status c = check_input(plan, n, pos, q, static_cast<hipStream_t>(stream));
    if (c != PSWFE_OK) return c;
  }
  return from_hip(run_pipeline(plan, n, pos, q, phi, vec, (flags & PSWFE_VEC_GRAD) ? 1 : 0, energy,
                               (flags & PSWFE_TOTAL) != 0, static_cast<hipStream_t>(stream)));
}
}  // namespace

pswfe_status pswfe_compute(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* force,
                           double* energy, void* stream) {
  return compute_impl(plan, n, pos, q, phi, force, 0, energy, stream);
}

pswfe_status pswfe_compute_grad(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* grad,
                                double* energy, void* stream) {
  return compute_impl(plan, n, pos, q, phi, grad, PSWFE_VEC_GRAD, energy, stream);
}

pswfe_status pswfe_compute_ex(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                              double* energy, int32_t flags, void* stream) {
  return compute_impl(plan, n, pos, q, phi, vec, flags, energy, stream);
}

pswfe_status pswfe_batch_compute(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* force,
                                 double* energy, void* stream) {
  return batch_impl(plan, pos, q, phi, force, 0, energy, stream);
}

pswfe_status pswfe_batch_compute_grad(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* grad,
                                      double* energy, void* stream) {
  return batch_impl(plan, pos, q, phi, grad, PSWFE_VEC_GRAD, energy, stream);
}

pswfe_status pswfe_batch_compute_ex(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* vec,
                                    double* energy, int32_t flags, void* stream) {
  return batch_impl(plan, pos, q, phi, vec, flags, energy, stream);
}

pswfe_status pswfe_local(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                         double* energy, int32_t flags, void* stream) {
  if (!plan || n < 0 || (flags & ~PSWFE_VEC_GRAD) || !plan->local_ok) return PSWFE_E_ARG;
  if (plan->batch ? n != plan->d.n_max : n > plan->d.n_max) return plan->batch ? PSWFE_E_ARG : PSWFE_E_CAPACITY;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  return from_hip(pswfe::launch_local(plan->d, n, pos, q, phi, vec, (flags & PSWFE_VEC_GRAD) ? 1 : 0, energy, false,
                                      static_cast<hipStream_t>(stream)));
}

pswfe_status pswfe_host_local(const pswfe_params* pp, int64_t count, const double* r, double* R, double* dRr,
                              double* info) {
  if (!pp || count < 0 || (count > 0 && !r)) return PSWFE_E_ARG;
  pswfe::Params p{};
  const pswfe_status st = params_from_c(pp, &p);
  if (st != PSWFE_OK) return st;
  if (p.split != pswfe::kSplitPswf) return PSWFE_E_ARG;
  pswfe::LocalTable t;
  pswfe::build_local_table(p, local_fit_tolerance(PSWFE_FP64), &t);
  for (int64_t i = 0; i < count; ++i) {
    const double ri = r[i];
    double Ri = 0.0, dRi = 0.0;
    if (ri > 0.0 && ri < p.rc) {
      const double g = ri * ri / (p.rc * p.rc) - 0.5;
      double G = t.coef[t.deg], dG = 0.0;
      for (int k = t.deg - 1; k >= 0; --k) {
        dG = dG * g + G;
        G = G * g + t.coef[k];
      }
      Ri = 1.0 / ri - t.K * G;
      dRi = -1.0 / (ri * ri * ri) - 2.0 * t.K / (p.rc * p.rc) * dG;
    }
    if (R) R[i] = Ri;
    if (dRr) dRr[i] = dRi;
  }
  if (info) {
    info[0] = t.deg;
    info[1] = t.fit_err;
    info[2] = t.K;
  }
  return PSWFE_OK;
}

namespace {
// pswfe_compute_noalloc: per device, the scratch array's device address and the configuration
// whose constant part it holds; and a few host-side plans bound to the scratch array, one per
// (parameters, precision, n, device), reused by later calls of that configuration.
constexpr int kNoAllocDevices = 64;
constexpr int kNoAllocSlots = 8;
struct NoAllocDevice {
  unsigned char* ptr = nullptr;
  const pswfe_plan* resident = nullptr;
};
struct NoAllocSlot {
  pswfe_params key{};
  int32_t prec = -1;
  int64_t n = -1;
  int device = -1;
  pswfe_plan* plan = nullptr;
  uint64_t used = 0;
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc_dev[kNoAllocDevices];
NoAllocSlot g_noalloc_slot[kNoAllocSlots];
uint64_t g_noalloc_clock = 0;

// Device address of the scratch array on `device` (current), taken once.
hipError_t noalloc_scratch(int device, unsigned char** out) {
  NoAllocDevice& dv = g_noalloc_dev[device];
  if (!dv.ptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    dv.ptr = static_cast<unsigned char*>(ptr);
  }
  *out = dv.ptr;
  return hipSuccess;
}
}  // namespace

pswfe_status pswfe_compute_noalloc(const pswfe_params* pp, int32_t prec, int64_t n, const void* pos, const void* q,
                                   void* phi, void* force, double* energy, void* stream) {
  if (!pp || n < 0 || n > (int64_t(1) << 31) - 1 || (n > 0 && (!pos || !q))) return PSWFE_E_ARG;
  if (prec != PSWFE_FP32 && prec != PSWFE_FP64 && prec != PSWFE_FP32_ARITH) return PSWFE_E_PREC;
  std::vector<pswfe::Params> ps(1);
  {
    const pswfe_status st = params_from_c(pp, &ps[0]);
    if (st != PSWFE_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) device = -1;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocSlot* slot = nullptr;
  for (NoAllocSlot& c : g_noalloc_slot)
    if (c.plan && c.device == device && c.prec == prec && c.n == n && std::memcmp(&c.key, pp, sizeof(*pp)) == 0)
      slot = &c;
  if (!slot) {
    // the layout's size is checked before any device call; the scratch address is taken only
    // for a configuration that fits
    pswfe_plan* plan = nullptr;
    Placement place;
    place.external = true;
    place.capacity = kNoAllocBytes;
    pswfe_status st = build_plan(ps, prec, n, nullptr, nullptr, &plan, place);
    if (st != PSWFE_OK) return st;
    if (device < 0 || device >= kNoAllocDevices) return PSWFE_E_HIP;
    if (noalloc_scratch(device, &place.base) != hipSuccess) return PSWFE_E_HIP;
    st = build_plan(ps, prec, n, nullptr, nullptr, &plan, place);
    if (st != PSWFE_OK) return st;
    slot = &g_noalloc_slot[0];
    for (NoAllocSlot& c : g_noalloc_slot)
      if (!c.plan || c.used < slot->used) slot = &c;
    if (slot->plan) {
      // the evicted plan's tables may be the scratch array's current contents
      (void)hipDeviceSynchronize();
      for (NoAllocDevice& dv : g_noalloc_dev)
        if (dv.resident == slot->plan) dv.resident = nullptr;
      free_plan(slot->plan);
    }
    slot->key = *pp;
    slot->prec = prec;
    slot->n = n;
    slot->device = device;
    slot->plan = plan;
  }
  slot->used = ++g_noalloc_clock;
  pswfe_plan* plan = slot->plan;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return PSWFE_E_HIP;
  if (cap != hipStreamCaptureStatusNone) return PSWFE_E_ARG;  // the upload below reads host memory
  NoAllocDevice& dv = g_noalloc_dev[device];
  hipError_t e = hipSuccess;
  if (dv.resident != plan) {
    e = hipMemcpyAsync(plan->base, plan->img.data(), plan->img.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) dv.resident = plan;
  }
  for (size_t k = 0; k < plan->zero.size() && e == hipSuccess; ++k)
    e = pswfe::launch_zero(plan->base + plan->zero[k].first, plan->zero[k].second, s);
  if (e == hipSuccess) e = run_pipeline(plan, n, pos, q, phi, force, 0, energy, false, s);
  return from_hip(e);
}

pswfe_status pswfe_spread(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* grid, void* stream) {
  if (!plan || plan->batch || n < 0 || !grid) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && (!pos || !q)) return PSWFE_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const pswfe::DevPlan& d = plan->d;
  hipError_t e = pswfe::launch_bin(d, n, pos, q, nullptr, s);
  if (e == hipSuccess) e = pswfe::launch_spread(d, s);
  if (e == hipSuccess) e = pswfe::launch_drain(d, grid, s);
  return from_hip(e);
}

pswfe_status pswfe_transform(pswfe_plan* plan, const void* grid_in, void* grid_out, void* stream) {
  if (!plan || plan->batch || !grid_in || !grid_out) return PSWFE_E_ARG;
  return from_hip(pswfe::launch_transform(plan->d, grid_in, grid_out, static_cast<hipStream_t>(stream)));
}

pswfe_status pswfe_interpolate(pswfe_plan* plan, int64_t n, const void* pos, const void* grid, void* phi, void* grad,
                               void* stream) {
  if (!plan || plan->batch || n < 0 || !grid) return PSWFE_E_ARG;
  if (n > plan->d.n_max) return PSWFE_E_CAPACITY;
  if (n > 0 && !pos) return PSWFE_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const pswfe::DevPlan& d = plan->d;
  hipError_t e = pswfe::launch_bin(d, n, pos, nullptr, nullptr, s);
  if (e == hipSuccess && n > 0) e = pswfe::launch_gather(d, grid, phi, grad, 1, false, nullptr, s);
  return from_hip(e);
}

}  // extern "C"
