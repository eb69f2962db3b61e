/*
 * pswfe — PSWF fast Ewald summation, long-range (Fourier-space) part, for AMD MI355X (gfx950).
 *
 * Method: Bostrom, Tornberg, af Klinteberg, "Fast Ewald summation using prolate spheroidal
 * wave functions" (arXiv 2602.16591). The library evaluates, for n point charges rho_j at
 * positions x_j in the periodic box [0, L)^3 (Sec. 2.1; charge neutral, Sec. 1), or a cuboid
 * [0, L) x [0, Ly) x [0, Lz) (Sec. 6.1, remark on cuboid domains),
 *
 *   phi_i = phi_i^far + phi_i^self         (Sec. 3.1), plus on request the real-space residual
 *                                           phi_i^local (Sec. 3.1.1): the full Ewald sum
 *   F_i   = -rho_i grad phi_i              (Remark in Sec. 3.1, eq. force)
 *   E     = 1/2 sum_i rho_i phi_i          (Remark in Sec. 3.1)
 *
 * with phi^far computed by the fast Fourier-space summation of Alg. 2 using the PSWF mollifier
 * (Sec. 4.2) and the PSWF window (Sec. 4.3), and parameters from Alg. 3 (Sec. 6). The Gaussian
 * split and the Gaussian and B-spline windows the paper compares with (Sec. 4.3.1, Sec. 7.3.1-7.4)
 * run through the same pipeline (pswfe_variant_params).
 * Units: no Coulomb constant (Sec. 1, eq. potential1); phi is charge / length.
 *
 * Conventions for every entry point
 *  - Return value: a pswfe_status; nothing is thrown across this interface.
 *  - "device" pointers are coarse-grained HIP device allocations (hipMalloc, or the storage of
 *    a torch tensor on the GPU) owned by the caller; the library never frees them. Managed or
 *    fine-grained memory is not supported: outputs are summed with hardware float64 atomics,
 *    which are defined on coarse-grained memory only. "host" pointers are ordinary CPU memory.
 *  - Inputs are not validated on the device unless PSWFE_CHECK_INPUT is passed (see pswfe_flags).
 *    Without it, a particle with a non-finite position is given a NaN charge, so it poisons the
 *    outputs it reaches (for the long-range part, every output and the energy of its system)
 *    instead of being moved silently into the box, as a non-finite charge does; and a system
 *    whose charges do not sum to zero carries the uniform neutralising background implied by
 *    dropping the k = 0 mode (Sec. 3.1.2).
 *  - Floating-point arrays are in the plan's precision: float for PSWFE_FP32 and
 *    PSWFE_FP32_ARITH, double for PSWFE_FP64. The energy is always a double.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Every compute
 *    entry point only enqueues work: it performs no allocation and no host synchronisation
 *    (except with PSWFE_CHECK_INPUT), so it may be captured into a HIP graph. Calls on one plan must not overlap in time
 *    (a plan owns one set of work buffers).
 */
#ifndef PSWFE_H
#define PSWFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PSWFE_OK = 0,
  PSWFE_E_ARG = 1,        /* null pointer, n < 0, L <= 0, bad enum value, rc >= L/2 ...   */
  PSWFE_E_EPS_RANGE = 2,  /* eps outside [1e-14, 0.1], or c_s / c_w beyond the PSWF range  */
  PSWFE_E_GRID = 3,       /* m not an even 2,3,5,7-smooth size in [8, 512], or P > m, P > 32 */
  PSWFE_E_ALLOC = 4,      /* device allocation failed (plan creation only)                 */
  PSWFE_E_HIP = 5,        /* a HIP runtime call or kernel launch failed                    */
  PSWFE_E_CAPACITY = 6,   /* n larger than the plan's n_max                                */
  PSWFE_E_PREC = 7,       /* unknown precision                                             */
  PSWFE_E_NONNEUTRAL = 8, /* PSWFE_CHECK_INPUT: |sum q| > 1e-6 sum |q| in some system          */
  PSWFE_E_NONFINITE = 9   /* PSWFE_CHECK_INPUT: a position or charge is NaN or infinite        */
} pswfe_status;

typedef enum {
  PSWFE_TOL_REL = 0,      /* c_s = log(1/eps): relative error target (Sec. 6.2.1)           */
  PSWFE_TOL_ABS = 1       /* c_s = W0(2 (B_s/eps)^2)/2: absolute RMS target (eq. cs_dimless) */
} pswfe_tolmode;

/* Plan precision. PSWFE_FP32: float32 inputs, grids and outputs, with window values, products and
 * per-tile sums in float64 (error about 1e-8 relative from the arithmetic). PSWFE_FP32_ARITH: the
 * same float32 storage, with window values, products and sums in float32 in spreading (on the
 * float32 matrix cores) and interpolation; tiles are added into a float64 grid, or, on grids of
 * 2^20 points and more over all systems, into a float32 grid with float32 atomic adds; the self
 * term and energy are float64 (for eps >= 1e-6: about 3e-7 relative on systems of neutral
 * molecules, where grid values cancel). PSWFE_FP64: float64 throughout. */
typedef enum { PSWFE_FP32 = 0, PSWFE_FP64 = 1, PSWFE_FP32_ARITH = 2 } pswfe_prec;

/* Flags of the *_ex compute entry points (bitwise or). */
typedef enum {
  PSWFE_VEC_GRAD = 1,  /* the vector output is grad phi (not the force -rho grad phi)          */
  PSWFE_TOTAL = 2,     /* add the real-space residual: phi, forces and energy of the full Ewald
                          sum phi_far + phi_local + phi_self (Sec. 3.1, eq. Ewald split)       */
  PSWFE_CHECK_INPUT = 4 /* before any other work, sum each system's charges and |charges| in
                          float64 and count non-finite positions and charges on the device, wait
                          for the result on the host, and return PSWFE_E_NONFINITE or
                          PSWFE_E_NONNEUTRAL (|sum q| > 1e-6 sum |q|; the k = 0 mode is dropped,
                          Sec. 3.1.2) without computing anything. The call then synchronises
                          `stream`, so it cannot be captured into a HIP graph: under capture it
                          returns PSWFE_E_ARG. Outputs are untouched when a check fails.       */
} pswfe_flags;

/* Kernel split (Sec. 3.1) and window (Table 2). The method of the paper is PSWF/PSWF; the
 * other choices are the configurations it is compared with (Sec. 4.3.1, Sec. 7.3.1-7.4) and run
 * through the same pipeline (parameters from pswfe_variant_params). */
typedef enum {
  PSWFE_SPLIT_PSWF = 0,   /* PSWF mollifier (Sec. 4.2), band limited to c_s / r_c             */
  PSWFE_SPLIT_GAUSS = 1   /* Gaussian mollifier (Example 1), sigma = r_c / sqrt(c_s)          */
} pswfe_split;

typedef enum {
  PSWFE_WINDOW_PSWF = 0,    /* psi_0^{c_w}(x / alpha) / psi_0^{c_w}(0) (Sec. 4.3)             */
  PSWFE_WINDOW_GAUSS = 1,   /* exp(-c_g (x / alpha)^2) on |x| <= alpha, free-space transform */
  PSWFE_WINDOW_BSPLINE = 2  /* cardinal B-spline B_P(x / h), SPME scaling (Sec. 7.1)          */
} pswfe_window;

/* Method parameters (Alg. 3). The first block is what the kernels use; the *_alg fields are
 * the unrounded results of Alg. 3 steps 1-3, kept for reference. */
typedef struct {
  double L;          /* box side                                                           */
  double eps;        /* requested tolerance                                                */
  double rc;         /* cutoff radius = support of the mollifier (Sec. 4.2)                 */
  double cs;         /* mollifier bandlimit, = pi rc m / L (eq. csrc)                        */
  double cw;         /* window bandlimit,    = pi P / 2   (eq. cwP)                          */
  double alpha;      /* window half width,   = P h / 2   (Sec. 6.3)                          */
  double h;          /* grid spacing L / m                                                  */
  double lambda0_s;  /* lambda_0(c_s), for the self term -2 rho / (rc lambda_0) (Sec. 3.1)  */
  double cs_alg, cw_alg, alpha_alg;
  int32_t m;         /* grid points per dimension (even, 2,3,5,7-smooth)                    */
  int32_t P;         /* window support in grid points per dimension                         */
  int32_t tol_mode;  /* pswfe_tolmode                                                       */
  int32_t split;     /* pswfe_split (PSWFE_SPLIT_PSWF from pswfe_choose_params)              */
  int32_t window;    /* pswfe_window (PSWFE_WINDOW_PSWF from pswfe_choose_params)            */
  int32_t reserved;  /* 0                                                                    */
  double cg;         /* Gaussian window shape c_g (PSWFE_WINDOW_GAUSS only)                  */
  /* Cuboid boxes [0, L) x [0, Ly) x [0, Lz) (Sec. 6.1, remark on cuboid domains): sides and grid
   * sizes along y and z; 0 means equal to L and m (a cube). Grid spacings h_d = L_d / m_d; L, m,
   * h and alpha above are the x values; the window has the same P and c_w along every axis. */
  double Ly, Lz;
  int32_t my, mz;
} pswfe_params;

typedef struct pswfe_plan pswfe_plan;

/* Alg. 3 (Sec. 6.4) with these readings: the W_{-1} branch for c_w; m rounded up to an even
 * size with prime factors 2, 3, 5, 7; P from the final m; the kernels then use c_s = pi rc m/L,
 * c_w = pi P / 2, alpha = P h / 2; A_s = 5 and A_s/A_w = 4 sqrt(5) / pi^{3/2}.
 *   eps       tolerance, 1e-14 <= eps <= 0.1
 *   L         box side (> 0)
 *   rc        cutoff radius; <= 0 selects it from m (if m > 0) or else from n (64 neighbours)
 *   m         prescribed grid size, or 0 to let Alg. 3 choose it
 *   n         number of particles (used only by the default rc rule)
 *   q_l2      ||rho||_2 (PSWFE_TOL_ABS only)
 *   tol_mode  pswfe_tolmode
 *   out       host pointer, written on success
 * Host only; touches no GPU. */
pswfe_status pswfe_choose_params(double eps, double L, double rc, int32_t m, int64_t n, double q_l2,
                                 int32_t tol_mode, pswfe_params* out);

/* Alg. 3 for a cuboid box [0, Lx) x [0, Ly) x [0, Lz) (Sec. 6.1, remark on cuboid domains): the
 * parameters of the cube of side L_min = min(Lx, Ly, Lz) with the same particle density and
 * charge density (n and ||rho||^2 scaled by L_min^3 / (Lx Ly Lz)) fix r_c, c_s, c_w and P and the
 * spacing h = L_min / m; then m_d is the smallest even 2,3,5,7-smooth size with L_d / m_d <= h.
 * Arguments as for pswfe_choose_params (m: prescribed grid size along the shortest side, or 0).
 * With Lx = Ly = Lz this is pswfe_choose_params. Host only. */
pswfe_status pswfe_choose_params_box(double eps, double Lx, double Ly, double Lz, double rc, int32_t m, int64_t n,
                                     double q_l2, int32_t tol_mode, pswfe_params* out);

/* Oversampled grid for PSWF/PSWF parameters (from pswfe_choose_params[_box]): each m_d becomes the
 * smallest even 2,3,5,7-smooth size >= sigma m_d; with the effective factor sigma' = min_d
 * m_d / (2 k_band,d), k_band,d = c_s L_d / (2 pi r_c), the window bandlimit becomes
 * c_w = pi P (1 - 1/(2 sigma')) (the gap between the band edge and its first alias, times alpha)
 * and P the smallest support with c_w >= the base's c_w (pi P / 2 from Alg. 3), so P shrinks by
 * about 1 / (2 - 1/sigma'); sigma = 1 returns the base grid and support. The split
 * (r_c, c_s) is unchanged. The paper names oversampling as future work; the reading is stated in
 * the design notes and pinned against the direct sum. sigma in [1, 4]; PSWFE_E_ARG for other
 * splits or windows, PSWFE_E_GRID if a size would exceed 512. Host only. */
pswfe_status pswfe_oversample_params(const pswfe_params* base, double sigma, pswfe_params* out);

/* Parameters of a comparison configuration (Sec. 7.3.1-7.4): the split and the window are
 * chosen independently and the grid size m and support P are given (the paper's comparisons
 * search them for each tolerance). Fills h = L/m, alpha = P h / 2, c_w = pi P / 2, lambda_0(c_s)
 * and the *_alg fields (= the used values).
 *   split, window  pswfe_split, pswfe_window
 *   L, rc          box side, cutoff radius (rc < L/2)
 *   cs             PSWF split: bandlimit c_s (band edge c_s / r_c, modes |k| <= c_s L/(2 pi r_c));
 *                  Gaussian split: (r_c / sigma)^2 (eq. directsumexample), modes |k| <= m/2
 *   m, P           grid size (even, 2,3,5,7-smooth, 8..512) and support (3..24, P <= m)
 *   cg             Gaussian window shape; <= 0 selects 0.8 pi P / 2 (ignored for other windows)
 *   eps            tolerance the window polynomials are fitted to (as for pswfe_choose_params)
 *   out            host pointer, written on success
 * Returns PSWFE_E_ARG for an unknown split or window or a non-positive length, PSWFE_E_GRID
 * for m or P out of range, PSWFE_E_EPS_RANGE for c_s > 40 or eps outside [1e-14, 0.1].
 * Plans made from these parameters compute phi_far + phi_self, forces and energy as usual; the
 * real-space residual (PSWFE_TOTAL, pswfe_local) is available for the PSWF split only. Host
 * only. */
pswfe_status pswfe_variant_params(int32_t split, int32_t window, double L, double rc, double cs, int32_t m,
                                  int32_t P, double cg, double eps, pswfe_params* out);

/* Creates a plan: precomputes in float64 on the host the PSWF Legendre coefficients (App. B),
 * the k-space scaling tables (eq. diag_scale, eq. MhatPSWF, Table 2), the piecewise-polynomial
 * window (Remark after eq. force) and the FFT twiddles; allocates the device work buffers
 * (grid, spectrum, particle bins) for up to n_max particles on the current HIP device, and, when
 * the real-space residual is available, a stream of default priority, two events and 32 bytes
 * of float64 scratch per particle for PSWFE_TOTAL calls. Everything is released by
 * pswfe_plan_destroy.
 *   p      host pointer to parameters (from pswfe_choose_params, or filled by the caller)
 *   prec   pswfe_prec
 *   n_max  largest n accepted by pswfe_compute (>= 0)
 *   out    host pointer receiving the plan; NULL on failure. */
pswfe_status pswfe_plan_create(const pswfe_params* p, int32_t prec, int64_t n_max, pswfe_plan** out);

/* As pswfe_plan_create with an explicit tile edge (in grid cells) for binning, spreading and
 * interpolation: particles are processed per tile of tile^3 cells, each with an LDS copy of
 * the grid points its supports touch (tiles of edge 8 spread by register columns, others by
 * LDS atomics). tile = 0 picks the default (8, reduced to fit the LDS limits and small grids);
 * a tile that does not fit the LDS limits is reduced until it does. Used by the autotuner of
 * the Python layer. tile < 0 or tile > m -> PSWFE_E_ARG. */
pswfe_status pswfe_plan_create_tiled(const pswfe_params* p, int32_t prec, int64_t n_max, int32_t tile,
                                     pswfe_plan** out);

/* Tile edge a plan uses (system 0 of a batch; 0 for NULL). */
int32_t pswfe_plan_tile(const pswfe_plan* plan);

/* Frees the plan and its device buffers (synchronises the device first). NULL is a no-op. */
pswfe_status pswfe_plan_destroy(pswfe_plan* plan);

/* Full Alg. 2 plus self term and energy, in one stream:
 *   pos     device, n x 3 (row-major x, y, z), any real values (wrapped mod L)
 *   q       device, n charges (should sum to zero: the k = 0 mode is dropped, Sec. 3.1.2)
 *   phi     device, n outputs phi_far + phi_self, or NULL to skip
 *   force   device, n x 3 outputs -rho_i grad phi_far, or NULL to skip
 *   energy  device, one double: 1/2 sum rho_i (phi_far + phi_self), or NULL to skip
 *   stream  hipStream_t or NULL
 * Outputs are in input order. n = 0 writes energy 0 and nothing else. */
pswfe_status pswfe_compute(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi,
                           void* force, double* energy, void* stream);

/* pswfe_compute for callers that cannot allocate device memory (serving loops and harnesses that
 * forbid hipMalloc): no plan object; every buffer of the pipeline (tables, descriptors, grids,
 * spectrum, particle bins) lives in one library-owned device array of 64 MiB per GPU, held until
 * the process ends, so the call allocates no device memory. Arguments as for pswfe_compute, with
 * the plan replaced by its parameters and precision:
 *   p, prec  parameters (as for pswfe_plan_create) and pswfe_prec
 *   n        number of particles (0 <= n < 2^31); pos, q, phi, force, energy, stream as for pswfe_compute
 * The configuration's buffers must fit the array: about 17 m^3 (float32) or 25 m^3 (float64)
 * bytes of grids and spectrum plus, per particle, 36 (float32) or 52 (float64) bytes below
 * 200,000 particles and 52 or 84 bytes from there on (the two-level sort of large systems keeps a
 * staging copy of the records), and a few KiB of tables (the 64^3 water box with 30,000
 * particles needs about 6 MiB; a 128^3 float32 grid fits up to about 600,000 particles); larger
 * configurations return PSWFE_E_CAPACITY before any
 * device work. The first call of a configuration (parameters,
 * precision, n) on a GPU builds its tables on the host (host memory; the last 8 configurations
 * are kept); a call uploads them into the array (a host-to-device copy on `stream`) when another
 * configuration used it last, clears the grid and bin counters with fill kernels, and runs the
 * pipeline. The upload reads host memory, so under graph capture the call returns PSWFE_E_ARG.
 * Every call on a GPU shares that GPU's array and leaves its contents there: calls that overlap
 * in time on one GPU (on different streams) race and give wrong results. */
pswfe_status pswfe_compute_noalloc(const pswfe_params* p, int32_t prec, int64_t n, const void* pos, const void* q,
                                   void* phi, void* force, double* energy, void* stream);

/* As pswfe_compute, but `grad` receives grad phi_far (n x 3, not multiplied by -rho): the
 * field needed by adjoints of losses that depend on phi (a second apply with charges g gives
 * A g, and d/dx_i of g^T A q = g_i grad phi_i[q] + q_i grad phi_i[g], A symmetric, eq. matform). */
pswfe_status pswfe_compute_grad(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi,
                                void* grad, double* energy, void* stream);

/* pswfe_compute / pswfe_compute_grad with flags (pswfe_flags). With PSWFE_TOTAL the outputs are
 * the full Ewald potential, force and energy: the real-space residual
 *   phi_local,i = sum'_j rho_j R(|x_i - x_j|),  R(r) = (1 - Phi(r)) / r for r < r_c, 0 beyond
 * (Sec. 3.1.1, eq. R; minimum image, self pair excluded) is added to phi_far + phi_self, its
 * force -rho_i grad phi_local,i to the force and 1/2 sum rho_i phi_local,i to the energy.
 * R is evaluated from a float64 polynomial fit of Phi(r)/r in r^2 (relative error below 1e-15
 * in float64 plans, 1e-10 in float32 plans); pairs are found in cells of edge
 * L / floor(L / r_c) >= r_c (every pair of the system when L < 3 r_c). The residual runs on a
 * stream the plan owns, started by an event recorded on `stream` and joined back to `stream`
 * before interpolation, so the call stays ordered on `stream` (and can be captured into a HIP
 * graph from it); as for every call, calls on one plan must not run concurrently.
 * PSWFE_TOTAL needs r_c < L/2 and the PSWF split for every system (else PSWFE_E_ARG); unknown
 * flag bits -> PSWFE_E_ARG. */
pswfe_status pswfe_compute_ex(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                              double* energy, int32_t flags, void* stream);

/* The real-space residual alone (Sec. 3.1.1): phi_local (n), its force -rho grad phi_local (or,
 * with PSWFE_VEC_GRAD, grad phi_local; n x 3) and energy 1/2 sum rho_i phi_local,i (one double
 * per system), written to the device outputs (any may be NULL). Single-system plans take
 * n <= n_max particles; batch plans exactly the packed total (else PSWFE_E_ARG). PSWF split
 * only (else PSWFE_E_ARG). */
pswfe_status pswfe_local(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* phi, void* vec,
                         double* energy, int32_t flags, void* stream);

/* Host view of the residual the kernels evaluate, for verification: R(r_i) and R'(r_i)/r_i for
 * count radii (0 outside (0, r_c)); info[0..2] = polynomial degree, fit error (relative to
 * Phi(r)/r at 0), K = 2 / (lambda_0 psi_0(0) r_c). Any output may be NULL. PSWF split only
 * (else PSWFE_E_ARG). */
pswfe_status pswfe_host_local(const pswfe_params* p, int64_t count, const double* r, double* R, double* dRr,
                              double* info);

/* Batches of independent systems (each its own box, parameters and particles; Alg. 2 applied
 * to each with its own parameters, as a single-system plan would). All systems share the
 * precision. Binning and each FFT pass run as one kernel launch over all systems; spreading
 * and interpolation run one launch per distinct window support P among the systems. A batch
 * call therefore enqueues a fixed handful of launches, whatever the number of systems, and
 * can be captured into one HIP graph.
 *   nsys     number of systems, 1 <= nsys <= 2^20
 *   params   host array of nsys parameter sets (pswfe_choose_params per system)
 *   counts   host array of nsys particle counts (>= 0, sum < 2^31); fixed for the plan
 *   prec     pswfe_prec
 *   tiles    host array of nsys tile edges (as pswfe_plan_create_tiled; 0 = default: 8, reduced
 *            to fit the LDS limits), or NULL for all defaults
 *   out      host pointer receiving the plan; NULL on failure.
 * The particles of system s occupy the packed rows [offset_s, offset_s + counts[s]) of every
 * particle array, offset_s = counts[0] + ... + counts[s-1]. */
pswfe_status pswfe_batch_plan_create(int32_t nsys, const pswfe_params* params, const int64_t* counts,
                                     int32_t prec, const int32_t* tiles, pswfe_plan** out);

/* pswfe_compute for every system of a batch plan:
 *   pos     device, N x 3 packed positions, N = sum of counts; system s's rows are wrapped mod L_s
 *   q       device, N packed charges (each system should be neutral)
 *   phi     device, N outputs (or NULL);  force: device, N x 3 outputs (or NULL)
 *   energy  device, nsys doubles, energy of each system (or NULL)
 * A plan from pswfe_plan_create is rejected (PSWFE_E_ARG), as are batch plans passed to the
 * single-system entry points. */
pswfe_status pswfe_batch_compute(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* force,
                                 double* energy, void* stream);

/* As pswfe_batch_compute with grad phi_far (N x 3) in place of the forces (see
 * pswfe_compute_grad). */
pswfe_status pswfe_batch_compute_grad(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* grad,
                                      double* energy, void* stream);

/* pswfe_batch_compute with flags, as pswfe_compute_ex. */
pswfe_status pswfe_batch_compute_ex(pswfe_plan* plan, const void* pos, const void* q, void* phi, void* vec,
                                    double* energy, int32_t flags, void* stream);

/* Number of systems of a plan (1 for single-system plans, 0 for NULL). */
int32_t pswfe_plan_num_systems(const pswfe_plan* plan);

/* Host description of system s of a plan: its parameters, the first packed row, the particle
 * count (single-system plans: 0 and n_max) and the tile edge; any output may be NULL.
 * s out of range -> PSWFE_E_ARG. */
pswfe_status pswfe_plan_system(const pswfe_plan* plan, int32_t s, pswfe_params* params, int64_t* offset,
                               int64_t* count, int32_t* tile);

/* Alg. 2 step 1 alone (eq. spread_def): grid[(lz*m + ly)*m + lx] = sum_j q_j
 * phitilde(x_j - h l) for the m x my x mz grid points (m^3 for a cube), written to the device
 * array `grid` (plan precision, x fastest, z slowest). */
pswfe_status pswfe_spread(pswfe_plan* plan, int64_t n, const void* pos, const void* q, void* grid,
                          void* stream);

/* Alg. 2 steps 2-4 alone: b = F^{-1} C D F a (eq. matform) from the device grid `grid_in` to
 * the device grid `grid_out` (both m x my x mz, z slowest; may alias). */
pswfe_status pswfe_transform(pswfe_plan* plan, const void* grid_in, void* grid_out, void* stream);

/* Alg. 2 step 5 alone (eq. FastEwaldSteps34, eq. force) from the device grid `grid` (m x my x mz):
 * phi = interpolated values (no self term), grad = device n x 3 gradients; either may be NULL. */
pswfe_status pswfe_interpolate(pswfe_plan* plan, int64_t n, const void* pos, const void* grid,
                               void* phi, void* grad, void* stream);

/* Host-only views of the float64 precompute, for verification (no GPU needed).
 * pswfe_host_pswf: psi_0^c(x), d/dx psi_0^c(x) for |x| <= 1, lambda_0(c) and chi_0(c) (App. B);
 *   any output pointer may be NULL.
 * pswfe_host_tables: for parameters p and precision prec, fills (each may be NULL)
 *   tm[0 .. 3(m/2)^2]   radial scaling T_M[|k|^2] = h^6 Mhat(k) / V in the band, 0 outside and at 0,
 *   w[0 .. m/2]         1 / phihat_1(2 pi k / L)^2,
 *   coef[0 .. P(deg+1)) window polynomial coefficients (piece j, power k at j*(deg+1)+k),
 *   info[0..3]          deg, max fit error, max fit error of the derivative, self coefficient
 *                       2 / (rc lambda_0(c_s));
 *   the *_len arguments give the capacity of each array (in doubles); too small -> PSWFE_E_ARG. */
pswfe_status pswfe_host_pswf(double c, double x, double* psi, double* dpsi, double* lambda0, double* chi0);
pswfe_status pswfe_host_tables(const pswfe_params* p, int32_t prec, double* tm, int64_t tm_len, double* w,
                               int64_t w_len, double* coef, int64_t coef_len, double* info);

/* Instrumentation (not for hot loops): records a pair of HIP events on the compute stream
 * around one pipeline stage of each following call on this plan, for up to max_calls calls.
 *   stage: 0 binning, 1 spreading, 2 x R2C FFT, 3 y FFT, 4 z FFT + scaling + inverse z FFT,
 *          5 inverse y FFT, 6 x C2R FFT, 7 interpolation, 8 the whole compute call,
 *          9 the real-space residual; -1 turns timing off and frees the events.
 * pswfe_timing_enable synchronises the device and creates the events (host allocation).
 * pswfe_timing_read waits for the last recorded event and returns the summed elapsed time (ms)
 * and the number of timed calls since enable or the previous read, then resets the count. */
pswfe_status pswfe_timing_enable(pswfe_plan* plan, int32_t stage, int32_t max_calls);
pswfe_status pswfe_timing_read(pswfe_plan* plan, double* total_ms, int64_t* calls);

/* Effective parameters of a plan (host copy; system 0 of a batch). */
pswfe_status pswfe_plan_params(const pswfe_plan* plan, pswfe_params* out);

/* Static description of a string for a status code (never NULL). */
const char* pswfe_status_str(pswfe_status s);

/* Library version string, e.g. "pswfe 0.1 gfx950". */
const char* pswfe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSWFE_H */
