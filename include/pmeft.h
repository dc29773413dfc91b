/*
 * pmeft.h -- C ABI of libpmeft.so: the particle-mesh gravity step of the
 * cubic-screening EFT of dark energy on one AMD Instinct MI355X (gfx950).
 *
 * The step (Secs. 3.1-3.5 of the paper): Cloud-in-Cell deposit (Sec. 3.6.2),
 * the Newtonian Poisson equation with Geff/G (eq. phipsi_mod), the nonlinear
 * scalar-field equation with Vainshtein screening (eq. chi_scm, discretised as
 * in Sec. 3.2 and solved by FAS multigrid, Sec. 3.4), the fifth force added to
 * the Newtonian one (eq. force) with the 5-point gradient (Sec. 3.5.2), and
 * CIC interpolation of the acceleration with the kick.
 *
 * Conventions shared by every entry point
 *   - Code units (Sec. 3.1): box of unit side, h = 1/ng, positions in [0,1).
 *   - Grids are periodic and cell centred; cell (i,j,k) sits at
 *     ((i+1/2)h, (j+1/2)h, (k+1/2)h).  Field arrays passed in or out are
 *     C order [i][j][k] (k fastest), ng^3 elements of the chosen dtype.
 *   - Particle arrays are structures of arrays: 3 consecutive blocks of np
 *     elements (x block, y block, z block), same dtype as the fields;
 *     0 < np <= 2^30.
 *   - Every pointer argument is a device pointer unless marked HOST.  The
 *     caller owns every buffer.  The library never allocates device memory:
 *     all scratch lives in the caller's workspace `ws` of at least
 *     pm_workspace_bytes() bytes (256-byte aligned).
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream).  Calls that fill a HOST report synchronise the stream before
 *     returning; the others only enqueue.
 *   - Return value: PM_OK (0) or a negative PM_E* code; nothing aborts.  On
 *     PM_ENOCONV the output holds the last iterate and the report is filled.
 *   - Concurrent calls that share a workspace race; calls with separate
 *     workspaces may run concurrently on different streams.
 */
#ifndef PMEFT_H
#define PMEFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *pm_stream_t; /* hipStream_t */

enum {
    PM_OK = 0,
    PM_EINVAL = -1,      /* null pointer, unsupported ng (see pm_grid_levels), np <= 0, bad option */
    PM_EUNSTABLE = -2,   /* nu <= 0 while xi != 0: no viable model (Sec. 2.5 requires nu > 0) */
    PM_ENOCONV = -3,     /* max_vcycles reached before rel_tol */
    PM_ENONFINITE = -4,  /* NaN/Inf met in the input or the residual */
    PM_EHIP = -5,        /* a HIP runtime call failed */
    PM_ENOMEM = -6       /* workspace smaller than pm_workspace_bytes() */
};

typedef enum { PM_F32 = 0, PM_F64 = 1 } pm_dtype;

/* Arithmetic of the multigrid solves.  PM_PREC_F64: every level in FP64.
 * PM_PREC_MIXED: smoothing, restriction, prolongation in FP32; the fine-grid
 * residual, the defect correction of the FP64 iterate, the convergence test
 * and the coarsest-grid solve in FP64.  Each outer step (FP64 residual, test,
 * correction) runs two FP32 V-cycles; the nonlinear scalar field finishes in
 * FP64 once its residual nears the FP32 representation limit. */
typedef enum { PM_PREC_F64 = 0, PM_PREC_MIXED = 1 } pm_prec;

/* Initial guess of a solve: zero; the values passed in the output array
 * (e.g. the previous time step, Sec. 3.5.1); the linearised solution
 * lap chi = mu_chi s delta (Sec. 3.5.1, first time step); or the learned
 * warm start (scalar field only): the network of ws_unet_forward predicts the
 * nonlinear part t of the normalised source lap chi / (s mu_chi) = delta + t,
 * and one linear full-multigrid pass on lap chi0 = s mu_chi (delta + t - <t>)
 * gives the guess.  The guess sets the cost of a solve, never its answer. */
typedef enum { PM_GUESS_ZERO = 0, PM_GUESS_GIVEN = 1, PM_GUESS_LINEAR = 2, PM_GUESS_LEARNED = 3 } pm_guess;

/* Model parameters as the paper states them (eq. alpha-a, Sec. 2.4). */
typedef struct {
    double omega_m0;   /* present-day matter density (flat LCDM background, Sec. 3.5.2) */
    double alpha_b0;   /* braiding today */
    double alpha_m0;   /* Planck-mass run rate today */
    double a;          /* scale factor of the step */
    int screening;     /* 1: full eq. chi_scm; 0: linearised option (C4 := 0, Sec. 3.5.1) */
    int alpha_b_dot;   /* 1: keep alphadot_B/H in C2 (Sec. 2.2); 0: drop it (static test, Sec. 3.6.1) */
} pm_eft_params;

/* Derived scalars (FP64).  nu, xi, mu_chi, mu_Psi: eq. linearised; C2, C4:
 * Sec. 2.2; s = 3/2 (Geff/G) a Omega_m0 and K = C4/(4 E^2 a^4): prefactors of
 * eqs. phipsi_mod and chi_scm, which read lap Psi_N = s delta and
 * nu lap chi - xi s delta - K [(lap chi)^2 - d_i d_j chi d_i d_j chi] = 0.
 * lambda = K s xi / nu^2 is the one parameter the scalar equation depends on
 * once chi is measured in units of s mu_chi h^2. */
typedef struct {
    double omega_m_a, E2, alpha_b, alpha_m, geff, C2, C4, nu, xi, mu_chi, mu_psi, s, K, lambda;
} pm_eft_coeffs;

typedef struct {
    double rel_tol;    /* stop when ||r||_2 / ||source||_2 <= rel_tol (source: s delta for Psi_N,
                          xi s delta / nu for chi) */
    int max_vcycles;   /* <= 64 is recorded in residual_hist */
    int n_pre, n_post; /* red-black Gauss-Seidel sweeps before / after the coarse correction */
    int precision;     /* pm_prec */
    int guess;         /* pm_guess */
    /* PM_GUESS_LEARNED only (else ignored): the network's FP32 parameters
     * (ws_unet_param_count values, device) and a device workspace of at least
     * ws_unet_workspace_bytes(ng, 0) bytes, 256-byte aligned.  ng must be a
     * multiple of 64; otherwise the solve returns PM_EINVAL. */
    const float *learned_params;
    void *learned_ws;
    size_t learned_ws_bytes;
    /* Smoother of every level: PM_SMOOTH_RBGS (0, default), red-black
     * Gauss-Seidel with the Laplacian-form Newton update (Sec. 3.2.2); or
     * PM_SMOOTH_JACOBI, the pointwise local solve of PySCo (Secs. 3.2.1 and
     * 3.5.1): every cell takes the root of its local equation from the
     * previous iterate's neighbours, under-relaxed as
     * chi <- w chi* + (1 - w) chi with w = jacobi_weight (0 means 0.6).  The
     * root is the same branch as the Newton update's, so both smoothers
     * converge to the same discrete solution; the Jacobi smoother runs the
     * per-level grid-wide kernels only. */
    int smoother;
    double jacobi_weight;
} pm_mg_opts;

enum { PM_SMOOTH_RBGS = 0, PM_SMOOTH_JACOBI = 1 };

typedef struct {
    int status;                 /* PM_OK or PM_ENOCONV / PM_ENONFINITE */
    int vcycles;                /* V-cycles performed */
    double rel_residual;        /* of the returned iterate */
    double residual_hist[64];   /* rel. residual before V-cycle i (i < 64); with PM_PREC_MIXED, before
                                   each outer defect-correction step (two FP32 V-cycles each), then
                                   before each V-cycle of an FP64 finish */
    double mean_shift;          /* mean of the quadratic-root Laplacian removed on the fine grid */
    long long clamped_cells;    /* void cells on the fine grid (Sec. 3.3) */
    float ms;                   /* wall time of the solve (HIP events) */
} pm_mg_report;

typedef struct {
    pm_mg_report poisson, scalar;
    float ms_deposit, ms_force, ms_total;
} pm_step_report;

/* Coefficients at the given parameters (HOST in, HOST out).  Returns
 * PM_EUNSTABLE if nu <= 0 while xi != 0 (the coefficients are still filled). */
int pm_eft_coefficients(const pm_eft_params *p /* HOST */, pm_eft_coeffs *out /* HOST */);

/* Number of multigrid levels for ng (ng halved while even and ng/2 >= 4,
 * coarsest grid 4^3 or 6^3); 0 if ng is not supported (ng < 8 or ng > 1024,
 * or the coarsest grid would be odd or larger than 6^3). */
int pm_grid_levels(int ng);

/* Workspace bytes for any entry point at this size (np may be 0 for the
 * grid-only calls).  With np > 0 (pm_step) it also holds a second per-solve
 * region and a second delta hierarchy, so that the step's two solves (and the
 * warm start's modified delta) run side by side. */
size_t pm_workspace_bytes(int ng, long long np, pm_dtype dtype, pm_prec prec);

/* CIC deposit (Sec. 3.6.2): rho_c = (ng^3/np) sum_p W(x_p - x_c), the tent
 * W = prod_d max(0, 1 - |dx_d|/h) with periodic wrap.  pos: SoA 3 x np in
 * [0,1); rho: ng^3 out, density in units of the mean.  Accumulation is in
 * 2^-40 fixed point, so the result does not depend on particle order. */
int pm_deposit(const void *pos, long long np, pm_dtype dtype, int ng, void *rho,
               void *ws, size_t ws_bytes, pm_stream_t stream);

/* The CIC deposit of pm_deposit without a caller workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the call allocates
 * nothing; its scratch (the fixed-point accumulator, the packed density and
 * the reduction partials, 16 bytes per cell plus 128 KiB) lives in a device
 * array of pm_deposit_noalloc_max_bytes() = 33 MiB inside the library, one
 * per GPU, held until the process ends.  Same arguments and result as
 * pm_deposit (bit for bit); ng up to 128 (PM_ENOMEM beyond: the scratch
 * array is too small), PM_EINVAL as pm_deposit.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents (the
 * accumulator is cleared by each call): calls that overlap on one GPU, on
 * any streams, race. */
size_t pm_deposit_noalloc_max_bytes(void);
int pm_deposit_noalloc(const void *pos, long long np, pm_dtype dtype, int ng, void *rho, pm_stream_t stream);

/* Newtonian potential (eq. phipsi_mod with Geff/G inside s): solve
 * lap_7 Psi_N = s (rho - 1 - <rho - 1>), <Psi_N> = 0, by red-black
 * Gauss-Seidel V-cycles.  rho: ng^3 in; psi: ng^3 in (guess if GIVEN) / out. */
int mg_poisson_solve(const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
                     const pm_mg_opts *opts /* HOST */, void *psi, pm_mg_report *rep /* HOST, nullable */,
                     void *ws, size_t ws_bytes, pm_stream_t stream);

/* Scalar field (eq. chi_scm, discretised as in Sec. 3.2: 7-point Laplacian,
 * 3-point second and 4-point cross derivatives): the periodic system
 *   lap_h chi = Lq - <Lq>,  Lq = -2 G / (nu + sqrt(nu^2 + (8/3) K G)),
 *   G = K T - xi s delta,  T = squared traceless part of the discrete Hessian,
 * with <chi> = 0.  Void cells, where the spherical existence condition
 * nu^2 - (8/3) K xi s delta >= 0 fails (Sec. 3.3), take the discriminant 0,
 * Lq = 3 nu/(4K).  FAS V-cycles (Sec. 3.4) with red-black Gauss-Seidel
 * Newton updates chi <- (S - h^2 (Lq - <Lq>))/6 (Sec. 3.2.2).  xi = 0 returns
 * chi = 0.  rho: ng^3 in; chi: ng^3 in (guess if GIVEN) / out. */
int mg_scalar_solve(const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
                    const pm_mg_opts *opts /* HOST */, void *chi, pm_mg_report *rep /* HOST, nullable */,
                    void *ws, size_t ws_bytes, pm_stream_t stream);

/* Force and kick (eq. force, Sec. 3.5.2): g = -D5 (Psi_N + xi chi) on the
 * grid with the 5-point stencil, interpolated to the particles with the CIC
 * kernel; vel += g * dt_kick.  psi, chi: ng^3 in; pos: 3 x np in; vel: 3 x np
 * in/out; acc_out: 3 x np out or NULL. */
int pm_force_interp(const void *psi, const void *chi, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
                    const void *pos, long long np, void *vel, double dt_kick, void *acc_out,
                    void *ws, size_t ws_bytes, pm_stream_t stream);

/* One PM gravity step: deposit, Poisson, scalar field, force, kick and, if
 * dt_drift != 0, drift pos += vel * dt_drift (mod 1).  psi and chi (ng^3) are
 * outputs and, with guess GIVEN, carry the previous step's fields in.  The
 * two solves depend on the deposit's delta only and run side by side: the
 * scalar-field solve (with PM_GUESS_LEARNED, after the network's forward pass
 * and the warm-start pass) is issued by a library worker thread on a second
 * stream owned by the library (one per device, created on first use, default
 * priority), ordered after the deposit and before the force by events; the
 * Poisson solve and all other work stay on `stream`, and the call returns
 * once both solves have finished their host-side convergence tests.  The
 * results are those of running the solves one after the other.  Overlapping
 * calls on one device share the second stream: correct, but their scalar
 * solves serialise. */
int pm_step(void *pos, void *vel, long long np, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
            const pm_mg_opts *poisson_opts /* HOST */, const pm_mg_opts *scalar_opts /* HOST */,
            double dt_kick, double dt_drift, void *psi, void *chi, pm_step_report *rep /* HOST, nullable */,
            void *ws, size_t ws_bytes, pm_stream_t stream);

/* Arrangement of pm_step's two solves, process-wide: side_by_side 1 (the
 * default) as described above; 0: both solves (and the learned warm start's
 * network) are issued from the calling thread on `stream` alone, Poisson
 * first, so that all of the step's work is ordered on the caller's stream
 * and no library thread or stream is used (same results; slower, since the
 * solves no longer overlap).  Returns the previous setting. */
int pm_set_step_concurrency(int side_by_side);

/* Bardeen potentials (eqs. phipsi_mod) from the Newtonian part Psi_N (lap
 * Psi_N = s delta, the psi of mg_poisson_solve / pm_step) and the scalar
 * field chi at the parameters' a: Psi = Psi_N + (alpha_B - alpha_M) chi, the
 * potential the particles feel; Phi = Psi_N + alpha_B chi; and Psi + Phi, the
 * combination that lensing sees (Sec. 1).  With screening off, chi =
 * mu_chi Psi_N and these reduce to mu_Psi Psi_N and mu_Phi Psi_N (eq.
 * linearised).  All arrays ng^3 natural order of dtype; each output nullable
 * (not all three).  Only enqueues; no workspace. */
int pm_potentials(const void *psi_n, const void *chi, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
                  void *psi_out, void *phi_out, void *lens_out, pm_stream_t stream);

/* Multi-step evolution: kick-drift-kick leapfrog of the particles in the
 * code time of Sec. 3.1, dt~ = da / (a^3 E(a)) (dx/dt~ = v, dv/dt~ = -grad Psi),
 * from a_start to a_end in nsteps steps uniform in a (log_spacing 0) or in
 * ln a (1).  pos, vel: 3 x np SoA at a_start (velocities in code units,
 * synchronous with the positions); on return both are at a_end.  The force
 * is evaluated nsteps + 1 times, at every a_k (one pm_step each, the model's
 * coefficients taken at a_k): the kick of evaluation k spans
 * [a_{k-1/2}, a_{k+1/2}] (clipped to [a_start, a_end]; half steps at the
 * midpoint of the spacing variable) and its drift [a_k, a_{k+1}].  The first
 * evaluation uses the guesses of the options; every later one starts both
 * solves from the previous step's fields (Sec. 3.5.1).  psi, chi: ng^3
 * (dtype) out, the fields of the last evaluation (in: guesses if GIVEN).
 * The parameters' a is ignored.  The report (HOST, nullable) sums the
 * V-cycles.  Returns PM_OK, PM_ENOCONV if some solve stopped at max_vcycles
 * (the run continues), or the first hard error; PM_EUNSTABLE if nu <= 0 at
 * some a_k while xi != 0 (checked before anything runs).  Workspace as for
 * pm_step. */
typedef struct {
    int status, steps, force_evaluations, max_scalar_vcycles;
    long long poisson_vcycles, scalar_vcycles, clamped_cells_last;
    double max_rel_residual, a_end;
    float ms_total;
} pm_evolve_report;

int pm_evolve(void *pos, void *vel, long long np, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
              double a_start, double a_end, int nsteps, int log_spacing, const pm_mg_opts *poisson_opts /* HOST */,
              const pm_mg_opts *scalar_opts /* HOST */, void *psi, void *chi, pm_evolve_report *rep /* HOST */,
              void *ws, size_t ws_bytes, pm_stream_t stream);

/* The code-time interval int_{a0}^{a1} da / (a^3 E(a)) of the flat LCDM
 * background (Sec. 3.1), as pm_evolve uses it for its kicks and drifts; NAN
 * for invalid arguments.  HOST only. */
double pm_code_time(double a0, double a1, double omega_m0);

/* ---- Power spectrum and boost (Sec. 3.6.2, Sec. 4.2) ----------------------
 * P(k) of a periodic field sampled on an n^3 grid (n a power of two, 8..1024)
 * in a box of side `box`: the 3D discrete Fourier transform F of the field
 * (FP64, computed by the library's FFT kernels) and the shell averages
 *   P_b = box^3 <|F_m|^2> / n^6,  k_b = (2 pi / box) <|m|>
 * over the integer wave vectors m (components in [-n/2, n/2)) with
 * b + 1/2 <= |m| < b + 3/2, b = 0 .. nbins - 1 (the zero mode is never
 * counted); count_b is the number of modes.  nbins <= n / 2; the paper keeps
 * the bins below half the estimator grid's Nyquist wavenumber, nbins = n / 4.
 * No window deconvolution.  Outputs are HOST arrays of nbins (each
 * nullable); the call synchronises the stream.  The shell sums use FP64
 * atomics in LDS: reruns agree to rounding, not bit for bit.
 * pm_particle_power first deposits the particles (3 x np SoA, dtype) with the
 * CIC kernel of pm_deposit on the n^3 estimator grid (finer than the particle
 * grid, to push aliasing to higher k) and transforms rho - 1.
 * Workspace: pm_power_workspace_bytes(n, particles) bytes (particles = 1 for
 * pm_particle_power), 256-byte aligned.  Errors: PM_EINVAL, PM_ENOMEM,
 * PM_EHIP. */
size_t pm_power_workspace_bytes(int n, int particles);
int pm_field_power(const void *field, int n, pm_dtype dtype, double box, int nbins, double *k_out /* HOST */,
                   double *pk_out /* HOST */, double *count_out /* HOST */, void *ws, size_t ws_bytes,
                   pm_stream_t stream);
int pm_particle_power(const void *pos, long long np, pm_dtype dtype, int n, double box, int nbins,
                      double *k_out /* HOST */, double *pk_out /* HOST */, double *count_out /* HOST */, void *ws,
                      size_t ws_bytes, pm_stream_t stream);

/* Power-spectrum boost R(k) = P_num(k) / P_den(k) of a simulation pair
 * (Sec. 4.2), smoothed over the bins with a one-dimensional Gaussian filter
 * of width sigma_k in k (the paper smooths its boosts this way):
 * r_b = sum_c w_bc R_c / sum_c w_bc, w_bc = exp(-(k_c - k_b)^2 / (2 sigma_k^2));
 * sigma_k = 0 returns R unsmoothed.  HOST arrays of nbins.  PM_ENONFINITE if
 * some P_den is 0 or a ratio is not finite; PM_EINVAL for bad arguments. */
int pm_boost(const double *k /* HOST */, const double *pk_num /* HOST */, const double *pk_den /* HOST */, int nbins,
             double sigma_k, double *r_out /* HOST */);

/* Particle sort: reorders the particles (pos, and vel and ids when given)
 * by the cell of their CIC base corner, key (i0 ng + j0) ng + k0 with
 * i0 = floor(x ng - 1/2) mod ng per axis (Sec. 3.6.2's CIC), so that
 * neighbouring particles sit together in memory and the deposit's and
 * interpolation's footprints stay compact.  Stable (equal keys keep their
 * order) and deterministic; particles with unusable coordinates take the last
 * cell.  pos, vel: 3 x np SoA of dtype (vel nullable); ids: np int64
 * (nullable).  Workspace: pm_sort_workspace_bytes(np, dtype), 256-byte
 * aligned.  The deposit's result does not depend on the order (it is exact
 * in fixed point); the sort changes cost only. */
size_t pm_sort_workspace_bytes(long long np, pm_dtype dtype);
int pm_sort_particles(void *pos, void *vel, long long *ids, long long np, int ng, pm_dtype dtype, void *ws,
                      size_t ws_bytes, pm_stream_t stream);

/* ---- Batched solves ------------------------------------------------------
 * Many independent scalar-field problems (a parameter scan, several boxes;
 * the batched scan of Sec. 4's parameter studies) in one call.  Each problem
 * has its own grid size, precision of its arrays, parameters and hierarchy;
 * its result and report equal those of mg_scalar_solve on the same problem
 * bit for bit.  Problems of one grid size and dtype form a group, solved in
 * lockstep: every kernel of the solve is one launch for all members still
 * iterating (grid rows select the member), so small grids fill the GPU
 * together; a member leaves at its own convergence test, and the mixed-
 * precision members that finish in FP64 do so together.  Members with
 * screening off (linear) are solved one after another.  The largest grid's
 * group runs on `stream`; beside it, from library worker threads, the second
 * largest on the library's second stream (the one pm_step uses) and the
 * others, one after another, on a third library stream, ordered by events
 * after the work already on `stream`; `stream` waits for them before
 * anything enqueued after the call.  The call
 * returns when every problem is solved (all output arrays complete).  opts
 * apply to every problem (PM_GUESS_LEARNED is not accepted here).  Workspace
 * (mg_batched_workspace_bytes, 256-byte aligned): every group's members'
 * solver workspaces side by side, each group with a small control area.
 * Returns PM_OK, PM_ENOCONV if some problem stopped at max_vcycles, or the
 * first hard error; reps (HOST, nprob entries, nullable) receive the
 * per-problem reports (ms: the time of the problem's group). */
typedef struct {
    const void *rho;     /* ng^3 density (device), natural order */
    void *chi;           /* ng^3 out (guess in if GIVEN) */
    int ng;
    pm_dtype dtype;      /* of rho and chi */
    pm_eft_params p;
} pm_problem;

size_t mg_batched_workspace_bytes(const pm_problem *probs /* HOST */, int nprob, int precision);
int mg_scalar_solve_batched(const pm_problem *probs /* HOST */, int nprob, const pm_mg_opts *opts /* HOST */,
                            pm_mg_report *reps /* HOST, nullable */, void *ws, size_t ws_bytes, pm_stream_t stream);

/* ---- Launch shapes and the autotuner --------------------------------------
 * Two launch choices are kept per (finest grid ng, word size of the
 * hierarchy: 8 for FP64 levels, 4 for the FP32 levels of PM_PREC_MIXED):
 *  - block_cycle_grid: the coarse end of every V-cycle (and of full
 *    multigrid) runs as one single-workgroup launch from the first level
 *    whose grid is at most this (0: every level launches its own kernels);
 *  - tiled_smoother (0 off, 1 small tiles, 2 large tiles, 3 largest
 *    tiles): the large levels (grid >= 64, divisible by 8 and by 64 or 128)
 *    use the 2.5D-tiled red-black half-sweep, whose cell updates equal the
 *    untiled ones bit for bit; large tiles (8 rows x 64 packed cells x 16
 *    planes, 8 in FP64) replace small ones (4 rows x 64 or 8 rows x 32, 8
 *    planes) where they still give 512 tiles, and the largest (16 rows x 64 x
 *    16 planes) replace large ones under the same rule; 4: the largest tiles
 *    for the transfers, and every red-black sweep of a level whose tiles (8
 *    rows by 32 packed cells in FP64, 64 in FP32) divide it into at least
 *    256 tiles runs both colours in one launch: each tile updates its red
 *    cells plus a one-cell halo one plane ahead of its black cells, which
 *    take those new red values, so the sweep reads the old values once (the
 *    black half then takes the lagged mean the red half takes).
 * Defaults 8 and 1.  They change the cost of a cycle, and the grouping of
 * the partial sums behind the lagged means, not the converged answer.
 * pm_autotune times full multigrid + 3 V-cycles of the scalar field on a
 * synthetic density (uniform hash noise per cell in [0.2, 1.8], rough at every
 * scale) for every candidate (block_cycle_grid in off, 8, 16, 32, 64;
 * tiled_smoother 0, 1, 2, 3, 4) and keeps the fastest for (ng, precision);
 * workspace: pm_autotune_workspace_bytes.  pm_tune_save / pm_tune_load write and read
 * the table as text lines "ng word_bytes block_cycle_grid tiled_smoother".
 * The table is process-wide. */
size_t pm_autotune_workspace_bytes(int ng, int precision);
int pm_autotune(int ng, int precision, void *ws, size_t ws_bytes, pm_stream_t stream);
int pm_get_launch_shape(int ng, int word_bytes, int *block_cycle_grid /* HOST */, int *tiled_smoother /* HOST */);
int pm_set_launch_shape(int ng, int word_bytes, int block_cycle_grid, int tiled_smoother);
int pm_tune_save(const char *path);
int pm_tune_load(const char *path);

/* ---- Learned warm start ------------------------------------------------
 * A 3-level 3D U-Net maps the density contrast and (alpha_B0, alpha_M0, a)
 * to the nonlinear part of the scalar field's normalised source,
 *   t = lap_h chi / (s mu_chi) - delta,
 * which vanishes where the field is unscreened (lap chi = mu_chi s delta in
 * linear theory, eq. linearised) and carries the Vainshtein suppression in
 * dense cells.  The source is local where chi is not, so the network predicts
 * t and a linear multigrid pass turns delta + t into the guess
 * (PM_GUESS_LEARNED above).  Input channels: standardised ln(1 + delta +
 * 1e-3) and the three parameters broadcast; 3x3x3 periodic convolutions with
 * ReLU (16-16 / 32-32 / 64-64 channels on grids n, n/2, n/4), 2x2x2 average
 * pooling, nearest-neighbour upsampling, skip concatenations (96 -> 32,
 * 48 -> 16) and a 1x1x1 head.  Convolutions run on the matrix cores in BF16
 * with FP32 accumulation; activations are BF16.  delta = rho - <rho>.
 *
 * Parameters: one FP32 device array of ws_unet_param_count() values: for each
 * convolution in order (l1a 4->16, l1b 16->16, l2a 16->32, l2b 32->32, l3a
 * 32->64, l3b 64->64, l4a 96->32, l4b 32->32, l5a 48->16, l5b 16->16) its
 * weight W[27][cin][cout] (tap t = (di+1)*9 + (dj+1)*3 + (dk+1) for the
 * neighbour offset (di, dj, dk)) followed by its bias[cout]; then the head's
 * 16 weights and 1 bias.  ng must be a multiple of 64 (64..1024).  Workspaces
 * are device memory, 256-byte aligned, owned by the caller; sizes from
 * ws_unet_workspace_bytes (training = 0: inference, also enough for
 * PM_GUESS_LEARNED; 1: training).  Errors: PM_EINVAL (null pointer, bad ng,
 * misaligned workspace), PM_ENOMEM (workspace too small), PM_EHIP. */
long long ws_unet_param_count(void);
size_t ws_unet_workspace_bytes(int ng, int training);

/* Forward pass.  rho: ng^3 FP64 density (natural order); yhat_out: ng^3 FP32,
 * the predicted t (natural order).  Inference evaluates the two decoder
 * layers that read nearest-neighbour upsampled tensors in the polyphase form
 * (per output parity, a 2x2x2 convolution of the coarse tensor with summed
 * taps) where the coarse grid is a multiple of 64; it differs from the
 * training forward pass only by the BF16 rounding of those summed weights. */
int ws_unet_forward(const float *params, const double *rho, int ng, const pm_eft_params *p /* HOST */,
                    float *yhat_out, void *ws, size_t ws_bytes, pm_stream_t stream);

/* The learned warm start's initial scalar field chi_0 itself (north-star
 * grown form (4)): the network's source prediction t for the density rho
 * (ng^3 natural order, dtype), then one linear full-multigrid pass on
 * lap chi_0 = s mu_chi (delta + t - <t>) -- exactly the guess that
 * PM_GUESS_LEARNED starts the scalar-field solve from.  chi0_out: ng^3
 * (dtype), mean-free (zero where the scalar equation is linear or xi = 0:
 * no learned guess is taken there).  learned_ws: ws_unet_workspace_bytes(ng,
 * 0) bytes; ws: a solver workspace (pm_workspace_bytes(ng, 0, dtype,
 * PM_PREC_F64)).  ng a multiple of 64.  Errors as mg_scalar_solve. */
int ws_unet_guess(const float *params, const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
                  void *chi0_out, void *learned_ws, size_t learned_ws_bytes, void *ws, size_t ws_bytes,
                  pm_stream_t stream);

/* Forward pass in the training form (spec grown form (4): the network
 * is trained by the library's own forward and backward kernels): the same
 * network as ws_unet_forward, but the two decoder layers read explicit
 * nearest-neighbour upsampled tensors (no polyphase rewrite), the first layer
 * reads the padded 4-channel input, and every activation the backward pass
 * reads stays in ws, a training workspace (ws_unet_workspace_bytes(ng, 1)
 * bytes).  yhat_out: ng^3 FP32, natural order (nullable).  Errors as above. */
int ws_unet_forward_train(const float *params, const double *rho, int ng, const pm_eft_params *p /* HOST */,
                          float *yhat_out, void *ws, size_t ws_bytes, pm_stream_t stream);

/* Backward pass (reverse-mode differentiation of the training forward pass):
 * the gradient of a scalar loss L with respect to every parameter, given
 * dloss_dyhat = dL/dyhat (ng^3 FP32, natural order).  ws must hold the
 * activations of the preceding ws_unet_forward_train call with the same
 * params and ng (nothing in between may have used ws).  grad_out
 * (ws_unet_param_count FP32, parameter layout above) is overwritten.
 * Activation gradients are BF16 between layers (rounded after each
 * convolution's input gradient, each upsampling's and pooling's adjoint);
 * weight and bias gradients accumulate in FP32 per block and are summed in
 * block order, so a rerun gives the same bits. */
int ws_unet_backward(const float *params, const float *dloss_dyhat, int ng, float *grad_out, void *ws,
                     size_t ws_bytes, pm_stream_t stream);

/* Adam (Kingma & Ba, with bias correction) on FP32 parameters, after optional
 * global-norm clipping: g <- g min(1, grad_clip / ||g||_2) when grad_clip > 0;
 * m <- beta1 m + (1 - beta1) g; v <- beta2 v + (1 - beta2) g^2;
 * params <- params - lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step))
 * + eps).  params, grads, m, v: n FP32 (device; grads is only read); step >= 1
 * counts the updates so far including this one.  grad_norm (HOST, nullable)
 * receives ||g||_2 before clipping (the call then synchronises the stream).
 * ws: ws_adam_workspace_bytes(n) bytes, 256-byte aligned (the norm's partial
 * sums).  Errors: PM_EINVAL (null pointer, n <= 0 or >= 2^31, step < 1,
 * lr < 0, beta outside [0, 1), eps <= 0, grad_clip < 0, misaligned ws),
 * PM_ENOMEM, PM_EHIP. */
size_t ws_adam_workspace_bytes(long long n);
int ws_adam_step(float *params, const float *grads, float *m, float *v, long long n, long long step, double lr,
                 double beta1, double beta2, double eps, double grad_clip, double *grad_norm /* HOST */, void *ws,
                 size_t ws_bytes, pm_stream_t stream);

/* One training step on one sample, the composition of the three calls above:
 * ws_unet_forward_train, the MSE loss mean (yhat - t)^2 against the target
 * t = lap_h chi / (s mu_chi) - delta of the solved field chi_target (ng^3
 * FP64, natural order; 7-point Laplacian) and its gradient dL/dyhat =
 * 2 (yhat - t) / ng^3, ws_unet_backward and (if lr > 0) ws_adam_step with
 * beta1 0.9, beta2 0.999, eps 1e-8 on params with moment arrays adam_m,
 * adam_v.  grad_out (param_count FP32, nullable) receives the unclipped
 * gradients; *loss and *grad_norm (HOST, nullable) the sample's loss and
 * ||g||_2 (either makes the call synchronise the stream). */
int ws_unet_train_step(float *params, float *adam_m, float *adam_v, long long step, double lr, double grad_clip,
                       const double *rho, const double *chi_target, int ng, const pm_eft_params *p /* HOST */,
                       float *grad_out, double *loss /* HOST */, double *grad_norm /* HOST */, void *ws,
                       size_t ws_bytes, pm_stream_t stream);

/* Read-back of a tensor of the training workspace ws (for testing the
 * backward pass stage by stage on the network's own BF16 values): gradient
 * 0, the activation that ws_unet_forward_train left; gradient 1, its
 * gradient as ws_unet_backward left it (ReLU masks applied, skip gradients
 * added; tensor 0 has none).  Tensor index 0..12 = input (16 channels, the
 * first 4 used), l1a out (16), [upsampled l4b out (32) | l1b out (16)] (48),
 * pool 1 (16), l2a out (32), [upsampled l3b out (64) | l2b out (32)] (96),
 * pool 2 (32), l3a out (64), l3b out (64), l4a out (32), l4b out (32), l5a
 * out (16), l5b out (16); grid ng, ng/2 or ng/4 per tensor as the network
 * runs it.  out: (grid^3 x channels) FP32, channels-last natural order. */
int ws_unet_tensor(const void *ws, int ng, int tensor, int gradient, float *out, pm_stream_t stream);

/* One 3x3x3 periodic convolution on BF16 channels-last tensors with FP32
 * output (for testing the kernels): mode 0 forward out[n^3][cout] =
 * b + conv(x); mode 1 input gradient out[n^3][cin] from dy[n^3][cout]; mode
 * 2 weight gradient out[27][cin][cout] from x and dy (summed in a fixed
 * order: deterministic); mode 3 the forward of a layer whose first 2cin/3
 * input channels are the nearest-neighbour upsampling of x (a coarse
 * (n/2)^3 x 2cin/3 tensor) and whose last cin/3 channels are dy (n^3 x
 * cin/3), evaluated in the polyphase form the network uses at inference
 * ((cin, cout) = (48, 16) or (96, 32), n a multiple of 128); mode 4 the
 * network's last layer with its output head as inference runs them, out[n^3]
 * = hb + sum_o hw[o] relu(b[o] + conv(x)[o]) (cin = cout = 16, n a multiple
 * of 64; b holds the 16 biases, then hw[16], then hb).  w: FP32
 * W[27][cin][cout] (device); n a multiple of 16; ws: 256-byte aligned, at
 * least 2 * W + 4 * 240 * (27 cin cout + cout) bytes with W = 54 *
 * pad16(cin) * pad16(cout) rounded up to 256. */
int ws_conv3(int mode, int n, int cin, int cout, const void *x_bf16, const void *dy_bf16, const float *w,
             const float *b, float *out, void *ws, size_t ws_bytes, pm_stream_t stream);

/* The network's first layer as inference runs it (for testing the kernel):
 * the 4-channel input [f, x1, x2, x3] with x1..x3 the same at every voxel
 * (the broadcast parameters), out[n^3][16] = b + conv(input) (FP32, no
 * ReLU), computed as a single-channel convolution of f (n^3 BF16, natural
 * order) plus the broadcast channels' constant.  w: FP32 W[27][4][16], b[16]
 * (device); xc: HOST [3]; n a multiple of 64. */
int ws_conv3_first(int n, const void *f_bf16, const float *w, const float *b, const float *xc /* HOST [3] */,
                   float *out, pm_stream_t stream);

/* Self-check of the workspace plan for (ng, np, dtype, prec), on the host
 * only (no device work, no allocation): every multigrid level view and
 * colour buffer lies inside pm_workspace_bytes(ng, np, dtype, prec), no two
 * arrays that a level's kernels write overlap, the levels halve down to a
 * 4^3 or 6^3 grid, and for every start level of the single-workgroup coarse
 * cycle the levels it keeps resident fit the LDS it requests (within its
 * budget).  PM_OK, or PM_EINVAL if any of these fails or the size is
 * unsupported. */
int pm_plan_check(int ng, long long np, pm_dtype dtype, pm_prec prec);

/* Measurement hooks.  While enabled, each launch of the finest-level
 * red-black smoother (a half-sweep, or a fused two-colour sweep) is
 * bracketed by HIP events on the stream it runs on (a fixed pool of 16384
 * launches; later launches go untimed).  pm_kernel_timing_read synchronises
 * on the recorded events, returns per-slot totals and launch counts (slots:
 * 0 scalar field FP64, 1 scalar field FP32, 2 Poisson FP64, 3 Poisson FP32
 * for half-sweeps; 4..7 the same for fused sweeps) and clears them.  Not for
 * concurrent use from several threads while timing is on. */
int pm_kernel_timing_enable(int on);
int pm_kernel_timing_read(double *total_ms /* HOST [8] */, long long *launches /* HOST [8] */);

const char *pm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PMEFT_H */
