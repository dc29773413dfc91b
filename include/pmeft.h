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
 * and the coarsest-grid solve in FP64. */
typedef enum { PM_PREC_F64 = 0, PM_PREC_MIXED = 1 } pm_prec;

/* Initial guess of a solve: zero; the values passed in the output array
 * (e.g. the previous time step, Sec. 3.5.1); or the linearised solution
 * lap chi = mu_chi s delta (Sec. 3.5.1, first time step). */
typedef enum { PM_GUESS_ZERO = 0, PM_GUESS_GIVEN = 1, PM_GUESS_LINEAR = 2 } pm_guess;

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
} pm_mg_opts;

typedef struct {
    int status;                 /* PM_OK or PM_ENOCONV / PM_ENONFINITE */
    int vcycles;                /* V-cycles performed */
    double rel_residual;        /* of the returned iterate */
    double residual_hist[64];   /* rel. residual before V-cycle i (i < 64) */
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
 * grid-only calls). */
size_t pm_workspace_bytes(int ng, long long np, pm_dtype dtype, pm_prec prec);

/* CIC deposit (Sec. 3.6.2): rho_c = (ng^3/np) sum_p W(x_p - x_c), the tent
 * W = prod_d max(0, 1 - |dx_d|/h) with periodic wrap.  pos: SoA 3 x np in
 * [0,1); rho: ng^3 out, density in units of the mean.  Accumulation is in
 * 2^-40 fixed point, so the result does not depend on particle order. */
int pm_deposit(const void *pos, long long np, pm_dtype dtype, int ng, void *rho,
               void *ws, size_t ws_bytes, pm_stream_t stream);

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
 * outputs and, with guess GIVEN, carry the previous step's fields in. */
int pm_step(void *pos, void *vel, long long np, int ng, pm_dtype dtype, const pm_eft_params *p /* HOST */,
            const pm_mg_opts *poisson_opts /* HOST */, const pm_mg_opts *scalar_opts /* HOST */,
            double dt_kick, double dt_drift, void *psi, void *chi, pm_step_report *rep /* HOST, nullable */,
            void *ws, size_t ws_bytes, pm_stream_t stream);

/* ---- Learned warm start ------------------------------------------------
 * A 3-level 3D U-Net maps the density and (alpha_B0, alpha_M0, a) to an
 * initial scalar field; multigrid then finishes the solve as usual (pass the
 * result with PM_GUESS_GIVEN).  Input channels: standardised ln(rho + 1e-3)
 * and the three parameters broadcast; 3x3x3 periodic convolutions with ReLU
 * (16-16 / 32-32 / 64-64 channels on grids n, n/2, n/4), 2x2x2 average
 * pooling, nearest-neighbour upsampling, skip concatenations (96 -> 32,
 * 48 -> 16) and a 1x1x1 head.  The output yhat is the field in units of
 * h^2 s mu_chi: chi0 = h^2 s mu_chi (yhat - <yhat>).  Convolutions run on the
 * matrix cores in BF16 with FP32 accumulation; activations are BF16.
 *
 * Parameters: one FP32 device array of ws_unet_param_count() values: for each
 * convolution in order (l1a 4->16, l1b 16->16, l2a 16->32, l2b 32->32, l3a
 * 32->64, l3b 64->64, l4a 96->32, l4b 32->32, l5a 48->16, l5b 16->16) its
 * weight W[27][cin][cout] (tap t = (di+1)*9 + (dj+1)*3 + (dk+1) for the
 * neighbour offset (di, dj, dk)) followed by its bias[cout]; then the head's
 * 16 weights and 1 bias.  ng must be a multiple of 64. */
long long ws_unet_param_count(void);
size_t ws_unet_workspace_bytes(int ng, int training);

/* Forward pass.  rho: ng^3 FP64 density (natural order); yhat_out: ng^3 FP32
 * or NULL; chi_out: ng^3 of `dtype` (the initial field chi0) or NULL. */
int ws_unet_forward(const float *params, const double *rho, int ng, const pm_eft_params *p /* HOST */,
                    float *yhat_out, void *chi_out, pm_dtype dtype, void *ws, size_t ws_bytes, pm_stream_t stream);

/* One training step on one sample: forward, MSE loss against the target
 * field chi_target (ng^3 FP64, converted to units of h^2 s mu_chi),
 * backward, and (if lr > 0) an Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias correction with `step` >= 1) on the FP32 params with moment arrays
 * adam_m, adam_v.  grad_out (param_count FP32, nullable) receives the
 * gradients; *loss (HOST, nullable) the sample's loss (this call then
 * synchronises the stream).  Weight gradients accumulate with FP32 atomics,
 * so their last bits depend on scheduling. */
int ws_unet_train_step(float *params, float *adam_m, float *adam_v, long long step, double lr, const double *rho,
                       const double *chi_target, int ng, const pm_eft_params *p /* HOST */, float *grad_out,
                       double *loss /* HOST */, void *ws, size_t ws_bytes, pm_stream_t stream);

/* One 3x3x3 periodic convolution on BF16 channels-last tensors with FP32
 * output (for testing the kernels): mode 0 forward out[n^3][cout] =
 * b + conv(x); mode 1 input gradient out[n^3][cin] from dy[n^3][cout]; mode
 * 2 weight gradient out[27][cin][cout] from x and dy.  w: FP32 W[27][cin][cout]
 * (device); ws: at least 2 * 27 * pad16(cin) * pad16(cout) * 2 + 512 bytes. */
int ws_conv3(int mode, int n, int cin, int cout, const void *x_bf16, const void *dy_bf16, const float *w,
             const float *b, float *out, void *ws, size_t ws_bytes, pm_stream_t stream);

/* Measurement hooks.  While enabled, each launch of the finest-level
 * red-black smoother (one colour per launch) is bracketed by HIP events on
 * the stream it runs on (a fixed pool of 16384 launches; later launches go
 * untimed).  pm_kernel_timing_read synchronises on the recorded events,
 * returns per-slot totals and launch counts (slots: 0 scalar field FP64,
 * 1 scalar field FP32, 2 Poisson FP64, 3 Poisson FP32) and clears them.
 * Not for concurrent use from several threads while timing is on. */
int pm_kernel_timing_enable(int on);
int pm_kernel_timing_read(double *total_ms /* HOST [4] */, long long *launches /* HOST [4] */);

const char *pm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PMEFT_H */
