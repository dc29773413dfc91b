/*
 * Oracle: plain FP64 FAS multigrid for the code-unit scalar-field equation.
 * TEST INFRASTRUCTURE ONLY -- used by tests/, the smoke check and the CPU
 * baseline; the product path never links or calls it.
 *
 * Equation (eq. chi_scm, Sec. 3.1), per cell, with the discretisation of
 * Sec. 3.2.1 (7-point Laplacian, 3-point second derivatives, 4-point cross
 * derivatives) and the operator splitting of Sec. 3.2.2 (w = 1/3):
 *
 *     nu L - xi s delta - K [ (2/3) L^2 - T ] = 0 ,
 *
 * where L is the discrete Laplacian of chi and T the squared traceless part
 * of the discrete Hessian, which does not contain the centre cell.  With
 * G = K T - b (b = xi s delta) the branch that is continuous with the
 * linear solution (Sec. 3.2.1, minus root) is
 *
 *     Lq(G) = -2 G / (nu + sqrt(nu^2 + (8/3) K G)) ,
 *
 * and in void cells, where the spherical-cell existence condition of Sec.
 * 3.3 fails, the discriminant is set to zero, i.e. Lq = 3 nu / (4 K) (see
 * root_lap).  On a periodic grid the quadratic-root
 * Laplacian has its mean subtracted (Sec. 3.2.2), so the discrete system is
 *
 *     lap_h chi = Lq(G(chi)) - <Lq(G(chi))> ,   <chi> = 0 .
 *
 * Smoother: Jacobi (Sec. 3.4) with the Newton update of Sec. 3.2.2,
 * chi_new = chi_old - (L~ - L_bar)/(-6/h^2) = (S - h^2 L_bar)/6, applied with
 * the under-relaxation 0.6 chi* + 0.4 chi of Sec. 3.5.1.  Multigrid: FAS
 * V-cycle (Sec. 3.4), 8-child average restriction, cell-centred trilinear
 * prolongation of the coarse correction.
 *
 * The same routine solves a linear Poisson problem lap u = b by passing
 * nu = 1, K = 0.
 *
 * Grids are cell centred; each level stores chi with one ghost layer,
 * (n+2)^3 values, filled either periodically or from given Dirichlet values
 * (zero for the coarse-grid correction).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n;
    double h;
    double *u;     /* (n+2)^3 chi with ghosts */
    double *gval;  /* (n+2)^3 Dirichlet ghost values, or NULL (periodic) */
    double *b;     /* n^3 source b = xi s delta */
    double *tau;   /* n^3 FAS source (zero on the finest level) */
    double *u0;    /* n^3 restricted fine chi, kept for the correction */
    double *lq;    /* n^3 scratch: quadratic-root Laplacian */
    double *w;     /* n^3 scratch */
} level_t;

typedef struct {
    int periodic;
    double nu, K, omega;
    int npre, npost;
    long long clamped;
} params_t;

static inline long pidx(int n, int i, int j, int k)
{
    return ((long)(i + 1) * (n + 2) + (j + 1)) * (n + 2) + (k + 1);
}

static inline long cidx(int n, int i, int j, int k)
{
    return ((long)i * n + j) * n + k;
}

static inline int wrap(int i, int n)
{
    return (i % n + n) % n;
}

/* Fill the ghost layer: periodic images, or the stored Dirichlet values
 * (NULL gval with periodic == 0 means zero ghosts). */
static void fill_ghost_cell(level_t *L, int periodic, int zero_ghosts, int i, int j, int k)
{
    int n = L->n;
    long p = pidx(n, i, j, k);
    if (periodic)
        L->u[p] = L->u[pidx(n, wrap(i, n), wrap(j, n), wrap(k, n))];
    else if (zero_ghosts || L->gval == NULL)
        L->u[p] = 0.0;
    else
        L->u[p] = L->gval[p];
}

static void fill_ghosts(level_t *L, int periodic, int zero_ghosts)
{
    int n = L->n;
    for (int i = -1; i <= n; i++)
        for (int j = -1; j <= n; j++) {
            if (i < 0 || i >= n || j < 0 || j >= n) {
                for (int k = -1; k <= n; k++)
                    fill_ghost_cell(L, periodic, zero_ghosts, i, j, k);
            } else {
                fill_ghost_cell(L, periodic, zero_ghosts, i, j, -1);
                fill_ghost_cell(L, periodic, zero_ghosts, i, j, n);
            }
        }
}

/* Face sum S, per-axis face sums and the centre-free shear T at one cell. */
static inline void local_terms(const double *u, int n, int i, int j, int k, double h,
                               double *S, double *T)
{
    long c = pidx(n, i, j, k);
    long sx = (long)(n + 2) * (n + 2), sy = n + 2, sz = 1;
    double ax = u[c + sx] + u[c - sx];
    double ay = u[c + sy] + u[c - sy];
    double az = u[c + sz] + u[c - sz];
    double dxy = (u[c + sx + sy] - u[c + sx - sy] - u[c - sx + sy] + u[c - sx - sy]) / (4.0 * h * h);
    double dxz = (u[c + sx + sz] - u[c + sx - sz] - u[c - sx + sz] + u[c - sx - sz]) / (4.0 * h * h);
    double dyz = (u[c + sy + sz] - u[c + sy - sz] - u[c - sy + sz] + u[c - sy - sz]) / (4.0 * h * h);
    double h4 = h * h * h * h;
    /* D_xx - D_yy = (ax - ay)/h^2, etc.: the centre value cancels. */
    double t_diag = ((ax - ay) * (ax - ay) + (ay - az) * (ay - az) + (az - ax) * (az - ax)) / (3.0 * h4);
    *S = ax + ay + az;
    *T = t_diag + 2.0 * (dxy * dxy + dxz * dxz + dyz * dyz);
}

/* Root of -(2/3) K L^2 + nu L + G = 0 on the linear branch, G = K T - b.
 *
 * Void cells (Sec. 3.3): treating the cell's mass as spherically symmetric,
 * a real solution exists only if nu^2 - (8/3) K b >= 0 (the condition
 * nu^2 - 2 A C4 xi >= 0 with A taken from the cell's own delta).  Where it
 * fails the discriminant is set to zero, so the root is the vertex
 * 3 nu / (4 K).  In every other cell the discriminant
 * nu^2 + (8/3) K G = (nu^2 - (8/3) K b) + (8/3) K^2 T is non-negative. */
static inline double root_lap(double b, double T, double nu, double K, int *clamped)
{
    double dsph = nu * nu - (8.0 / 3.0) * K * b;
    if (dsph < 0.0) {
        *clamped = 1;
        return 3.0 * nu / (4.0 * K);
    }
    double G = K * T - b;
    double disc = dsph + (8.0 / 3.0) * K * K * T;
    return -2.0 * G / (nu + sqrt(disc));
}

/* lq[c] = Lq(G(u)) + tau[c] for every cell; returns its mean. u's ghosts must
 * be current. */
static double eval_lq(level_t *L, const params_t *P, long long *nclamp)
{
    int n = L->n;
    double sum = 0.0;
    long long ncl = 0;
#pragma omp parallel for reduction(+ : sum, ncl) schedule(static) if (n >= 24)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                double S, T;
                int cl = 0;
                local_terms(L->u, n, i, j, k, L->h, &S, &T);
                long c = cidx(n, i, j, k);
                double v = root_lap(L->b[c], T, P->nu, P->K, &cl) + L->tau[c];
                L->lq[c] = v;
                sum += v;
                ncl += cl;
            }
    if (nclamp)
        *nclamp = ncl;
    return sum / ((double)n * n * n);
}

/* One damped Jacobi sweep of the Newton update. */
static void jacobi_sweep(level_t *L, const params_t *P, int zero_ghosts)
{
    int n = L->n;
    double h2 = L->h * L->h;
    fill_ghosts(L, P->periodic, zero_ghosts);
    double mean = eval_lq(L, P, NULL);
    double c = P->periodic ? mean : 0.0;
#pragma omp parallel for schedule(static) if (n >= 24)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long p = pidx(n, i, j, k);
                double S = L->u[p + (long)(n + 2) * (n + 2)] + L->u[p - (long)(n + 2) * (n + 2)] +
                           L->u[p + n + 2] + L->u[p - (n + 2)] + L->u[p + 1] + L->u[p - 1];
                long q = cidx(n, i, j, k);
                double lbar = L->lq[q] - c;
                double star = (S - h2 * lbar) / 6.0;
                L->w[q] = (1.0 - P->omega) * L->u[p] + P->omega * star;
            }
#pragma omp parallel for schedule(static) if (n >= 24)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                L->u[pidx(n, i, j, k)] = L->w[cidx(n, i, j, k)];
}

/* r = Lq + tau - <Lq + tau> - lap u  (periodic) or Lq + tau - lap u. Returns
 * sum r^2. */
static double residual(level_t *L, const params_t *P, double *r, int zero_ghosts, long long *nclamp)
{
    int n = L->n;
    double h2 = L->h * L->h;
    fill_ghosts(L, P->periodic, zero_ghosts);
    double mean = eval_lq(L, P, nclamp);
    double c = P->periodic ? mean : 0.0;
    double ss = 0.0;
#pragma omp parallel for reduction(+ : ss) schedule(static) if (n >= 24)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long p = pidx(n, i, j, k);
                double S = L->u[p + (long)(n + 2) * (n + 2)] + L->u[p - (long)(n + 2) * (n + 2)] +
                           L->u[p + n + 2] + L->u[p - (n + 2)] + L->u[p + 1] + L->u[p - 1];
                double lap = (S - 6.0 * L->u[p]) / h2;
                long q = cidx(n, i, j, k);
                double v = L->lq[q] - c - lap;
                r[q] = v;
                ss += v * v;
            }
    return ss;
}

/* Average of the 8 children of each coarse cell. */
static void restrict_avg(int nc, const double *fine, double *coarse)
{
    int nf = 2 * nc;
#pragma omp parallel for schedule(static) if (nc >= 24)
    for (int I = 0; I < nc; I++)
        for (int J = 0; J < nc; J++)
            for (int K = 0; K < nc; K++) {
                double s = 0.0;
                for (int a = 0; a < 2; a++)
                    for (int b = 0; b < 2; b++)
                        for (int c = 0; c < 2; c++)
                            s += fine[cidx(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
                coarse[cidx(nc, I, J, K)] = 0.125 * s;
            }
}

static void vcycle(level_t *lv, int l, int nlev, params_t *P);

/* Solve the coarsest level by repeated sweeps. */
static void coarsest_solve(level_t *L, params_t *P, int zero_ghosts)
{
    int n = L->n;
    double r0 = sqrt(residual(L, P, L->w, zero_ghosts, NULL));
    for (int it = 0; it < 20000; it++) {
        jacobi_sweep(L, P, zero_ghosts);
        if ((it & 15) == 15) {
            double r = sqrt(residual(L, P, L->w, zero_ghosts, NULL));
            if (r <= 1e-13 * r0 || r < 1e-300)
                break;
        }
    }
    (void)n;
}

/* Cell-centred trilinear interpolation of the coarse correction, added to
 * the fine interior. */
static void prolong_add(level_t *F, level_t *C, int periodic)
{
    int nc = C->n, nf = F->n;
    /* e = u_H - u0_H on the coarse grid, with ghosts (periodic wrap or 0). */
    double *e = (double *)malloc(sizeof(double) * (size_t)(nc + 2) * (nc + 2) * (nc + 2));
    for (int i = -1; i <= nc; i++)
        for (int j = -1; j <= nc; j++)
            for (int k = -1; k <= nc; k++) {
                long p = pidx(nc, i, j, k);
                int in = (i >= 0 && i < nc && j >= 0 && j < nc && k >= 0 && k < nc);
                if (in)
                    e[p] = C->u[p] - C->u0[cidx(nc, i, j, k)];
                else if (periodic) {
                    int ii = wrap(i, nc), jj = wrap(j, nc), kk = wrap(k, nc);
                    e[p] = C->u[pidx(nc, ii, jj, kk)] - C->u0[cidx(nc, ii, jj, kk)];
                } else
                    e[p] = 0.0;
            }
#pragma omp parallel for schedule(static) if (nf >= 24)
    for (int i = 0; i < nf; i++)
        for (int j = 0; j < nf; j++)
            for (int k = 0; k < nf; k++) {
                int I = i >> 1, J = j >> 1, K = k >> 1;
                int di = (i & 1) ? 1 : -1, dj = (j & 1) ? 1 : -1, dk = (k & 1) ? 1 : -1;
                double v = 0.0;
                for (int a = 0; a < 2; a++)
                    for (int b = 0; b < 2; b++)
                        for (int c = 0; c < 2; c++) {
                            double wgt = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            v += wgt * e[pidx(nc, I + a * di, J + b * dj, K + c * dk)];
                        }
                F->u[pidx(nf, i, j, k)] += v;
            }
    free(e);
}

/* tau_H = R r_h + lap_H(R u_h) - Lq_H(R u_h): the FAS coarse source. */
static void fas_coarse_source(level_t *F, level_t *C, params_t *P, int zero_ghosts_c)
{
    int nc = C->n;
    double h2 = C->h * C->h;
    /* R r_h is already in C->tau; C->u interior holds R u_h. */
    double *rr = C->w;
    memcpy(rr, C->tau, sizeof(double) * (size_t)nc * nc * nc);
    memset(C->tau, 0, sizeof(double) * (size_t)nc * nc * nc);
    fill_ghosts(C, P->periodic, zero_ghosts_c);
    eval_lq(C, P, NULL); /* lq = Lq_H(R u) since tau = 0 here */
#pragma omp parallel for schedule(static) if (nc >= 24)
    for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++)
            for (int k = 0; k < nc; k++) {
                long p = pidx(nc, i, j, k);
                double S = C->u[p + (long)(nc + 2) * (nc + 2)] + C->u[p - (long)(nc + 2) * (nc + 2)] +
                           C->u[p + nc + 2] + C->u[p - (nc + 2)] + C->u[p + 1] + C->u[p - 1];
                double lap = (S - 6.0 * C->u[p]) / h2;
                long q = cidx(nc, i, j, k);
                C->tau[q] = rr[q] + lap - C->lq[q];
            }
    (void)F;
}

/* V-cycle on level l (0 = finest).  On coarse levels of a Dirichlet problem
 * the correction equation is solved with the coarse ghosts held at the
 * restricted boundary values, which cancel in the FAS source. */
static void vcycle(level_t *lv, int l, int nlev, params_t *P)
{
    level_t *L = &lv[l];
    int zg = 0; /* ghosts: periodic, or the level's Dirichlet values */
    if (l == nlev - 1) {
        coarsest_solve(L, P, zg);
        return;
    }
    for (int s = 0; s < P->npre; s++)
        jacobi_sweep(L, P, zg);
    level_t *C = &lv[l + 1];
    int nc = C->n;
    residual(L, P, L->w, zg, NULL);
    restrict_avg(nc, L->w, C->tau);
    /* R u_h into the coarse interior and u0 */
    {
        int nf = L->n;
        double *ui = (double *)malloc(sizeof(double) * (size_t)nf * nf * nf);
        for (int i = 0; i < nf; i++)
            for (int j = 0; j < nf; j++)
                for (int k = 0; k < nf; k++)
                    ui[cidx(nf, i, j, k)] = L->u[pidx(nf, i, j, k)];
        restrict_avg(nc, ui, C->u0);
        free(ui);
        for (int i = 0; i < nc; i++)
            for (int j = 0; j < nc; j++)
                for (int k = 0; k < nc; k++)
                    C->u[pidx(nc, i, j, k)] = C->u0[cidx(nc, i, j, k)];
    }
    fas_coarse_source(L, C, P, zg);
    vcycle(lv, l + 1, nlev, P);
    prolong_add(L, C, P->periodic);
    for (int s = 0; s < P->npost; s++)
        jacobi_sweep(L, P, zg);
}

static double norm2(const double *x, long n)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static) if (n >= 32768)
    for (long i = 0; i < n; i++)
        s += x[i] * x[i];
    return sqrt(s);
}

/*
 * Solve on an n^3 grid (n = 2^k * m, coarsened while n is even and n/2 >= 4).
 *   b      : n^3 source xi s delta (C order, k fastest)
 *   gval   : (n+2)^3 Dirichlet ghost values of chi, or NULL for periodic
 *   chi    : n^3 in: initial guess; out: solution (mean-free if periodic)
 *   report : [0] relative residual ||r||/||b/nu||, [1] V-cycles,
 *            [2] clamped cells, [3] status (0 ok, -3 not converged)
 * Returns the status.
 */
int orc_chi_solve(int n, double h, const double *b, const double *gval, double nu, double K,
                  double tol, int max_cycles, int npre, int npost, double omega,
                  double *chi, double *report)
{
    params_t P = {gval == NULL, nu, K, omega, npre, npost, 0};
    int nlev = 1;
    for (int m = n; m % 2 == 0 && m / 2 >= 4; m /= 2)
        nlev++;
    level_t *lv = (level_t *)calloc((size_t)nlev, sizeof(level_t));
    int m = n;
    double hh = h;
    for (int l = 0; l < nlev; l++) {
        size_t pc = (size_t)(m + 2) * (m + 2) * (m + 2), cc = (size_t)m * m * m;
        lv[l].n = m;
        lv[l].h = hh;
        lv[l].u = (double *)calloc(pc, sizeof(double));
        lv[l].b = (double *)calloc(cc, sizeof(double));
        lv[l].tau = (double *)calloc(cc, sizeof(double));
        lv[l].u0 = (double *)calloc(cc, sizeof(double));
        lv[l].lq = (double *)calloc(cc, sizeof(double));
        lv[l].w = (double *)calloc(cc, sizeof(double));
        lv[l].gval = NULL;
        m /= 2;
        hh *= 2.0;
    }
    memcpy(lv[0].b, b, sizeof(double) * (size_t)n * n * n);
    for (int l = 1; l < nlev; l++)
        restrict_avg(lv[l].n, lv[l - 1].b, lv[l].b);
    if (gval) {
        /* Dirichlet ghosts: the given values on the finest level; on coarse
         * levels the ghosts of the correction problem are held fixed, so any
         * consistent value works -- use the average of the adjacent fine
         * ghosts' images, approximated by sampling the finest ghost layer. */
        size_t pc0 = (size_t)(n + 2) * (n + 2) * (n + 2);
        lv[0].gval = (double *)malloc(sizeof(double) * pc0);
        memcpy(lv[0].gval, gval, sizeof(double) * pc0);
        for (int l = 1; l < nlev; l++) {
            int mc = lv[l].n, mf = lv[l - 1].n;
            size_t pc = (size_t)(mc + 2) * (mc + 2) * (mc + 2);
            lv[l].gval = (double *)calloc(pc, sizeof(double));
            for (int i = -1; i <= mc; i++)
                for (int j = -1; j <= mc; j++)
                    for (int k = -1; k <= mc; k++) {
                        int fi = i < 0 ? -1 : (i >= mc ? mf : 2 * i);
                        int fj = j < 0 ? -1 : (j >= mc ? mf : 2 * j);
                        int fk = k < 0 ? -1 : (k >= mc ? mf : 2 * k);
                        lv[l].gval[pidx(mc, i, j, k)] = lv[l - 1].gval[pidx(mf, fi, fj, fk)];
                    }
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                lv[0].u[pidx(n, i, j, k)] = chi[cidx(n, i, j, k)];

    long cc0 = (long)n * n * n;
    double bnorm = norm2(lv[0].b, cc0) / fabs(nu);
    if (bnorm == 0.0)
        bnorm = 1.0;
    int status = -3, cyc;
    double rel = 0.0;
    long long ncl = 0;
    for (cyc = 0; cyc <= max_cycles; cyc++) {
        rel = sqrt(residual(&lv[0], &P, lv[0].w, 0, &ncl)) / bnorm;
        if (!(rel == rel)) {
            status = -4;
            break;
        }
        if (rel <= tol) {
            status = 0;
            break;
        }
        if (cyc == max_cycles)
            break;
        vcycle(lv, 0, nlev, &P);
    }
    double mean = 0.0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                mean += lv[0].u[pidx(n, i, j, k)];
    mean = P.periodic ? mean / (double)cc0 : 0.0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                chi[cidx(n, i, j, k)] = lv[0].u[pidx(n, i, j, k)] - mean;
    report[0] = rel;
    report[1] = (double)(cyc > max_cycles ? max_cycles : cyc);
    report[2] = (double)ncl;
    report[3] = (double)status;
    for (int l = 0; l < nlev; l++) {
        free(lv[l].u);
        free(lv[l].b);
        free(lv[l].tau);
        free(lv[l].u0);
        free(lv[l].lq);
        free(lv[l].w);
        free(lv[l].gval);
    }
    free(lv);
    return status;
}

/*
 * Evaluate the discrete operator pieces at a given chi (no solve):
 *   lap (n^3), lq = Lq(G) (n^3, before mean subtraction), T (n^3),
 *   r = lq - <lq> - lap (periodic) or lq - lap (Dirichlet).
 * Any output pointer may be NULL.  Returns the number of clamped cells.
 */
long long orc_chi_operator(int n, double h, const double *b, const double *gval, double nu, double K,
                           const double *chi, double *lap, double *lq, double *T, double *r)
{
    level_t L;
    memset(&L, 0, sizeof(L));
    params_t P = {gval == NULL, nu, K, 0.0, 0, 0, 0};
    size_t pc = (size_t)(n + 2) * (n + 2) * (n + 2), cc = (size_t)n * n * n;
    L.n = n;
    L.h = h;
    L.u = (double *)calloc(pc, sizeof(double));
    L.b = (double *)malloc(sizeof(double) * cc);
    memcpy(L.b, b, sizeof(double) * cc);
    L.tau = (double *)calloc(cc, sizeof(double));
    L.lq = (double *)calloc(cc, sizeof(double));
    L.gval = gval ? (double *)gval : NULL;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                L.u[pidx(n, i, j, k)] = chi[cidx(n, i, j, k)];
    fill_ghosts(&L, P.periodic, 0);
    long long ncl = 0;
    double mean = eval_lq(&L, &P, &ncl);
    double c = P.periodic ? mean : 0.0;
    double h2 = h * h;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long p = pidx(n, i, j, k);
                long q = cidx(n, i, j, k);
                double S, Tv;
                local_terms(L.u, n, i, j, k, h, &S, &Tv);
                double lp = (S - 6.0 * L.u[p]) / h2;
                if (lap)
                    lap[q] = lp;
                if (lq)
                    lq[q] = L.lq[q];
                if (T)
                    T[q] = Tv;
                if (r)
                    r[q] = L.lq[q] - c - lp;
            }
    free(L.u);
    free(L.b);
    free(L.tau);
    free(L.lq);
    return ncl;
}
