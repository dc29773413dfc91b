// Multigrid kernels for the Poisson and scalar-field solves (gfx950).
//
// Discrete operator (Sec. 3.2): 7-point Laplacian, 3-point second
// derivatives, 4-point cross derivatives.  The scalar-field equation
// nu L - b - K [(2/3) L^2 - T] = 0 (eq. chi_scm after the operator splitting
// of Sec. 3.2.2 with w = 1/3; b = xi s delta) has the per-cell root
//   Lq = -2 G / (nu + sqrt(nu^2 + (8/3) K G)),  G = K T - b,
// on the branch continuous with the linear solution (Sec. 3.2.1).  Void
// cells (Sec. 3.3) are those where the spherical-cell existence condition
// nu^2 - (8/3) K b >= 0 fails; their discriminant is set to zero, giving
// Lq = 3 nu / (4 K).  Elsewhere the discriminant equals
// (nu^2 - (8/3) K b) + (8/3) K^2 T >= 0.  A level solves
//   lap x = Lq(x) + tau - <Lq(x) + tau>
// (tau = 0 on the finest level), the mean being the lagged one of the last
// half-sweeps (Sec. 3.2.2 subtracts the mean of the root Laplacian).
//
// The Newton update of Sec. 3.2.2 reduces to x <- (S - h^2 (Lq + tau - c))/6
// with S the face-neighbour sum; Lq does not depend on the centre cell.  The
// 12 edge neighbours of the scalar-field stencil have the cell's own colour,
// so each half-sweep reads its own colour from one buffer and writes the new
// values into another (no cell reads a value written in the same launch).
#include "mg_stencil.h"

#include <math.h>

#include <algorithm>

namespace pmeft {

namespace {
thread_local Group t_group;
}
const Group &cur_group() { return t_group; }
void set_cur_group(const Group &g) { t_group = g; }
GroupScope::GroupScope(const Group &g) : prev(t_group) { t_group = g; }
GroupScope::~GroupScope() { t_group = prev; }

// Per-thread stage of the finalize kernels: thread t adds, in order, the
// rows b = t, t + kBlock, ... (< nblocks) of the partials, each value q into
// acc[q].  All of a thread's rows are loaded (64 bytes each) before any is
// added, so the stage waits for memory once; rows past nblocks add +0, which
// leaves every sum bitwise what the row-by-row loop gives.
constexpr int kFinRows = kMaxBlocks / kBlock;
__device__ __forceinline__ void finalize_rows(const double *__restrict__ partials, int nblocks, double acc[8])
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 v[kFinRows][4];
#pragma unroll
    for (int u = 0; u < kFinRows; u++) {
        const int b = threadIdx.x + u * kBlock;
        const d2 *row = reinterpret_cast<const d2 *>(partials + (size_t)b * 8);
#pragma unroll
        for (int h = 0; h < 4; h++)
            v[u][h] = b < nblocks ? row[h] : d2{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < 8; q++)
        acc[q] = 0.0;
#pragma unroll
    for (int u = 0; u < kFinRows; u++)
#pragma unroll
        for (int q = 0; q < 8; q++)
            acc[q] += v[u][q >> 1][q & 1];
}

// One block: out[q] = sum over blocks b (in order) of partials[b * 8 + q].
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials, int nblocks, int nv,
                                                     double *__restrict__ out, Group grp)
{
    const long long go = group_offset(grp);
    partials = gshift(partials, go);
    out = gshift(out, go);
    __shared__ double sm[8][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double acc[8];
    finalize_rows(partials, nblocks, acc);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        if (q >= nv)
            break;
        double a = acc[q];
        for (int off = 32; off > 0; off >>= 1)
            a += __shfl_down(a, off, 64);
        if (lane == 0)
            sm[q][wid] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; w++)
            t += sm[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
}

void launch_finalize(const ReduceSlot &rs, const Span &sp, int nv, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, group_grid(1), dim3(kBlock), 0, st, (const double *)rs.partials, (int)sp.nblocks, nv,
                       out, cur_group());
}

// k_finalize for the six sums of the mixed-precision outer residual, which
// also writes the next lagged means (lag64[0] = sum 2, lag64[1] = 0,
// lag32[0..1] = sums 4, 5), saving the copies a separate launch would need.
__global__ __launch_bounds__(kBlock) void k_finalize_outer(const double *__restrict__ partials, int nblocks,
                                                           double *__restrict__ out, double *__restrict__ lag64,
                                                           double *__restrict__ lag32, Group grp)
{
    const long long go = group_offset(grp);
    partials = gshift(partials, go);
    out = gshift(out, go);
    lag64 = gshift(lag64, go);
    lag32 = gshift(lag32, go);
    constexpr int nv = 6;
    __shared__ double sm[nv][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double acc[8];
    finalize_rows(partials, nblocks, acc);
#pragma unroll
    for (int q = 0; q < nv; q++) {
        double a = acc[q];
        for (int off = 32; off > 0; off >>= 1)
            a += __shfl_down(a, off, 64);
        if (lane == 0)
            sm[q][wid] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; w++)
            t += sm[threadIdx.x][w];
        out[threadIdx.x] = t;
        if (threadIdx.x == 2)
            lag64[0] = t;
        else if (threadIdx.x == 4 || threadIdx.x == 5)
            lag32[threadIdx.x - 4] = t;
    } else if (threadIdx.x == nv) {
        lag64[1] = 0.0;
    }
}

// ------------------------------------------------------- residual/restrict
template <typename T, typename R, bool NL>
__device__ __forceinline__ T cell_residual(const LevelView<R> &F, const R *xr, const R *xb, int c, int i, int j, int kh,
                                           unsigned e, T cmean, const SolveConsts &sc, T &lq_plus_tau, int &isv)
{
    const R *own = c ? xb : xr;
    const R *oth = c ? xr : xb;
    T tsh;
    const T S = stencil_terms<T, R>(own, oth, F.n, F.nh, c, i, j, kh, NL, tsh);
    const T ih2 = (T)(1.0 / (F.h * F.h));
    const T b = (T)sc.beta * (T)(c ? F.db : F.dr)[e];
    const T lq = root_lap<T>(b, tsh * ih2 * ih2, sc, NL, isv);
    const R *tc = c ? F.tb : F.tr;
    const T v = lq + (tc ? (T)tc[e] : (T)0);
    const T lap = (S - (T)6 * (T)own[e]) * ih2;
    lq_plus_tau = v;
    return v - cmean - lap;
}

// Coarse cell e (natural order): residual of its 8 children, their average
// into the coarse tau, the average of the children's x into the coarse x and
// x0; acc += (sum r^2, sum r, sum Lq + tau, void cells).
template <typename R, bool NL>
__device__ __forceinline__ void restrict_cell(const LevelView<R> &F, const R *__restrict__ xr, const R *__restrict__ xb,
                                              double cm, const LevelView<R> &C, R *__restrict__ cxr,
                                              R *__restrict__ cxb, const SolveConsts &sc, unsigned e, double acc[4])
{
    const int nc = C.n, nch = C.nh;
    int I, J, K;
    split(e, nc, nc, I, J, K);
    const int cc = (I + J + K) & 1;
    const unsigned ec = ((unsigned)I * nc + J) * nch + (K >> 1);
    double sr = 0.0, sx = 0.0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int i = 2 * I + a, j = 2 * J + b;
            const unsigned ef = ((unsigned)i * F.n + j) * F.nh + K;
#pragma unroll
            for (int fc = 0; fc < 2; fc++) {
                // in the level's own precision (the FP32 levels of the mixed
                // solve need FP32 residuals only); sums in FP64
                R lqt_r;
                int isv;
                const double r = (double)cell_residual<R, R, NL>(F, xr, xb, fc, i, j, K, ef, (R)cm, sc, lqt_r, isv);
                const double lqt = (double)lqt_r;
                sr += r;
                sx += (double)(fc ? xb : xr)[ef];
                acc[0] += r * r;
                acc[1] += r;
                acc[2] += lqt;
                acc[3] += (double)isv;
            }
        }
    const R rx = (R)(0.125 * sx);
    (cc ? C.tb : C.tr)[ec] = (R)(0.125 * sr);
    (cc ? cxb : cxr)[ec] = rx;
    (cc ? C.x0b : C.x0r)[ec] = rx;
}

// One thread per coarse cell, in natural (I, J, K) order so that
// consecutive threads read consecutive fine elements: residual of its 8
// children, their average into the coarse tau, the average of the
// children's x into the coarse x and x0.
template <typename R, bool NL>
__global__ __launch_bounds__(kBlock) void k_residual_restrict(LevelView<R> F, const R *__restrict__ xr,
                                                              const R *__restrict__ xb, const double *__restrict__ csum,
                                                              LevelView<R> C, R *__restrict__ cxr,
                                                              R *__restrict__ cxb, ReduceSlot rs, SolveConsts sc,
                                                              Span sp, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    gshift_view(C, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    csum = gshift(csum, go);
    cxr = gshift(cxr, go);
    cxb = gshift(cxb, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    const double cm = (csum[0] + csum[1]) / (2.0 * (double)F.half);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    restrict_cell<R, NL>(F, xr, xb, cm, C, cxr, cxb, sc, e, acc);
    block_partials<4>(acc, rs, sp);
}

template <typename R>
void launch_residual_restrict(const LevelView<R> &F, const R *xr, const R *xb, const double *csum,
                              const LevelView<R> &C, R *cxr, R *cxb, ReduceSlot rs, SolveConsts sc, bool nonlinear,
                              hipStream_t st, bool norms, int tiled)
{
    Span spt;
    if (launch_residual_restrict_tiled<R>(F, xr, xb, csum, C, cxr, cxb, rs, sc, nonlinear, st, tiled, &spt)) {
        if (norms)
            launch_finalize(rs, spt, 4, rs.out, st);
        return;
    }
    const Span sp = make_span(2 * C.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_residual_restrict<R, true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb,
                           csum, C, cxr, cxb, rs, sc, sp, cur_group());
    else
        hipLaunchKernelGGL((k_residual_restrict<R, false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb,
                           csum, C, cxr, cxb, rs, sc, sp, cur_group());
    if (norms)
        launch_finalize(rs, sp, 4, rs.out, st);
}

// ------------------------------------------------------------ FAS source
// Element e of the level (both colours, colour 1 from half on): tau += lap x
// - Lq(x) unless accumulate_only; acc[colour] += Lq + tau.
template <typename R, bool NL>
__device__ __forceinline__ void fas_cell(const LevelView<R> &C, const R *__restrict__ xr, const R *__restrict__ xb,
                                         const SolveConsts &sc, unsigned e, int accumulate_only, double acc[2])
{
    const double ih2 = 1.0 / (C.h * C.h);
    const unsigned half = (unsigned)C.half;
    const int c = e >= half;
    const unsigned ec = e - (c ? half : 0u);
    int i, j, kh;
    split(ec, C.nh, C.n, i, j, kh);
    const R *own = c ? xb : xr;
    const R *oth = c ? xr : xb;
    double tsh;
    const double S = stencil_terms<double, R>(own, oth, C.n, C.nh, c, i, j, kh, NL, tsh);
    const double b = sc.beta * (double)(c ? C.db : C.dr)[ec];
    int isv;
    const double lq = root_lap<double>(b, tsh * ih2 * ih2, sc, NL, isv);
    R *tc = c ? C.tb : C.tr;
    double t = tc ? (double)tc[ec] : 0.0;
    if (!accumulate_only) {
        const double lap = (S - 6.0 * (double)own[ec]) * ih2;
        t += lap - lq;
        tc[ec] = (R)t;
        t = (double)(R)t;
    }
    acc[c] += lq + t;
}

// tau += lap x - Lq(x) (or, with accumulate_only, leave tau) and store the
// per-colour sums of Lq + tau.
template <typename R, bool NL>
__global__ __launch_bounds__(kBlock) void k_fas_tau(LevelView<R> C, const R *__restrict__ xr,
                                                    const R *__restrict__ xb, ReduceSlot rs, SolveConsts sc, Span sp,
                                                    int accumulate_only, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(C, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    double acc[2] = {0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    fas_cell<R, NL>(C, xr, xb, sc, e, accumulate_only, acc);
    block_partials<2>(acc, rs, sp);
}

template <typename R>
void launch_fas_tau(const LevelView<R> &C, const R *xr, const R *xb, double *csum, ReduceSlot rs, SolveConsts sc,
                    bool nonlinear, bool accumulate_only, hipStream_t st, int tiled, bool zero_iterate)
{
    const int acc_only = (accumulate_only || C.tr == nullptr) ? 1 : 0;
    Span spt;
    if (launch_fas_tau_tiled<R>(C, xr, xb, rs, sc, nonlinear, acc_only, st, tiled, &spt, zero_iterate)) {
        launch_finalize(rs, spt, 2, csum, st);
        return;
    }
    const Span sp = make_span(2 * C.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_fas_tau<R, true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, C, xr, xb, rs, sc, sp,
                           acc_only, cur_group());
    else
        hipLaunchKernelGGL((k_fas_tau<R, false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, C, xr, xb, rs, sc, sp,
                           acc_only, cur_group());
    launch_finalize(rs, sp, 2, csum, st);
}

// ------------------------------------------------------------- prolongation
template <typename R>
__device__ __forceinline__ double coarse_at(const R *cr, const R *cb, int nc, int nch, int I, int J, int K)
{
    const unsigned o = ((unsigned)I * nc + J) * nch + (K >> 1);
    return (double)(((I + J + K) & 1) ? cb[o] : cr[o]);
}

// Cell-centred trilinear prolongation, one thread per coarse cell (natural
// order): the 27 coarse values around it are interpolated axis by axis
// (weights 3/4, 1/4) to its 8 children.  CORR: add P (x_H - x0_H) to the
// fine iterate (coarse-grid correction); !CORR: write P x_H (full
// approximation, used to start full multigrid).
template <typename R, bool CORR>
__device__ __forceinline__ void prolong_cell(const LevelView<R> &F, R *__restrict__ xr, R *__restrict__ xb,
                                             const LevelView<R> &C, const R *__restrict__ cxr,
                                             const R *__restrict__ cxb, unsigned e);

template <typename R, bool CORR>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelView<R> F, R *__restrict__ xr, R *__restrict__ xb,
                                                    LevelView<R> C, const R *__restrict__ cxr,
                                                    const R *__restrict__ cxb, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    gshift_view(C, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    cxr = gshift(cxr, go);
    cxb = gshift(cxb, go);
    PM_SPAN_LOOP(e, sp)
    prolong_cell<R, CORR>(F, xr, xb, C, cxr, cxb, e);
}

template <typename R, bool CORR>
__device__ __forceinline__ void prolong_cell(const LevelView<R> &F, R *__restrict__ xr, R *__restrict__ xb,
                                             const LevelView<R> &C, const R *__restrict__ cxr,
                                             const R *__restrict__ cxb, unsigned e)
{
    const int nc = C.n, nch = C.nh;
    {
        int I, J, K;
        split(e, nc, nc, I, J, K);
        const int Is[3] = {wrap_dn(I - 1, nc), I, wrap_up(I + 1, nc)};
        const int Js[3] = {wrap_dn(J - 1, nc), J, wrap_up(J + 1, nc)};
        const int Ks[3] = {wrap_dn(K - 1, nc), K, wrap_up(K + 1, nc)};
        double lk[3][3][2];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                double v[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    v[c] = coarse_at(cxr, cxb, nc, nch, Is[a], Js[b], Ks[c]);
                    if (CORR)
                        v[c] -= coarse_at(C.x0r, C.x0b, nc, nch, Is[a], Js[b], Ks[c]);
                }
                lk[a][b][0] = 0.75 * v[1] + 0.25 * v[0];
                lk[a][b][1] = 0.75 * v[1] + 0.25 * v[2];
            }
#pragma unroll
        for (int aa = 0; aa < 2; aa++)
#pragma unroll
            for (int bb = 0; bb < 2; bb++) {
                const int i = 2 * I + aa, j = 2 * J + bb;
                const unsigned ef = ((unsigned)i * F.n + j) * F.nh + K;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    double lj[3];
#pragma unroll
                    for (int a = 0; a < 3; a++)
                        lj[a] = 0.75 * lk[a][1][c] + 0.25 * lk[a][bb ? 2 : 0][c];
                    const double v = 0.75 * lj[1] + 0.25 * lj[aa ? 2 : 0];
                    R *x = ((aa + bb + c) & 1) ? xb : xr;
                    if (CORR)
                        x[ef] = (R)((double)x[ef] + v);
                    else
                        x[ef] = (R)v;
                }
            }
    }
}

template <typename R>
void launch_prolong_correct(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                            hipStream_t st, int tiled)
{
    if (launch_prolong_tiled<R>(F, xr, xb, C, cxr, cxb, true, st, tiled))
        return;
    const Span sp = make_span(2 * C.half);
    hipLaunchKernelGGL((k_prolong<R, true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, C, cxr, cxb, sp,
                       cur_group());
}

template <typename R>
void launch_prolong_full(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                         hipStream_t st, int tiled)
{
    if (launch_prolong_tiled<R>(F, xr, xb, C, cxr, cxb, false, st, tiled))
        return;
    const Span sp = make_span(2 * C.half);
    hipLaunchKernelGGL((k_prolong<R, false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, C, cxr, cxb, sp,
                       cur_group());
}

// ------------------------------------------------------------- coarsest
// One workgroup, n <= 6: red-black Gauss-Seidel in FP64 in LDS with the exact
// mean of Lq + tau recomputed before every half-sweep, until the largest
// update falls below kCoarseTol of the largest value or `sweeps` sweeps are
// done (the coarse correction needs far less than the V-cycle's per-cycle
// reduction).
constexpr int kCoarseMax = 216;
constexpr double kCoarseTol = 1e-10;
// ... or below kCoarseRel of the largest accumulated change of the solve (the
// coarse-grid correction is then resolved to about 1%, well below the
// V-cycle's per-cycle reduction of about a tenth)
constexpr double kCoarseRel = 1e-2;

// Device part, for any block size >= n^3 that is a multiple of 64 (all
// threads of the block must call it).
template <typename R, bool NL>
__device__ void coarsest_solve(const LevelView<R> &C, R *xr, R *xb, const SolveConsts &sc, int sweeps, double tol)
{
    __shared__ double x[kCoarseMax], d[kCoarseMax], t[kCoarseMax];
    __shared__ double red[16][2], cred[16];
    const int n = C.n, nh = C.nh, N = n * n * n;
    const int q = threadIdx.x, nw = blockDim.x >> 6;
    int i = 0, j = 0, k = 0, col = 0;
    long long off = 0;
    if (q < N) {
        i = q / (n * n);
        j = (q / n) % n;
        k = q % n;
        col = (i + j + k) & 1;
        off = ((long long)i * n + j) * nh + (k >> 1);
        x[q] = (double)(col ? xb : xr)[off];
        d[q] = (double)(col ? C.db : C.dr)[off];
        const R *tc = col ? C.tb : C.tr;
        t[q] = tc ? (double)tc[off] : 0.0;
    }
    __syncthreads();
    const double xstart = q < N ? x[q] : 0.0;
    const double h2 = C.h * C.h, ih2 = 1.0 / h2;
    auto at = [&](int a, int b, int c) -> double {
        a = a < 0 ? a + n : (a >= n ? a - n : a);
        b = b < 0 ? b + n : (b >= n ? b - n : b);
        c = c < 0 ? c + n : (c >= n ? c - n : c);
        return x[(a * n + b) * n + c];
    };
    const int lane = q & 63, wid = q >> 6;
    for (int sw = 0; sw < sweeps; sw++) {
        double maxd = 0.0;
        for (int colour = 0; colour < 2; colour++) {
            double S = 0.0, val = 0.0;
            if (q < N) {
                const double ax = at(i + 1, j, k) + at(i - 1, j, k);
                const double ay = at(i, j + 1, k) + at(i, j - 1, k);
                const double az = at(i, j, k + 1) + at(i, j, k - 1);
                S = ax + ay + az;
                double tsh = 0.0;
                if (NL) {
                    const double dxy = at(i + 1, j + 1, k) - at(i + 1, j - 1, k) - at(i - 1, j + 1, k) + at(i - 1, j - 1, k);
                    const double dxz = at(i + 1, j, k + 1) - at(i + 1, j, k - 1) - at(i - 1, j, k + 1) + at(i - 1, j, k - 1);
                    const double dyz = at(i, j + 1, k + 1) - at(i, j + 1, k - 1) - at(i, j - 1, k + 1) + at(i, j - 1, k - 1);
                    tsh = ((ax - ay) * (ax - ay) + (ay - az) * (ay - az) + (az - ax) * (az - ax)) / 3.0 +
                          0.125 * (dxy * dxy + dxz * dxz + dyz * dyz);
                }
                int isv;
                val = root_lap<double>(sc.beta * d[q], tsh * ih2 * ih2, sc, NL, isv) + t[q];
            }
            double s = val;
            for (int o = 32; o > 0; o >>= 1)
                s += __shfl_down(s, o, 64);
            if (lane == 0)
                red[wid][0] = s;
            __syncthreads();
            double tot = 0.0;
            for (int w = 0; w < nw; w++)
                tot += red[w][0];
            const double cmean = tot / (double)N;
            double nx = 0.0;
            if (q < N && col == colour) {
                nx = (S - h2 * (val - cmean)) / 6.0;
                maxd = fmax(maxd, fabs(nx - x[q]));
            }
            __syncthreads();
            if (q < N && col == colour)
                x[q] = nx;
            __syncthreads();
        }
        double mx = 0.0, md = maxd, mc = 0.0;
        if (q < N) {
            mx = fabs(x[q]);
            mc = fabs(x[q] - xstart);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mx = fmax(mx, __shfl_down(mx, o, 64));
            md = fmax(md, __shfl_down(md, o, 64));
            mc = fmax(mc, __shfl_down(mc, o, 64));
        }
        if (lane == 0) {
            red[wid][0] = mx;
            red[wid][1] = md;
            cred[wid] = mc;
        }
        __syncthreads();
        double gx = 0.0, gd = 0.0, gc = 0.0;
        for (int w = 0; w < nw; w++) {
            gx = fmax(gx, red[w][0]);
            gd = fmax(gd, red[w][1]);
            gc = fmax(gc, cred[w]);
        }
        __syncthreads();
        if (gd <= tol * gx || gd <= kCoarseRel * gc)
            break;
    }
    if (q < N)
        (col ? xb : xr)[off] = (R)x[q];
    __syncthreads();
}

// The 4^3 coarsest grid in one wavefront: lane q holds cell q = (i n + j) n + k
// and reads its neighbours with cross-lane shuffles, so a sweep needs no
// barrier.  Same iteration as coarsest_solve (red-black Gauss-Seidel with the
// exact mean of Lq + tau before every half-sweep, same stopping rules).
// Called by the 64 lanes of one wave.
template <typename R, bool NL>
__device__ void coarsest_wave(const LevelView<R> &C, R *xr, R *xb, const SolveConsts &sc, int sweeps, double tol)
{
    constexpr int n = 4, nh = 2;
    const int q = threadIdx.x & 63;
    const int i = q >> 4, j = (q >> 2) & 3, k = q & 3;
    const int col = (i + j + k) & 1;
    const long long off = ((long long)i * n + j) * nh + (k >> 1);
    double x = (double)(col ? xb : xr)[off];
    const double xstart = x;
    const double d = (double)(col ? C.db : C.dr)[off];
    const R *tc = col ? C.tb : C.tr;
    const double t = tc ? (double)tc[off] : 0.0;
    const double h2 = C.h * C.h, ih2 = 1.0 / h2;
    auto lane = [&](int a, int b, int c) { return (((a + n) & 3) << 4) | (((b + n) & 3) << 2) | ((c + n) & 3); };
    auto wsum = [](double v) {
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o, 64);
        return v;
    };
    auto wmax = [](double v) {
        for (int o = 32; o > 0; o >>= 1)
            v = fmax(v, __shfl_xor(v, o, 64));
        return v;
    };
    for (int sw = 0; sw < sweeps; sw++) {
        double maxd = 0.0;
        for (int colour = 0; colour < 2; colour++) {
            const double ax = __shfl(x, lane(i + 1, j, k), 64) + __shfl(x, lane(i - 1, j, k), 64);
            const double ay = __shfl(x, lane(i, j + 1, k), 64) + __shfl(x, lane(i, j - 1, k), 64);
            const double az = __shfl(x, lane(i, j, k + 1), 64) + __shfl(x, lane(i, j, k - 1), 64);
            const double S = ax + ay + az;
            double tsh = 0.0;
            if (NL) {
                const double dxy = __shfl(x, lane(i + 1, j + 1, k), 64) - __shfl(x, lane(i + 1, j - 1, k), 64) -
                                   __shfl(x, lane(i - 1, j + 1, k), 64) + __shfl(x, lane(i - 1, j - 1, k), 64);
                const double dxz = __shfl(x, lane(i + 1, j, k + 1), 64) - __shfl(x, lane(i + 1, j, k - 1), 64) -
                                   __shfl(x, lane(i - 1, j, k + 1), 64) + __shfl(x, lane(i - 1, j, k - 1), 64);
                const double dyz = __shfl(x, lane(i, j + 1, k + 1), 64) - __shfl(x, lane(i, j + 1, k - 1), 64) -
                                   __shfl(x, lane(i, j - 1, k + 1), 64) + __shfl(x, lane(i, j - 1, k - 1), 64);
                tsh = ((ax - ay) * (ax - ay) + (ay - az) * (ay - az) + (az - ax) * (az - ax)) / 3.0 +
                      0.125 * (dxy * dxy + dxz * dxz + dyz * dyz);
            }
            int isv;
            const double val = root_lap<double>(sc.beta * d, tsh * ih2 * ih2, sc, NL, isv) + t;
            const double cmean = wsum(val) / 64.0;
            if (col == colour) {
                const double nx = (S - h2 * (val - cmean)) / 6.0;
                maxd = fmax(maxd, fabs(nx - x));
                x = nx;
            }
        }
        const double gx = wmax(fabs(x)), gd = wmax(maxd), gc = wmax(fabs(x - xstart));
        if (gd <= tol * gx || gd <= kCoarseRel * gc)
            break;
    }
    (col ? xb : xr)[off] = (R)x;
}

template <typename R, bool NL>
__global__ __launch_bounds__(kBlock) void k_coarsest(LevelView<R> C, R *xr, R *xb, SolveConsts sc, int sweeps,
                                                     double tol, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(C, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    gconsts(sc, grp);
    if (C.n == 4) {
        if (threadIdx.x < 64)
            coarsest_wave<R, NL>(C, xr, xb, sc, sweeps, tol);
        return;
    }
    coarsest_solve<R, NL>(C, xr, xb, sc, sweeps, tol);
}

template <typename R>
void launch_coarsest(const LevelView<R> &C, R *xr, R *xb, SolveConsts sc, bool nonlinear, int sweeps, hipStream_t st)
{
    if (nonlinear)
        hipLaunchKernelGGL((k_coarsest<R, true>), group_grid(1), dim3(kBlock), 0, st, C, xr, xb, sc, sweeps, kCoarseTol,
                           cur_group());
    else
        hipLaunchKernelGGL((k_coarsest<R, false>), group_grid(1), dim3(kBlock), 0, st, C, xr, xb, sc, sweeps, kCoarseTol,
                           cur_group());
}

// ------------------------------------------------------------- transfers
template <typename R>
__global__ __launch_bounds__(kBlock) void k_restrict_field(int nc, const R *__restrict__ fr, const R *__restrict__ fb,
                                                           R *__restrict__ cr, R *__restrict__ cb, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    fr = gshift(fr, go);
    fb = gshift(fb, go);
    cr = gshift(cr, go);
    cb = gshift(cb, go);
    const int nch = nc / 2, nf = 2 * nc, nfh = nc;
    PM_SPAN_LOOP(e, sp)
    {
        int I, J, K;
        split(e, nc, nc, I, J, K);
        double t = 0.0;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                const unsigned ef = ((unsigned)(2 * I + a) * nf + (2 * J + b)) * nfh + K;
                t += (double)fr[ef] + (double)fb[ef];
            }
        const unsigned ec = ((unsigned)I * nc + J) * nch + (K >> 1);
        (((I + J + K) & 1) ? cb : cr)[ec] = (R)(0.125 * t);
    }
}

template <typename R>
void launch_restrict_field(int nc, const R *fr, const R *fb, R *cr, R *cb, hipStream_t st)
{
    const Span sp = make_span((unsigned long long)nc * nc * nc);
    hipLaunchKernelGGL((k_restrict_field<R>), group_grid(sp.nblocks), dim3(kBlock), 0, st, nc, fr, fb, cr, cb, sp,
                       cur_group());
}

__global__ __launch_bounds__(kBlock) void k_cast_f64_f32(const double *__restrict__ s, float *__restrict__ d, Span sp,
                                                         Group grp)
{
    const long long go = group_offset(grp);
    s = gshift(s, go);
    d = gshift(d, go);
    PM_SPAN_LOOP(e, sp)
    d[e] = (float)s[e];
}

void launch_cast_f64_f32(const double *src, float *dst, long long n, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_cast_f64_f32, group_grid(sp.nblocks), dim3(kBlock), 0, st, src, dst, sp, cur_group());
}

// Device-to-device copy in 16-byte words: the runtime's copy kernel moved
// about 2.6 TB/s at 128 MiB and 1.6 TB/s at 1 GiB here.  Unaligned or
// ragged copies go to hipMemcpyAsync.
__global__ __launch_bounds__(kBlock) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   unsigned long long n)
{
    for (unsigned long long q = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; q < n;
         q += (unsigned long long)gridDim.x * kBlock)
        dst[q] = src[q];
}

hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    if (bytes == 0)
        return hipSuccess;
    if ((((uintptr_t)dst) | ((uintptr_t)src) | bytes) & 15u)
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    const unsigned long long n = bytes / 16;
    const unsigned nb = (unsigned)std::min<unsigned long long>((n + kBlock - 1) / kBlock, 65536ull);
    hipLaunchKernelGGL(k_copy16, dim3(nb), dim3(kBlock), 0, st, (const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

// natural [i][j][k] (float or double) -> packed double, y = scale * x + shift.
// A thread takes the natural pair k = 2 kh, 2 kh + 1 of row (i, j): one red
// and one black cell, both halves of a cache line read at once.
template <typename Tn>
__global__ __launch_bounds__(kBlock) void k_nat_to_packed(const Tn *__restrict__ nat, double *__restrict__ packed, int n,
                                                          double scale, double shift, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    nat = gshift(nat, go);
    packed = gshift(packed, go);
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    PM_SPAN_LOOP(ec, sp)
    {
        int i, j, kh;
        split(ec, nh, n, i, j, kh);
        const Tn *in = nat + ((unsigned)i * n + j) * n + 2 * kh;
        const double v0 = scale * (double)in[0] + shift, v1 = scale * (double)in[1] + shift;
        const bool red_even = ((i + j) & 1) == 0;  // the red cell of the pair sits at k = 2 kh + ((i + j) & 1)
        packed[ec] = red_even ? v0 : v1;
        packed[half + ec] = red_even ? v1 : v0;
    }
}

void launch_natural_to_packed(const void *nat, pm_dtype dt, double *packed, int n, double scale, double shift,
                              hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n * n * (n / 2));
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_nat_to_packed<double>), group_grid(sp.nblocks), dim3(kBlock), 0, st,
                           (const double *)nat, packed, n, scale, shift, sp, cur_group());
    else
        hipLaunchKernelGGL((k_nat_to_packed<float>), group_grid(sp.nblocks), dim3(kBlock), 0, st, (const float *)nat,
                           packed, n, scale, shift, sp, cur_group());
}

// packed double -> natural, subtracting sum_ptr[0] / n^3 (the mean) if given
// and adding `add`.  A thread writes the natural pair k = 2 kh, 2 kh + 1 of
// row (i, j) from its red and its black cell, so both halves of a cache line
// are written together (red and black a half-array apart in time left the
// writes of each line split).
template <typename Tn>
__global__ __launch_bounds__(kBlock) void k_packed_to_nat(const double *__restrict__ packed, Tn *__restrict__ nat, int n,
                                                          const double *sum_ptr, double add, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    packed = gshift(packed, go);
    nat = gshift(nat, go);
    sum_ptr = gshift(sum_ptr, go);
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    const double shift = sum_ptr ? sum_ptr[0] / (2.0 * (double)half) : 0.0;
    PM_SPAN_LOOP(ec, sp)
    {
        int i, j, kh;
        split(ec, nh, n, i, j, kh);
        const Tn r = (Tn)(packed[ec] - shift + add), b = (Tn)(packed[half + ec] - shift + add);
        const bool red_even = ((i + j) & 1) == 0;  // the red cell of the pair sits at k = 2 kh + ((i + j) & 1)
        Tn *out = nat + ((unsigned)i * n + j) * n + 2 * kh;
        out[0] = red_even ? r : b;
        out[1] = red_even ? b : r;
    }
}

void launch_packed_to_natural(const double *packed, void *nat, pm_dtype dt, int n, double add, const double *sum_ptr,
                              hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n * n * (n / 2));
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_packed_to_nat<double>), group_grid(sp.nblocks), dim3(kBlock), 0, st, packed,
                           (double *)nat, n, sum_ptr, add, sp, cur_group());
    else
        hipLaunchKernelGGL((k_packed_to_nat<float>), group_grid(sp.nblocks), dim3(kBlock), 0, st, packed,
                           (float *)nat, n, sum_ptr, add, sp, cur_group());
}

// ------------------------------------------------------------ mixed precision
// NL: FAS form (the FP32 level carries the full approximation x32 = fl(x64)).
// !NL: correction form for the linear problem: the FP32 level solves
// lap e = r64 - <r64> from e = 0 (its source beta is 0), so FP32 rounding of
// the iterate never enters.
template <bool NL>
__global__ __launch_bounds__(kBlock) void k_mixed_outer(LevelView<double> F, const double *__restrict__ xr,
                                                        const double *__restrict__ xb, const double *__restrict__ csum64,
                                                        LevelView<float> G, float *__restrict__ x32r,
                                                        float *__restrict__ x32b, ReduceSlot rs, SolveConsts sc,
                                                        Span sp, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    gshift_view(G, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    csum64 = gshift(csum64, go);
    x32r = gshift(x32r, go);
    x32b = gshift(x32b, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    const double cm = (csum64[0] + csum64[1]) / (2.0 * (double)F.half);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double ih2 = 1.0 / (F.h * F.h);
    const float ih2f = (float)ih2;
    const unsigned half = (unsigned)F.half;
    const int n = F.n, nh = F.nh;
    const unsigned lb = span_block(sp);
    const unsigned e0 = lb * sp.chunk + threadIdx.x;
    const unsigned e1 = min(sp.total, (lb + 1) * sp.chunk);
    int c = e0 >= half;
    unsigned ef = e0 - (c ? half : 0u);
    int i = 0, j = 0, kh = 0;
    if (e0 < e1)
        split(ef, nh, n, i, j, kh);
    for (unsigned e = e0; e < e1;) {
        const double *own = c ? xb : xr;
        const double *oth = c ? xr : xb;
        // the 18 neighbours once, for both the FP64 residual and the FP32
        // operator of x32 = fl(x64) (each neighbour rounded on load)
        const int p = (i + j + c) & 1;
        const int km = wrap_dn(kh - 1 + p, nh), kp = wrap_up(kh + p, nh);
        const int ip = wrap_up(i + 1, n), im = wrap_dn(i - 1, n);
        const int jp = wrap_up(j + 1, n), jm = wrap_dn(j - 1, n);
        const unsigned r00 = ((unsigned)i * n + j) * nh, rp0 = ((unsigned)ip * n + j) * nh;
        const unsigned rm0 = ((unsigned)im * n + j) * nh, r0p = ((unsigned)i * n + jp) * nh;
        const unsigned r0m = ((unsigned)i * n + jm) * nh;
        double v[18];
        v[0] = oth[rp0 + kh];
        v[1] = oth[rm0 + kh];
        v[2] = oth[r0p + kh];
        v[3] = oth[r0m + kh];
        v[4] = oth[r00 + kp];
        v[5] = oth[r00 + km];
        if (NL) {
            const unsigned rpp = ((unsigned)ip * n + jp) * nh, rpm = ((unsigned)ip * n + jm) * nh;
            const unsigned rmp = ((unsigned)im * n + jp) * nh, rmm = ((unsigned)im * n + jm) * nh;
            v[6] = own[rpp + kh];
            v[7] = own[rpm + kh];
            v[8] = own[rmp + kh];
            v[9] = own[rmm + kh];
            v[10] = own[rp0 + kp];
            v[11] = own[rp0 + km];
            v[12] = own[rm0 + kp];
            v[13] = own[rm0 + km];
            v[14] = own[r0p + kp];
            v[15] = own[r0p + km];
            v[16] = own[r0m + kp];
            v[17] = own[r0m + km];
        } else {
            for (int q = 6; q < 18; q++)
                v[q] = 0.0;
        }
        const double x64 = own[ef];
        double tsh;
        const double S = stencil_eval<double>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], v[11],
                                              v[12], v[13], v[14], v[15], v[16], v[17], NL, tsh);
        const double dv = (c ? F.db : F.dr)[ef];
        const double b = sc.beta * dv;
        int isv;
        const double lq = root_lap<double>(b, tsh * ih2 * ih2, sc, NL, isv);
        const double r = lq - cm - (S - 6.0 * x64) * ih2;
        acc[0] += r * r;
        acc[1] += r;
        acc[2] += lq;
        acc[3] += (double)isv;
        if (!NL) {
            (c ? x32b : x32r)[ef] = 0.0f;
            (c ? G.tb : G.tr)[ef] = (float)r;
            acc[4 + c] += (double)(float)r;
        } else {
            float tsh32;
            const float S32 = stencil_eval<float>(
                (float)v[0], (float)v[1], (float)v[2], (float)v[3], (float)v[4], (float)v[5], (float)v[6],
                (float)v[7], (float)v[8], (float)v[9], (float)v[10], (float)v[11], (float)v[12], (float)v[13],
                (float)v[14], (float)v[15], (float)v[16], (float)v[17], true, tsh32);
            const float x32 = (float)x64;
            const float b32 = (float)sc.beta * (float)dv;  // the FP32 level's delta is fl32 of the FP64 one
            int isv32;
            const float lq32 = root_lap<float>(b32, tsh32 * ih2f * ih2f, sc, true, isv32);
            const float lap32 = (S32 - 6.0f * x32) * ih2f;
            const float tau32 = (float)r + lap32 - lq32;
            (c ? x32b : x32r)[ef] = x32;
            (c ? G.tb : G.tr)[ef] = tau32;
            acc[4 + c] += (double)(lq32 + tau32);
        }
        e += kBlock;
        if (e < e1) {  // step by kBlock cells; re-split when crossing into colour 1
            if (!c && e >= half) {
                c = 1;
                ef = e - half;
                split(ef, nh, n, i, j, kh);
            } else {
                ef += kBlock;
                kh += kBlock;
                while (kh >= nh) {
                    kh -= nh;
                    if (++j == n) {
                        j = 0;
                        ++i;
                    }
                }
            }
        }
    }
    block_partials<6>(acc, rs, sp);
}

bool launch_mixed_outer_residual(const LevelView<double> &F64, const double *xr, const double *xb, const double *csum64,
                                 const LevelView<float> &F32, float *x32r, float *x32b, ReduceSlot rs,
                                 SolveConsts sc, bool nonlinear, hipStream_t st, int tiled, double *lag64,
                                 double *lag32, const MixedCorr *corr, bool zero_iterate)
{
    auto finish = [&](const Span &s) {
        if (lag64 && lag32)
            hipLaunchKernelGGL(k_finalize_outer, group_grid(1), dim3(kBlock), 0, st, (const double *)rs.partials,
                               (int)s.nblocks, rs.out, lag64, lag32, cur_group());
        else
            launch_finalize(rs, s, 6, rs.out, st);
    };
    Span spt;
    if (launch_mixed_outer_tiled(F64, xr, xb, csum64, F32, x32r, x32b, rs, sc, nonlinear, st, tiled, &spt, corr,
                                 zero_iterate)) {
        finish(spt);
        return true;
    }
    if (corr)
        return false;
    const Span sp = make_span(2 * F64.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_mixed_outer<true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F64, xr, xb, csum64, F32,
                           x32r, x32b, rs, sc, sp, cur_group());
    else
        hipLaunchKernelGGL((k_mixed_outer<false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F64, xr, xb, csum64,
                           F32, x32r, x32b, rs, sc, sp, cur_group());
    finish(sp);
    return true;
}

// x64 += fl32(x32 - fl32(x64)) (NL: the FP32 level started from fl32(x64))
// or x64 += x32 (the linear correction form, started from 0).
template <bool NL>
__global__ __launch_bounds__(kBlock) void k_mixed_correct(double *__restrict__ x64, const float *__restrict__ x32r,
                                                          const float *__restrict__ x32b, unsigned half, Span sp,
                                                          Group grp)
{
    const long long go = group_offset(grp);
    x64 = gshift(x64, go);
    x32r = gshift(x32r, go);
    x32b = gshift(x32b, go);
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ec = e - (c ? half : 0u);
        const double x = x64[e];
        const float v = c ? x32b[ec] : x32r[ec];
        const float d = NL ? v - (float)x : v;
        x64[e] = x + (double)d;
    }
}

void launch_mixed_correct(double *x64, const float *x32r, const float *x32b, long long half, bool nonlinear,
                          hipStream_t st)
{
    const Span sp = make_span(2 * half);
    if (nonlinear)
        hipLaunchKernelGGL((k_mixed_correct<true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, x64, x32r, x32b,
                           (unsigned)half, sp, cur_group());
    else
        hipLaunchKernelGGL((k_mixed_correct<false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, x64, x32r, x32b,
                           (unsigned)half, sp, cur_group());
}

// ------------------------------------------------------------ residual norm
template <bool NL>
__global__ __launch_bounds__(kBlock) void k_residual_norm(LevelView<double> F, const double *__restrict__ xr,
                                                          const double *__restrict__ xb, const double *__restrict__ csum,
                                                          ReduceSlot rs, SolveConsts sc, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    csum = gshift(csum, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    const double cm = (csum[0] + csum[1]) / (2.0 * (double)F.half);
    double acc[4] = {0, 0, 0, 0};
    const unsigned half = (unsigned)F.half;
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ef = e - (c ? half : 0u);
        int i, j, kh;
        split(ef, F.nh, F.n, i, j, kh);
        double lqt;
        int isv;
        const double r = cell_residual<double, double, NL>(F, xr, xb, c, i, j, kh, ef, cm, sc, lqt, isv);
        acc[0] += r * r;
        acc[1] += r;
        acc[2] += lqt;
        acc[3] += (double)isv;
    }
    block_partials<4>(acc, rs, sp);
}

void launch_residual_norm(const LevelView<double> &F, const double *xr, const double *xb, const double *csum,
                          ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st)
{
    const Span sp = make_span(2 * F.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_residual_norm<true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, rs, sc,
                           sp, cur_group());
    else
        hipLaunchKernelGGL((k_residual_norm<false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, rs,
                           sc, sp, cur_group());
    launch_finalize(rs, sp, 4, rs.out, st);
}

// ------------------------------------------------------------ small helpers
__global__ __launch_bounds__(kBlock) void k_field_sum(const double *__restrict__ x, ReduceSlot rs, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    x = gshift(x, go);
    gshift_slot(rs, go);
    double acc[2] = {0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    {
        const double v = x[e];
        acc[0] += v;
        acc[1] += v * v;
    }
    block_partials<2>(acc, rs, sp);
}

void launch_field_sum(const double *x, long long n, ReduceSlot rs, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_field_sum, group_grid(sp.nblocks), dim3(kBlock), 0, st, x, rs, sp, cur_group());
    launch_finalize(rs, sp, 2, rs.out, st);
}

__global__ __launch_bounds__(kBlock) void k_subtract_mean(double *__restrict__ x, const double *sum_ptr, Span sp,
                                                          Group grp)
{
    const long long go = group_offset(grp);
    x = gshift(x, go);
    sum_ptr = gshift(sum_ptr, go);
    const double m = sum_ptr[0] / (double)sp.total;
    PM_SPAN_LOOP(e, sp)
    x[e] -= m;
}

void launch_subtract_mean(double *x, long long n, const double *sum_ptr, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_subtract_mean, group_grid(sp.nblocks), dim3(kBlock), 0, st, x, sum_ptr, sp, cur_group());
}

__global__ __launch_bounds__(kBlock) void k_scale(const double *__restrict__ x, double *__restrict__ y, double a, Span sp,
                                                  Group grp)
{
    const long long go = group_offset(grp);
    x = gshift(x, go);
    y = gshift(y, go);
    PM_SPAN_LOOP(e, sp)
    y[e] = a * x[e];
}

void launch_scale(const double *x, double *y, double a, long long n, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_scale, group_grid(sp.nblocks), dim3(kBlock), 0, st, x, y, a, sp, cur_group());
}

// src[0 .. count-1] into host memory, then the sequence number (one lane, a
// system-scope release between them), for a host that polls the sequence
// number instead of synchronising the stream.
__global__ void k_publish(const double *__restrict__ src, int count, double *dst, unsigned *seqp, unsigned seq)
{
    if (threadIdx.x == 0) {
        for (int q = 0; q < count; q++)
            dst[q] = src[q];
        __threadfence_system();
        *(volatile unsigned *)seqp = seq;
    }
}

void launch_publish(const double *src, int count, double *dst, unsigned *seqp, unsigned seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, st, src, count, dst, seqp, seq);
}

// dst[s * count + q] = src[q] of slot s (slot s at src + s * stride bytes),
// for the m slots of a group: their norms in one contiguous readback.
__global__ __launch_bounds__(kBlock) void k_gather_slots(const double *__restrict__ src, long long stride, int m,
                                                         int count, double *__restrict__ dst)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < m * count) {
        const int s = t / count, q = t - s * count;
        dst[t] = *reinterpret_cast<const double *>(reinterpret_cast<const char *>(src) + (long long)s * stride +
                                                   (long long)q * sizeof(double));
    }
}

void launch_gather_slots(const double *src, long long stride, int m, int count, double *dst, hipStream_t st)
{
    const int n = m * count;
    hipLaunchKernelGGL(k_gather_slots, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, stride, m, count,
                       dst);
}

// Zero fill as a kernel (not hipMemsetAsync), 64-bit indices: the
// workspace can exceed 2^32 words.
__global__ __launch_bounds__(kBlock) void k_zero(uint32_t *__restrict__ p, long long nw, Group grp)
{
    p = gshift(p, group_offset(grp));
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < nw; e += (long long)gridDim.x * kBlock)
        p[e] = 0u;
}

void launch_zero(void *p, size_t bytes, hipStream_t st)
{
    const long long nw = (long long)(bytes / 4);
    long long b = (nw + kBlock - 1) / kBlock;
    if (b > kMaxBlocks)
        b = kMaxBlocks;
    hipLaunchKernelGGL(k_zero, group_grid((unsigned)(b < 1 ? 1 : b)), dim3(kBlock), 0, st, (uint32_t *)p, nw,
                       cur_group());
}

// explicit instantiations
template void launch_residual_restrict<double>(const LevelView<double> &, const double *, const double *,
                                               const double *, const LevelView<double> &, double *, double *,
                                               ReduceSlot, SolveConsts, bool, hipStream_t, bool, int);
template void launch_residual_restrict<float>(const LevelView<float> &, const float *, const float *, const double *,
                                              const LevelView<float> &, float *, float *, ReduceSlot, SolveConsts,
                                              bool, hipStream_t, bool, int);
template void launch_fas_tau<double>(const LevelView<double> &, const double *, const double *, double *, ReduceSlot,
                                     SolveConsts, bool, bool, hipStream_t, int, bool);
template void launch_fas_tau<float>(const LevelView<float> &, const float *, const float *, double *, ReduceSlot,
                                    SolveConsts, bool, bool, hipStream_t, int, bool);
template void launch_prolong_correct<double>(const LevelView<double> &, double *, double *, const LevelView<double> &,
                                             const double *, const double *, hipStream_t, int);
template void launch_prolong_correct<float>(const LevelView<float> &, float *, float *, const LevelView<float> &,
                                            const float *, const float *, hipStream_t, int);
template void launch_prolong_full<double>(const LevelView<double> &, double *, double *, const LevelView<double> &,
                                          const double *, const double *, hipStream_t, int);
template void launch_prolong_full<float>(const LevelView<float> &, float *, float *, const LevelView<float> &,
                                         const float *, const float *, hipStream_t, int);
template void launch_coarsest<double>(const LevelView<double> &, double *, double *, SolveConsts, bool, int,
                                      hipStream_t);
template void launch_coarsest<float>(const LevelView<float> &, float *, float *, SolveConsts, bool, int, hipStream_t);
template void launch_restrict_field<double>(int, const double *, const double *, double *, double *, hipStream_t);
template void launch_restrict_field<float>(int, const float *, const float *, float *, float *, hipStream_t);

// ------------------------------------------------------------ block cycle
// The V-cycle (or the coarse part of full multigrid) from level l0 down, run
// by one workgroup: on coarse grids a launch per operation costs more than
// the operation, so the whole sub-cycle becomes one launch.  The cell updates
// are the functions of the grid-wide kernels; the lagged mean of a level is
// the exact per-colour sum of its last half-sweeps (no deferred fold).
template <typename R>
__device__ __forceinline__ void block_sum2(double a, double b, double *out2, double (*red)[2])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if (lane == 0) {
        red[wid][0] = a;
        red[wid][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < nw; w++) {
            sa += red[w][0];
            sb += red[w][1];
        }
        out2[0] = sa;
        out2[1] = sb;
    }
    __syncthreads();
}

// Levels lr..L-1 of a block cycle live in LDS for the whole launch: every
// operation on them is bound by memory latency, not bandwidth.  A resident
// level holds its delta, its tau (if it has one), x0 (below l0 only) and the
// two colour buffers, each 2 half elements; at most kBlockLdsBytes in all.
constexpr size_t kBlockLdsBytes = 48 * 1024;
__host__ __device__ constexpr unsigned block_level_elems(long long half, bool has_tau, bool has_x0)
{
    return (unsigned)(2 * half) * (3u + (has_tau ? 1u : 0u) + (has_x0 ? 1u : 0u));
}

template <typename R, bool NL>
__global__ __launch_bounds__(kBlockCycleThreads) void k_block_cycle(BlockHier<R> Barg, int l0, int fmg, int n_pre,
                                                                    int n_post, SolveConsts sc,
                                                                    const double *__restrict__ csum_l0, int cur_bits,
                                                                    int coarse_sweeps, int lr, Group grp)
{
    // the level table lives in LDS: indexed by level at run time, a kernel
    // argument would be copied to private memory.  The helpers below capture
    // by value: a by-reference capture of the arguments (sc, the sweep
    // counts, tid) would keep them in private memory too, read in every loop.
    __shared__ BlockHier<R> B;
    const long long go = group_offset(grp);
    csum_l0 = gshift(csum_l0, go);
    gconsts(sc, grp);
    if (threadIdx.x == 0) {
        B = Barg;
        for (int l = 0; l < kMaxLevels; l++) {
            gshift_view(B.L[l], go);
            B.buf[l][0] = gshift(B.buf[l][0], go);
            B.buf[l][1] = gshift(B.buf[l][1], go);
        }
    }
    __shared__ int cur[kMaxLevels][2];
    __shared__ double cs[kMaxLevels][2];
    __shared__ double red[16][2];
    __shared__ double tmp2[2];
    const unsigned tid = threadIdx.x, nt = blockDim.x;
    const int L = Barg.nlev;  // B is read only after the barrier below
    if (tid == 0) {
        for (int l = 0; l < kMaxLevels; l++) {
            cur[l][0] = cur[l][1] = 0;
            cs[l][0] = cs[l][1] = 0.0;
        }
        if (!fmg) {
            cur[l0][0] = cur_bits & 1;
            cur[l0][1] = (cur_bits >> 1) & 1;
            cs[l0][0] = csum_l0[0];
            cs[l0][1] = csum_l0[1];
        }
    }
    __syncthreads();
    // Move the resident levels into LDS.  Delta and tau are inputs (tau of
    // every level below l0 is still read by full multigrid), level l0's two
    // colour buffers are inputs and outputs; the rest is written in the cycle
    // before it is read.  The views in B are repointed level by level, once
    // all threads have copied through the old pointers.
    extern __shared__ __align__(16) unsigned char bc_dyn[];
    __shared__ R *gx0[2];
    if (lr < L) {
        R *lds = reinterpret_cast<R *>(bc_dyn);
        unsigned o = 0;
        for (int m = lr; m < L; m++) {
            const unsigned half = (unsigned)B.L[m].half, tot = 2u * half;
            const bool has_t = B.L[m].tr != nullptr, has_x0 = m > l0 && B.L[m].x0r != nullptr;
            R *d = lds + o;
            R *t = d + tot;
            R *x0 = t + (has_t ? tot : 0u);
            R *b0 = x0 + (has_x0 ? tot : 0u);
            R *b1 = b0 + tot;
            o += block_level_elems(half, has_t, has_x0);
            for (unsigned e = tid; e < tot; e += nt) {
                const bool red_half = e < half;
                d[e] = red_half ? B.L[m].dr[e] : B.L[m].db[e - half];
                if (has_t)
                    t[e] = red_half ? B.L[m].tr[e] : B.L[m].tb[e - half];
                if (m == l0) {
                    b0[e] = B.buf[m][0][e];
                    b1[e] = B.buf[m][1][e];
                }
            }
            __syncthreads();
            if (tid == 0) {
                if (m == l0) {
                    gx0[0] = B.buf[m][0];
                    gx0[1] = B.buf[m][1];
                }
                B.L[m].dr = d;
                B.L[m].db = d + half;
                if (has_t) {
                    B.L[m].tr = t;
                    B.L[m].tb = t + half;
                }
                if (has_x0) {
                    B.L[m].x0r = x0;
                    B.L[m].x0b = x0 + half;
                }
                B.buf[m][0] = b0;
                B.buf[m][1] = b1;
            }
            __syncthreads();
        }
    }
    auto coarsest = [=](const LevelView<R> &Cv, R *cr, R *cb) {
        if (Cv.n == 4) {  // uniform branch: one wave solves, the block waits
            if (tid < 64)
                coarsest_wave<R, NL>(Cv, cr, cb, sc, coarse_sweeps, kCoarseTol);
            __syncthreads();
        } else {
            coarsest_solve<R, NL>(Cv, cr, cb, sc, coarse_sweeps, kCoarseTol);
        }
    };
    auto xr = [=](int l) -> R * { return B.buf[l][cur[l][0]]; };
    auto xb = [=](int l) -> R * { return B.buf[l][cur[l][1]] + B.L[l].half; };
    auto half_sweep = [=](int m, int colour) {
        const LevelView<R> &Lv = B.L[m];
        const int own = cur[m][colour];
        const unsigned half = (unsigned)Lv.half;
        R *src = B.buf[m][own] + (colour ? half : 0u);
        R *dst = B.buf[m][1 - own] + (colour ? half : 0u);
        const R *oth = B.buf[m][cur[m][1 - colour]] + (colour ? 0u : half);
        const R cmean = (R)((cs[m][0] + cs[m][1]) / (2.0 * (double)half));
        const R h2 = (R)(Lv.h * Lv.h), ih2 = (R)(1.0 / (Lv.h * Lv.h));
        const R *dc = colour ? Lv.db : Lv.dr;
        const R *tc = colour ? Lv.tb : Lv.tr;
        double acc = 0.0;
        for (unsigned e = tid; e < half; e += nt) {
            int i, j, kh;
            split(e, Lv.nh, Lv.n, i, j, kh);
            acc += (double)smooth_cell<R, NL>(src, oth, dst, dc, tc, Lv.n, Lv.nh, colour, i, j, kh, e, cmean, h2, ih2,
                                             sc);
        }
        block_sum2<R>(acc, 0.0, tmp2, red);
        if (tid == 0) {
            cs[m][colour] = tmp2[0];
            cur[m][colour] = 1 - own;
        }
        __syncthreads();
    };
    auto fas = [=](int m, int acc_only) {
        double acc[2] = {0.0, 0.0};
        const unsigned tot = 2u * (unsigned)B.L[m].half;
        R *x_r = xr(m), *x_b = xb(m);
        for (unsigned e = tid; e < tot; e += nt)
            fas_cell<R, NL>(B.L[m], x_r, x_b, sc, e, acc_only, acc);
        block_sum2<R>(acc[0], acc[1], tmp2, red);
        if (tid == 0) {
            cs[m][0] = tmp2[0];
            cs[m][1] = tmp2[1];
        }
        __syncthreads();
    };
    auto vcycle = [=](int l) {
        for (int m = l; m < L - 1; m++) {
            for (int s = 0; s < n_pre; s++) {
                half_sweep(m, 0);
                half_sweep(m, 1);
            }
            const double cm = (cs[m][0] + cs[m][1]) / (2.0 * (double)B.L[m].half);
            R *cxr = B.buf[m + 1][0], *cxb = B.buf[m + 1][0] + B.L[m + 1].half;
            const unsigned tot = 2u * (unsigned)B.L[m + 1].half;
            R *x_r = xr(m), *x_b = xb(m);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (unsigned e = tid; e < tot; e += nt)
                restrict_cell<R, NL>(B.L[m], x_r, x_b, cm, B.L[m + 1], cxr, cxb, sc, e, acc);
            __syncthreads();
            if (tid == 0)
                cur[m + 1][0] = cur[m + 1][1] = 0;
            __syncthreads();
            fas(m + 1, 0);
        }
        coarsest(B.L[L - 1], xr(L - 1), xb(L - 1));
        for (int m = L - 2; m >= l; m--) {
            const unsigned tot = 2u * (unsigned)B.L[m + 1].half;
            R *x_r = xr(m), *x_b = xb(m), *c_r = xr(m + 1), *c_b = xb(m + 1);
            for (unsigned e = tid; e < tot; e += nt)
                prolong_cell<R, true>(B.L[m], x_r, x_b, B.L[m + 1], c_r, c_b, e);
            __syncthreads();
            for (int s = 0; s < n_post; s++) {
                half_sweep(m, 0);
                half_sweep(m, 1);
            }
        }
    };
    if (fmg) {
        R *xc = B.buf[L - 1][0];
        const unsigned totc = 2u * (unsigned)B.L[L - 1].half;
        for (unsigned e = tid; e < totc; e += nt)
            xc[e] = (R)0;
        __syncthreads();
        coarsest(B.L[L - 1], xc, xc + B.L[L - 1].half);
        for (int l = L - 2; l >= l0; l--) {
            const unsigned tot = 2u * (unsigned)B.L[l + 1].half;
            R *x_r = B.buf[l][0], *x_b = B.buf[l][0] + B.L[l].half, *c_r = xr(l + 1), *c_b = xb(l + 1);
            for (unsigned e = tid; e < tot; e += nt)
                prolong_cell<R, false>(B.L[l], x_r, x_b, B.L[l + 1], c_r, c_b, e);
            __syncthreads();
            if (tid == 0)
                cur[l][0] = cur[l][1] = 0;
            __syncthreads();
            fas(l, 1);
            vcycle(l);
        }
    } else {
        vcycle(l0);
    }
    if (lr <= l0) {  // level l0 resident: its colour buffers go back
        __syncthreads();
        const unsigned tot = 2u * (unsigned)B.L[l0].half;
        for (unsigned e = tid; e < tot; e += nt) {
            gx0[0][e] = B.buf[l0][0][e];
            gx0[1][e] = B.buf[l0][1][e];
        }
    }
}

// The coarsest levels (from l0 down) that fit in kBlockLdsBytes become
// resident: returns their LDS bytes and the first resident level in *lr
// (B.nlev: none).
template <typename R>
size_t block_cycle_lds(const BlockHier<R> &B, int l0, int *lr_out)
{
    int lr = B.nlev;
    size_t bytes = 0;
    for (int m = B.nlev - 1; m >= l0; m--) {
        const size_t b = sizeof(R) * block_level_elems(B.L[m].half, B.L[m].tr != nullptr,
                                                       m > l0 && B.L[m].x0r != nullptr);
        if (bytes + b > kBlockLdsBytes)
            break;
        bytes += b;
        lr = m;
    }
    *lr_out = lr;
    return bytes;
}
template size_t block_cycle_lds<float>(const BlockHier<float> &, int, int *);
template size_t block_cycle_lds<double>(const BlockHier<double> &, int, int *);

size_t block_cycle_lds_limit() { return kBlockLdsBytes; }

template <typename R>
void launch_block_cycle(const BlockHier<R> &B, int l0, bool fmg, int n_pre, int n_post, SolveConsts sc, bool nonlinear,
                        const double *csum_l0, int cur_bits, int coarse_sweeps, hipStream_t st)
{
    int lr = B.nlev;
    const size_t bytes = block_cycle_lds(B, l0, &lr);
    if (nonlinear)
        hipLaunchKernelGGL((k_block_cycle<R, true>), group_grid(1), dim3(kBlockCycleThreads), bytes, st, B, l0,
                           fmg ? 1 : 0, n_pre, n_post, sc, csum_l0, cur_bits, coarse_sweeps, lr, cur_group());
    else
        hipLaunchKernelGGL((k_block_cycle<R, false>), group_grid(1), dim3(kBlockCycleThreads), bytes, st, B, l0,
                           fmg ? 1 : 0, n_pre, n_post, sc, csum_l0, cur_bits, coarse_sweeps, lr, cur_group());
}

template void launch_block_cycle<float>(const BlockHier<float> &, int, bool, int, int, SolveConsts, bool,
                                        const double *, int, int, hipStream_t);
template void launch_block_cycle<double>(const BlockHier<double> &, int, bool, int, int, SolveConsts, bool,
                                         const double *, int, int, hipStream_t);

}  // namespace pmeft
