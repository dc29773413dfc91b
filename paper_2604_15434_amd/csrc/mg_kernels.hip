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
#include "pmeft_internal.h"

#include <math.h>

namespace pmeft {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrap_up(int i, int n) { return i >= n ? i - n : i; }
__device__ __forceinline__ int wrap_dn(int i, int n) { return i < 0 ? i + n : i; }

// Void-cell test and root of the local quadratic, computed in the type T.
template <typename T>
__device__ __forceinline__ T root_lap(T b, T Tsh, const SolveConsts &sc, bool nonlinear, int &is_void)
{
    const T nu = (T)sc.nu;
    if (!nonlinear) {
        is_void = 0;
        return b / nu;
    }
    const T K = (T)sc.K;
    const T dsph = nu * nu - (T)(8.0 / 3.0) * K * b;
    if (dsph < (T)0) {
        is_void = 1;
        return (T)0.75 * nu / K;
    }
    is_void = 0;
    const T G = K * Tsh - b;
    const T disc = dsph + (T)(8.0 / 3.0) * K * K * Tsh;
    return (T)-2 * G / (nu + sqrt(disc));
}

// Operator pieces from the 18 neighbour values of a cell: the six face
// neighbours (other colour: x+, x-, y+, y-, z+, z-) and the twelve edge
// neighbours (own colour: (i+-1, j+-1) at k; (i+-1) at k+-1; (j+-1) at
// k+-1).  Returns S (face sum); sets Tsh (squared traceless Hessian times h^4)
// when nonlinear.
template <typename T>
__device__ __forceinline__ T stencil_eval(T oxp, T oxm, T oyp, T oym, T ozp, T ozm, T epp, T epm, T emp, T emm,
                                          T xpp, T xpm, T xmp, T xmm, T ypp, T ypm, T ymp, T ymm, bool nonlinear,
                                          T &tsh_h4)
{
    const T ax = oxp + oxm;
    const T ay = oyp + oym;
    const T az = ozp + ozm;
    tsh_h4 = (T)0;
    if (nonlinear) {
        const T dxy = epp - epm - emp + emm;
        const T dxz = xpp - xpm - xmp + xmm;
        const T dyz = ypp - ypm - ymp + ymm;
        const T exy = ax - ay, eyz = ay - az, ezx = az - ax;
        // (1/3) sum (D_ll - D_mm)^2 + 2 sum D_lm^2, all times h^4, with
        // D_lm = d_lm / (4 h^2).
        tsh_h4 = (exy * exy + eyz * eyz + ezx * ezx) * (T)(1.0 / 3.0) + (dxy * dxy + dxz * dxz + dyz * dyz) * (T)0.125;
    }
    return ax + ay + az;
}

// Operator pieces at cell (i, j, kh) of colour c.  `own` is the colour-c
// block, `oth` the other block; values are loaded as Ts and computed as T.
// In the packed layout the k-neighbours of (i, j, kh) sit at kh - 1 + p and
// kh + p with p = (i + j + c) & 1.
template <typename T, typename Ts>
__device__ __forceinline__ T stencil_terms(const Ts *__restrict__ own, const Ts *__restrict__ oth, int n, int nh, int c,
                                           int i, int j, int kh, bool nonlinear, T &tsh_h4)
{
    const int p = (i + j + c) & 1;
    const int km = wrap_dn(kh - 1 + p, nh);
    const int kp = wrap_up(kh + p, nh);
    const int ip = wrap_up(i + 1, n), im = wrap_dn(i - 1, n);
    const int jp = wrap_up(j + 1, n), jm = wrap_dn(j - 1, n);
    const unsigned r00 = ((unsigned)i * n + j) * nh;
    const unsigned rp0 = ((unsigned)ip * n + j) * nh;
    const unsigned rm0 = ((unsigned)im * n + j) * nh;
    const unsigned r0p = ((unsigned)i * n + jp) * nh;
    const unsigned r0m = ((unsigned)i * n + jm) * nh;
    if (!nonlinear)
        return stencil_eval<T>((T)oth[rp0 + kh], (T)oth[rm0 + kh], (T)oth[r0p + kh], (T)oth[r0m + kh],
                               (T)oth[r00 + kp], (T)oth[r00 + km], (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0,
                               (T)0, (T)0, (T)0, (T)0, false, tsh_h4);
    const unsigned rpp = ((unsigned)ip * n + jp) * nh;
    const unsigned rpm = ((unsigned)ip * n + jm) * nh;
    const unsigned rmp = ((unsigned)im * n + jp) * nh;
    const unsigned rmm = ((unsigned)im * n + jm) * nh;
    return stencil_eval<T>((T)oth[rp0 + kh], (T)oth[rm0 + kh], (T)oth[r0p + kh], (T)oth[r0m + kh], (T)oth[r00 + kp],
                           (T)oth[r00 + km], (T)own[rpp + kh], (T)own[rpm + kh], (T)own[rmp + kh], (T)own[rmm + kh],
                           (T)own[rp0 + kp], (T)own[rp0 + km], (T)own[rm0 + kp], (T)own[rm0 + km], (T)own[r0p + kp],
                           (T)own[r0p + km], (T)own[r0m + kp], (T)own[r0m + km], true, tsh_h4);
}

// One block: out[q] = sum over blocks b (in order) of partials[b * 8 + q].
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials, int nblocks, int nv,
                                                     double *__restrict__ out)
{
    __shared__ double sm[8][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int q = 0; q < nv; q++) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock)
            acc += partials[(size_t)b * 8 + q];
        for (int off = 32; off > 0; off >>= 1)
            acc += __shfl_down(acc, off, 64);
        if (lane == 0)
            sm[q][wid] = acc;
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
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, (const double *)rs.partials, (int)sp.nblocks, nv,
                       out);
}

// ---------------------------------------------------------------- smoothing
// Block 0 of a half-sweep: csum_out = csum_in with the colour of the previous
// half-sweep at this level (prev_colour; -1 none) replaced by the sum of its
// per-block partials, in block order.
__device__ __forceinline__ void fold_previous(const double *__restrict__ csum_in, double *__restrict__ csum_out,
                                              const double *__restrict__ prev, int prev_nblocks, int prev_colour)
{
    __shared__ double fin[kBlock / 64];
    double t = 0.0;
    if (prev_colour >= 0)
        for (int q = threadIdx.x; q < prev_nblocks; q += kBlock)
            t += prev[(size_t)q * 8];
    for (int off = 32; off > 0; off >>= 1)
        t += __shfl_down(t, off, 64);
    if ((threadIdx.x & 63) == 0)
        fin[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = csum_in[threadIdx.x];
        if ((int)threadIdx.x == prev_colour) {
            v = 0.0;
            for (int w = 0; w < kBlock / 64; w++)
                v += fin[w];
        }
        csum_out[threadIdx.x] = v;
    }
}

// Local update of one cell of colour `colour` (element e = (i, j, kh)):
// x_new = (S - h^2 (Lq + tau - cmean)) / 6; returns Lq + tau.
template <typename R, bool NL>
__device__ __forceinline__ R smooth_cell(const R *__restrict__ xc_old, const R *__restrict__ xo, R *__restrict__ xc_new,
                                         const R *__restrict__ dc, const R *__restrict__ tc, int n, int nh, int colour,
                                         int i, int j, int kh, unsigned e, R cmean, R h2, R ih2, const SolveConsts &sc)
{
    R tsh;
    const R S = stencil_terms<R, R>(xc_old, xo, n, nh, colour, i, j, kh, NL, tsh);
    const R b = (R)sc.beta * dc[e];
    int isv;
    const R lq = root_lap<R>(b, tsh * ih2 * ih2, sc, NL, isv);
    const R v = lq + (tc ? tc[e] : (R)0);
    xc_new[e] = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
    return v;
}

// One half-sweep of colour `colour`.  The lagged mean c = <Lq + tau> comes
// from csum_in (per-colour sums).  Block 0 also folds the partial sums of the
// previous half-sweep at this level (prev, prev_nblocks, prev_colour; colour
// -1 = none) into csum_out, which the next half-sweep reads: the mean thus
// lags by about one sweep, needs no extra launch, and stays deterministic
// (every launch reads only values completed by earlier launches).
template <typename R, bool NL>
__global__ __launch_bounds__(kBlock) void k_smooth(LevelView<R> L, int colour, const R *__restrict__ xc_old,
                                                   const R *__restrict__ xo, R *__restrict__ xc_new,
                                                   const double *__restrict__ csum_in, double *__restrict__ csum_out,
                                                   const double *__restrict__ prev, int prev_nblocks, int prev_colour,
                                                   ReduceSlot rs, SolveConsts sc, Span sp)
{
    const int n = L.n, nh = L.nh;
    const R cmean = (R)((csum_in[0] + csum_in[1]) / (2.0 * (double)L.half));
    const R h2 = (R)(L.h * L.h);
    const R ih2 = (R)(1.0 / (L.h * L.h));
    const R *dc = colour ? L.db : L.dr;
    const R *tc = colour ? L.tb : L.tr;
    double acc[1] = {0.0};
    const unsigned lb = span_block(sp);
    const unsigned e0 = lb * sp.chunk + threadIdx.x;
    const unsigned e1 = min(sp.total, (lb + 1) * sp.chunk);
    int i, j, kh;
    if (e0 < e1)
        split(e0, nh, n, i, j, kh);
    for (unsigned e = e0; e < e1;) {
        acc[0] += (double)smooth_cell<R, NL>(xc_old, xo, xc_new, dc, tc, n, nh, colour, i, j, kh, e, cmean, h2, ih2, sc);
        e += kBlock;
        if (e < e1) {  // step (i, j, kh) by kBlock cells without dividing
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
    block_partials<1>(acc, rs, sp);
    if (blockIdx.x == 0)
        fold_previous(csum_in, csum_out, prev, prev_nblocks, prev_colour);
}

// 2.5D-tiled half-sweep for the large levels: a tile is TJ = 256/TK rows in
// j by TK elements in kh by kTilePlanes planes in i; its block keeps a
// three-plane window of both colours (one halo row / element on each side) in
// LDS and marches along i, issuing the next plane's loads into registers
// before computing the current plane.  Each cell update is k_smooth's
// arithmetic on the same operands (bitwise the same value); only the
// grouping of the per-block partial sums of Lq + tau differs.  Blocks take
// tiles lb, lb + nblocks, ... so that nblocks <= kMaxBlocks.
constexpr int kTilePlanes = 8;

template <typename R, bool NL, int TK>
__global__ __launch_bounds__(kBlock) void k_smooth_tile(LevelView<R> L, int colour, const R *__restrict__ xc_old,
                                                        const R *__restrict__ xo, R *__restrict__ xc_new,
                                                        const double *__restrict__ csum_in, double *__restrict__ csum_out,
                                                        const double *__restrict__ prev, int prev_nblocks,
                                                        int prev_colour, ReduceSlot rs, SolveConsts sc, Span sp,
                                                        unsigned ntiles)
{
    constexpr int TJ = kBlock / TK;
    constexpr int W = (TJ + 2) * (TK + 2);  // window elements per plane and colour
    constexpr int PER = (2 * W + kBlock - 1) / kBlock;
    __shared__ R win[2][3][TJ + 2][TK + 2];  // [0]: own colour, [1]: other colour
    const int n = L.n, nh = L.nh;
    const int nK = nh / TK, nI = n / kTilePlanes;
    const R cmean = (R)((csum_in[0] + csum_in[1]) / (2.0 * (double)L.half));
    const R h2 = (R)(L.h * L.h);
    const R ih2 = (R)(1.0 / (L.h * L.h));
    const R *dc = colour ? L.db : L.dr;
    const R *tc = colour ? L.tb : L.tr;
    const int tj = threadIdx.x / TK, tk = threadIdx.x % TK;
    double acc[1] = {0.0};
    R pre[PER];
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        const int ib = (int)(tile % nI), kb = (int)((tile / nI) % nK), jb = (int)(tile / ((unsigned)nI * nK));
        const int i0 = ib * kTilePlanes, j0 = jb * TJ, k0 = kb * TK;
        // window element q of a plane: colour q / W, row (q % W) / (TK + 2), column (q % W) % (TK + 2)
        auto fetch = [&](int ii) {
            ii = ii < 0 ? ii + n : (ii >= n ? ii - n : ii);
#pragma unroll
            for (int u = 0; u < PER; u++) {
                const int q = threadIdx.x + u * kBlock;
                if (q < 2 * W) {
                    const int which = q / W, r = (q % W) / (TK + 2), c = (q % W) % (TK + 2);
                    int jj = j0 - 1 + r, kk = k0 - 1 + c;
                    jj = jj < 0 ? jj + n : (jj >= n ? jj - n : jj);
                    kk = kk < 0 ? kk + nh : (kk >= nh ? kk - nh : kk);
                    pre[u] = (which ? xo : xc_old)[((unsigned)ii * n + jj) * nh + kk];
                }
            }
        };
        auto store = [&](int slot) {
#pragma unroll
            for (int u = 0; u < PER; u++) {
                const int q = threadIdx.x + u * kBlock;
                if (q < 2 * W) {
                    const int which = q / W, r = (q % W) / (TK + 2), c = (q % W) % (TK + 2);
                    win[which][slot][r][c] = pre[u];
                }
            }
        };
        fetch(i0 - 1);
        store(0);
        fetch(i0);
        store(1);
        fetch(i0 + 1);
        store(2);
        __syncthreads();
        for (int t = 0; t < kTilePlanes; t++) {
            const int i = i0 + t;
            const int sm = t % 3, s0 = (t + 1) % 3, sp1 = (t + 2) % 3;  // planes i - 1, i, i + 1
            if (t + 1 < kTilePlanes)
                fetch(i + 2);  // into registers, stored after this plane
            const int j = j0 + tj, kh = k0 + tk;
            const int p = (i + j + colour) & 1;
            const int a = tj + 1, b = tk + 1;        // window coordinates of the cell
            const int bm = tk + p, bp = tk + 1 + p;  // its kh - 1 + p and kh + p neighbours
            R tsh;
            R S;
            if (NL)
                S = stencil_eval<R>(win[1][sp1][a][b], win[1][sm][a][b], win[1][s0][a + 1][b], win[1][s0][a - 1][b],
                                    win[1][s0][a][bp], win[1][s0][a][bm], win[0][sp1][a + 1][b], win[0][sp1][a - 1][b],
                                    win[0][sm][a + 1][b], win[0][sm][a - 1][b], win[0][sp1][a][bp],
                                    win[0][sp1][a][bm], win[0][sm][a][bp], win[0][sm][a][bm], win[0][s0][a + 1][bp],
                                    win[0][s0][a + 1][bm], win[0][s0][a - 1][bp], win[0][s0][a - 1][bm], true, tsh);
            else
                S = stencil_eval<R>(win[1][sp1][a][b], win[1][sm][a][b], win[1][s0][a + 1][b], win[1][s0][a - 1][b],
                                    win[1][s0][a][bp], win[1][s0][a][bm], (R)0, (R)0, (R)0, (R)0, (R)0, (R)0, (R)0,
                                    (R)0, (R)0, (R)0, (R)0, (R)0, false, tsh);
            const unsigned e = ((unsigned)i * n + j) * nh + kh;
            const R bsrc = (R)sc.beta * dc[e];
            int isv;
            const R lq = root_lap<R>(bsrc, tsh * ih2 * ih2, sc, NL, isv);
            const R v = lq + (tc ? tc[e] : (R)0);
            xc_new[e] = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
            acc[0] += (double)v;
            __syncthreads();
            if (t + 1 < kTilePlanes)
                store(sm);  // plane i + 2 replaces plane i - 1
            __syncthreads();
        }
    }
    block_partials<1>(acc, rs, sp);
    if (blockIdx.x == 0)
        fold_previous(csum_in, csum_out, prev, prev_nblocks, prev_colour);
}

// Whether the tiled half-sweep applies to a level (and with which TK).
static inline int tile_width(int n)
{
    if (n < 64 || n % kTilePlanes)
        return 0;
    const int nh = n / 2;
    if (nh % 64 == 0 && n % (kBlock / 64) == 0)
        return 64;
    if (nh % 32 == 0 && n % (kBlock / 32) == 0)
        return 32;
    return 0;
}

template <typename R>
void launch_smooth(const LevelView<R> &L, int colour, const R *xc_old, const R *xo, R *xc_new, const double *csum_in,
                   double *csum_out, const double *prev, int prev_nblocks, int prev_colour, ReduceSlot rs,
                   SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out, bool tiled)
{
    const int tk = tiled ? tile_width(L.n) : 0;
    if (tk) {
        // Span only carries the block count (XCD mapping, partials)
        const unsigned ntiles = (unsigned)((L.n / (kBlock / tk)) * (L.nh / tk) * (L.n / kTilePlanes));
        Span sp;
        unsigned nb = ntiles < (unsigned)kMaxBlocks ? ntiles : (unsigned)kMaxBlocks;
        if (nb >= 8)
            nb -= nb % 8;
        sp.nblocks = nb;
        sp.chunk = kBlock;
        sp.total = nb * kBlock;
        *nblocks_out = (int)nb;
#define PM_TILE(NLV, TKV)                                                                                              \
    hipLaunchKernelGGL((k_smooth_tile<R, NLV, TKV>), dim3(nb), dim3(kBlock), 0, st, L, colour, xc_old, xo, xc_new,      \
                       csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, ntiles)
        if (nonlinear) {
            if (tk == 64)
                PM_TILE(true, 64);
            else
                PM_TILE(true, 32);
        } else {
            if (tk == 64)
                PM_TILE(false, 64);
            else
                PM_TILE(false, 32);
        }
#undef PM_TILE
        return;
    }
    const Span sp = make_span(L.half);
    *nblocks_out = (int)sp.nblocks;
    if (nonlinear)
        hipLaunchKernelGGL((k_smooth<R, true>), dim3(sp.nblocks), dim3(kBlock), 0, st, L, colour, xc_old, xo, xc_new,
                           csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp);
    else
        hipLaunchKernelGGL((k_smooth<R, false>), dim3(sp.nblocks), dim3(kBlock), 0, st, L, colour, xc_old, xo, xc_new,
                           csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp);
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
                double lqt;
                int isv;
                const double r = cell_residual<double, R, NL>(F, xr, xb, fc, i, j, K, ef, cm, sc, lqt, isv);
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
                                                              Span sp)
{
    const double cm = (csum[0] + csum[1]) / (2.0 * (double)F.half);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    restrict_cell<R, NL>(F, xr, xb, cm, C, cxr, cxb, sc, e, acc);
    block_partials<4>(acc, rs, sp);
}

template <typename R>
void launch_residual_restrict(const LevelView<R> &F, const R *xr, const R *xb, const double *csum,
                              const LevelView<R> &C, R *cxr, R *cxb, ReduceSlot rs, SolveConsts sc, bool nonlinear,
                              hipStream_t st)
{
    const Span sp = make_span(2 * C.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_residual_restrict<R, true>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, C,
                           cxr, cxb, rs, sc, sp);
    else
        hipLaunchKernelGGL((k_residual_restrict<R, false>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, C,
                           cxr, cxb, rs, sc, sp);
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
                                                    int accumulate_only)
{
    double acc[2] = {0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    fas_cell<R, NL>(C, xr, xb, sc, e, accumulate_only, acc);
    block_partials<2>(acc, rs, sp);
}

template <typename R>
void launch_fas_tau(const LevelView<R> &C, const R *xr, const R *xb, double *csum, ReduceSlot rs, SolveConsts sc,
                    bool nonlinear, bool accumulate_only, hipStream_t st)
{
    const Span sp = make_span(2 * C.half);
    const int acc_only = (accumulate_only || C.tr == nullptr) ? 1 : 0;
    if (nonlinear)
        hipLaunchKernelGGL((k_fas_tau<R, true>), dim3(sp.nblocks), dim3(kBlock), 0, st, C, xr, xb, rs, sc, sp,
                           acc_only);
    else
        hipLaunchKernelGGL((k_fas_tau<R, false>), dim3(sp.nblocks), dim3(kBlock), 0, st, C, xr, xb, rs, sc, sp,
                           acc_only);
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
                                                    const R *__restrict__ cxb, Span sp)
{
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
                            hipStream_t st)
{
    const Span sp = make_span(2 * C.half);
    hipLaunchKernelGGL((k_prolong<R, true>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, C, cxr, cxb, sp);
}

template <typename R>
void launch_prolong_full(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                         hipStream_t st)
{
    const Span sp = make_span(2 * C.half);
    hipLaunchKernelGGL((k_prolong<R, false>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, C, cxr, cxb, sp);
}

// ------------------------------------------------------------- coarsest
// One workgroup, n <= 6: red-black Gauss-Seidel in FP64 in LDS with the exact
// mean of Lq + tau recomputed before every half-sweep, until the largest
// update falls below 1e-14 of the largest value or `sweeps` sweeps are done.
constexpr int kCoarseMax = 216;
constexpr double kCoarseTol = 1e-14;

// Device part, for any block size >= n^3 that is a multiple of 64 (all
// threads of the block must call it).
template <typename R, bool NL>
__device__ void coarsest_solve(const LevelView<R> &C, R *xr, R *xb, const SolveConsts &sc, int sweeps, double tol)
{
    __shared__ double x[kCoarseMax], d[kCoarseMax], t[kCoarseMax];
    __shared__ double red[16][2];
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
        double mx = 0.0, md = maxd;
        if (q < N)
            mx = fabs(x[q]);
        for (int o = 32; o > 0; o >>= 1) {
            mx = fmax(mx, __shfl_down(mx, o, 64));
            md = fmax(md, __shfl_down(md, o, 64));
        }
        if (lane == 0) {
            red[wid][0] = mx;
            red[wid][1] = md;
        }
        __syncthreads();
        double gx = 0.0, gd = 0.0;
        for (int w = 0; w < nw; w++) {
            gx = fmax(gx, red[w][0]);
            gd = fmax(gd, red[w][1]);
        }
        __syncthreads();
        if (gd <= tol * gx)
            break;
    }
    if (q < N)
        (col ? xb : xr)[off] = (R)x[q];
    __syncthreads();
}

template <typename R, bool NL>
__global__ __launch_bounds__(kBlock) void k_coarsest(LevelView<R> C, R *xr, R *xb, SolveConsts sc, int sweeps,
                                                     double tol)
{
    coarsest_solve<R, NL>(C, xr, xb, sc, sweeps, tol);
}

template <typename R>
void launch_coarsest(const LevelView<R> &C, R *xr, R *xb, SolveConsts sc, bool nonlinear, int sweeps, hipStream_t st)
{
    if (nonlinear)
        hipLaunchKernelGGL((k_coarsest<R, true>), dim3(1), dim3(kBlock), 0, st, C, xr, xb, sc, sweeps, kCoarseTol);
    else
        hipLaunchKernelGGL((k_coarsest<R, false>), dim3(1), dim3(kBlock), 0, st, C, xr, xb, sc, sweeps, kCoarseTol);
}

// ------------------------------------------------------------- transfers
template <typename R>
__global__ __launch_bounds__(kBlock) void k_restrict_field(int nc, const R *__restrict__ fr, const R *__restrict__ fb,
                                                           R *__restrict__ cr, R *__restrict__ cb, Span sp)
{
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
    hipLaunchKernelGGL((k_restrict_field<R>), dim3(sp.nblocks), dim3(kBlock), 0, st, nc, fr, fb, cr, cb, sp);
}

__global__ __launch_bounds__(kBlock) void k_cast_f64_f32(const double *__restrict__ s, float *__restrict__ d, Span sp)
{
    PM_SPAN_LOOP(e, sp)
    d[e] = (float)s[e];
}

void launch_cast_f64_f32(const double *src, float *dst, long long n, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_cast_f64_f32, dim3(sp.nblocks), dim3(kBlock), 0, st, src, dst, sp);
}

// natural [i][j][k] (float or double) -> packed double, y = scale * x + shift
template <typename Tn>
__global__ __launch_bounds__(kBlock) void k_nat_to_packed(const Tn *__restrict__ nat, double *__restrict__ packed, int n,
                                                          double scale, double shift, Span sp)
{
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ec = e - (c ? half : 0u);
        int i, j, kh;
        split(ec, nh, n, i, j, kh);
        const int k = 2 * kh + ((i + j + c) & 1);
        packed[e] = scale * (double)nat[((unsigned)i * n + j) * n + k] + shift;
    }
}

void launch_natural_to_packed(const void *nat, pm_dtype dt, double *packed, int n, double scale, double shift,
                              hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n * n * n);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_nat_to_packed<double>), dim3(sp.nblocks), dim3(kBlock), 0, st, (const double *)nat,
                           packed, n, scale, shift, sp);
    else
        hipLaunchKernelGGL((k_nat_to_packed<float>), dim3(sp.nblocks), dim3(kBlock), 0, st, (const float *)nat, packed,
                           n, scale, shift, sp);
}

// packed double -> natural, subtracting sum_ptr[0] / n^3 (the mean) if given
// and adding `add`
template <typename Tn>
__global__ __launch_bounds__(kBlock) void k_packed_to_nat(const double *__restrict__ packed, Tn *__restrict__ nat, int n,
                                                          const double *sum_ptr, double add, Span sp)
{
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    const double shift = sum_ptr ? sum_ptr[0] / (2.0 * (double)half) : 0.0;
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ec = e - (c ? half : 0u);
        int i, j, kh;
        split(ec, nh, n, i, j, kh);
        const int k = 2 * kh + ((i + j + c) & 1);
        nat[((unsigned)i * n + j) * n + k] = (Tn)(packed[e] - shift + add);
    }
}

void launch_packed_to_natural(const double *packed, void *nat, pm_dtype dt, int n, double add, const double *sum_ptr,
                              hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n * n * n);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_packed_to_nat<double>), dim3(sp.nblocks), dim3(kBlock), 0, st, packed, (double *)nat, n,
                           sum_ptr, add, sp);
    else
        hipLaunchKernelGGL((k_packed_to_nat<float>), dim3(sp.nblocks), dim3(kBlock), 0, st, packed, (float *)nat, n,
                           sum_ptr, add, sp);
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
                                                        Span sp)
{
    const double cm = (csum64[0] + csum64[1]) / (2.0 * (double)F.half);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const float ih2f = (float)(1.0 / (F.h * F.h));
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
        if (!NL) {
            (c ? x32b : x32r)[ef] = 0.0f;
            (c ? G.x0b : G.x0r)[ef] = 0.0f;
            (c ? G.tb : G.tr)[ef] = (float)r;
            acc[4 + c] += (double)(float)r;
            continue;
        }
        // FP32 operator of x32 = fl(x64), each neighbour rounded on load
        const double *own = c ? xb : xr;
        const double *oth = c ? xr : xb;
        float tsh;
        const float S = stencil_terms<float, double>(own, oth, F.n, F.nh, c, i, j, kh, NL, tsh);
        const float x32 = (float)own[ef];
        const float b = (float)sc.beta * (c ? G.db : G.dr)[ef];
        int isv32;
        const float lq32 = root_lap<float>(b, tsh * ih2f * ih2f, sc, NL, isv32);
        const float lap32 = (S - 6.0f * x32) * ih2f;
        const float tau32 = (float)r + lap32 - lq32;
        (c ? x32b : x32r)[ef] = x32;
        (c ? G.x0b : G.x0r)[ef] = x32;
        (c ? G.tb : G.tr)[ef] = tau32;
        acc[4 + c] += (double)(lq32 + tau32);
    }
    block_partials<6>(acc, rs, sp);
}

void launch_mixed_outer_residual(const LevelView<double> &F64, const double *xr, const double *xb, const double *csum64,
                                 const LevelView<float> &F32, float *x32r, float *x32b, double *, ReduceSlot rs,
                                 SolveConsts sc, bool nonlinear, hipStream_t st)
{
    const Span sp = make_span(2 * F64.half);
    if (nonlinear)
        hipLaunchKernelGGL((k_mixed_outer<true>), dim3(sp.nblocks), dim3(kBlock), 0, st, F64, xr, xb, csum64, F32, x32r,
                           x32b, rs, sc, sp);
    else
        hipLaunchKernelGGL((k_mixed_outer<false>), dim3(sp.nblocks), dim3(kBlock), 0, st, F64, xr, xb, csum64, F32,
                           x32r, x32b, rs, sc, sp);
    launch_finalize(rs, sp, 6, rs.out, st);
}

__global__ __launch_bounds__(kBlock) void k_mixed_correct(double *__restrict__ x64, const float *__restrict__ x32r,
                                                          const float *__restrict__ x32b, const float *__restrict__ x0r,
                                                          const float *__restrict__ x0b, unsigned half, Span sp)
{
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ec = e - (c ? half : 0u);
        const float d = c ? x32b[ec] - x0b[ec] : x32r[ec] - x0r[ec];
        x64[e] += (double)d;
    }
}

void launch_mixed_correct(double *x64, const float *x32r, const float *x32b, const float *x0r, const float *x0b,
                          long long half, hipStream_t st)
{
    const Span sp = make_span(2 * half);
    hipLaunchKernelGGL(k_mixed_correct, dim3(sp.nblocks), dim3(kBlock), 0, st, x64, x32r, x32b, x0r, x0b,
                       (unsigned)half, sp);
}

// ------------------------------------------------------------ residual norm
template <bool NL>
__global__ __launch_bounds__(kBlock) void k_residual_norm(LevelView<double> F, const double *__restrict__ xr,
                                                          const double *__restrict__ xb, const double *__restrict__ csum,
                                                          ReduceSlot rs, SolveConsts sc, Span sp)
{
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
        hipLaunchKernelGGL((k_residual_norm<true>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, rs, sc, sp);
    else
        hipLaunchKernelGGL((k_residual_norm<false>), dim3(sp.nblocks), dim3(kBlock), 0, st, F, xr, xb, csum, rs, sc, sp);
    launch_finalize(rs, sp, 4, rs.out, st);
}

// ------------------------------------------------------------ small helpers
__global__ __launch_bounds__(kBlock) void k_field_sum(const double *__restrict__ x, ReduceSlot rs, Span sp)
{
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
    hipLaunchKernelGGL(k_field_sum, dim3(sp.nblocks), dim3(kBlock), 0, st, x, rs, sp);
    launch_finalize(rs, sp, 2, rs.out, st);
}

__global__ __launch_bounds__(kBlock) void k_subtract_mean(double *__restrict__ x, const double *sum_ptr, Span sp)
{
    const double m = sum_ptr[0] / (double)sp.total;
    PM_SPAN_LOOP(e, sp)
    x[e] -= m;
}

void launch_subtract_mean(double *x, long long n, const double *sum_ptr, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_subtract_mean, dim3(sp.nblocks), dim3(kBlock), 0, st, x, sum_ptr, sp);
}

__global__ __launch_bounds__(kBlock) void k_scale(const double *__restrict__ x, double *__restrict__ y, double a, Span sp)
{
    PM_SPAN_LOOP(e, sp)
    y[e] = a * x[e];
}

void launch_scale(const double *x, double *y, double a, long long n, hipStream_t st)
{
    const Span sp = make_span(n);
    hipLaunchKernelGGL(k_scale, dim3(sp.nblocks), dim3(kBlock), 0, st, x, y, a, sp);
}

// Zero fill as a kernel (not hipMemsetAsync), 64-bit indices: the
// workspace can exceed 2^32 words.
__global__ __launch_bounds__(kBlock) void k_zero(uint32_t *__restrict__ p, long long nw)
{
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < nw; e += (long long)gridDim.x * kBlock)
        p[e] = 0u;
}

void launch_zero(void *p, size_t bytes, hipStream_t st)
{
    const long long nw = (long long)(bytes / 4);
    long long b = (nw + kBlock - 1) / kBlock;
    if (b > kMaxBlocks)
        b = kMaxBlocks;
    hipLaunchKernelGGL(k_zero, dim3((int)(b < 1 ? 1 : b)), dim3(kBlock), 0, st, (uint32_t *)p, nw);
}

// explicit instantiations
template void launch_smooth<double>(const LevelView<double> &, int, const double *, const double *, double *,
                                    const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                    hipStream_t, int *, bool);
template void launch_smooth<float>(const LevelView<float> &, int, const float *, const float *, float *,
                                   const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                   hipStream_t, int *, bool);
template void launch_residual_restrict<double>(const LevelView<double> &, const double *, const double *,
                                               const double *, const LevelView<double> &, double *, double *,
                                               ReduceSlot, SolveConsts, bool, hipStream_t);
template void launch_residual_restrict<float>(const LevelView<float> &, const float *, const float *, const double *,
                                              const LevelView<float> &, float *, float *, ReduceSlot, SolveConsts,
                                              bool, hipStream_t);
template void launch_fas_tau<double>(const LevelView<double> &, const double *, const double *, double *, ReduceSlot,
                                     SolveConsts, bool, bool, hipStream_t);
template void launch_fas_tau<float>(const LevelView<float> &, const float *, const float *, double *, ReduceSlot,
                                    SolveConsts, bool, bool, hipStream_t);
template void launch_prolong_correct<double>(const LevelView<double> &, double *, double *, const LevelView<double> &,
                                             const double *, const double *, hipStream_t);
template void launch_prolong_correct<float>(const LevelView<float> &, float *, float *, const LevelView<float> &,
                                            const float *, const float *, hipStream_t);
template void launch_prolong_full<double>(const LevelView<double> &, double *, double *, const LevelView<double> &,
                                          const double *, const double *, hipStream_t);
template void launch_prolong_full<float>(const LevelView<float> &, float *, float *, const LevelView<float> &,
                                         const float *, const float *, hipStream_t);
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

template <typename R, bool NL>
__global__ __launch_bounds__(kBlockCycleThreads) void k_block_cycle(BlockHier<R> Barg, int l0, int fmg, int n_pre,
                                                                    int n_post, SolveConsts sc,
                                                                    const double *__restrict__ csum_l0, int cur_bits,
                                                                    int coarse_sweeps)
{
    // the level table lives in LDS: indexed by level at run time, a kernel
    // argument would be copied to private memory
    __shared__ BlockHier<R> B;
    if (threadIdx.x == 0)
        B = Barg;
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
    auto xr = [&](int l) -> R * { return B.buf[l][cur[l][0]]; };
    auto xb = [&](int l) -> R * { return B.buf[l][cur[l][1]] + B.L[l].half; };
    auto half_sweep = [&](int m, int colour) {
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
    auto fas = [&](int m, int acc_only) {
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
    auto vcycle = [&](int l) {
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
        coarsest_solve<R, NL>(B.L[L - 1], xr(L - 1), xb(L - 1), sc, coarse_sweeps, kCoarseTol);
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
        coarsest_solve<R, NL>(B.L[L - 1], xc, xc + B.L[L - 1].half, sc, coarse_sweeps, kCoarseTol);
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
}

template <typename R>
void launch_block_cycle(const BlockHier<R> &B, int l0, bool fmg, int n_pre, int n_post, SolveConsts sc, bool nonlinear,
                        const double *csum_l0, int cur_bits, int coarse_sweeps, hipStream_t st)
{
    if (nonlinear)
        hipLaunchKernelGGL((k_block_cycle<R, true>), dim3(1), dim3(kBlockCycleThreads), 0, st, B, l0, fmg ? 1 : 0,
                           n_pre, n_post, sc, csum_l0, cur_bits, coarse_sweeps);
    else
        hipLaunchKernelGGL((k_block_cycle<R, false>), dim3(1), dim3(kBlockCycleThreads), 0, st, B, l0, fmg ? 1 : 0,
                           n_pre, n_post, sc, csum_l0, cur_bits, coarse_sweeps);
}

template void launch_block_cycle<float>(const BlockHier<float> &, int, bool, int, int, SolveConsts, bool,
                                        const double *, int, int, hipStream_t);
template void launch_block_cycle<double>(const BlockHier<double> &, int, bool, int, int, SolveConsts, bool,
                                         const double *, int, int, hipStream_t);

}  // namespace pmeft
