// 2.5D-tiled kernels that evaluate the operator at both colours of a large
// level (gfx950): the fused fine residual + restriction, the coarse FAS
// source and the outer FP64 residual of the mixed-precision solve; and the
// tiled prolongation.  Each
// block walks a tile of TJ = 2 * 256 / TK rows by TK packed elements along i
// through the LDS plane ring of tile_window.h; thread (tp, tk) owns rows
// j0 + 2 tp and j0 + 2 tp + 1 at element k0 + tk, both colours, so that the
// 8 children of a coarse cell (2 planes x 2 rows x 2 colours) meet in one
// thread.  The per-cell arithmetic is that of the grid-wide kernels in
// mg_kernels.hip (same operands, same order); only the grouping of the
// per-block partial sums differs.
#include "tile_window.h"

#include <math.h>

namespace pmeft {

namespace {

// Launch geometry of a tiled both-colour kernel on a level of n cells per
// side: TK = 64 where nh allows it, else 32; PL = 8 planes per tile, or 4 when
// that leaves fewer than 1024 tiles.  Returns false where no geometry fits.
struct PairTiles {
    int TK = 0, PL = 0;
    unsigned ntiles = 0;
    Span sp;
};

bool pair_tiles(int n, int tiled, PairTiles &g)
{
    if (!tiled || n < 128)
        return false;
    const int nh = n / 2;
    g.TK = nh % 64 == 0 ? 64 : (nh % 32 == 0 ? 32 : 0);
    if (!g.TK)
        return false;
    const int TJ = 2 * kBlock / g.TK;
    if (n % TJ || n % 8)
        return false;
    const unsigned per_plane_set = (unsigned)(n / TJ) * (unsigned)(nh / g.TK);
    g.PL = per_plane_set * (unsigned)(n / 8) >= 1024 ? 8 : 4;
    g.ntiles = per_plane_set * (unsigned)(n / g.PL);
    unsigned nb = g.ntiles < (unsigned)kMaxBlocks ? g.ntiles : (unsigned)kMaxBlocks;
    if (nb >= 8)
        nb -= nb % 8;
    g.sp.nblocks = nb;
    g.sp.chunk = kBlock;
    g.sp.total = nb * kBlock;
    return true;
}

}  // namespace

// ------------------------------------------------ fused residual + restrict
// As k_residual_restrict: residual r = Lq + tau - c - lap x of the fine cells
// (in the level's precision R), coarse tau <- 8-child average of r, coarse x
// and x0 <- 8-child average of x; acc += (sum r^2, sum r, sum Lq + tau, void
// cells).  Child order within a coarse cell: plane, row, colour.
template <typename R, bool NL, int TK, int PL>
__global__ __launch_bounds__(kBlock) void k_residual_restrict_tile(LevelView<R> F, const R *__restrict__ xr,
                                                                   const R *__restrict__ xb,
                                                                   const double *__restrict__ csum, LevelView<R> C,
                                                                   R *__restrict__ cxr, R *__restrict__ cxb,
                                                                   ReduceSlot rs, SolveConsts sc, Span sp,
                                                                   unsigned ntiles, Group grp)
{
    static_assert(PL % 2 == 0, "plane pairs");
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
    constexpr int TJ = 2 * kBlock / TK;
    __shared__ RingSlots<R, TK, TJ> win;  // [0]: red, [1]: black
    const int n = F.n, nh = F.nh, nI = n / PL, nK = nh / TK;
    const int nc = C.n, nch = C.nh;
    const R cm = (R)((csum[0] + csum[1]) / (2.0 * (double)F.half));
    const R ih2 = (R)(1.0 / (F.h * F.h));
    const int tp = threadIdx.x / TK, tk = threadIdx.x % TK;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    PlaneRing<R, TK, TJ> ring;
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = ib * PL, j0 = jb * TJ, k0 = kb * TK;
        ring.setup(xr, xb, n, nh, j0, k0);
        ring.prime(win, i0);
        const unsigned e00 = ((unsigned)i0 * n + j0 + 2 * tp) * nh + k0 + tk;
        R dcur[2][2], tcur[2][2], dnxt[2][2], tnxt[2][2];  // [row][colour]
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const unsigned e = e00 + b * nh;
                dcur[b][c] = (c ? F.db : F.dr)[e];
                const R *tc = c ? F.tb : F.tr;
                tcur[b][c] = tc ? tc[e] : (R)0;
            }
        __syncthreads();
        double sr = 0.0, sx = 0.0;
#pragma unroll 1
        for (int t = 0; t < PL; t++) {
            const int i = i0 + t;
            const int sm = t & 3, s0 = (t + 1) & 3, sp1 = (t + 2) & 3;
            if (t + 1 < PL) {
                ring.fetch(i + 2);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const unsigned e = e00 + (unsigned)(t + 1) * ring.plane + b * nh;
                        dnxt[b][c] = (c ? F.db : F.dr)[e];
                        const R *tc = c ? F.tb : F.tr;
                        tnxt[b][c] = tc ? tc[e] : (R)0;
                    }
            }
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int j = j0 + 2 * tp + b, a = 2 * tp + b + 1;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const int p = (i + j + c) & 1;
                    R tsh;
                    const R S = ring_stencil<R, R, TK, TJ>(win, c, sm, s0, sp1, a, tk, p, NL, tsh);
                    const R xo = win[c][s0][a][tk + 1];
                    const R bsrc = (R)sc.beta * dcur[b][c];
                    int isv;
                    const R lq = root_lap<R>(bsrc, tsh * ih2 * ih2, sc, NL, isv);
                    const R v = lq + tcur[b][c];
                    const R lap = (S - (R)6 * xo) * ih2;
                    const double r = (double)(v - cm - lap);
                    sr += r;
                    sx += (double)xo;
                    acc[0] += r * r;
                    acc[1] += r;
                    acc[2] += (double)v;
                    acc[3] += (double)isv;
                }
            }
            if (t & 1) {  // plane pair complete: coarse cell (i / 2, j0 / 2 + tp, k0 + tk)
                const int I = i >> 1, J = (j0 >> 1) + tp, K = k0 + tk;
                const int cc = (I + J + K) & 1;
                const unsigned ec = ((unsigned)I * nc + J) * nch + (K >> 1);
                const R rx = (R)(0.125 * sx);
                (cc ? C.tb : C.tr)[ec] = (R)(0.125 * sr);
                (cc ? cxb : cxr)[ec] = rx;
                (cc ? C.x0b : C.x0r)[ec] = rx;
                sr = 0.0;
                sx = 0.0;
            }
            if (t + 1 < PL) {
                ring.store(win, (t + 3) & 3);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        dcur[b][c] = dnxt[b][c];
                        tcur[b][c] = tnxt[b][c];
                    }
            }
            __syncthreads();
        }
    }
    block_partials<4>(acc, rs, sp);
}

// --------------------------------------------------------- coarse FAS source
// As k_fas_tau: tau += lap x - Lq(x) (in FP64, stored as R) unless
// accumulate_only; acc[colour] += Lq + tau.  ZX: x is zero (nothing of it is
// loaded; its stencil terms are the zeros the general path computes).
template <typename R, bool NL, int TK, int PL, bool ZX>
__global__ __launch_bounds__(kBlock) void k_fas_tau_tile(LevelView<R> L, const R *__restrict__ xr,
                                                         const R *__restrict__ xb, ReduceSlot rs, SolveConsts sc,
                                                         Span sp, unsigned ntiles, int accumulate_only, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(L, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    constexpr int TJ = 2 * kBlock / TK;
    __shared__ RingSlots<R, TK, TJ> win;
    const int n = L.n, nh = L.nh, nI = n / PL, nK = nh / TK;
    const double ih2 = 1.0 / (L.h * L.h);
    const int tp = threadIdx.x / TK, tk = threadIdx.x % TK;
    const unsigned plane = (unsigned)n * nh;
    double acc[2] = {0.0, 0.0};
    PlaneRing<R, TK, TJ> ring;
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = ib * PL, j0 = jb * TJ, k0 = kb * TK;
        if constexpr (!ZX) {
            ring.setup(xr, xb, n, nh, j0, k0);
            ring.prime(win, i0);
        }
        const unsigned e00 = ((unsigned)i0 * n + j0 + 2 * tp) * nh + k0 + tk;
        R dcur[2][2], tcur[2][2], dnxt[2][2], tnxt[2][2];
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const unsigned e = e00 + b * nh;
                dcur[b][c] = (c ? L.db : L.dr)[e];
                const R *tc = c ? L.tb : L.tr;
                tcur[b][c] = tc ? tc[e] : (R)0;
            }
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < PL; t++) {
            const int i = i0 + t;
            const int sm = t & 3, s0 = (t + 1) & 3, sp1 = (t + 2) & 3;
            if (t + 1 < PL) {
                if constexpr (!ZX)
                    ring.fetch(i + 2);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const unsigned e = e00 + (unsigned)(t + 1) * plane + b * nh;
                        dnxt[b][c] = (c ? L.db : L.dr)[e];
                        const R *tc = c ? L.tb : L.tr;
                        tnxt[b][c] = tc ? tc[e] : (R)0;
                    }
            }
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int j = j0 + 2 * tp + b, a = 2 * tp + b + 1;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const int p = (i + j + c) & 1;
                    double tsh = 0.0, S = 0.0;
                    if constexpr (!ZX)
                        S = ring_stencil<double, R, TK, TJ>(win, c, sm, s0, sp1, a, tk, p, NL, tsh);
                    const double bsrc = sc.beta * (double)dcur[b][c];
                    int isv;
                    const double lq = root_lap<double>(bsrc, tsh * ih2 * ih2, sc, NL, isv);
                    double tv = (double)tcur[b][c];
                    if (!accumulate_only) {
                        const double lap = (S - 6.0 * (ZX ? 0.0 : (double)win[c][s0][a][tk + 1])) * ih2;
                        tv += lap - lq;
                        (c ? L.tb : L.tr)[((unsigned)i * n + j) * nh + k0 + tk] = (R)tv;
                        tv = (double)(R)tv;
                    }
                    acc[c] += lq + tv;
                }
            }
            if (t + 1 < PL) {
                if constexpr (!ZX)
                    ring.store(win, (t + 3) & 3);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        dcur[b][c] = dnxt[b][c];
                        tcur[b][c] = tnxt[b][c];
                    }
            }
            __syncthreads();
        }
    }
    block_partials<2>(acc, rs, sp);
}

// ---------------------------------------------------- mixed-precision outer
// As k_mixed_outer: FP64 residual of the FP64 iterate (norm partials in
// acc[0..3]), x32 = fl(x64) into the FP32 level's x, and the FP32 target
// tau32 = fl(r) + lap32 x32 - Lq32(x32) (nonlinear) or tau32 = fl(r) with
// x32 = 0 (linear); acc[4 + colour] += Lq32 + tau32.  CORR: the iterate is
// first corrected by the FP32 result of the previous V-cycles (MixedCorr),
// value by value as the window loads it, with k_mixed_correct's arithmetic;
// the corrected values of the tile's own cells go to cr.yr / cr.yb.  ZX: the
// iterate is zero (a solve's first step from a zero start), so nothing of it
// is loaded and its stencil terms are the zeros the general path computes.
template <bool NL, int TK, int PL, bool CORR, bool ZX>
__global__ __launch_bounds__(kBlock) void k_mixed_outer_tile(LevelView<double> F, const double *__restrict__ xr,
                                                             const double *__restrict__ xb,
                                                             const double *__restrict__ csum64, LevelView<float> G,
                                                             float *__restrict__ x32r, float *__restrict__ x32b,
                                                             ReduceSlot rs, SolveConsts sc, Span sp, unsigned ntiles,
                                                             MixedCorr cr, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    gshift_view(G, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    csum64 = gshift(csum64, go);
    x32r = gshift(x32r, go);
    x32b = gshift(x32b, go);
    cr.vr = gshift(cr.vr, go);
    cr.vb = gshift(cr.vb, go);
    cr.yr = gshift(cr.yr, go);
    cr.yb = gshift(cr.yb, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    constexpr int TJ = 2 * kBlock / TK;
    __shared__ RingSlots<double, TK, TJ> win;
    const int n = F.n, nh = F.nh, nI = n / PL, nK = nh / TK;
    const double cm = (csum64[0] + csum64[1]) / (2.0 * (double)F.half);
    const double ih2 = 1.0 / (F.h * F.h);
    const float ih2f = (float)ih2;
    const int tp = threadIdx.x / TK, tk = threadIdx.x % TK;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    using Ring = PlaneRing<double, TK, TJ>;
    Ring ring;
    // CORR: the FP32 values of this thread's window elements (same offsets as
    // the ring's), loaded with them and folded in just before the LDS store
    const float *vsrc[Ring::PER];
    float vpre[Ring::PER];
    const unsigned plane = (unsigned)n * nh;
    auto fetch = [&](int ii) {
        if constexpr (ZX)
            return;
        ring.fetch(ii);
        if constexpr (CORR) {
            const int iw = ii < 0 ? ii + n : (ii >= n ? ii - n : ii);
            const unsigned base = (unsigned)iw * ring.plane;
#pragma unroll
            for (int u = 0; u < Ring::PER; u++)
                if (u < Ring::FULL || threadIdx.x + u * kBlock < 2 * Ring::W)
                    vpre[u] = vsrc[u][base + ring.poff[u]];
        }
    };
    auto store = [&](int slot) {
        if constexpr (CORR) {
#pragma unroll
            for (int u = 0; u < Ring::PER; u++)
                if (u < Ring::FULL || threadIdx.x + u * kBlock < 2 * Ring::W) {
                    const double x = ring.pre[u];
                    const float d = NL ? vpre[u] - (float)x : vpre[u];
                    ring.pre[u] = x + (double)d;
                }
        }
        if constexpr (!ZX)
            ring.store(win, slot);
    };
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = ib * PL, j0 = jb * TJ, k0 = kb * TK;
        if constexpr (!ZX)
            ring.setup(xr, xb, n, nh, j0, k0);
        if constexpr (CORR) {
#pragma unroll
            for (int u = 0; u < Ring::PER; u++) {
                const int q = threadIdx.x + u * kBlock;
                vsrc[u] = (q < 2 * Ring::W ? q : 0) < Ring::W ? cr.vr : cr.vb;
            }
        }
        fetch(i0 - 1);
        store(0);
        fetch(i0);
        store(1);
        fetch(i0 + 1);
        store(2);
        const unsigned e00 = ((unsigned)i0 * n + j0 + 2 * tp) * nh + k0 + tk;
        // (the FP32 level's delta is fl32 of the FP64 one: rounded here
        // instead of loaded)
        double dcur[2][2], dnxt[2][2];
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int c = 0; c < 2; c++)
                dcur[b][c] = (c ? F.db : F.dr)[e00 + b * nh];
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < PL; t++) {
            const int i = i0 + t;
            const int sm = t & 3, s0 = (t + 1) & 3, sp1 = (t + 2) & 3;
            if (t + 1 < PL) {
                fetch(i + 2);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++)
                        dnxt[b][c] = (c ? F.db : F.dr)[e00 + (unsigned)(t + 1) * plane + b * nh];
            }
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int j = j0 + 2 * tp + b, a = 2 * tp + b + 1;
                const unsigned e = ((unsigned)i * n + j) * nh + k0 + tk;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const int p = (i + j + c) & 1;
                    double tsh = 0.0, S = 0.0, x64 = 0.0;
                    if constexpr (!ZX) {
                        S = ring_stencil<double, double, TK, TJ>(win, c, sm, s0, sp1, a, tk, p, NL, tsh);
                        x64 = win[c][s0][a][tk + 1];
                    }
                    if constexpr (CORR)
                        (c ? cr.yb : cr.yr)[e] = x64;
                    int isv;
                    const double lq = root_lap<double>(sc.beta * dcur[b][c], tsh * ih2 * ih2, sc, NL, isv);
                    const double r = lq - cm - (S - 6.0 * x64) * ih2;
                    acc[0] += r * r;
                    acc[1] += r;
                    acc[2] += lq;
                    acc[3] += (double)isv;
                    if (!NL) {
                        (c ? x32b : x32r)[e] = 0.0f;
                        (c ? G.tb : G.tr)[e] = (float)r;
                        acc[4 + c] += (double)(float)r;
                    } else {
                        float tsh32 = 0.0f, S32 = 0.0f;
                        if constexpr (!ZX)
                            S32 = ring_stencil<float, double, TK, TJ>(win, c, sm, s0, sp1, a, tk, p, true, tsh32);
                        const float x32 = (float)x64;
                        int isv32;
                        const float lq32 =
                            root_lap<float>((float)sc.beta * (float)dcur[b][c], tsh32 * ih2f * ih2f, sc, true, isv32);
                        const float lap32 = (S32 - 6.0f * x32) * ih2f;
                        const float tau32 = (float)r + lap32 - lq32;
                        (c ? x32b : x32r)[e] = x32;
                        (c ? G.tb : G.tr)[e] = tau32;
                        acc[4 + c] += (double)(lq32 + tau32);
                    }
                }
            }
            if (t + 1 < PL) {
                store((t + 3) & 3);
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++)
                        dcur[b][c] = dnxt[b][c];
            }
            __syncthreads();
        }
    }
    block_partials<6>(acc, rs, sp);
}

// ------------------------------------------------------------- prolongation
// As k_prolong (trilinear cell-centred, weights 3/4 and 1/4 axis by axis, in
// the same order), tiled over coarse cells: a block walks RPc = 256 / TKc
// coarse rows by TKc coarse cells along I, keeping coarse planes I - 1, I,
// I + 1 (x_H - x0_H, or x_H for the full-approximation start, in FP64 and in
// natural K order) in a four-slot LDS ring; thread (tp, tk) writes the 8
// children of coarse cell (I, J0 + tp, K0 + tk).
template <typename R, bool CORR, int TKc, int PLc>
__global__ __launch_bounds__(kBlock) void k_prolong_tile(LevelView<R> F, R *__restrict__ xr, R *__restrict__ xb,
                                                         LevelView<R> C, const R *__restrict__ cxr,
                                                         const R *__restrict__ cxb, Span sp, unsigned ntiles,
                                                         Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(F, go);
    gshift_view(C, go);
    xr = gshift(xr, go);
    xb = gshift(xb, go);
    cxr = gshift(cxr, go);
    cxb = gshift(cxb, go);
    constexpr int RPc = kBlock / TKc;
    constexpr int WR = RPc + 2, WC = TKc + 2, W = WR * WC;
    constexpr int PER = (W + kBlock - 1) / kBlock;
    __shared__ double win[4][WR][WC];
    const int nc = C.n, nch = C.nh, n = F.n, nh = F.nh;
    const int nI = nc / PLc, nK = nc / TKc;
    const int tp = threadIdx.x / TKc, tk = threadIdx.x % TKc;
    const unsigned cplane = (unsigned)nc * nch;
    double *wflat = &win[0][0][0];
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int I0 = ib * PLc, J0 = jb * RPc, K0 = kb * TKc;
        // window element q: row q / WC (J = J0 - 1 + row), column q % WC
        // (K = K0 - 1 + column); packed offset within a plane and J + K parity
        unsigned poff[PER];
        int par[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int q = threadIdx.x + u * kBlock;
            const int qq = q < W ? q : 0;
            int Jw = J0 - 1 + qq / WC, Kw = K0 - 1 + qq % WC;
            Jw = Jw < 0 ? Jw + nc : (Jw >= nc ? Jw - nc : Jw);
            Kw = Kw < 0 ? Kw + nc : (Kw >= nc ? Kw - nc : Kw);
            poff[u] = (unsigned)Jw * nch + (Kw >> 1);
            par[u] = (Jw + Kw) & 1;
        }
        double pre[PER];
        auto fetch = [&](int I) {
            I = I < 0 ? I + nc : (I >= nc ? I - nc : I);
            const unsigned base = (unsigned)I * cplane;
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kBlock < W) {
                    const int cc = (I + par[u]) & 1;
                    const unsigned o = base + poff[u];
                    double v = (double)(cc ? cxb : cxr)[o];
                    if (CORR)
                        v -= (double)(cc ? C.x0b : C.x0r)[o];
                    pre[u] = v;
                }
        };
        auto store = [&](int slot) {
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kBlock < W)
                    wflat[slot * W + threadIdx.x + u * kBlock] = pre[u];
        };
        fetch(I0 - 1);
        store(0);
        fetch(I0);
        store(1);
        fetch(I0 + 1);
        store(2);
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < PLc; t++) {
            const int I = I0 + t, J = J0 + tp, K = K0 + tk;
            const int sl[3] = {t & 3, (t + 1) & 3, (t + 2) & 3};  // planes I - 1, I, I + 1
            if (t + 1 < PLc)
                fetch(I + 2);
            R xf[2][2][2];  // fine iterate of the children [aa][bb][c]
            if (CORR) {
#pragma unroll
                for (int aa = 0; aa < 2; aa++)
#pragma unroll
                    for (int bb = 0; bb < 2; bb++) {
                        const unsigned ef = ((unsigned)(2 * I + aa) * n + 2 * J + bb) * nh + K;
#pragma unroll
                        for (int c = 0; c < 2; c++)
                            xf[aa][bb][c] = (((aa + bb + c) & 1) ? xb : xr)[ef];
                    }
            }
            double lk[3][3][2];
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    const double *row = &win[sl[a]][tp + b][tk];
                    lk[a][b][0] = 0.75 * row[1] + 0.25 * row[0];
                    lk[a][b][1] = 0.75 * row[1] + 0.25 * row[2];
                }
#pragma unroll
            for (int aa = 0; aa < 2; aa++)
#pragma unroll
                for (int bb = 0; bb < 2; bb++) {
                    const unsigned ef = ((unsigned)(2 * I + aa) * n + 2 * J + bb) * nh + K;
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        double lj[3];
#pragma unroll
                        for (int a = 0; a < 3; a++)
                            lj[a] = 0.75 * lk[a][1][c] + 0.25 * lk[a][bb ? 2 : 0][c];
                        const double v = 0.75 * lj[1] + 0.25 * lj[aa ? 2 : 0];
                        R *x = ((aa + bb + c) & 1) ? xb : xr;
                        x[ef] = CORR ? (R)((double)xf[aa][bb][c] + v) : (R)v;
                    }
                }
            if (t + 1 < PLc)
                store((t + 3) & 3);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ launchers
#define PM_PAIR_DISPATCH(KERNEL_TK_PL)                                                                                 \
    if (g.TK == 64 && g.PL == 8)                                                                                       \
        KERNEL_TK_PL(64, 8);                                                                                           \
    else if (g.TK == 64)                                                                                               \
        KERNEL_TK_PL(64, 4);                                                                                           \
    else if (g.PL == 8)                                                                                                \
        KERNEL_TK_PL(32, 8);                                                                                           \
    else                                                                                                               \
        KERNEL_TK_PL(32, 4);

template <typename R>
bool launch_residual_restrict_tiled(const LevelView<R> &F, const R *xr, const R *xb, const double *csum,
                                    const LevelView<R> &C, R *cxr, R *cxb, ReduceSlot rs, SolveConsts sc,
                                    bool nonlinear, hipStream_t st, int tiled, Span *sp_out)
{
    PairTiles g;
    if (!pair_tiles(F.n, tiled, g))
        return false;
#define PM_RR(TKV, PLV)                                                                                                \
    do {                                                                                                               \
        if (nonlinear)                                                                                                 \
            hipLaunchKernelGGL((k_residual_restrict_tile<R, true, TKV, PLV>), group_grid(g.sp.nblocks), dim3(kBlock), \
                               0, st, F, xr, xb, csum, C, cxr, cxb, rs, sc, g.sp, g.ntiles, cur_group());              \
        else                                                                                                           \
            hipLaunchKernelGGL((k_residual_restrict_tile<R, false, TKV, PLV>), group_grid(g.sp.nblocks), dim3(kBlock), \
                               0, st, F, xr, xb, csum, C, cxr, cxb, rs, sc, g.sp, g.ntiles, cur_group());              \
    } while (0)
    PM_PAIR_DISPATCH(PM_RR)
#undef PM_RR
    *sp_out = g.sp;
    return true;
}

template <typename R>
bool launch_fas_tau_tiled(const LevelView<R> &L, const R *xr, const R *xb, ReduceSlot rs, SolveConsts sc,
                          bool nonlinear, int accumulate_only, hipStream_t st, int tiled, Span *sp_out,
                          bool zero_iterate)
{
    PairTiles g;
    if (!pair_tiles(L.n, tiled, g))
        return false;
#define PM_FT1(NLV, TKV, PLV, ZV)                                                                                      \
    hipLaunchKernelGGL((k_fas_tau_tile<R, NLV, TKV, PLV, ZV>), group_grid(g.sp.nblocks), dim3(kBlock), 0, st, L, xr,  \
                       xb, rs, sc, g.sp, g.ntiles, accumulate_only, cur_group())
#define PM_FT(TKV, PLV)                                                                                                \
    do {                                                                                                               \
        if (nonlinear && zero_iterate)                                                                                 \
            PM_FT1(true, TKV, PLV, true);                                                                              \
        else if (nonlinear)                                                                                            \
            PM_FT1(true, TKV, PLV, false);                                                                             \
        else if (zero_iterate)                                                                                         \
            PM_FT1(false, TKV, PLV, true);                                                                             \
        else                                                                                                           \
            PM_FT1(false, TKV, PLV, false);                                                                            \
    } while (0)
    PM_PAIR_DISPATCH(PM_FT)
#undef PM_FT
#undef PM_FT1
    *sp_out = g.sp;
    return true;
}

bool mixed_outer_tiles(int n, int tiled)
{
    PairTiles g;
    return pair_tiles(n, tiled, g);
}

bool launch_mixed_outer_tiled(const LevelView<double> &F64, const double *xr, const double *xb, const double *csum64,
                              const LevelView<float> &F32, float *x32r, float *x32b, ReduceSlot rs, SolveConsts sc,
                              bool nonlinear, hipStream_t st, int tiled, Span *sp_out, const MixedCorr *corr,
                              bool zero_iterate)
{
    PairTiles g;
    if (!pair_tiles(F64.n, tiled, g))
        return false;
    const MixedCorr cr = corr ? *corr : MixedCorr{};
#define PM_MO1(NLV, TKV, PLV, CV, ZV)                                                                                  \
    hipLaunchKernelGGL((k_mixed_outer_tile<NLV, TKV, PLV, CV, ZV>), group_grid(g.sp.nblocks), dim3(kBlock), 0, st,    \
                       F64, xr, xb, csum64, F32, x32r, x32b, rs, sc, g.sp, g.ntiles, cr, cur_group())
#define PM_MO2(NLV, TKV, PLV)                                                                                          \
    do {                                                                                                               \
        if (corr)                                                                                                      \
            PM_MO1(NLV, TKV, PLV, true, false);                                                                        \
        else if (zero_iterate)                                                                                         \
            PM_MO1(NLV, TKV, PLV, false, true);                                                                        \
        else                                                                                                           \
            PM_MO1(NLV, TKV, PLV, false, false);                                                                       \
    } while (0)
#define PM_MO(TKV, PLV)                                                                                                \
    do {                                                                                                               \
        if (nonlinear)                                                                                                 \
            PM_MO2(true, TKV, PLV);                                                                                    \
        else                                                                                                           \
            PM_MO2(false, TKV, PLV);                                                                                   \
    } while (0)
    PM_PAIR_DISPATCH(PM_MO)
#undef PM_MO
#undef PM_MO2
#undef PM_MO1
    *sp_out = g.sp;
    return true;
}
#undef PM_PAIR_DISPATCH

template <typename R>
bool launch_prolong_tiled(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                          bool corr, hipStream_t st, int tiled)
{
    const int nc = C.n;
    if (!tiled || nc < 64)
        return false;
    const int TKc = nc % 64 == 0 ? 64 : (nc % 32 == 0 ? 32 : 0);
    if (!TKc || nc % (kBlock / TKc) || nc % 4)
        return false;
    const unsigned per_set = (unsigned)(nc / (kBlock / TKc)) * (unsigned)(nc / TKc);
    const int PLc = per_set * (unsigned)(nc / 4) >= 1024 ? 4 : 2;
    const unsigned ntiles = per_set * (unsigned)(nc / PLc);
    Span sp;
    unsigned nb = ntiles < (unsigned)kMaxBlocks ? ntiles : (unsigned)kMaxBlocks;
    if (nb >= 8)
        nb -= nb % 8;
    sp.nblocks = nb;
    sp.chunk = kBlock;
    sp.total = nb * kBlock;
#define PM_PT(CV, TKV, PLV)                                                                                            \
    hipLaunchKernelGGL((k_prolong_tile<R, CV, TKV, PLV>), group_grid(nb), dim3(kBlock), 0, st, F, xr, xb, C, cxr, cxb, \
                       sp, ntiles, cur_group())
#define PM_PT_C(TKV, PLV)                                                                                              \
    do {                                                                                                               \
        if (corr)                                                                                                      \
            PM_PT(true, TKV, PLV);                                                                                     \
        else                                                                                                           \
            PM_PT(false, TKV, PLV);                                                                                    \
    } while (0)
    if (TKc == 64 && PLc == 4)
        PM_PT_C(64, 4);
    else if (TKc == 64)
        PM_PT_C(64, 2);
    else if (PLc == 4)
        PM_PT_C(32, 4);
    else
        PM_PT_C(32, 2);
#undef PM_PT_C
#undef PM_PT
    return true;
}

template bool launch_residual_restrict_tiled<double>(const LevelView<double> &, const double *, const double *,
                                                     const double *, const LevelView<double> &, double *, double *,
                                                     ReduceSlot, SolveConsts, bool, hipStream_t, int, Span *);
template bool launch_residual_restrict_tiled<float>(const LevelView<float> &, const float *, const float *,
                                                    const double *, const LevelView<float> &, float *, float *,
                                                    ReduceSlot, SolveConsts, bool, hipStream_t, int, Span *);
template bool launch_fas_tau_tiled<double>(const LevelView<double> &, const double *, const double *, ReduceSlot,
                                           SolveConsts, bool, int, hipStream_t, int, Span *, bool);
template bool launch_prolong_tiled<double>(const LevelView<double> &, double *, double *, const LevelView<double> &,
                                           const double *, const double *, bool, hipStream_t, int);
template bool launch_prolong_tiled<float>(const LevelView<float> &, float *, float *, const LevelView<float> &,
                                          const float *, const float *, bool, hipStream_t, int);
template bool launch_fas_tau_tiled<float>(const LevelView<float> &, const float *, const float *, ReduceSlot,
                                          SolveConsts, bool, int, hipStream_t, int, Span *, bool);

}  // namespace pmeft
