// Red-black half-sweeps of the multigrid levels (gfx950): the grid-wide
// kernel for every level and the 2.5D-tiled kernel for the large levels.
// The operator and the cell update are those of mg_stencil.h.
#include "tile_window.h"

#include <math.h>

namespace pmeft {

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
                                                   ReduceSlot rs, SolveConsts sc, Span sp, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(L, go);
    xc_old = gshift(xc_old, go);
    xo = gshift(xo, go);
    xc_new = gshift(xc_new, go);
    csum_in = gshift(csum_in, go);
    csum_out = gshift(csum_out, go);
    prev = gshift(prev, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
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

// 2.5D-tiled half-sweep for the large levels: a tile is TJ = CJ * 256 / TK
// rows in j by TK elements in kh by PL planes in i; each thread computes CJ
// cells of a plane (rows tj, tj + 256/TK, ...).  The block keeps a
// three-plane window of both colours (one halo row / element on each side) in
// a four-slot LDS ring and marches along i, issuing the next plane's loads
// into registers before computing the current plane and storing them into the
// free slot after it (one barrier per plane).  Each cell update is k_smooth's
// arithmetic on the same operands (bitwise the same value); only the
// grouping of the per-block partial sums of Lq + tau differs.  Blocks take
// tiles lb, lb + nblocks, ... so that nblocks <= kMaxBlocks.
template <typename R, bool NL, int TK, int CJ, int PL>
__global__ __launch_bounds__(kBlock) void k_smooth_tile(LevelView<R> L, int colour, const R *__restrict__ xc_old,
                                                        const R *__restrict__ xo, R *__restrict__ xc_new,
                                                        const double *__restrict__ csum_in, double *__restrict__ csum_out,
                                                        const double *__restrict__ prev, int prev_nblocks,
                                                        int prev_colour, ReduceSlot rs, SolveConsts sc, Span sp,
                                                        unsigned ntiles, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(L, go);
    xc_old = gshift(xc_old, go);
    xo = gshift(xo, go);
    xc_new = gshift(xc_new, go);
    csum_in = gshift(csum_in, go);
    csum_out = gshift(csum_out, go);
    prev = gshift(prev, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    constexpr int RS = kBlock / TK;  // rows per pass of the block
    constexpr int TJ = CJ * RS;
    __shared__ RingSlots<R, TK, TJ> win;  // [0]: own colour, [1]: other colour
    const int n = L.n, nh = L.nh;
    const int nK = nh / TK, nI = n / PL;
    const R cmean = (R)((csum_in[0] + csum_in[1]) / (2.0 * (double)L.half));
    const R h2 = (R)(L.h * L.h);
    const R ih2 = (R)(1.0 / (L.h * L.h));
    const R *dc = colour ? L.db : L.dr;
    const R *tc = colour ? L.tb : L.tr;
    const int tj = threadIdx.x / TK, tk = threadIdx.x % TK;
    double acc[1] = {0.0};
    PlaneRing<R, TK, TJ, NL ? 2 : 1> ring;
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = ib * PL, j0 = jb * TJ, k0 = kb * TK;
        ring.setup(xc_old, xo, n, nh, j0, k0);
        ring.prime(win, i0);
        // density and tau of this thread's cells, one plane ahead as well
        const unsigned e00 = ((unsigned)i0 * n + j0 + tj) * nh + k0 + tk;
        R dcur[CJ], tcur[CJ], dnxt[CJ], tnxt[CJ];
#pragma unroll
        for (int cj = 0; cj < CJ; cj++) {
            dcur[cj] = dc[e00 + cj * RS * nh];
            tcur[cj] = tc ? tc[e00 + cj * RS * nh] : (R)0;
        }
        __syncthreads();
        for (int t = 0; t < PL; t++) {
            const int i = i0 + t;
            const int sm = t & 3, s0 = (t + 1) & 3, sp1 = (t + 2) & 3;  // planes i - 1, i, i + 1
            if (t + 1 < PL) {
                ring.fetch(i + 2);  // into registers, stored after this plane
#pragma unroll
                for (int cj = 0; cj < CJ; cj++) {
                    const unsigned en = e00 + (unsigned)(t + 1) * ring.plane + cj * RS * nh;
                    dnxt[cj] = dc[en];
                    tnxt[cj] = tc ? tc[en] : (R)0;
                }
            }
#pragma unroll
            for (int cj = 0; cj < CJ; cj++) {
                const int j = j0 + tj + cj * RS, kh = k0 + tk;
                const int p = (i + j + colour) & 1;
                R tsh;
                const R S = ring_stencil<R, R, TK, TJ>(win, 0, sm, s0, sp1, tj + cj * RS + 1, tk, p, NL, tsh);
                const unsigned e = ((unsigned)i * n + j) * nh + kh;
                const R tv = tcur[cj];
                const R bsrc = (R)sc.beta * dcur[cj];
                int isv;
                const R lq = root_lap<R>(bsrc, tsh * ih2 * ih2, sc, NL, isv);
                const R v = lq + tv;
                xc_new[e] = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
                acc[0] += (double)v;
            }
            if (t + 1 < PL) {
                ring.store(win, (t + 3) & 3);
#pragma unroll
                for (int cj = 0; cj < CJ; cj++) {
                    dcur[cj] = dnxt[cj];
                    tcur[cj] = tnxt[cj];
                }
            }
            __syncthreads();
        }
    }
    block_partials<1>(acc, rs, sp);
    if (blockIdx.x == 0)
        fold_previous(csum_in, csum_out, prev, prev_nblocks, prev_colour);
}

// Tile configuration of a level for a tiling choice (1: small tiles, 2:
// large tiles where they still give at least 512 tiles, else small; 3: the
// largest tiles where they still give 512, else as 2): 0 = untiled; 1 = (TK
// 64, CJ 2, 16 planes, 8 in FP64); 2 = (TK 64, CJ 1, 8 planes); 3 = (TK 32,
// CJ 1, 8 planes); 4 = (TK 64, CJ 4, 16 planes).  Larger tiles re-read less
// halo (j and i halos of 2 rows and 2 planes per tile), which counts where
// the level's working set does not stay in the last-level cache (FP64 at
// 256^3), at the price of LDS (two FP64 blocks per CU with CJ 4).
constexpr int kMinTiles = 256;

static inline int tile_config(int n, int choice)
{
    if (choice == 0 || n < 64)
        return 0;
    const int nh = n / 2;
    if (choice == 3 && nh % 64 == 0 && n % 16 == 0 && (n / 16) * (nh / 64) * (n / 16) >= 512)
        return 4;
    if (choice >= 2 && nh % 64 == 0 && n % 16 == 0 && (n / 8) * (nh / 64) * (n / 16) >= 512)
        return 1;
    // small tiles only where they still occupy the chip: a level with fewer
    // than kMinTiles of them runs the grid-wide kernel (more blocks)
    if (nh % 64 == 0 && n % 8 == 0 && (n / 4) * (nh / 64) * (n / 8) >= kMinTiles)
        return 2;
    if (nh % 32 == 0 && n % 8 == 0 && (n / 8) * (nh / 32) * (n / 8) >= kMinTiles)
        return 3;
    return 0;
}

template <typename R>
void launch_smooth(const LevelView<R> &L, int colour, const R *xc_old, const R *xo, R *xc_new, const double *csum_in,
                   double *csum_out, const double *prev, int prev_nblocks, int prev_colour, ReduceSlot rs,
                   SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out, int tiled)
{
    const int cfg = tile_config(L.n, tiled);
    if (cfg) {
        // FP64 large tiles march 8 planes: three such blocks fit a CU (LDS), and
        // 16-plane tiles would leave a third of the last round of blocks idle
        constexpr int PL1 = sizeof(R) == 8 ? 8 : 16;
        const int TK = cfg == 3 ? 32 : 64;
        const int TJ = (cfg == 4 ? 4 : (cfg == 1 ? 2 : 1)) * kBlock / TK;
        const int PL = cfg == 4 ? 16 : (cfg == 1 ? PL1 : 8);
        const unsigned ntiles = (unsigned)((L.n / TJ) * (L.nh / TK) * (L.n / PL));
        // Span only carries the block count (XCD mapping, partials)
        Span sp;
        unsigned nb = ntiles < (unsigned)kMaxBlocks ? ntiles : (unsigned)kMaxBlocks;
        if (nb >= 8)
            nb -= nb % 8;
        sp.nblocks = nb;
        sp.chunk = kBlock;
        sp.total = nb * kBlock;
        *nblocks_out = (int)nb;
#define PM_TILE(NLV, TKV, CJV, PLV)                                                                                    \
    hipLaunchKernelGGL((k_smooth_tile<R, NLV, TKV, CJV, PLV>), group_grid(nb), dim3(kBlock), 0, st, L, colour, xc_old, \
                       xo, xc_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, ntiles, cur_group())
        if (nonlinear) {
            if (cfg == 4)
                PM_TILE(true, 64, 4, 16);
            else if (cfg == 1)
                PM_TILE(true, 64, 2, PL1);
            else if (cfg == 2)
                PM_TILE(true, 64, 1, 8);
            else
                PM_TILE(true, 32, 1, 8);
        } else {
            if (cfg == 4)
                PM_TILE(false, 64, 4, 16);
            else if (cfg == 1)
                PM_TILE(false, 64, 2, PL1);
            else if (cfg == 2)
                PM_TILE(false, 64, 1, 8);
            else
                PM_TILE(false, 32, 1, 8);
        }
#undef PM_TILE
        return;
    }
    const Span sp = make_span(L.half);
    *nblocks_out = (int)sp.nblocks;
    if (nonlinear)
        hipLaunchKernelGGL((k_smooth<R, true>), group_grid(sp.nblocks), dim3(kBlock), 0, st, L, colour, xc_old, xo,
                           xc_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, cur_group());
    else
        hipLaunchKernelGGL((k_smooth<R, false>), group_grid(sp.nblocks), dim3(kBlock), 0, st, L, colour, xc_old, xo,
                           xc_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, cur_group());
}

template void launch_smooth<double>(const LevelView<double> &, int, const double *, const double *, double *,
                                    const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                    hipStream_t, int *, int);
template void launch_smooth<float>(const LevelView<float> &, int, const float *, const float *, float *,
                                   const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                   hipStream_t, int *, int);

}  // namespace pmeft
