// Both colours of a red-black Gauss-Seidel sweep in one launch (gfx950), for
// the large levels.  A block owns a tile of TJ rows (j) by TK packed elements
// (kh) and marches along i over PL planes.  At plane i it updates the red
// cells of plane i + 1 on the tile plus a one-cell halo in j and kh, then
// the black cells of plane i on the tile, whose face neighbours are those new
// red values: the sweep reads each colour's old values once and writes each
// new value once (3 words per cell with the source, 4 with the FAS source
// tau), where two half-sweep launches read the red values twice.  The red
// cells of the halo, and of planes i0 - 1 and i0 + PL, are updated by
// neighbouring tiles as well; only the tile's own cells are written.
//
// LDS: a five-slot ring of old planes i - 1 .. i + 2 (both colours, two-cell
// halo; the slot of plane i - 2 takes the prefetched plane i + 3) and a
// three-slot ring of the new red planes i - 1 .. i + 1 (one-cell halo).  Each
// cell's update is that of the half-sweep kernels on the same operands; the
// black half uses the lagged mean the red half uses (one launch), so a
// fused sweep differs from two half-sweeps by the mean's lag only.
#include "tile_window.h"

#include <math.h>

namespace pmeft {

namespace {

// Operator pieces (S, and Tsh when nonlinear) of a cell from its other-
// colour planes (om, o0, op: planes i - 1, i, i + 1; the cell at row ro,
// column co, row length ldo) and own-colour planes (wm, w0, wp; row rw,
// column cw, row length ldw); p = (i + j + colour) & 1 selects the packed
// k-neighbours kh - 1 + p and kh + p.
template <typename T, typename R>
__device__ __forceinline__ T planes_stencil(const R *om, const R *o0, const R *op, int ldo, int ro, int co,
                                            const R *wm, const R *w0, const R *wp, int ldw, int rw, int cw, int p,
                                            bool nonlinear, T &tsh)
{
    const int oc = ro * ldo + co, wc = rw * ldw + cw;
    if (!nonlinear)
        return stencil_eval<T>((T)op[oc], (T)om[oc], (T)o0[oc + ldo], (T)o0[oc - ldo], (T)o0[oc + p],
                               (T)o0[oc - 1 + p], (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0,
                               (T)0, false, tsh);
    return stencil_eval<T>((T)op[oc], (T)om[oc], (T)o0[oc + ldo], (T)o0[oc - ldo], (T)o0[oc + p], (T)o0[oc - 1 + p],
                           (T)wp[wc + ldw], (T)wp[wc - ldw], (T)wm[wc + ldw], (T)wm[wc - ldw], (T)wp[wc + p],
                           (T)wp[wc - 1 + p], (T)wm[wc + p], (T)wm[wc - 1 + p], (T)w0[wc + ldw + p],
                           (T)w0[wc + ldw - 1 + p], (T)w0[wc - ldw + p], (T)w0[wc - ldw - 1 + p], true, tsh);
}

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace

// One full red-black sweep of a level.  xr_old / xb_old: the colours' current
// buffers; xr_new / xb_new: the other buffers.  Partial sums of Lq + tau per
// block: red in slot 0, black in slot 1 (block_partials<2>); block 0 folds
// the previous launch's partials (fold_previous).
template <typename R, bool NL, int TK, int TJ, int PL, bool PF>
__global__ __launch_bounds__(kBlock) void k_sweep2_tile(LevelView<R> L, const R *__restrict__ xr_old,
                                                        const R *__restrict__ xb_old, R *__restrict__ xr_new,
                                                        R *__restrict__ xb_new, const double *__restrict__ csum_in,
                                                        double *__restrict__ csum_out,
                                                        const double *__restrict__ prev, int prev_nblocks,
                                                        int prev_colour, ReduceSlot rs, SolveConsts sc, Span sp,
                                                        unsigned ntiles)
{
    constexpr int NC = NL ? 2 : 1;  // the linear update reads no old value of its own colour
    constexpr int CB = NL ? 1 : 0;  // ring index of the black colour
    constexpr int WJ = TJ + 4, WK = TK + 4, W = WJ * WK;  // old-value window (two-cell halo)
    constexpr int RJ = TJ + 2, RK = TK + 2, RW = RJ * RK;  // new red window (one-cell halo)
    constexpr int LPER = (NC * W + kBlock - 1) / kBlock;    // old-plane elements per thread
    constexpr int RPER = (RW + kBlock - 1) / kBlock;         // red window cells per thread
    constexpr int BPER = TJ * TK / kBlock;                   // black cells per thread
    static_assert(TJ * TK % kBlock == 0, "black cells per thread");
    __shared__ R old[NC][5][WJ][WK];
    __shared__ R rn[3][RJ][RK];
    const int n = L.n, nh = L.nh;
    const unsigned plane = (unsigned)n * nh;
    const int nK = nh / TK, nJ = n / TJ, nI = n / PL;
    (void)nJ;
    const R cmean = (R)((csum_in[0] + csum_in[1]) / (2.0 * (double)L.half));
    const R h2 = (R)(L.h * L.h);
    const R ih2 = (R)(1.0 / (L.h * L.h));
    const R beta = (R)sc.beta;
    const unsigned tid = threadIdx.x;
    double acc[2] = {0.0, 0.0};
    R *oldf = &old[0][0][0][0];
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = ib * PL, j0 = jb * TJ, k0 = kb * TK;
        // this thread's old-window elements q = tid + u kBlock: colour q / W,
        // row (q % W) / WK, column (q % W) % WK (recomputed at each use)
        R pre[LPER];
        auto fetch = [&](int ii) {
            const unsigned base = (unsigned)wrapc(ii, n) * plane;
#pragma unroll
            for (int u = 0; u < LPER; u++) {
                const int q = (int)tid + u * kBlock;
                if (u * kBlock + kBlock <= NC * W || q < NC * W) {
                    const int col = q / W, rr = (q % W) / WK, cc = (q % W) % WK;
                    const unsigned off = base + (unsigned)wrapc(j0 - 2 + rr, n) * nh + wrapc(k0 - 2 + cc, nh);
                    pre[u] = (NL && col == 0) ? xr_old[off] : xb_old[off];
                }
            }
        };
        auto store = [&](int slot) {
#pragma unroll
            for (int u = 0; u < LPER; u++) {
                const int q = (int)tid + u * kBlock;
                if (u * kBlock + kBlock <= NC * W || q < NC * W)
                    oldf[(q / W) * 5 * W + slot * W + q % W] = pre[u];
            }
        };
        auto oslot = [&](int q) { return (q - i0 + 7) % 5; };  // plane q >= i0 - 2
        auto rslot = [&](int q) { return (q - i0 + 4) % 3; };  // plane q >= i0 - 1
        // red window cells: global offset within a plane (wrapped)
        unsigned roff[RPER];
#pragma unroll
        for (int u = 0; u < RPER; u++) {
            const int w = (int)tid + u * kBlock, ww = w < RW ? w : 0;
            roff[u] = (unsigned)wrapc(j0 - 1 + ww / RK, n) * nh + wrapc(k0 - 1 + ww % RK, nh);
        }
        auto load_red_src = [&](int q, R (&d)[RPER], R (&t)[RPER]) {
            const unsigned base = (unsigned)wrapc(q, n) * plane;
#pragma unroll
            for (int u = 0; u < RPER; u++)
                if ((int)tid + u * kBlock < RW) {
                    d[u] = L.dr[base + roff[u]];
                    t[u] = L.tr ? L.tr[base + roff[u]] : (R)0;
                }
        };
        auto load_black_src = [&](int q, R (&d)[BPER], R (&t)[BPER]) {
            const unsigned base = (unsigned)wrapc(q, n) * plane;
#pragma unroll
            for (int u = 0; u < BPER; u++) {
                const int w = (int)tid + u * kBlock;
                const unsigned e = base + (unsigned)(j0 + w / TK) * nh + k0 + w % TK;
                d[u] = L.db[e];
                t[u] = L.tb ? L.tb[e] : (R)0;
            }
        };
        // red cells of plane q (window), new values into rn[rslot(q)]; the
        // tile's own cells of planes i0 .. i0 + PL - 1 also go to xr_new
        auto red_plane = [&](int q, const R (&d)[RPER], const R (&t)[RPER]) {
            const R *bm = &old[CB][oslot(q - 1)][0][0], *b0 = &old[CB][oslot(q)][0][0],
                    *bp = &old[CB][oslot(q + 1)][0][0];
            const R *rm = &old[0][oslot(q - 1)][0][0], *r0 = &old[0][oslot(q)][0][0],
                    *rp = &old[0][oslot(q + 1)][0][0];
            R *dst = &rn[rslot(q)][0][0];
            const bool own_plane = q >= i0 && q < i0 + PL;
            const unsigned base = (unsigned)wrapc(q, n) * plane;
#pragma unroll
            for (int u = 0; u < RPER; u++) {
                const int w = (int)tid + u * kBlock;
                if (w >= RW)
                    continue;
                const int r = w / RK, c = w % RK;
                const int p = (q + j0 - 1 + r) & 1;
                R tsh;
                const R S = planes_stencil<R, R>(bm, b0, bp, WK, r + 1, c + 1, rm, r0, rp, WK, r + 1, c + 1, p, NL,
                                                 tsh);
                int isv;
                const R lq = root_lap<R>(beta * d[u], tsh * ih2 * ih2, sc, NL, isv);
                const R v = lq + t[u];
                const R x = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
                dst[w] = x;
                if (own_plane && r >= 1 && r <= TJ && c >= 1 && c <= TK) {
                    xr_new[base + roff[u]] = x;
                    acc[0] += (double)v;
                }
            }
        };
        // black cells of plane i (tile), faces from the new red ring
        auto black_plane = [&](int i, const R (&d)[BPER], const R (&t)[BPER]) {
            const R *wm = &old[CB][oslot(i - 1)][0][0], *w0 = &old[CB][oslot(i)][0][0],
                    *wp = &old[CB][oslot(i + 1)][0][0];
            const R *om = &rn[rslot(i - 1)][0][0], *o0 = &rn[rslot(i)][0][0], *op = &rn[rslot(i + 1)][0][0];
            const unsigned base = (unsigned)i * plane;
#pragma unroll
            for (int u = 0; u < BPER; u++) {
                const int w = (int)tid + u * kBlock;
                const int r = w / TK, c = w % TK;
                const int p = (i + j0 + r + 1) & 1;
                R tsh;
                const R S = planes_stencil<R, R>(om, o0, op, RK, r + 1, c + 1, wm, w0, wp, WK, r + 2, c + 2, p, NL,
                                                 tsh);
                int isv;
                const R lq = root_lap<R>(beta * d[u], tsh * ih2 * ih2, sc, NL, isv);
                const R v = lq + t[u];
                xb_new[base + (unsigned)(j0 + r) * nh + k0 + c] = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
                acc[1] += (double)v;
            }
        };
        // prologue: old planes i0 - 2 .. i0 + 2, new red planes i0 - 1 and i0
        __syncthreads();  // the previous tile's last reads of the rings are done
        for (int q = i0 - 2; q <= i0 + 2; q++) {
            fetch(q);
            store(oslot(q));
        }
        R rd[RPER], rt[RPER], bd[BPER], bt[BPER];
        load_red_src(i0 - 1, rd, rt);
        __syncthreads();
        red_plane(i0 - 1, rd, rt);
        load_red_src(i0, rd, rt);
        red_plane(i0, rd, rt);
        if (PF) {  // sources one plane ahead
            load_red_src(i0 + 1, rd, rt);
            load_black_src(i0, bd, bt);
        }
        for (int s = 0; s < PL; s++) {
            const int i = i0 + s;
            R rdn[RPER], rtn[RPER], bdn[BPER], btn[BPER];
            const bool more_old = i + 3 <= i0 + PL + 1;
            if (more_old)
                fetch(i + 3);
            if (!PF) {  // this plane's sources, issued with the old plane's loads
                load_red_src(i + 1, rd, rt);
                load_black_src(i, bd, bt);
            } else if (s + 1 < PL) {
                load_red_src(i + 2, rdn, rtn);
                load_black_src(i + 1, bdn, btn);
            }
            red_plane(i + 1, rd, rt);
            __syncthreads();  // new red plane i + 1 complete
            black_plane(i, bd, bt);
            if (more_old)
                store(oslot(i + 3));  // the slot of plane i - 2, last read in the previous step
            __syncthreads();
            if (PF && s + 1 < PL) {
#pragma unroll
                for (int u = 0; u < RPER; u++) {
                    rd[u] = rdn[u];
                    rt[u] = rtn[u];
                }
#pragma unroll
                for (int u = 0; u < BPER; u++) {
                    bd[u] = bdn[u];
                    bt[u] = btn[u];
                }
            }
        }
    }
    block_partials<2>(acc, rs, sp);
    if (blockIdx.x == 0)
        fold_previous(csum_in, csum_out, prev, prev_nblocks, prev_colour);
}

// the sources of the next plane are loaded one plane ahead (measured
// faster than loading them with the plane's old values: 124 against 211 us
// for an FP64 sweep at 256^3)
constexpr bool kSweep2Prefetch = true;

// Tile shape of the fused sweep for a level (false: the level does not take
// it): FP64 16 rows by 32 packed elements, FP32 8 rows by 64 (the shapes
// measured fastest within the LDS and registers of two blocks per CU), PL =
// 32 planes where that still gives 512 tiles, else 16.
template <typename R>
static bool sweep2_shape(int n, int &TK, int &PL, unsigned &ntiles)
{
    const int nh = n / 2, TJ = sizeof(R) == 8 ? 16 : 8;
    TK = sizeof(R) == 8 ? 32 : 64;
    if (n < 64 || nh % TK || n % TJ || n % 16)
        return false;
    PL = (n % 32 == 0 && (n / 32) * (n / TJ) * (nh / TK) >= 512) ? 32 : 16;
    ntiles = (unsigned)((n / PL) * (n / TJ) * (nh / TK));
    return true;
}

bool sweep2_fits(int n, int word_bytes)
{
    int TK = 0, PL = 0;
    unsigned nt = 0;
    return word_bytes == 8 ? sweep2_shape<double>(n, TK, PL, nt) : sweep2_shape<float>(n, TK, PL, nt);
}

template <typename R>
bool launch_sweep2(const LevelView<R> &L, const R *xr_old, const R *xb_old, R *xr_new, R *xb_new,
                   const double *csum_in, double *csum_out, const double *prev, int prev_nblocks, int prev_colour,
                   ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out)
{
    int TK = 0, PL = 0;
    unsigned ntiles = 0;
    if (sc.jacobi || !sweep2_shape<R>(L.n, TK, PL, ntiles))
        return false;
    Span sp;
    unsigned nb = ntiles < (unsigned)kMaxBlocks ? ntiles : (unsigned)kMaxBlocks;
    if (nb >= 8)
        nb -= nb % 8;
    sp.nblocks = nb;
    sp.chunk = kBlock;
    sp.total = nb * kBlock;
    *nblocks_out = (int)nb;
    constexpr int TKV = sizeof(R) == 8 ? 32 : 64, TJV = sizeof(R) == 8 ? 16 : 8;
#define PM_SWEEP2(NLV, PLV)                                                                                            \
    hipLaunchKernelGGL((k_sweep2_tile<R, NLV, TKV, TJV, PLV, kSweep2Prefetch>), dim3(nb), dim3(kBlock), 0, st, L,     \
                       xr_old, xb_old, xr_new, xb_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, \
                       ntiles)
    if (nonlinear) {
        if (PL == 32)
            PM_SWEEP2(true, 32);
        else
            PM_SWEEP2(true, 16);
    } else {
        if (PL == 32)
            PM_SWEEP2(false, 32);
        else
            PM_SWEEP2(false, 16);
    }
#undef PM_SWEEP2
    return true;
}

template bool launch_sweep2<double>(const LevelView<double> &, const double *, const double *, double *, double *,
                                    const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                    hipStream_t, int *);
template bool launch_sweep2<float>(const LevelView<float> &, const float *, const float *, float *, float *,
                                   const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                   hipStream_t, int *);

}  // namespace pmeft
