// LDS plane ring of the 2.5D-tiled multigrid kernels (gfx950): a block owns a
// tile of TJ rows (j) by TK packed elements (kh) and marches along i.  The
// ring holds planes i - 1, i and i + 1 of both colour arrays of a packed
// level, with a one-row / one-element periodic halo on each side, in four
// slots: the loads of plane i + 2 are issued into registers before plane i is
// computed and stored into the free slot after it, so one barrier per plane
// suffices (the free slot held plane i - 2, last read before the previous
// barrier).
#pragma once

#include "mg_stencil.h"

namespace pmeft {

template <typename R, int TK, int TJ>
using RingSlots = R[2][4][TJ + 2][TK + 2];

// NCOL = 1 loads colour 1 (a1) only: the linear smoother reads no neighbour
// of its own colour.
template <typename R, int TK, int TJ, int NCOL = 2>
struct PlaneRing {
    static constexpr int W = (TJ + 2) * (TK + 2);  // window elements per plane and colour
    static constexpr int PER = (NCOL * W + kBlock - 1) / kBlock;
    static constexpr int FULL = NCOL * W / kBlock;  // elements u < FULL exist for every thread
    const R *src[PER];  // this thread's window elements: source array,
    unsigned poff[PER]; // offset within a plane (periodic wrap applied),
    int loff[PER];      // and LDS offset within slot 0
    R pre[PER];
    unsigned plane;
    int n;

    // Element q of a plane's window: colour q / W, row (q % W) / (TK + 2),
    // column (q % W) % (TK + 2); colour 0 comes from a0, colour 1 from a1.
    __device__ __forceinline__ void setup(const R *a0, const R *a1, int n_, int nh, int j0, int k0)
    {
        n = n_;
        plane = (unsigned)n_ * nh;
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int q = threadIdx.x + u * kBlock;
            const int qq = q < NCOL * W ? q : 0;
            const int which = NCOL == 2 ? qq / W : 1, r = (qq % W) / (TK + 2), c = (qq % W) % (TK + 2);
            int jj = j0 - 1 + r, kk = k0 - 1 + c;
            jj = jj < 0 ? jj + n_ : (jj >= n_ ? jj - n_ : jj);
            kk = kk < 0 ? kk + nh : (kk >= nh ? kk - nh : kk);
            src[u] = which ? a1 : a0;
            poff[u] = (unsigned)jj * nh + kk;
            loff[u] = (which * 4 * (TJ + 2) + r) * (TK + 2) + c;
        }
    }
    // plane ii (periodic) into registers
    __device__ __forceinline__ void fetch(int ii)
    {
        ii = ii < 0 ? ii + n : (ii >= n ? ii - n : ii);
        const unsigned base = (unsigned)ii * plane;
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (u < FULL || threadIdx.x + u * kBlock < NCOL * W)
                pre[u] = src[u][base + poff[u]];
    }
    // the fetched plane into ring slot `slot`
    __device__ __forceinline__ void store(RingSlots<R, TK, TJ> &win, int slot)
    {
        R *w = &win[0][0][0][0];
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (u < FULL || threadIdx.x + u * kBlock < NCOL * W)
                w[loff[u] + slot * (TJ + 2) * (TK + 2)] = pre[u];
    }
    // planes i0 - 1, i0, i0 + 1 into slots 0, 1, 2 (the caller then syncs)
    __device__ __forceinline__ void prime(RingSlots<R, TK, TJ> &win, int i0)
    {
        fetch(i0 - 1);
        store(win, 0);
        fetch(i0);
        store(win, 1);
        fetch(i0 + 1);
        store(win, 2);
    }
};

// Operator pieces (S, and Tsh when nonlinear; see stencil_eval) of the cell at
// window row a, column tk + 1 of the plane in slot s0, whose own colour sits
// in win[ow]; sm and sp1 are the slots of planes i - 1 and i + 1 and
// p = (i + j + colour) & 1.  Values stored as R are computed as T.
template <typename T, typename R, int TK, int TJ>
__device__ __forceinline__ T ring_stencil(const RingSlots<R, TK, TJ> &win, int ow, int sm, int s0, int sp1, int a,
                                          int tk, int p, bool nonlinear, T &tsh)
{
    const int b = tk + 1, bm = tk + p, bp = tk + 1 + p;
    const int ot = 1 - ow;
    if (!nonlinear)
        return stencil_eval<T>((T)win[ot][sp1][a][b], (T)win[ot][sm][a][b], (T)win[ot][s0][a + 1][b],
                               (T)win[ot][s0][a - 1][b], (T)win[ot][s0][a][bp], (T)win[ot][s0][a][bm], (T)0, (T)0,
                               (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, false, tsh);
    return stencil_eval<T>((T)win[ot][sp1][a][b], (T)win[ot][sm][a][b], (T)win[ot][s0][a + 1][b],
                           (T)win[ot][s0][a - 1][b], (T)win[ot][s0][a][bp], (T)win[ot][s0][a][bm],
                           (T)win[ow][sp1][a + 1][b], (T)win[ow][sp1][a - 1][b], (T)win[ow][sm][a + 1][b],
                           (T)win[ow][sm][a - 1][b], (T)win[ow][sp1][a][bp], (T)win[ow][sp1][a][bm],
                           (T)win[ow][sm][a][bp], (T)win[ow][sm][a][bm], (T)win[ow][s0][a + 1][bp],
                           (T)win[ow][s0][a + 1][bm], (T)win[ow][s0][a - 1][bp], (T)win[ow][s0][a - 1][bm], true, tsh);
}

// Tile walk order: tile t -> (ib, kb, jb) with ib fastest, so that a block's
// consecutive tiles (and the blocks of one XCD, which take consecutive
// logical indices) share halo planes in the L2.
__device__ __forceinline__ void tile_coords(unsigned tile, int nI, int nK, int &ib, int &kb, int &jb)
{
    ib = (int)(tile % nI);
    kb = (int)((tile / nI) % nK);
    jb = (int)(tile / ((unsigned)nI * nK));
}

}  // namespace pmeft
