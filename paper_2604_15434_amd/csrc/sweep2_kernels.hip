// Both colours of a red-black Gauss-Seidel sweep in one launch (gfx950), for
// the large levels.  A block owns a tile of TJ rows (j) by TK packed elements
// (kh) and marches along i over a chunk of planes.  The two colours run one
// plane apart in a software pipeline: the step at plane i updates the red
// cells of plane i + 2 on the tile plus a one-cell halo in j and kh, and the
// black cells of plane i on the tile, whose face neighbours are the new red
// values of planes i - 1 .. i + 1, finished in earlier steps.  The two halves
// of a step are independent, so one barrier per plane suffices, and the old
// values of plane i + 5 are loaded during the step that stores plane i + 4:
// a whole step hides each load.  The sweep reads each colour's old values
// once and writes each new value once (3 words per cell with the source, 4
// with the FAS source tau), where two half-sweep launches read the red values
// twice.  The red cells of the halo, and of the planes just outside the
// chunk, are updated by neighbouring tiles as well; only the tile's own cells
// are written.
//
// LDS rings (two-cell halo for the old values, one-cell for the new red):
//   red colour, old:   planes i + 1 .. i + 3 read, i + 4 stored  (4 slots)
//   black colour, old: planes i - 1 .. i + 3 read, i + 4 stored  (6 slots;
//                      the linear update reads i + 1 .. i + 3: 4 slots)
//   red colour, new:   planes i - 1 .. i + 1 read, i + 2 written (4 slots)
// Each cell's update is that of the half-sweep kernels on the same operands;
// the black half uses the lagged mean the red half uses (one launch), so a
// fused sweep differs from two half-sweeps by the mean's lag only.
#include "tile_window.h"

#include <math.h>

#include <atomic>
#include <type_traits>

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

template <int TK, int TJ, bool NL>
struct Sweep2Dims {
    static constexpr int WJ = TJ + 4, WK = TK + 4, W = WJ * WK;  // old window
    static constexpr int RJ = TJ + 2, RK = TK + 2, RW = RJ * RK;  // new red window
    static constexpr int NR = NL ? 4 : 0, NB = NL ? 6 : 4;       // old ring slots per colour
};

}  // namespace

// One full red-black sweep of a level.  xr_old / xb_old: the colours' current
// buffers; xr_new / xb_new: the other buffers.  Tile t covers columns (jb, kb)
// and the chunk ib of nI chunks along i (planes ib n / nI .. (ib + 1) n / nI
// - 1).  Partial sums of Lq + tau per block: red in slot 0, black in slot 1
// (block_partials<2>); block 0 folds the previous launch's partials
// (fold_previous).
template <typename R, bool NL, int TK, int TJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_sweep2_tile(LevelView<R> L, const R *__restrict__ xr_old,
                                                        const R *__restrict__ xb_old, R *__restrict__ xr_new,
                                                        R *__restrict__ xb_new, const double *__restrict__ csum_in,
                                                        double *__restrict__ csum_out,
                                                        const double *__restrict__ prev, int prev_nblocks,
                                                        int prev_colour, ReduceSlot rs, SolveConsts sc, Span sp,
                                                        unsigned ntiles, int nI, Group grp)
{
    const long long go = group_offset(grp);
    gshift_view(L, go);
    xr_old = gshift(xr_old, go);
    xb_old = gshift(xb_old, go);
    xr_new = gshift(xr_new, go);
    xb_new = gshift(xb_new, go);
    csum_in = gshift(csum_in, go);
    csum_out = gshift(csum_out, go);
    prev = gshift(prev, go);
    gshift_slot(rs, go);
    gconsts(sc, grp);
    using D = Sweep2Dims<TK, TJ, NL>;
    constexpr int W = D::W, WK = D::WK, RW = D::RW, RK = D::RK, NR = D::NR, NB = D::NB;
    constexpr int NC = NL ? 2 : 1;  // colours loaded (the linear update reads no old value of its own colour)
    constexpr int LPER = (NC * W + kBlock - 1) / kBlock;  // old-plane elements per thread
    constexpr int RPER = (RW + kBlock - 1) / kBlock;      // red window cells per thread
    constexpr int BPER = TJ * TK / kBlock;                // black cells per thread
    static_assert(TJ * TK % kBlock == 0, "black cells per thread");
    __shared__ R ring[(NR + NB) * W];  // red colour slots, then black colour slots
    __shared__ R rn[4 * RW];
    const int n = L.n, nh = L.nh;
    const unsigned plane = (unsigned)n * nh;
    const int nK = nh / TK;
    const R cmean = (R)((csum_in[0] + csum_in[1]) / (2.0 * (double)L.half));
    const R h2 = (R)(L.h * L.h);
    const R ih2 = (R)(1.0 / (L.h * L.h));
    const R beta = (R)sc.beta;
    const int tid = (int)threadIdx.x;
    double acc[2] = {0.0, 0.0};
    for (unsigned tile = span_block(sp); tile < ntiles; tile += sp.nblocks) {
        int ib, kb, jb;
        tile_coords(tile, nI, nK, ib, kb, jb);
        const int i0 = (int)((long long)ib * n / nI), len = (int)((long long)(ib + 1) * n / nI) - i0;
        const int j0 = jb * TJ, k0 = kb * TK;
        const int last_old = i0 + len + 1;  // the last old plane any step reads
        auto red_slot = [&](int q) { return &ring[((q - i0 + 8) & 3) * W]; };
        auto black_slot = [&](int q) { return &ring[(NR + (q - i0 + 12) % NB) * W]; };
        auto new_slot = [&](int q) { return &rn[((q - i0 + 8) & 3) * RW]; };
        // this thread's old-window elements q = tid + u kBlock: red colour
        // for q < W when NL, black otherwise, at element q mod W of the
        // window; poff holds its offset within a plane
        auto is_red = [&](int u) { return NL && tid + u * kBlock < W; };
        unsigned poff[LPER];
#pragma unroll
        for (int u = 0; u < LPER; u++) {
            const int q = tid + u * kBlock, qq = q < NC * W ? q : 0;
            const int e = qq % W, rr = e / WK, cc = e % WK;
            poff[u] = (unsigned)wrapc(j0 - 2 + rr, n) * nh + wrapc(k0 - 2 + cc, nh);
        }
        R pre[LPER];
        auto fetch = [&](int ii) {
            const unsigned base = (unsigned)wrapc(ii, n) * plane;
#pragma unroll
            for (int u = 0; u < LPER; u++)
                if ((u + 1) * kBlock <= NC * W || tid + u * kBlock < NC * W)
                    pre[u] = (is_red(u) ? xr_old : xb_old)[base + poff[u]];
        };
        auto store = [&](int ii) {
            R *rs_ = red_slot(ii), *bs_ = black_slot(ii);
#pragma unroll
            for (int u = 0; u < LPER; u++)
                if ((u + 1) * kBlock <= NC * W || tid + u * kBlock < NC * W) {
                    const int q = tid + u * kBlock;
                    if (is_red(u))
                        rs_[q] = pre[u];
                    else
                        bs_[NL ? q - W : q] = pre[u];
                }
        };
        // red window cells: offset within a plane (wrapped)
        unsigned roff[RPER];
#pragma unroll
        for (int u = 0; u < RPER; u++) {
            const int w = tid + u * kBlock, ww = w < RW ? w : 0;
            roff[u] = (unsigned)wrapc(j0 - 1 + ww / RK, n) * nh + wrapc(k0 - 1 + ww % RK, nh);
        }
        auto load_red_src = [&](int q, R (&d)[RPER], R (&t)[RPER]) {
            const unsigned base = (unsigned)wrapc(q, n) * plane;
#pragma unroll
            for (int u = 0; u < RPER; u++) {
                d[u] = (R)0;
                t[u] = (R)0;
                if (tid + u * kBlock < RW) {
                    d[u] = L.dr[base + roff[u]];
                    t[u] = L.tr ? L.tr[base + roff[u]] : (R)0;
                }
            }
        };
        auto load_black_src = [&](int q, R (&d)[BPER], R (&t)[BPER]) {
            const unsigned base = (unsigned)q * plane;
#pragma unroll
            for (int u = 0; u < BPER; u++) {
                const int w = tid + u * kBlock;
                const unsigned e = base + (unsigned)(j0 + w / TK) * nh + k0 + w % TK;
                d[u] = L.db[e];
                t[u] = L.tb ? L.tb[e] : (R)0;
            }
        };
        // red cells of plane q (window) into the new-red ring; the tile's own
        // cells of the chunk's planes also go to xr_new
        auto red_compute = [&](int q, const R (&d)[RPER], const R (&t)[RPER], R (&xv)[RPER], R (&vv)[RPER]) {
            const R *bm = black_slot(q - 1), *b0 = black_slot(q), *bp = black_slot(q + 1);
            const R *rm = NL ? red_slot(q - 1) : bm, *r0 = NL ? red_slot(q) : b0, *rp = NL ? red_slot(q + 1) : bp;
#pragma unroll
            for (int u = 0; u < RPER; u++) {
                // threads past the window compute its last cell and drop it
                const int w0 = tid + u * kBlock, w = w0 < RW ? w0 : RW - 1;
                const int r = w / RK, c = w % RK;
                const int p = (q + j0 - 1 + r) & 1;
                R tsh;
                const R S = planes_stencil<R, R>(bm, b0, bp, WK, r + 1, c + 1, rm, r0, rp, WK, r + 1, c + 1, p, NL,
                                                 tsh);
                const R lq = root_lap_select<R>(beta * d[u], tsh * ih2 * ih2, sc, NL);
                vv[u] = lq + t[u];
                xv[u] = (S - h2 * (vv[u] - cmean)) * (R)(1.0 / 6.0);
            }
        };
        auto red_store = [&](int q, const R (&xv)[RPER], const R (&vv)[RPER]) {
            R *dst = new_slot(q);
            const bool own_plane = q >= i0 && q < i0 + len;
            const unsigned base = (unsigned)wrapc(q, n) * plane;
#pragma unroll
            for (int u = 0; u < RPER; u++) {
                const int w = tid + u * kBlock, r = w / RK, c = w % RK;
                if (w < RW) {
                    dst[w] = xv[u];
                    if (own_plane && r >= 1 && r <= TJ && c >= 1 && c <= TK) {
                        xr_new[base + roff[u]] = xv[u];
                        acc[0] += (double)vv[u];
                    }
                }
            }
        };
        // black cells of plane i (tile), faces from the new red ring
        auto black_compute = [&](int i, const R (&d)[BPER], const R (&t)[BPER], R (&xv)[BPER], R (&vv)[BPER]) {
            const R *wm = black_slot(i - 1), *w0 = black_slot(i), *wp = black_slot(i + 1);
            const R *om = new_slot(i - 1), *o0 = new_slot(i), *op = new_slot(i + 1);
#pragma unroll
            for (int u = 0; u < BPER; u++) {
                const int w = tid + u * kBlock;
                const int r = w / TK, c = w % TK;
                const int p = (i + j0 + r + 1) & 1;
                R tsh;
                const R S = planes_stencil<R, R>(om, o0, op, RK, r + 1, c + 1, wm, w0, wp, WK, r + 2, c + 2, p, NL,
                                                 tsh);
                const R lq = root_lap_select<R>(beta * d[u], tsh * ih2 * ih2, sc, NL);
                vv[u] = lq + t[u];
                xv[u] = (S - h2 * (vv[u] - cmean)) * (R)(1.0 / 6.0);
            }
        };
        auto black_store = [&](int i, const R (&xv)[BPER], const R (&vv)[BPER]) {
            const unsigned base = (unsigned)i * plane;
#pragma unroll
            for (int u = 0; u < BPER; u++) {
                const int w = tid + u * kBlock;
                xb_new[base + (unsigned)(j0 + w / TK) * nh + k0 + w % TK] = xv[u];
                acc[1] += (double)vv[u];
            }
        };
        // prologue: old planes i0 - 2 .. i0 into the rings, plane i0 + 1 into
        // registers, the red sources of plane i0 - 1
        __syncthreads();  // the previous tile's last reads of the rings are done
        for (int q = i0 - 2; q <= i0; q++) {
            fetch(q);
            store(q);
        }
        fetch(i0 + 1);
        R rd[RPER], rt[RPER], bd[BPER], bt[BPER];
        load_red_src(i0 - 1, rd, rt);
        __syncthreads();
        // step s at plane i = i0 + s: store plane i + 4, load plane i + 5,
        // red of plane i + 2 (DR: s <= len - 2), black of plane i (DB: s >=
        // 0); the flags are constants, so that within a step the compiler
        // interleaves the cells of both halves
        auto step = [&](int s, auto DR, auto DB) {
            constexpr bool do_red = decltype(DR)::value, do_black = decltype(DB)::value;
            const int i = i0 + s;
            if (i + 4 <= last_old)
                store(i + 4);
            if (i + 5 <= last_old)
                fetch(i + 5);
            R rdn[RPER], rtn[RPER], bdn[BPER], btn[BPER];
            const bool red_next = s + 1 <= len - 2, black_next = s + 1 >= 0 && s + 1 < len;
            if (red_next)
                load_red_src(i + 3, rdn, rtn);
            if (black_next)
                load_black_src(i + 1, bdn, btn);
            // both halves computed before either is stored
            R rx[RPER], rv[RPER], bx[BPER], bv[BPER];
            if constexpr (do_red)
                red_compute(i + 2, rd, rt, rx, rv);
            if constexpr (do_black)
                black_compute(i, bd, bt, bx, bv);
            if constexpr (do_red)
                red_store(i + 2, rx, rv);
            if constexpr (do_black)
                black_store(i, bx, bv);
            __syncthreads();
            if (red_next) {
#pragma unroll
                for (int u = 0; u < RPER; u++) {
                    rd[u] = rdn[u];
                    rt[u] = rtn[u];
                }
            }
            if (black_next) {
#pragma unroll
                for (int u = 0; u < BPER; u++) {
                    bd[u] = bdn[u];
                    bt[u] = btn[u];
                }
            }
        };
        using yes = std::true_type;
        using no = std::false_type;
        for (int s = -3; s < 0; s++)
            step(s, yes{}, no{});
        for (int s = 0; s <= len - 2; s++)
            step(s, yes{}, yes{});
        step(len - 1, no{}, yes{});
    }
    block_partials<2>(acc, rs, sp);
    if (blockIdx.x == 0)
        fold_previous(csum_in, csum_out, prev, prev_nblocks, prev_colour);
}

// Tile shape of the fused sweep per word size: FP64 8 rows by 32 packed
// elements, FP32 8 by 64 (three blocks per CU within the LDS).
template <typename R>
struct Sweep2Shape {
    static constexpr int TJ = 8, TK = sizeof(R) == 8 ? 32 : 64;
};

namespace {

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (!cus[dev]) {
        int c = 0;
        cus[dev] = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0 ? c
                                                                                                                : 256;
    }
    return cus[dev];
}

// Resident blocks per CU of the fused kernel (the occupancy the runtime
// reports for its registers and LDS), queried once.
template <typename R, bool NL>
int sweep2_blocks_per_cu()
{
    static std::atomic<int> cached{0};
    int v = cached.load(std::memory_order_relaxed);
    if (!v) {
        using S = Sweep2Shape<R>;
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sweep2_tile<R, NL, S::TK, S::TJ>, kBlock, 0) !=
                hipSuccess ||
            b < 1)
            b = 1;
        v = b > 8 ? 8 : b;
        cached.store(v, std::memory_order_relaxed);
    }
    return v;
}

// Chunks along i and tiles of a level (false: the level does not take the
// fused sweep).  Resident slots: the kernel's blocks per CU on every CU.  The
// chunk count nI (chunks of at least 8 planes) minimises rounds x (chunk
// length + 5), the rounds of resident blocks the tiles take times a tile's
// steps with its prologue, so that the tiles fill whole rounds of slots.
// Levels with fewer than 256 tiles at the shortest chunks are left to the
// half-sweeps.
template <typename R>
bool sweep2_plan(int n, bool nl, int &nI, unsigned &ntiles)
{
    using S = Sweep2Shape<R>;
    const int nh = n / 2;
    if (n < 64 || nh % S::TK || n % S::TJ)
        return false;
    const long long columns = (long long)(n / S::TJ) * (nh / S::TK);
    if (columns * (n / 8) < 256)
        return false;
    const long long slots =
        (long long)(nl ? sweep2_blocks_per_cu<R, true>() : sweep2_blocks_per_cu<R, false>()) * device_cus();
    double best = 0.0;
    nI = 1;
    for (int c = 1; c <= n / 8; c++) {
        const long long rounds = (columns * c + slots - 1) / slots;
        const double cost = (double)rounds * ((double)n / c + 5.0);
        if (c == 1 || cost < best - 1e-9) {
            best = cost;
            nI = c;
        }
    }
    ntiles = (unsigned)(columns * nI);
    return ntiles >= 256;
}

}  // namespace

bool sweep2_fits(int n, int word_bytes)
{
    int nI = 0;
    unsigned nt = 0;
    return word_bytes == 8 ? sweep2_plan<double>(n, true, nI, nt) : sweep2_plan<float>(n, true, nI, nt);
}

template <typename R>
bool launch_sweep2(const LevelView<R> &L, const R *xr_old, const R *xb_old, R *xr_new, R *xb_new,
                   const double *csum_in, double *csum_out, const double *prev, int prev_nblocks, int prev_colour,
                   ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out)
{
    int nI = 0;
    unsigned ntiles = 0;
    if (sc.jacobi || !sweep2_plan<R>(L.n, nonlinear, nI, ntiles))
        return false;
    Span sp;
    unsigned nb = ntiles < (unsigned)kMaxBlocks ? ntiles : (unsigned)kMaxBlocks;
    if (nb >= 8)
        nb -= nb % 8;
    sp.nblocks = nb;
    sp.chunk = kBlock;
    sp.total = nb * kBlock;
    *nblocks_out = (int)nb;
    using S = Sweep2Shape<R>;
    if (nonlinear)
        hipLaunchKernelGGL((k_sweep2_tile<R, true, S::TK, S::TJ>), group_grid(nb), dim3(kBlock), 0, st, L, xr_old,
                           xb_old, xr_new, xb_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, ntiles,
                           nI, cur_group());
    else
        hipLaunchKernelGGL((k_sweep2_tile<R, false, S::TK, S::TJ>), group_grid(nb), dim3(kBlock), 0, st, L, xr_old,
                           xb_old, xr_new, xb_new, csum_in, csum_out, prev, prev_nblocks, prev_colour, rs, sc, sp, ntiles,
                           nI, cur_group());
    return true;
}

template bool launch_sweep2<double>(const LevelView<double> &, const double *, const double *, double *, double *,
                                    const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                    hipStream_t, int *);
template bool launch_sweep2<float>(const LevelView<float> &, const float *, const float *, float *, float *,
                                   const double *, double *, const double *, int, int, ReduceSlot, SolveConsts, bool,
                                   hipStream_t, int *);

}  // namespace pmeft
