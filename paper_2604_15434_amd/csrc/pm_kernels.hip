// Particle-mesh kernels: Cloud-in-Cell deposit (Sec. 3.6.2), the 5-point
// gradient of the total potential (Sec. 3.5.2, eq. force) and the CIC
// interpolation of the acceleration with the kick.
//
// CIC convention: a particle at x lies between the centres of cells i0 and
// i0 + 1 with u = x ng - 1/2, i0 = floor(u), f = u - i0; weights (1 - f) and f
// per axis, periodic wrap.  The same kernel is used to deposit and to
// interpolate, so a lone particle feels no force from itself.
#include "pmeft_internal.h"

#include <math.h>

#include <algorithm>

namespace pmeft {

__device__ __forceinline__ int wrapn(int i, int n)
{
    if (i >= 0 && i < n)
        return i;
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Base cell and fraction along one axis.  Non-finite or absurd coordinates
// (beyond +-2^30 cells) return false: the particle is skipped rather than
// indexing out of range.
__device__ __forceinline__ bool cic_axis(double x, int ng, int &i0, int &i1, double &f)
{
    const double u = x * (double)ng - 0.5;
    if (!(u > -1073741824.0 && u < 1073741824.0))
        return false;
    const double fl = floor(u);
    f = u - fl;
    const int ii = (int)fl;
    i0 = wrapn(ii, ng);
    i1 = wrapn(ii + 1, ng);
    return true;
}

// ------------------------------------------------------------------ deposit
// Each corner weight w in [0, 1] is added as round(w * 2^40) to a 64-bit
// integer, which makes the sum independent of particle order (bitwise
// reproducible) and loses at most 2^-41 per weight.
//
// A chunk is kDepChunk consecutive particles.  Particles of a PM code are
// stored in (roughly) spatial order, so a chunk's CIC footprint is a small
// box: the block accumulates it in LDS with 64-bit LDS atomics and then adds
// each touched cell to the grid with one global atomic, instead of 8
// contended global atomics per particle.  A chunk whose box does not fit the
// LDS tile (scattered order, or a chunk that straddles the periodic boundary)
// falls back to direct global atomics.  Each block walks chunks lb, lb + nb,
// ... (consecutive chunks on one XCD share boundary cells in its L2); a
// thread keeps the cells and fractions of its kDepPer particles between the
// box reduction (wave shuffles, then one LDS slot per wave) and the deposit,
// and the positions of the block's next chunk are already loading.
constexpr int kDepChunk = 1024;
constexpr int kDepPer = kDepChunk / kBlock;
constexpr int kDepTile = 8192;  // 64 KB of 64-bit counters

template <typename Tp>
__global__ __launch_bounds__(kBlock) void k_deposit_tiled(const Tp *__restrict__ pos, unsigned np, int ng,
                                                          unsigned long long *__restrict__ acc, unsigned nchunks,
                                                          const unsigned *__restrict__ sorted_flag)
{
    if (sorted_flag && sorted_flag[0] == 0u)  // the input is row-sorted: the gather deposits it
        return;
    __shared__ unsigned long long tile[kDepTile];
    __shared__ int wbox[kBlock / 64][6];  // per wave: min x, y, z, max x, y, z of the base cells
    const unsigned nb = gridDim.x;
    const unsigned lb = (nb % 8) ? blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Tp cur[3][kDepPer], nxt[3][kDepPer];
    auto load = [&](unsigned chunk, Tp(&dst)[3][kDepPer]) {
#pragma unroll
        for (int u = 0; u < kDepPer; u++) {
            const unsigned p = chunk * kDepChunk + threadIdx.x + u * kBlock;
#pragma unroll
            for (int d = 0; d < 3; d++)
                dst[d][u] = p < np ? pos[(size_t)d * np + p] : (Tp)0;
        }
    };
    if (lb < nchunks)
        load(lb, cur);
    for (unsigned chunk = lb; chunk < nchunks; chunk += nb) {
        if (chunk + nb < nchunks)
            load(chunk + nb, nxt);
        // base cells and fractions of this thread's particles
        int c0[3][kDepPer], c1[3][kDepPer];
        double fr[3][kDepPer];
        bool ok[kDepPer];
        int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-1, -1, -1};
#pragma unroll
        for (int u = 0; u < kDepPer; u++) {
            const unsigned p = chunk * kDepChunk + threadIdx.x + u * kBlock;
            ok[u] = p < np;
#pragma unroll
            for (int d = 0; d < 3; d++)
                ok[u] = ok[u] && cic_axis((double)cur[d][u], ng, c0[d][u], c1[d][u], fr[d][u]);
            if (ok[u])
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    mn[d] = min(mn[d], c0[d][u]);
                    mx[d] = max(mx[d], c0[d][u]);
                }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int d = 0; d < 3; d++) {
                mn[d] = min(mn[d], __shfl_xor(mn[d], off, 64));
                mx[d] = max(mx[d], __shfl_xor(mx[d], off, 64));
            }
        if (lane == 0)
#pragma unroll
            for (int d = 0; d < 3; d++) {
                wbox[wave][d] = mn[d];
                wbox[wave][3 + d] = mx[d];
            }
        __syncthreads();  // also: the previous chunk's flush has read the tile
        int bmin[3], bmax[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            bmin[d] = wbox[0][d];
            bmax[d] = wbox[0][3 + d];
#pragma unroll
            for (int w = 1; w < kBlock / 64; w++) {
                bmin[d] = min(bmin[d], wbox[w][d]);
                bmax[d] = max(bmax[d], wbox[w][3 + d]);
            }
        }
        // box of base cells [bmin, bmax] plus one for the upper corners
        const int ex = bmax[0] - bmin[0] + 2, ey = bmax[1] - bmin[1] + 2, ez = bmax[2] - bmin[2] + 2;
        const bool use_tile = bmax[0] >= 0 && (long long)ex * ey * ez <= kDepTile;
        const int vol = use_tile ? ex * ey * ez : 0;
        for (int t = threadIdx.x; t < vol; t += kBlock)
            tile[t] = 0ull;
        __syncthreads();  // wbox read and the tile cleared
#pragma unroll
        for (int u = 0; u < kDepPer; u++) {
            if (!ok[u])
                continue;
            const double wx[2] = {1.0 - fr[0][u], fr[0][u]}, wy[2] = {1.0 - fr[1][u], fr[1][u]},
                         wz[2] = {1.0 - fr[2][u], fr[2][u]};
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int bb = 0; bb < 2; bb++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const double w = wx[a] * wy[bb] * wz[c];
                        const unsigned long long q = (unsigned long long)(w * kFixScale + 0.5);
                        if (!q)
                            continue;
                        if (use_tile) {
                            const int li = ((c0[0][u] - bmin[0] + a) * ey + (c0[1][u] - bmin[1] + bb)) * ez +
                                           (c0[2][u] - bmin[2] + c);
                            atomicAdd(&tile[li], q);
                        } else {
                            const int gi = a ? c1[0][u] : c0[0][u], gj = bb ? c1[1][u] : c0[1][u],
                                      gk = c ? c1[2][u] : c0[2][u];
                            atomicAdd(&acc[((unsigned)gi * ng + gj) * ng + gk], q);
                        }
                    }
        }
        __syncthreads();
        // cell t -> (ii, jj, kk) by float reciprocals: exact for t < 2^13 (the
        // quotient's error is below 2^-20 of it, its distance to an integer
        // at least 1/(2 ez))
        const float rez = 1.0f / (float)ez, rey = 1.0f / (float)ey;
        for (int t = threadIdx.x; t < vol; t += kBlock) {
            const unsigned long long v = tile[t];
            if (!v)
                continue;
            const int r = __float2int_rz(((float)t + 0.5f) * rez), kk = t - r * ez;
            const int ii = __float2int_rz(((float)r + 0.5f) * rey), jj = r - ii * ey;
            int gi = bmin[0] + ii, gj = bmin[1] + jj, gk = bmin[2] + kk;
            gi = gi >= ng ? gi - ng : gi;
            gj = gj >= ng ? gj - ng : gj;
            gk = gk >= ng ? gk - ng : gk;
            atomicAdd(&acc[((unsigned)gi * ng + gj) * ng + gk], v);
        }
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int u = 0; u < kDepPer; u++)
                cur[d][u] = nxt[d][u];
    }
}

void launch_deposit_fixed(const void *pos, long long np, pm_dtype dt, int ng, unsigned long long *acc, hipStream_t st)
{
    const unsigned nchunks = (unsigned)((np + kDepChunk - 1) / kDepChunk);
    // two 64 KB-tile blocks fit a CU: 512 blocks walk the chunks
    unsigned nb = nchunks < 512u ? nchunks : 512u;
    if (nb >= 8)
        nb -= nb % 8;
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_deposit_tiled<double>), dim3(nb), dim3(kBlock), 0, st, (const double *)pos,
                           (unsigned)np, ng, acc, nchunks, (const unsigned *)nullptr);
    else
        hipLaunchKernelGGL((k_deposit_tiled<float>), dim3(nb), dim3(kBlock), 0, st, (const float *)pos, (unsigned)np,
                           ng, acc, nchunks, (const unsigned *)nullptr);
}

// ------------------------------------------------------- gather deposit
// Particles stored in the order of their CIC base row (i0, j0) (as
// pm_sort_particles leaves them) let each cell collect its own sum: a
// target row (I, J) receives from the particles of the four base rows
// (I - a, J - b), a, b in {0, 1}, which are contiguous ranges of the
// particle arrays.  A block sums a target row's ng cells in LDS (64-bit
// integer atomics, the same 2^-40 rounding of every weight as the scatter,
// so the grid is bitwise the scatter's) and writes each cell once: no global
// atomics and no clearing of the grid.  k_row_index finds the rows' first
// particles and flags input that is not in base-row order (or has an
// unusable x or y coordinate); then the scatter deposits instead.  The choice is made on
// the device, so the deposit still only enqueues.
template <typename Tp>
__device__ __forceinline__ int base_row(const Tp *__restrict__ pos, unsigned np, unsigned p, int ng)
{
    int x0, x1, y0, y1;
    double fx, fy;
    if (!cic_axis((double)pos[p], ng, x0, x1, fx) || !cic_axis((double)pos[np + p], ng, y0, y1, fy))
        return -1;
    return x0 * ng + y0;
}

// flag[0]: 1 if the input is not row-sorted (cleared before the launch);
// rowstart[r] = first particle of base row r, rowstart[ng^2] = np.
template <typename Tp>
__global__ __launch_bounds__(kBlock) void k_row_index(const Tp *__restrict__ pos, unsigned np, int ng,
                                                      unsigned *__restrict__ rowstart, unsigned *__restrict__ flag)
{
    const int nrows = ng * ng;
    for (unsigned p = blockIdx.x * kBlock + threadIdx.x; p < np; p += gridDim.x * kBlock) {
        const int r = base_row(pos, np, p, ng);
        const int prev = p > 0 ? base_row(pos, np, p - 1, ng) : -1;
        if (r < 0 || (p > 0 && prev < 0) || prev > r) {
            flag[0] = 1u;
            continue;
        }
        for (int q = prev + 1; q <= r; q++)
            rowstart[q] = p;
        if (p == np - 1)
            for (int q = r + 1; q <= nrows; q++)
                rowstart[q] = np;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_if_unsorted(unsigned long long *__restrict__ acc, unsigned long long n,
                                                             const unsigned *__restrict__ flag)
{
    if (flag[0] == 0u)
        return;
    for (unsigned long long e = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (unsigned long long)gridDim.x * kBlock)
        acc[e] = 0ull;
}

template <typename Tp>
__global__ __launch_bounds__(kBlock) void k_deposit_gather(const Tp *__restrict__ pos, unsigned np, int ng,
                                                           const unsigned *__restrict__ rowstart,
                                                           const unsigned *__restrict__ flag,
                                                           unsigned long long *__restrict__ acc, unsigned rows_per_block)
{
    if (flag[0] != 0u)
        return;
    __shared__ unsigned long long row[1024];
    const unsigned nb = gridDim.x;
    // XCD-aware: the blocks of one XCD take one contiguous range of rows, so
    // the four source rows of neighbouring target rows stay in its L2
    const unsigned lb = (nb % 8) ? blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const unsigned nrows = (unsigned)ng * ng;
    const unsigned r0 = lb * rows_per_block, r1 = min(nrows, r0 + rows_per_block);
    for (unsigned R = r0; R < r1; R++) {
        const int I = (int)(R / (unsigned)ng), J = (int)(R - (unsigned)I * ng);
        for (int k = threadIdx.x; k < ng; k += kBlock)
            row[k] = 0ull;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int i0 = I - a < 0 ? I - a + ng : I - a, j0 = J - b < 0 ? J - b + ng : J - b;
                const unsigned src = (unsigned)i0 * ng + j0;
                const unsigned s = rowstart[src], e = rowstart[src + 1];
                for (unsigned p = s + threadIdx.x; p < e; p += kBlock) {
                    int x0, x1, y0, y1, z0, z1;
                    double fx, fy, fz;
                    cic_axis((double)pos[p], ng, x0, x1, fx);
                    cic_axis((double)pos[np + p], ng, y0, y1, fy);
                    // (x and y were checked by k_row_index; a particle whose
                    // z is unusable is skipped, as the scatter skips it)
                    if (!cic_axis((double)pos[2 * (size_t)np + p], ng, z0, z1, fz))
                        continue;
                    // the scatter's weight products, in its order
                    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const double w = wx[a] * wy[b] * wz[c];
                        const unsigned long long q = (unsigned long long)(w * kFixScale + 0.5);
                        if (q)
                            atomicAdd(&row[c ? z1 : z0], q);
                    }
                }
            }
        __syncthreads();
        for (int k = threadIdx.x; k < ng; k += kBlock)
            acc[(size_t)R * ng + k] = row[k];
        __syncthreads();
    }
}

size_t deposit_index_bytes(int ng) { return sizeof(unsigned) * ((size_t)ng * ng + 1 + 64); }

// Deposit into acc (ng^3 fixed point): the gather where the particles are in
// base-row order, else the scatter (acc cleared first in that case only).
// idx: deposit_index_bytes(ng) bytes of scratch.
void launch_deposit_auto(const void *pos, long long np, pm_dtype dt, int ng, unsigned long long *acc, void *idx,
                         hipStream_t st)
{
    unsigned *flag = (unsigned *)idx, *rowstart = flag + 64;
    launch_zero(flag, 256, st);
    const unsigned nbi = (unsigned)std::min<long long>((np + kBlock - 1) / kBlock, 4096);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_row_index<double>), dim3(nbi), dim3(kBlock), 0, st, (const double *)pos, (unsigned)np,
                           ng, rowstart, flag);
    else
        hipLaunchKernelGGL((k_row_index<float>), dim3(nbi), dim3(kBlock), 0, st, (const float *)pos, (unsigned)np, ng,
                           rowstart, flag);
    const unsigned long long n3 = (unsigned long long)ng * ng * ng;
    hipLaunchKernelGGL(k_zero_if_unsorted, dim3(2048), dim3(kBlock), 0, st, acc, n3, (const unsigned *)flag);
    const unsigned nchunks = (unsigned)((np + kDepChunk - 1) / kDepChunk);
    unsigned nb = nchunks < 512u ? nchunks : 512u;
    if (nb >= 8)
        nb -= nb % 8;
    const unsigned nrows = (unsigned)ng * ng;
    // 16384 blocks (4 target rows each at 256^3): the gather at 256^3 takes
    // 8 % less time than with 4096 blocks of 16 rows
    unsigned gb = nrows < 16384u ? nrows : 16384u;
    if (gb >= 8)
        gb -= gb % 8;
    const unsigned rpb = (nrows + gb - 1) / gb;
    if (dt == PM_F64) {
        hipLaunchKernelGGL((k_deposit_tiled<double>), dim3(nb), dim3(kBlock), 0, st, (const double *)pos,
                           (unsigned)np, ng, acc, nchunks, (const unsigned *)flag);
        hipLaunchKernelGGL((k_deposit_gather<double>), dim3(gb), dim3(kBlock), 0, st, (const double *)pos,
                           (unsigned)np, ng, (const unsigned *)rowstart, (const unsigned *)flag, acc, rpb);
    } else {
        hipLaunchKernelGGL((k_deposit_tiled<float>), dim3(nb), dim3(kBlock), 0, st, (const float *)pos, (unsigned)np,
                           ng, acc, nchunks, (const unsigned *)flag);
        hipLaunchKernelGGL((k_deposit_gather<float>), dim3(gb), dim3(kBlock), 0, st, (const float *)pos, (unsigned)np,
                           ng, (const unsigned *)rowstart, (const unsigned *)flag, acc, rpb);
    }
}

// fixed point (natural layout) -> packed delta_raw = rho - 1, with its sum.
__global__ __launch_bounds__(kBlock) void k_fixed_to_delta(const unsigned long long *__restrict__ acc, int n,
                                                           double rho_scale, double *__restrict__ delta, ReduceSlot rs,
                                                           Span sp)
{
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    double s[1] = {0.0};
    PM_SPAN_LOOP(e, sp)
    {
        const int c = e >= half;
        const unsigned ec = e - (c ? half : 0u);
        int i, j, kh;
        split(ec, nh, n, i, j, kh);
        const int k = 2 * kh + ((i + j + c) & 1);
        const double rho = (double)acc[((unsigned)i * n + j) * n + k] * (rho_scale / kFixScale);
        const double d = rho - 1.0;
        delta[e] = d;
        s[0] += d;
    }
    block_partials<1>(s, rs, sp);
}

void launch_fixed_to_delta(const unsigned long long *acc, int ng, double rho_scale, double *delta_packed, ReduceSlot rs,
                           hipStream_t st)
{
    const Span sp = make_span((unsigned long long)ng * ng * ng);
    hipLaunchKernelGGL(k_fixed_to_delta, dim3(sp.nblocks), dim3(kBlock), 0, st, acc, ng, rho_scale, delta_packed, rs,
                       sp);
    launch_finalize(rs, sp, 1, rs.out, st);
}

// ----------------------------------------------------------------- gradient
__device__ __forceinline__ double ld_packed(const double *f, int n, int nh, long long half, int i, int j, int k)
{
    const int c = (i + j + k) & 1;
    return f[(c ? (unsigned)half : 0u) + ((unsigned)i * n + j) * nh + (k >> 1)];
}

// g = -D5 Psi_tot, D5 f_i = (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h),
// Psi_tot = Psi_N + xi chi; written as (gx, gy, gz, 0) per cell in natural
// order.
template <typename Tg>
__global__ __launch_bounds__(kBlock) void k_gradient(const double *__restrict__ psi, const double *__restrict__ chi,
                                                     double xi, int n, Tg *__restrict__ g4, Span sp)
{
    const int nh = n / 2;
    const long long half = (long long)n * n * nh;
    const double s = -(double)n / 12.0;  // -1/(12 h)
    PM_SPAN_LOOP(e, sp)
    {
        int i, j, k;
        split((unsigned)e, (unsigned)n, (unsigned)n, i, j, k);
        auto P = [&](int a, int b, int c) -> double {
            a = a < 0 ? a + n : (a >= n ? a - n : a);
            b = b < 0 ? b + n : (b >= n ? b - n : b);
            c = c < 0 ? c + n : (c >= n ? c - n : c);
            double v = ld_packed(psi, n, nh, half, a, b, c);
            if (chi)
                v += xi * ld_packed(chi, n, nh, half, a, b, c);
            return v;
        };
        const double gx = s * (P(i - 2, j, k) - 8.0 * P(i - 1, j, k) + 8.0 * P(i + 1, j, k) - P(i + 2, j, k));
        const double gy = s * (P(i, j - 2, k) - 8.0 * P(i, j - 1, k) + 8.0 * P(i, j + 1, k) - P(i, j + 2, k));
        const double gz = s * (P(i, j, k - 2) - 8.0 * P(i, j, k - 1) + 8.0 * P(i, j, k + 1) - P(i, j, k + 2));
        Tg *o = g4 + 4 * (size_t)e;
        o[0] = (Tg)gx;
        o[1] = (Tg)gy;
        o[2] = (Tg)gz;
        o[3] = (Tg)0;
    }
}

// The same gradient, 2.5D-tiled for n % 64 == 0: a block owns 4 CJ rows (j)
// by 64 cells (k) and walks PL planes along i, keeping Psi_tot of planes
// i - 2 .. i + 2 (with a two-cell halo in j and k, in natural order) in a
// six-slot LDS ring: the next plane is fetched into registers before the
// current one is computed and stored into the free slot after it (one
// barrier per plane).  Thread (tj, tk) computes rows tj, tj + 4, ... of the
// tile.  Same operands and expression as k_gradient.
constexpr int kGradK = 64, kGradPL = 16, kGradCJ = 2;

template <typename Tg, int CJ>
__global__ __launch_bounds__(kBlock) void k_gradient_tile(const double *__restrict__ psi,
                                                          const double *__restrict__ chi, double xi, int n,
                                                          Tg *__restrict__ g4, unsigned ntiles)
{
    constexpr int RS = kBlock / kGradK, ROWS = RS * CJ;
    constexpr int WR = ROWS + 4, WC = kGradK + 4, W = WR * WC;
    constexpr int PER = (W + kBlock - 1) / kBlock;
    __shared__ double win[6][WR][WC];
    const int nh = n / 2;
    const unsigned half = (unsigned)n * n * nh;
    const double s = -(double)n / 12.0;
    const int nI = n / kGradPL, nK = n / kGradK;
    const int tj = threadIdx.x / kGradK, tk = threadIdx.x % kGradK;
    const unsigned nb = gridDim.x;
    const unsigned lb = (nb % 8) ? blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    double *wflat = &win[0][0][0];
    for (unsigned t = lb; t < ntiles; t += nb) {
        const int ib = (int)(t % nI), kb = (int)((t / nI) % nK), jb = (int)(t / ((unsigned)nI * nK));
        const int i0 = ib * kGradPL, j0 = jb * ROWS, k0 = kb * kGradK;
        // window element q: row q / WC (j = j0 - 2 + row), column q % WC
        // (k = k0 - 2 + column); packed offset within a plane and j + k parity
        unsigned poff[PER];
        int par[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int q = threadIdx.x + u * kBlock;
            const int qq = q < W ? q : 0;
            int j = j0 - 2 + qq / WC, k = k0 - 2 + qq % WC;
            j = j < 0 ? j + n : (j >= n ? j - n : j);
            k = k < 0 ? k + n : (k >= n ? k - n : k);
            poff[u] = (unsigned)j * nh + (k >> 1);
            par[u] = (j + k) & 1;
        }
        double pre[PER];
        auto fetch = [&](int ii) {
            ii = ii < 0 ? ii + n : (ii >= n ? ii - n : ii);
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kBlock < W) {
                    const unsigned o = (((ii + par[u]) & 1) ? half : 0u) + (unsigned)ii * n * nh + poff[u];
                    double v = psi[o];
                    if (chi)
                        v += xi * chi[o];
                    pre[u] = v;
                }
        };
        auto store = [&](int slot) {
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kBlock < W)
                    wflat[slot * W + threadIdx.x + u * kBlock] = pre[u];
        };
#pragma unroll 1
        for (int d = 0; d < 5; d++) {
            fetch(i0 - 2 + d);
            store(d);
        }
        __syncthreads();
#pragma unroll 1
        for (int p = 0; p < kGradPL; p++) {
            const int i = i0 + p;
            if (p + 1 < kGradPL)
                fetch(i + 3);
#pragma unroll
            for (int cj = 0; cj < CJ; cj++) {
                const int r = tj + cj * RS + 2, c = tk + 2;
                const double *m2 = &win[p % 6][r][c], *m1 = &win[(p + 1) % 6][r][c], *c0 = &win[(p + 2) % 6][r][c];
                const double *p1 = &win[(p + 3) % 6][r][c], *p2 = &win[(p + 4) % 6][r][c];
                const double gx = s * (m2[0] - 8.0 * m1[0] + 8.0 * p1[0] - p2[0]);
                const double gy = s * (c0[-2 * WC] - 8.0 * c0[-WC] + 8.0 * c0[WC] - c0[2 * WC]);
                const double gz = s * (c0[-2] - 8.0 * c0[-1] + 8.0 * c0[1] - c0[2]);
                typedef Tg Tg4 __attribute__((ext_vector_type(4)));
                Tg4 o;
                o[0] = (Tg)gx;
                o[1] = (Tg)gy;
                o[2] = (Tg)gz;
                o[3] = (Tg)0;
                *(Tg4 *)(g4 + 4 * ((size_t)((unsigned)i * n + j0 + tj + cj * RS) * n + k0 + tk)) = o;
            }
            if (p + 1 < kGradPL)
                store((p + 5) % 6);  // plane i + 3 replaces plane i - 3
            __syncthreads();
        }
    }
}

void launch_gradient(const double *psi, const double *chi, double xi, int ng, void *g4, pm_dtype dt, hipStream_t st)
{
    constexpr int rows = kBlock / kGradK * kGradCJ;
    if (ng % kGradK == 0 && ng % kGradPL == 0 && ng % rows == 0) {
        const unsigned ntiles = (unsigned)(ng / rows) * (ng / kGradK) * (ng / kGradPL);
        unsigned nb = ntiles < 2048u ? ntiles : 2048u;
        if (nb >= 8)
            nb -= nb % 8;
        if (dt == PM_F64)
            hipLaunchKernelGGL((k_gradient_tile<double, kGradCJ>), dim3(nb), dim3(kBlock), 0, st, psi, chi, xi, ng,
                               (double *)g4, ntiles);
        else
            hipLaunchKernelGGL((k_gradient_tile<float, kGradCJ>), dim3(nb), dim3(kBlock), 0, st, psi, chi, xi, ng,
                               (float *)g4, ntiles);
        return;
    }
    const Span sp = make_span((unsigned long long)ng * ng * ng);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_gradient<double>), dim3(sp.nblocks), dim3(kBlock), 0, st, psi, chi, xi, ng,
                           (double *)g4, sp);
    else
        hipLaunchKernelGGL((k_gradient<float>), dim3(sp.nblocks), dim3(kBlock), 0, st, psi, chi, xi, ng, (float *)g4,
                           sp);
}

// ---------------------------------------------------------- interpolation
// CIC interpolation of g at each particle, kick, optional drift.  A thread
// takes UNR particles (kBlock apart) per pass and issues all their position
// and corner loads before the arithmetic on any of them; a particle with a
// non-finite coordinate reads cell 0 and gets zero acceleration.
constexpr int kInterpUnr = 2;

template <typename T, int UNR>
__global__ __launch_bounds__(kBlock) void k_interp_kick(const T *__restrict__ g4, int ng, T *__restrict__ pos,
                                                        unsigned np, T *__restrict__ vel, double dt_kick,
                                                        double dt_drift, T *__restrict__ acc_out, Span sp)
{
    typedef T T4 __attribute__((ext_vector_type(4)));
    const unsigned b0 = span_block(sp) * sp.chunk;
    const unsigned end = min(sp.total, b0 + sp.chunk);
    for (unsigned p0 = b0 + threadIdx.x; p0 < end; p0 += UNR * kBlock) {
        unsigned pp[UNR];
        bool live[UNR], ok[UNR];
        double x[UNR][3], fr[UNR][3];
        int c0[UNR][3], c1[UNR][3];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const unsigned p = p0 + u * kBlock;
            live[u] = p < end;
            pp[u] = live[u] ? p : p0;
#pragma unroll
            for (int d = 0; d < 3; d++)
                x[u][d] = (double)pos[(size_t)d * np + pp[u]];
        }
        T4 g[UNR][8];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            ok[u] = true;
#pragma unroll
            for (int d = 0; d < 3; d++)
                ok[u] = ok[u] && cic_axis(x[u][d], ng, c0[u][d], c1[u][d], fr[u][d]);
            if (!ok[u])
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    c0[u][d] = c1[u][d] = 0;
                    fr[u][d] = 0.0;
                }
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const unsigned cell = ((unsigned)(a ? c1[u][0] : c0[u][0]) * ng + (b ? c1[u][1] : c0[u][1])) * ng +
                                              (c ? c1[u][2] : c0[u][2]);
                        g[u][4 * a + 2 * b + c] = *(const T4 *)(g4 + 4 * (size_t)cell);  // one 16- or 32-byte load
                    }
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            double ax = 0.0, ay = 0.0, az = 0.0;
            const double wx[2] = {1.0 - fr[u][0], fr[u][0]}, wy[2] = {1.0 - fr[u][1], fr[u][1]},
                         wz[2] = {1.0 - fr[u][2], fr[u][2]};
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const double w = wx[a] * wy[b] * wz[c];
                        const T4 gv = g[u][4 * a + 2 * b + c];
                        ax += w * (double)gv[0];
                        ay += w * (double)gv[1];
                        az += w * (double)gv[2];
                    }
            if (!ok[u])
                ax = ay = az = 0.0;
            if (!live[u])
                continue;
            const unsigned p = pp[u];
            const double vx = (double)vel[p] + ax * dt_kick;
            const double vy = (double)vel[np + p] + ay * dt_kick;
            const double vz = (double)vel[2 * np + p] + az * dt_kick;
            vel[p] = (T)vx;
            vel[np + p] = (T)vy;
            vel[2 * np + p] = (T)vz;
            if (acc_out) {
                acc_out[p] = (T)ax;
                acc_out[np + p] = (T)ay;
                acc_out[2 * np + p] = (T)az;
            }
            if (dt_drift != 0.0 && ok[u]) {
                double xn = x[u][0] + vx * dt_drift;
                double yn = x[u][1] + vy * dt_drift;
                double zn = x[u][2] + vz * dt_drift;
                xn -= floor(xn);
                yn -= floor(yn);
                zn -= floor(zn);
                pos[p] = (T)(xn >= 1.0 ? 0.0 : xn);
                pos[np + p] = (T)(yn >= 1.0 ? 0.0 : yn);
                pos[2 * np + p] = (T)(zn >= 1.0 ? 0.0 : zn);
            }
        }
    }
}

void launch_interp_kick(const void *g4, int ng, pm_dtype dt, void *pos, long long np, void *vel, double dt_kick,
                        double dt_drift, void *acc_out, hipStream_t st)
{
    const Span sp = make_span(np);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_interp_kick<double, kInterpUnr>), dim3(sp.nblocks), dim3(kBlock), 0, st,
                           (const double *)g4, ng, (double *)pos, (unsigned)np, (double *)vel, dt_kick, dt_drift,
                           (double *)acc_out, sp);
    else
        hipLaunchKernelGGL((k_interp_kick<float, kInterpUnr>), dim3(sp.nblocks), dim3(kBlock), 0, st,
                           (const float *)g4, ng, (float *)pos, (unsigned)np, (float *)vel, dt_kick, dt_drift,
                           (float *)acc_out, sp);
}

// Bardeen potentials from Psi_N and chi (natural order, same dtype):
// Psi = Psi_N + c_psi chi, Phi = Psi_N + c_phi chi, Psi + Phi; each output
// nullable.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_potentials(const T *__restrict__ psi_n, const T *__restrict__ chi,
                                                       double c_psi, double c_phi, T *__restrict__ psi,
                                                       T *__restrict__ phi, T *__restrict__ lens, Span sp)
{
    PM_SPAN_LOOP(e, sp)
    {
        const double pn = (double)psi_n[e], x = (double)chi[e];
        const double a = pn + c_psi * x, b = pn + c_phi * x;
        if (psi)
            psi[e] = (T)a;
        if (phi)
            phi[e] = (T)b;
        if (lens)
            lens[e] = (T)(a + b);
    }
}

void launch_potentials(const void *psi_n, const void *chi, pm_dtype dt, long long n3, double c_psi, double c_phi,
                       void *psi, void *phi, void *lens, hipStream_t st)
{
    const Span sp = make_span(n3);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_potentials<double>), dim3(sp.nblocks), dim3(kBlock), 0, st, (const double *)psi_n,
                           (const double *)chi, c_psi, c_phi, (double *)psi, (double *)phi, (double *)lens, sp);
    else
        hipLaunchKernelGGL((k_potentials<float>), dim3(sp.nblocks), dim3(kBlock), 0, st, (const float *)psi_n,
                           (const float *)chi, c_psi, c_phi, (float *)psi, (float *)phi, (float *)lens, sp);
}

// ------------------------------------------------------------ particle sort
// Stable LSD radix sort of the particles by the cell of their CIC base
// corner, key = (i0 ng + j0) ng + k0 (particles with unusable coordinates
// take the last cell).  8-bit digits; per pass: per-tile digit histograms,
// one exclusive scan over (digit, tile), and a scatter in which each element's
// rank among equal digits of its tile comes from wave ballots, so the order
// of equal keys is the input order and the result is deterministic.
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;  // elements per tile
constexpr int kScanChunk = 2048;                // entries per scan block

template <typename Tp>
__global__ __launch_bounds__(kBlock) void k_sort_keys(const Tp *__restrict__ pos, unsigned np, int ng,
                                                      unsigned *__restrict__ keys, unsigned *__restrict__ vals)
{
    const unsigned last = (unsigned)ng * ng * ng - 1u;
    for (unsigned p = blockIdx.x * kBlock + threadIdx.x; p < np; p += gridDim.x * kBlock) {
        int x0, x1, y0, y1, z0, z1;
        double fx, fy, fz;
        const bool ok = cic_axis((double)pos[p], ng, x0, x1, fx) && cic_axis((double)pos[np + p], ng, y0, y1, fy) &&
                        cic_axis((double)pos[2 * (size_t)np + p], ng, z0, z1, fz);
        keys[p] = ok ? ((unsigned)x0 * ng + y0) * ng + z0 : last;
        vals[p] = p;
    }
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const unsigned *__restrict__ keys, unsigned n, int shift,
                                                       unsigned ntiles, unsigned *__restrict__ hist)
{
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const unsigned t0 = blockIdx.x * kSortTile;
    for (unsigned e = t0 + threadIdx.x; e < min(n, t0 + kSortTile); e += kBlock)
        atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of x[0..n) in chunks: each block scans its chunk and writes the chunk total
__global__ __launch_bounds__(kBlock) void k_scan_chunks(unsigned *__restrict__ x, unsigned n,
                                                        unsigned *__restrict__ totals)
{
    __shared__ unsigned s[kBlock];
    constexpr int per = kScanChunk / kBlock;
    const unsigned base = blockIdx.x * kScanChunk + threadIdx.x * per;
    unsigned v[per], sum = 0;
    for (int q = 0; q < per; q++) {
        v[q] = base + q < n ? x[base + q] : 0u;
        sum += v[q];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
        const unsigned t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    unsigned run = s[threadIdx.x] - sum;
    for (int q = 0; q < per; q++) {
        if (base + q < n)
            x[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == kBlock - 1)
        totals[blockIdx.x] = s[kBlock - 1];
}

// one block: exclusive scan of the chunk totals (any count), then add to the chunks
__global__ __launch_bounds__(kBlock) void k_scan_totals(unsigned *__restrict__ totals, unsigned nchunks)
{
    __shared__ unsigned s[kBlock];
    __shared__ unsigned carry;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (unsigned b0 = 0; b0 < nchunks; b0 += kBlock) {
        const unsigned i = b0 + threadIdx.x;
        const unsigned v = i < nchunks ? totals[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const unsigned t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunks)
            totals[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0)
            carry += s[kBlock - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(unsigned *__restrict__ x, unsigned n,
                                                     const unsigned *__restrict__ totals)
{
    const unsigned add = totals[blockIdx.x];
    for (unsigned e = blockIdx.x * kScanChunk + threadIdx.x; e < min(n, (blockIdx.x + 1) * kScanChunk); e += kBlock)
        x[e] += add;
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const unsigned *__restrict__ kin,
                                                          const unsigned *__restrict__ vin, unsigned n, int shift,
                                                          unsigned ntiles, const unsigned *__restrict__ offs,
                                                          unsigned *__restrict__ kout, unsigned *__restrict__ vout)
{
    __shared__ unsigned run[256];        // elements of each digit already placed by this tile
    __shared__ unsigned wc[kBlock / 64][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run[threadIdx.x] = 0;
    const unsigned t0 = blockIdx.x * kSortTile;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortItems; r++) {
        for (int w = 0; w < kBlock / 64; w++)
            wc[w][threadIdx.x] = 0;
        __syncthreads();
        const unsigned e = t0 + r * kBlock + threadIdx.x;
        const bool valid = e < n;
        const unsigned key = valid ? kin[e] : 0u;
        const unsigned val = valid ? vin[e] : 0u;
        const unsigned d = (key >> shift) & 255u;
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        // m: valid lanes of this wave with digit d
        const unsigned rank_w = (unsigned)__popcll(m & lt);
        if (valid && rank_w == 0)
            wc[wave][d] = (unsigned)__popcll(m);
        __syncthreads();
        if (valid) {
            unsigned before = run[d] + rank_w;
            for (int w = 0; w < wave; w++)
                before += wc[w][d];
            const unsigned pos = offs[(size_t)d * ntiles + blockIdx.x] + before;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        unsigned add = 0;
        for (int w = 0; w < kBlock / 64; w++)
            add += wc[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute3(const T *__restrict__ src, T *__restrict__ dst,
                                                     const unsigned *__restrict__ perm, unsigned np)
{
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < np; i += gridDim.x * kBlock) {
        const unsigned p = perm[i];
        dst[i] = src[p];
        dst[(size_t)np + i] = src[(size_t)np + p];
        dst[2 * (size_t)np + i] = src[2 * (size_t)np + p];
    }
}

__global__ __launch_bounds__(kBlock) void k_permute_ids(const long long *__restrict__ src, long long *__restrict__ dst,
                                                        const unsigned *__restrict__ perm, unsigned np)
{
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < np; i += gridDim.x * kBlock)
        dst[i] = src[perm[i]];
}

static unsigned sort_tiles(unsigned long long np) { return (unsigned)((np + kSortTile - 1) / kSortTile); }

size_t sort_workspace_bytes(unsigned long long np, int word)
{
    const unsigned nt = sort_tiles(np);
    const size_t nh = (size_t)256 * nt;
    const size_t nchunks = (nh + kScanChunk - 1) / kScanChunk;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 4 * al(sizeof(unsigned) * np) + al(sizeof(unsigned) * nh) + al(sizeof(unsigned) * nchunks) +
           al((size_t)3 * word * np);
}

// Sort; pos, vel (nullable) 3 x np SoA of dtype; ids (nullable) np int64.
int launch_sort_particles(void *pos, void *vel, long long *ids, unsigned np, int ng, pm_dtype dt, char *ws,
                          hipStream_t st)
{
    const unsigned nt = sort_tiles(np);
    const size_t nh = (size_t)256 * nt;
    const unsigned nchunks = (unsigned)((nh + kScanChunk - 1) / kScanChunk);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    unsigned *k0 = (unsigned *)ws;
    unsigned *v0 = (unsigned *)(ws + al(sizeof(unsigned) * np));
    unsigned *k1 = (unsigned *)(ws + 2 * al(sizeof(unsigned) * np));
    unsigned *v1 = (unsigned *)(ws + 3 * al(sizeof(unsigned) * np));
    unsigned *hist = (unsigned *)(ws + 4 * al(sizeof(unsigned) * np));
    unsigned *tot = (unsigned *)((char *)hist + al(sizeof(unsigned) * nh));
    char *scratch = (char *)tot + al(sizeof(unsigned) * nchunks);
    const unsigned nb = std::min(4096u, (np + kBlock - 1) / kBlock);
    if (dt == PM_F64)
        hipLaunchKernelGGL((k_sort_keys<double>), dim3(nb), dim3(kBlock), 0, st, (const double *)pos, np, ng, k0, v0);
    else
        hipLaunchKernelGGL((k_sort_keys<float>), dim3(nb), dim3(kBlock), 0, st, (const float *)pos, np, ng, k0, v0);
    const unsigned long long maxkey = (unsigned long long)ng * ng * ng - 1ull;
    int bits = 0;
    while ((maxkey >> bits) != 0ull)
        bits++;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nt), dim3(kBlock), 0, st, k0, np, shift, nt, hist);
        hipLaunchKernelGGL(k_scan_chunks, dim3(nchunks), dim3(kBlock), 0, st, hist, (unsigned)nh, tot);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, st, tot, nchunks);
        hipLaunchKernelGGL(k_scan_add, dim3(nchunks), dim3(kBlock), 0, st, hist, (unsigned)nh, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nt), dim3(kBlock), 0, st, k0, v0, np, shift, nt, hist, k1, v1);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    // v0: the permutation (sorted position -> original index)
    const size_t word = dt == PM_F64 ? 8 : 4;
    void *arrays[2] = {pos, vel};
    for (int a = 0; a < 2; a++) {
        if (!arrays[a])
            continue;
        if (dt == PM_F64)
            hipLaunchKernelGGL((k_permute3<double>), dim3(nb), dim3(kBlock), 0, st, (const double *)arrays[a],
                               (double *)scratch, v0, np);
        else
            hipLaunchKernelGGL((k_permute3<float>), dim3(nb), dim3(kBlock), 0, st, (const float *)arrays[a],
                               (float *)scratch, v0, np);
        if (hipMemcpyAsync(arrays[a], scratch, 3 * word * np, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PM_EHIP;
    }
    if (ids) {
        // the key buffer k1 (np words) and v1 are free now: 8 * np bytes from k1 on
        long long *tmp = (long long *)k1;
        hipLaunchKernelGGL(k_permute_ids, dim3(nb), dim3(kBlock), 0, st, ids, tmp, v0, np);
        if (hipMemcpyAsync(ids, tmp, sizeof(long long) * np, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PM_EHIP;
    }
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP;
}

}  // namespace pmeft
