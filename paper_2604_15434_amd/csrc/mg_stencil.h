// Device functions of the multigrid stencils shared by the smoothers, the
// transfer kernels and the block cycle: the local root of the scalar-field
// equation, the 19-point operator pieces in the packed red-black layout,
// the cell update of a half-sweep and the fold of per-block partial sums.
#pragma once

#include "pmeft_internal.h"

#include <math.h>

namespace pmeft {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrap_up(int i, int n) { return i >= n ? i - n : i; }
__device__ __forceinline__ int wrap_dn(int i, int n) { return i < 0 ? i + n : i; }

// FP64 square root and reciprocal from the hardware estimates (v_rsq_f64,
// v_rcp_f64) refined by two Newton steps each: relative error near 1 ulp, at
// about half the instructions of the IEEE-rounded sequences.  sqrt_nr returns
// 0 for x <= 1e-280 (there sqrt(x) < 1e-140, far below any value it is added
// to here).
__device__ __forceinline__ double sqrt_nr(double x)
{
    const bool pos = x > 1e-280;
    const double xs = pos ? x : 1.0;
    double y = __builtin_amdgcn_rsq(xs);
    y = fma(0.5 * y, fma(-xs * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-xs * y, y, 1.0), y);
    return pos ? xs * y : 0.0;
}
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Root of the local quadratic without a branch: both cases are evaluated
// with the operations of root_lap below and the void value is selected, so
// that a kernel updating several cells per thread can interleave them.
template <typename T>
__device__ __forceinline__ T root_lap_select(T b, T Tsh, const SolveConsts &sc, bool nonlinear)
{
    const T nu = (T)sc.nu;
    if (!nonlinear)
        return b / nu;
    const T K = (T)sc.K;
    const T dsph = nu * nu - (T)(8.0 / 3.0) * K * b;
    const T G = K * Tsh - b;
    const T disc = dsph + (T)(8.0 / 3.0) * K * K * Tsh;
    T r;
    if constexpr (sizeof(T) == 4)
        r = (T)-2 * G * __builtin_amdgcn_rcpf(nu + __builtin_amdgcn_sqrtf(disc));
    else
        r = (T)-2 * G * rcp_nr(nu + sqrt_nr(disc));
    // r is pinned (an empty asm statement that reads it): otherwise the
    // compiler turns the select back into a branch around r and its operand
    // loads
    asm volatile("" ::"v"(r));
    return dsph < (T)0 ? (T)0.75 * nu / K : r;
}

// Void-cell test and root of the local quadratic, computed in the type T.
template <typename T>
__device__ __forceinline__ T root_lap(T b, T Tsh, const SolveConsts &sc, bool nonlinear, int &is_void)
{
    const T nu = (T)sc.nu;
    if (!nonlinear) {
        is_void = 0;
        return b / nu;
    }
    // Tsh is pinned here (an empty asm statement that reads it): otherwise the
    // compiler sinks the loads of its operands into the non-void branch below,
    // and every cell waits for two rounds of memory latency instead of one
    asm volatile("" ::"v"(Tsh));
    const T K = (T)sc.K;
    const T dsph = nu * nu - (T)(8.0 / 3.0) * K * b;
    if (dsph < (T)0) {
        is_void = 1;
        return (T)0.75 * nu / K;
    }
    is_void = 0;
    const T G = K * Tsh - b;
    const T disc = dsph + (T)(8.0 / 3.0) * K * K * Tsh;
    if constexpr (sizeof(T) == 4)  // FP32 smoothing: hardware sqrt and reciprocal (1 ulp each)
        return (T)-2 * G * __builtin_amdgcn_rcpf(nu + __builtin_amdgcn_sqrtf(disc));
    else
        return (T)-2 * G * rcp_nr(nu + sqrt_nr(disc));
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

// ---------------------------------------------------------------- smoothing
// Block 0 of a half-sweep: csum_out = csum_in with the colour of the previous
// launch at this level (prev_colour; -1 none, 2 both: a fused two-colour
// sweep, whose partials hold red in slot 0 and black in slot 1) replaced by
// the sum of its per-block partials, in block order.
__device__ __forceinline__ void fold_previous(const double *__restrict__ csum_in, double *__restrict__ csum_out,
                                              const double *__restrict__ prev, int prev_nblocks, int prev_colour)
{
    __shared__ double fin[2][kBlock / 64];
    double t[2] = {0.0, 0.0};
    if (prev_colour >= 0)
        for (int q = threadIdx.x; q < prev_nblocks; q += kBlock) {
            t[0] += prev[(size_t)q * 8];
            if (prev_colour == 2)
                t[1] += prev[(size_t)q * 8 + 1];
        }
    for (int c = 0; c < 2; c++) {
        for (int off = 32; off > 0; off >>= 1)
            t[c] += __shfl_down(t[c], off, 64);
        if ((threadIdx.x & 63) == 0)
            fin[c][threadIdx.x >> 6] = t[c];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = csum_in[threadIdx.x];
        const int slot = prev_colour == 2 ? (int)threadIdx.x : 0;
        if ((int)threadIdx.x == prev_colour || prev_colour == 2) {
            v = 0.0;
            for (int w = 0; w < kBlock / 64; w++)
                v += fin[slot][w];
        }
        csum_out[threadIdx.x] = v;
    }
}

// Local update of one cell of colour `colour` (element e = (i, j, kh)):
// x_new = (S - h^2 (Lq + tau - cmean)) / 6 (blended with the old value for
// the Jacobi smoother); returns Lq + tau.
template <typename R, bool NL>
__device__ __forceinline__ R smooth_cell(const R *__restrict__ xc_old, const R *__restrict__ xo, R *__restrict__ xc_new,
                                         const R *__restrict__ dc, const R *__restrict__ tc, int n, int nh, int colour,
                                         int i, int j, int kh, unsigned e, R cmean, R h2, R ih2, const SolveConsts &sc)
{
    R tsh;
    const R tv = tc ? tc[e] : (R)0;
    const R dv = dc[e];
    const R S = stencil_terms<R, R>(xc_old, xo, n, nh, colour, i, j, kh, NL, tsh);
    asm volatile("" ::"v"(tv), "v"(dv));  // loaded with the stencil operands, not after the root
    const R b = (R)sc.beta * dv;
    int isv;
    const R lq = root_lap<R>(b, tsh * ih2 * ih2, sc, NL, isv);
    const R v = lq + tv;
    R xn = (S - h2 * (v - cmean)) * (R)(1.0 / 6.0);
    if (sc.jacobi)  // under-relaxed Jacobi: blend with the cell's previous value
        xn = (R)sc.omega * xn + (R)(1.0 - sc.omega) * xc_old[e];
    xc_new[e] = xn;
    return v;
}

}  // namespace pmeft
