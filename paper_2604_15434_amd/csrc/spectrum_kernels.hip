// Power spectrum of a periodic field or of a particle load (the estimator
// the paper applies to its runs, Sec. 3.6.2 and Sec. 4.2): Cloud-in-Cell
// density on a grid (finer than the particle grid to push aliasing out),
// a 3D discrete Fourier transform, and the average of |delta_k|^2 over
// spherical shells of width k_f = 2 pi / L, kept below a wavenumber cut (the
// paper keeps k < k_Nyquist / 2 of the estimator's grid).  P(k) =
// L^3 <|F_k|^2> / N^6 with F the unnormalised transform of the N^3 field.
//
// The transform is three passes of batched radix-2 FFTs, one per axis, in
// FP64: a block loads C lines of N points (the contiguous axis: C whole
// lines; the strided axes: N rows of C neighbouring lines, so every row
// is a C-element contiguous run), transforms them in LDS (bit-reversed load,
// log2 N butterfly stages with one barrier each, twiddles from a per-block
// table), and writes them back in place.
#include "pmeft_internal.h"

#include <math.h>
#include <string.h>

namespace pmeft {

void launch_deposit_fixed(const void *pos, long long np, pm_dtype dt, int ng, unsigned long long *acc,
                          hipStream_t st);

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftLdsBytes = 48 * 1024;  // line data per block (the twiddles add n / 2 complex values)
constexpr int kMaxFftN = 1024;

inline int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n)
        l++;
    return l;
}

// lines per block: the largest power of two C <= min(16, N) with C * N complex
// doubles within kFftLdsBytes (C divides N)
inline int fft_lines(int n)
{
    int c = n < 16 ? n : 16;
    while (c > 1 && (size_t)c * n * 16 > (size_t)kFftLdsBytes)
        c /= 2;
    return c;
}

__device__ __forceinline__ unsigned bitrev(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

// AXIS 2: k (contiguous); 1: j (stride N); 0: i (stride N^2).  sign -1:
// forward transform (exp(-2 pi i t f / N)).
template <int AXIS>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(double2 *__restrict__ data, int n, int lg, int C,
                                                          double sign)
{
    extern __shared__ __align__(16) unsigned char fft_lds[];
    double2 *s = reinterpret_cast<double2 *>(fft_lds);  // [C][n]
    double2 *tw = s + (size_t)C * n;                      // [n / 2]
    const unsigned tid = threadIdx.x;
    for (int m = tid; m < n / 2; m += kFftThreads) {
        double sn, cs;
        sincospi(sign * 2.0 * (double)m / (double)n, &sn, &cs);
        tw[m] = make_double2(cs, sn);
    }
    const unsigned g = blockIdx.x;  // line group
    const unsigned nn = (unsigned)n;
    const unsigned total = (unsigned)C * nn;
    // element (c, t) of the group <-> global address
    auto addr = [&](unsigned c, unsigned t) -> size_t {
        if (AXIS == 2)
            return ((size_t)g * C + c) * nn + t;
        const unsigned groups_per_row = nn / (unsigned)C;
        const unsigned a = g / groups_per_row, k0 = (g - a * groups_per_row) * (unsigned)C;
        if (AXIS == 1)  // lines (i = a, k = k0 + c) along j
            return ((size_t)a * nn + t) * nn + k0 + c;
        return ((size_t)t * nn + a) * nn + k0 + c;  // lines (j = a, k) along i
    };
    for (unsigned e = tid; e < total; e += kFftThreads) {
        unsigned c, t;
        if (AXIS == 2) {
            c = e / nn;
            t = e - c * nn;
        } else {
            t = e / (unsigned)C;
            c = e - t * (unsigned)C;
        }
        s[(size_t)c * nn + bitrev(t, lg)] = data[addr(c, t)];
    }
    __syncthreads();
    const unsigned nbf = total / 2;  // butterflies per stage
    for (int st = 1; st <= lg; st++) {
        const unsigned half = 1u << (st - 1), stride = nn >> st;  // twiddle index step
        for (unsigned b = tid; b < nbf; b += kFftThreads) {
            const unsigned c = b / (nn / 2), q = b - c * (nn / 2);
            const unsigned grp = q >> (st - 1), pos = q & (half - 1);
            const unsigned i0 = c * nn + (grp << st) + pos, i1 = i0 + half;
            const double2 w = tw[pos * stride];
            const double2 u = s[i0], v = s[i1];
            const double2 vw = make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
            s[i0] = make_double2(u.x + vw.x, u.y + vw.y);
            s[i1] = make_double2(u.x - vw.x, u.y - vw.y);
        }
        __syncthreads();
    }
    for (unsigned e = tid; e < total; e += kFftThreads) {
        unsigned c, t;
        if (AXIS == 2) {
            c = e / nn;
            t = e - c * nn;
        } else {
            t = e / (unsigned)C;
            c = e - t * (unsigned)C;
        }
        data[addr(c, t)] = s[(size_t)c * nn + t];
    }
}

// real field (natural order) -> complex
template <typename T>
__global__ __launch_bounds__(kBlock) void k_real_to_complex(const T *__restrict__ f, double2 *__restrict__ z,
                                                            size_t n3)
{
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n3; e += (size_t)gridDim.x * kBlock)
        z[e] = make_double2((double)f[e], 0.0);
}

// fixed-point CIC accumulator -> complex density contrast rho - 1
__global__ __launch_bounds__(kBlock) void k_fixed_to_complex(const unsigned long long *__restrict__ acc,
                                                             double rho_scale, double2 *__restrict__ z, size_t n3)
{
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n3; e += (size_t)gridDim.x * kBlock)
        z[e] = make_double2((double)acc[e] * rho_scale - 1.0, 0.0);
}

// Shell sums of |F|^2 * scale, of k / k_f and of the mode count, per block
// (LDS histograms with FP64 atomics, then the block's partials to
// part[block][3][nbins]).  Bin b holds b + 1/2 <= |m| < b + 3/2 with m the
// integer wave vector (numpy's fftfreq convention: index n/2 is -n/2).
constexpr int kPkBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_pk_bin(const double2 *__restrict__ z, int n, int nbins, double scale,
                                                   double *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char pk_lds[];
    double *h = reinterpret_cast<double *>(pk_lds);  // [3][nbins]
    for (int q = threadIdx.x; q < 3 * nbins; q += kBlock)
        h[q] = 0.0;
    __syncthreads();
    const unsigned n3 = (unsigned)n * n * n;  // n <= 1024: below 2^31
    const unsigned un = (unsigned)n;
    const int hn = n / 2;
    for (unsigned e = blockIdx.x * kBlock + threadIdx.x; e < n3; e += gridDim.x * kBlock) {
        const unsigned r = e / un, k = e - r * un;
        const unsigned i = r / un, j = r - i * un;
        const int mi = (int)i < hn ? (int)i : (int)i - n, mj = (int)j < hn ? (int)j : (int)j - n,
                  mk = (int)k < hn ? (int)k : (int)k - n;
        const long long m2 = (long long)mi * mi + (long long)mj * mj + (long long)mk * mk;
        const double km = sqrt((double)m2);
        const double bf = floor(km - 0.5);
        if (m2 == 0 || bf >= (double)nbins)
            continue;
        const int b = (int)bf;
        const double2 v = z[e];
        atomicAdd(&h[b], (v.x * v.x + v.y * v.y) * scale);
        atomicAdd(&h[nbins + b], km);
        atomicAdd(&h[2 * nbins + b], 1.0);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 3 * nbins; q += kBlock)
        part[(size_t)blockIdx.x * 3 * nbins + q] = h[q];
}

// out[q] = sum over blocks, in block order
__global__ __launch_bounds__(kBlock) void k_pk_finalize(const double *__restrict__ part, int nblocks, int nq,
                                                        double *__restrict__ out)
{
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= nq)
        return;
    double t = 0.0;
    for (int b = 0; b < nblocks; b++)
        t += part[(size_t)b * nq + q];
    out[q] = t;
}

struct PkPlan {
    size_t z = 0, acc = 0, part = 0, out = 0, total = 0;
};

size_t take(size_t &cur, size_t bytes)
{
    const size_t o = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return o;
}

bool pk_plan(PkPlan &P, int n, bool particles)
{
    if (n < 8 || n > kMaxFftN || (n & (n - 1)))
        return false;
    P = PkPlan();
    size_t c = 0;
    const size_t n3 = (size_t)n * n * n;
    P.z = take(c, sizeof(double2) * n3);
    if (particles)
        P.acc = take(c, sizeof(unsigned long long) * n3);
    P.part = take(c, sizeof(double) * 3 * (n / 2) * kPkBlocks);
    P.out = take(c, sizeof(double) * 3 * (n / 2));
    P.total = c + 256;
    return true;
}

int fft3d_forward(double2 *z, int n, hipStream_t st)
{
    const int lg = ilog2(n), C = fft_lines(n);
    if (C < 1 || n % C)
        return PM_EINVAL;
    const unsigned groups = (unsigned)((size_t)n * n / C);
    const size_t lds = sizeof(double2) * ((size_t)C * n + n / 2);
    hipLaunchKernelGGL((k_fft_axis<2>), dim3(groups), dim3(kFftThreads), lds, st, z, n, lg, C, -1.0);
    hipLaunchKernelGGL((k_fft_axis<1>), dim3(groups), dim3(kFftThreads), lds, st, z, n, lg, C, -1.0);
    hipLaunchKernelGGL((k_fft_axis<0>), dim3(groups), dim3(kFftThreads), lds, st, z, n, lg, C, -1.0);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP;
}

// transform z (n^3, filled), bin, copy the shells to the host
int bin_power(char *ws, const PkPlan &P, int n, double box, int nbins, double *k_out, double *pk_out,
              double *count_out, hipStream_t st)
{
    double2 *z = reinterpret_cast<double2 *>(ws + P.z);
    int e = fft3d_forward(z, n, st);
    if (e)
        return e;
    const double n3 = (double)n * n * n;
    const double scale = box * box * box / (n3 * n3);
    double *part = reinterpret_cast<double *>(ws + P.part), *out = reinterpret_cast<double *>(ws + P.out);
    hipLaunchKernelGGL(k_pk_bin, dim3(kPkBlocks), dim3(kBlock), sizeof(double) * 3 * nbins, st, z, n, nbins, scale,
                       part);
    const int nq = 3 * nbins;
    hipLaunchKernelGGL(k_pk_finalize, dim3((nq + kBlock - 1) / kBlock), dim3(kBlock), 0, st, part, kPkBlocks, nq, out);
    if (hipGetLastError() != hipSuccess)
        return PM_EHIP;
    double *host = (double *)malloc(sizeof(double) * nq);
    if (!host)
        return PM_EHIP;
    if (hipMemcpyAsync(host, out, sizeof(double) * nq, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        free(host);
        return PM_EHIP;
    }
    const double kf = 2.0 * M_PI / box;
    for (int b = 0; b < nbins; b++) {
        const double cnt = host[2 * nbins + b];
        if (count_out)
            count_out[b] = cnt;
        if (k_out)
            k_out[b] = cnt > 0.0 ? kf * host[nbins + b] / cnt : 0.0;
        if (pk_out)
            pk_out[b] = cnt > 0.0 ? host[b] / cnt : 0.0;
    }
    free(host);
    return PM_OK;
}

int pk_setup(int n, double box, int nbins, bool particles, void *ws, size_t ws_bytes, PkPlan &P)
{
    if (!ws || ((uintptr_t)ws & 255) || !(box > 0.0) || nbins < 1 || nbins > n / 2)
        return PM_EINVAL;
    if (!pk_plan(P, n, particles))
        return PM_EINVAL;
    if (ws_bytes < P.total)
        return PM_ENOMEM;
    return PM_OK;
}

}  // namespace
}  // namespace pmeft

using namespace pmeft;

extern "C" {

size_t pm_power_workspace_bytes(int n, int particles)
{
    PkPlan P;
    return pk_plan(P, n, particles != 0) ? P.total : 0;
}

int pm_field_power(const void *field, int n, pm_dtype dtype, double box, int nbins, double *k_out, double *pk_out,
                   double *count_out, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!field || (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    PkPlan P;
    int e = pk_setup(n, box, nbins, false, ws, ws_bytes, P);
    if (e)
        return e;
    hipStream_t st = (hipStream_t)stream;
    double2 *z = reinterpret_cast<double2 *>((char *)ws + P.z);
    const size_t n3 = (size_t)n * n * n;
    if (dtype == PM_F64)
        hipLaunchKernelGGL((k_real_to_complex<double>), dim3(2048), dim3(kBlock), 0, st, (const double *)field, z, n3);
    else
        hipLaunchKernelGGL((k_real_to_complex<float>), dim3(2048), dim3(kBlock), 0, st, (const float *)field, z, n3);
    return bin_power((char *)ws, P, n, box, nbins, k_out, pk_out, count_out, st);
}

int pm_particle_power(const void *pos, long long np, pm_dtype dtype, int n, double box, int nbins, double *k_out,
                      double *pk_out, double *count_out, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!pos || np <= 0 || np > (1LL << 30) || (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    PkPlan P;
    int e = pk_setup(n, box, nbins, true, ws, ws_bytes, P);
    if (e)
        return e;
    hipStream_t st = (hipStream_t)stream;
    const size_t n3 = (size_t)n * n * n;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>((char *)ws + P.acc);
    launch_zero(acc, sizeof(unsigned long long) * n3, st);
    launch_deposit_fixed(pos, np, dtype, n, acc, st);
    double2 *z = reinterpret_cast<double2 *>((char *)ws + P.z);
    hipLaunchKernelGGL(k_fixed_to_complex, dim3(2048), dim3(kBlock), 0, st, (const unsigned long long *)acc,
                       (double)n3 / (double)np / kFixScale, z, n3);
    return bin_power((char *)ws, P, n, box, nbins, k_out, pk_out, count_out, st);
}

int pm_boost(const double *k, const double *pk_num, const double *pk_den, int nbins, double sigma_k, double *r_out)
{
    if (!k || !pk_num || !pk_den || !r_out || nbins < 1 || !(sigma_k >= 0.0))
        return PM_EINVAL;
    for (int b = 0; b < nbins; b++)
        if (!(pk_den[b] != 0.0) || !isfinite(pk_num[b] / pk_den[b]))
            return PM_ENONFINITE;
    for (int b = 0; b < nbins; b++) {
        if (sigma_k == 0.0) {
            r_out[b] = pk_num[b] / pk_den[b];
            continue;
        }
        double sw = 0.0, s = 0.0;
        for (int c = 0; c < nbins; c++) {
            const double d = (k[c] - k[b]) / sigma_k;
            const double w = exp(-0.5 * d * d);
            sw += w;
            s += w * pk_num[c] / pk_den[c];
        }
        r_out[b] = s / sw;
    }
    return PM_OK;
}

}  // extern "C"
