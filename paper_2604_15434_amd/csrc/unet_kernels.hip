// Kernels of the learned warm start: a 3-level 3D U-Net on the periodic grid.
//
// Activations are channels-last bf16 tensors (voxel-major, channels
// contiguous); a tensor view is (pointer, row stride in elements, channel
// offset), so a convolution can read or write one slice of a concatenation
// buffer.  Convolutions are implicit GEMMs on the MFMA unit (BF16 operands,
// FP32 accumulation) with the 27 taps (periodic neighbours) and the input
// channels as the K index:
//   k_conv3          one-plane kernel: a wave computes 16 consecutive voxels
//                    along k times 16 output channels per tile
//                    (v_mfma_f32_16x16x16_bf16);
//   k_conv3_lds      the plane's neighbourhood staged in LDS (grids that are
//                    multiples of 64, more than 48 input channels);
//   k_conv3_march    grids that are multiples of 64, up to 48 input channels:
//                    blocks march along i over input planes (three-slot LDS
//                    ring), each feeding three output planes' accumulators
//                    (v_mfma_f32_16x16x32_bf16);
//   k_conv3_in1      the first layer at inference (one density channel);
//   k_upconv_poly    decoder layers on upsampled tensors at inference
//                    (polyphase form on the coarse grid);
//   k_updec_march    the decoder layer on the 16-channel level at inference,
//                    skip channels and polyphase sum in one march;
//   k_conv3_wgrad    weight and bias gradients (voxels as the K index);
//   k_pack_jobs      every weight layout the kernels read, in one launch.
// MFMA operand layout (16x16xK, K = 16 or 32, L = K / 4 values per lane):
// lane l supplies A[l%16][L(l/16)+i] and B[L(l/16)+i][l%16], i < L, and
// receives D[4(l/16)+i][l%16], i = 0..3.
#include "pmeft_internal.h"

#include <math.h>

namespace pmeft {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)  // inf / nan: truncate, keep nan quiet
        return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ void tap_offsets(int t, int &di, int &dj, int &dk)
{
    di = t / 9 - 1;
    dj = (t / 3) % 3 - 1;
    dk = t % 3 - 1;
}

static inline unsigned xcd_blocks(unsigned nb) { return nb >= 8 ? (nb + 7) / 8 * 8 : nb; }

__device__ __forceinline__ unsigned xcd_block(unsigned nb_real)
{
    const unsigned b = blockIdx.x, g = gridDim.x;
    if (g % 8)
        return b;
    return (b % 8) * (g / 8) + b / 8;
}

// ---------------------------------------------------------------- convolution
// out[v][out_off + o] = act(bias[o] + sum_t sum_c in[v + s d_t][in_off + c] * Wp[t][o][c])
// with s = +1 (forward) or -1 (input gradient, Wp packed as the transpose).
// cin_pad, cout_pad: multiples of 16; only o < cout is written.
// A wave computes MT*16 consecutive voxels along k of one (i, j) row times
// COT*16 output channels.  For each of the 9 (di, dj) neighbour rows and
// 16-channel input slice it first issues all 3*MT activation and 3*COT weight
// fragment loads (the three dk taps), then the 3*MT*COT MFMAs, so the loads
// of a row overlap instead of serialising behind each MFMA.
template <int MT, int COT>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t *__restrict__ in, int in_stride, int in_off, int cin_pad,
                                               const uint16_t *__restrict__ wp, int cout_pad,
                                               const float *__restrict__ bias, int cout, void *__restrict__ out,
                                               int out_stride, int out_off, int out_f32, int n, int flip, int relu,
                                               unsigned nseg)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned seg = xcd_block(0) * 4 + wave;
    if (seg >= nseg)
        return;
    const int segs_row = n / (16 * MT);
    const unsigned row = seg / segs_row;
    const int k0 = (int)(seg - row * segs_row) * 16 * MT;
    const int i = (int)(row / n), j = (int)(row - (row / n) * n);
    const int r = lane & 15, q = lane >> 4;
    const int co_base = blockIdx.y * COT * 16;
    const int sgn = flip ? -1 : 1;
    f32x4 acc[MT][COT];
#pragma unroll
    for (int m = 0; m < MT; m++)
#pragma unroll
        for (int t = 0; t < COT; t++)
            acc[m][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // voxel offsets along k of this lane's rows for dk = -1, 0, +1 (input side)
    int kk[3][MT];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int m = 0; m < MT; m++)
            kk[d][m] = wrapi(k0 + 16 * m + r + sgn * (d - 1), n);
    for (int dij = 0; dij < 9; dij++) {
        const int di = sgn * (dij / 3 - 1), dj = sgn * (dij % 3 - 1);
        const int ii = wrapi(i + di, n), jj = wrapi(j + dj, n);
        const uint16_t *rowp = in + (size_t)((ii * n + jj) * n) * in_stride + in_off + 4 * q;
        const uint16_t *wrow = wp + ((size_t)(dij * 3) * cout_pad + co_base + r) * cin_pad + 4 * q;
        for (int c0 = 0; c0 < cin_pad; c0 += 16) {
            bf16x4 a[3][MT], b[3][COT];
#pragma unroll
            for (int d = 0; d < 3; d++) {
#pragma unroll
                for (int m = 0; m < MT; m++)
                    a[d][m] = *(const bf16x4 *)(rowp + (size_t)kk[d][m] * in_stride + c0);
#pragma unroll
                for (int t = 0; t < COT; t++)
                    b[d][t] = *(const bf16x4 *)(wrow + ((size_t)d * cout_pad + t * 16) * cin_pad + c0);
            }
#pragma unroll
            for (int d = 0; d < 3; d++)
#pragma unroll
                for (int m = 0; m < MT; m++)
#pragma unroll
                    for (int t = 0; t < COT; t++)
                        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[d][m], b[d][t], acc[m][t], 0, 0, 0);
        }
    }
    const size_t vbase = (size_t)((i * n + j) * n + k0);
#pragma unroll
    for (int t = 0; t < COT; t++) {
        const int o = co_base + t * 16 + r;
        if (o >= cout)
            continue;
        const float bo = bias ? bias[o] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; m++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                float v = acc[m][t][e] + bo;
                if (relu)
                    v = fmaxf(v, 0.f);
                const size_t idx = (vbase + 16 * m + 4 * q + e) * out_stride + out_off + o;
                if (out_f32)
                    ((float *)out)[idx] = v;
                else
                    ((uint16_t *)out)[idx] = f2bf(v);
            }
    }
}

// LDS-staged variant for grids with n % 64 == 0: a block computes a tile of
// 4 RW rows (j) x 64 voxels (k) of one plane (i) for COT*16 output channels.
// For every 16-channel input slice it stages the 3 x (4 RW + 2) x 66 voxel
// neighbourhood of the tile in LDS (voxel stride 20 bf16 = 40 bytes, which
// spreads a wave's 8-byte fragment reads over distinct banks), then each wave
// (RW rows) runs the 27 taps x 4 RW voxel tiles x COT channel tiles from LDS.
// Every block reads the same weights, so each fragment feeding RW rows' MFMAs
// halves their L2 traffic at RW = 2.  The weights are the MFMA's A operand:
// a lane holds four consecutive output channels of one voxel (vector stores
// when the view is 4-aligned).
constexpr int kCvK = 64, kCvStride = 20;

template <int COT, int RW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv3_lds(const uint16_t *__restrict__ in, int in_stride, int in_off,
                                                   int cin_pad, const uint16_t *__restrict__ wp, int cout_pad,
                                                   const float *__restrict__ bias, int cout, void *__restrict__ out,
                                                   int out_stride, int out_off, int out_f32, int n, int flip, int relu,
                                                   unsigned ntiles)
{
    constexpr int ROWS = 4 * RW, WR = ROWS + 2, WVOX = 3 * WR * (kCvK + 2);
    __shared__ __align__(16) uint16_t tile[WVOX * kCvStride];
    const unsigned t = xcd_block(0);
    if (t >= ntiles)
        return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int nkt = n / kCvK, njt = n / ROWS;
    const int kt = (int)(t % nkt), jt = (int)((t / nkt) % njt), i = (int)(t / ((unsigned)nkt * njt));
    const int j0 = jt * ROWS, k0 = kt * kCvK;
    const int co_base = blockIdx.y * COT * 16;
    const int sgn = flip ? -1 : 1;
    const bool vec = out_stride % 4 == 0 && out_off % 4 == 0;
    f32x4 acc[RW][4][COT];
#pragma unroll
    for (int w = 0; w < RW; w++)
#pragma unroll
        for (int m = 0; m < 4; m++)
#pragma unroll
            for (int u = 0; u < COT; u++)
                acc[w][m][u] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // weight fragments of tap `tap` and input slice c0 for this lane (a
    // uniform base plus the lane's offset)
    const unsigned wlane = (unsigned)((co_base + r) * cin_pad + 4 * q);
    auto load_b = [&](int tap, int c0, bf16x4 *dst) {
#pragma unroll
        for (int u = 0; u < COT; u++) {
            const uint16_t *wt = wp + ((size_t)tap * cout_pad + u * 16) * cin_pad + c0;
            dst[u] = *(const bf16x4 *)(wt + wlane);
        }
    };
    // staging of one 16-channel input slice: this thread's 8-byte chunks of
    // the neighbourhood in three batches, each with all its loads issued
    // before any is stored
    constexpr int NST = (WVOX * 4 + 255) / 256, NB = (NST + 2) / 3;
    const int part = threadIdx.x & 3;
    auto stage = [&](int c0, int st0) {
        uint2 stg[NB];
#pragma unroll
        for (int u = 0; u < NB; u++) {
            const int v = (threadIdx.x >> 2) + 64 * (st0 + u);
            if (st0 + u < NST && v < WVOX) {
                const int pl = v / (WR * (kCvK + 2));
                const int rem = v - pl * WR * (kCvK + 2);
                const int row = rem / (kCvK + 2), col = rem - row * (kCvK + 2);
                const int ii = wrapi(i + pl - 1, n), jj = wrapi(j0 + row - 1, n), kk = wrapi(k0 + col - 1, n);
                stg[u] = *(const uint2 *)(in + (size_t)((ii * n + jj) * n + kk) * in_stride + in_off + c0 + 4 * part);
            }
        }
        // voxel v = (plane * WR + row) * 66 + col, 16 channels as 4 x 8 bytes
#pragma unroll
        for (int u = 0; u < NB; u++) {
            const int v = (threadIdx.x >> 2) + 64 * (st0 + u);
            if (st0 + u < NST && v < WVOX)
                *(uint2 *)(tile + v * kCvStride + 4 * part) = stg[u];
        }
    };
    // one tap: the MFMAs of tap `tap` on weights bc while the weights of tap
    // + 2 load into bl (the slot of the tap computed last; the last two taps
    // reload tap 26, unconditionally, so the wait counts stay static)
    auto tap_step = [&](int tap, int c0, const bf16x4 *bc, bf16x4 *bl) {
        load_b(tap + 2 < 27 ? tap + 2 : 26, c0, bl);
        int di, dj, dk;
        tap_offsets(tap, di, dj, dk);
        const int pl = 1 + sgn * di, colb = 1 + r + sgn * dk;
#pragma unroll
        for (int w = 0; w < RW; w++) {
            const int row = 1 + RW * wave + w + sgn * dj;
            const uint16_t *tb = tile + ((pl * WR + row) * (kCvK + 2) + colb) * kCvStride + 4 * q;
            bf16x4 a[4];
#pragma unroll
            for (int m = 0; m < 4; m++)
                a[m] = *(const bf16x4 *)(tb + 16 * m * kCvStride);
#pragma unroll
            for (int m = 0; m < 4; m++)
#pragma unroll
                for (int u = 0; u < COT; u++)
                    acc[w][m][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bc[u], a[m], acc[w][m][u], 0, 0, 0);
        }
    };
    for (int c0 = 0; c0 < cin_pad; c0 += 16) {
        // weights two taps ahead in a ring of three register slots; the first
        // two taps' load with the slice
        bf16x4 b0[COT], b1[COT], b2[COT];
        load_b(0, c0, b0);
        load_b(1, c0, b1);
        stage(c0, 0);
        stage(c0, NB);
        stage(c0, 2 * NB);
        __syncthreads();
#pragma unroll 1
        for (int t3 = 0; t3 < 27; t3 += 3) {
            tap_step(t3, c0, b0, b2);
            tap_step(t3 + 1, c0, b1, b0);
            tap_step(t3 + 2, c0, b2, b1);
        }
        __syncthreads();
    }
    // lane (r, q) holds channels 4q .. 4q + 3 (+ 16 u) of voxel 16 m + r
#pragma unroll
    for (int w = 0; w < RW; w++) {
        const size_t vbase = (size_t)((i * n + j0 + RW * wave + w) * n + k0);
#pragma unroll
        for (int u = 0; u < COT; u++) {
            const int o0 = co_base + u * 16 + 4 * q;
            float bo[4];
#pragma unroll
            for (int e = 0; e < 4; e++)
                bo[e] = (bias && o0 + e < cout) ? bias[o0 + e] : 0.f;
#pragma unroll
            for (int m = 0; m < 4; m++) {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; e++)
                    v[e] = relu ? fmaxf(acc[w][m][u][e] + bo[e], 0.f) : acc[w][m][u][e] + bo[e];
                const size_t idx = (vbase + 16 * m + r) * out_stride + out_off + o0;
                if (vec && o0 + 3 < cout) {
                    if (out_f32)
                        *(f32x4 *)((float *)out + idx) = (f32x4){v[0], v[1], v[2], v[3]};
                    else
                        *(u16x4 *)((uint16_t *)out + idx) = (u16x4){f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        if (o0 + e < cout) {
                            if (out_f32)
                                ((float *)out)[idx + e] = v[e];
                            else
                                ((uint16_t *)out)[idx + e] = f2bf(v[e]);
                        }
                }
            }
        }
    }
}

template <int MT>
static void launch_conv3_mt(const uint16_t *in, int in_stride, int in_off, int cin_pad, const uint16_t *wp,
                            int cout_pad, const float *bias, int cout, void *out, int out_stride, int out_off,
                            bool out_f32, int n, bool flip, bool relu, hipStream_t st)
{
    const unsigned nseg = (unsigned)n * n * (n / (16 * MT));
    const unsigned nbx = xcd_blocks((nseg + 3) / 4);
    // output tiles per wave: the largest of 4, 3, 2, 1 that divides the tile count
    const int tiles = cout_pad / 16;
    const int cot = tiles % 4 == 0 ? 4 : (tiles % 3 == 0 ? 3 : (tiles % 2 == 0 ? 2 : 1));
    dim3 grid(nbx, cout_pad / (cot * 16));
#define PM_CONV(C)                                                                                                     \
    hipLaunchKernelGGL((k_conv3<MT, C>), grid, dim3(256), 0, st, in, in_stride, in_off, cin_pad, wp, cout_pad, bias,   \
                       cout, out, out_stride, out_off, out_f32 ? 1 : 0, n, flip ? 1 : 0, relu ? 1 : 0, nseg)
    if (cot == 4)
        PM_CONV(4);
    else if (cot == 3)
        PM_CONV(3);
    else if (cot == 2)
        PM_CONV(2);
    else
        PM_CONV(1);
#undef PM_CONV
}

// Plane-marching variant for grids with n % 64 == 0 and at most 48 input
// channels (8-aligned views): a block of 8 waves owns 4 rows (j) by 64 voxels
// (k), two waves per row of 32 voxels, and walks the input planes s = i0 - 1
// .. i0 + PL of its PL output planes i0 .. i0 + PL - 1.  Input plane s
// (6 x 66 voxels, all input channels, in an LDS ring of three slots: plane
// s + 2 loads while s is computed) feeds the output planes s - 1, s and s + 1
// through the taps with di = +1, 0, -1 (forward; mirrored for the input
// gradient), held in three rolling accumulators: every activation fragment
// read from LDS feeds three MFMAs, and output plane s - 1 is complete after
// plane s.  Per input plane the K index runs over the 9 (dj, dk) taps and the
// channels, in chunks of 32 on v_mfma_f32_16x16x32_bf16 (a chunk may span two
// taps: each lane's 8 values lie in one tap, 8-aligned channels) and a final
// 16 on the 16x16x16 form when 9 * cin_pad is not a multiple of 32; each
// output still sums its taps in order.  The voxel stride in LDS is an odd
// number of 16-byte units (the 16-byte fragment reads of 8 consecutive lanes
// then fall in distinct banks).  PL = 2 mod 3, so the steps between the two
// boundary steps at each end come in whole rounds of the three slots.

constexpr int kMarchThreads = 512;

// Planes per tile of the plane-marching convolution (2 mod 3): long tiles
// where the grid still has a tile per block slot, else 32 / 8.
static inline int march_planes(int n)
{
    if (n >= 256 && n % 128 == 0)
        return 128;
    return n >= 128 ? 32 : 8;
}

template <int V>
struct IConst {
    static constexpr int value = V;
};

//
// HD (one 16-channel output tile, ReLU): the network's 1x1x1 output head is
// applied in the epilogue, out[v] = hb + sum_o hw[o] relu(conv[v][o]) as
// FP32 in natural voxel order, and the 16-channel activation is never stored
// (nor rounded to BF16, as the unfused form rounds it).  The channel sum runs
// over the 16 lanes of a row of the MFMA result (row rotations 8, 4, 2, 1).
template <int CS, int COT, bool HD = false>
__global__ __launch_bounds__(kMarchThreads) __attribute__((amdgpu_waves_per_eu(CS == 1 && COT == 1 ? 4 : 1))) void k_conv3_march(const uint16_t *__restrict__ in, int in_stride, int in_off,
                                                     const uint16_t *__restrict__ wp, int cout_pad,
                                                     const float *__restrict__ bias, int cout, void *__restrict__ out,
                                                     int out_stride, int out_off, int out_f32, int n, int flip,
                                                     int relu, unsigned ntiles, int PL, const float *__restrict__ hw,
                                                     const float *__restrict__ hb)
{
    static_assert(!HD || COT == 1, "the head reads one output tile");
    // TR: weights as the A operand, so the result is D[channel][voxel] and a
    // lane holds four consecutive channels of one voxel (vector stores when
    // the output view is 4-aligned); the head keeps D[voxel][channel]
    constexpr bool TR = !HD;
    const bool vec = out_stride % 4 == 0 && out_off % 4 == 0;
    constexpr int CP = 16 * CS;                 // input channels (padded)
    constexpr int SV = CP + 8;                  // LDS voxel stride (halfwords)
    constexpr int WV = 6 * 66;                  // voxels per staged plane
    constexpr int NCH = WV * (CP / 8);          // 16-byte chunks per plane
    constexpr int PER = (NCH + kMarchThreads - 1) / kMarchThreads;
    constexpr int KP = 9 * CP;                  // GEMM K per input plane
    constexpr int NK = KP / 32, TAIL = KP % 32;
    __shared__ __align__(16) uint16_t ring[3 * WV * SV];
    const int wave = threadIdx.x >> 7, mh = ((threadIdx.x >> 6) & 1) * 2;  // row, first m-tile
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int nkt = n / 64, nit = n / PL;
    const int co_base = blockIdx.y * COT * 16;
    const int sgn = flip ? -1 : 1;
    const size_t plane_elems = (size_t)n * n * in_stride;
    const unsigned nb = gridDim.x;
    const unsigned lb = (nb % 8) ? blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    // B fragments of output offset e (output plane s - 1 + e takes input plane
    // s through the tap with di = sgn (1 - e)) and K chunk c; in registers for
    // the whole block where they fit
    constexpr bool BREG = COT == 1 && CS <= 2;
    auto wfrag8 = [&](const uint16_t *w, int e, int c, int u) {
        const int kk = 32 * c + 8 * q, tap = (1 + sgn * (1 - e)) * 9 + kk / CP, ch = kk % CP;
        return __builtin_bit_cast(bf16x8, *(const u32x4 *)(w + ((size_t)tap * cout_pad + co_base + u * 16 + r) * CP + ch));
    };
    auto wfrag4 = [&](const uint16_t *w, int e, int u) {
        const int kk = 32 * NK + 4 * q, tap = (1 + sgn * (1 - e)) * 9 + kk / CP, ch = kk % CP;
        return *(const bf16x4 *)(w + ((size_t)tap * cout_pad + co_base + u * 16 + r) * CP + ch);
    };
    bf16x8 bw[BREG ? 3 : 1][BREG ? NK : 1][COT];
    bf16x4 bt[BREG && TAIL ? 3 : 1][COT];
    if constexpr (BREG) {
#pragma unroll
        for (int e = 0; e < 3; e++)
#pragma unroll
            for (int u = 0; u < COT; u++) {
#pragma unroll
                for (int c = 0; c < NK; c++)
                    bw[e][c][u] = wfrag8(wp, e, c, u);
                if constexpr (TAIL != 0)
                    bt[e][u] = wfrag4(wp, e, u);
            }
    }
    for (unsigned t = lb; t < ntiles; t += nb) {
        const int ib = (int)(t % nit), kt = (int)((t / nit) % nkt), jt = (int)(t / ((unsigned)nit * nkt));
        const int i0 = ib * PL, j0 = jt * 4, k0 = kt * 64;
        // this thread's staging chunks: within-plane source offset and LDS offset
        unsigned soff[PER];
        int loff[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int c = threadIdx.x + u * kMarchThreads;
            const int cc = c < NCH ? c : 0;
            const int v = cc / (CP / 8), part = cc % (CP / 8);
            const int row = v / 66, col = v % 66;
            const int jj = wrapi(j0 + row - 1, n), kk = wrapi(k0 + col - 1, n);
            soff[u] = (unsigned)((jj * n + kk) * in_stride + in_off + 8 * part);
            loff[u] = v * SV + 8 * part;
        }
        u32x4 pre[PER];
        auto fetch = [&](int ii) {
            const uint16_t *base = in + (size_t)wrapi(ii, n) * plane_elems;
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kMarchThreads < NCH)
                    pre[u] = *(const u32x4 *)(base + soff[u]);
        };
        auto put = [&](int slot) {
            uint16_t *dst = ring + slot * WV * SV;
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kMarchThreads < NCH)
                    *(u32x4 *)(dst + loff[u]) = pre[u];
        };
        fetch(i0 - 1);
        put(0);
        fetch(i0);
        put(1);
        __syncthreads();
        f32x4 acc[3][2][COT];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int m = 0; m < 2; m++)
#pragma unroll
                for (int u = 0; u < COT; u++)
                    acc[a][m][u] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // output plane o from its accumulators
        auto store_plane = [&](int o, const f32x4 (&ac)[2][COT]) {
            const size_t vbase = ((size_t)o * n + j0 + wave) * n + k0;
            if constexpr (HD) {
                // lane (r, q) holds channel r of voxels 16 (mh + m) + 4 q + e
                const float bo = bias[r], ho = hw[r];
                float sm[2][4];
#pragma unroll
                for (int m = 0; m < 2; m++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        float v = ho * fmaxf(ac[m][0][e] + bo, 0.f);
                        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
                        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
                        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xf, 0xf, false));
                        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));
                        sm[m][e] = v;
                    }
                // every lane of a row now holds the row's eight sums; lane r < 8
                // writes voxel 16 (mh + r / 4) + 4 q + r % 4
                const int mm = (r >> 2) & 1, ee = r & 3;
                float y = sm[0][0];
#pragma unroll
                for (int m = 0; m < 2; m++)
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        y = (mm == m && ee == e) ? sm[m][e] : y;
                if (r < 8)
                    ((float *)out)[vbase + 16 * (mh + mm) + 4 * q + ee] = hb[0] + y;
            } else {
                // lane (r, q) holds channels 4q .. 4q + 3 (+ 16 u) of voxel 16 (mh + m) + r
#pragma unroll
                for (int u = 0; u < COT; u++) {
                    const int o0 = co_base + u * 16 + 4 * q;
                    float bo[4];
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        bo[e] = (bias && o0 + e < cout) ? bias[o0 + e] : 0.f;
#pragma unroll
                    for (int m = 0; m < 2; m++) {
                        float v[4];
#pragma unroll
                        for (int e = 0; e < 4; e++)
                            v[e] = relu ? fmaxf(ac[m][u][e] + bo[e], 0.f) : ac[m][u][e] + bo[e];
                        const size_t idx = (vbase + 16 * (mh + m) + r) * out_stride + out_off + o0;
                        if (vec && o0 + 3 < cout) {
                            if (out_f32)
                                *(f32x4 *)((float *)out + idx) = (f32x4){v[0], v[1], v[2], v[3]};
                            else
                                *(u16x4 *)((uint16_t *)out + idx) =
                                    (u16x4){f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; e++)
                                if (o0 + e < cout) {
                                    if (out_f32)
                                        ((float *)out)[idx + e] = v[e];
                                    else
                                        ((uint16_t *)out)[idx + e] = f2bf(v[e]);
                                }
                        }
                    }
                }
            }
        };
        // one input plane s whose ring slot (and the accumulator slot of output
        // plane s - 1) is JM; LD: plane s + 2 is still to be staged; ST: output
        // plane s - 1 lies in the tile
        auto step = [&](int s, auto JM, auto LD, auto ST) {
            constexpr int jm = decltype(JM)::value;
            if constexpr (decltype(LD)::value)
                fetch(s + 2);
            const uint16_t *sl = ring + jm * WV * SV;
            // without register-resident weights each step loads its own
            // (the empty asm keeps them from being hoisted out of the loops)
            const uint16_t *ws = wp;
            if constexpr (!BREG)
                asm volatile("" : "+s"(ws));
            auto chunk = [&](int c) {
                const int kk = 32 * c + 8 * q, tip = kk / CP, ch = kk % CP;
                const int dj = tip / 3 - 1, dk = tip % 3 - 1;
                const int ab = ((1 + wave + sgn * dj) * 66 + 1 + 16 * mh + r + sgn * dk) * SV + ch;
                bf16x8 a[2];
#pragma unroll
                for (int m = 0; m < 2; m++)
                    a[m] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(sl + ab + 16 * m * SV));
#pragma unroll
                for (int e = 0; e < 3; e++) {
                    bf16x8 b[COT];
#pragma unroll
                    for (int u = 0; u < COT; u++)
                        b[u] = BREG ? bw[BREG ? e : 0][BREG ? c : 0][u] : wfrag8(ws, e, c, u);
#pragma unroll
                    for (int m = 0; m < 2; m++)
#pragma unroll
                        for (int u = 0; u < COT; u++)
                            acc[(jm + e) % 3][m][u] =
                                TR ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[u], a[m], acc[(jm + e) % 3][m][u], 0, 0, 0)
                                   : __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[u], acc[(jm + e) % 3][m][u], 0, 0, 0);
                }
            };
            if constexpr (BREG) {
#pragma unroll
                for (int c = 0; c < NK; c++)
                    chunk(c);
            } else {
#pragma unroll 2
                for (int c = 0; c < NK; c++)
                    chunk(c);
            }
            if constexpr (TAIL != 0) {
                const int kk = 32 * NK + 4 * q, tip = kk / CP, ch = kk % CP;
                const int dj = tip / 3 - 1, dk = tip % 3 - 1;
                const int ab = ((1 + wave + sgn * dj) * 66 + 1 + 16 * mh + r + sgn * dk) * SV + ch;
                bf16x4 a[2];
#pragma unroll
                for (int m = 0; m < 2; m++)
                    a[m] = *(const bf16x4 *)(sl + ab + 16 * m * SV);
#pragma unroll
                for (int e = 0; e < 3; e++) {
                    bf16x4 b[COT];
#pragma unroll
                    for (int u = 0; u < COT; u++)
                        b[u] = BREG ? bt[BREG ? e : 0][u] : wfrag4(ws, e, u);
#pragma unroll
                    for (int m = 0; m < 2; m++)
#pragma unroll
                        for (int u = 0; u < COT; u++)
                            acc[(jm + e) % 3][m][u] =
                                TR ? __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b[u], a[m], acc[(jm + e) % 3][m][u], 0, 0, 0)
                                   : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], b[u], acc[(jm + e) % 3][m][u], 0, 0, 0);
                }
            }
            // the epilogue is kept apart from the MFMAs around it (scheduling
            // barriers): with the compiler free to interleave the two, the
            // head instance's results varied from run to run
            if constexpr (decltype(ST)::value) {
                __builtin_amdgcn_sched_barrier(0);
                store_plane(s - 1, acc[jm]);
                __builtin_amdgcn_sched_barrier(0);
            }
            // the slot of plane s - 1 (stored, or outside the tile) becomes plane s + 2's
#pragma unroll
            for (int m = 0; m < 2; m++)
#pragma unroll
                for (int u = 0; u < COT; u++)
                    acc[jm][m][u] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if constexpr (decltype(LD)::value)
                put((jm + 2) % 3);
            __syncthreads();
        };
        // input planes i0 - 1 and i0 (no complete output plane yet), then whole
        // rounds of three, then i0 + PL - 1 and i0 + PL (nothing left to stage)
        step(i0 - 1, IConst<0>(), IConst<1>(), IConst<0>());
        step(i0, IConst<1>(), IConst<1>(), IConst<0>());
        for (int s = i0 + 1; s < i0 + PL - 1; s += 3) {
            step(s, IConst<2>(), IConst<1>(), IConst<1>());
            step(s + 1, IConst<0>(), IConst<1>(), IConst<1>());
            step(s + 2, IConst<1>(), IConst<1>(), IConst<1>());
        }
        step(i0 + PL - 1, IConst<2>(), IConst<0>(), IConst<1>());
        step(i0 + PL, IConst<0>(), IConst<0>(), IConst<1>());
    }
}

// Convolution of a nearest-neighbour upsampled tensor, evaluated on the
// coarse grid (inference).  A fine voxel v = 2P + pi (parity pi per axis) sees
// the coarse parent of v + d for its 27 taps d; along an axis the three taps
// fall on two coarse offsets, pi - 1 and pi, so the layer restricted to the
// upsampled channels is, per parity, a 2 x 2 x 2 convolution of the coarse
// tensor with weights summed over the taps that share a coarse offset (the
// polyphase form; 8 x 8 instead of 27 taps per output).  Wp[p][e][o][c]: parity
// p = 4 pi_i + 2 pi_j + pi_k, coarse tap e = 4 e_i + 2 e_j + e_k, offset
// e - 1 + pi per axis.  The block stages the 3 x 6 x (KT + 2) coarse
// neighbourhood of 4 coarse rows x KT coarse voxels (all CIN channels) in LDS
// (KT small enough for three blocks per CU).  Wave w owns the two parities
// (pi_i, pi_j) = (w / 2, w % 2), pi_k = 0, 1, for all four rows: per parity it
// runs the 8 taps x CIN/32 K-chunks on v_mfma_f32_16x16x32_bf16, each weight
// fragment feeding the four rows (every block reads the same weights, so
// fewer fragment loads per output keep them off the L2's critical path).
// Epilogue: out[v][ooff + o] =
// act(bias[o] + add[v][o] + sum), with add the rest of the layer (the other
// input channels, FP32, cout per voxel) computed beforehand; out may be add
// itself when FP32.
template <int CIN, int COT, int KT, bool F32OUT, bool RELU>
__global__ __launch_bounds__(256) void k_upconv_poly(const uint16_t *__restrict__ in, int nc,
                                                     const uint16_t *__restrict__ wp, int cout_pad,
                                                     const float *__restrict__ bias, const float *add, void *out,
                                                     int out_stride, int out_off, unsigned ntiles)
{
    constexpr int SV = CIN + 8;  // odd number of 16-byte units
    constexpr int WK = KT + 2, WV = 3 * 6 * WK;
    constexpr int NCH = WV * (CIN / 8);
    constexpr int MT = KT / 16;
    __shared__ __align__(16) uint16_t tile[WV * SV];
    const unsigned t = xcd_block(0);
    if (t >= ntiles)
        return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int nkt = nc / KT, njt = nc / 4;
    const int kt = (int)(t % nkt), jt = (int)((t / nkt) % njt), I = (int)(t / ((unsigned)nkt * njt));
    const int J0 = jt * 4, K0 = kt * KT;
    const int co_base = blockIdx.y * COT * 16;
    for (int c = threadIdx.x; c < NCH; c += 256) {
        const int v = c / (CIN / 8), part = c % (CIN / 8);
        const int pl = v / (6 * WK), rem = v - pl * 6 * WK, row = rem / WK, col = rem - row * WK;
        const int ii = wrapi(I + pl - 1, nc), jj = wrapi(J0 + row - 1, nc), kk = wrapi(K0 + col - 1, nc);
        *(u32x4 *)(tile + v * SV + 8 * part) =
            *(const u32x4 *)(in + ((size_t)((ii * nc + jj) * nc + kk)) * CIN + 8 * part);
    }
    __syncthreads();
    const int nf = 2 * nc;
    const int pi = wave >> 1, pj = wave & 1;
    // Every output channel group is whole and every view 4-aligned (the
    // launcher checks), so loads and stores are 4-channel vectors with no
    // branch to split the load pipeline: both parities' addends load before
    // the first parity is computed.
    constexpr int NCK = CIN / 32;
    typedef f32x4 AddRegs[4][MT][COT];
    const int cout = cout_pad;
    f32x4 bo[COT];
#pragma unroll
    for (int u = 0; u < COT; u++) {
        const int o0 = co_base + u * 16 + 4 * q;
#pragma unroll
        for (int e = 0; e < 4; e++)
            bo[u][e] = bias ? bias[o0 + e] : 0.f;
    }
    // fine voxel of parity (pi, pj, pk) above coarse voxel (I, J0 + row, K0 + 16 m + r)
    auto fine_voxel = [&](int row, int pk, int m) {
        const int J = J0 + row, K = K0 + 16 * m + r;
        return ((size_t)(2 * I + pi) * nf + 2 * J + pj) * nf + 2 * K + pk;
    };
    auto load_add = [&](int pk, AddRegs &addv) {
#pragma unroll
        for (int row = 0; row < 4; row++)
#pragma unroll
            for (int m = 0; m < MT; m++)
#pragma unroll
                for (int u = 0; u < COT; u++)
                    addv[row][m][u] = *(const f32x4 *)(add + fine_voxel(row, pk, m) * cout + co_base + u * 16 + 4 * q);
    };
    auto compute = [&](int pk, const AddRegs &addv) {
        const int p = 4 * pi + 2 * pj + pk;
        f32x4 acc[4][MT][COT];
#pragma unroll
        for (int row = 0; row < 4; row++)
#pragma unroll
            for (int m = 0; m < MT; m++)
#pragma unroll
                for (int u = 0; u < COT; u++)
                    acc[row][m][u] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int oi = (e >> 2) - 1 + pi, oj = ((e >> 1) & 1) - 1 + pj, ok = (e & 1) - 1 + pk;
#pragma unroll
            for (int c = 0; c < NCK; c++) {
                bf16x8 b[COT];
#pragma unroll
                for (int u = 0; u < COT; u++)
                    b[u] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(wp + ((size_t)(p * 8 + e) * cout_pad + co_base +
                                                                             u * 16 + r) * CIN + 32 * c + 8 * q));
#pragma unroll
                for (int row = 0; row < 4; row++) {
                    const int ab = ((1 + oi) * 6 + 1 + row + oj) * WK + 1 + r + ok;  // window voxel of m = 0
#pragma unroll
                    for (int m = 0; m < MT; m++) {
                        const bf16x8 a =
                            __builtin_bit_cast(bf16x8, *(const u32x4 *)(tile + (ab + 16 * m) * SV + 32 * c + 8 * q));
#pragma unroll
                        for (int u = 0; u < COT; u++)
                            acc[row][m][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[u], a, acc[row][m][u], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int row = 0; row < 4; row++)
#pragma unroll
            for (int u = 0; u < COT; u++) {
                const int o0 = co_base + u * 16 + 4 * q;
#pragma unroll
                for (int m = 0; m < MT; m++) {
                    float v[4];
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        v[e] = acc[row][m][u][e] + bo[u][e] + addv[row][m][u][e];
                        if (RELU)
                            v[e] = fmaxf(v[e], 0.f);
                    }
                    // out may alias add: same elements, same thread
                    const size_t oi_ = fine_voxel(row, pk, m) * out_stride + out_off + o0;
                    if constexpr (F32OUT)
                        *(f32x4 *)((float *)out + oi_) = (f32x4){v[0], v[1], v[2], v[3]};
                    else
                        *(u16x4 *)((uint16_t *)out + oi_) =
                            (u16x4){f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
                }
            }
    };
#pragma unroll 1
    for (int pk = 0; pk < 2; pk++) {
        AddRegs addv;
        load_add(pk, addv);
        compute(pk, addv);
    }
}

// The decoder layer on the upsampled 16-channel level in one kernel
// (inference): 16 skip channels at the fine grid n plus 32 coarse channels
// at n/2 seen through nearest-neighbour upsampling, 16 outputs.  It marches
// the fine input planes like k_conv3_march (three-slot ring, three rolling
// accumulators of the skip channels' 27 taps), and when fine output plane o
// is complete adds the polyphase sum of the coarse tensor (parity p = 4 pi_i
// + 2 pi_j + pi_k, 8 coarse taps, k_upconv_poly's weights Wp[p][e][o][c]),
// the bias and the ReLU.  Wave w owns fine row j0 + w / 2 (pi_j = w / 2 mod
// 2) and the parity pi_k = w mod 2 of the block's 64 voxels (two tiles of 16
// voxels at stride 2), so its polyphase weights (two parities, pi_i = 0, 1)
// stay in registers beside the skip weights.  The fine planes sit in LDS
// de-interleaved by k parity (even voxels, then odd), so the stride-2 tiles
// read consecutive voxel slots; the coarse planes (4 rows x 34 voxels) sit
// in a ring of three slots, one staged every second step.  Each output is
// bias + skip sum + polyphase sum in the order of the two-kernel form
// (k_conv3_march into an FP32 scratch, then k_upconv_poly), and the same
// value.  PL even and 2 mod 3, so the main loop runs in rounds of six steps.
template <bool F32OUT, bool RELU>
__global__ __launch_bounds__(kMarchThreads) void k_updec_march(const uint16_t *__restrict__ skip, int skip_stride,
                                                               int skip_off, const uint16_t *__restrict__ coarse,
                                                               const uint16_t *__restrict__ wsub,
                                                               const uint16_t *__restrict__ wpoly,
                                                               const float *__restrict__ bias, void *__restrict__ out,
                                                               int out_stride, int out_off, int n, unsigned ntiles,
                                                               int PL)
{
    constexpr int SV = 24;                       // fine voxel stride (halfwords): 16 channels + pad
    constexpr int WV = 6 * 66;                   // fine voxel slots per plane
    constexpr int NCH = WV * 2, PER = (NCH + kMarchThreads - 1) / kMarchThreads;
    constexpr int SVC = 40;                      // coarse voxel stride: 32 channels + pad
    constexpr int WVC = 4 * 34;                  // coarse voxel slots per plane
    constexpr int NCHC = WVC * 4, PERC = (NCHC + kMarchThreads - 1) / kMarchThreads;
    __shared__ __align__(16) uint16_t ring[3 * WV * SV];
    __shared__ __align__(16) uint16_t cring[3 * WVC * SVC];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = w >> 1, pk = w & 1, pj = row & 1;
    const int r = lane & 15, q = lane >> 4;
    const int nc = n / 2;
    const int nkt = n / 64, nit = n / PL;
    const size_t plane_elems = (size_t)n * n * skip_stride;
    const size_t cplane_elems = (size_t)nc * nc * 32;
    const unsigned nb = gridDim.x;
    const unsigned lb = (nb % 8) ? blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    // skip weights [27][16][16]: chunk c of input plane offset e (tap di = 1 - e)
    bf16x8 bw[3][4];
    bf16x4 bt[3];
#pragma unroll
    for (int e = 0; e < 3; e++) {
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int kk = 32 * c + 8 * q, tap = (2 - e) * 9 + kk / 16, ch = kk % 16;
            bw[e][c] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(wsub + (tap * 16 + r) * 16 + ch));
        }
        const int tap = (2 - e) * 9 + 8;
        bt[e] = *(const bf16x4 *)(wsub + (tap * 16 + r) * 16 + 4 * q);
    }
    // polyphase weights of this wave's parities (pi_i = 0, 1)
    bf16x8 pw[2][8];
#pragma unroll
    for (int pi = 0; pi < 2; pi++)
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int p = 4 * pi + 2 * pj + pk;
            pw[pi][e] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(wpoly + ((p * 8 + e) * 16 + r) * 32 + 8 * q));
        }
    f32x4 bo;
#pragma unroll
    for (int e = 0; e < 4; e++)
        bo[e] = bias ? bias[4 * q + e] : 0.f;
    for (unsigned t = lb; t < ntiles; t += nb) {
        const int ib = (int)(t % nit), kt = (int)((t / nit) % nkt), jt = (int)(t / ((unsigned)nit * nkt));
        const int i0 = ib * PL, j0 = jt * 4, k0 = kt * 64;
        unsigned soff[PER], csoff[PERC];
        int loff[PER], cloff[PERC];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int c = threadIdx.x + u * kMarchThreads;
            const int cc = c < NCH ? c : 0;
            const int v = cc / 2, part = cc % 2;
            const int rw = v / 66, col = v % 66;
            const int jj = wrapi(j0 + rw - 1, n), kk = wrapi(k0 + col - 1, n);
            soff[u] = (unsigned)((jj * n + kk) * skip_stride + skip_off + 8 * part);
            loff[u] = (rw * 66 + (col & 1) * 33 + (col >> 1)) * SV + 8 * part;
        }
#pragma unroll
        for (int u = 0; u < PERC; u++) {
            const int c = threadIdx.x + u * kMarchThreads;
            const int cc = c < NCHC ? c : 0;
            const int v = cc / 4, part = cc % 4;
            const int rw = v / 34, col = v % 34;
            const int jj = wrapi(j0 / 2 + rw - 1, nc), kk = wrapi(k0 / 2 + col - 1, nc);
            csoff[u] = (unsigned)((jj * nc + kk) * 32 + 8 * part);
            cloff[u] = v * SVC + 8 * part;
        }
        u32x4 pre[PER], prec[PERC];
        auto fetch = [&](int ii) {
            const uint16_t *base = skip + (size_t)wrapi(ii, n) * plane_elems;
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kMarchThreads < NCH)
                    pre[u] = *(const u32x4 *)(base + soff[u]);
        };
        auto put = [&](int slot) {
            uint16_t *dst = ring + slot * WV * SV;
#pragma unroll
            for (int u = 0; u < PER; u++)
                if (threadIdx.x + u * kMarchThreads < NCH)
                    *(u32x4 *)(dst + loff[u]) = pre[u];
        };
        // coarse plane cp lives in slot (cp - (i0 / 2 - 1)) mod 3
        auto cslot = [&](int cp) { return (cp - i0 / 2 + 1) % 3; };
        auto cfetch = [&](int cp) {
            const uint16_t *base = coarse + (size_t)wrapi(cp, nc) * cplane_elems;
#pragma unroll
            for (int u = 0; u < PERC; u++)
                if (threadIdx.x + u * kMarchThreads < NCHC)
                    prec[u] = *(const u32x4 *)(base + csoff[u]);
        };
        auto cput = [&](int cp) {
            uint16_t *dst = cring + cslot(cp) * WVC * SVC;
#pragma unroll
            for (int u = 0; u < PERC; u++)
                if (threadIdx.x + u * kMarchThreads < NCHC)
                    *(u32x4 *)(dst + cloff[u]) = prec[u];
        };
        fetch(i0 - 1);
        put(0);
        fetch(i0);
        put(1);
        cfetch(i0 / 2 - 1);
        cput(i0 / 2 - 1);
        cfetch(i0 / 2);
        cput(i0 / 2);
        __syncthreads();
        f32x4 acc[3][2];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int m = 0; m < 2; m++)
                acc[a][m] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // fine output plane o (parity PI along i): polyphase sum, bias, skip sum, ReLU, store
        auto finish = [&](int o, auto PI, const f32x4 (&ac)[2]) {
            constexpr int pi = decltype(PI)::value;
            const int I = o >> 1;
            f32x4 ap[2] = {(f32x4){0.f, 0.f, 0.f, 0.f}, (f32x4){0.f, 0.f, 0.f, 0.f}};
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int oi = (e >> 2) - 1 + pi, oj = ((e >> 1) & 1) - 1 + pj, ok = (e & 1) - 1 + pk;
                const uint16_t *cs = cring + cslot(I + oi) * WVC * SVC;
                const int cb = (((row >> 1) + oj + 1) * 34 + r + ok + 1) * SVC + 8 * q;
#pragma unroll
                for (int m = 0; m < 2; m++) {
                    const bf16x8 b = __builtin_bit_cast(bf16x8, *(const u32x4 *)(cs + cb + 16 * m * SVC));
                    ap[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pw[pi][e], b, ap[m], 0, 0, 0);
                }
            }
            const int j = j0 + row;
#pragma unroll
            for (int m = 0; m < 2; m++) {
                const size_t vf = ((size_t)o * n + j) * n + k0 + 2 * (16 * m + r) + pk;
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    v[e] = ap[m][e] + bo[e] + ac[m][e];
                    if (RELU)
                        v[e] = fmaxf(v[e], 0.f);
                }
                const size_t oi_ = vf * out_stride + out_off + 4 * q;
                if constexpr (F32OUT)
                    *(f32x4 *)((float *)out + oi_) = (f32x4){v[0], v[1], v[2], v[3]};
                else
                    *(u16x4 *)((uint16_t *)out + oi_) = (u16x4){f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
            }
        };
        // input plane s in ring slot JM (also the accumulator slot of output
        // plane s - 1); LD: fine plane s + 2 still to stage; ST: output plane
        // s - 1 in the tile, of parity PI; CLD: coarse plane s / 2 + 1 to stage
        auto step = [&](int s, auto JM, auto LD, auto ST, auto PI, auto CLD) {
            constexpr int jm = decltype(JM)::value;
            if constexpr (decltype(LD)::value)
                fetch(s + 2);
            if constexpr (decltype(CLD)::value)
                cfetch(s / 2 + 1);
            const uint16_t *sl = ring + jm * WV * SV;
#pragma unroll
            for (int c = 0; c < 5; c++) {
                // K chunk c (c = 4: the last tap alone, 16 wide)
                const int kk = c < 4 ? 32 * c + 8 * q : 128 + 4 * q, tip = kk / 16, ch = kk % 16;
                const int dj = tip / 3 - 1, dk = tip % 3 - 1;
                const int kl = pk + 1 + dk;  // fine k offset (window slot) of lane r's voxel, less 2 (16 m + r)
                const int ab = ((1 + row + dj) * 66 + (kl & 1) * 33 + r + (kl >> 1)) * SV + ch;
#pragma unroll
                for (int m = 0; m < 2; m++) {
                    if (c < 4) {
                        const bf16x8 a = __builtin_bit_cast(bf16x8, *(const u32x4 *)(sl + ab + 16 * m * SV));
#pragma unroll
                        for (int e = 0; e < 3; e++)
                            acc[(jm + e) % 3][m] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[e][c < 4 ? c : 0], a, acc[(jm + e) % 3][m], 0, 0, 0);
                    } else {
                        const bf16x4 a = *(const bf16x4 *)(sl + ab + 16 * m * SV);
#pragma unroll
                        for (int e = 0; e < 3; e++)
                            acc[(jm + e) % 3][m] =
                                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bt[e], a, acc[(jm + e) % 3][m], 0, 0, 0);
                    }
                }
            }
            if constexpr (decltype(ST)::value) {
                // kept apart from the MFMAs around it, as in k_conv3_march
                __builtin_amdgcn_sched_barrier(0);
                finish(s - 1, PI, acc[jm]);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int m = 0; m < 2; m++)
                acc[jm][m] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if constexpr (decltype(LD)::value)
                put((jm + 2) % 3);
            if constexpr (decltype(CLD)::value)
                cput(s / 2 + 1);
            __syncthreads();
        };
        using I0 = IConst<0>;
        using I1 = IConst<1>;
        using I2 = IConst<2>;
        step(i0 - 1, I0(), I1(), I0(), I0(), I0());
        step(i0, I1(), I1(), I0(), I0(), I1());
        for (int s = i0 + 1; s < i0 + PL - 1; s += 6) {
            step(s, I2(), I1(), I1(), I0(), I0());
            step(s + 1, I0(), I1(), I1(), I1(), I1());
            step(s + 2, I1(), I1(), I1(), I0(), I0());
            step(s + 3, I2(), I1(), I1(), I1(), I1());
            step(s + 4, I0(), I1(), I1(), I0(), I0());
            step(s + 5, I1(), I1(), I1(), I1(), I1());
        }
        step(i0 + PL - 1, I2(), I0(), I1(), I0(), I0());
        step(i0 + PL, I0(), I0(), I1(), I1(), I0());
    }
}

// The fused decoder layer above: skip (n^3 x 16, view), coarse ((n/2)^3 x 32,
// compact), wsub [27][16][16] and wpoly [64][16][32] as packed by
// k_pack_conv_sub and k_pack_poly.  Returns false (nothing launched) for
// grids or views it does not handle.
bool launch_updec16(const uint16_t *skip, int skip_stride, int skip_off, const uint16_t *coarse, const uint16_t *wsub,
                    const uint16_t *wpoly, const float *bias, void *out, int out_stride, int out_off, bool out_f32,
                    bool relu, int n, hipStream_t st)
{
    if (n % 64 || skip_stride % 8 || skip_off % 8 || out_stride % 4 || out_off % 4 || out_f32 == relu)
        return false;
    const int PL = march_planes(n);
    const unsigned ntiles = (unsigned)(n / 4) * (n / 64) * (n / PL);
    unsigned nb = ntiles < 2048u ? ntiles : 2048u;
    if (nb >= 8)
        nb -= nb % 8;
#define PM_UPDEC(F, RL)                                                                                               \
    hipLaunchKernelGGL((k_updec_march<F, RL>), dim3(nb), dim3(kMarchThreads), 0, st, skip, skip_stride, skip_off,    \
                       coarse, wsub, wpoly, bias, out, out_stride, out_off, n, ntiles, PL)
    if (out_f32)
        PM_UPDEC(true, false);
    else
        PM_UPDEC(false, true);
#undef PM_UPDEC
    return true;
}

// Polyphase weights of k_upconv_poly from layer weights w[27][cin][cout]
// (FP32) restricted to input channels [0, cup): Wp[p][e][o][c] = sum of
// w[t][c][o] over the taps t whose coarse offset for parity p is e, in tap
// order, rounded once to BF16.
__device__ __forceinline__ void pack_poly(const float *__restrict__ w, int cin, int cout, int cup, int cout_pad,
                                          uint16_t *__restrict__ wp, int x0, int dx)
{
    const int total = 64 * cout_pad * cup;
    for (int x = x0; x < total; x += dx) {
        const int c = x % cup, o = (x / cup) % cout_pad, pe = x / (cup * cout_pad);
        const int p = pe >> 3, e = pe & 7;
        float s = 0.f;
        if (o < cout)
            for (int t = 0; t < 27; t++) {
                int di, dj, dk;
                tap_offsets(t, di, dj, dk);
                // coarse offset of tap d for parity pi: floor((pi + d) / 2), as e = that + 1 - pi
                const int ei = ((((p >> 2) + di + 2) >> 1) - 1) + 1 - (p >> 2);
                const int ej = (((((p >> 1) & 1) + dj + 2) >> 1) - 1) + 1 - ((p >> 1) & 1);
                const int ek = ((((p & 1) + dk + 2) >> 1) - 1) + 1 - (p & 1);
                if (ei == (e >> 2) && ej == ((e >> 1) & 1) && ek == (e & 1))
                    s += w[((size_t)t * cin + c) * cout + o];
            }
        wp[x] = f2bf(s);
    }
}
__global__ __launch_bounds__(256) void k_pack_poly(const float *__restrict__ w, int cin, int cout, int cup,
                                                   int cout_pad, uint16_t *__restrict__ wp)
{
    pack_poly(w, cin, cout, cup, cout_pad, wp, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

// Conv weights of input channels [c0, c0 + csub) of a layer, packed like
// k_pack_conv's forward layout ([27][cout_pad][csub_pad]).
__device__ __forceinline__ void pack_conv_sub(const float *__restrict__ w, int cin, int cout, int c0, int csub,
                                              int csub_pad, int cout_pad, uint16_t *__restrict__ wf, int x0, int dx)
{
    const int total = 27 * cout_pad * csub_pad;
    for (int x = x0; x < total; x += dx) {
        const int c = x % csub_pad, o = (x / csub_pad) % cout_pad, t = x / (csub_pad * cout_pad);
        const float v = (c < csub && o < cout) ? w[((size_t)t * cin + c0 + c) * cout + o] : 0.f;
        wf[x] = f2bf(v);
    }
}
__global__ __launch_bounds__(256) void k_pack_conv_sub(const float *__restrict__ w, int cin, int cout, int c0,
                                                       int csub, int csub_pad, int cout_pad, uint16_t *__restrict__ wf)
{
    pack_conv_sub(w, cin, cout, c0, csub, csub_pad, cout_pad, wf, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

void launch_pack_poly(const float *w, int cin, int cout, int cup, int cout_pad, uint16_t *wp, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_poly, dim3(128), dim3(256), 0, st, w, cin, cout, cup, cout_pad, wp);
}

void launch_pack_conv_sub(const float *w, int cin, int cout, int c0, int csub, int csub_pad, int cout_pad,
                          uint16_t *wf, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_conv_sub, dim3(128), dim3(256), 0, st, w, cin, cout, c0, csub, csub_pad, cout_pad, wf);
}

// Returns false (nothing launched) for channel counts without an instance.
bool launch_upconv_poly(const uint16_t *in, int cup, int nc, const uint16_t *wp, int cout_pad, const float *bias,
                        const float *add, int cout, void *out, int out_stride, int out_off, bool out_f32, bool relu,
                        hipStream_t st)
{
    // the two forms in use: BF16 activation with ReLU (inference) and FP32
    // without (the layer on its own); whole channel groups, 4-aligned views
    if (nc % 64 || cout != cout_pad || out_stride % 4 || out_off % 4 || out_f32 == relu)
        return false;
#define PM_UPCONV(CI, C, KTV, F, RL, NT)                                                                                \
    hipLaunchKernelGGL((k_upconv_poly<CI, C, KTV, F, RL>), dim3(xcd_blocks(NT), 1), dim3(256), 0, st, in, nc, wp,     \
                       cout_pad, bias, add, out, out_stride, out_off, NT)
    if (cup == 32 && cout_pad == 16) {
        const unsigned ntiles = (unsigned)nc * (nc / 4) * (nc / 32);
        if (out_f32)
            PM_UPCONV(32, 1, 32, true, false, ntiles);
        else
            PM_UPCONV(32, 1, 32, false, true, ntiles);
        return true;
    }
    if (cup == 64 && cout_pad == 32) {
        const unsigned ntiles = (unsigned)nc * (nc / 4) * (nc / 16);
        if (out_f32)
            PM_UPCONV(64, 2, 16, true, false, ntiles);
        else
            PM_UPCONV(64, 2, 16, false, true, ntiles);
        return true;
    }
#undef PM_UPCONV
    return false;
}


// 16 -> 16 convolution with ReLU followed by the 1x1x1 head (yhat, FP32,
// natural order); false when the grid has no plane-marching instance.
bool launch_conv3_head(const uint16_t *in, int in_stride, int in_off, const uint16_t *wp, const float *bias,
                       const float *hw, const float *hb, float *yhat, int n, hipStream_t st)
{
    if (n % 64 || in_stride % 8 || in_off % 8)
        return false;
    const int PL = march_planes(n);
    const unsigned ntiles = (unsigned)(n / 4) * (n / 64) * (n / PL);
    unsigned nb = ntiles < 2048u ? ntiles : 2048u;
    if (nb >= 8)
        nb -= nb % 8;
    hipLaunchKernelGGL((k_conv3_march<1, 1, true>), dim3(nb, 1), dim3(kMarchThreads), 0, st, in, in_stride,
                       in_off, wp, 16, bias, 16, (void *)yhat, 1, 0, 1, n, 0, 1, ntiles, PL, hw, hb);
    return true;
}

void launch_conv3(const uint16_t *in, int in_stride, int in_off, int cin_pad, const uint16_t *wp, int cout_pad,
                  const float *bias, int cout, void *out, int out_stride, int out_off, bool out_f32, int n, bool flip,
                  bool relu, hipStream_t st)
{
    if (n % 64 == 0 && cin_pad <= 48 && in_stride % 8 == 0 && in_off % 8 == 0) {
        const int PL = march_planes(n);
        const unsigned ntiles = (unsigned)(n / 4) * (n / 64) * (n / PL);
        unsigned nb = ntiles < 2048u ? ntiles : 2048u;
        if (nb >= 8)
            nb -= nb % 8;
        dim3 grid(nb, cout_pad / 16);
#define PM_CONVM(CSV, C)                                                                                              \
    hipLaunchKernelGGL((k_conv3_march<CSV, C>), grid, dim3(kMarchThreads), 0, st, in, in_stride, in_off, wp, cout_pad, \
                       bias, cout, out, out_stride, out_off, out_f32 ? 1 : 0, n, flip ? 1 : 0, relu ? 1 : 0, ntiles,   \
                       PL, nullptr, nullptr)
        if (cin_pad == 16)
            PM_CONVM(1, 1);
        else if (cin_pad == 32)
            PM_CONVM(2, 1);
        else
            PM_CONVM(3, 1);
#undef PM_CONVM
        return;
    }
    if (n % kCvK == 0 && in_stride % 4 == 0 && in_off % 4 == 0) {
        // two rows per wave (8-row tiles)
        const unsigned ntiles = (unsigned)n * (n / 8) * (n / kCvK);
        const int tiles = cout_pad / 16;
        const int cot = tiles % 4 == 0 ? 4 : (tiles % 3 == 0 ? 3 : (tiles % 2 == 0 ? 2 : 1));
        dim3 grid(xcd_blocks(ntiles), cout_pad / (cot * 16));
#define PM_CONVL(C)                                                                                                    \
    hipLaunchKernelGGL((k_conv3_lds<C, 2>), grid, dim3(256), 0, st, in, in_stride, in_off, cin_pad, wp, cout_pad,      \
                       bias, cout, out, out_stride, out_off, out_f32 ? 1 : 0, n, flip ? 1 : 0, relu ? 1 : 0, ntiles)
        if (cot == 4)
            PM_CONVL(4);
        else if (cot == 3)
            PM_CONVL(3);
        else if (cot == 2)
            PM_CONVL(2);
        else
            PM_CONVL(1);
#undef PM_CONVL
        return;
    }
    if (n % 64 == 0)
        launch_conv3_mt<4>(in, in_stride, in_off, cin_pad, wp, cout_pad, bias, cout, out, out_stride, out_off,
                           out_f32, n, flip, relu, st);
    else if (n % 32 == 0)
        launch_conv3_mt<2>(in, in_stride, in_off, cin_pad, wp, cout_pad, bias, cout, out, out_stride, out_off,
                           out_f32, n, flip, relu, st);
    else
        launch_conv3_mt<1>(in, in_stride, in_off, cin_pad, wp, cout_pad, bias, cout, out, out_stride, out_off,
                           out_f32, n, flip, relu, st);
}

// Weight and bias gradients:
//   dW[t][c][o] = sum_v x[v + d_t][x_off + c] dy[v][dy_off + o],  db[o] = sum_v dy[v][dy_off + o].
// GEMMs with the voxels as the reduction index on v_mfma_f32_16x16x16_bf16:
// A[m = c][k = voxel] from x, B[k = voxel][n = o] from dy, D[c][o].  A block
// owns one (16-channel c tile, 16-channel o tile) pair and a contiguous range
// of units; a unit is a row segment (SEG = min(64, n) voxels along k of row
// j) marched over PLW planes i.  The block keeps rows j - 1 .. j + 1 of
// planes i - 1 .. i + 2 of x (SEG + 2 voxels: the k halo) in a four-slot LDS
// ring and the dy segment of plane i in a two-slot one, voxel-major with a
// padded voxel stride; per plane it stages only the new plane's three rows,
// whose loads were issued before the previous plane was computed.  Wave w
// (nine per block) owns the neighbour row (di, dj) = (w / 3 - 1, w % 3 - 1)
// and its three taps 3w .. 3w + 2: a lane reads six consecutive voxels of
// one channel once and forms the A operands of the three k offsets from
// them.  Every block writes its partial sums; k_wgrad_reduce adds them in
// block order, so the gradients do not depend on scheduling.  vec: the views
// allow 16-byte loads of 16-channel tiles (strides and offsets multiples of
// 8, padded channel counts within the strides), else 2-byte loads.
constexpr int kWgBlocks = 240;
constexpr int kWgThreads = 576;  // nine waves
constexpr int kWgSeg = 64;       // voxels per row segment (n if smaller)
constexpr int kWgPlanes = 16;    // planes per unit (n if smaller)
constexpr int kWgVS = 24;        // LDS voxel stride in halfwords (16 channels + pad)
constexpr int kWgXW = kWgSeg + 2;
constexpr int kWgSlotX = 3 * kWgXW * kWgVS;  // one plane: three rows
constexpr int kWgSlotD = kWgSeg * kWgVS;

__host__ __device__ __forceinline__ int wgrad_seg(int n) { return n < kWgSeg ? n : kWgSeg; }
__host__ __device__ __forceinline__ int wgrad_planes(int n) { return n < kWgPlanes ? n : kWgPlanes; }

static inline unsigned wgrad_blocks(int n)
{
    const unsigned units = (unsigned)(n / wgrad_planes(n)) * n * (unsigned)(n / wgrad_seg(n));
    return units < (unsigned)kWgBlocks ? (units ? units : 1) : (unsigned)kWgBlocks;
}

size_t wgrad_partial_floats(int cin, int cout) { return (size_t)kWgBlocks * (27 * (size_t)cin * cout + cout); }

__global__ __launch_bounds__(kWgThreads) void k_conv3_wgrad(const uint16_t *__restrict__ x, int x_stride, int x_off,
                                                            int cin, const uint16_t *__restrict__ dy, int dy_stride,
                                                            int dy_off, int cout, float *__restrict__ part, int n,
                                                            int vec)
{
    __shared__ __align__(16) uint16_t lds[4 * kWgSlotX + 2 * kWgSlotD];
    uint16_t *const xr = lds, *const dr = lds + 4 * kWgSlotX;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int otiles = (cout + 15) / 16;
    const int ct = blockIdx.y / otiles, ot = blockIdx.y - (blockIdx.y / otiles) * otiles;
    const int c0 = ct * 16, o0 = ot * 16;
    const int seg = wgrad_seg(n), pl = wgrad_planes(n), nsr = n / seg, nkc = seg / 16;
    const int nxc = 3 * (seg + 2) * 2, nch = nxc + seg * 2;  // 16-byte chunks per plane step
    const unsigned units = (unsigned)(n / pl) * n * (unsigned)nsr;
    const unsigned u0 = (unsigned)(((unsigned long long)blockIdx.x * units) / gridDim.x);
    const unsigned u1 = (unsigned)(((unsigned long long)(blockIdx.x + 1) * units) / gridDim.x);
    // this thread's chunk of a plane step (one at most: nch <= 3 * 66 * 2 + 128 < 576):
    // an x row (dj) and voxel, or a dy voxel; first channel; LDS offset in its slot
    const int e = threadIdx.x;
    const bool isx = e < nxc, has = e < nch;
    int c_dj = 0, c_vx = 0, c_ch = 0, c_off = 0;
    if (isx) {
        const int rw = e / ((seg + 2) * 2), rem = e - rw * (seg + 2) * 2;
        c_dj = rw - 1;
        c_vx = (rem >> 1) - 1;
        c_ch = c0 + 8 * (rem & 1);
        c_off = (rw * kWgXW + (rem >> 1)) * kWgVS + 8 * (rem & 1);
    } else if (has) {
        const int rem = e - nxc;
        c_vx = rem >> 1;
        c_ch = o0 + 8 * (rem & 1);
        c_off = (rem >> 1) * kWgVS + 8 * (rem & 1);
    }
    const int lim = isx ? cin : cout;
    const bool ok = has && c_ch < lim, full = c_ch + 8 <= lim;
    // chunk of plane II (x rows j - 1 .. j + 1) or of dy row (II, j), segment k0
    auto fetch = [&](int II, int j, int k0, bool want_x, bool want_d) -> u32x4 {
        u32x4 v = {0u, 0u, 0u, 0u};
        if (!ok || (isx ? !want_x : !want_d))
            return v;
        const uint16_t *src;
        if (isx) {
            const int ii = wrapi(II, n), jj = wrapi(j + c_dj, n), kk = wrapi(k0 + c_vx, n);
            src = x + ((size_t)((ii * n + jj) * n + kk)) * x_stride + x_off + c_ch;
        } else {
            src = dy + ((size_t)((II * n + j) * n + k0 + c_vx)) * dy_stride + dy_off + c_ch;
        }
        if (vec) {
            v = *(const u32x4 *)src;
            if (!full)
#pragma unroll
                for (int h = 0; h < 4; h++) {
                    const unsigned lo = c_ch + 2 * h < lim ? 0xffffu : 0u;
                    const unsigned hi = c_ch + 2 * h + 1 < lim ? 0xffff0000u : 0u;
                    v[h] &= lo | hi;
                }
        } else {
#pragma unroll
            for (int h = 0; h < 4; h++) {
                const unsigned lo = c_ch + 2 * h < lim ? src[2 * h] : 0u;
                const unsigned hi = c_ch + 2 * h + 1 < lim ? src[2 * h + 1] : 0u;
                v[h] = lo | (hi << 16);
            }
        }
        return v;
    };
    const int di = wave / 3 - 1, dj = wave % 3 - 1;
    f32x4 acc[3];
#pragma unroll
    for (int d = 0; d < 3; d++)
        acc[d] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (unsigned un = u0; un < u1; un++) {
        const unsigned col = un / (unsigned)(n / pl);  // (j, segment): planes fastest
        const int i0 = (int)(un - col * (unsigned)(n / pl)) * pl;
        const int j = (int)(col / (unsigned)nsr), k0 = (int)(col - (col / (unsigned)nsr) * (unsigned)nsr) * seg;
        // prime: x planes i0 - 1, i0, i0 + 1 into slots 0, 1, 2; dy of plane i0 into slot 0
        __syncthreads();  // the previous unit's operands have been read
        if (isx) {
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const u32x4 v = fetch(i0 - 1 + d, j, k0, true, false);
                if (has)
                    *(u32x4 *)(xr + d * kWgSlotX + c_off) = v;
            }
        } else if (has) {
            *(u32x4 *)(dr + c_off) = fetch(i0, j, k0, false, true);
        }
        // next loads: x plane i0 + 2, dy of plane i0 + 1 (rows within the unit's planes)
        u32x4 pre = isx ? fetch(i0 + 2, j, k0, true, false)
                        : (pl > 1 ? fetch(i0 + 1, j, k0, false, true) : (u32x4){0u, 0u, 0u, 0u});
        __syncthreads();
        for (int p = 0; p < pl; p++) {
            const int i = i0 + p;
            // operands of this plane: dy segment (B, all taps), then the wave's x row
            const uint16_t *dseg = dr + (p & 1) * kWgSlotD;
            const uint16_t *xrow = xr + ((p + 1 + di) & 3) * kWgSlotX + (dj + 1) * kWgXW * kWgVS;
#pragma unroll
            for (int kc = 0; kc < kWgSeg / 16; kc++)
                if (kc < nkc) {
                    bf16x4 b;
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        b[u] = (short)dseg[(16 * kc + 4 * q + u) * kWgVS + r];
                    if (wave == 0)
#pragma unroll
                        for (int u = 0; u < 4; u++)
                            bsum += bf2f((uint16_t)b[u]);
                    short xv[6];  // window voxels 16 kc + 4q .. + 5 (offsets -1 .. 4), channel r
#pragma unroll
                    for (int u = 0; u < 6; u++)
                        xv[u] = (short)xrow[(16 * kc + 4 * q + u) * kWgVS + r];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        const bf16x4 a = (bf16x4){xv[d], xv[d + 1], xv[d + 2], xv[d + 3]};
                        acc[d] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[d], 0, 0, 0);
                    }
                }
            if (p + 1 < pl) {
                // plane i + 2 into the x slot of plane i - 2, dy of plane i + 1 into the other dy slot
                // (both last read before the previous barrier)
                if (has)
                    *(u32x4 *)((isx ? xr + ((p + 3) & 3) * kWgSlotX : dr + ((p + 1) & 1) * kWgSlotD) + c_off) = pre;
                if (p + 2 < pl)
                    pre = isx ? fetch(i + 3, j, k0, true, false) : fetch(i + 2, j, k0, false, true);
            }
            __syncthreads();
        }
    }
    // lane (r, q) holds dW[3 wave + d][c0 + 4q + e][o0 + r]
    float *pb = part + (size_t)blockIdx.x * (27 * (size_t)cin * cout + cout);
    const int o = o0 + r;
    if (o < cout)
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int e4 = 0; e4 < 4; e4++) {
                const int c = c0 + 4 * q + e4;
                if (c < cin)
                    pb[((size_t)(3 * wave + d) * cin + c) * cout + o] = acc[d][e4];
            }
    // bias: wave 0, lanes r, r + 16, r + 32, r + 48 hold partial sums of o0 + r
    if (ct == 0 && wave == 0) {
        bsum += __shfl_down(bsum, 32, 64);
        bsum += __shfl_down(bsum, 16, 64);
        if (lane < 16 && o < cout)
            pb[27 * (size_t)cin * cout + o] = bsum;
    }
}

// dw[e] = sum_b part[b][e] (e over 27 cin cout), db[o] = sum_b part[b][27 cin cout + o]
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part, unsigned nb, int cin, int cout,
                                                      float *__restrict__ dw, float *__restrict__ db)
{
    const size_t nw = 27 * (size_t)cin * cout, stride = nw + cout;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < stride; e += (size_t)gridDim.x * 256) {
        float s = 0.f;
#pragma unroll 16
        for (unsigned b = 0; b < nb; b++)
            s += part[(size_t)b * stride + e];
        if (e < nw)
            dw[e] = s;
        else if (db)
            db[e - nw] = s;
    }
}

void launch_conv3_wgrad(const uint16_t *x, int x_stride, int x_off, int cin, const uint16_t *dy, int dy_stride,
                        int dy_off, int cout, float *dw, float *db, float *part, int n, hipStream_t st)
{
    const unsigned nb = wgrad_blocks(n);
    dim3 grid(nb, ((cin + 15) / 16) * ((cout + 15) / 16));
    const int vec = x_stride % 8 == 0 && x_off % 8 == 0 && x_off + (cin + 15) / 16 * 16 <= x_stride &&
                    dy_stride % 8 == 0 && dy_off % 8 == 0 && dy_off + (cout + 15) / 16 * 16 <= dy_stride;
    hipLaunchKernelGGL(k_conv3_wgrad, grid, dim3(kWgThreads), 0, st, x, x_stride, x_off, cin, dy, dy_stride, dy_off,
                       cout, part, n, vec);
    const size_t total = 27 * (size_t)cin * cout + cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, nb, cin, cout,
                       dw, db);
}

// ---------------------------------------------------------------- elementwise
// dy[v][off + c] *= (y[v][y_off + c] > 0)
__global__ __launch_bounds__(256) void k_relu_bwd(uint16_t *__restrict__ dy, int dstride, int doff,
                                                  const uint16_t *__restrict__ y, int ystride, int yoff, int C,
                                                  unsigned nvox)
{
    const unsigned total = nvox * (unsigned)C;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / C;
        const int c = (int)(e - v * C);
        if (!(bf2f(y[(size_t)v * ystride + yoff + c]) > 0.f))
            dy[(size_t)v * dstride + doff + c] = 0;
    }
}

void launch_relu_bwd(uint16_t *dy, int dstride, int doff, const uint16_t *y, int ystride, int yoff, int C,
                     unsigned nvox, hipStream_t st)
{
    hipLaunchKernelGGL(k_relu_bwd, dim3(2048), dim3(256), 0, st, dy, dstride, doff, y, ystride, yoff, C, nvox);
}

// 2x2x2 average pooling: out (n/2)^3 x C from in n^3 (slice in_off..)
__global__ __launch_bounds__(256) void k_pool(const uint16_t *__restrict__ in, int istride, int ioff,
                                              uint16_t *__restrict__ out, int ostride, int ooff, int C, int nc)
{
    const unsigned total = (unsigned)nc * nc * nc * C;
    const int nf = 2 * nc;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / C;
        const int c = (int)(e - v * C);
        const int K = (int)(v % nc), J = (int)((v / nc) % nc), I = (int)(v / ((unsigned)nc * nc));
        float s = 0.f;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int d = 0; d < 2; d++)
                    s += bf2f(in[((size_t)((2 * I + a) * nf + 2 * J + b) * nf + 2 * K + d) * istride + ioff + c]);
        out[(size_t)v * ostride + ooff + c] = f2bf(0.125f * s);
    }
}

// d_in[child] += d_out[parent] / 8 (accumulating into the existing gradient)
__global__ __launch_bounds__(256) void k_pool_bwd(const uint16_t *__restrict__ dout, int ostride, int ooff,
                                                  uint16_t *__restrict__ din, int istride, int ioff, int C, int nf)
{
    const unsigned total = (unsigned)nf * nf * nf * C;
    const int nc = nf / 2;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / C;
        const int c = (int)(e - v * C);
        const int k = (int)(v % nf), j = (int)((v / nf) % nf), i = (int)(v / ((unsigned)nf * nf));
        const size_t p = (size_t)((i / 2) * nc + j / 2) * nc + k / 2;
        const size_t di = (size_t)v * istride + ioff + c;
        din[di] = f2bf(bf2f(din[di]) + 0.125f * bf2f(dout[p * ostride + ooff + c]));
    }
}

// nearest-neighbour upsampling into a slice: out[child][ooff + c] = in[parent][c]
__global__ __launch_bounds__(256) void k_up(const uint16_t *__restrict__ in, int istride, int ioff,
                                            uint16_t *__restrict__ out, int ostride, int ooff, int C, int nf)
{
    const unsigned total = (unsigned)nf * nf * nf * C;
    const int nc = nf / 2;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / C;
        const int c = (int)(e - v * C);
        const int k = (int)(v % nf), j = (int)((v / nf) % nf), i = (int)(v / ((unsigned)nf * nf));
        const size_t p = (size_t)((i / 2) * nc + j / 2) * nc + k / 2;
        out[(size_t)v * ostride + ooff + c] = in[p * istride + ioff + c];
    }
}

// d_in[parent][c] = sum over children of d_out[child][ooff + c]
__global__ __launch_bounds__(256) void k_up_bwd(const uint16_t *__restrict__ dout, int ostride, int ooff,
                                                uint16_t *__restrict__ din, int istride, int ioff, int C, int nc)
{
    const unsigned total = (unsigned)nc * nc * nc * C;
    const int nf = 2 * nc;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / C;
        const int c = (int)(e - v * C);
        const int K = (int)(v % nc), J = (int)((v / nc) % nc), I = (int)(v / ((unsigned)nc * nc));
        float s = 0.f;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int d = 0; d < 2; d++)
                    s += bf2f(dout[((size_t)((2 * I + a) * nf + 2 * J + b) * nf + 2 * K + d) * ostride + ooff + c]);
        din[(size_t)v * istride + ioff + c] = f2bf(s);
    }
}

// The same two maps, 8 channels (16 bytes) per thread, for 8-aligned views;
// thread e covers voxel e / (C / 8), channels 8 (e % (C / 8)) .. + 7.
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_pool8(const uint16_t *__restrict__ in, int istride, int ioff,
                                               uint16_t *__restrict__ out, int ostride, int ooff, int C, int nc)
{
    const int G = C / 8;
    const unsigned total = (unsigned)nc * nc * nc * G;
    const int nf = 2 * nc;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / G;
        const int c = 8 * (int)(e - v * G);
        const int K = (int)(v % nc), J = (int)((v / nc) % nc), I = (int)(v / ((unsigned)nc * nc));
        float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int d = 0; d < 2; d++) {
                    const u16x8 x = *(const u16x8 *)(in + ((size_t)((2 * I + a) * nf + 2 * J + b) * nf + 2 * K + d) *
                                                              istride +
                                                      ioff + c);
#pragma unroll
                    for (int h = 0; h < 8; h++)
                        sum[h] += bf2f(x[h]);
                }
        u16x8 y;
#pragma unroll
        for (int h = 0; h < 8; h++)
            y[h] = f2bf(0.125f * sum[h]);
        *(u16x8 *)(out + (size_t)v * ostride + ooff + c) = y;
    }
}

__global__ __launch_bounds__(256) void k_up8(const uint16_t *__restrict__ in, int istride, int ioff,
                                             uint16_t *__restrict__ out, int ostride, int ooff, int C, int nf)
{
    const int G = C / 8;
    const unsigned total = (unsigned)nf * nf * nf * G;
    const int nc = nf / 2;
    for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const unsigned v = e / G;
        const int c = 8 * (int)(e - v * G);
        const int k = (int)(v % nf), j = (int)((v / nf) % nf), i = (int)(v / ((unsigned)nf * nf));
        const size_t p = (size_t)((i / 2) * nc + j / 2) * nc + k / 2;
        *(u16x8 *)(out + (size_t)v * ostride + ooff + c) = *(const u16x8 *)(in + p * istride + ioff + c);
    }
}

static inline bool aligned8(int C, int s1, int o1, int s2, int o2)
{
    return C % 8 == 0 && s1 % 8 == 0 && o1 % 8 == 0 && s2 % 8 == 0 && o2 % 8 == 0;
}

void launch_pool(const uint16_t *in, int istride, int ioff, uint16_t *out, int ostride, int ooff, int C, int nc,
                 hipStream_t st)
{
    if (aligned8(C, istride, ioff, ostride, ooff))
        hipLaunchKernelGGL(k_pool8, dim3(4096), dim3(256), 0, st, in, istride, ioff, out, ostride, ooff, C, nc);
    else
        hipLaunchKernelGGL(k_pool, dim3(2048), dim3(256), 0, st, in, istride, ioff, out, ostride, ooff, C, nc);
}
void launch_pool_bwd(const uint16_t *dout, int ostride, int ooff, uint16_t *din, int istride, int ioff, int C, int nf,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_bwd, dim3(2048), dim3(256), 0, st, dout, ostride, ooff, din, istride, ioff, C, nf);
}
void launch_up(const uint16_t *in, int istride, int ioff, uint16_t *out, int ostride, int ooff, int C, int nf,
               hipStream_t st)
{
    if (aligned8(C, istride, ioff, ostride, ooff))
        hipLaunchKernelGGL(k_up8, dim3(4096), dim3(256), 0, st, in, istride, ioff, out, ostride, ooff, C, nf);
    else
        hipLaunchKernelGGL(k_up, dim3(2048), dim3(256), 0, st, in, istride, ioff, out, ostride, ooff, C, nf);
}
void launch_up_bwd(const uint16_t *dout, int ostride, int ooff, uint16_t *din, int istride, int ioff, int C, int nc,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_up_bwd, dim3(2048), dim3(256), 0, st, dout, ostride, ooff, din, istride, ioff, C, nc);
}

// ---------------------------------------------------------------- input / head
// The density contrast comes in the solver's packed red-black layout: voxel
// (i, j, k) of colour c = (i + j + k) & 1 sits at c * n^3/2 + (i n + j) n/2 + k/2.
__device__ __forceinline__ unsigned packed_index(unsigned v, int n)
{
    const int k = (int)(v % (unsigned)n);
    const unsigned row = v / (unsigned)n;  // i * n + j
    const int ij = (int)(row / (unsigned)n) + (int)(row % (unsigned)n);
    const unsigned half = (unsigned)n * n * (n / 2);
    return ((ij + k) & 1) * half + row * (unsigned)(n / 2) + (unsigned)(k >> 1);
}

__device__ __forceinline__ double feature_of(double delta) { return log(fmax(1.0 + delta, 0.0) + 1e-3); }

// partial sums of l = ln(1 + delta + 1e-3) and l^2
__global__ __launch_bounds__(kBlock) void k_feature_stats(const double *__restrict__ delta, ReduceSlot rs, Span sp)
{
    double acc[2] = {0.0, 0.0};
    PM_SPAN_LOOP(e, sp)
    {
        const double l = feature_of(delta[e]);
        acc[0] += l;
        acc[1] += l * l;
    }
    block_partials<2>(acc, rs, sp);
}

void launch_feature_stats(const double *delta_packed, unsigned long long n3, ReduceSlot rs, hipStream_t st)
{
    const Span sp = make_span(n3);
    hipLaunchKernelGGL(k_feature_stats, dim3(sp.nblocks), dim3(kBlock), 0, st, delta_packed, rs, sp);
    launch_finalize(rs, sp, 2, rs.out, st);
}

// x0[v][0..15] = (standardised l, alpha_B0, alpha_M0, a, 0 ...), natural voxel order
__global__ __launch_bounds__(256) void k_unet_input(const double *__restrict__ delta, int n,
                                                    const double *__restrict__ stats, float ab0, float am0, float a,
                                                    uint16_t *__restrict__ x0)
{
    const unsigned nvox = (unsigned)n * n * n;
    const double mean = stats[0] / nvox;
    const double var = fmax(stats[1] / nvox - mean * mean, 1e-30);
    const double inv = 1.0 / sqrt(var);
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256) {
        const float l = (float)((feature_of(delta[packed_index(v, n)]) - mean) * inv);
        uint16_t *o = x0 + (size_t)v * 16;
        o[0] = f2bf(l);
        o[1] = f2bf(ab0);
        o[2] = f2bf(am0);
        o[3] = f2bf(a);
        for (int c = 4; c < 16; c++)
            o[c] = 0;
    }
}

void launch_unet_input(const double *delta_packed, int n, const double *stats, float ab0, float am0, float a,
                       uint16_t *x0, hipStream_t st)
{
    hipLaunchKernelGGL(k_unet_input, dim3(2048), dim3(256), 0, st, delta_packed, n, stats, ab0, am0, a, x0);
}

// Inference input: the density channel alone, f[v] = bf16(standardised
// feature), natural order; the three broadcast channels enter the first
// layer as a constant (k_conv3_in1).
__global__ __launch_bounds__(256) void k_unet_feature(const double *__restrict__ delta, int n,
                                                      const double *__restrict__ stats, uint16_t *__restrict__ f)
{
    const unsigned nvox = (unsigned)n * n * n;
    const double mean = stats[0] / nvox;
    const double var = fmax(stats[1] / nvox - mean * mean, 1e-30);
    const double inv = 1.0 / sqrt(var);
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256)
        f[v] = f2bf((float)((feature_of(delta[packed_index(v, n)]) - mean) * inv));
}

void launch_unet_feature(const double *delta_packed, int n, const double *stats, uint16_t *f, hipStream_t st)
{
    hipLaunchKernelGGL(k_unet_feature, dim3(2048), dim3(256), 0, st, delta_packed, n, stats, f);
}

// First layer at inference (4 -> 16 channels, ReLU).  Channels 1..3 of its
// input are the same value at every voxel and the padding is periodic, so
// their taps add a per-channel constant: out[v][o] = relu(b'[o] + sum_t
// f[v + d_t] W[t][0][o]) with b'[o] = b[o] + sum_{t, c >= 1} bf16(x_c)
// bf16(W[t][c][o]) (the operands the general convolution would multiply).
// The remaining single-channel convolution is one 16x16x32 MFMA per 16
// voxels: A[m = o][k = tap] the weights (taps 27..31 zero), B[k = tap][n =
// voxel] gathered from LDS, so the result D[o][v] gives each lane four
// consecutive channels of one voxel (one 8-byte store; 16 bytes with F32
// output, no ReLU: the test form).  Block: 4 waves, one row j each, 64
// voxels along k, marching PL planes along i with planes i - 1 .. i + 2 of
// the 6 x 66 window in a ring of four slots; the loads run four planes ahead
// through a register queue (a plane costs only four MFMAs per wave, far less
// than a load's latency).  w: FP32 weights w[t][c][o] of the 4-channel
// layer.
template <bool F32>
__global__ __launch_bounds__(256) void k_conv3_in1(const uint16_t *__restrict__ f, const float *__restrict__ w,
                                                   const float *__restrict__ b, float x1, float x2, float x3,
                                                   void *__restrict__ out, int out_stride, int out_off, int n, int PL)
{
    constexpr int RW = 66, PW = 6 * RW;  // window plane: 6 rows x 66 voxels
    __shared__ uint16_t ring[4 * PW];
    __shared__ float part[27 * 16];
    __shared__ float beff[16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const unsigned nkt = (unsigned)(n / 64), nit = (unsigned)(n / PL);
    const unsigned tile = xcd_block(0);
    const int ib = (int)(tile % nit), kt = (int)((tile / nit) % nkt), jt = (int)(tile / (nit * nkt));
    const int i0 = ib * PL, j0 = jt * 4, k0 = kt * 64;
    // the broadcast channels' constant: 27 x 16 partial sums, then per channel
    {
        const float xb1 = bf2f(f2bf(x1)), xb2 = bf2f(f2bf(x2)), xb3 = bf2f(f2bf(x3));
        for (int x = threadIdx.x; x < 27 * 16; x += 256) {
            const float *wt = w + (size_t)(x >> 4) * 64 + (x & 15);
            part[x] = xb1 * bf2f(f2bf(wt[16])) + xb2 * bf2f(f2bf(wt[32])) + xb3 * bf2f(f2bf(wt[48]));
        }
    }
    // this thread's window elements (two at most: 396 per plane)
    unsigned soff[2];
    int loff[2];
    bool has[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const int e = threadIdx.x + 256 * u;
        has[u] = e < PW;
        const int ee = has[u] ? e : 0, row = ee / RW, col = ee - row * RW;
        soff[u] = (unsigned)(wrapi(j0 + row - 1, n) * n + wrapi(k0 + col - 1, n));
        loff[u] = ee;
    }
    // pre[d]: plane i + 2 + d of the current plane i (a queue of four)
    uint16_t pre[4][2];
    const size_t plane = (size_t)n * n;
#define PM_IN1_FETCH(D, II)                                                                                            \
    do {                                                                                                               \
        const uint16_t *src_ = f + (size_t)wrapi((II), n) * plane;                                                     \
        _Pragma("unroll") for (int u = 0; u < 2; u++) if (has[u]) pre[D][u] = src_[soff[u]];                          \
    } while (0)
#define PM_IN1_STORE(D, SLOT)                                                                                          \
    do {                                                                                                               \
        _Pragma("unroll") for (int u = 0; u < 2; u++) if (has[u]) ring[(SLOT) * PW + loff[u]] = pre[D][u];           \
    } while (0)
    PM_IN1_FETCH(0, i0 - 1);
    PM_IN1_STORE(0, 0);
    PM_IN1_FETCH(0, i0);
    PM_IN1_STORE(0, 1);
    PM_IN1_FETCH(0, i0 + 1);
    PM_IN1_STORE(0, 2);
    PM_IN1_FETCH(0, i0 + 2);
    PM_IN1_FETCH(1, i0 + 3);
    PM_IN1_FETCH(2, i0 + 4);
    // A: lane (r, q) holds W[t][0][r] for the taps t = 8q .. 8q + 7; the B
    // gather of voxel r reads window row 1 + wave + dj, column 1 + dk + r
    bf16x8 a;
    int roff[8], dio[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const int t = 8 * q + u;
        int di, dj, dk;
        tap_offsets(t < 27 ? t : 13, di, dj, dk);
        a[u] = t < 27 ? __builtin_bit_cast(__bf16, f2bf(w[(size_t)t * 64 + r])) : __builtin_bit_cast(__bf16, (uint16_t)0);
        roff[u] = t < 27 ? (1 + wave + dj) * RW + 1 + dk : -1;
        dio[u] = di;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float sb = b[threadIdx.x];
        for (int t = 0; t < 27; t++)
            sb += part[t * 16 + threadIdx.x];
        beff[threadIdx.x] = sb;
    }
    __syncthreads();
    const float bq[4] = {beff[4 * q], beff[4 * q + 1], beff[4 * q + 2], beff[4 * q + 3]};
    for (int p = 0; p < PL; p++) {
        const int i = i0 + p;
        if (p + 4 < PL)
            PM_IN1_FETCH(3, i + 5);
        int toff[8];
#pragma unroll
        for (int u = 0; u < 8; u++)
            toff[u] = roff[u] >= 0 ? ((p + 1 + dio[u]) & 3) * PW + roff[u] : -1;
        const size_t vrow = ((size_t)i * n + j0 + wave) * n + k0;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            bf16x8 bv;
#pragma unroll
            for (int u = 0; u < 8; u++)
                bv[u] = toff[u] >= 0 ? __builtin_bit_cast(__bf16, ring[toff[u] + 16 * m + r])
                                     : __builtin_bit_cast(__bf16, (uint16_t)0);
            const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, (f32x4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            // lane (r, q): channels 4q .. 4q + 3 of voxel 16 m + r
            const size_t idx = (vrow + 16 * m + r) * out_stride + out_off + 4 * q;
            if constexpr (F32) {
                *(f32x4 *)((float *)out + idx) = (f32x4){d[0] + bq[0], d[1] + bq[1], d[2] + bq[2], d[3] + bq[3]};
            } else {
                u16x4 y;
#pragma unroll
                for (int e = 0; e < 4; e++)
                    y[e] = f2bf(fmaxf(d[e] + bq[e], 0.f));
                *(u16x4 *)((uint16_t *)out + idx) = y;
            }
        }
        // plane i + 2 into the slot of plane i - 2 (last read before the previous barrier)
        if (p + 1 < PL) {
            PM_IN1_STORE(0, (p + 3) & 3);
#pragma unroll
            for (int d = 0; d < 3; d++)
#pragma unroll
                for (int u = 0; u < 2; u++)
                    pre[d][u] = pre[d + 1][u];
        }
        __syncthreads();
    }
#undef PM_IN1_STORE
#undef PM_IN1_FETCH
}

// false unless n % 64 == 0 and the output view is 4-aligned
bool launch_conv3_in1(const uint16_t *f, const float *w, const float *b, float x1, float x2, float x3, void *out,
                      int out_stride, int out_off, bool out_f32, int n, hipStream_t st)
{
    if (n % 64 || out_stride % 4 || out_off % 4)
        return false;
    const int PL = n >= 256 ? 16 : 8;
    const unsigned ntiles = (unsigned)(n / PL) * (n / 4) * (n / 64);
    if (out_f32)
        hipLaunchKernelGGL(k_conv3_in1<true>, dim3(ntiles), dim3(256), 0, st, f, w, b, x1, x2, x3, out, out_stride,
                           out_off, n, PL);
    else
        hipLaunchKernelGGL(k_conv3_in1<false>, dim3(ntiles), dim3(256), 0, st, f, w, b, x1, x2, x3, out, out_stride,
                           out_off, n, PL);
    return true;
}

// Training target t = lap7(chi) / (h^2 s mu_chi) - delta (natural order out);
// chi natural FP64, delta packed.
__global__ __launch_bounds__(256) void k_source_target(const double *__restrict__ chi,
                                                       const double *__restrict__ delta, int n, double inv_scale,
                                                       float *__restrict__ t)
{
    const unsigned nvox = (unsigned)n * n * n;
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256) {
        const int k = (int)(v % (unsigned)n), j = (int)((v / n) % (unsigned)n), i = (int)(v / ((unsigned)n * n));
        const int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
        const int jp = j + 1 == n ? 0 : j + 1, jm = j == 0 ? n - 1 : j - 1;
        const int kp = k + 1 == n ? 0 : k + 1, km = k == 0 ? n - 1 : k - 1;
        const double lap = chi[((unsigned)ip * n + j) * n + k] + chi[((unsigned)im * n + j) * n + k] +
                           chi[((unsigned)i * n + jp) * n + k] + chi[((unsigned)i * n + jm) * n + k] +
                           chi[((unsigned)i * n + j) * n + kp] + chi[((unsigned)i * n + j) * n + km] - 6.0 * chi[v];
        t[v] = (float)(lap * inv_scale - delta[packed_index(v, n)]);
    }
}

void launch_source_target(const double *chi, const double *delta_packed, int n, double inv_scale, float *t,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_source_target, dim3(2048), dim3(256), 0, st, chi, delta_packed, n, inv_scale, t);
}

// yhat[v] = hb + sum_c hw[c] * b5[v][c]
__global__ __launch_bounds__(256) void k_head(const uint16_t *__restrict__ b5, const float *__restrict__ hw,
                                              const float *__restrict__ hb, unsigned nvox, float *__restrict__ yhat)
{
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256) {
        float s = hb[0];
        const uint16_t *h = b5 + (size_t)v * 16;
        for (int c = 0; c < 16; c++)
            s += hw[c] * bf2f(h[c]);
        yhat[v] = s;
    }
}

void launch_head(const uint16_t *b5, const float *hw, const float *hb, unsigned nvox, float *yhat, hipStream_t st)
{
    hipLaunchKernelGGL(k_head, dim3(2048), dim3(256), 0, st, b5, hw, hb, nvox, yhat);
}

// Backward of the output head yhat = hb + sum_c hw[c] b5[c].  With y given:
// MSE loss L = mean (yhat - y)^2 and dyhat = 2 (yhat - y) / N; with y null,
// `yhat` already holds dL/dyhat.  db5 = dyhat hw (masked by b5 > 0, the ReLU
// of the layer below), rounded to BF16.  Each block writes its partial sums
// of the head's 17 gradients and of the loss to part[block * 18 + q]; the
// one-block k_head_finalize adds them in block order (deterministic).
__global__ __launch_bounds__(256) void k_head_loss_bwd(const float *__restrict__ yhat, const float *__restrict__ y,
                                                       const uint16_t *__restrict__ b5, const float *__restrict__ hw,
                                                       unsigned nvox, uint16_t *__restrict__ db5,
                                                       float *__restrict__ part)
{
    __shared__ float sm[18][4];
    float gw[16], gb = 0.f, ls = 0.f;
    for (int c = 0; c < 16; c++)
        gw[c] = 0.f;
    const float sc = 2.0f / (float)nvox;
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256) {
        float g;
        if (y) {
            const float d = yhat[v] - y[v];
            ls += d * d;
            g = sc * d;
        } else {
            g = yhat[v];
        }
        gb += g;
        const uint16_t *h = b5 + (size_t)v * 16;
        uint16_t *dh = db5 + (size_t)v * 16;
        for (int c = 0; c < 16; c++) {
            const float hv = bf2f(h[c]);
            gw[c] += g * hv;
            dh[c] = hv > 0.f ? f2bf(g * hw[c]) : (uint16_t)0;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int q = 0; q < 18; q++) {
        float x = q < 16 ? gw[q] : (q == 16 ? gb : ls);
        for (int off = 32; off > 0; off >>= 1)
            x += __shfl_down(x, off, 64);
        if (lane == 0)
            sm[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < 18)
        part[(size_t)blockIdx.x * 18 + threadIdx.x] =
            sm[threadIdx.x][0] + sm[threadIdx.x][1] + sm[threadIdx.x][2] + sm[threadIdx.x][3];
}

// ghw[16], ghb[1] (overwritten) and, when loss is not null, the mean loss.
__global__ __launch_bounds__(64) void k_head_finalize(const float *__restrict__ part, unsigned nb,
                                                      float *__restrict__ ghw, float *__restrict__ ghb,
                                                      float *__restrict__ loss, unsigned nvox)
{
    const int q = threadIdx.x;
    if (q >= 18)
        return;
    float t = 0.f;
    for (unsigned b = 0; b < nb; b++)
        t += part[(size_t)b * 18 + q];
    if (q < 16)
        ghw[q] = t;
    else if (q == 16)
        ghb[0] = t;
    else if (loss)
        loss[0] = t / (float)nvox;
}

size_t head_partial_floats() { return 1024 * 18; }

void launch_head_loss_bwd(const float *yhat, const float *y, const uint16_t *b5, const float *hw, unsigned nvox,
                          uint16_t *db5, float *ghw, float *ghb, float *loss, float *part, hipStream_t st)
{
    unsigned nb = (nvox + 255) / 256;
    if (nb > 1024)
        nb = 1024;
    hipLaunchKernelGGL(k_head_loss_bwd, dim3(nb), dim3(256), 0, st, yhat, y, b5, hw, nvox, db5, part);
    hipLaunchKernelGGL(k_head_finalize, dim3(1), dim3(64), 0, st, (const float *)part, nb, ghw, ghb, y ? loss : nullptr,
                       nvox);
}

// ---------------------------------------------------------------- parameters
// Pack fp32 W[27][cin][cout] into bf16 Wf[27][cout_pad][cin_pad] (forward)
// and Wd[27][cin_pad][cout_pad] (input gradient: output channels = cin).
__device__ __forceinline__ void pack_conv(const float *__restrict__ w, int cin, int cout, int cin_pad, int cout_pad,
                                          uint16_t *__restrict__ wf, uint16_t *__restrict__ wd, size_t x0, size_t dx)
{
    const size_t total = (size_t)27 * cin_pad * cout_pad;
    for (size_t e = x0; e < total; e += dx) {
        const int t = (int)(e / ((size_t)cin_pad * cout_pad));
        const int rem = (int)(e - (size_t)t * cin_pad * cout_pad);
        const int c = rem / cout_pad, o = rem % cout_pad;
        const float v = (c < cin && o < cout) ? w[((size_t)t * cin + c) * cout + o] : 0.f;
        const uint16_t b = f2bf(v);
        wf[((size_t)t * cout_pad + o) * cin_pad + c] = b;
        if (wd)
            wd[((size_t)t * cin_pad + c) * cout_pad + o] = b;
    }
}
__global__ __launch_bounds__(256) void k_pack_conv(const float *__restrict__ w, int cin, int cout, int cin_pad,
                                                   int cout_pad, uint16_t *__restrict__ wf, uint16_t *__restrict__ wd)
{
    pack_conv(w, cin, cout, cin_pad, cout_pad, wf, wd, (size_t)blockIdx.x * 256 + threadIdx.x, (size_t)gridDim.x * 256);
}

// All of a network's weight packings in one launch: grid row y runs job y
// (the element loops of the packing kernels).
__global__ __launch_bounds__(256) void k_pack_jobs(PackJobs jobs)
{
    const PackJob &J = jobs.job[blockIdx.y];
    const int x0 = blockIdx.x * 256 + threadIdx.x, dx = gridDim.x * 256;
    if (J.kind == 0)
        pack_conv(J.w, J.cin, J.cout, J.a, J.b, J.d0, J.d1, (size_t)x0, (size_t)dx);
    else if (J.kind == 1)
        pack_poly(J.w, J.cin, J.cout, J.a, J.b, J.d0, x0, dx);
    else
        pack_conv_sub(J.w, J.cin, J.cout, J.a, J.b, J.c, J.d, J.d0, x0, dx);
}

void launch_pack_jobs(const PackJobs &jobs, hipStream_t st)
{
    if (jobs.n > 0)
        hipLaunchKernelGGL(k_pack_jobs, dim3(64, jobs.n), dim3(256), 0, st, jobs);
}

void launch_pack_conv(const float *w, int cin, int cout, int cin_pad, int cout_pad, uint16_t *wf, uint16_t *wd,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_conv, dim3(256), dim3(256), 0, st, w, cin, cout, cin_pad, cout_pad, wf, wd);
}

// sum of squares of the gradient (global-norm clipping)
__global__ __launch_bounds__(kBlock) void k_sumsq(const float *__restrict__ g, ReduceSlot rs, Span sp)
{
    double acc[1] = {0.0};
    PM_SPAN_LOOP(e, sp)
    acc[0] += (double)g[e] * (double)g[e];
    block_partials<1>(acc, rs, sp);
}

void launch_sumsq(const float *g, long long n, ReduceSlot rs, hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n);
    hipLaunchKernelGGL(k_sumsq, dim3(sp.nblocks), dim3(kBlock), 0, st, g, rs, sp);
    launch_finalize(rs, sp, 1, rs.out, st);
}

// Adam (Kingma & Ba) with bias correction on FP32 master weights; the
// gradient is scaled by min(1, clip / ||g||) when clip > 0 (||g||^2 in gsq).
// omb1 = 1 - b1 and omb2 = 1 - b2 come from the host, formed in FP64: in
// FP32, 1 - b2 from a rounded b2 = 0.999 would be off by 1e-5 relative.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, long long n, float lr, float b1, float omb1,
                                              float b2, float omb2, float eps, float c1, float c2,
                                              const double *__restrict__ gsq, float clip)
{
    const double gn = sqrt(gsq[0]);
    const float scale = (clip > 0.f && gn > (double)clip) ? (float)((double)clip / gn) : 1.f;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float gg = scale * g[e];
        const float mm = b1 * m[e] + omb1 * gg;
        const float vv = b2 * v[e] + omb2 * gg * gg;
        m[e] = mm;
        v[e] = vv;
        w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

void launch_adam(float *w, const float *g, float *m, float *v, long long n, double lr, double b1, double b2,
                 double eps, long long step, const double *gsq, double clip, hipStream_t st)
{
    const float c1 = (float)(1.0 - pow(b1, (double)step)), c2 = (float)(1.0 - pow(b2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, st, w, g, m, v, n, (float)lr, (float)b1, (float)(1.0 - b1),
                       (float)b2, (float)(1.0 - b2), (float)eps, c1, c2, gsq, (float)clip);
}

// bf16 <-> f32 helpers for tests and the output path
__global__ __launch_bounds__(256) void k_bf16_slice_to_f32(const uint16_t *__restrict__ s, int stride, int off, int C,
                                                           float *__restrict__ d, size_t nvox)
{
    const size_t total = nvox * (size_t)C;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const size_t v = e / C;
        d[e] = bf2f(s[v * stride + off + (e - v * C)]);
    }
}

void launch_bf16_slice_to_f32(const uint16_t *s, int stride, int off, int C, float *d, size_t nvox, hipStream_t st)
{
    hipLaunchKernelGGL(k_bf16_slice_to_f32, dim3(1024), dim3(256), 0, st, s, stride, off, C, d, nvox);
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *__restrict__ s, uint16_t *__restrict__ d, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
        d[e] = f2bf(s[e]);
}

void launch_f32_to_bf16(const float *s, uint16_t *d, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(1024), dim3(256), 0, st, s, d, n);
}

__global__ __launch_bounds__(kBlock) void k_f32_sum(const float *__restrict__ x, ReduceSlot rs, Span sp)
{
    double acc[1] = {0.0};
    PM_SPAN_LOOP(e, sp)
    acc[0] += (double)x[e];
    block_partials<1>(acc, rs, sp);
}

// delta[packed(v)] += yhat[v] - <yhat>: the learned source delta + t
__global__ __launch_bounds__(256) void k_add_source(const float *__restrict__ yhat, int n,
                                                    const double *__restrict__ ysum, double *__restrict__ delta)
{
    const unsigned nvox = (unsigned)n * n * n;
    const double mean = ysum[0] / nvox;
    for (unsigned v = blockIdx.x * 256 + threadIdx.x; v < nvox; v += gridDim.x * 256)
        delta[packed_index(v, n)] += (double)yhat[v] - mean;
}

void launch_add_source(const float *yhat, int n, double *delta_packed, ReduceSlot rs, hipStream_t st)
{
    const Span sp = make_span((unsigned long long)n * n * n);
    hipLaunchKernelGGL(k_f32_sum, dim3(sp.nblocks), dim3(kBlock), 0, st, yhat, rs, sp);
    launch_finalize(rs, sp, 1, rs.out, st);
    hipLaunchKernelGGL(k_add_source, dim3(2048), dim3(256), 0, st, yhat, n, (const double *)rs.out, delta_packed);
}

}  // namespace pmeft
