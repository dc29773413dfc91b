// Internal declarations shared by the HIP sources of libpmeft.so.
//
// Grid storage inside the library ("packed red/black"): a level with n cells
// per side (n even) stores its n^3 values as two colour blocks of n^3/2
// elements, colour c = (i + j + k) & 1.  Within a colour block the element
// (i, j, kh) holds the cell (i, j, k = 2 kh + ((i + j + c) & 1)), with kh
// fastest.  Consecutive threads then touch consecutive addresses, a half-sweep
// of red-black Gauss-Seidel reads and writes dense arrays, and the 8 children
// of a coarse cell (I, J, K) sit at kh = K in rows (2I+a, 2J+b) of both
// colours.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pmeft.h"

namespace pmeft {

constexpr int kBlock = 256;          // threads per block of the grid kernels
constexpr int kMaxLevels = 12;
constexpr double kFixScale = 1099511627776.0;  // 2^40: deposit fixed point

// Index arithmetic is 32-bit (grids are capped at 1024^3, so n^3 < 2^31):
// 64-bit integer division is emulated on the GPU and would dominate these
// bandwidth-bound kernels.  split() decodes a linear index over rows of
// length nh and planes of n rows.
__device__ __forceinline__ void split(unsigned e, unsigned nh, unsigned n, int &i, int &j, int &kh)
{
    const unsigned row = e / nh;
    kh = (int)(e - row * nh);
    const unsigned ii = row / n;
    j = (int)(row - ii * n);
    i = (int)ii;
}

// Work distribution of the grid kernels.  The hardware hands block b to
// XCD b mod 8, and each XCD has its own L2.  A block therefore works on one
// contiguous chunk of `chunk` elements, and the chunks are ordered so that
// the blocks an XCD receives cover one contiguous slab of the grid: the
// planes a stencil reads around a cell are then mostly in that XCD's L2
// instead of being fetched once per XCD.
struct Span {
    unsigned total;    // elements
    unsigned chunk;    // elements per block (multiple of kBlock)
    unsigned nblocks;  // launched blocks (multiple of 8 when >= 8)
};

constexpr int kMaxBlocks = 2048;  // 8 blocks per CU on 256 CUs

inline Span make_span(unsigned long long total, unsigned max_blocks = kMaxBlocks)
{
    Span sp;
    sp.total = (unsigned)total;
    if (total == 0) {
        sp.chunk = kBlock;
        sp.nblocks = 1;
        return sp;
    }
    unsigned long long b = (total + kBlock - 1) / kBlock;
    if (b > max_blocks)
        b = max_blocks;
    if (b >= 8)
        b -= b % 8;
    if (b < 1)
        b = 1;
    unsigned long long ch = (total + b - 1) / b;
    ch = (ch + kBlock - 1) / kBlock * kBlock;
    sp.chunk = (unsigned)ch;
    sp.nblocks = (unsigned)((total + ch - 1) / ch);
    if (sp.nblocks >= 8 && sp.nblocks % 8)
        sp.nblocks += 8 - sp.nblocks % 8;  // trailing blocks get empty chunks
    if (sp.nblocks < 1)
        sp.nblocks = 1;
    return sp;
}

__device__ __forceinline__ unsigned span_block(const Span &sp)
{
    const unsigned b = blockIdx.x;
    if (sp.nblocks % 8)
        return b;
    const unsigned per = sp.nblocks / 8;
    return (b % 8) * per + b / 8;
}

#define PM_SPAN_LOOP(e, sp)                                                                                            \
    for (unsigned e##_end_ = min((sp).total, (span_block(sp) + 1) * (sp).chunk),                                     \
                  e = span_block(sp) * (sp).chunk + threadIdx.x;                                                      \
         e < e##_end_; e += kBlock)

// Scalars of one solve, by value into every kernel.
struct SolveConsts {
    double nu;     // coefficient of lap chi (1 for the Poisson solve)
    double K;      // screening prefactor (0 for Poisson or the linearised option)
    double beta;   // source b = beta * delta (s for Poisson, xi s for chi)
    // Smoother: red-black Gauss-Seidel (jacobi 0), or Jacobi sweeps under-
    // relaxed as x <- omega x* + (1 - omega) x with x* the local root from the
    // previous iterate's neighbours (jacobi 1).
    double omega = 1.0;
    int jacobi = 0;
};

// Device view of one multigrid level (pointers are to packed arrays).
template <typename R>
struct LevelView {
    int n;           // cells per side
    int nh;          // n / 2
    long long half;  // n^3 / 2
    double h;        // cell size
    const R *dr, *db;   // delta, red / black blocks
    R *tr, *tb;         // FAS source tau (null on the finest level of an F64 solve)
    R *x0r, *x0b;       // restricted fine iterate (coarse levels)
};

// Weight packing jobs of the learned warm start's network, run in one launch:
// kind 0 convolution (a = cin_pad, b = cout_pad, d0 forward and d1 input-
// gradient layout or null), 1 polyphase (a = coarse channels, b = cout_pad),
// 2 a channel range (a = first channel, b = count, c = padded count, d =
// cout_pad).
struct PackJob {
    int kind;
    const float *w;
    int cin, cout, a, b, c, d;
    uint16_t *d0, *d1;
};
constexpr int kMaxPackJobs = 16;
struct PackJobs {
    PackJob job[kMaxPackJobs];
    int n;
};
void launch_pack_jobs(const PackJobs &jobs, hipStream_t st);

// Reduction scratch inside the workspace: every block of a reducing kernel
// writes its partial sums (8 slots per block); a one-block finalize kernel
// launched right after adds them in block order (deterministic, and no
// device-scope fence inside the reducing kernel).
struct ReduceSlot {
    double *partials;   // kMaxBlocks * 8
    unsigned *counter;  // unused (kept zero)
    double *out;        // finalised sums
};

// A pending mixed-precision correction of the FP64 iterate x64 by the FP32
// level-0 iterate v of the last V-cycles: x64 += fl32(v - fl32(x64)) for the
// nonlinear (full-approximation) form, x64 += v for the linear correction
// form.  The tiled outer residual applies it to every value it loads and
// writes the corrected iterate of its own cells to yr / yb (not the arrays
// it reads: neighbouring tiles still read the old values).
struct MixedCorr {
    const float *vr = nullptr, *vb = nullptr;
    double *yr = nullptr, *yb = nullptr;
};

// Grouped launches.  Problems of one shape solved together sit in workspace
// slots `stride` bytes apart; every pointer a solver kernel receives is the
// one of slot 0, and grid row blockIdx.y works on slot map[blockIdx.y] (the
// row itself without a map), so one launch covers the same step of every
// problem in the group.  Per-slot solve constants (nu, K, beta) replace the
// argument's when `sc` is set (see gconsts).  stride 0 is a single problem: no pointer
// moves and the kernels do exactly what they do without a group.
struct Group {
    long long stride = 0;              // bytes between slots
    const int *map = nullptr;          // device: slot of grid row y (null: y)
    const SolveConsts *sc = nullptr;   // device: per-slot constants (null: the argument's)
    int rows = 1;                      // grid rows (host side: gridDim.y)
};

__device__ __forceinline__ int group_slot(const Group &g) { return g.map ? g.map[blockIdx.y] : (int)blockIdx.y; }
__device__ __forceinline__ long long group_offset(const Group &g)
{
    return g.stride ? (long long)group_slot(g) * g.stride : 0;
}
template <typename T>
__device__ __forceinline__ T *gshift(T *p, long long off)
{
    return p ? reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<void *>(static_cast<const void *>(p))) + off)
             : p;
}
template <typename R>
__device__ __forceinline__ void gshift_view(LevelView<R> &L, long long off)
{
    L.dr = gshift(L.dr, off);
    L.db = gshift(L.db, off);
    L.tr = gshift(L.tr, off);
    L.tb = gshift(L.tb, off);
    L.x0r = gshift(L.x0r, off);
    L.x0b = gshift(L.x0b, off);
}
__device__ __forceinline__ void gshift_slot(ReduceSlot &rs, long long off)
{
    rs.partials = gshift(rs.partials, off);
    rs.counter = gshift(rs.counter, off);
    rs.out = gshift(rs.out, off);
}
// A zero K or beta in the argument stays zero: the host zeroes them for the
// correction equation of a linear problem and for the linear guess.
__device__ __forceinline__ void gconsts(SolveConsts &sc, const Group &g)
{
    if (g.sc) {
        const SolveConsts &t = g.sc[group_slot(g)];
        sc.nu = t.nu;
        if (sc.K != 0.0)
            sc.K = t.K;
        if (sc.beta != 0.0)
            sc.beta = t.beta;
    }
}

// The group the launchers of this host thread use (a single problem unless a
// GroupScope is open).
const Group &cur_group();
void set_cur_group(const Group &g);
struct GroupScope {
    Group prev;
    explicit GroupScope(const Group &g);
    ~GroupScope();
};
inline dim3 group_grid(unsigned nblocks) { return dim3(nblocks, (unsigned)cur_group().rows); }

// Block reduction of NV doubles; thread 0 stores the block's sums at
// partials[logical block * 8 + q].  The k_finalize launch that follows adds
// the partials in block order, so results do not depend on scheduling.
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], const ReduceSlot &rs, const Span &sp)
{
    __shared__ double sm[NV][kBlock / 64];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1)
            x += __shfl_down(x, off, 64);
        v[q] = x;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++)
            sm[q][wid] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned lb = span_block(sp);
#pragma unroll
        for (int q = 0; q < NV; q++) {
            double t = 0.0;
            for (int w = 0; w < kBlock / 64; w++)
                t += sm[q][w];
            rs.partials[(size_t)lb * 8 + q] = t;
        }
    }
}

// Sums the partials of the preceding reducing launch (nv values) into out.
void launch_finalize(const ReduceSlot &rs, const Span &sp, int nv, double *out, hipStream_t st);

// ---- launchers (mg_kernels.hip) ------------------------------------------
// One red-black half-sweep (see k_smooth).  Writes its per-block partial
// sums of Lq + tau to rs.partials and returns the block count.
template <typename R>
void launch_smooth(const LevelView<R> &L, int colour, const R *xc_old, const R *xo, R *xc_new, const double *csum_in,
                   double *csum_out, const double *prev, int prev_nblocks, int prev_colour, ReduceSlot rs,
                   SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out, int tiled);

// Both colours of one red-black sweep in one launch (the 2.5D-tiled fused
// sweep of sweep2_kernels.hip): red from (xr_old, xb_old) into xr_new, then
// black from (xb_old, new red) into xb_new.  Returns false, launching
// nothing, where the level does not tile that way or the smoother is Jacobi.
template <typename R>
bool launch_sweep2(const LevelView<R> &L, const R *xr_old, const R *xb_old, R *xr_new, R *xb_new,
                   const double *csum_in, double *csum_out, const double *prev, int prev_nblocks, int prev_colour,
                   ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st, int *nblocks_out);
// whether a level of n cells per side takes the fused sweep
bool sweep2_fits(int n, int word_bytes);

// Fine-level residual r = Lq + tau - c - lap x fused with the 8-child
// restriction into the coarse level: coarse tau <- R r, coarse x <- R x (also
// into x0).  Accumulates sum r^2, sum r, sum Lq+tau into rs.out[0..2] and the
// void-cell count into rs.out[3].
// tiled != 0 selects the 2.5D-tiled kernel on levels with n >= 128.
template <typename R>
void launch_residual_restrict(const LevelView<R> &F, const R *xr, const R *xb, const double *csum,
                              const LevelView<R> &C, R *cxr, R *cxb, ReduceSlot rs, SolveConsts sc, bool nonlinear,
                              hipStream_t st, bool norms = true, int tiled = 0);

// Coarse FAS source: tau += lap x - Lq(x) (unless accumulate_only or the
// level has no tau); writes sum(Lq + tau) per colour into csum[0..1].
// zero_iterate: x is known to be zero (nothing of it is read where the
// level tiles; the sums are bitwise those of reading the zeros).
template <typename R>
void launch_fas_tau(const LevelView<R> &C, const R *xr, const R *xb, double *csum, ReduceSlot rs, SolveConsts sc,
                    bool nonlinear, bool accumulate_only, hipStream_t st, int tiled = 0, bool zero_iterate = false);

// The 2.5D-tiled variants (tile_kernels.hip): return false, launching
// nothing, where the level is too small or its shape does not tile; else
// launch and return the partial-sum span for the finalize.
template <typename R>
bool launch_residual_restrict_tiled(const LevelView<R> &F, const R *xr, const R *xb, const double *csum,
                                    const LevelView<R> &C, R *cxr, R *cxb, ReduceSlot rs, SolveConsts sc,
                                    bool nonlinear, hipStream_t st, int tiled, Span *sp_out);
template <typename R>
bool launch_fas_tau_tiled(const LevelView<R> &L, const R *xr, const R *xb, ReduceSlot rs, SolveConsts sc,
                          bool nonlinear, int accumulate_only, hipStream_t st, int tiled, Span *sp_out,
                          bool zero_iterate = false);
bool launch_mixed_outer_tiled(const LevelView<double> &F64, const double *xr, const double *xb, const double *csum64,
                              const LevelView<float> &F32, float *x32r, float *x32b, ReduceSlot rs, SolveConsts sc,
                              bool nonlinear, hipStream_t st, int tiled, Span *sp_out, const MixedCorr *corr,
                              bool zero_iterate);
// Whether the mixed outer residual of a level of n cells per side runs tiled
// (and can therefore take a pending correction).
bool mixed_outer_tiles(int n, int tiled);

// Fine x += P (x_H - x0_H), trilinear cell-centred prolongation.
template <typename R>
void launch_prolong_correct(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr,
                            const R *cxb, hipStream_t st, int tiled = 0);

// Fine x = P x_H (full-approximation prolongation, to start full multigrid).
template <typename R>
void launch_prolong_full(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                         hipStream_t st, int tiled = 0);
// Tiled prolongation on coarse levels with n >= 64 (false: nothing launched).
template <typename R>
bool launch_prolong_tiled(const LevelView<R> &F, R *xr, R *xb, const LevelView<R> &C, const R *cxr, const R *cxb,
                          bool corr, hipStream_t st, int tiled);

// Coarsest level solved by one workgroup in FP64.
template <typename R>
void launch_coarsest(const LevelView<R> &C, R *xr, R *xb, SolveConsts sc, bool nonlinear, int sweeps,
                     hipStream_t st);

// delta hierarchy: coarse = 8-child average of fine.
template <typename R>
void launch_restrict_field(int nc, const R *fr, const R *fb, R *cr, R *cb, hipStream_t st);

// FP64 fine delta -> FP32 copy (mixed precision hierarchy).
void launch_cast_f64_f32(const double *src, float *dst, long long n, hipStream_t st);
// device-to-device copy (16-byte words where aligned, else hipMemcpyAsync)
hipError_t launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st);

// Natural [i][j][k] <-> packed red/black conversion; dtype of the natural
// array is float or double, the packed array is double.
void launch_natural_to_packed(const void *nat, pm_dtype dt, double *packed, int n, double scale, double shift,
                              hipStream_t st);
// nat = packed - (sum_ptr ? sum_ptr[0] / n^3 : 0) + add
void launch_packed_to_natural(const double *packed, void *nat, pm_dtype dt, int n, double add, const double *sum_ptr,
                              hipStream_t st);

// Mixed precision outer step: FP64 residual of (x64, delta64) with norm
// partials, cast x32 = fl(x64) into the level-0 x (0 for the linear
// correction form) and the FP32 FAS target tau32 = fl(r64) + lap32 x32 -
// Lq32(x32); per-colour sums of Lq32 + tau32 into csum32.
// The six sums go to rs.out; with lag64 / lag32 set, the same final stage
// also writes the next lagged means: lag64[0] = out[2], lag64[1] = 0,
// lag32[0..1] = out[4..5] (lag64 may be csum64: the residual kernel has
// read it by then).  With corr set (tiled levels only, see
// mixed_outer_tiles) the residual is that of the corrected iterate, which
// goes to corr->yr / yb; returns false, launching nothing, where corr is set
// and the level does not tile.
bool launch_mixed_outer_residual(const LevelView<double> &F64, const double *xr, const double *xb,
                                 const double *csum64, const LevelView<float> &F32, float *x32r, float *x32b,
                                 ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st, int tiled = 0,
                                 double *lag64 = nullptr, double *lag32 = nullptr, const MixedCorr *corr = nullptr,
                                 bool zero_iterate = false);
// The correction of MixedCorr applied on its own: x64 += fl32(x32 - fl32(x64))
// (nonlinear) or x64 += x32 (linear).
void launch_mixed_correct(double *x64, const float *x32r, const float *x32b, long long half, bool nonlinear,
                          hipStream_t st);

// Plain FP64 residual norm (no restriction) of the finest level.
void launch_residual_norm(const LevelView<double> &F, const double *xr, const double *xb, const double *csum,
                          ReduceSlot rs, SolveConsts sc, bool nonlinear, hipStream_t st);

// Sum of a packed double field (rs.out[0]).
void launch_field_sum(const double *x, long long n, ReduceSlot rs, hipStream_t st);
// x -= shift (shift read from device *shift_sum / n)
void launch_subtract_mean(double *x, long long n, const double *sum_ptr, hipStream_t st);
// y = a * x
void launch_scale(const double *x, double *y, double a, long long n, hipStream_t st);
void launch_zero(void *p, size_t bytes, hipStream_t st);
// dst[0 .. count-1] = src (dst in host memory the device can write), then
// *seqp = seq after a system-scope fence
void launch_publish(const double *src, int count, double *dst, unsigned *seqp, unsigned seq, hipStream_t st);
// dst[s * count + q] = src[q] of slot s = 0 .. m-1 (slots `stride` bytes apart);
// not a grouped launch (one grid covers every slot)
void launch_gather_slots(const double *src, long long stride, int m, int count, double *dst, hipStream_t st);

// ---- particle sort (pm_kernels.hip) --------------------------------------
size_t sort_workspace_bytes(unsigned long long np, int word);
int launch_sort_particles(void *pos, void *vel, long long *ids, unsigned np, int ng, pm_dtype dt, char *ws,
                          hipStream_t st);

// ---- block cycle: the coarse part of a V-cycle in one workgroup ---------
constexpr int kBlockCycleThreads = 512;
template <typename R>
struct BlockHier {
    int nlev;
    LevelView<R> L[kMaxLevels];
    R *buf[kMaxLevels][2];
};
// fmg = false: V-cycle from level l0 (its tau set, its per-colour sums in
// csum_l0, its colour buffers cur_bits (bit c = buffer of colour c)); each
// colour of level l0 ends in buffer cur ^ ((n_pre + n_post) & 1).
// fmg = true: full multigrid from the coarsest level up to l0 (taus set);
// level l0 ends in buffer (n_pre + n_post) & 1.
template <typename R>
void launch_block_cycle(const BlockHier<R> &B, int l0, bool fmg, int n_pre, int n_post, SolveConsts sc, bool nonlinear,
                        const double *csum_l0, int cur_bits, int coarse_sweeps, hipStream_t st);
// LDS bytes of the levels a block cycle from l0 keeps resident (the first
// resident level in *lr) and the budget they must fit.
template <typename R>
size_t block_cycle_lds(const BlockHier<R> &B, int l0, int *lr);
size_t block_cycle_lds_limit();

// ---- learned warm start (unet_api.hip) -----------------------------------
// Forward pass: copy delta (packed, mean-free) to `save` and run the network
// on that copy, leaving its source prediction t in the workspace; delta
// itself is only read (by the copy), so this may run on a second stream
// while other work reads delta.
// packed: the weights were already packed into ws by unet_learned_pack (for
// these params), so the pass skips that.
int unet_learned_forward(const float *params, const double *delta_packed, double *save, int ng,
                         const pm_eft_params &p, void *ws, size_t ws_bytes, hipStream_t st, bool packed = false);
// The weights' MFMA layouts into ws (inference form), ahead of
// unet_learned_forward(..., packed = true): they depend on params only.
int unet_learned_pack(const float *params, int ng, void *ws, size_t ws_bytes, hipStream_t st);
// delta -> delta + t - <t> with the t of the preceding forward pass.
int unet_add_learned_source(void *ws, int ng, double *delta_packed, hipStream_t st);
double *unet_save_area(void *ws, int ng);

// ---- particle kernels (pm_kernels.hip) -----------------------------------
void launch_deposit_fixed(const void *pos, long long np, pm_dtype dt, int ng, unsigned long long *acc,
                          hipStream_t st);
// The deposit pm_deposit and pm_step use: the gather over particles in CIC
// base-row order, else the scatter (decided on the device; acc need not be
// cleared).  idx: deposit_index_bytes(ng) bytes of workspace.
size_t deposit_index_bytes(int ng);
void launch_deposit_auto(const void *pos, long long np, pm_dtype dt, int ng, unsigned long long *acc, void *idx,
                         hipStream_t st);
// acc (fixed point) -> packed delta = rho - 1 (FP64); sum into rs.out[0]
void launch_fixed_to_delta(const unsigned long long *acc, int ng, double rho_scale, double *delta_packed,
                           ReduceSlot rs, hipStream_t st);
// g = -D5 (psi + xi chi) from packed FP64 fields -> interleaved (gx, gy, gz, 0)
void launch_gradient(const double *psi, const double *chi, double xi, int ng, void *g4, pm_dtype dt,
                     hipStream_t st);
void launch_interp_kick(const void *g4, int ng, pm_dtype dt, void *pos, long long np, void *vel,
                        double dt_kick, double dt_drift, void *acc_out, hipStream_t st);
// Psi = Psi_N + c_psi chi, Phi = Psi_N + c_phi chi, Psi + Phi (natural order;
// outputs nullable)
void launch_potentials(const void *psi_n, const void *chi, pm_dtype dt, long long n3, double c_psi, double c_phi,
                       void *psi, void *phi, void *lens, hipStream_t st);

}  // namespace pmeft
