// Host side of libpmeft.so: coefficients, workspace planning, the multigrid
// drivers (FP64 and mixed precision) and the C ABI declared in pmeft.h.
#include "pmeft_internal.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace pmeft {

// ------------------------------------------------------------ coefficients
// Secs. 2.2-2.5 and 3.1 (see pmeft.h for the definitions).
static int coefficients(const pm_eft_params &p, pm_eft_coeffs &c)
{
    const double om0 = p.omega_m0, a = p.a;
    if (!(om0 > 0.0 && om0 < 1.0) || !(a > 0.0))
        return PM_EINVAL;
    const double om = om0 / (om0 + (1.0 - om0) * a * a * a);
    const double E2 = om0 / (a * a * a) + 1.0 - om0;
    const double ab = p.alpha_b0 * (1.0 - om) / (1.0 - om0);
    const double am = p.alpha_m0 * (1.0 - om) / (1.0 - om0);
    const double geff = pow(om, p.alpha_m0 / (3.0 * (1.0 - om0)));
    const double hdot = -1.5 * om;                         // Hdot / H^2
    const double abdot = p.alpha_b_dot ? 3.0 * om * ab : 0.0;  // d alpha_B / d ln a
    const double C2 = -am + ab * (1.0 + am) + (1.0 + ab) * hdot + abdot + 1.5 * om * geff;
    const double C4 = p.screening ? (-4.0 * ab + 2.0 * am) : 0.0;
    c.omega_m_a = om;
    c.E2 = E2;
    c.alpha_b = ab;
    c.alpha_m = am;
    c.geff = geff;
    c.C2 = C2;
    c.C4 = C4;
    c.nu = 2.0 * ab * am - ab * ab - C2;
    c.xi = ab - am;
    c.s = 1.5 * geff * a * om0;
    c.K = C4 / (4.0 * E2 * a * a * a * a);
    c.mu_chi = c.nu != 0.0 ? c.xi / c.nu : 0.0;
    c.mu_psi = c.nu != 0.0 ? 1.0 + c.xi * c.xi / c.nu : 1.0;
    c.lambda = c.nu != 0.0 ? c.K * c.s * c.xi / (c.nu * c.nu) : 0.0;
    if (c.xi != 0.0 && !(c.nu > 0.0))
        return PM_EUNSTABLE;
    return PM_OK;
}

static int grid_levels(int ng)
{
    if (ng < 8 || ng > 1024)
        return 0;
    int n = ng, l = 1;
    while (n % 2 == 0 && n / 2 >= 4) {
        n /= 2;
        l++;
    }
    if (n != 4 && n != 6)
        return 0;
    return l;
}

// ----------------------------------------------------------- workspace plan
enum { kPrecF64 = 1, kPrecMixed = 2 };

struct Plan {
    int ng = 0, nlev = 0;
    long long N = 0, np = 0;
    int n[kMaxLevels] = {};
    size_t total = 0;
    size_t red_partials = 0, red_counter = 0, red_out = 0, csum64 = 0, csum32 = 0, outer_out = 0, sm_partials = 0;
    size_t delta64[kMaxLevels] = {};
    size_t psi64 = 0, chi64 = 0;
    size_t p64[kMaxLevels] = {}, q64[kMaxLevels] = {}, t64[kMaxLevels] = {}, x064[kMaxLevels] = {};
    size_t d32[kMaxLevels] = {}, p32[kMaxLevels] = {}, q32[kMaxLevels] = {}, t32[kMaxLevels] = {},
           x032[kMaxLevels] = {};
    size_t fixacc = 0, g4 = 0, depidx = 0;
    size_t dalt64[kMaxLevels] = {}, dalt32[kMaxLevels] = {};  // step plans: the warm start's delta hierarchy
    int precs = 0;
    // Everything one solve writes (reductions, lagged means, the hierarchy
    // buffers) sits in [solve_lo, solve_lo + solve_bytes); a step plan holds a
    // second such region at solve2 so that its two solves can run side by side.
    size_t solve_lo = 0, solve_bytes = 0, solve2 = 0;
};

static size_t take(size_t &cur, size_t bytes)
{
    const size_t o = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return o;
}

static bool make_plan(Plan &P, int ng, long long np, pm_dtype dt, int precs)
{
    P = Plan();
    P.nlev = grid_levels(ng);
    if (!P.nlev)
        return false;
    P.ng = ng;
    P.np = np;
    P.precs = precs;
    P.N = (long long)ng * ng * ng;
    for (int l = 0, m = ng; l < P.nlev; l++, m /= 2)
        P.n[l] = m;
    size_t c = 0;
    // shared by both solves (read-only while they run)
    for (int l = 0; l < P.nlev; l++)
        P.delta64[l] = take(c, sizeof(double) * (size_t)P.n[l] * P.n[l] * P.n[l]);
    P.psi64 = take(c, sizeof(double) * P.N);
    P.chi64 = take(c, sizeof(double) * P.N);
    if (precs & kPrecMixed)
        for (int l = 0; l < P.nlev; l++)
            P.d32[l] = take(c, sizeof(float) * (size_t)P.n[l] * P.n[l] * P.n[l]);
    if (np > 0) {
        P.fixacc = take(c, sizeof(unsigned long long) * P.N);
        P.depidx = take(c, deposit_index_bytes(ng));
        P.g4 = take(c, (dt == PM_F64 ? sizeof(double) : sizeof(float)) * 4 * P.N);
        for (int l = 0; l < P.nlev; l++) {
            const size_t m3 = (size_t)P.n[l] * P.n[l] * P.n[l];
            P.dalt64[l] = take(c, sizeof(double) * m3);
            if (precs & kPrecMixed)
                P.dalt32[l] = take(c, sizeof(float) * m3);
        }
    }
    // one solve's own region
    P.solve_lo = c;
    P.red_partials = take(c, sizeof(double) * 8 * kMaxBlocks);
    P.red_counter = take(c, 256);
    P.red_out = take(c, sizeof(double) * 8);
    P.outer_out = take(c, sizeof(double) * 8);
    P.csum64 = take(c, sizeof(double) * 2 * 2 * kMaxLevels);
    P.csum32 = take(c, sizeof(double) * 2 * 2 * kMaxLevels);
    P.sm_partials = take(c, sizeof(double) * 8 * kMaxBlocks * 2 * kMaxLevels);
    if (precs & kPrecF64) {
        for (int l = 0; l < P.nlev; l++) {
            const size_t m3 = (size_t)P.n[l] * P.n[l] * P.n[l];
            if (l > 0)
                P.p64[l] = take(c, sizeof(double) * m3);
            P.q64[l] = take(c, sizeof(double) * m3);
            if (l > 0) {
                P.t64[l] = take(c, sizeof(double) * m3);
                P.x064[l] = take(c, sizeof(double) * m3);
            }
        }
    }
    if (precs & kPrecMixed) {
        for (int l = 0; l < P.nlev; l++) {
            const size_t m3 = (size_t)P.n[l] * P.n[l] * P.n[l];
            P.p32[l] = take(c, sizeof(float) * m3);
            P.q32[l] = take(c, sizeof(float) * m3);
            P.t32[l] = take(c, sizeof(float) * m3);
            P.x032[l] = take(c, sizeof(float) * m3);
        }
    }
    P.solve_bytes = c - P.solve_lo;
    if (np > 0) {
        P.solve2 = c;
        c += P.solve_bytes;
    }
    P.total = c + 256;
    return true;
}

// Moves every offset of the per-solve region to start at `to` (the layout
// inside the region is unchanged).
static void rebase_solve(Plan &P, size_t to)
{
    const size_t d = to - P.solve_lo;
    for (size_t *f : {&P.red_partials, &P.red_counter, &P.red_out, &P.outer_out, &P.csum64, &P.csum32, &P.sm_partials})
        *f += d;
    for (int l = 0; l < P.nlev; l++) {
        if (P.precs & kPrecF64) {
            if (l > 0) {
                P.p64[l] += d;
                P.t64[l] += d;
                P.x064[l] += d;
            }
            P.q64[l] += d;
        }
        if (P.precs & kPrecMixed) {
            P.p32[l] += d;
            P.q32[l] += d;
            P.t32[l] += d;
            P.x032[l] += d;
        }
    }
    P.solve_lo = to;
}

// ---------------------------------------------------------------- context
struct Ctx {
    Plan P;
    char *ws = nullptr;
    hipStream_t st = nullptr;
    ReduceSlot rs;
    double *csum64 = nullptr, *csum32 = nullptr, *outer_out = nullptr, *sm_partials = nullptr;
    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

#define PM_HIP(call)                                                                                                   \
    do {                                                                                                               \
        if ((call) != hipSuccess)                                                                                      \
            return PM_EHIP;                                                                                            \
    } while (0)

static int launched()
{
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP;
}

// Pointers of the context's per-solve region (from its plan); the reduction
// counter is cleared on the context's stream.
static void bind_solve(Ctx &C)
{
    C.rs.partials = C.at<double>(C.P.red_partials);
    C.rs.counter = C.at<unsigned>(C.P.red_counter);
    C.rs.out = C.at<double>(C.P.red_out);
    C.csum64 = C.at<double>(C.P.csum64);
    C.csum32 = C.at<double>(C.P.csum32);
    C.outer_out = C.at<double>(C.P.outer_out);
    C.sm_partials = C.at<double>(C.P.sm_partials);
    launch_zero(C.ws + C.P.red_counter, 256, C.st);
}

static int setup_ctx(Ctx &C, void *ws, size_t ws_bytes, int ng, long long np, pm_dtype dt, int precs,
                     pm_stream_t stream)
{
    if (!ws)
        return PM_EINVAL;
    if (!make_plan(C.P, ng, np, dt, precs))
        return PM_EINVAL;
    if (ws_bytes < C.P.total)
        return PM_ENOMEM;
    // 256-byte alignment of the caller's buffer
    if (((uintptr_t)ws) & 255)
        return PM_EINVAL;
    C.ws = (char *)ws;
    C.st = (hipStream_t)stream;
    bind_solve(C);
    return launched();
}

// ---- small readbacks -------------------------------------------------------
// A solve reads a few norms back after every V-cycle.  The device writes them
// into pinned, coherent host memory followed by a sequence number
// (launch_publish), and the host polls the sequence number: no copy launch
// and no stream synchronisation, which shortens the idle gap before the next
// cycle's launches.  Mailboxes come from a process-wide pool: a host thread
// leases one per device on first use and returns it when it exits (pm_step
// starts a worker thread per step).
namespace {
constexpr int kMailDevices = 16;
constexpr size_t kMailBytes = 16384, kMailSeqOff = 12288;  // values: up to 1536 doubles
struct Mailbox {
    double *vals = nullptr;
    unsigned *seq = nullptr;
    unsigned next = 0;
};
std::mutex g_mail_mu;
std::vector<Mailbox *> g_mail_free[kMailDevices];
struct MailLease {
    Mailbox *m[kMailDevices] = {};
    ~MailLease()
    {
        std::lock_guard<std::mutex> g(g_mail_mu);
        for (int d = 0; d < kMailDevices; d++)
            if (m[d])
                g_mail_free[d].push_back(m[d]);
    }
};
thread_local MailLease t_mail;

Mailbox *mailbox()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMailDevices)
        return nullptr;
    if (t_mail.m[dev])
        return t_mail.m[dev];
    {
        std::lock_guard<std::mutex> g(g_mail_mu);
        if (!g_mail_free[dev].empty()) {
            t_mail.m[dev] = g_mail_free[dev].back();
            g_mail_free[dev].pop_back();
            return t_mail.m[dev];
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, kMailBytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
        return nullptr;
    Mailbox *M = new Mailbox;
    M->vals = (double *)p;
    M->seq = (unsigned *)((char *)p + kMailSeqOff);
    *(volatile unsigned *)M->seq = 0u;
    t_mail.m[dev] = M;
    return M;
}
}  // namespace

// count doubles at dev, written by the work queued on C.st, into host[].
static int read_out(Ctx &C, const double *dev, double *host, int count)
{
    Mailbox *M = mailbox();
    if (!M || sizeof(double) * count > kMailSeqOff) {
        PM_HIP(hipMemcpyAsync(host, dev, sizeof(double) * count, hipMemcpyDeviceToHost, C.st));
        PM_HIP(hipStreamSynchronize(C.st));
        return PM_OK;
    }
    const unsigned seq = ++M->next;
    launch_publish(dev, count, M->vals, M->seq, seq, C.st);
    PM_HIP(hipGetLastError());
    volatile unsigned *s = M->seq;
    long long spins = 0;
    while (*s != seq) {
        if (++spins > (1LL << 26)) {  // a long wait: synchronise the stream (which reports its errors)
            PM_HIP(hipStreamSynchronize(C.st));
            if (*s != seq)
                return PM_EHIP;
            break;
        }
    }
    for (int q = 0; q < count; q++)
        host[q] = ((volatile double *)M->vals)[q];
    return PM_OK;
}

// Hierarchy of one precision: per-level ping-pong buffers and flags telling
// which buffer holds the current red / black values, double-buffered
// per-colour sums of Lq + tau (the lagged mean) and the partial sums of the
// last half-sweep still to be folded into them.
template <typename R>
struct Hier {
    int nlev = 0;
    LevelView<R> L[kMaxLevels];
    R *buf[kMaxLevels][2];
    int cur[kMaxLevels][2];  // [level][colour] -> buffer index
    double *csum = nullptr;  // [2][kMaxLevels][2]
    double *parts = nullptr; // [kMaxLevels][2][kMaxBlocks * 8]
    int cs[kMaxLevels];      // current csum buffer per level
    int pend_col[kMaxLevels], pend_nb[kMaxLevels], next_part[kMaxLevels];
    int block_l0 = kMaxLevels;  // levels from here down run as one block cycle
    int tiled = 1;              // 2.5D-tiled smoother: 0 off, 1 small, 2 large, 3 largest tiles
    bool fused = false;         // large levels sweep both colours in one launch
    BlockHier<R> block() const
    {
        BlockHier<R> B;
        B.nlev = nlev;
        for (int l = 0; l < kMaxLevels; l++) {
            B.L[l] = L[l];
            B.buf[l][0] = buf[l][0];
            B.buf[l][1] = buf[l][1];
        }
        return B;
    }
    R *xr(int l) { return buf[l][cur[l][0]]; }
    R *xb(int l) { return buf[l][cur[l][1]] + L[l].half; }
    double *csum_cur(int l) { return csum + ((size_t)cs[l] * kMaxLevels + l) * 2; }
    double *csum_alt(int l) { return csum + ((size_t)(cs[l] ^ 1) * kMaxLevels + l) * 2; }
    double *part(int l, int k) { return parts + ((size_t)l * 2 + k) * 8 * kMaxBlocks; }
    // the level's mean was just set exactly (csum_cur); nothing pending
    void fresh(int l) { pend_col[l] = -1; }
    void init_state(int l)
    {
        cur[l][0] = cur[l][1] = 0;
        cs[l] = 0;
        pend_col[l] = -1;
        pend_nb[l] = 0;
        next_part[l] = 0;
    }
};

template <typename R>
static LevelView<R> make_view(int n, double h, const R *d, R *t, R *x0)
{
    LevelView<R> v;
    v.n = n;
    v.nh = n / 2;
    v.half = (long long)n * n * (n / 2);
    v.h = h;
    v.dr = d;
    v.db = d ? d + v.half : nullptr;
    v.tr = t;
    v.tb = t ? t + v.half : nullptr;
    v.x0r = x0;
    v.x0b = x0 ? x0 + v.half : nullptr;
    return v;
}

// ---- launch-shape table --------------------------------------------------
// Per (finest grid, word size): the largest grid of the levels that run as
// one block cycle, and whether the large levels use the 2.5D-tiled smoother;
// set by pm_autotune, defaults kBlockCycleDefault and tiled.
constexpr int kBlockCycleDefault = 8;
struct Shape {
    int ng, word, block_n, tiled;
};
struct TuneTable {
    std::mutex mu;
    std::vector<Shape> rows;
};
static TuneTable g_tune;

static Shape launch_shape(int ng, int word)
{
    std::lock_guard<std::mutex> g(g_tune.mu);
    for (const auto &e : g_tune.rows)
        if (e.ng == ng && e.word == word)
            return e;
    return Shape{ng, word, kBlockCycleDefault, 1};
}

static void set_shape(const Shape &sh)
{
    std::lock_guard<std::mutex> g(g_tune.mu);
    for (auto &e : g_tune.rows)
        if (e.ng == sh.ng && e.word == sh.word) {
            e = sh;
            return;
        }
    g_tune.rows.push_back(sh);
}

template <typename R>
static void set_block_level(Hier<R> &H, int ng)
{
    const Shape sh = launch_shape(ng, (int)sizeof(R));
    H.tiled = sh.tiled > 3 ? 3 : sh.tiled;  // 4: the largest tiles for the transfers, fused sweeps
    H.fused = sh.tiled == 4;
    H.block_l0 = kMaxLevels;
    for (int l = 0; l < H.nlev - 1; l++)
        if (H.L[l].n <= sh.block_n) {
            H.block_l0 = l;
            break;
        }
}

static void build_hier64(Ctx &C, Hier<double> &H, double *master)
{
    const Plan &P = C.P;
    H.nlev = P.nlev;
    H.csum = C.csum64;
    for (int l = 0; l < P.nlev; l++) {
        const double h = 1.0 / P.n[l];
        H.L[l] = make_view<double>(P.n[l], h, C.at<double>(P.delta64[l]), l ? C.at<double>(P.t64[l]) : nullptr,
                                   l ? C.at<double>(P.x064[l]) : nullptr);
        H.buf[l][0] = l ? C.at<double>(P.p64[l]) : master;
        H.buf[l][1] = C.at<double>(P.q64[l]);
        H.init_state(l);
    }
    H.parts = C.sm_partials;
    set_block_level(H, P.ng);
}

static void build_hier32(Ctx &C, Hier<float> &H)
{
    const Plan &P = C.P;
    H.nlev = P.nlev;
    H.csum = C.csum32;
    for (int l = 0; l < P.nlev; l++) {
        const double h = 1.0 / P.n[l];
        H.L[l] = make_view<float>(P.n[l], h, C.at<float>(P.d32[l]), C.at<float>(P.t32[l]), C.at<float>(P.x032[l]));
        H.buf[l][0] = C.at<float>(P.p32[l]);
        H.buf[l][1] = C.at<float>(P.q32[l]);
        H.init_state(l);
    }
    H.parts = C.sm_partials;
    set_block_level(H, P.ng);
}

// ------------------------------------------------------- kernel timing
// Opt-in measurement: while enabled, every launch of the finest-level
// smoother is bracketed by two HIP events recorded on the launch stream.
// Slots: 0 scalar field FP64, 1 scalar field FP32, 2 Poisson FP64,
// 3 Poisson FP32.
struct KernelTiming {
    std::mutex mu;
    std::atomic<bool> on{false};  // read by the step's worker thread too
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> slot_of_pair;
};
static KernelTiming g_kt;
constexpr size_t kTimingPairs = 16384;
constexpr int kTimingSlots = 8;  // 0..3 half-sweeps, 4..7 fused sweeps (same order)

template <typename R>
static void smooth(Ctx &C, Hier<R> &H, int l, int colour, SolveConsts sc, bool nl)
{
    const int own = H.cur[l][colour];
    const long long half = H.L[l].half;
    R *src = H.buf[l][own] + (colour ? half : 0);
    R *dst = H.buf[l][1 - own] + (colour ? half : 0);
    const R *oth = H.buf[l][H.cur[l][1 - colour]] + (colour ? 0 : half);
    if (sc.jacobi && colour == 1)  // Jacobi: the red values from before this sweep's red half
        oth = H.buf[l][1 - H.cur[l][0]];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (l == 0 && g_kt.on.load(std::memory_order_relaxed)) {
        std::lock_guard<std::mutex> g(g_kt.mu);
        if (g_kt.used + 2 <= g_kt.pool.size()) {
            e0 = g_kt.pool[g_kt.used];
            e1 = g_kt.pool[g_kt.used + 1];
            g_kt.used += 2;
            g_kt.slot_of_pair.push_back((sizeof(R) == 4 ? 1 : 0) + (nl ? 0 : 2));
        }
    }
    if (e0)
        (void)hipEventRecord(e0, C.st);
    ReduceSlot rs = C.rs;
    const int k = H.next_part[l];
    rs.partials = H.part(l, k);
    int nb = 0;
    launch_smooth<R>(H.L[l], colour, src, oth, dst, H.csum_cur(l), H.csum_alt(l), H.part(l, k ^ 1), H.pend_nb[l],
                     H.pend_col[l], rs, sc, nl, C.st, &nb, sc.jacobi ? 0 : H.tiled);
    if (e1)
        (void)hipEventRecord(e1, C.st);
    H.cur[l][colour] = 1 - own;
    H.cs[l] ^= 1;
    H.pend_col[l] = colour;
    H.pend_nb[l] = nb;
    H.next_part[l] = k ^ 1;
}

// One full sweep of level l: both colours in one launch where the level
// takes the fused sweep, else two half-sweeps.
template <typename R>
static void sweep(Ctx &C, Hier<R> &H, int l, SolveConsts sc, bool nl)
{
    if (H.fused && !sc.jacobi && sweep2_fits(H.L[l].n, (int)sizeof(R))) {
        const long long half = H.L[l].half;
        const int orr = H.cur[l][0], ob = H.cur[l][1];
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (l == 0 && g_kt.on.load(std::memory_order_relaxed)) {
            std::lock_guard<std::mutex> g(g_kt.mu);
            if (g_kt.used + 2 <= g_kt.pool.size()) {
                e0 = g_kt.pool[g_kt.used];
                e1 = g_kt.pool[g_kt.used + 1];
                g_kt.used += 2;
                g_kt.slot_of_pair.push_back(4 + (sizeof(R) == 4 ? 1 : 0) + (nl ? 0 : 2));
            }
        }
        if (e0)
            (void)hipEventRecord(e0, C.st);
        ReduceSlot rs = C.rs;
        const int k = H.next_part[l];
        rs.partials = H.part(l, k);
        int nb = 0;
        const bool done = launch_sweep2<R>(H.L[l], H.buf[l][orr], H.buf[l][ob] + half, H.buf[l][1 - orr],
                                           H.buf[l][1 - ob] + half, H.csum_cur(l), H.csum_alt(l), H.part(l, k ^ 1),
                                           H.pend_nb[l], H.pend_col[l], rs, sc, nl, C.st, &nb);
        if (e1)
            (void)hipEventRecord(e1, C.st);
        if (done) {
            H.cur[l][0] = 1 - orr;
            H.cur[l][1] = 1 - ob;
            H.cs[l] ^= 1;
            H.pend_col[l] = 2;
            H.pend_nb[l] = nb;
            H.next_part[l] = k ^ 1;
            return;
        }
    }
    smooth(C, H, l, 0, sc, nl);
    smooth(C, H, l, 1, sc, nl);
}

constexpr int kCoarseSweeps = 100;

// V-cycle below level l (level l's tau and csum are set).  Levels below get
// their x from restriction into buffer 0.
template <typename R>
static void vcycle_from(Ctx &C, Hier<R> &H, int l, const pm_mg_opts &o, SolveConsts sc, bool nl)
{
    if (l >= H.block_l0 && l < H.nlev - 1) {
        const int bits = H.cur[l][0] | (H.cur[l][1] << 1);
        launch_block_cycle<R>(H.block(), l, false, o.n_pre, o.n_post, sc, nl, H.csum_cur(l), bits, kCoarseSweeps,
                              C.st);
        const int f = (o.n_pre + o.n_post) & 1;
        H.cur[l][0] ^= f;
        H.cur[l][1] ^= f;
        return;
    }
    if (l == H.nlev - 1) {
        launch_coarsest<R>(H.L[l], H.xr(l), H.xb(l), sc, nl, kCoarseSweeps, C.st);
        return;
    }
    for (int s = 0; s < o.n_pre; s++)
        sweep(C, H, l, sc, nl);
    H.cur[l + 1][0] = H.cur[l + 1][1] = 0;
    launch_residual_restrict<R>(H.L[l], H.xr(l), H.xb(l), H.csum_cur(l), H.L[l + 1], H.xr(l + 1), H.xb(l + 1), C.rs,
                                sc, nl, C.st, false, H.tiled);
    launch_fas_tau<R>(H.L[l + 1], H.xr(l + 1), H.xb(l + 1), H.csum_cur(l + 1), C.rs, sc, nl, false, C.st, H.tiled);
    H.fresh(l + 1);
    vcycle_from(C, H, l + 1, o, sc, nl);
    launch_prolong_correct<R>(H.L[l], H.xr(l), H.xb(l), H.L[l + 1], H.xr(l + 1), H.xb(l + 1), C.st, H.tiled);
    for (int s = 0; s < o.n_post; s++)
        sweep(C, H, l, sc, nl);
}

// Full multigrid start from a zero iterate: each level's problem takes the
// restricted source of the level above (the level-0 tau, if any, restricted
// down; zero otherwise), the coarsest is solved, and each finer level starts
// from the prolongated solution of the coarser one and gets one V-cycle.
template <typename R>
static void fmg_start(Ctx &C, Hier<R> &H, const pm_mg_opts &o, SolveConsts sc, bool nl)
{
    const int L = H.nlev;
    for (int l = 1; l < L; l++) {
        LevelView<R> &F = H.L[l - 1], &G = H.L[l];
        if (F.tr)
            launch_restrict_field<R>(G.n, F.tr, F.tb, G.tr, G.tb, C.st);
        else
            launch_zero(G.tr, sizeof(R) * 2 * G.half, C.st);
    }
    int top = L - 2;
    if (H.block_l0 < L - 1) {
        launch_block_cycle<R>(H.block(), H.block_l0, true, o.n_pre, o.n_post, sc, nl, nullptr, 0, kCoarseSweeps, C.st);
        const int f = (o.n_pre + o.n_post) & 1;
        H.cur[H.block_l0][0] = H.cur[H.block_l0][1] = f;
        top = H.block_l0 - 1;
        if (H.block_l0 == 0) {
            // the caller smooths level 0 next: set its per-colour sums exactly
            launch_fas_tau<R>(H.L[0], H.xr(0), H.xb(0), H.csum_cur(0), C.rs, sc, nl, true, C.st, H.tiled);
            H.fresh(0);
        }
    } else {
        H.cur[L - 1][0] = H.cur[L - 1][1] = 0;
        launch_zero(H.buf[L - 1][0], sizeof(R) * 2 * H.L[L - 1].half, C.st);
        launch_coarsest<R>(H.L[L - 1], H.xr(L - 1), H.xb(L - 1), sc, nl, kCoarseSweeps, C.st);
    }
    for (int l = top; l >= 0; l--) {
        H.cur[l][0] = H.cur[l][1] = 0;
        launch_prolong_full<R>(H.L[l], H.xr(l), H.xb(l), H.L[l + 1], H.xr(l + 1), H.xb(l + 1), C.st, H.tiled);
        launch_fas_tau<R>(H.L[l], H.xr(l), H.xb(l), H.csum_cur(l), C.rs, sc, nl, true, C.st, H.tiled);
        H.fresh(l);
        vcycle_from(C, H, l, o, sc, nl);
    }
}

struct SolveOut {
    int status = PM_OK, vcycles = 0;
    double rel = 0.0, hist[64] = {}, mean_shift = 0.0;
    long long clamped = 0;
};

static void record(SolveOut &so, int i, double rel)
{
    if (i < 64)
        so.hist[i] = rel;
    so.rel = rel;
}

// Problems of one shape solved in lockstep (mg_scalar_solve_batched): slot s
// of the group has its workspace stride * s bytes after slot 0's, which the
// context C addresses; every launch covers the active slots (the device map
// lists them), and each slot's convergence test drops it from the map.  One
// problem is the group {slot 0} with stride 0: no map and plain launches.
struct GroupRun {
    int m = 1;                     // slots
    long long stride = 0;          // bytes between slots
    int *dmap = nullptr;           // device map [m] (grouped runs)
    const SolveConsts *dsc = nullptr;  // device per-slot constants (grouped runs)
    double *dgather = nullptr;     // device [m * 8]: the slots' norms, gathered for one readback
    std::vector<int> active{0};    // active slots, ascending
    std::vector<int> uploaded;     // the list the device map holds
    hipStream_t st = nullptr;      // the stream of the group's launches
    bool grouped() const { return stride != 0; }
};

// Makes G's active list this thread's launch group.  A changed list is
// copied into the device map in stream order and waited for: launches before
// it read the old map, launches after it the new one, and the host list may
// change again at once.
static int group_bind(GroupRun &G)
{
    if (!G.grouped()) {
        set_cur_group(Group());
        return PM_OK;
    }
    if (G.active.empty())
        return PM_OK;
    if (G.uploaded != G.active) {
        PM_HIP(hipMemcpyAsync(G.dmap, G.active.data(), sizeof(int) * G.active.size(), hipMemcpyHostToDevice, G.st));
        PM_HIP(hipStreamSynchronize(G.st));
        G.uploaded = G.active;
    }
    Group g;
    g.stride = G.stride;
    g.map = G.dmap;
    g.sc = G.dsc;
    g.rows = (int)G.active.size();
    set_cur_group(g);
    return PM_OK;
}

// count doubles at dev (slot 0's address) for every slot: host[s * count + q]
static int read_group(Ctx &C, const GroupRun &G, const double *dev, double *host, int count)
{
    if (!G.grouped())
        return read_out(C, dev, host, count);
    launch_gather_slots(dev, G.stride, G.m, count, G.dgather, C.st);
    return read_out(C, G.dgather, host, count * G.m);
}

// Device-to-device copy of `bytes` from src to dst (slot 0 addresses) for slot s.
static int slot_copy(Ctx &C, const GroupRun &G, int s, void *dst, const void *src, size_t bytes)
{
    const long long o = (long long)s * G.stride;
    PM_HIP(launch_copy_bytes((char *)dst + o, (const char *)src + o, bytes, C.st));
    return PM_OK;
}

// FP64 solve of one field held packed in `master` (initial guess in, solution
// out), for every active slot of G.  src_norm[s] = ||beta delta / nu||_2 of
// slot s; limit[s]: its V-cycle budget (null: o.max_vcycles).  mean_set: the
// fine level's lagged mean already holds the exact mean of Lq of the guess
// (the mixed solve's last outer step wrote it), so it is not evaluated again.
static int solve_f64(Ctx &C, GroupRun &G, double *master, SolveConsts sc, bool nl, const pm_mg_opts &o,
                     const double *src_norm, SolveOut *so, bool zero_start, const int *limit = nullptr,
                     bool mean_set = false)
{
    int e = group_bind(G);
    if (e)
        return e;
    Hier<double> H;
    build_hier64(C, H, master);
    if (sc.jacobi)  // (the single-workgroup coarse cycle smooths by Gauss-Seidel only)
        H.block_l0 = kMaxLevels;
    const long long N = C.P.N;
    int fmg = 0;
    if (zero_start && o.max_vcycles > 0) {
        fmg_start<double>(C, H, o, sc, nl);  // counts as the first V-cycle
        fmg = 1;
    } else {
        // exact mean of Lq on the fine level for the first half-sweep
        if (!mean_set)
            launch_fas_tau<double>(H.L[0], H.xr(0), H.xb(0), H.csum_cur(0), C.rs, sc, nl, true, C.st, H.tiled);
        H.fresh(0);
    }
    std::vector<double> out(4 * (size_t)G.m);
    const long long half = H.L[0].half;
    for (int it = fmg;; it++) {
        for (int s = 0; s < o.n_pre; s++)
            sweep(C, H, 0, sc, nl);
        H.cur[1][0] = H.cur[1][1] = 0;
        launch_residual_restrict<double>(H.L[0], H.xr(0), H.xb(0), H.csum_cur(0), H.L[1], H.xr(1), H.xb(1), C.rs, sc,
                                         nl, C.st, true, H.tiled);
        e = read_group(C, G, C.rs.out, out.data(), 4);
        if (e)
            return e;
        std::vector<int> next;
        for (int s : G.active) {
            const double *q = &out[(size_t)s * 4];
            SolveOut &r = so[s];
            const double r2 = fmax(q[0] - q[1] * q[1] / (double)N, 0.0);
            const double rel = sqrt(r2) / src_norm[s];
            record(r, it - fmg, rel);
            r.mean_shift = q[2] / (double)N;
            r.clamped = (long long)q[3];
            bool done = true;
            if (!isfinite(rel))
                r.status = PM_ENONFINITE;
            else if (rel <= o.rel_tol)
                r.status = PM_OK;
            else if (it >= (limit ? limit[s] : o.max_vcycles))
                r.status = PM_ENOCONV;
            else
                done = false;
            if (!done) {
                next.push_back(s);
                continue;
            }
            r.vcycles = it;
            // bring both colours back into the master buffer
            if (H.cur[0][0] && (e = slot_copy(C, G, s, master, H.buf[0][1], sizeof(double) * half)))
                return e;
            if (H.cur[0][1] && (e = slot_copy(C, G, s, master + half, H.buf[0][1] + half, sizeof(double) * half)))
                return e;
        }
        G.active = next;
        if (G.active.empty())
            break;
        if ((e = group_bind(G)))
            return e;
        launch_fas_tau<double>(H.L[1], H.xr(1), H.xb(1), H.csum_cur(1), C.rs, sc, nl, false, C.st, H.tiled);
        H.fresh(1);
        vcycle_from(C, H, 1, o, sc, nl);
        launch_prolong_correct<double>(H.L[0], H.xr(0), H.xb(0), H.L[1], H.xr(1), H.xb(1), C.st, H.tiled);
        for (int s = 0; s < o.n_post; s++)
            sweep(C, H, 0, sc, nl);
    }
    return launched();
}

// Mixed precision.  Every outer step evaluates the FP64 residual of the FP64
// iterate (convergence test included) and hands the defect to kMixedInner
// FP32 V-cycles whose result corrects the FP64 iterate.
//  - Linear problems (Poisson, linearised option): the FP32 V-cycle solves
//    the correction equation lap e = r from e = 0, so the iteration has no
//    FP32 floor.
//  - The nonlinear scalar field: the FP32 level carries the full
//    approximation (FAS), which is accurate only down to the FP32 rounding
//    of the iterate's Laplacian (~1e-6 relative residual on fine grids).
//    Once the FP64 residual is within `kMixedSwitch` of that floor, or a
//    cycle stops paying (reduction worse than 0.6), the remaining V-cycles
//    run in FP64.
constexpr double kMixedSwitchNL = 3e-6;
constexpr int kMixedInner = 2;        // FP32 V-cycles per outer step
constexpr double kMixedStall = 0.36;  // an outer step must reduce the residual at least this much (0.6 per V-cycle)

// final_residual = false: once the cycle budget is spent, the last outer
// residual (which changes nothing but the report) and its readback are
// skipped; for callers that read no residual.  zero_start: the master
// iterate holds zeros (every caller clears it first) and the first V-cycle
// is a full-multigrid start.  For every active slot of G
// (see solve_f64); slots that finish in FP64 do so together, after the FP32
// phase of the whole group.
static int solve_mixed(Ctx &C, GroupRun &G, double *master, SolveConsts sc, bool nl, const pm_mg_opts &o,
                       const double *src_norm, SolveOut *so, bool zero_start, bool final_residual = true)
{
    int e = group_bind(G);
    if (e)
        return e;
    Hier<float> H;
    build_hier32(C, H);
    if (sc.jacobi)
        H.block_l0 = kMaxLevels;
    const long long N = C.P.N;
    LevelView<double> F64 = make_view<double>(C.P.n[0], 1.0 / C.P.n[0], C.at<double>(C.P.delta64[0]), nullptr, nullptr);
    const long long half = F64.half;
    // exact initial mean of Lq64 (zero_start: the master iterate is zero,
    // which the level's tiled kernels then take without reading it)
    launch_fas_tau<double>(F64, master, master + half, C.csum64, C.rs, sc, nl, true, C.st, H.tiled, zero_start);
    ReduceSlot ro = C.rs;
    ro.out = C.outer_out;
    // the FP32 correction equation of a linear problem has no source term
    SolveConsts sc32 = sc;
    if (!nl) {
        sc32.K = 0.0;
        sc32.beta = 0.0;
    }
    const double switch_tol = fmax(kMixedSwitchNL, 30.0 * o.rel_tol);
    std::vector<double> out(4 * (size_t)G.m), prev(G.m, 0.0);
    std::vector<int> cyc_of(G.m, 0), it_of(G.m, 0), to_f64;
    int cyc = 0;  // FP32 V-cycles (the same for every slot still in the FP32 phase)
    // The FP64 iterate lives in `cur`: the master buffer, or the level's
    // second FP64 buffer after an odd number of corrections applied out of
    // place by the tiled outer step.  `pending`: the FP32 V-cycles since the
    // last outer step have not corrected it yet (the next outer step does).
    // Applied out of place from 256^3 up: on smaller levels the separate
    // correction launch costs less than the fused loads add to the outer
    // step's latency.
    double *cur = master, *alt = C.at<double>(C.P.q64[0]);
    const bool fuse = (C.P.precs & kPrecF64) && C.P.n[0] >= 256 && mixed_outer_tiles(C.P.n[0], H.tiled);
    bool pending = false;
    auto to_master = [&](int s) {
        return cur == master ? PM_OK : slot_copy(C, G, s, master, cur, sizeof(double) * 2 * half);
    };
    for (int it = 0;; it++) {
        if (!final_residual && it > 0 && cyc >= o.max_vcycles) {
            if (pending)
                launch_mixed_correct(cur, H.xr(0), H.xb(0), half, nl, C.st);
            for (int s : G.active) {
                if ((e = to_master(s)))
                    return e;
                so[s].status = PM_ENOCONV;
                so[s].vcycles = cyc;
            }
            G.active.clear();
            break;
        }
        MixedCorr mc;
        const bool fused = pending && fuse;
        if (fused) {
            mc.vr = H.xr(0);
            mc.vb = H.xb(0);
            mc.yr = alt;
            mc.yb = alt + half;
            // x32 goes to the other buffer of each colour (v is read there)
            H.cur[0][0] ^= 1;
            H.cur[0][1] ^= 1;
        } else {
            if (pending)
                launch_mixed_correct(cur, H.xr(0), H.xb(0), half, nl, C.st);
            H.cur[0][0] = H.cur[0][1] = 0;
        }
        // (its final stage also sets the lagged means for the next outer
        // residual and the FP32 level 0)
        if (!launch_mixed_outer_residual(F64, cur, cur + half, C.csum64, H.L[0], H.xr(0), H.xb(0), ro, sc, nl, C.st,
                                         H.tiled, C.csum64, H.csum_cur(0), fused ? &mc : nullptr,
                                         zero_start && it == 0))
            return PM_EINVAL;
        if (fused)
            std::swap(cur, alt);
        pending = false;
        H.fresh(0);
        e = read_group(C, G, C.outer_out, out.data(), 4);
        if (e)
            return e;
        std::vector<int> next;
        double rel_last = 0.0, prev_last = 0.0;
        for (int s : G.active) {
            const double *q = &out[(size_t)s * 4];
            SolveOut &r = so[s];
            const double r2 = fmax(q[0] - q[1] * q[1] / (double)N, 0.0);
            const double rel = sqrt(r2) / src_norm[s];
            record(r, it, rel);
            r.mean_shift = q[2] / (double)N;
            r.clamped = (long long)q[3];
            r.vcycles = cyc;
            bool leaves = true;  // the slot's FP32 phase ends here
            if (!isfinite(rel)) {
                r.status = PM_ENONFINITE;
            } else if (rel <= o.rel_tol) {
                r.status = PM_OK;
            } else if (cyc >= o.max_vcycles) {
                r.status = PM_ENOCONV;
            } else if (nl && (rel <= switch_tol || (it > 0 && rel > kMixedStall * prev[s]))) {
                cyc_of[s] = cyc;
                it_of[s] = it;
                to_f64.push_back(s);
            } else {
                prev_last = prev[s];
                rel_last = rel;
                prev[s] = rel;
                next.push_back(s);
                leaves = false;
            }
            if (leaves && (e = to_master(s)))
                return e;
        }
        G.active = next;
        if (G.active.empty())
            break;
        if ((e = group_bind(G)))
            return e;
        // kMixedInner FP32 V-cycles per FP64 defect correction: the FP64
        // residual and correction are paid once for all of them.  A linear
        // problem converges at a steady rate per V-cycle; when one cycle at
        // the last outer step's rate (with a 2x margin) reaches the tolerance,
        // the final outer step runs one cycle only.  Only with one problem
        // active: members of a lockstep group run the same cycles.
        int inner = kMixedInner;
        if (!nl && G.active.size() == 1 && it >= 2 && prev_last > 0.0) {  // (the first step includes the FMG start)
            const double per_cycle = pow(rel_last / prev_last, 1.0 / kMixedInner);
            if (per_cycle < 1.0 && 2.0 * rel_last * per_cycle <= o.rel_tol)
                inner = 1;
        }
        for (int v = 0; v < inner && cyc < o.max_vcycles; v++, cyc++) {
            if (it == 0 && v == 0 && zero_start)
                fmg_start<float>(C, H, o, sc32, nl);
            else
                vcycle_from<float>(C, H, 0, o, sc32, nl);
        }
        pending = true;
    }
    e = launched();
    if (e || to_f64.empty())
        return e;
    // finish in FP64 from the current iterates
    std::sort(to_f64.begin(), to_f64.end());
    std::vector<SolveOut> s64(G.m);
    std::vector<int> limit(G.m, 0);
    for (int s : to_f64)
        limit[s] = o.max_vcycles - cyc_of[s];
    G.active = to_f64;
    e = solve_f64(C, G, master, sc, nl, o, src_norm, s64.data(), false, limit.data(), true);
    if (e)
        return e;
    for (int s : to_f64) {
        SolveOut &r = so[s];
        // the FP64 phase's residuals follow the FP32 phase's, from the
        // switching outer step's own
        for (int i = 0; i <= s64[s].vcycles && it_of[s] + i < 64; i++)
            r.hist[it_of[s] + i] = s64[s].hist[i];
        r.vcycles = cyc_of[s] + s64[s].vcycles;
        r.rel = s64[s].rel;
        r.status = s64[s].status;
        r.mean_shift = s64[s].mean_shift;
        r.clamped = s64[s].clamped;
    }
    return PM_OK;
}

// coarse delta levels (8-cell averages) and FP32 copies from the fine level
static void delta_levels(Ctx &C)
{
    const Plan &P = C.P;
    for (int l = 1; l < P.nlev; l++) {
        const long long fh = (long long)P.n[l - 1] * P.n[l - 1] * (P.n[l - 1] / 2);
        const long long ch = (long long)P.n[l] * P.n[l] * (P.n[l] / 2);
        double *f = C.at<double>(P.delta64[l - 1]);
        double *c = C.at<double>(P.delta64[l]);
        launch_restrict_field<double>(P.n[l], f, f + fh, c, c + ch, C.st);
    }
    if (P.precs & kPrecMixed)
        for (int l = 0; l < P.nlev; l++)
            launch_cast_f64_f32(C.at<double>(P.delta64[l]), C.at<float>(P.d32[l]),
                                (long long)P.n[l] * P.n[l] * P.n[l], C.st);
}

// delta hierarchy from the packed fine delta (mean removed here) + FP32 copy
// after_mean (optional) is called once the fine delta is mean-free on C.st,
// before the coarse levels and the norm: work that needs only the fine delta
// can start there.
static int prepare_delta(Ctx &C, double *delta_sq_sum, const std::function<int()> &after_mean = nullptr)
{
    const Plan &P = C.P;
    double *d0 = C.at<double>(P.delta64[0]);
    launch_field_sum(d0, P.N, C.rs, C.st);
    launch_subtract_mean(d0, P.N, C.rs.out, C.st);
    if (after_mean) {
        const int e = after_mean();
        if (e)
            return e;
    }
    delta_levels(C);
    launch_field_sum(d0, P.N, C.rs, C.st);
    double out[2];
    int e = read_out(C, C.rs.out, out, 2);
    if (e)
        return e;
    *delta_sq_sum = out[1];
    if (!isfinite(out[0]) || !isfinite(out[1]))
        return PM_ENONFINITE;
    return launched();
}

static void fill_report(pm_mg_report *rep, const SolveOut &so, float ms)
{
    if (!rep)
        return;
    memset(rep, 0, sizeof(*rep));
    rep->status = so.status;
    rep->vcycles = so.vcycles;
    rep->rel_residual = so.rel;
    for (int i = 0; i < 64; i++)
        rep->residual_hist[i] = so.hist[i];
    rep->mean_shift = so.mean_shift;
    rep->clamped_cells = so.clamped;
    rep->ms = ms;
}

static bool opts_ok(const pm_mg_opts *o)
{
    return o && o->rel_tol > 0.0 && o->max_vcycles >= 0 && o->n_pre >= 0 && o->n_post >= 0 && o->n_pre + o->n_post > 0 &&
           (o->precision == PM_PREC_F64 || o->precision == PM_PREC_MIXED) && o->guess >= PM_GUESS_ZERO &&
           o->guess <= PM_GUESS_LEARNED &&
           (o->guess != PM_GUESS_LEARNED || (o->learned_params && o->learned_ws)) &&
           (o->smoother == PM_SMOOTH_RBGS || o->smoother == PM_SMOOTH_JACOBI) &&
           o->jacobi_weight >= 0.0 && o->jacobi_weight <= 1.0;
}

// The mixed path also needs the FP64 hierarchy: the nonlinear solve finishes
// its last V-cycles in FP64.
static int prec_bits(const pm_mg_opts *o) { return o->precision == PM_PREC_MIXED ? (kPrecMixed | kPrecF64) : kPrecF64; }

// final_residual: see solve_mixed (the FP64 path always tests).
static int run_solve_group(Ctx &C, GroupRun &G, double *master, SolveConsts sc, bool nl, const pm_mg_opts &o,
                           const double *src_norm, SolveOut *so, bool zero_start, bool final_residual = true)
{
    return o.precision == PM_PREC_MIXED
               ? solve_mixed(C, G, master, sc, nl, o, src_norm, so, zero_start, final_residual)
               : solve_f64(C, G, master, sc, nl, o, src_norm, so, zero_start);
}

// One problem: the group {slot 0}.
static int run_solve(Ctx &C, double *master, SolveConsts sc, bool nl, const pm_mg_opts &o, double src_norm,
                     SolveOut &so, bool zero_start, bool final_residual = true)
{
    GroupRun G;
    return run_solve_group(C, G, master, sc, nl, o, &src_norm, &so, zero_start, final_residual);
}

// Solve constants with the smoother the options ask for.
static SolveConsts consts(double nu, double K, double beta, const pm_mg_opts &o)
{
    SolveConsts sc{nu, K, beta};
    if (o.smoother == PM_SMOOTH_JACOBI) {
        sc.jacobi = 1;
        sc.omega = o.jacobi_weight > 0.0 ? o.jacobi_weight : 0.6;
    }
    return sc;
}

// Poisson: lap psi = s delta (nu = 1, K = 0, beta = s).
static int poisson_core(Ctx &C, const pm_eft_coeffs &cf, const pm_mg_opts &o, SolveOut &so, double dsq)
{
    double *m = C.at<double>(C.P.psi64);
    if (o.guess != PM_GUESS_GIVEN)
        launch_zero(m, sizeof(double) * C.P.N, C.st);
    SolveConsts sc = consts(1.0, 0.0, cf.s, o);
    const double src = fabs(cf.s) * sqrt(dsq);
    if (src == 0.0) {
        launch_zero(m, sizeof(double) * C.P.N, C.st);
        so = SolveOut();
        return launched();
    }
    return run_solve(C, m, sc, false, o, src, so, o.guess != PM_GUESS_GIVEN);
}

static int learned_ok(int ng, const pm_mg_opts &o)
{
    if (ng % 64 || ng < 64)
        return PM_EINVAL;
    if (o.learned_ws_bytes < ws_unet_workspace_bytes(ng, 0))
        return PM_ENOMEM;
    return PM_OK;
}

// Learned warm start: one linear full-multigrid pass on
// nu lap chi0 = xi s (delta + t - <t>), t from the network.  forward_done: the
// network's forward pass was already issued (and waited for) by the caller.
// separate: the pass's delta is built in the plan's second delta hierarchy
// (step plans), so the shared one is never modified and a concurrent solve
// may read it; otherwise delta is modified in place and restored afterwards.
static int learned_guess(Ctx &C, const pm_eft_params &p, const pm_eft_coeffs &cf, const pm_mg_opts &o, double src,
                         bool forward_done, bool separate)
{
    const int ng = C.P.ng;
    int e = learned_ok(ng, o);
    if (e)
        return e;
    double *d0 = C.at<double>(C.P.delta64[0]);
    double *save = unet_save_area(o.learned_ws, ng);
    if (!forward_done) {
        e = unet_learned_forward(o.learned_params, d0, save, ng, p, o.learned_ws, o.learned_ws_bytes, C.st);
        if (e)
            return e;
    }
    Ctx G = C;  // the guess pass: C's solve region, its own delta when separate
    if (separate) {
        if (!C.P.dalt64[0])
            return PM_EINVAL;
        for (int l = 0; l < C.P.nlev; l++) {
            G.P.delta64[l] = C.P.dalt64[l];
            G.P.d32[l] = C.P.dalt32[l];
        }
        PM_HIP(launch_copy_bytes(G.at<double>(G.P.delta64[0]), save, sizeof(double) * C.P.N, C.st));
    }
    e = unet_add_learned_source(o.learned_ws, ng, G.at<double>(G.P.delta64[0]), C.st);
    if (e)
        return e;
    delta_levels(G);
    pm_mg_opts lo = o;
    lo.rel_tol = 1e-30;  // the pass itself, no convergence test
    lo.max_vcycles = 1;
    SolveOut tmp;
    e = run_solve(G, C.at<double>(C.P.chi64), consts(cf.nu, 0.0, cf.xi * cf.s, o), false, lo, src, tmp, true, false);
    if (e)
        return e;
    if (separate)
        return launched();
    PM_HIP(launch_copy_bytes(d0, save, sizeof(double) * C.P.N, C.st));
    delta_levels(C);
    return launched();
}

// Scalar field: nu lap chi - xi s delta - K N(chi) = 0 (beta = xi s).
static int scalar_core(Ctx &C, const pm_eft_params &p, const pm_eft_coeffs &cf, const pm_mg_opts &o, SolveOut &so,
                       double dsq, bool forward_done = false, bool separate_delta = false)
{
    double *m = C.at<double>(C.P.chi64);
    so = SolveOut();
    if (cf.xi == 0.0) {
        launch_zero(m, sizeof(double) * C.P.N, C.st);
        return launched();
    }
    const bool nl = cf.K != 0.0;
    const double src = fabs(cf.xi * cf.s / cf.nu) * sqrt(dsq);
    if (src == 0.0) {
        launch_zero(m, sizeof(double) * C.P.N, C.st);
        return launched();
    }
    SolveConsts sc = consts(cf.nu, cf.K, cf.xi * cf.s, o);
    if (o.guess != PM_GUESS_GIVEN)
        launch_zero(m, sizeof(double) * C.P.N, C.st);
    if (o.guess == PM_GUESS_LEARNED && nl) {
        int e = learned_guess(C, p, cf, o, src, forward_done, separate_delta);
        if (e)
            return e;
        return run_solve(C, m, sc, nl, o, src, so, false);
    }
    if (o.guess == PM_GUESS_LINEAR && nl) {
        pm_mg_opts lo = o;
        lo.rel_tol = 1e-3;
        lo.max_vcycles = 4;
        SolveOut tmp;
        SolveConsts lin = consts(cf.nu, 0.0, cf.xi * cf.s, o);
        int e = run_solve(C, m, lin, false, lo, src, tmp, true);
        if (e)
            return e;
    }
    return run_solve(C, m, sc, nl, o, src, so, o.guess == PM_GUESS_ZERO || o.guess == PM_GUESS_LEARNED);
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s)
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, st);
    }
    float stop()
    {
        mark();
        return ms();
    }
    // end of the timed span, read later with ms() (no host wait here)
    void mark() { (void)hipEventRecord(b, st); }
    float ms()
    {
        float v = 0.f;
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&v, a, b);
        return v;
    }
    ~Timer()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

static int grid_solve(const void *rho, int ng, pm_dtype dt, const pm_eft_params *p, const pm_mg_opts *o, void *out,
                      pm_mg_report *rep, void *ws, size_t wsb, pm_stream_t stream, bool scalar)
{
    if (!rho || !p || !out || !opts_ok(o) || (dt != PM_F32 && dt != PM_F64))
        return PM_EINVAL;
    pm_eft_coeffs cf;
    int e = coefficients(*p, cf);
    if (e == PM_EINVAL || (scalar && e == PM_EUNSTABLE))
        return e;
    Ctx C;
    e = setup_ctx(C, ws, wsb, ng, 0, dt, prec_bits(o), stream);
    if (e)
        return e;
    Timer tm(C.st);
    // rho -> packed delta = rho - 1 (mean removed in prepare_delta)
    launch_natural_to_packed(rho, dt, C.at<double>(C.P.delta64[0]), ng, 1.0, -1.0, C.st);
    double dsq = 0.0;
    e = prepare_delta(C, &dsq);
    if (e)
        return e;
    double *m = C.at<double>(scalar ? C.P.chi64 : C.P.psi64);
    if (o->guess == PM_GUESS_GIVEN)
        launch_natural_to_packed(out, dt, m, ng, 1.0, 0.0, C.st);
    SolveOut so;
    e = scalar ? scalar_core(C, *p, cf, *o, so, dsq) : poisson_core(C, cf, *o, so, dsq);
    if (e)
        return e;
    launch_field_sum(m, C.P.N, C.rs, C.st);
    launch_packed_to_natural(m, out, dt, ng, 0.0, C.rs.out, C.st);
    e = launched();
    if (e)
        return e;
    fill_report(rep, so, tm.stop());
    return so.status;
}

}  // namespace pmeft

using namespace pmeft;

extern "C" {

int pm_eft_coefficients(const pm_eft_params *p, pm_eft_coeffs *out)
{
    if (!p || !out)
        return PM_EINVAL;
    return coefficients(*p, *out);
}

int pm_grid_levels(int ng) { return grid_levels(ng); }

size_t pm_workspace_bytes(int ng, long long np, pm_dtype dtype, pm_prec prec)
{
    Plan P;
    const int bits = prec == PM_PREC_F64 ? kPrecF64 : (kPrecF64 | kPrecMixed);
    if (!make_plan(P, ng, np < 0 ? 0 : np, dtype, bits))
        return 0;
    return P.total;
}

size_t pm_sort_workspace_bytes(long long np, pm_dtype dtype)
{
    if (np <= 0 || np > (1LL << 30) || (dtype != PM_F32 && dtype != PM_F64))
        return 0;
    return sort_workspace_bytes((unsigned long long)np, dtype == PM_F64 ? 8 : 4);
}

int pm_sort_particles(void *pos, void *vel, long long *ids, long long np, int ng, pm_dtype dtype, void *ws,
                      size_t ws_bytes, pm_stream_t stream)
{
    if (!pos || !ws || ((uintptr_t)ws & 255) || np <= 0 || np > (1LL << 30) || ng < 8 || ng > 1024 ||
        (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    if (ws_bytes < pm_sort_workspace_bytes(np, dtype))
        return PM_ENOMEM;
    return launch_sort_particles(pos, vel, ids, (unsigned)np, ng, dtype, (char *)ws, (hipStream_t)stream);
}

int pm_deposit(const void *pos, long long np, pm_dtype dtype, int ng, void *rho, void *ws, size_t ws_bytes,
               pm_stream_t stream)
{
    if (!pos || !rho || np <= 0 || np > (1LL << 30) || (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    Ctx C;
    int e = setup_ctx(C, ws, ws_bytes, ng, np, dtype, 0, stream);
    if (e)
        return e;
    unsigned long long *acc = C.at<unsigned long long>(C.P.fixacc);
    launch_deposit_auto(pos, np, dtype, ng, acc, C.ws + C.P.depidx, C.st);
    double *d0 = C.at<double>(C.P.delta64[0]);
    launch_fixed_to_delta(acc, ng, (double)C.P.N / (double)np, d0, C.rs, C.st);
    // rho = delta_raw + 1 in natural order
    launch_packed_to_natural(d0, rho, dtype, ng, 1.0, nullptr, C.st);
    e = launched();
    if (e)
        return e;
    return PM_OK;
}

int mg_poisson_solve(const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p, const pm_mg_opts *opts,
                     void *psi, pm_mg_report *rep, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    return grid_solve(rho, ng, dtype, p, opts, psi, rep, ws, ws_bytes, stream, false);
}

int mg_scalar_solve(const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p, const pm_mg_opts *opts,
                    void *chi, pm_mg_report *rep, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    return grid_solve(rho, ng, dtype, p, opts, chi, rep, ws, ws_bytes, stream, true);
}

int ws_unet_guess(const float *params, const void *rho, int ng, pm_dtype dtype, const pm_eft_params *p,
                  void *chi0_out, void *learned_ws, size_t learned_ws_bytes, void *ws, size_t ws_bytes,
                  pm_stream_t stream)
{
    if (!params || !learned_ws || !rho || !p || !chi0_out || (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    pm_eft_coeffs cf;
    int e = coefficients(*p, cf);
    if (e)
        return e;
    Ctx C;
    e = setup_ctx(C, ws, ws_bytes, ng, 0, dtype, kPrecF64, stream);
    if (e)
        return e;
    launch_natural_to_packed(rho, dtype, C.at<double>(C.P.delta64[0]), ng, 1.0, -1.0, C.st);
    double dsq = 0.0;
    e = prepare_delta(C, &dsq);
    if (e)
        return e;
    double *m = C.at<double>(C.P.chi64);
    launch_zero(m, sizeof(double) * C.P.N, C.st);
    const double src = cf.nu != 0.0 ? fabs(cf.xi * cf.s / cf.nu) * sqrt(dsq) : 0.0;
    if (cf.xi != 0.0 && cf.K != 0.0 && src > 0.0) {  // (otherwise no learned guess: chi_0 = 0)
        pm_mg_opts o{};
        o.rel_tol = 1e-30;
        o.max_vcycles = 1;
        o.n_pre = 1;
        o.n_post = 2;
        o.precision = PM_PREC_F64;
        o.guess = PM_GUESS_LEARNED;
        o.learned_params = params;
        o.learned_ws = learned_ws;
        o.learned_ws_bytes = learned_ws_bytes;
        e = learned_guess(C, *p, cf, o, src, false, false);
        if (e)
            return e;
    }
    launch_field_sum(m, C.P.N, C.rs, C.st);
    launch_packed_to_natural(m, chi0_out, dtype, ng, 0.0, C.rs.out, C.st);
    return launched();
}

// ---- grouped batched solves ----------------------------------------------
// The library's second stream (one per device, created on first use, default
// priority, non-blocking): pm_step runs its scalar-field solve on it while the
// Poisson solve runs on the caller's stream, and a batched solve its smaller
// grids' groups beside the largest.  Overlapping calls on one device share
// it, which stays correct (each call orders its work with events of its own)
// but serialises their work on it.
namespace {
struct SideStream {
    hipStream_t s = nullptr;
};
std::mutex g_side_mu;
SideStream g_side[64][2];

// which: 0 the second stream, 1 a third one (batched solves only)
int side_stream(SideStream **out, int which = 0)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || which < 0 || which > 1)
        return PM_EHIP;
    std::lock_guard<std::mutex> g(g_side_mu);
    SideStream &S = g_side[dev][which];
    if (!S.s && hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) != hipSuccess)
        return PM_EHIP;
    *out = &S;
    return PM_OK;
}
}  // namespace

// The problems are grouped by (grid, dtype of their arrays), largest grid
// first, and each group is solved in lockstep: one launch per kernel of the
// solve covers every problem of the group still iterating (Group), each in
// its own workspace slot.  The largest group runs on the caller's stream;
// beside it the second largest on the library's second stream and the
// others, one after another, on a third (their latency-bound small grids fill
// the large group's gaps).  Each group has its own region and control area
// of the workspace.
namespace {
struct BatchGroup {
    int ng = 0;
    pm_dtype dt = PM_F32;
    std::vector<int> idx;  // problem indices
    size_t slice = 0;      // bytes per slot
};

// control area per slot: its map entry and two constants tables
constexpr size_t kBatchCtlPerSlot = sizeof(int) + 2 * sizeof(SolveConsts) + 8 * sizeof(double);

bool batch_groups(const pm_problem *probs, int nprob, int precision, std::vector<BatchGroup> &out)
{
    out.clear();
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; i++)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].ng > probs[b].ng; });
    for (int i : order) {
        BatchGroup *g = nullptr;
        for (auto &x : out)
            if (x.ng == probs[i].ng && x.dt == probs[i].dtype)
                g = &x;
        if (!g) {
            out.emplace_back();
            g = &out.back();
            g->ng = probs[i].ng;
            g->dt = probs[i].dtype;
            const size_t b = pm_workspace_bytes(g->ng, 0, g->dt, (pm_prec)precision);
            if (b == 0)
                return false;
            g->slice = (b + 255) & ~(size_t)255;
        }
        g->idx.push_back(i);
    }
    return true;
}

size_t batch_ctl_bytes(int nprob) { return ((size_t)nprob * kBatchCtlPerSlot + 4 * 256 + 255) & ~(size_t)255; }

// Workspace layout of a batch: group k's region (slots) then its control
// area, groups one after another; off[k] is group k's region offset and
// off[gs.size()] the total.
void batch_layout(const std::vector<BatchGroup> &gs, std::vector<size_t> &off)
{
    off.assign(gs.size() + 1, 0);
    for (size_t k = 0; k < gs.size(); k++)
        off[k + 1] = off[k] + gs[k].slice * gs[k].idx.size() + batch_ctl_bytes((int)gs[k].idx.size());
}

struct GroupReset {
    ~GroupReset() { set_cur_group(Group()); }
};

// One group in lockstep: the steps of grid_solve and scalar_core for every
// slot, each launch covering the slots that take it.
int solve_group(const pm_problem *probs, const BatchGroup &bg, const pm_mg_opts &o, pm_mg_report *reps,
                std::vector<int> &codes, char *region, char *ctl, hipStream_t st)
{
    const int m = (int)bg.idx.size();
    const int ng = bg.ng;
    Ctx C;
    int e = setup_ctx(C, region, bg.slice, ng, 0, bg.dt, prec_bits(&o), st);
    if (e)
        return e;
    GroupReset reset;
    GroupRun G;
    G.m = m;
    G.stride = (long long)bg.slice;
    G.st = C.st;
    G.dmap = reinterpret_cast<int *>(ctl);
    // control area: map [m] | constants [m] | linear-guess constants [m] | gathered norms [m * 8]
    SolveConsts *dsc = reinterpret_cast<SolveConsts *>(ctl + (((size_t)m * sizeof(int) + 255) & ~(size_t)255));
    SolveConsts *dlin = dsc + m;
    G.dgather = reinterpret_cast<double *>(
        reinterpret_cast<char *>(dsc) + ((2 * (size_t)m * sizeof(SolveConsts) + 255) & ~(size_t)255));
    std::vector<pm_eft_coeffs> cf(m);
    std::vector<SolveConsts> tsc(m), tlin(m);
    std::vector<double> dsq(m, 0.0), src(m, 0.0);
    std::vector<SolveOut> so(m);
    std::vector<int> live;  // slots still in the run
    for (int s = 0; s < m; s++) {
        const int i = bg.idx[s];
        const int ce = coefficients(probs[i].p, cf[s]);
        if (ce == PM_EINVAL || ce == PM_EUNSTABLE) {
            codes[i] = ce;
            continue;
        }
        tsc[s] = consts(cf[s].nu, cf[s].K, cf[s].xi * cf[s].s, o);
        tlin[s] = consts(cf[s].nu, 0.0, cf[s].xi * cf[s].s, o);
        live.push_back(s);
    }
    if (live.empty())
        return PM_OK;
    PM_HIP(hipMemcpyAsync(dsc, tsc.data(), sizeof(SolveConsts) * m, hipMemcpyHostToDevice, C.st));
    PM_HIP(hipMemcpyAsync(dlin, tlin.data(), sizeof(SolveConsts) * m, hipMemcpyHostToDevice, C.st));
    PM_HIP(hipStreamSynchronize(C.st));
    const long long N = C.P.N;
    const size_t esz = bg.dt == PM_F64 ? sizeof(double) : sizeof(float);
    double *stage = C.at<double>(C.P.psi64);  // natural-order staging of rho and chi (the scalar solve leaves psi free)
    double *d0 = C.at<double>(C.P.delta64[0]);
    double *m0 = C.at<double>(C.P.chi64);
    auto bind = [&](const std::vector<int> &slots) {
        G.active = slots;
        return group_bind(G);
    };
    // a problem's array <-> its slot's staging area
    auto stage_in = [&](int s, const void *user) {
        return hipMemcpyAsync((char *)stage + (long long)s * G.stride, user, esz * N, hipMemcpyDeviceToDevice, C.st) ==
                       hipSuccess
                   ? PM_OK
                   : PM_EHIP;
    };
    auto stage_out = [&](int s, void *user) {
        return hipMemcpyAsync(user, (const char *)stage + (long long)s * G.stride, esz * N, hipMemcpyDeviceToDevice,
                              C.st) == hipSuccess
                   ? PM_OK
                   : PM_EHIP;
    };
    Timer tm(C.st);
    // rho -> packed delta = rho - 1, mean removed, coarse levels, norms
    for (int s : live)
        if ((e = stage_in(s, probs[bg.idx[s]].rho)))
            return e;
    if ((e = bind(live)))
        return e;
    launch_zero(C.ws + C.P.red_counter, 256, C.st);
    launch_natural_to_packed(stage, bg.dt, d0, ng, 1.0, -1.0, C.st);
    launch_field_sum(d0, N, C.rs, C.st);
    launch_subtract_mean(d0, N, C.rs.out, C.st);
    delta_levels(C);
    launch_field_sum(d0, N, C.rs, C.st);
    std::vector<double> out(2 * (size_t)m);
    if ((e = read_group(C, G, C.rs.out, out.data(), 2)))
        return e;
    std::vector<int> ok, zero, nlset, linset;
    for (int s : live) {
        if (!isfinite(out[2 * s]) || !isfinite(out[2 * s + 1])) {
            codes[bg.idx[s]] = PM_ENONFINITE;
            continue;
        }
        dsq[s] = out[2 * s + 1];
        ok.push_back(s);
        src[s] = fabs(cf[s].xi * cf[s].s / cf[s].nu) * sqrt(dsq[s]);
        if (cf[s].xi == 0.0 || src[s] == 0.0)
            zero.push_back(s);
        else
            (cf[s].K != 0.0 ? nlset : linset).push_back(s);
    }
    if (ok.empty())
        return launched();
    if (o.guess == PM_GUESS_GIVEN) {
        for (int s : ok)
            if ((e = stage_in(s, probs[bg.idx[s]].chi)))
                return e;
        if ((e = bind(ok)))
            return e;
        launch_natural_to_packed(stage, bg.dt, m0, ng, 1.0, 0.0, C.st);
    }
    if (!zero.empty()) {  // no source: chi = 0
        if ((e = bind(zero)))
            return e;
        launch_zero(m0, sizeof(double) * N, C.st);
    }
    G.dsc = dsc;
    // the nonlinear members in lockstep, then the linear ones (screening off)
    // one at a time: a linear mixed-precision solve may end with one FP32
    // cycle instead of two, which members would decide differently
    std::vector<std::vector<int>> runs;
    if (!nlset.empty())
        runs.push_back(nlset);
    for (int s : linset)
        runs.push_back({s});
    for (const auto &set : runs) {
        const bool nl = cf[set[0]].K != 0.0;
        if (o.guess != PM_GUESS_GIVEN) {
            if ((e = bind(set)))
                return e;
            launch_zero(m0, sizeof(double) * N, C.st);
        }
        if (o.guess == PM_GUESS_LINEAR && nl) {
            pm_mg_opts lo = o;
            lo.rel_tol = 1e-3;
            lo.max_vcycles = 4;
            std::vector<SolveOut> tmp(m);
            G.dsc = dlin;
            G.active = set;
            e = run_solve_group(C, G, m0, tlin[set[0]], false, lo, src.data(), tmp.data(), true);
            G.dsc = dsc;
            if (e)
                return e;
        }
        G.active = set;
        e = run_solve_group(C, G, m0, tsc[set[0]], nl, o, src.data(), so.data(),
                            o.guess == PM_GUESS_ZERO || o.guess == PM_GUESS_LEARNED);
        if (e)
            return e;
    }
    // packed chi -> natural (mean removed) -> the problems' arrays
    G.dsc = nullptr;
    if ((e = bind(ok)))
        return e;
    launch_field_sum(m0, N, C.rs, C.st);
    launch_packed_to_natural(m0, stage, bg.dt, ng, 0.0, C.rs.out, C.st);
    if ((e = launched()))
        return e;
    for (int s : ok)
        if ((e = stage_out(s, probs[bg.idx[s]].chi)))
            return e;
    const float ms = tm.stop();
    for (int s : ok) {
        const int i = bg.idx[s];
        codes[i] = so[s].status;
        if (reps)
            fill_report(&reps[i], so[s], ms);
    }
    return launched();
}
}  // namespace

size_t mg_batched_workspace_bytes(const pm_problem *probs, int nprob, int precision)
{
    if (!probs || nprob <= 0 || (precision != PM_PREC_F64 && precision != PM_PREC_MIXED))
        return 0;
    std::vector<BatchGroup> gs;
    if (!batch_groups(probs, nprob, precision, gs))
        return 0;
    std::vector<size_t> off;
    batch_layout(gs, off);
    return off.back();
}

int mg_scalar_solve_batched(const pm_problem *probs, int nprob, const pm_mg_opts *opts, pm_mg_report *reps, void *ws,
                            size_t ws_bytes, pm_stream_t stream)
{
    if (!probs || nprob <= 0 || !opts_ok(opts) || opts->guess == PM_GUESS_LEARNED || !ws || ((uintptr_t)ws & 255))
        return PM_EINVAL;
    for (int i = 0; i < nprob; i++)
        if (!probs[i].rho || !probs[i].chi || (probs[i].dtype != PM_F32 && probs[i].dtype != PM_F64))
            return PM_EINVAL;
    const size_t need = mg_batched_workspace_bytes(probs, nprob, opts->precision);
    if (need == 0)
        return PM_EINVAL;
    if (ws_bytes < need)
        return PM_ENOMEM;
    std::vector<BatchGroup> gs;
    if (!batch_groups(probs, nprob, opts->precision, gs))
        return PM_EINVAL;
    std::vector<size_t> off;
    batch_layout(gs, off);
    std::vector<int> codes(nprob, PM_OK);  // (the groups write disjoint entries)
    auto run = [&](size_t k, hipStream_t st) {
        char *region = (char *)ws + off[k];
        return solve_group(probs, gs[k], *opts, reps, codes, region, region + gs[k].slice * gs[k].idx.size(), st);
    };
    if (reps)
        for (int i = 0; i < nprob; i++)
            memset(&reps[i], 0, sizeof(reps[i]));
    int e = PM_OK;
    if (gs.size() == 1) {
        e = run(0, (hipStream_t)stream);
    } else {
        // the second largest group on the second stream, the rest one after
        // another on a third, each from a worker thread (a group reads back
        // its norms from the host between its steps)
        const int nside = gs.size() > 2 ? 2 : 1;
        SideStream *S[2] = {nullptr, nullptr};
        for (int q = 0; q < nside; q++)
            if ((e = side_stream(&S[q], q)))
                return e;
        int dev = 0;
        PM_HIP(hipGetDevice(&dev));
        hipEvent_t ready = nullptr, done = nullptr;
        PM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(ready);
            return PM_EHIP;
        }
        bool ordered = hipEventRecord(ready, (hipStream_t)stream) == hipSuccess;
        for (int q = 0; q < nside; q++)
            ordered = ordered && hipStreamWaitEvent(S[q]->s, ready, 0) == hipSuccess;
        if (!ordered) {
            (void)hipEventDestroy(ready);
            (void)hipEventDestroy(done);
            return PM_EHIP;
        }
        int ex[2] = {PM_OK, PM_OK};
        auto rest = [&](int q) {
            if (hipSetDevice(dev) != hipSuccess) {
                ex[q] = PM_EHIP;
                return;
            }
            const size_t k0 = 1 + (size_t)q, k1 = q == 0 && nside == 2 ? 2 : gs.size();
            for (size_t k = k0; k < k1 && !ex[q]; k++)
                ex[q] = run(k, S[q]->s);
        };
        std::thread worker[2];
        bool threaded[2] = {false, false};
        for (int q = 0; q < nside; q++) {
            try {
                worker[q] = std::thread(rest, q);
                threaded[q] = true;
            } catch (...) {  // no thread: the same work from this thread, after the largest group's
            }
        }
        e = run(0, (hipStream_t)stream);
        for (int q = 0; q < nside; q++) {
            if (threaded[q])
                worker[q].join();
            else
                rest(q);
        }
        // on every path the caller's stream waits for the side streams' work
        bool waited = true;
        for (int q = 0; q < nside; q++)
            waited = waited && hipEventRecord(done, S[q]->s) == hipSuccess &&
                     hipStreamWaitEvent((hipStream_t)stream, done, 0) == hipSuccess;
        (void)hipEventDestroy(ready);
        (void)hipEventDestroy(done);
        for (int q = 0; q < nside && !e; q++)
            e = ex[q];
        if (!e && !waited)
            e = PM_EHIP;
    }
    if (e)
        return e;
    int rc = PM_OK;
    for (int i = 0; i < nprob; i++) {
        if (codes[i] != PM_OK && codes[i] != PM_ENOCONV && (rc == PM_OK || rc == PM_ENOCONV))
            rc = codes[i];
        else if (codes[i] == PM_ENOCONV && rc == PM_OK)
            rc = PM_ENOCONV;
    }
    return rc;
}

// ---- autotuner ------------------------------------------------------------
// Synthetic density for timing: rho = 0.2 + 1.6 u per cell with u uniform in
// [0, 1) from an integer hash of the cell index (mean 1, rough at every
// scale), so that full multigrid + 3 V-cycles converge like a real field and
// the mixed solve stays in its FP32 cycles while it is timed.
__device__ __forceinline__ unsigned hash32(unsigned x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void k_synth_rho(double *rho, int n)
{
    const unsigned long long n3 = (unsigned long long)n * n * n;
    for (unsigned long long e = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; e < n3;
         e += (unsigned long long)gridDim.x * blockDim.x)
        rho[e] = 0.2 + 1.6 * ((double)hash32((unsigned)e * 2654435761u + 12345u) * (1.0 / 4294967296.0));
}

size_t pm_autotune_workspace_bytes(int ng, int precision)
{
    if (precision != PM_PREC_F64 && precision != PM_PREC_MIXED)
        return 0;
    const size_t b = pm_workspace_bytes(ng, 0, PM_F64, (pm_prec)precision);
    if (b == 0)
        return 0;
    return ((b + 255) & ~(size_t)255) + 2 * (((sizeof(double) * (size_t)ng * ng * ng) + 255) & ~(size_t)255);
}

int pm_get_launch_shape(int ng, int word_bytes, int *block_cycle_grid, int *tiled_smoother)
{
    if ((word_bytes != 4 && word_bytes != 8) || !block_cycle_grid || !tiled_smoother)
        return PM_EINVAL;
    const Shape sh = launch_shape(ng, word_bytes);
    *block_cycle_grid = sh.block_n;
    *tiled_smoother = sh.tiled;
    return PM_OK;
}

int pm_set_launch_shape(int ng, int word_bytes, int block_cycle_grid, int tiled_smoother)
{
    if ((word_bytes != 4 && word_bytes != 8) || block_cycle_grid < 0 || ng < 8 || tiled_smoother < 0 ||
        tiled_smoother > 4)
        return PM_EINVAL;
    set_shape(Shape{ng, word_bytes, block_cycle_grid, tiled_smoother});
    return PM_OK;
}

int pm_autotune(int ng, int precision, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    const size_t need = pm_autotune_workspace_bytes(ng, precision);
    if (need == 0 || !ws || ((uintptr_t)ws & 255))
        return PM_EINVAL;
    if (ws_bytes < need)
        return PM_ENOMEM;
    const size_t solver = (pm_workspace_bytes(ng, 0, PM_F64, (pm_prec)precision) + 255) & ~(size_t)255;
    const size_t field = ((sizeof(double) * (size_t)ng * ng * ng) + 255) & ~(size_t)255;
    double *rho = (double *)((char *)ws + solver);
    double *chi = (double *)((char *)ws + solver + field);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_synth_rho, dim3(1024), dim3(256), 0, st, rho, ng);
    PM_HIP(hipGetLastError());
    const pm_eft_params p{0.3071, -0.5, 0.1, 1.0, 1, 1};
    pm_mg_opts o{};
    o.rel_tol = 1e-30;  // fixed work: full multigrid + 3 V-cycles
    o.max_vcycles = 4;
    o.n_pre = 1;
    o.n_post = 2;
    o.precision = precision;
    o.guess = PM_GUESS_ZERO;
    const int word = precision == PM_PREC_MIXED ? 4 : 8;
    const int cands[5] = {0, 8, 16, 32, 64};
    Shape best = launch_shape(ng, word);
    float best_ms = 1e30f;
    for (int tiled = 0; tiled < 5; tiled++)
        for (int c = 0; c < 5; c++) {
            const int n = cands[c];
            if (n >= ng)
                continue;
            const Shape sh{ng, word, n, tiled};
            set_shape(sh);
            float ms = 1e30f;
            for (int rep = 0; rep < 4; rep++) {  // first run warms up
                pm_mg_report r;
                const int e = grid_solve(rho, ng, PM_F64, &p, &o, chi, &r, ws, solver, stream, true);
                if (e != PM_OK && e != PM_ENOCONV) {
                    set_shape(best);
                    return e;
                }
                if (rep > 0)
                    ms = std::min(ms, r.ms);
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = sh;
            }
        }
    set_shape(best);
    return PM_OK;
}

int pm_tune_save(const char *path)
{
    if (!path)
        return PM_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f)
        return PM_EINVAL;
    std::lock_guard<std::mutex> g(g_tune.mu);
    fprintf(f, "# pmeft launch shapes: ng word_bytes block_cycle_grid tiled_smoother\n");
    for (const auto &e : g_tune.rows)
        fprintf(f, "%d %d %d %d\n", e.ng, e.word, e.block_n, e.tiled);
    fclose(f);
    return PM_OK;
}

int pm_tune_load(const char *path)
{
    if (!path)
        return PM_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f)
        return PM_EINVAL;
    char line[256];
    int rc = PM_OK;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n')
            continue;
        int ng, word, n, tiled;
        if (sscanf(line, "%d %d %d %d", &ng, &word, &n, &tiled) != 4 || (word != 4 && word != 8) || n < 0 ||
            ng < 8 || tiled < 0 || tiled > 4) {
            rc = PM_EINVAL;
            break;
        }
        set_shape(Shape{ng, word, n, tiled});
    }
    fclose(f);
    return rc;
}

int pm_force_interp(const void *psi, const void *chi, int ng, pm_dtype dtype, const pm_eft_params *p, const void *pos,
                    long long np, void *vel, double dt_kick, void *acc_out, void *ws, size_t ws_bytes,
                    pm_stream_t stream)
{
    if (!psi || !pos || !vel || !p || np <= 0 || np > (1LL << 30) || (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    pm_eft_coeffs cf;
    int e = coefficients(*p, cf);
    if (e == PM_EINVAL)
        return e;
    Ctx C;
    e = setup_ctx(C, ws, ws_bytes, ng, np, dtype, 0, stream);
    if (e)
        return e;
    double *ps = C.at<double>(C.P.psi64), *ch = C.at<double>(C.P.chi64);
    launch_natural_to_packed(psi, dtype, ps, ng, 1.0, 0.0, C.st);
    if (chi)
        launch_natural_to_packed(chi, dtype, ch, ng, 1.0, 0.0, C.st);
    void *g4 = C.ws + C.P.g4;
    launch_gradient(ps, chi ? ch : nullptr, cf.xi, ng, g4, dtype, C.st);
    launch_interp_kick(g4, ng, dtype, const_cast<void *>(pos), np, vel, dt_kick, 0.0, acc_out, C.st);
    return launched();
}


// The Poisson and scalar-field solves of a step depend on delta only, so they
// run side by side: the scalar field (after the warm start's network and
// pass, built on the plan's second delta hierarchy) on the side stream,
// driven by a worker thread through the plan's second per-solve region, the
// Poisson solve on the caller's stream in this thread.  Each solve's launches
// and convergence reads stay those of running it alone, so the results do not
// change; the latency-bound coarse levels of one overlap the other's large
// levels.
// Also writes psi_out (natural order, mean removed) right after the Poisson
// solve, while the scalar solve still runs, and chi_out on the side stream
// right after the scalar solve: the caller's stream then waits only for the
// solve itself (its force pass overlaps the conversion) and gets *conv, an
// event after the conversion, to wait on before it ends (null: the
// conversion was not issued, and the caller converts).
// forward_done: the warm start's forward pass is already on the side stream.
static int solve_both(Ctx &C, const pm_eft_params &p, const pm_eft_coeffs &cf, const pm_mg_opts &po,
                      const pm_mg_opts &so, double dsq, void *psi_out, void *chi_out, pm_dtype dtype, SolveOut &sp,
                      SolveOut &sx, float &ms_p, float &ms_x, bool forward_done, hipEvent_t *conv)
{
    *conv = nullptr;
    SideStream *S = nullptr;
    int e = side_stream(&S);
    if (e)
        return e;
    int dev = 0;
    PM_HIP(hipGetDevice(&dev));
    hipEvent_t ready = nullptr, done = nullptr, cdone = nullptr;
    PM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(ready);
        return PM_EHIP;
    }
    if (hipEventCreateWithFlags(&cdone, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(ready);
        (void)hipEventDestroy(done);
        return PM_EHIP;
    }
    Ctx C1 = C;
    rebase_solve(C1.P, C.P.solve2);
    C1.st = S->s;
    e = hipEventRecord(ready, C.st) == hipSuccess && hipStreamWaitEvent(C1.st, ready, 0) == hipSuccess ? PM_OK
                                                                                                      : PM_EHIP;
    if (e) {
        (void)hipEventDestroy(ready);
        (void)hipEventDestroy(done);
        return e;
    }
    bind_solve(C1);
    int ex = PM_OK;
    bool converted = false;  // chi_out issued on the side stream, done recorded before it
    auto scalar_job = [&]() {
        if (hipSetDevice(dev) != hipSuccess) {
            ex = PM_EHIP;
            return;
        }
        Timer tx(C1.st);
        ex = scalar_core(C1, p, cf, so, sx, dsq, forward_done, true);
        if (ex)
            return;
        ms_x = tx.stop();
        if (hipEventRecord(done, C1.st) != hipSuccess) {
            ex = PM_EHIP;
            return;
        }
        double *ch = C1.at<double>(C1.P.chi64);
        launch_field_sum(ch, C1.P.N, C1.rs, C1.st);
        launch_packed_to_natural(ch, chi_out, dtype, C1.P.ng, 0.0, C1.rs.out, C1.st);
        ex = launched();
        if (!ex)
            ex = hipEventRecord(cdone, C1.st) == hipSuccess ? PM_OK : PM_EHIP;
        converted = !ex;
    };
    std::thread worker;
    bool threaded = true;
    try {
        worker = std::thread(scalar_job);
    } catch (...) {  // no thread: the same work, issued from this thread first
        threaded = false;
    }
    if (!threaded)
        scalar_job();
    {
        Timer tp(C.st);
        e = poisson_core(C, cf, po, sp, dsq);
        if (!e) {
            ms_p = tp.stop();
            double *ps = C.at<double>(C.P.psi64);
            launch_field_sum(ps, C.P.N, C.rs, C.st);
            launch_packed_to_natural(ps, psi_out, dtype, C.P.ng, 0.0, C.rs.out, C.st);
            e = launched();
        }
    }
    if (threaded)
        worker.join();
    // on every path the caller's stream waits for the scalar solve's work:
    // for the solve now and the conversion through *conv, or (the conversion
    // not issued) for everything now
    bool waited = (converted || hipEventRecord(done, C1.st) == hipSuccess) &&
                  hipStreamWaitEvent(C.st, done, 0) == hipSuccess;
    if (!e)
        e = ex;
    if (!e && !waited)
        e = PM_EHIP;
    if (converted) {
        if (!e)
            *conv = cdone;  // the caller waits on it after its force pass
        else                // an error: the caller's stream covers the conversion now
            (void)hipStreamWaitEvent(C.st, cdone, 0);
    }
    if (!*conv)
        (void)hipEventDestroy(cdone);
    (void)hipEventDestroy(ready);
    (void)hipEventDestroy(done);
    return e;
}

// Process-wide choice of pm_step's solve arrangement (pm_set_step_concurrency).
static std::atomic<int> g_step_side{1};

int pm_set_step_concurrency(int side_by_side)
{
    return g_step_side.exchange(side_by_side ? 1 : 0);
}

int pm_step(void *pos, void *vel, long long np, int ng, pm_dtype dtype, const pm_eft_params *p,
            const pm_mg_opts *poisson_opts, const pm_mg_opts *scalar_opts, double dt_kick, double dt_drift, void *psi,
            void *chi, pm_step_report *rep, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!pos || !vel || !psi || !chi || !p || np <= 0 || np > (1LL << 30) || !opts_ok(poisson_opts) || !opts_ok(scalar_opts) ||
        (dtype != PM_F32 && dtype != PM_F64))
        return PM_EINVAL;
    pm_eft_coeffs cf;
    int e = coefficients(*p, cf);
    if (e)
        return e;
    Ctx C;
    e = setup_ctx(C, ws, ws_bytes, ng, np, dtype, prec_bits(poisson_opts) | prec_bits(scalar_opts), stream);
    if (e)
        return e;
    // With the learned warm start the network runs on the scalar solve's
    // stream: its weights are packed there first, beside the deposit (they
    // depend on the parameters only), and its forward pass starts as soon as
    // the fine delta is mean-free, beside the rest of the delta preparation.
    const bool side = g_step_side.load() != 0;
    const bool learned = side && scalar_opts->guess == PM_GUESS_LEARNED && cf.K != 0.0 && cf.xi != 0.0;
    SideStream *S = nullptr;
    if (learned) {
        e = learned_ok(ng, *scalar_opts);
        if (!e)
            e = side_stream(&S);
        if (e)
            return e;
    }
    bool fwd = false;  // work that uses the caller's buffers is queued on S
    auto after_caller = [&]() -> int {  // S waits for the caller's stream as it is now
        hipEvent_t ev = nullptr;
        PM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const bool ok = hipEventRecord(ev, C.st) == hipSuccess && hipStreamWaitEvent(S->s, ev, 0) == hipSuccess;
        (void)hipEventDestroy(ev);
        return ok ? PM_OK : PM_EHIP;
    };
    auto start_network = [&]() -> int {
        if (!learned)
            return PM_OK;
        const int r = after_caller();
        if (r)
            return r;
        fwd = true;  // (set before the call: on failure part of it may be queued)
        return unet_learned_forward(scalar_opts->learned_params, C.at<double>(C.P.delta64[0]),
                                    unet_save_area(scalar_opts->learned_ws, ng), ng, *p, scalar_opts->learned_ws,
                                    scalar_opts->learned_ws_bytes, S->s, true);
    };
    // on an error return after work was queued on S: the caller's stream
    // must not run ahead of that work's use of its buffers
    auto wait_network = [&]() {
        hipEvent_t ev = nullptr;
        if (fwd && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
            (void)hipEventRecord(ev, S->s);
            (void)hipStreamWaitEvent(C.st, ev, 0);
            (void)hipEventDestroy(ev);
        }
    };
    if (learned) {
        e = after_caller();
        if (!e) {
            fwd = true;
            e = unet_learned_pack(scalar_opts->learned_params, ng, scalar_opts->learned_ws,
                                  scalar_opts->learned_ws_bytes, S->s);
        }
        if (e) {
            wait_network();
            return e;
        }
    }
    Timer tall(C.st);
    // deposit -> packed delta
    Timer tdep(C.st);
    unsigned long long *acc = C.at<unsigned long long>(C.P.fixacc);
    launch_deposit_auto(pos, np, dtype, ng, acc, C.ws + C.P.depidx, C.st);
    launch_fixed_to_delta(acc, ng, (double)C.P.N / (double)np, C.at<double>(C.P.delta64[0]), C.rs, C.st);
    double dsq = 0.0;
    e = prepare_delta(C, &dsq, start_network);
    if (e) {
        wait_network();
        return e;
    }
    tdep.mark();
    double *ps = C.at<double>(C.P.psi64), *ch = C.at<double>(C.P.chi64);
    if (poisson_opts->guess == PM_GUESS_GIVEN)
        launch_natural_to_packed(psi, dtype, ps, ng, 1.0, 0.0, C.st);
    if (scalar_opts->guess == PM_GUESS_GIVEN)
        launch_natural_to_packed(chi, dtype, ch, ng, 1.0, 0.0, C.st);
    SolveOut sp, sx;
    float ms_p = 0.0f, ms_x = 0.0f;
    hipEvent_t conv = nullptr;  // chi's conversion issued on the side stream (solve_both)
    if (cf.K == 0.0) {
        // Linearised option (screening off) or no scalar field: chi obeys
        // nu lap chi = xi s delta with the same 7-point Laplacian as Psi_N,
        // so chi = mu_chi Psi_N exactly and the step costs one Poisson solve
        // (eq. linearised; Psi_N + xi chi = mu_Psi Psi_N).  The scalar report
        // takes the Poisson solve's residual, which the scaling leaves
        // unchanged, with no V-cycles of its own.
        Timer tp(C.st);
        e = poisson_core(C, cf, *poisson_opts, sp, dsq);
        if (e)
            return e;
        ms_p = tp.stop();
        launch_scale(ps, ch, cf.mu_chi, C.P.N, C.st);
        launch_field_sum(ps, C.P.N, C.rs, C.st);
        launch_packed_to_natural(ps, psi, dtype, ng, 0.0, C.rs.out, C.st);
        sx = sp;
        sx.vcycles = 0;
        for (int i = 0; i < 64; i++)
            sx.hist[i] = i == 0 ? sp.rel : 0.0;
        e = launched();
    } else if (!side) {
        // both solves on the caller's stream, issued from this thread
        {
            Timer tp(C.st);
            e = poisson_core(C, cf, *poisson_opts, sp, dsq);
            if (e)
                return e;
            ms_p = tp.stop();
        }
        launch_field_sum(ps, C.P.N, C.rs, C.st);
        launch_packed_to_natural(ps, psi, dtype, ng, 0.0, C.rs.out, C.st);
        Timer tx(C.st);
        e = scalar_core(C, *p, cf, *scalar_opts, sx, dsq);
        if (!e)
            ms_x = tx.stop();
    } else {
        e = solve_both(C, *p, cf, *poisson_opts, *scalar_opts, dsq, psi, chi, dtype, sp, sx, ms_p, ms_x, fwd, &conv);
    }
    if (e) {
        wait_network();  // (solve_both waits itself once its worker has started)
        return e;
    }
    Timer tf(C.st);
    void *g4 = C.ws + C.P.g4;
    launch_gradient(ps, ch, cf.xi, ng, g4, dtype, C.st);
    launch_interp_kick(g4, ng, dtype, pos, np, vel, dt_kick, dt_drift, nullptr, C.st);
    tf.mark();
    if (conv) {  // chi was converted on the side stream beside the force pass
        const bool w = hipStreamWaitEvent(C.st, conv, 0) == hipSuccess;
        (void)hipEventDestroy(conv);
        if (!w)
            return PM_EHIP;
    } else {
        launch_field_sum(ch, C.P.N, C.rs, C.st);
        launch_packed_to_natural(ch, chi, dtype, ng, 0.0, C.rs.out, C.st);
    }
    e = launched();
    if (e)
        return e;
    const float ms_all = tall.stop();
    if (rep) {
        memset(rep, 0, sizeof(*rep));
        fill_report(&rep->poisson, sp, ms_p);
        fill_report(&rep->scalar, sx, ms_x);
        rep->ms_deposit = tdep.ms();
        rep->ms_force = tf.ms();
        rep->ms_total = ms_all;
    }
    if (sp.status)
        return sp.status;
    return sx.status;
}

int pm_potentials(const void *psi_n, const void *chi, int ng, pm_dtype dtype, const pm_eft_params *p, void *psi_out,
                  void *phi_out, void *lens_out, pm_stream_t stream)
{
    if (!psi_n || !chi || !p || ng < 1 || ng > 1024 || (dtype != PM_F32 && dtype != PM_F64) ||
        (!psi_out && !phi_out && !lens_out))
        return PM_EINVAL;
    pm_eft_coeffs cf;
    const int e = coefficients(*p, cf);
    if (e == PM_EINVAL)
        return e;
    launch_potentials(psi_n, chi, dtype, (long long)ng * ng * ng, cf.xi, cf.alpha_b, psi_out, phi_out, lens_out,
                      (hipStream_t)stream);
    return launched();
}

// Time variable of the equations of motion in code units (Sec. 3.1):
// dt~ = H0 dt / a^2 = da / (a^3 E(a)), E^2 = Omega_m0 a^-3 + 1 - Omega_m0.
// Integral over [a0, a1] by composite 8-point Gauss-Legendre quadrature on
// 32 panels; the nodes come from Newton's method on the Legendre polynomial
// P_8 (three-term recurrence), started from the asymptotic estimate
// cos(pi (i - 1/4) / (n + 1/2)).
static void gauss_legendre8(double x[8], double w[8])
{
    const int n = 8;
    for (int i = 1; i <= n; i++) {
        double z = cos(M_PI * (i - 0.25) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        x[i - 1] = z;
        w[i - 1] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static double code_time(double a0, double a1, double om0)
{
    double x[8], w[8];
    gauss_legendre8(x, w);
    const int panels = 32;
    const double hpan = (a1 - a0) / panels;
    double sum = 0.0;
    for (int q = 0; q < panels; q++) {
        const double lo = a0 + q * hpan, mid = lo + 0.5 * hpan;
        for (int i = 0; i < 8; i++) {
            const double a = mid + 0.5 * hpan * x[i];
            const double E = sqrt(om0 / (a * a * a) + 1.0 - om0);
            sum += 0.5 * hpan * w[i] / (a * a * a * E);
        }
    }
    return sum;
}

int pm_evolve(void *pos, void *vel, long long np, int ng, pm_dtype dtype, const pm_eft_params *p, double a_start,
              double a_end, int nsteps, int log_spacing, const pm_mg_opts *poisson_opts, const pm_mg_opts *scalar_opts,
              void *psi, void *chi, pm_evolve_report *rep, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!p || !poisson_opts || !scalar_opts || nsteps < 1 || nsteps > 100000 || !(a_start > 0.0) ||
        !(a_end > a_start) || !opts_ok(poisson_opts) || !opts_ok(scalar_opts))
        return PM_EINVAL;
    pm_eft_params q = *p;
    // the whole interval must be a valid model (nu > 0 where xi != 0)
    for (int k = 0; k <= nsteps; k++) {
        pm_eft_coeffs cf;
        q.a = log_spacing ? a_start * pow(a_end / a_start, (double)k / nsteps)
                          : a_start + (a_end - a_start) * k / nsteps;
        const int e = coefficients(q, cf);
        if (e)
            return e;
    }
    auto a_at = [&](double k) {  // k may be half-integer
        return log_spacing ? a_start * pow(a_end / a_start, k / nsteps) : a_start + (a_end - a_start) * k / nsteps;
    };
    if (rep)
        memset(rep, 0, sizeof(*rep));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    PM_HIP(hipEventCreate(&t0));
    PM_HIP(hipEventCreate(&t1));
    (void)hipEventRecord(t0, (hipStream_t)stream);
    int status = PM_OK;
    pm_mg_opts po = *poisson_opts, so = *scalar_opts;
    for (int k = 0; k <= nsteps; k++) {
        // kick from a_{k-1/2} (a_0 at the start) to a_{k+1/2} (a_N at the end),
        // then drift from a_k to a_{k+1} (none after the last force)
        const double ak = a_at(k);
        const double kick_lo = k == 0 ? ak : a_at(k - 0.5), kick_hi = k == nsteps ? ak : a_at(k + 0.5);
        const double dk = code_time(kick_lo, kick_hi, p->omega_m0);
        const double dd = k == nsteps ? 0.0 : code_time(ak, a_at(k + 1), p->omega_m0);
        q.a = ak;
        pm_step_report sr;
        const int e = pm_step(pos, vel, np, ng, dtype, &q, &po, &so, dk, dd, psi, chi, &sr, ws, ws_bytes, stream);
        if (e && e != PM_ENOCONV) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return e;
        }
        if (e)
            status = e;
        if (rep) {
            rep->force_evaluations++;
            rep->poisson_vcycles += sr.poisson.vcycles;
            rep->scalar_vcycles += sr.scalar.vcycles;
            rep->max_scalar_vcycles = std::max(rep->max_scalar_vcycles, sr.scalar.vcycles);
            rep->max_rel_residual = std::max(rep->max_rel_residual, std::max(sr.poisson.rel_residual,
                                                                             sr.scalar.rel_residual));
            rep->clamped_cells_last = sr.scalar.clamped_cells;
        }
        // the next step starts from this step's fields (Sec. 3.5.1)
        po.guess = PM_GUESS_GIVEN;
        so.guess = PM_GUESS_GIVEN;
    }
    float ms = 0.f;
    (void)hipEventRecord(t1, (hipStream_t)stream);
    (void)hipEventSynchronize(t1);
    (void)hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rep) {
        rep->steps = nsteps;
        rep->a_end = a_at(nsteps);
        rep->ms_total = ms;
        rep->status = status;
    }
    return status;
}

double pm_code_time(double a0, double a1, double omega_m0)
{
    if (!(a0 > 0.0) || !(a1 > 0.0) || !(omega_m0 > 0.0 && omega_m0 <= 1.0))
        return NAN;
    return code_time(a0, a1, omega_m0);
}

// Host self-check of a workspace plan (no device work): every level view and
// colour buffer the kernels receive lies inside the workspace and no two
// arrays a kernel writes overlap; the levels halve down to a 4^3 or 6^3 grid;
// and for every block-cycle start level the resident levels fit the LDS the
// launch requests, which stays within the budget.  The hierarchies are
// built exactly as the solves build them, from a base address of 256.
}  // extern "C"
namespace pmeft {
namespace {
struct Extent {
    size_t lo, hi;
    const char *what;
};
template <typename R>
bool check_hier(const Hier<R> &H, const char *base, size_t total, std::vector<Extent> &ext)
{
    auto in = [&](const void *p, long long elems, const char *what) {
        if (!p)
            return true;
        const size_t lo = (size_t)((const char *)p - base), hi = lo + sizeof(R) * (size_t)elems;
        if ((const char *)p < base || hi > total)
            return false;
        ext.push_back(Extent{lo, hi, what});
        return true;
    };
    for (int l = 0; l < H.nlev; l++) {
        const LevelView<R> &L = H.L[l];
        if (L.half != (long long)L.n * L.n * (L.n / 2) || L.nh * 2 != L.n)
            return false;
        if (l > 0 && L.n * 2 != H.L[l - 1].n)
            return false;
        // the red / black halves of each array are adjacent
        if ((L.db && L.db != L.dr + L.half) || (L.tb && L.tb != L.tr + L.half) ||
            (L.x0b && L.x0b != L.x0r + L.half))
            return false;
        if (!in(L.dr, 2 * L.half, "delta") || !in(L.tr, 2 * L.half, "tau") || !in(L.x0r, 2 * L.half, "x0") ||
            !in(H.buf[l][0], 2 * L.half, "buf0") || !in(H.buf[l][1], 2 * L.half, "buf1"))
            return false;
    }
    const int nc = H.L[H.nlev - 1].n;
    if (nc != 4 && nc != 6)
        return false;
    BlockHier<R> B = H.block();
    for (int l0 = 0; l0 < H.nlev - 1; l0++) {
        int lr = H.nlev;
        const size_t bytes = block_cycle_lds(B, l0, &lr);
        if (bytes > block_cycle_lds_limit() || lr < l0 || lr > H.nlev)
            return false;
        size_t need = 0;  // the kernel's own layout of the resident levels
        for (int m = lr; m < H.nlev; m++)
            need += sizeof(R) * 2 * (size_t)B.L[m].half *
                    (3 + (B.L[m].tr ? 1 : 0) + (m > l0 && B.L[m].x0r ? 1 : 0));
        if (need != bytes)
            return false;
    }
    return true;
}
}  // namespace
}  // namespace pmeft
extern "C" {

int pm_plan_check(int ng, long long np, pm_dtype dtype, pm_prec prec)
{
    if ((dtype != PM_F32 && dtype != PM_F64) || np < 0)
        return PM_EINVAL;
    int precs = prec == PM_PREC_F64 ? kPrecF64 : (kPrecMixed | kPrecF64);
    Ctx C;
    if (!make_plan(C.P, ng, np, dtype, precs))
        return PM_EINVAL;
    char *base = (char *)(uintptr_t)256;
    C.ws = base;
    std::vector<Ctx> ctxs{C};
    if (np > 0) {  // the step's second per-solve region
        Ctx C2 = C;
        rebase_solve(C2.P, C.P.solve2);
        if (C2.P.solve_lo + C2.P.solve_bytes > C.P.total)
            return PM_EINVAL;
        ctxs.push_back(C2);
    }
    for (Ctx &X : ctxs) {
        X.csum64 = X.at<double>(X.P.csum64);
        X.csum32 = X.at<double>(X.P.csum32);
        X.sm_partials = X.at<double>(X.P.sm_partials);
        std::vector<Extent> ext;
        Hier<double> H64;
        if (!(precs & kPrecF64))
            return PM_EINVAL;
        for (double *master : {X.at<double>(X.P.psi64), X.at<double>(X.P.chi64)}) {
            ext.clear();
            build_hier64(X, H64, master);
            if (!check_hier(H64, base, X.P.total, ext))
                return PM_EINVAL;
            // arrays written by the hierarchy's kernels never overlap each other
            std::sort(ext.begin(), ext.end(), [](const Extent &a, const Extent &b) { return a.lo < b.lo; });
            for (size_t i = 1; i < ext.size(); i++)
                if (ext[i].lo < ext[i - 1].hi)
                    return PM_EINVAL;
        }
        if (precs & kPrecMixed) {
            Hier<float> H32;
            ext.clear();
            build_hier32(X, H32);
            if (!check_hier(H32, base, X.P.total, ext))
                return PM_EINVAL;
            std::sort(ext.begin(), ext.end(), [](const Extent &a, const Extent &b) { return a.lo < b.lo; });
            for (size_t i = 1; i < ext.size(); i++)
                if (ext[i].lo < ext[i - 1].hi)
                    return PM_EINVAL;
        }
        // per-solve scratch inside the workspace
        if (X.P.sm_partials + sizeof(double) * 8 * kMaxBlocks * 2 * kMaxLevels > X.P.total ||
            X.P.red_partials + sizeof(double) * 8 * kMaxBlocks > X.P.total)
            return PM_EINVAL;
    }
    return PM_OK;
}

int pm_kernel_timing_enable(int on)
{
    std::lock_guard<std::mutex> g(g_kt.mu);
    if (on && g_kt.pool.empty()) {
        g_kt.pool.resize(2 * kTimingPairs);
        for (auto &e : g_kt.pool)
            if (hipEventCreate(&e) != hipSuccess)
                return PM_EHIP;
    }
    g_kt.on.store(on != 0);
    return PM_OK;
}

int pm_kernel_timing_read(double *total_ms /* HOST [8] */, long long *launches /* HOST [8] */)
{
    if (!total_ms || !launches)
        return PM_EINVAL;
    std::lock_guard<std::mutex> g(g_kt.mu);
    for (int q = 0; q < kTimingSlots; q++) {
        total_ms[q] = 0.0;
        launches[q] = 0;
    }
    for (size_t k = 0; k < g_kt.slot_of_pair.size(); k++) {
        float ms = 0.f;
        if (hipEventSynchronize(g_kt.pool[2 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_kt.pool[2 * k], g_kt.pool[2 * k + 1]) != hipSuccess)
            return PM_EHIP;
        total_ms[g_kt.slot_of_pair[k]] += ms;
        launches[g_kt.slot_of_pair[k]] += 1;
    }
    g_kt.used = 0;
    g_kt.slot_of_pair.clear();
    return PM_OK;
}

const char *pm_strerror(int code)
{
    switch (code) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument (null pointer, unsupported grid size or option)";
    case PM_EUNSTABLE: return "unstable model: nu <= 0 with xi != 0";
    case PM_ENOCONV: return "multigrid did not reach the tolerance within max_vcycles";
    case PM_ENONFINITE: return "non-finite value in the input or the residual";
    case PM_EHIP: return "HIP runtime error";
    case PM_ENOMEM: return "workspace too small";
    default: return "unknown error";
    }
}

}  // extern "C"
