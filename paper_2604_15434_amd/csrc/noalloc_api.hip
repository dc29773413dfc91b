// Allocation-free CIC deposit: pm_deposit_noalloc (declared in pmeft.h).
// Its scratch lives in a file-scope device array of this library (one copy
// per GPU, held until the process ends) instead of a caller workspace, for
// callers that cannot allocate device memory.
#include "pmeft_internal.h"

#include <mutex>

namespace pmeft {

// The scratch array holds the fixed-point accumulator (8 bytes per cell),
// the packed delta (8 bytes per cell) and the reduction partials: grids up
// to 128^3.  Host code never passes `scratch` itself (its name on the host
// is a stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
namespace {
constexpr size_t kScratchBytes = 33u << 20;  // 33 MiB
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[64] = {};

int scratch_ptr(char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return PM_EHIP;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return PM_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = (char *)g_scratch_dev[dev];
    return PM_OK;
}

// offsets inside the scratch array for an ng^3 deposit
struct ScratchLayout {
    size_t acc, delta, partials, out, total;
};
ScratchLayout scratch_layout(int ng)
{
    ScratchLayout L;
    const size_t n3 = (size_t)ng * ng * ng;
    size_t c = 0;
    L.acc = c;
    c += (sizeof(unsigned long long) * n3 + 255) & ~(size_t)255;
    L.delta = c;
    c += (sizeof(double) * n3 + 255) & ~(size_t)255;
    L.partials = c;
    c += sizeof(double) * 8 * kMaxBlocks;
    L.out = c;
    c += 256;
    L.total = c;
    return L;
}
}  // namespace
}  // namespace pmeft

using namespace pmeft;

extern "C" {

size_t pm_deposit_noalloc_max_bytes(void) { return kScratchBytes; }

int pm_deposit_noalloc(const void *pos, long long np, pm_dtype dtype, int ng, void *rho, pm_stream_t stream)
{
    if (!pos || !rho || np <= 0 || np > (1LL << 30) || (dtype != PM_F32 && dtype != PM_F64) || !pm_grid_levels(ng))
        return PM_EINVAL;
    const ScratchLayout L = scratch_layout(ng);
    if (L.total > kScratchBytes)
        return PM_ENOMEM;
    char *base = nullptr;
    const int e = scratch_ptr(&base);
    if (e)
        return e;
    hipStream_t st = (hipStream_t)stream;
    const long long n3 = (long long)ng * ng * ng;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(base + L.acc);
    double *d0 = reinterpret_cast<double *>(base + L.delta);
    ReduceSlot rs;
    rs.partials = reinterpret_cast<double *>(base + L.partials);
    rs.counter = nullptr;
    rs.out = reinterpret_cast<double *>(base + L.out);
    // the launches of pm_deposit, on the scratch array; the accumulator is
    // cleared first (every call on a GPU shares the array)
    launch_zero(acc, sizeof(unsigned long long) * n3, st);
    launch_deposit_fixed(pos, np, dtype, ng, acc, st);
    launch_fixed_to_delta(acc, ng, (double)n3 / (double)np, d0, rs, st);
    launch_packed_to_natural(d0, rho, dtype, ng, 1.0, nullptr, st);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP;
}

}  // extern "C"
