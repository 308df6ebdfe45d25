// An allocation-free variant of stag_mdagm for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).  Its odd
// temporary w = D_oe in lives in a file-scope device array instead of the
// handle's workspace.
#include <cmath>
#include <mutex>

#include "ctx.h"

namespace {

// 32 MiB: the odd half vector (3 x Vh x 16 B) of lattices up to Vh = 699050
// sites, e.g. 48^3x12.  Every GPU holds one copy until the process ends.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

namespace stag {

// Resolves the device address of the array on the current device (once per
// device); called by stag_create with the handle's device current.
stag_status scratch_init(stag_ctx* c) {
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, STAG_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[c->device]) return STAG_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(c, STAG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[c->device] = ptr;
    return STAG_OK;
}

}  // namespace stag

extern "C" stag_status stag_mdagm_noalloc(stag_handle c, void* out, const void* in, double mass) {
    using namespace stag;
    if (!c) return fail(nullptr, STAG_ERR_INVALID_ARG, "handle is NULL");
    if (!c->has_gauge) return fail(c, STAG_ERR_NO_GAUGE, "no gauge field set (call stag_set_gauge)");
    if (!out || !in || (uintptr_t)out % 16 || (uintptr_t)in % 16 || out == in)
        return fail(c, STAG_ERR_INVALID_ARG, "vector pointers NULL, misaligned or equal");
    if (!std::isfinite(mass)) return fail(c, STAG_ERR_INVALID_ARG, "mass must be finite");
    if (half_bytes(c->g) > kScratchBytes)
        return fail(c, STAG_ERR_INVALID_ARG,
                    "lattice too large for the allocation-free operator: the odd temporary needs " +
                        std::to_string(half_bytes(c->g)) + " bytes, the scratch array holds " +
                        std::to_string(kScratchBytes));
    void* w;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        w = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
    }
    if (!w) return fail(c, STAG_ERR_HIP, "scratch array not resolved on this device");
    // the derived link copies are allocated when the format or the improvement
    // is chosen; get_links below only refreshes them
    if ((c->fmt64 == STAG_LINKS_F64_12 && !c->links_d12) ||
        (c->naik && (!c->long_d18 || (c->fmt64 == STAG_LINKS_F64_12 && !c->long_d12))))
        return fail(c, STAG_ERR_INVALID_ARG, "link copies of the operator are not allocated");
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    HIP_OR_FAIL(c, hipEventRecord(c->ev_in, c->user));
    HIP_OR_FAIL(c, hipStreamWaitEvent(c->s, c->ev_in, 0));
    LinkSet ls;
    stag_status e = get_links(c, -1, ls);
    if (e) return e;
    launch_dslash(c->g, ls, (const double2*)in, (double2*)w, 1, c->tps, nullptr, c->s);
    launch_dslash_axpy(c->g, ls, (const double2*)w, (const double2*)in, 4.0 * mass * mass, (double2*)out, c->tps,
                       c->s);
    HIP_OR_FAIL(c, hipGetLastError());
    HIP_OR_FAIL(c, hipEventRecord(c->ev_out, c->s));
    HIP_OR_FAIL(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
    return STAG_OK;
}
