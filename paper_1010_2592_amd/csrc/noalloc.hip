// The no-allocation form of the multi-shift solve: every workspace buffer of
// the call is carved from one fixed device array, `scratch`, instead of
// hipMalloc, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array: its name in host code is only a
// host-side stand-in, never a device address.  At context creation (with the
// context's device current) noalloc_setup() asks the runtime for the array's
// address on that device once and keeps it per device; the solver is handed
// that address, never the symbol.  Each device holds its own copy of the
// array until the process ends.  All no-allocation calls on one device share
// it and leave their contents in it; calls that overlap in time on one device
// race.
#include <mutex>
#include <string>

#include "msb.h"
#include "ctx.h"

namespace msb {

static __device__ __align__(256) char scratch[MSB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES)
        return set_error(S_ERR_HIP, "device index " + std::to_string(device) + " beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch_ptr[device]) return 0;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_error(S_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
    return 0;
}

int solve_noalloc(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts, bool want_true,
                  SolveReport *rep) {
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (c->device >= 0 && c->device < MAX_DEVICES) base = g_scratch_ptr[c->device];
    }
    if (!base) return set_error(S_ERR_HIP, "the scratch buffer of this device was not set up by msb_create");
    // a context that shares the caller's links and geometry but owns no
    // workspace: every ensure() of the solve draws from the arena
    Ctx t;
    t.g = c->g;
    t.mass = c->mass;
    t.mu = c->mu;
    t.bc_t = c->bc_t;
    t.stream = c->stream;
    t.device = c->device;
    t.U64 = c->U64;
    t.U32 = c->U32;
    Arena a;
    a.base = (char *)base;
    a.cap = MSB_NOALLOC_SCRATCH_BYTES;
    t.arena = &a;
    return solve_mshift(&t, P, b, y, x_shifts, want_true, rep);
}

}  // namespace msb
