// pft_cl_step_static: the field step with the semi-implicit step's work
// memory in a fixed device array of the library, for callers that cannot
// allocate (include/pft.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

// ------------------------------------------------------- fixed work memory --
// pft_cl_step_static takes the semi-implicit step's work memory from this
// array instead of buffers the context allocates.  Host code never uses the
// array's name as an address: each device's copy is found once with
// hipGetSymbolAddress and kept per device.
static __device__ __align__(256) unsigned char scratch[PFT_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// The address of the current device's copy of the array (looked up on the
// first call on that device).
pft_status scratch_address(pft_ctx* c, unsigned char** out)
{
    int dev = -1;
    PFT_HIP(c, hipGetDevice(&dev));
    if (dev != c->device) return c->fail(PFT_E_INVALID, "the context's device (%d) must be current, not %d", c->device, dev);
    if (dev < 0 || dev >= kMaxDevices) return c->fail(PFT_E_DEVICE, "device ordinal %d beyond the library's table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return c->fail(PFT_E_DEVICE, "hipGetSymbolAddress of the work array failed: %s", hipGetErrorString(e));
        }
        g_scratch_at[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_at[dev]);
    return PFT_OK;
}
}  // namespace

extern "C" {

pft_status pft_cl_step_static(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
                              double* Q, double* H)
{
    if (!c) return PFT_E_INVALID;
    if (!st) return c->fail(PFT_E_INVALID, "step parameters are NULL");
    if (st->update != 1) return cl_step(c, wp, wm, st, phi_a, phi_b, Q, H, nullptr);  // no work memory
    // the layout: R [M], then between walls X and W [Me each], then |k|^2 [3][pitch]
    const pft_params& p = c->p;
    const int n[3] = {p.nx, p.ny, p.nz};
    int pitch = 0;
    int64_t Me = 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int ne = p.bc[ax] ? 2 * n[ax] : n[ax];
        Me *= ne;
        pitch = std::max(pitch, ne);
    }
    const bool walls = p.bc[0] || p.bc[1] || p.bc[2];
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t offX = up((size_t)c->M * sizeof(double2));
    const size_t offK = offX + (walls ? 2 * up((size_t)Me * sizeof(double2)) : 0);
    const size_t need = offK + up(3 * (size_t)pitch * sizeof(double));
    if (need > (size_t)PFT_STATIC_SCRATCH_BYTES)
        return c->fail(PFT_E_UNSUPPORTED, "pft_cl_step_static: the semi-implicit step needs %zu bytes of work memory, "
                       "more than the fixed %zu", need, (size_t)PFT_STATIC_SCRATCH_BYTES);
    unsigned char* base = nullptr;
    const pft_status sa = scratch_address(c, &base);
    if (sa) return sa;
    SisBufs sb;
    sb.R = reinterpret_cast<double2*>(base);
    if (walls) {
        sb.X = reinterpret_cast<double2*>(base + offX);
        sb.W = reinterpret_cast<double2*>(base + offX + up((size_t)Me * sizeof(double2)));
    }
    sb.k2 = reinterpret_cast<const double*>(base + offK);
    sb.pitch = pitch;
    return cl_step(c, wp, wm, st, phi_a, phi_b, Q, H, &sb);
}

}  // extern "C"
