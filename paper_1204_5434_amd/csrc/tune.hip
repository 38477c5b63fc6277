// Kernel-variant autotuner: every axis length has a few compiled variants of
// its passes; pft_autotune times them and makes the fastest the default for
// contexts created afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.h"

namespace pft::rt {

// Kernel variant per (precision, axis length, kind: 0 = z pass, 1 = x pass,
// 2 = y pass), used by contexts created afterwards; filled by pft_autotune or
// pft_tune_load (also from $PFT_TUNE_CACHE on the first pft_create).
namespace {
int g_tune[2][257][3] = {};
std::once_flag g_tune_env;
}  // namespace

int tuned_variant(int prec, int n, int kind)
{
    int n1, n2, w;
    const int v = (n >= 0 && n <= 256) ? g_tune[prec & 1][n][kind] : 0;
    return pft::axis_variant(n, v, &n1, &n2, &w) ? v : 0;
}

void tune_env_once()
{
    std::call_once(g_tune_env, [] {
        if (const char* path = std::getenv("PFT_TUNE_CACHE")) (void)pft_tune_load(path);
    });
}

}  // namespace pft::rt

// ============================================================== autotuner ==
namespace {

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Side length A of the two other axes of the timing grid (A * A * N <= 4 Mi sites).
int tune_side(int N)
{
    const int sides[] = {256, 192, 128, 96, 64, 48, 32, 24, 16, 8};
    for (int a : sides)
        if ((int64_t)a * a * N <= (int64_t)4 << 20) return a;
    return 8;
}

// Average duration (ms) of `reps` launches of one pass kind with variant v.
template <typename T>
double time_variant(pft_ctx* c, int kind, int v, int reps)
{
    cx<T>* w0 = static_cast<cx<T>*>(c->work);
    const cx<T>* e = etab<T>(c, 0);
    // the passes in their Richardson-step form, as the sweeps run them
    auto launch = [&]() -> hipError_t {
        if (kind == 0) {
            // z pass completing one step and starting the next
            pft::ZArgs<T> a{};
            a.nlines = (int64_t)c->p.nx * c->p.ny;
            a.U = static_cast<cx<T>*>(c->U);
            a.V = static_cast<cx<T>*>(c->V);
            a.qout = w0;
            a.scheme = PFT_RQM4;
            a.has_prev = 1;
            a.has_next = 1;
            a.Ep = e;
            a.En = e;
            a.gh_p = gptr<T>(c, 0, 0, 2);
            a.gh_n = gptr<T>(c, 0, 0, 2);
            a.gf_n = gptr<T>(c, 0, 1, 2);
            return pft::launch_zpass<T>(c->p.nz, v, a, c->stream);
        }
        const int64_t nynz = (int64_t)c->p.ny * c->p.nz;
        pft::SArgs<T> a{};
        a.U = static_cast<cx<T>*>(c->U);
        a.V = static_cast<cx<T>*>(c->V);
        if (kind == 1) {
            // x pass on both arrays with the field multiply
            a.opU = {gptr<T>(c, 0, 0, 0), e, gptr<T>(c, 0, 0, 0), nullptr};
            a.opV = {gptr<T>(c, 0, 1, 0), e, nullptr, nullptr};
            a.S = nynz;
            return pft::launch_spass<T>(0, c->p.nx, v, nynz, a, 1, c->stream);
        }
        // y pass on both arrays (the first y pass of a Richardson step)
        a.opU = {gptr<T>(c, 0, 0, 1), nullptr, nullptr, nullptr};
        a.opV = {gptr<T>(c, 0, 1, 1), nullptr, nullptr, nullptr};
        a.S = c->p.nz;
        a.slab_stride = nynz;
        return pft::launch_spass<T>(1, c->p.ny, v, c->p.nz, a, c->p.nx, c->stream);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    double ms = -1;
    bool ok = launch() == hipSuccess && launch() == hipSuccess;  // warm-up
    if (ok) ok = hipEventRecord(e0, c->stream) == hipSuccess;
    for (int i = 0; ok && i < reps; ++i) ok = launch() == hipSuccess;
    if (ok) ok = hipEventRecord(e1, c->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float t = 0.f;
    if (ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

extern "C" {

pft_status pft_autotune(int32_t precision, const int32_t* sizes, int32_t nsizes, void* hip_stream, int32_t* choices,
                        double* timings)
{
    if ((precision != PFT_C128 && precision != PFT_C64) || !sizes || nsizes < 1) return PFT_E_INVALID;
    for (int i = 0; i < nsizes; ++i)
        if (!pft::axis_supported(sizes[i])) return PFT_E_UNSUPPORTED;
    for (int i = 0; i < nsizes; ++i) {
        const int N = sizes[i];
        const int A = tune_side(N);
        for (int kind = 0; kind < 3; ++kind) {
            // lines of length N along z (kind 0), x (1) or y (2)
            const int ax = kind == 0 ? 2 : kind - 1;
            pft_params p{};
            p.nx = ax == 0 ? N : A;
            p.ny = ax == 1 ? N : A;
            p.nz = ax == 2 ? N : A;
            p.lx = 0.1 * p.nx;
            p.ly = 0.1 * p.ny;
            p.lz = 0.1 * p.nz;
            p.ns = 2;
            p.f = 0.5;
            p.chiN = 10;
            p.C = 1;
            p.precision = precision;
            p.scheme = PFT_SPLIT2;
            pft_ctx* c = nullptr;
            pft_status st = pft_create(&p, hip_stream, &c);
            if (st) return st;
            // the timed inputs: zeros are fine for timing (no data-dependent work)
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->work), (int64_t)(c->M * c->elem / 16));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 4, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->E), (int64_t)(c->M * c->elem / 4));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->U), (int64_t)(c->M * c->elem / 16));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->V), (int64_t)(c->M * c->elem / 16));
            int best = 0;
            double best_ms = -1;
            for (int v = 0; v < PFT_MAX_VARIANTS; ++v) {
                int n1, n2, w;
                double ms = -1;
                if (pft::axis_variant(N, v, &n1, &n2, &w))
                    ms = precision == PFT_C128 ? time_variant<double>(c, kind, v, 10) : time_variant<float>(c, kind, v, 10);
                if (timings) timings[(i * 3 + kind) * PFT_MAX_VARIANTS + v] = ms;
                if (ms > 0 && (best_ms < 0 || ms < best_ms)) {
                    best_ms = ms;
                    best = v;
                }
            }
            pft_destroy(c);
            if (best_ms < 0) return PFT_E_DEVICE;
            g_tune[precision][N][kind] = best;
            if (choices) choices[i * 3 + kind] = best;
        }
    }
    return PFT_OK;
}

pft_status pft_tune_save(const char* path)
{
    if (!path) return PFT_E_INVALID;
    FILE* f = std::fopen(path, "w");
    if (!f) return PFT_E_INVALID;
    const std::string arch = device_arch();
    for (int prec = 0; prec < 2; ++prec)
        for (int n = 0; n <= 256; ++n)
            for (int kind = 0; kind < 3; ++kind)
                if (pft::axis_supported(n))
                    std::fprintf(f, "%s %d %d %d %d\n", arch.c_str(), prec, n, kind, g_tune[prec][n][kind]);
    std::fclose(f);
    return PFT_OK;
}

pft_status pft_tune_load(const char* path)
{
    if (!path) return PFT_E_INVALID;
    FILE* f = std::fopen(path, "r");
    if (!f) return PFT_E_INVALID;
    const std::string arch = device_arch();
    char a[64];
    int prec, n, kind, v;
    while (std::fscanf(f, "%63s %d %d %d %d", a, &prec, &n, &kind, &v) == 5) {
        int n1, n2, w;
        if (arch == a && (prec == 0 || prec == 1) && kind >= 0 && kind <= 2 && n >= 0 && n <= 256 &&
            pft::axis_variant(n, v, &n1, &n2, &w))
            g_tune[prec][n][kind] = v;
    }
    std::fclose(f);
    return PFT_OK;
}

pft_status pft_set_variant(pft_ctx* c, int32_t axis, int32_t variant)
{
    if (!c || axis < 0 || axis > 2) return PFT_E_INVALID;
    const int n = axis == 0 ? c->p.nx : axis == 1 ? c->p.ny : c->p.nz;
    int n1, n2, w;
    if (!pft::axis_variant(n, variant, &n1, &n2, &w)) return c->fail(PFT_E_UNSUPPORTED, "no variant %d for %d", variant, n);
    c->var[axis] = variant;
    return PFT_OK;
}

}  // extern "C"
