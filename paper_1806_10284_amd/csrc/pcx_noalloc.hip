// pcx_apply_Ar_noalloc: z = A_r y (eq. NFSEP) without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses that forbid it).
//
// The two buffers that pcx_apply_Ar takes from the plan on demand -- the per-wave-vector mode
// codes (n bytes) and the matvec workspace t (3n complex per vector, twice that for planes that
// take the two-pass path) -- live here in one file-scope device array of PCX_NOALLOC_SCRATCH_BYTES.
// Every device that loads the library holds its own copy until the process ends.  Its device
// address is looked up once per device (hipGetSymbolAddress, with that device current) when the
// first plan on the device is created; host code then uses only that address.  The W table of
// the fixed-size FP32 adjoint kernel is not used: those kernels form W per mode instead (same
// operator up to rounding order).  Calls on one device share the array, so calls that overlap on
// one device race; nothing in it has to start at zero (the codes and t are written before they
// are read).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "pcx_host.h"

namespace pcx {

static __device__ __align__(256) unsigned char scratch[PCX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
}  // namespace

// Called with `device` current (plan creation).  Looks up the array's address on this device once.
int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(PCX_E_DEVICE, "device %d out of range", device);
    std::call_once(g_once[device], [device] {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_status[device] = e;
        if (e == hipSuccess) g_ptr[device] = ptr;
    });
    if (g_status[device] != hipSuccess) return hip_fail(g_status[device], "scratch symbol address");
    return g_ptr[device] ? PCX_OK : fail(PCX_E_DEVICE, "scratch symbol address is null");
}

}  // namespace pcx

using namespace pcx;

extern "C" int pcx_apply_Ar_noalloc(pcx_plan* pp, const double kappa[3], int precision, const void* y, void* z,
                                    int nvec) {
    Plan* p = (Plan*)pp;
    if (!p || !kappa || !y || !z) return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: bad precision");
    if (nvec < 1) return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: nvec must be >= 1");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: non-finite kappa");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: permittivity not set");
    int rc = p->check_fits(precision);
    if (rc) return rc;
    const int dev = p->device;
    if (dev < 0 || dev >= kMaxDevices || !g_ptr[dev])
        return fail(PCX_E_DEVICE, "pcx_apply_Ar_noalloc: no scratch address for device %d", dev);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev)
        return fail(PCX_E_ARG, "pcx_apply_Ar_noalloc: the plan's device %d is not the current device", dev);
    // scratch layout: mode codes (n bytes, rounded up to 256), then the workspace t
    Grid g = p->grid(kappa);
    const int f = precision == PCX_FP64 ? 1 : 0;
    const size_t codes_bytes = ((size_t)p->n + 255) / 256 * 256;
    const size_t cplx = f ? sizeof(cx<double>) : sizeof(cx<float>);
    const size_t per_vec = (g.split[f] ? 2 : 1) * 3 * (size_t)p->n * cplx;
    const size_t need = codes_bytes + (size_t)nvec * per_vec;
    if (need > (size_t)PCX_NOALLOC_SCRATCH_BYTES)
        return fail(PCX_E_SIZE,
                    "pcx_apply_Ar_noalloc: %d vectors of this grid need %zu bytes of scratch, more than the %zu "
                    "available (at most %zu vectors)",
                    nvec, need, (size_t)PCX_NOALLOC_SCRATCH_BYTES,
                    ((size_t)PCX_NOALLOC_SCRATCH_BYTES - codes_bytes) / per_vec);
    unsigned char* base = (unsigned char*)g_ptr[dev];
    unsigned char* codes = base;
    void* t = base + codes_bytes;
    g.codes = codes;
    g.wtab[0] = g.wtab[1] = nullptr;
    hipError_t e = launch_modecode(g, codes, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_apply_Ar_noalloc: mode codes");
    if (f)
        e = launch_apply_Ar<double>(g, p->tables, (const double*)p->inv_epsn64, (const cx<double>*)y, (cx<double>*)z,
                                    (cx<double>*)t, nvec, p->stream);
    else
        e = launch_apply_Ar<float>(g, p->tables, (const float*)p->inv_epsn32, (const cx<float>*)y, (cx<float>*)z,
                                   (cx<float>*)t, nvec, p->stream);
    return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_apply_Ar_noalloc: launch");
}
