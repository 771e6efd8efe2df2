// fem_residual_noalloc: the FP64 Newton residual of fem_assemble for callers that
// cannot allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its element-term scratch is a static device
// array of this file, so the call allocates nothing.
#include <mutex>
#include <vector>

#include "solver.h"

namespace {

// Element terms of the residual: n_elems * 8 * ndpn doubles (node-major incidence
// order, every used entry written before it is read).  64 MiB: up to 349,525 elements
// with 3 dofs per node, 1,048,576 with 1.  Each device the library runs on holds its
// own copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;  // per device: the device address of `scratch`

// The device address of this device's copy of `scratch`.  The array's name is a
// host-side stand-in, not a device address; the runtime gives the address per
// device.  Looked up once per device, with that device current.
double *scratch_for(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device >= int(g_scratch_ptr.size())) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        FEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw fem::Error(FEM_EHIP, "hipGetSymbolAddress returned NULL for the static scratch array");
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" int fem_residual_noalloc(fem_handle *h, const double *u, const double *theta, double *residual,
                                    void *stream) {
    return fem::run_guarded([&] {
        if (h == nullptr) throw fem::Error(FEM_EINVAL, "handle is NULL");
        if (h->g.N == 0) return;
        if (!(u && theta && residual)) throw fem::Error(FEM_EINVAL, "u, theta and residual must be non-NULL");
        const size_t need = size_t(h->g.Ne) * 8 * size_t(h->g.nd) * sizeof(double);
        if (need > kScratchBytes)
            throw fem::Error(FEM_ENOMEM, "the mesh needs " + std::to_string(need) +
                                             " bytes of element scratch; the static buffer of "
                                             "fem_residual_noalloc holds " +
                                             std::to_string(kScratchBytes) +
                                             " (use fem_assemble with a workspace)");
        FEM_HIP(hipSetDevice(h->device));
        double *scr = scratch_for(h->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        fem::reset_status(h, s);
        fem::launch_residual(h, u, theta, 1.0, scr, residual, s);
    });
}
