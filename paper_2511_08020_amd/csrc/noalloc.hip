// pdg_vjp_static: the vector-Jacobian product of the residual with its workspace in a fixed
// device array, for callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is a file-scope __device__ array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code never passes the
// array's name to a kernel or a copy: in host code that name is a stand-in, not a device
// address.  Instead the address is looked up once per device with hipGetSymbolAddress, with
// that device current, and the looked-up pointer is used from then on.  The workspace needs no
// clearing: every entry the adjoint kernels read is written earlier in the same call.  All
// calls on one GPU share the array, so calls that overlap in time on one GPU race (use one
// stream, or serialise them).
#include <mutex>

#include "pdg_internal.h"

namespace pdg {
namespace {

constexpr size_t kScratchDoubles = (size_t)8 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of the current GPU's copy of `scratch` (looked up on the first call per GPU)
int scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the static workspace table");
        return PDG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress of the static workspace failed: ") + hipGetErrorString(e));
            return PDG_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PDG_OK;
}

size_t round_up_256b(size_t doubles) { return (doubles + 31) & ~(size_t)31; }

}  // namespace

int static_workspace_setup() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return PDG_EHIP;
    }
    double *p = nullptr;
    return scratch_address(dev, &p);
}

}  // namespace pdg

using namespace pdg;

extern "C" int pdg_vjp_static(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U) {
    if (!ctx) {
        set_error("null context");
        return PDG_EINVAL;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return PDG_EHIP;
    }
    if (dev != context_device(ctx)) {
        set_error("the current device is not the context's device");
        return PDG_EINVAL;
    }
    size_t lf = 0, lw = 0, ub = 0;
    adjoint_workspace(ctx, &lf, &lw, &ub);
    const size_t need = round_up_256b(lf) + round_up_256b(lw) + round_up_256b(ub);
    if (need > kScratchDoubles) {
        set_error("pdg_vjp_static: the mesh needs " + std::to_string(need * sizeof(double)) +
                  " bytes of workspace, the static workspace holds " +
                  std::to_string(kScratchDoubles * sizeof(double)));
        return PDG_EINVAL;
    }
    double *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc != PDG_OK) return rc;
    double *Lf = base;
    double *Lw = lw ? Lf + round_up_256b(lf) : nullptr;
    double *Ub = ub ? Lf + round_up_256b(lf) + round_up_256b(lw) : nullptr;
    return vjp_in(ctx, U, cot, grad_U, Lf, Lw, Ub);
}
