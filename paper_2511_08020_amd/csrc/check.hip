// Finiteness check of a state vector (failure detection): the smallest index of a NaN or
// infinite entry, by an integer minimum over the grid (the result does not depend on order).
#include <algorithm>

#include "kernels.h"

namespace pdg {

__global__ __launch_bounds__(256) void k_first_nonfinite(const double *__restrict__ U, int64_t n,
                                                          unsigned long long *first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long mine = (unsigned long long)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!isfinite(U[i])) {
            mine = (unsigned long long)i;
            break;  // later entries of this lane have larger indices
        }
    }
    if (mine < (unsigned long long)n) atomicMin(first, mine);
}

hipError_t launch_first_nonfinite(const double *U, int64_t n, unsigned long long *first, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_first_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, U, n, first);
    return hipGetLastError();
}

}  // namespace pdg
