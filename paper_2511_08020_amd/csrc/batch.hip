// Batched kernels: many independent meshes (any N, either equation set) advanced together.
//
// A work item is (mesh, first, count): `count` consecutive entries of that mesh's element list
// of one type, processed in order by one workgroup (the tile of the (type, N) launch).  Each
// (phase, type, N, equations) is one launch over the items of every mesh in the batch; the
// per-mesh kernel arguments (tables, geometry, state pointers, the stage's LSERK coefficients)
// are read from a device array indexed by the item's mesh.
#include "batch.h"
#include "phases.h"

namespace pdg {

template <int T, int N>
__global__ __launch_bounds__(128) void kb_trace(const StageArgs *__restrict__ A, const BatchItem *__restrict__ items) {
    __shared__ double smem[TraceLDS<T, N>::size];
    const BatchItem it = items[blockIdx.x];
    const StageArgs &a = A[it.mesh];
    for (int i = 0; i < it.count; ++i) {
        if (i) __syncthreads();
        trace_elem<T, N>(a, a.list[T][it.first + i], smem);
    }
}

// at least four waves per SIMD, as the per-type volume kernels
template <int T, int N, bool NS, bool CV>
__global__ __launch_bounds__((kVolBS<T, N>), 4) void kb_volume(const StageArgs *__restrict__ A,
                                                            const BatchItem *__restrict__ items) {
    __shared__ double smem[VolLDS<T, N, NS>::size];
    const BatchItem it = items[blockIdx.x];
    const StageArgs &a = A[it.mesh];
    for (int i = 0; i < it.count; ++i) {
        if (i) __syncthreads();
        volume_elem<T, N, NS, kVolBS<T, N>, false, Dm<T, N>::SLOTS, CV>(a, a.list[T][it.first + i], smem);
    }
}

template <int T, int N, bool NS, bool CV>
__global__ __launch_bounds__(kBS<N>) void kb_surface(const StageArgs *__restrict__ A,
                                                     const BatchItem *__restrict__ items) {
    __shared__ double smem[SurfLDS<T, N>::size];
    const BatchItem it = items[blockIdx.x];
    const StageArgs &a = A[it.mesh];
    for (int i = 0; i < it.count; ++i) {
        if (i) __syncthreads();
        surface_elem<T, N, NS, false, Dm<T, N>::SLOTS, CV>(a, a.list[T][it.first + i], smem);
    }
}

template <int T, int N, bool CV>
static void go_b_cv(int phase, bool ns, const StageArgs *A, const BatchItem *items, int n, hipStream_t s) {
    if (phase == 0) {
        hipLaunchKernelGGL((kb_trace<T, N>), dim3(n), dim3(128), 0, s, A, items);
    } else if (phase == 1) {
        if (!ns) {
            hipLaunchKernelGGL((kb_volume<T, N, false, CV>), dim3(n), dim3(kVolBS<T, N>), 0, s, A, items);
        } else if constexpr (N <= 5) {
            hipLaunchKernelGGL((kb_volume<T, N, true, CV>), dim3(n), dim3(kVolBS<T, N>), 0, s, A, items);
        }
    } else {
        if (!ns) {
            hipLaunchKernelGGL((kb_surface<T, N, false, CV>), dim3(n), dim3(kBS<N>), 0, s, A, items);
        } else if constexpr (N <= 5) {
            hipLaunchKernelGGL((kb_surface<T, N, true, CV>), dim3(n), dim3(kBS<N>), 0, s, A, items);
        }
    }
}
template <int T, int N>
static void go_b(int phase, bool ns, bool cv, const StageArgs *A, const BatchItem *items, int n, hipStream_t s) {
    if (cv) go_b_cv<T, N, true>(phase, ns, A, items, n, s);
    else go_b_cv<T, N, false>(phase, ns, A, items, n, s);
}

hipError_t launch_batch_phase(int type, int N, bool ns, bool cv, int phase, const StageArgs *A,
                              const BatchItem *items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (ns && N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_TN(go_b, phase, ns, cv, A, items, n_items, s);
    return hipGetLastError();
}

}  // namespace pdg
