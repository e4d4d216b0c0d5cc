// Volume phase in the entropy-stable split form and surface phase with the entropy-conservative
// two-point flux (per-type and work-queue kernels); see volume_elem and surface_elem.
#include "phases.h"

namespace pdg {

// CV: a mesh with curved elements (per-node metrics, averaged per node pair in the two-point
// fluxes; conforming faces, so only the narrow kernels)
template <int T, int N, bool NS, bool WIDE, bool CV = false>
__global__ __launch_bounds__((kVolBS<T, N>), 4) void k_volume_split(StageArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double smem[VolLDS<T, N, NS, true, S, CV>::size];
    volume_elem<T, N, NS, kVolBS<T, N>, true, S, CV>(a, (WIDE ? a.list_w : a.list_n)[T][blockIdx.x], smem);
}

constexpr int cmax4s(int a, int b, int c, int d) {
    return a > b ? (a > c ? (a > d ? a : d) : (c > d ? c : d)) : (b > c ? (b > d ? b : d) : (c > d ? c : d));
}

template <int N, bool NS, bool CV = false>
__global__ __launch_bounds__(kBS<N>) void k_volume_split_q(StageArgs a, const int32_t *qtb, uint64_t *qt) {
    constexpr int SZ = cmax4s(VolLDS<0, N, NS, true, Dm<0, N>::SLOTS, CV>::size, VolLDS<1, N, NS, true, Dm<1, N>::SLOTS, CV>::size,
                              VolLDS<2, N, NS, true, Dm<2, N>::SLOTS, CV>::size, VolLDS<3, N, NS, true, Dm<3, N>::SLOTS, CV>::size);
    __shared__ double smem[SZ];
    const long long t0 = queue_clock_begin();
    queue_type_loop<PDG_HEX>(a, qtb, [&](int e) { volume_elem<PDG_HEX, N, NS, kBS<N>, true, Dm<PDG_HEX, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PRISM>(a, qtb, [&](int e) { volume_elem<PDG_PRISM, N, NS, kBS<N>, true, Dm<PDG_PRISM, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PYR>(a, qtb, [&](int e) { volume_elem<PDG_PYR, N, NS, kBS<N>, true, Dm<PDG_PYR, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_TET>(a, qtb, [&](int e) { volume_elem<PDG_TET, N, NS, kBS<N>, true, Dm<PDG_TET, N>::SLOTS, CV>(a, e, smem); });
    queue_clock_end(qt, t0);
}

template <int T, int N, bool NS, bool WIDE, bool CV = false>
__global__ __launch_bounds__(kBS<N>) void k_surface_ec(StageArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double sgs[SurfLDS<T, N, S>::size];
    surface_elem<T, N, NS, true, S, CV>(a, (WIDE ? a.list_w : a.list_n)[T][blockIdx.x], sgs);
}

template <int N, bool NS, bool CV = false>
__global__ __launch_bounds__(kBS<N>) void k_surface_ec_q(StageArgs a, const int32_t *qtb, uint64_t *qt) {
    constexpr int SZ = cmax4s(SurfLDS<0, N>::size, SurfLDS<1, N>::size, SurfLDS<2, N>::size, SurfLDS<3, N>::size);
    __shared__ double smem[SZ];
    const long long t0 = queue_clock_begin();
    queue_type_loop<PDG_HEX>(a, qtb, [&](int e) { surface_elem<PDG_HEX, N, NS, true, Dm<PDG_HEX, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PRISM>(a, qtb, [&](int e) { surface_elem<PDG_PRISM, N, NS, true, Dm<PDG_PRISM, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PYR>(a, qtb, [&](int e) { surface_elem<PDG_PYR, N, NS, true, Dm<PDG_PYR, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_TET>(a, qtb, [&](int e) { surface_elem<PDG_TET, N, NS, true, Dm<PDG_TET, N>::SLOTS, CV>(a, e, smem); });
    queue_clock_end(qt, t0);
}

template <int T, int N, bool NS>
static void go_surf_ec_nw(const StageArgs &a, hipStream_t s) {
    if (a.mesh.nmet) {  // curved mesh: conforming faces, every element in the narrow list
        if (a.count_n[T]) hipLaunchKernelGGL((k_surface_ec<T, N, NS, false, true>), dim3(a.count_n[T]), dim3(Dm<T, N>::BS), 0, s, a);
        return;
    }
    if (a.count_n[T]) hipLaunchKernelGGL((k_surface_ec<T, N, NS, false>), dim3(a.count_n[T]), dim3(Dm<T, N>::BS), 0, s, a);
    if (a.count_w[T]) hipLaunchKernelGGL((k_surface_ec<T, N, NS, true>), dim3(a.count_w[T]), dim3(Dm<T, N>::BS), 0, s, a);
}
template <int T, int N>
static void go_surf_ec(const StageArgs &a, bool ns, hipStream_t s) {
    if (!ns) {
        go_surf_ec_nw<T, N, false>(a, s);
    } else if constexpr (N <= 5) {
        go_surf_ec_nw<T, N, true>(a, s);
    }
}

template <int N>
static void goq_surf_ec(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    const bool cv = a.mesh.nmet != nullptr;
    if (!ns) {
        if (cv) hipLaunchKernelGGL((k_surface_ec_q<N, false, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
        else hipLaunchKernelGGL((k_surface_ec_q<N, false>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
    } else if constexpr (N <= 5) {
        if (cv) hipLaunchKernelGGL((k_surface_ec_q<N, true, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
        else hipLaunchKernelGGL((k_surface_ec_q<N, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
    }
}

hipError_t launch_surface_ec(int N, bool ns, const StageArgs &a, int type, hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    if (ns && N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_TN(go_surf_ec, a, ns, s);
    return hipGetLastError();
}

hipError_t launch_surface_ec_queues(int N, bool ns, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                                    hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    if (ns && N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_N(goq_surf_ec, a, ns, qtb, nq, qt, s);
    return hipGetLastError();
}

template <int T, int N, bool NS>
static void go_vol_split_nw(const StageArgs &a, hipStream_t s) {
    if (a.mesh.nmet) {  // curved mesh: conforming faces, every element in the narrow list
        if (a.count_n[T]) hipLaunchKernelGGL((k_volume_split<T, N, NS, false, true>), dim3(a.count_n[T]), dim3(kVolBS<T, N>), 0, s, a);
        return;
    }
    if (a.count_n[T]) hipLaunchKernelGGL((k_volume_split<T, N, NS, false>), dim3(a.count_n[T]), dim3(kVolBS<T, N>), 0, s, a);
    if (a.count_w[T]) hipLaunchKernelGGL((k_volume_split<T, N, NS, true>), dim3(a.count_w[T]), dim3(kVolBS<T, N>), 0, s, a);
}
template <int T, int N>
static void go_vol_split(const StageArgs &a, bool ns, hipStream_t s) {
    if (!ns) {
        go_vol_split_nw<T, N, false>(a, s);
    } else if constexpr (N <= 5) {
        go_vol_split_nw<T, N, true>(a, s);
    }
}

template <int N>
static void goq_vol_split(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    const bool cv = a.mesh.nmet != nullptr;
    if (!ns) {
        if (cv) hipLaunchKernelGGL((k_volume_split_q<N, false, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
        else hipLaunchKernelGGL((k_volume_split_q<N, false>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
    } else if constexpr (N <= 5) {
        if (cv) hipLaunchKernelGGL((k_volume_split_q<N, true, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
        else hipLaunchKernelGGL((k_volume_split_q<N, true>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
    }
}

hipError_t launch_volume_split(int N, bool ns, const StageArgs &a, int type, hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    if (ns && N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_TN(go_vol_split, a, ns, s);
    return hipGetLastError();
}

hipError_t launch_volume_split_queues(int N, bool ns, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                                      hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    if (ns && N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_N(goq_vol_split, a, ns, qtb, nq, qt, s);
    return hipGetLastError();
}

}  // namespace pdg
