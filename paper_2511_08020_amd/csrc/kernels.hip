// Device kernels of the DG residual on mixed meshes (gfx950, FP64).
//
// One residual evaluation (paper Sec. 2, Eq. (1) and Algorithm 1) is three phases, each one
// workgroup per element, launched per element type:
//   trace    state at the n^2 points of every face side of the element (hexahedra: gather /
//            plane interpolation of nodal values; other types: phi_j at the points, E u~)
//   volume   nodal state (V u~ for modal elements), pointwise flux, contravariant transform,
//            sum-factorised weak derivative in LDS, and for modal elements the projection
//            P^ = M_D^-1 V^T W onto the modes (Algorithm 1); Navier-Stokes adds the BR1
//            gradients (nodal on hexahedra, modal on the other types) and the viscous normal
//            flux at the element's face points
//   surface  Lax-Friedrichs flux from both sides' traces (each side evaluates it with its own
//            outward normal; the flux is bitwise antisymmetric, so both sides see the same
//            value up to sign), lift, and either dU/dt or the LSERK stage update
// No floating-point atomics: every output is written by exactly one thread.
#include <cstdint>

#include "phases.h"

namespace pdg {

template <int T, int N>
__global__ __launch_bounds__(128) void k_trace(StageArgs a) {
    __shared__ double smem[TraceLDS<T, N>::size];
    trace_elem<T, N>(a, a.list[T][blockIdx.x], smem);
}

// at least four waves per SIMD: the modal kernels then fit in 128 registers without spilling.
// WIDE: the elements with more face sides than kSlotsNarrow (list_w), else the others (list_n)
// CV: a mesh with curved elements (per-node metrics, per-element mass matrices; conforming
// faces, so only the narrow kernels)
template <int T, int N, bool NS, bool WIDE, bool CV = false>
__global__ __launch_bounds__((kVolBS<T, N>), 4) void k_volume(StageArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double smem[VolLDS<T, N, NS, false, S>::size];
    volume_elem<T, N, NS, kVolBS<T, N>, false, S, CV>(a, (WIDE ? a.list_w : a.list_n)[T][blockIdx.x], smem);
}

template <int T, int N, bool NS, bool WIDE, bool CV = false>
__global__ __launch_bounds__(kBS<N>) void k_surface(StageArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double sgs[SurfLDS<T, N, S>::size];
    surface_elem<T, N, NS, false, S, CV>(a, (WIDE ? a.list_w : a.list_n)[T][blockIdx.x], sgs);
}

// ----------------------------------------------------------------- work-queue (segment) kernels
// One workgroup per queue: the elements [qb[q], qb[q+1]) of a contiguous Hilbert segment, of
// any type (the paper's contiguous SFC segments, Sec. 3), taken type by type so that only one
// type's code is live at a time (see queue_type_loop).
template <int N>
constexpr int cmax4(int a, int b, int c, int d) {
    return a > b ? (a > c ? (a > d ? a : d) : (c > d ? c : d)) : (b > c ? (b > d ? b : d) : (c > d ? c : d));
}

template <int N>
__global__ __launch_bounds__(kTraceQBS) void k_trace_q(StageArgs a, const int32_t *qtb, uint64_t *qt) {
    constexpr int SZ = cmax4<N>(TraceLDS<0, N>::size, TraceLDS<1, N>::size, TraceLDS<2, N>::size,
                                TraceLDS<3, N>::size);
    __shared__ double smem[SZ];
    const long long t0 = queue_clock_begin();
    queue_type_loop<PDG_HEX>(a, qtb, [&](int e) { trace_elem<PDG_HEX, N>(a, e, smem); });
    queue_type_loop<PDG_PRISM>(a, qtb, [&](int e) { trace_elem<PDG_PRISM, N>(a, e, smem); });
    queue_type_loop<PDG_PYR>(a, qtb, [&](int e) { trace_elem<PDG_PYR, N>(a, e, smem); });
    queue_type_loop<PDG_TET>(a, qtb, [&](int e) { trace_elem<PDG_TET, N>(a, e, smem); });
    queue_clock_end(qt, t0);
}

template <int N, bool NS, bool CV = false>
__global__ __launch_bounds__(kBS<N>, 2) void k_volume_q(StageArgs a, const int32_t *qtb, uint64_t *qt) {
    constexpr int SZ = cmax4<N>(VolLDS<0, N, NS>::size, VolLDS<1, N, NS>::size, VolLDS<2, N, NS>::size,
                                VolLDS<3, N, NS>::size);
    __shared__ double smem[SZ];
    const long long t0 = queue_clock_begin();
    constexpr int BS = kBS<N>;
    queue_type_loop<PDG_HEX>(a, qtb, [&](int e) { volume_elem<PDG_HEX, N, NS, BS, false, Dm<PDG_HEX, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PRISM>(a, qtb, [&](int e) { volume_elem<PDG_PRISM, N, NS, BS, false, Dm<PDG_PRISM, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PYR>(a, qtb, [&](int e) { volume_elem<PDG_PYR, N, NS, BS, false, Dm<PDG_PYR, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_TET>(a, qtb, [&](int e) { volume_elem<PDG_TET, N, NS, BS, false, Dm<PDG_TET, N>::SLOTS, CV>(a, e, smem); });
    queue_clock_end(qt, t0);
}

// workgroups per CU for four waves per SIMD, as the per-type surface kernels reach (at most 128
// registers; the compiler lowers the bound where LDS allows fewer workgroups)
template <int N>
constexpr int kSurfQBlocks = 16 / (kBS<N> / 64) > 1 ? 16 / (kBS<N> / 64) : 1;
template <int N, bool NS, bool CV = false>
__global__ __launch_bounds__(kBS<N>, kSurfQBlocks<N>) void k_surface_q(StageArgs a, const int32_t *qtb, uint64_t *qt) {
    constexpr int SZ = cmax4<N>(SurfLDS<0, N>::size, SurfLDS<1, N>::size, SurfLDS<2, N>::size,
                                SurfLDS<3, N>::size);
    __shared__ double smem[SZ];
    const long long t0 = queue_clock_begin();
    queue_type_loop<PDG_HEX>(a, qtb, [&](int e) { surface_elem<PDG_HEX, N, NS, false, Dm<PDG_HEX, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PRISM>(a, qtb, [&](int e) { surface_elem<PDG_PRISM, N, NS, false, Dm<PDG_PRISM, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_PYR>(a, qtb, [&](int e) { surface_elem<PDG_PYR, N, NS, false, Dm<PDG_PYR, N>::SLOTS, CV>(a, e, smem); });
    queue_type_loop<PDG_TET>(a, qtb, [&](int e) { surface_elem<PDG_TET, N, NS, false, Dm<PDG_TET, N>::SLOTS, CV>(a, e, smem); });
    queue_clock_end(qt, t0);
}

// ------------------------------------------------------------------- projection and nodal values
template <int T, int N>
__global__ __launch_bounds__(kBS<N>) void k_project(StageArgs a, const double *q, double *U) {
    using D = Dm<T, N>;
    constexpr int nn = D::nn, m = D::m, BS = D::BS;
    const int e = a.list[T][blockIdx.x];
    const int64_t off = a.mesh.off[e];
    const double *qe = q + (int64_t)e * 5 * nn;
    if constexpr (T == PDG_HEX) {
        for (int t = threadIdx.x; t < 5 * nn; t += BS) U[off + t] = qe[t];
    } else {
        // u~ = M_D^-1 V^T W J_D q  (the element's constant affine Jacobian cancels); curved
        // elements: u~ = M_e^-1 V^T W J q with the Jacobian at the nodes
        const bool cv = a.mesh.nmet != nullptr;
        __shared__ double sq[5 * nn];
        __shared__ double sr[5 * m];
        for (int t = threadIdx.x; t < 5 * nn; t += BS)
            sq[t] = qe[t] * (cv ? a.mesh.nmet[((int64_t)e * nn + t % nn) * 10] : a.tab[T].jd[t % nn]);
        __syncthreads();
        for (int t = threadIdx.x; t < 5 * m; t += BS) {
            const int v = t / m, j = t % m;
            const double *Pr = a.tab[T].VtW + (int64_t)j * nn;
            double acc = 0.0;
            for (int k = 0; k < nn; ++k) acc += Pr[k] * sq[v * nn + k];
            sr[t] = acc;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < 5 * m; t += BS) {
            const int v = t / m, j = t % m;
            const double *Mr = (cv ? a.mesh.minv + a.mesh.minv_off[e] : a.tab[T].Minv) + (int64_t)j * m;
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += Mr[k] * sr[v * m + k];
            U[off + t] = acc;
        }
    }
}

template <int T, int N>
__global__ __launch_bounds__(kBS<N>) void k_nodal(StageArgs a, const double *U, double *q) {
    using D = Dm<T, N>;
    constexpr int nn = D::nn, m = D::m, BS = D::BS;
    const int e = a.list[T][blockIdx.x];
    const int64_t off = a.mesh.off[e];
    double *qe = q + (int64_t)e * 5 * nn;
    if constexpr (T == PDG_HEX) {
        for (int t = threadIdx.x; t < 5 * nn; t += BS) qe[t] = U[off + t];
    } else {
        __shared__ double su[5 * m];
        for (int t = threadIdx.x; t < 5 * m; t += BS) su[t] = U[off + t];
        __syncthreads();
        const int k = threadIdx.x;
        if (k < nn) {
            const double *Vr = a.tab[T].V + (int64_t)k * m;
            double acc[5] = {0, 0, 0, 0, 0};
            for (int j = 0; j < m; ++j)
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] += Vr[j] * su[v * m + j];
#pragma unroll
            for (int v = 0; v < 5; ++v) qe[v * nn + k] = acc[v];
        }
    }
}

// ---------------------------------------------------------------------------------- launches
template <int T, int N>
static void go_trace(const StageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_trace<T, N>), dim3(a.count[T]), dim3(128), 0, s, a);
}
// the narrow and the wide part of a type's elements, one launch each
template <int T, int N, bool NS>
static void go_vol(const StageArgs &a, hipStream_t s) {
    if (a.mesh.nmet) {  // curved mesh: conforming faces, every element in the narrow list
        if (a.count_n[T]) hipLaunchKernelGGL((k_volume<T, N, NS, false, true>), dim3(a.count_n[T]), dim3(kVolBS<T, N>), 0, s, a);
        return;
    }
    if (a.count_n[T]) hipLaunchKernelGGL((k_volume<T, N, NS, false>), dim3(a.count_n[T]), dim3(kVolBS<T, N>), 0, s, a);
    if (a.count_w[T]) hipLaunchKernelGGL((k_volume<T, N, NS, true>), dim3(a.count_w[T]), dim3(kVolBS<T, N>), 0, s, a);
}
template <int T, int N>
static void go_vol_euler(const StageArgs &a, hipStream_t s) {
    go_vol<T, N, false>(a, s);
}
// Navier-Stokes kernels exist for N <= 5 (N = 6 would exceed the 160 KB of LDS per workgroup)
template <int T, int N>
static void go_vol_ns(const StageArgs &a, hipStream_t s) {
    if constexpr (N <= 5) go_vol<T, N, true>(a, s);
}
template <int T, int N, bool NS>
static void go_surf(const StageArgs &a, hipStream_t s) {
    if (a.mesh.nmet) {
        if (a.count_n[T]) hipLaunchKernelGGL((k_surface<T, N, NS, false, true>), dim3(a.count_n[T]), dim3(Dm<T, N>::BS), 0, s, a);
        return;
    }
    if (a.count_n[T]) hipLaunchKernelGGL((k_surface<T, N, NS, false>), dim3(a.count_n[T]), dim3(Dm<T, N>::BS), 0, s, a);
    if (a.count_w[T]) hipLaunchKernelGGL((k_surface<T, N, NS, true>), dim3(a.count_w[T]), dim3(Dm<T, N>::BS), 0, s, a);
}
template <int T, int N>
static void go_surf_euler(const StageArgs &a, hipStream_t s) {
    go_surf<T, N, false>(a, s);
}
template <int T, int N>
static void go_surf_ns(const StageArgs &a, hipStream_t s) {
    if constexpr (N <= 5) go_surf<T, N, true>(a, s);
}
template <int T, int N>
static void go_project(const StageArgs &a, const double *q, double *U, hipStream_t s) {
    hipLaunchKernelGGL((k_project<T, N>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a, q, U);
}
template <int T, int N>
static void go_nodal(const StageArgs &a, const double *U, double *q, hipStream_t s) {
    hipLaunchKernelGGL((k_nodal<T, N>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a, U, q);
}

hipError_t launch_trace(int N, const StageArgs &a, int type, hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    PDG_DISPATCH_TN(go_trace, a, s);
    return hipGetLastError();
}
hipError_t launch_volume(int N, bool ns, const StageArgs &a, int type, hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    if (ns) {
        PDG_DISPATCH_TN(go_vol_ns, a, s);
    } else {
        PDG_DISPATCH_TN(go_vol_euler, a, s);
    }
    return hipGetLastError();
}
hipError_t launch_surface(int N, bool ns, const StageArgs &a, int type, hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    if (ns) {
        PDG_DISPATCH_TN(go_surf_ns, a, s);
    } else {
        PDG_DISPATCH_TN(go_surf_euler, a, s);
    }
    return hipGetLastError();
}
template <int N>
static void goq_trace(const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    hipLaunchKernelGGL((k_trace_q<N>), dim3(nq * a.qsub), dim3(kTraceQBS), 0, s, a, qtb, qt);
}
template <int N, bool CV>
static void goq_vol_cv(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    if constexpr (N <= 5) {
        if (ns) { hipLaunchKernelGGL((k_volume_q<N, true, CV>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt); return; }
    }
    if (!ns) hipLaunchKernelGGL((k_volume_q<N, false, CV>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
}
template <int N>
static void goq_vol(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    if (a.mesh.nmet) goq_vol_cv<N, true>(a, ns, qtb, nq, qt, s);
    else goq_vol_cv<N, false>(a, ns, qtb, nq, qt, s);
}
template <int N, bool CV>
static void goq_surf_cv(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    if constexpr (N <= 5) {
        if (ns) { hipLaunchKernelGGL((k_surface_q<N, true, CV>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt); return; }
    }
    if (!ns) hipLaunchKernelGGL((k_surface_q<N, false, CV>), dim3(nq * a.qsub), dim3(kBS<N>), 0, s, a, qtb, qt);
}
template <int N>
static void goq_surf(const StageArgs &a, bool ns, const int32_t *qtb, int nq, uint64_t *qt, hipStream_t s) {
    if (a.mesh.nmet) goq_surf_cv<N, true>(a, ns, qtb, nq, qt, s);
    else goq_surf_cv<N, false>(a, ns, qtb, nq, qt, s);
}

hipError_t launch_queues(int N, bool ns, int phase, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                         hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    if (phase == 0) {
        PDG_DISPATCH_N(goq_trace, a, qtb, nq, qt, s);
    } else if (phase == 1) {
        PDG_DISPATCH_N(goq_vol, a, ns, qtb, nq, qt, s);
    } else {
        PDG_DISPATCH_N(goq_surf, a, ns, qtb, nq, qt, s);
    }
    return hipGetLastError();
}

template <int N>
static void occ_q(bool ns, int phase, int *nb) {
    const void *k = reinterpret_cast<const void *>(&k_trace_q<N>);
    int bs = kTraceQBS;
    if (phase == 1) {
        bs = kBS<N>;
        k = reinterpret_cast<const void *>(&k_volume_q<N, false>);
        if constexpr (N <= 5)
            if (ns) k = reinterpret_cast<const void *>(&k_volume_q<N, true>);
    } else if (phase == 2) {
        bs = kBS<N>;
        k = ns ? reinterpret_cast<const void *>(&k_surface_q<N, true>)
               : reinterpret_cast<const void *>(&k_surface_q<N, false>);
    }
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k, bs, 0);
}
static hipError_t occ_dispatch(int N, bool ns, int phase, int *nb) {
    PDG_DISPATCH_N(occ_q, ns, phase, nb);
    return hipSuccess;
}
int queue_occupancy(int N, bool ns, int phase) {
    int nb = 0;
    if (occ_dispatch(N, ns, phase, &nb) != hipSuccess || nb < 1) return 1;
    return nb;
}

hipError_t launch_project(int N, const StageArgs &a, int type, const double *q, double *U,
                          hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    PDG_DISPATCH_TN(go_project, a, q, U, s);
    return hipGetLastError();
}
hipError_t launch_nodal(int N, const StageArgs &a, int type, const double *U, double *q,
                        hipStream_t s) {
    if (a.count[type] == 0) return hipSuccess;
    PDG_DISPATCH_TN(go_nodal, a, U, q, s);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ SFC keys
// Skilling's transpose form of the Hilbert index (AIP Conf. Proc. 707, 2004), 3 axes
__global__ void k_sfc_keys(int n, const double *cen, double lo0, double lo1, double lo2, double scale,
                           uint64_t *keys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int B = 21;
    constexpr uint64_t MAXV = (1ull << B) - 1;
    const double lo[3] = {lo0, lo1, lo2};
    uint64_t X[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        // exactly one subtraction and one multiplication, no contraction
        const double v = floor(__dmul_rn(__dsub_rn(cen[3 * (int64_t)i + ax], lo[ax]), scale));
        X[ax] = v <= 0.0 ? 0ull : (v >= (double)MAXV ? MAXV : (uint64_t)v);
    }
    const uint64_t M = 1ull << (B - 1);
    for (uint64_t Q = M; Q > 1; Q >>= 1) {
        const uint64_t P = Q - 1;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (X[ax] & Q) {
                X[0] ^= P;
            } else {
                const uint64_t t = (X[0] ^ X[ax]) & P;
                X[0] ^= t;
                X[ax] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint64_t t = 0;
    for (uint64_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    X[0] ^= t; X[1] ^= t; X[2] ^= t;
    uint64_t key = 0;
    for (int b = B - 1; b >= 0; --b)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) key = (key << 1) | ((X[ax] >> b) & 1ull);
    keys[i] = key;
}

hipError_t launch_sfc_keys(int n, const double *centroid, const double lo[3], double scale,
                           uint64_t *keys, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sfc_keys, dim3((n + 255) / 256), dim3(256), 0, s, n, centroid, lo[0], lo[1],
                       lo[2], scale, keys);
    return hipGetLastError();
}

// ------------------------------------------------------------------------- element weights
__global__ void k_type_weights(int n, const int8_t *etype, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                               uint32_t *weight) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = etype[i];
    weight[i] = t == 0 ? w0 : (t == 1 ? w1 : (t == 2 ? w2 : w3));
}

hipError_t launch_type_weights(int n, const int8_t *etype, const uint32_t wt[4], uint32_t *weight, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_type_weights, dim3((n + 255) / 256), dim3(256), 0, s, n, etype, wt[0], wt[1], wt[2], wt[3],
                       weight);
    return hipGetLastError();
}

// ------------------------------------------------------------------------ weighted partition
// one workgroup: chunked exclusive u64 prefix sum of the weights, then midpoint queue bounds
__global__ __launch_bounds__(1024) void k_partition(int n, const uint32_t *w, int nq, int32_t *qb,
                                                    uint64_t *S) {
    __shared__ uint64_t part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (n + nt - 1) / nt;
    const int b0 = min(n, tid * chunk), b1 = min(n, b0 + chunk);
    uint64_t loc = 0;
    for (int i = b0; i < b1; ++i) loc += w[i];
    part[tid] = loc;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {  // inclusive Hillis-Steele scan of the chunk sums
        const uint64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - loc;
    for (int i = b0; i < b1; ++i) {
        S[i] = run;
        run += w[i];
    }
    const uint64_t W = part[nt - 1];
    __threadfence_block();
    __syncthreads();
    if (W == 0) {
        for (int q = tid; q <= nq; q += nt) qb[q] = q == nq ? n : 0;
        return;
    }
    // queue(i) = min(Q - 1, Q (2 S_i + w_i) / (2W)) in 128-bit arithmetic (S_i + w_i <= W < 2^63
    // for 32-bit weights and n < 2^31, so 2 S_i + w_i fits 64 bits; the product by Q may not)
    const auto queue_of = [&](int i) -> int64_t {
        const unsigned __int128 num = (unsigned __int128)(uint64_t)nq * (2 * S[i] + w[i]);
        const uint64_t qi = (uint64_t)(num / ((unsigned __int128)2 * W));
        return qi < (uint64_t)nq ? (int64_t)qi : (int64_t)nq - 1;
    };
    for (int i = tid; i < n; i += nt) {
        const int64_t qi = queue_of(i);
        const int64_t qprev = i == 0 ? -1 : queue_of(i - 1);
        for (int64_t q = qprev + 1; q <= qi; ++q) qb[q] = i;
        if (i == n - 1)
            for (int64_t q = qi + 1; q <= nq; ++q) qb[q] = n;
    }
}

hipError_t launch_partition(int n, const uint32_t *w, int nq, int32_t *qb, uint64_t *scratch,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_partition, dim3(1), dim3(1024), 0, s, n, w, nq, qb, scratch);
    return hipGetLastError();
}

}  // namespace pdg
