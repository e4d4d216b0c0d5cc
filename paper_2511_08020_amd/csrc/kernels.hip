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

#include "device.h"

namespace pdg {

// ------------------------------------------------------------------------------- trace phase
template <int T, int N>
struct TraceLDS {
    static constexpr int ops = 5 * Dm<T, N>::m;              // int64 op offsets per local side
    static constexpr int size = ops + Dm<T, N>::SLOTS;
};

template <int T, int N>
__device__ __forceinline__ void trace_elem(const StageArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m;
    double *su = smem;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + TraceLDS<T, N>::ops);
    const int64_t off = a.mesh.off[e];
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    for (int t = threadIdx.x; t < 5 * m; t += blockDim.x) su[t] = a.U[off + t];
    for (int t = threadIdx.x; t < s1 - s0; t += blockDim.x) sops[t] = a.ops.op_off[a.mesh.slot_op[s0 + t]];
    __syncthreads();
    if constexpr (T == PDG_HEX) {
        for (int t = threadIdx.x; t < (s1 - s0) * n2; t += blockDim.x) {
            const int sl = s0 + t / n2, p = t % n2;
            const int op = a.mesh.slot_op[sl];
            double acc[5] = {0, 0, 0, 0, 0};
            const int plane = a.ops.op_plane[op];
            if (a.ops.op_perm[op]) {
                const int k = plane_vol(plane, a.ops.idata[a.ops.op_ioff[op] + p], n);
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] = su[v * nn + k];
            } else {
                const double *I = a.ops.data + a.ops.op_off[op] + (int64_t)p * n2;
                for (int a2 = 0; a2 < n2; ++a2) {
                    const int k = plane_vol(plane, a2, n);
                    const double c = I[a2];
#pragma unroll
                    for (int v = 0; v < 5; ++v) acc[v] += c * su[v * nn + k];
                }
            }
            double *dst = a.Tq + (int64_t)sl * 5 * n2 + p;
#pragma unroll
            for (int v = 0; v < 5; ++v) dst[v * n2] = acc[v];
        }
    } else {
        // traces of all face sides at once: rows (side, point), E = phi(face points)
        const double *data = a.ops.data;
        double *Tq = a.Tq;
        mfma_gemm((s1 - s0) * n2, m, 5,
                  [&](int i, int k) { return data[sops[i / n2] + (int64_t)(i % n2) * m + k]; },
                  [&](int k, int c) { return su[c * m + k]; },
                  [&](int i, int c, double v) { Tq[((int64_t)(s0 + i / n2) * 5 + c) * n2 + i % n2] = v; });
    }
}

template <int T, int N>
__global__ __launch_bounds__(128) void k_trace(StageArgs a) {
    __shared__ double smem[TraceLDS<T, N>::size];
    trace_elem<T, N>(a, a.list[T][blockIdx.x], smem);
}

// ------------------------------------------------------------------------------ volume phase
// LDS of one element in the volume phase, laid out by buffer lifetime:
//   q    nodal state, later the weak derivative d                          5 nn
//   A    NS: volume part of the gradient, later the gradient at the nodes  12 nn
//   B    NS: face terms of all sides, later the gradient at face points     12 S n2
//        (modal: the state coefficients u~ live here before that)
//   C    NS modal: BR1 right-hand side and gradient coefficients           24 m
//        (the lifting variables, 4 nn, live here before that)
//   G    contravariant fluxes, 15 nn; aliases A, B and C once the gradients are consumed
template <int T, int N, bool NS>
struct VolLDS {
    using D = Dm<T, N>;
    static constexpr bool MODAL = T != PDG_HEX;
    static constexpr int nn = D::nn, m = D::m, n2 = D::n2;
    static constexpr int cmax(int x, int y) { return x > y ? x : y; }
    static constexpr int q = 0;
    static constexpr int dh = q + 5 * nn;
    static constexpr int ops = dh + 3 * D::n * D::n;
    static constexpr int A = ops + D::SLOTS;
    static constexpr int szA = NS ? 12 * nn : 0;
    static constexpr int B = A + szA;
    static constexpr int szB = NS ? 12 * (MODAL ? D::SLOTS : 1) * n2 : 0;
    static constexpr int C = B + cmax(szB, MODAL ? 5 * m : 0);
    static constexpr int szC = NS ? cmax(MODAL ? 24 * m : 0, 4 * nn) : 0;
    static constexpr int u = MODAL ? B : 0;       // u~ (5 m) before B is used
    static constexpr int w = C;                   // lifting variables (4 nn) before C is used
    static constexpr int G = NS ? A : C;          // fluxes after the gradient phase
    static constexpr int size = cmax(C + szC, G + 15 * nn);
};

template <int T, int N, bool NS>
__device__ __forceinline__ void volume_elem(const StageArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    using L = VolLDS<T, N, NS>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m, BS = D::BS;
    constexpr bool MODAL = T != PDG_HEX;
    double *sq = smem + L::q;
    double *sG = smem + L::G;
    double *sdh = smem + L::dh;
    double *su = smem + L::u;
    double *sgn = smem + L::A;
    double *sgm = smem + L::C;       // modal BR1 right-hand side (12 m)
    double *sgt = smem + L::C + 12 * m;  // modal BR1 gradient coefficients (12 m)
    double *sbuf = smem + L::B;      // face terms / gradient at the face points
    double *sw = smem + L::w;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + L::ops);

    const int tid = threadIdx.x;
    const int64_t off = a.mesh.off[e];
    const DevType &tab = a.tab[T];
    const double *geo = a.mesh.geo + 10 * (int64_t)e;
    const double Jaff = geo[0];
    const double iJ = 1.0 / Jaff;
    double cofT[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) cofT[i] = geo[1 + i];
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0;

    for (int t = tid; t < 3 * n * n; t += BS) sdh[t] = tab.dhat[t / (n * n)][t % (n * n)];
    for (int t = tid; t < nsl; t += BS) sops[t] = a.ops.op_off[a.mesh.slot_op[s0 + t]];
    if constexpr (MODAL) {
        for (int t = tid; t < 5 * m; t += BS) su[t] = a.U[off + t];
        __syncthreads();
        // nodal state q = V u~
        const double *V = tab.V;
        mfma_gemm(nn, m, 5, [&](int i, int k) { return V[i * m + k]; }, [&](int k, int c) { return su[c * m + k]; },
                  [&](int i, int c, double v) { sq[c * nn + i] = v; });
    }
    __syncthreads();

    const int k = tid;
    const bool act = k < nn;
    const int ii[3] = {k % n, (k / n) % n, k / (n * n)};
    const int stride[3] = {1, n, n * n};
    double q[5] = {1, 0, 0, 0, 1};
    if (act) {
        if constexpr (MODAL) {
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = sq[v * nn + k];
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = a.U[off + v * nn + k];
        }
    }

    double g[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) g[f] = 0.0;

    if constexpr (NS) {
        br1_gradients<T, N>(a, s0, s1, cofT, iJ, q, sops, sdh, sw, sgn, sbuf, sgm, sgt, g);
        // viscous normal flux Fv(q, g).n_out at this element's face points
        const int np = nsl * n2;
        for (int t = tid; t < np; t += BS) {
            const int sl = s0 + t / n2, p = t % n2;
            const int op = a.mesh.slot_op[sl];
            const double *sg = a.mesh.slot_geo + 4 * (int64_t)sl;
            double qa[5], gp[12];
#pragma unroll
            for (int v = 0; v < 5; ++v) qa[v] = a.Tq[((int64_t)sl * 5 + v) * n2 + p];
#pragma unroll
            for (int f = 0; f < 12; ++f) gp[f] = 0.0;
            if constexpr (MODAL) {
#pragma unroll
                for (int f = 0; f < 12; ++f) gp[f] = sbuf[f * np + t];
            } else {
                const int plane = a.ops.op_plane[op];
                if (a.ops.op_perm[op]) {
                    const int kk = plane_vol(plane, a.ops.idata[a.ops.op_ioff[op] + p], n);
#pragma unroll
                    for (int f = 0; f < 12; ++f) gp[f] = sgn[f * nn + kk];
                } else {
                    const double *I = a.ops.data + a.ops.op_off[op] + (int64_t)p * n2;
                    for (int a2 = 0; a2 < n2; ++a2) {
                        const int kk = plane_vol(plane, a2, n);
                        const double c = I[a2];
#pragma unroll
                        for (int f = 0; f < 12; ++f) gp[f] += c * sgn[f * nn + kk];
                    }
                }
            }
            double Fv[3][5];
            visc_flux(qa, gp, a.phys, Fv);
#pragma unroll
            for (int v = 0; v < 5; ++v)
                a.Fvn[((int64_t)sl * 5 + v) * n2 + p] = Fv[0][v] * sg[0] + Fv[1][v] * sg[1] + Fv[2][v] * sg[2];
        }
        __syncthreads();  // gradient buffers are dead from here on (the fluxes reuse them)
    }

    // pointwise flux and contravariant transform
    if (act) {
        double F[3][5];
        euler_flux(q, a.phys.gamma, a.phys.p_ref, F);
        if constexpr (NS) {
            double Fv[3][5];
            visc_flux(q, g, a.phys, Fv);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int v = 0; v < 5; ++v) F[c][v] -= Fv[c][v];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double Fh[3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                Fh[b] = cofT[b * 3 + 0] * F[0][v] + cofT[b * 3 + 1] * F[1][v] + cofT[b * 3 + 2] * F[2][v];
            if constexpr (MODAL) {
                const double *c = tab.cmet + k * 9;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax)
                    sG[(ax * 5 + v) * nn + k] = c[ax * 3 + 0] * Fh[0] + c[ax * 3 + 1] * Fh[1] + c[ax * 3 + 2] * Fh[2];
            } else {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) sG[(ax * 5 + v) * nn + k] = Fh[ax];
            }
        }
    }
    __syncthreads();
    // sum-factorised weak derivative d_k = sum_a sum_l Dhat_a[i_a][l] G^a(.. l ..)
    if (act) {
        double d[5] = {0, 0, 0, 0, 0};
        for (int ax = 0; ax < 3; ++ax) {
            const int base = k - ii[ax] * stride[ax];
            for (int l = 0; l < n; ++l) {
                const double dh = sdh[ax * n * n + ii[ax] * n + l];
                const int mm = base + l * stride[ax];
#pragma unroll
                for (int v = 0; v < 5; ++v) d[v] += dh * sG[(ax * 5 + v) * nn + mm];
            }
        }
        if constexpr (MODAL) {
#pragma unroll
            for (int v = 0; v < 5; ++v) sq[v * nn + k] = d[v];
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) a.Rp[off + v * nn + k] = d[v] * iJ;
        }
    }
    if constexpr (MODAL) {
        __syncthreads();
        // volume part of the modal right-hand side, V^T W d / J (M_D^-1 follows the lift)
        const double *VtW = tab.VtW;
        double *Rp = a.Rp + off;
        mfma_gemm(m, nn, 5, [&](int i, int kk) { return VtW[i * nn + kk]; },
                  [&](int kk, int c) { return sq[c * nn + kk]; },
                  [&](int i, int c, double v) { Rp[c * m + i] = v * iJ; });
    }
}

template <int T, int N, bool NS>
__global__ __launch_bounds__(kBS<N>) void k_volume(StageArgs a) {
    __shared__ double smem[VolLDS<T, N, NS>::size];
    volume_elem<T, N, NS>(a, a.list[T][blockIdx.x], smem);
}

// ----------------------------------------------------------------------------- surface phase
template <int T, int N>
struct SurfLDS {
    static constexpr int rhs = Dm<T, N>::SLOTS * 5 * Dm<T, N>::n2;
    static constexpr int ops = rhs + (T != PDG_HEX ? 5 * Dm<T, N>::m : 0);
    static constexpr int size = ops + Dm<T, N>::SLOTS;
};

template <int T, int N, bool NS>
__device__ __forceinline__ void surface_elem(const StageArgs &a, int e, double *sgs) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m, BS = D::BS;
    constexpr bool MODAL = T != PDG_HEX;
    const int tid = threadIdx.x;
    const int64_t off = a.mesh.off[e];
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0;
    const double Jaff = a.mesh.geo[10 * (int64_t)e];
    int64_t *sops = reinterpret_cast<int64_t *>(sgs + SurfLDS<T, N>::ops);
    for (int t = tid; t < nsl; t += BS) sops[t] = a.ops.op_off[a.mesh.slot_op[s0 + t]];
    for (int t = tid; t < nsl * n2; t += BS) {
        const int ls = t / n2, p = t % n2, sl = s0 + ls;
        const int nb = a.mesh.slot_nbr[sl];
        const double *sg = a.mesh.slot_geo + 4 * (int64_t)sl;
        double qa[5], qb[5], f[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qa[v] = a.Tq[((int64_t)sl * 5 + v) * n2 + p];
            qb[v] = a.Tq[((int64_t)nb * 5 + v) * n2 + p];
        }
        const double nv[3] = {sg[0], sg[1], sg[2]};
        lf_flux(qa, qb, nv, a.phys.gamma, a.phys.p_ref, f);
        if constexpr (NS) {
#pragma unroll
            for (int v = 0; v < 5; ++v)
                f[v] -= 0.5 * (a.Fvn[((int64_t)sl * 5 + v) * n2 + p] - a.Fvn[((int64_t)nb * 5 + v) * n2 + p]);
        }
        const double ws = a.ops.Wq[a.mesh.slot_kind[sl] * n2 + p] * sg[3];
#pragma unroll
        for (int v = 0; v < 5; ++v) sgs[(ls * 5 + v) * n2 + p] = ws * f[v];
    }
    __syncthreads();
    const double iJ = 1.0 / Jaff;
    if constexpr (MODAL) {
        // rhs = volume part - E^T (face terms) / J over all sides; then dU~/dt = M_D^-1 rhs
        double *srhs = sgs + SurfLDS<T, N>::rhs;
        const double *data = a.ops.data;
        const double *Rp = a.Rp + off;
        mfma_gemm(m, nsl * n2, 5,
                  [&](int i, int kk) { return data[sops[kk / n2] + (int64_t)n2 * m + (int64_t)i * n2 + kk % n2]; },
                  [&](int kk, int c) { return sgs[((kk / n2) * 5 + c) * n2 + kk % n2]; },
                  [&](int i, int c, double v) { srhs[c * m + i] = Rp[c * m + i] - v * iJ; });
        __syncthreads();
        const double *Minv = a.tab[T].Minv;
        const int mode = a.mode;
        const double rk_a = a.rk_a, rk_bdt = a.rk_bdt;
        double *out = a.out + off, *Kr = a.K + off, *Uw = a.Uw + off;
        mfma_gemm(m, m, 5, [&](int i, int kk) { return Minv[i * m + kk]; },
                  [&](int kk, int c) { return srhs[c * m + kk]; },
                  [&](int i, int c, double R) {
                      const int idx = c * m + i;
                      if (mode == 0) {
                          out[idx] = R;
                      } else {
                          const double Kn = (rk_a == 0.0) ? R : rk_a * Kr[idx] + R;
                          Kr[idx] = Kn;
                          Uw[idx] = Uw[idx] + rk_bdt * Kn;
                      }
                  });
    } else {
        const int k = tid;
        if (k < nn) {
            double lift[5] = {0, 0, 0, 0, 0};
            for (int sl = s0; sl < s1; ++sl) {
                const int op = a.mesh.slot_op[sl];
                const int a2 = vol_plane(a.ops.op_plane[op], k, n);
                if (a2 < 0) continue;
                const double *gs = sgs + (sl - s0) * 5 * n2;
                if (a.ops.op_perm[op]) {
                    const int p = a.ops.idata[a.ops.op_ioff[op] + n2 + a2];
#pragma unroll
                    for (int v = 0; v < 5; ++v) lift[v] += gs[v * n2 + p];
                } else {
                    const double *I = a.ops.data + a.ops.op_off[op];
                    for (int p = 0; p < n2; ++p) {
                        const double c = I[(int64_t)p * n2 + a2];
#pragma unroll
                        for (int v = 0; v < 5; ++v) lift[v] += c * gs[v * n2 + p];
                    }
                }
            }
            const double sc = iJ / a.tab[T].w[k];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const int64_t idx = off + v * nn + k;
                const double R = a.Rp[idx] - lift[v] * sc;
                if (a.mode == 0) {
                    a.out[idx] = R;
                } else {
                    const double Kn = (a.rk_a == 0.0) ? R : a.rk_a * a.K[idx] + R;
                    a.K[idx] = Kn;
                    a.Uw[idx] = a.Uw[idx] + a.rk_bdt * Kn;
                }
            }
        }
    }
}

template <int T, int N, bool NS>
__global__ __launch_bounds__(kBS<N>) void k_surface(StageArgs a) {
    __shared__ double sgs[SurfLDS<T, N>::size];
    surface_elem<T, N, NS>(a, a.list[T][blockIdx.x], sgs);
}

// ----------------------------------------------------------------- work-queue (segment) kernels
// One workgroup per queue: the elements [qb[q], qb[q+1]) of a contiguous Hilbert segment, of
// any type, processed in order (the paper's contiguous SFC segments, Sec. 3).
template <int N>
constexpr int cmax4(int a, int b, int c, int d) {
    return a > b ? (a > c ? (a > d ? a : d) : (c > d ? c : d)) : (b > c ? (b > d ? b : d) : (c > d ? c : d));
}

template <int N>
__global__ __launch_bounds__(kBS<N>) void k_trace_q(StageArgs a, const int32_t *qb) {
    constexpr int SZ = cmax4<N>(TraceLDS<0, N>::size, TraceLDS<1, N>::size, TraceLDS<2, N>::size,
                                TraceLDS<3, N>::size);
    __shared__ double smem[SZ];
    for (int e = qb[blockIdx.x]; e < qb[blockIdx.x + 1]; ++e) {
        switch (a.mesh.etype[e]) {
            case PDG_HEX: trace_elem<PDG_HEX, N>(a, e, smem); break;
            case PDG_PRISM: trace_elem<PDG_PRISM, N>(a, e, smem); break;
            case PDG_PYR: trace_elem<PDG_PYR, N>(a, e, smem); break;
            default: trace_elem<PDG_TET, N>(a, e, smem); break;
        }
        __syncthreads();
    }
}

template <int N, bool NS>
__global__ __launch_bounds__(kBS<N>) void k_volume_q(StageArgs a, const int32_t *qb) {
    constexpr int SZ = cmax4<N>(VolLDS<0, N, NS>::size, VolLDS<1, N, NS>::size, VolLDS<2, N, NS>::size,
                                VolLDS<3, N, NS>::size);
    __shared__ double smem[SZ];
    for (int e = qb[blockIdx.x]; e < qb[blockIdx.x + 1]; ++e) {
        switch (a.mesh.etype[e]) {
            case PDG_HEX: volume_elem<PDG_HEX, N, NS>(a, e, smem); break;
            case PDG_PRISM: volume_elem<PDG_PRISM, N, NS>(a, e, smem); break;
            case PDG_PYR: volume_elem<PDG_PYR, N, NS>(a, e, smem); break;
            default: volume_elem<PDG_TET, N, NS>(a, e, smem); break;
        }
        __syncthreads();
    }
}

template <int N, bool NS>
__global__ __launch_bounds__(kBS<N>) void k_surface_q(StageArgs a, const int32_t *qb) {
    constexpr int SZ = cmax4<N>(SurfLDS<0, N>::size, SurfLDS<1, N>::size, SurfLDS<2, N>::size,
                                SurfLDS<3, N>::size);
    __shared__ double smem[SZ];
    for (int e = qb[blockIdx.x]; e < qb[blockIdx.x + 1]; ++e) {
        switch (a.mesh.etype[e]) {
            case PDG_HEX: surface_elem<PDG_HEX, N, NS>(a, e, smem); break;
            case PDG_PRISM: surface_elem<PDG_PRISM, N, NS>(a, e, smem); break;
            case PDG_PYR: surface_elem<PDG_PYR, N, NS>(a, e, smem); break;
            default: surface_elem<PDG_TET, N, NS>(a, e, smem); break;
        }
        __syncthreads();
    }
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
        // u~ = M_D^-1 V^T W J_D q  (the element's constant affine Jacobian cancels)
        __shared__ double sq[5 * nn];
        __shared__ double sr[5 * m];
        for (int t = threadIdx.x; t < 5 * nn; t += BS) sq[t] = qe[t] * a.tab[T].jd[t % nn];
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
            const double *Mr = a.tab[T].Minv + (int64_t)j * m;
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
template <int T, int N>
static void go_vol_euler(const StageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_volume<T, N, false>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a);
}
// Navier-Stokes kernels exist for N <= 5 (N = 6 would exceed the 160 KB of LDS per workgroup)
template <int T, int N>
static void go_vol_ns(const StageArgs &a, hipStream_t s) {
    if constexpr (N <= 5) hipLaunchKernelGGL((k_volume<T, N, true>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a);
}
template <int T, int N>
static void go_surf_euler(const StageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_surface<T, N, false>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a);
}
template <int T, int N>
static void go_surf_ns(const StageArgs &a, hipStream_t s) {
    if constexpr (N <= 5) hipLaunchKernelGGL((k_surface<T, N, true>), dim3(a.count[T]), dim3(Dm<T, N>::BS), 0, s, a);
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
static void goq_trace(const StageArgs &a, const int32_t *qb, int nq, hipStream_t s) {
    hipLaunchKernelGGL((k_trace_q<N>), dim3(nq), dim3(kBS<N>), 0, s, a, qb);
}
template <int N>
static void goq_vol(const StageArgs &a, bool ns, const int32_t *qb, int nq, hipStream_t s) {
    if constexpr (N <= 5) {
        if (ns) { hipLaunchKernelGGL((k_volume_q<N, true>), dim3(nq), dim3(kBS<N>), 0, s, a, qb); return; }
    }
    if (!ns) hipLaunchKernelGGL((k_volume_q<N, false>), dim3(nq), dim3(kBS<N>), 0, s, a, qb);
}
template <int N>
static void goq_surf(const StageArgs &a, bool ns, const int32_t *qb, int nq, hipStream_t s) {
    if constexpr (N <= 5) {
        if (ns) { hipLaunchKernelGGL((k_surface_q<N, true>), dim3(nq), dim3(kBS<N>), 0, s, a, qb); return; }
    }
    if (!ns) hipLaunchKernelGGL((k_surface_q<N, false>), dim3(nq), dim3(kBS<N>), 0, s, a, qb);
}

hipError_t launch_queues(int N, bool ns, int phase, const StageArgs &a, const int32_t *qb, int nq,
                         hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    if (phase == 0) {
        PDG_DISPATCH_N(goq_trace, a, qb, nq, s);
    } else if (phase == 1) {
        PDG_DISPATCH_N(goq_vol, a, ns, qb, nq, s);
    } else {
        PDG_DISPATCH_N(goq_surf, a, ns, qb, nq, s);
    }
    return hipGetLastError();
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
    const uint64_t Q = (uint64_t)nq;
    for (int i = tid; i < n; i += nt) {
        const uint64_t qi = Q * (2 * S[i] + w[i]) / (2 * W);
        const int64_t qprev = i == 0 ? -1 : (int64_t)(Q * (2 * S[i - 1] + w[i - 1]) / (2 * W));
        for (int64_t q = qprev + 1; q <= (int64_t)qi; ++q) qb[q] = i;
        if (i == n - 1)
            for (int64_t q = (int64_t)qi + 1; q <= nq; ++q) qb[q] = n;
    }
}

hipError_t launch_partition(int n, const uint32_t *w, int nq, int32_t *qb, uint64_t *scratch,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_partition, dim3(1), dim3(1024), 0, s, n, w, nq, qb, scratch);
    return hipGetLastError();
}

}  // namespace pdg
