// Per-element phases of one residual evaluation (trace, volume, surface), shared by the
// per-type, work-queue and batched kernels.  Each function processes one element with the
// whole workgroup and the LDS block passed in.
#pragma once

#include "device.h"

namespace pdg {

// per-queue wall-clock ticks of a work-queue workgroup (constant-rate device clock), added to
// qt[q] by one lane; qt may be null
__device__ __forceinline__ long long queue_clock_begin() { return wall_clock64(); }
__device__ __forceinline__ void queue_clock_end(uint64_t *qt, long long t0) {
    __syncthreads();
    if (qt && threadIdx.x == 0) qt[blockIdx.x] += (uint64_t)(wall_clock64() - t0);
}

// ------------------------------------------------------------------------------- trace phase
// Work-queue kernels: qsub workgroups serve each queue (as several threads serve one rank);
// workgroup s of queue q = blockIdx.x / qsub runs body(e) for every qsub-th type-T element of
// the queue, list[T][qtb[4 q + T] + s + i qsub] below qtb[4 (q + 1) + T] (the type-T elements
// of the queue's segment, in segment order), with a barrier after each element.
template <int T, typename F>
__device__ __forceinline__ void queue_type_loop(const StageArgs &a, const int32_t *qtb, F &&body) {
    const int q = blockIdx.x / a.qsub, s = blockIdx.x - q * a.qsub;
    const int j1 = qtb[4 * (q + 1) + T];
    for (int j = qtb[4 * q + T] + s; j < j1; j += a.qsub) {
        body(a.list[T][j]);
        __syncthreads();
    }
}

template <int T, int N>
struct TraceLDS {
    static constexpr int size = 5 * Dm<T, N>::m;  // the element's stored values
};

template <int T, int N>
__device__ __forceinline__ void trace_elem(const StageArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m;
    double *su = smem;
    const int64_t off = a.mesh.off[e];
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    // energy relative to e_ref: nodal values (hexahedra) or the constant mode's coefficient
    const DevType &tab = a.tab[T];
    const double eshift = T == PDG_HEX ? a.phys.e_ref : tab.c0;
    for (int t = threadIdx.x; t < 5 * m; t += blockDim.x) {
        const double v = a.U[off + t];
        su[t] = (t >= 4 * m && (T == PDG_HEX || t == 4 * m)) ? v - eshift : v;
    }
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
#pragma unroll 1
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
        // one lane per face point: Tq = sum_j E[p][j] u~_j, with E^T read along j (coalesced over
        // the lanes' points).  Five right-hand sides use five of sixteen MFMA columns, so the
        // vector units do this product faster than the matrix cores.
        const int np = (s1 - s0) * n2;
        for (int t = threadIdx.x; t < np; t += blockDim.x) {
            const int ls = t / n2, p = t - ls * n2, sl = s0 + ls;
            const double *Et = a.ops.data + a.ops.op_off[a.mesh.slot_op[sl]] + (int64_t)n2 * m + p;
            double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll 5
            for (int j = 0; j < m; ++j) {
                const double ev = Et[(int64_t)j * n2];
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] += ev * su[v * m + j];
            }
            acc[4] += tab.dlt;
            double *dst = a.Tq + (int64_t)sl * 5 * n2 + p;
#pragma unroll
            for (int v = 0; v < 5; ++v) dst[v * n2] = acc[v];
        }
    }
}

// ------------------------------------------------------------------------------ volume phase
// LDS of one element in the volume phase, laid out by buffer lifetime:
//   q    nodal state, later the weak derivative d                          5 nn
//   dh, dm  1-D weak derivative tables; NS: strong derivative tables (BR1)   3 n^2 each
//   A    NS: volume part of the gradient, later the gradient at the nodes  12 nn
//   B    NS: face terms of all sides, later the gradient at face points     12 S n2
//        (modal: the state coefficients u~ live here before that)
//   C    NS modal: BR1 right-hand side and gradient coefficients     12 m (prisms) / 24 m
//        (the lifting variables, 4 nn, live here before that)
//   G    contravariant fluxes, 15 nn; aliases A, B and C once the gradients are consumed
// workgroup size of the per-type volume kernels: modal elements up to 128 volume nodes get twice
// the waves of one lane per node (the matrix-core contractions are spread over more waves)
template <int T, int N>
constexpr int kVolBS = (T != PDG_HEX && Dm<T, N>::BS <= 128) ? 2 * Dm<T, N>::BS : Dm<T, N>::BS;

// directions whose 1-D rule holds both end points (Gauss-Lobatto): the split form applies there;
// the collapsing directions of prisms, pyramids (third) and tetrahedra (second, third) are on
// left Gauss-Radau nodes
template <int T>
__host__ __device__ constexpr bool sbp_dir(int ax) {
    return T == PDG_HEX ? true : (T == PDG_TET ? ax == 0 : ax < 2);
}
template <int T>
constexpr int kSbpDirs = T == PDG_HEX ? 3 : (T == PDG_TET ? 1 : 2);

template <int T, int N, bool NS, bool SPLIT = false, int S = Dm<T, N>::SLOTS, bool CV = false>
struct VolLDS {
    using D = Dm<T, N>;
    static constexpr bool MODAL = T != PDG_HEX;
    static constexpr int nn = D::nn, m = D::m, n2 = D::n2;
    static constexpr int cmax(int x, int y) { return x > y ? x : y; }
    // Navier-Stokes on modal elements keeps no separate nodal-state block: V u~ lands in A
    // (read once per node before the gradient phase) and the weak derivative in C
    static constexpr bool ALIAS = NS && MODAL;
    static constexpr int q = 0;
    static constexpr int dh = q + (ALIAS ? 0 : 5 * nn);
    static constexpr int dm = dh + 3 * D::n * D::n;           // NS: strong 1-D derivatives (BR1)
    static constexpr int ops = dm + (NS ? 3 * D::n * D::n : 0);
    static constexpr int A = ops + S;
    static constexpr int szA = NS ? 12 * nn : 0;
    static constexpr int B = A + szA;
    static constexpr int szB = NS ? 12 * (MODAL ? S : 1) * n2 : 0;
    static constexpr int C = B + cmax(szB, MODAL ? 5 * m : 0);
    static constexpr int szC =
        NS ? cmax(cmax(MODAL ? 12 * m : 0, 4 * nn), ALIAS ? 5 * nn : 0) : 0;
    static constexpr int u = MODAL ? B : 0;       // u~ (5 m) before B is used
    static constexpr int w = C;                   // lifting variables (4 nn) before C is used
    static constexpr int G = NS ? A : C;          // fluxes after the gradient phase
    static constexpr int qv = ALIAS ? A : q;      // nodal state V u~ (5 nn)
    static constexpr int dd = ALIAS ? C : q;      // weak derivative (5 nn), read by V^T W d
    static constexpr int size_weak = cmax(C + szC, G + 15 * nn);
    // split form: (Q^T - Q)/w per direction (3 n^2), the nodes' two-point quantities (6 nn) and,
    // on modal elements, the contravariant vectors of the split directions (3 per direction, nn)
    // Navier-Stokes on modal elements: these blocks are filled once the gradient buffers are
    // dead and sit past the flux block, in face-gradient and coefficient space that the weak
    // derivative no longer uses (four workgroups per CU fit in LDS)
    static constexpr bool SALIAS = SPLIT && NS && MODAL;
    static constexpr int ds = SALIAS ? G + 15 * nn : size_weak;
    static constexpr int P = ds + 3 * D::n * D::n;
    static constexpr int AC = P + 6 * nn;
    // (curved hexahedra keep their per-node contravariant vectors there too)
    static constexpr int size = SPLIT ? cmax(size_weak, AC + ((MODAL || CV) ? 3 * kSbpDirs<T> * nn : 0)) : size_weak;
    // the two-point fluxes of one direction's node pairs, 5 n^2 n(n-1)/2 <= 15 nn for n <= 7,
    // reuse the flux block G once the weak derivative has read it
    static_assert(!SPLIT || 5 * D::n * D::n * (D::n * (D::n - 1) / 2) <= 15 * nn, "pair-flux block");
};

// CV: the mesh has curved elements (per-node metrics, per-element mass matrices); compiled apart so
// that the affine kernels carry none of it
template <int T, int N, bool NS, int BS = Dm<T, N>::BS, bool SPLIT = false, int S = Dm<T, N>::SLOTS,
          bool CV = false>
__device__ __forceinline__ void volume_elem(const StageArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    using L = VolLDS<T, N, NS, SPLIT, S, CV>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m;
    constexpr bool MODAL = T != PDG_HEX;
    double *sq = smem + L::qv;
    double *sdd = smem + L::dd;
    double *sG = smem + L::G;
    double *sdh = smem + L::dh;
    double *sdm = smem + L::dm;
    double *su = smem + L::u;
    double *sgn = smem + L::A;
    double *sgt = smem + L::C;       // modal BR1 gradient coefficients (12 m)
    double *sbuf = smem + L::B;      // face terms / gradient at the face points
    double *sw = smem + L::w;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + L::ops);

    const int tid = threadIdx.x;
    const int64_t off = a.mesh.off[e];
    const DevType &tab = a.tab[T];
    const double *geo = a.mesh.geo + 10 * (int64_t)e;
    const double Jaff = geo[0];
    double iJ = 1.0 / Jaff;
    double cofT[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) cofT[i] = geo[1 + i];
    // curved (trilinear) elements: this lane's node has its own contravariant rows (composed
    // with the collapse on the modal types, whose reference metric is then not applied) and its
    // own Jacobian; on hexahedra every use below (contravariant fluxes, BR1 gradients, 1/J) is then
    // per node, on the modal types M_e^-1 replaces M_D^-1 / J
    constexpr bool cv = CV;
    if (cv && tid < nn) {
        const double *mt = a.mesh.nmet + ((int64_t)e * nn + tid) * 10;
        iJ = 1.0 / mt[0];
#pragma unroll
        for (int i = 0; i < 9; ++i) cofT[i] = mt[1 + i];
    }
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0;

    for (int t = tid; t < 3 * n * n; t += BS) sdh[t] = tab.dhat[t / (n * n)][t % (n * n)];
    if constexpr (NS)
        for (int t = tid; t < 3 * n * n; t += BS) sdm[t] = tab.dmat[t / (n * n)][t % (n * n)];
    for (int t = tid; t < nsl; t += BS) sops[t] = (MODAL ? a.ops.op_poff : a.ops.op_off)[a.mesh.slot_op[s0 + t]];
    constexpr int KBm = (m + 15) / 16, KBnn = (nn + 15) / 16;
    if constexpr (MODAL) {
        // the energy's constant-mode coefficient less c0: V u~ then gives rho E - e_ref - dlt
        for (int t = tid; t < 5 * m; t += BS) su[t] = t == 4 * m ? a.U[off + t] - tab.c0 : a.U[off + t];
        __syncthreads();
        // nodal state q = V u~, energy relative to e_ref
        mfma_gemm_pk(nn, KBm, 5, [&](int i, int kb) { return tab.Vp + ((int64_t)i * KBm + kb) * 16; },
                     [&](int k, int c) { return su[c * m + kclamp(k, m)]; },
                     [&](int i, int c, double v) { sq[c * nn + i] = c == 4 ? v + tab.dlt : v; },
                     [&](int kb) { return ksteps_of(m, kb); });
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
            q[4] -= a.phys.e_ref;  // energy relative to e_ref (exact near the mean state)
        }
    }

    // the split form's (Q^T - Q)/w tables, per-node two-point quantities and contravariant vectors
    auto split_node_data = [&]() {
        for (int t = tid; t < 3 * n * n; t += BS) smem[L::ds + t] = tab.dskew[t / (n * n)][t % (n * n)];
        if (act) {
            double P[6];
            ec_prim(q, a.phys, P);
#pragma unroll
            for (int j = 0; j < 6; ++j) smem[L::P + j * nn + k] = P[j];
            if constexpr (MODAL || CV) {
                // this node's contravariant vectors of the split directions (curved elements:
                // the node's own rows, which hold the collapse)
                const double *c = tab.cmet + k * 9;
                int sd = 0;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    if (!sbp_dir<T>(ax)) continue;
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        smem[L::AC + (sd * 3 + cc) * nn + k] =
                            CV ? cofT[ax * 3 + cc]
                               : c[ax * 3 + 0] * cofT[cc] + c[ax * 3 + 1] * cofT[3 + cc] + c[ax * 3 + 2] * cofT[6 + cc];
                    ++sd;
                }
            }
        }
    };
    if constexpr (SPLIT && !L::SALIAS) split_node_data();

    double g[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) g[f] = 0.0;

    if constexpr (NS) {
        br1_gradients<T, N, BS, true, CV>(a, e, s0, s1, cofT, iJ, q, sops, sdm, sw, sgn, sbuf, sgt, g);
        // viscous normal flux Fv(q, g).n_out at this element's face points
        const int np = nsl * n2;
        for (int t = tid; t < np; t += BS) {
            const int sl = s0 + t / n2, p = t % n2;
            const int op = a.mesh.slot_op[sl];
            const double *sg = slot_geom<CV>(a.mesh, sl, p);
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
#pragma unroll 1
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
        if constexpr (L::SALIAS) split_node_data();
    }

    // directions with a weak volume term: all, or with the split form those on Gauss-Radau lines
    // and, for Navier-Stokes, every direction (the viscous flux keeps the weak term)
    constexpr bool WEAK0 = !SPLIT || NS || !sbp_dir<T>(0);
    constexpr bool WEAK1 = !SPLIT || NS || !sbp_dir<T>(1);
    constexpr bool WEAK2 = !SPLIT || NS || !sbp_dir<T>(2);
    constexpr bool ANYWEAK = WEAK0 || WEAK1 || WEAK2;
    // pointwise flux and contravariant transform
    if (act && ANYWEAK) {
        double F[3][5];
        euler_flux(q, a.phys, F);
        if constexpr (CV) {
            if (a.mesh.nmov) {
                // moving mesh: the flux relative to the grid, F - q xdot (energy absolute)
                const double *mv = a.mesh.nmov + ((int64_t)e * nn + k) * 4;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) F[c][v] -= (v == 4 ? q[4] + a.phys.e_ref : q[v]) * mv[1 + c];
            }
        }
        double Fv[3][5];
        if constexpr (NS) {
            // this node's gradients, read back from LDS (not kept in registers across the face loop)
            double gk[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) gk[f] = sgn[f * nn + k];
            visc_flux(q, gk, a.phys, Fv);
            if constexpr (!SPLIT) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) F[c][v] -= Fv[c][v];
            }
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double Fh[3], Fhv[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int b = 0; b < 3; ++b)
                Fh[b] = cofT[b * 3 + 0] * F[0][v] + cofT[b * 3 + 1] * F[1][v] + cofT[b * 3 + 2] * F[2][v];
            if constexpr (SPLIT && NS) {
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    Fhv[b] = cofT[b * 3 + 0] * Fv[0][v] + cofT[b * 3 + 1] * Fv[1][v] + cofT[b * 3 + 2] * Fv[2][v];
            }
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (SPLIT && !NS && sbp_dir<T>(ax)) continue;
                // split directions carry only the viscous part here
                double Fx[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) Fx[b] = (SPLIT && sbp_dir<T>(ax)) ? -Fhv[b] : Fh[b] - Fhv[b];
                if (MODAL && !cv) {
                    const double *c = tab.cmet + k * 9;
                    sG[(ax * 5 + v) * nn + k] = c[ax * 3 + 0] * Fx[0] + c[ax * 3 + 1] * Fx[1] + c[ax * 3 + 2] * Fx[2];
                } else {
                    sG[(ax * 5 + v) * nn + k] = Fx[ax];
                }
            }
        }
    }
    __syncthreads();
    // sum-factorised weak derivative d_k = sum_a sum_l Dhat_a[i_a][l] G^a(.. l ..)
    double d[5] = {0, 0, 0, 0, 0};
    if (act) {
        for (int ax = 0; ax < 3; ++ax) {
            if (!(ax == 0 ? WEAK0 : ax == 1 ? WEAK1 : WEAK2)) continue;
            const int base = k - ii[ax] * stride[ax];
            for (int l = 0; l < n; ++l) {
                const double dh = sdh[ax * n * n + ii[ax] * n + l];
                const int mm = base + l * stride[ax];
#pragma unroll
                for (int v = 0; v < 5; ++v) d[v] += dh * sG[(ax * 5 + v) * nn + mm];
            }
        }
    }
    if constexpr (SPLIT) {
        // flux differencing along the Gauss-Lobatto lines, one direction at a time:
        //   d_k += sum_l (Q^T - Q)[i][l]/w_i F#(q_k, q_m) . (a_k + a_m)/2.
        // The two-point flux is symmetric, so each unordered pair (i < j) of a line is evaluated
        // once by any lane (all lanes of the workgroup share the pairs) into sF[v][line][pair];
        // each node then gathers its n - 1 partners in ascending order.
        constexpr int NP = n * (n - 1) / 2;
        double *sF = sG;
        __syncthreads();  // the weak derivative has read G
        int sd = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (!sbp_dir<T>(ax)) continue;
            for (int t = tid; t < n * n * NP; t += BS) {
                const int line = t / NP, pp = t - line * NP;
                int i = 0, rem = pp;
                while (rem >= n - 1 - i) {
                    rem -= n - 1 - i;
                    ++i;
                }
                const int j = i + 1 + rem;
                const int base = ax == 0 ? n * line : ax == 1 ? (line % n) + n * n * (line / n) : line;
                const int ki = base + i * stride[ax], kj = base + j * stride[ax];
                double Pi[6], Pj[6], nv[3], f[5];
#pragma unroll
                for (int q6 = 0; q6 < 6; ++q6) {
                    Pi[q6] = smem[L::P + q6 * nn + ki];
                    Pj[q6] = smem[L::P + q6 * nn + kj];
                }
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    nv[cc] = (MODAL || CV) ? 0.5 * (smem[L::AC + (sd * 3 + cc) * nn + ki] + smem[L::AC + (sd * 3 + cc) * nn + kj])
                                   : cofT[ax * 3 + cc];
                ec_flux_prim(Pi, Pj, nv, a.phys.gamma, a.phys.p_ref, f);
#pragma unroll
                for (int v = 0; v < 5; ++v) sF[(v * n * n + line) * NP + pp] = f[v];
            }
            __syncthreads();
            if (act) {
                const int i = ii[ax];
                const int line = ax == 0 ? ii[1] + n * ii[2] : ax == 1 ? ii[0] + n * ii[2] : ii[0] + n * ii[1];
                const double *srow = smem + L::ds + ax * n * n + i * n;
                for (int l = 0; l < n; ++l) {
                    if (l == i) continue;
                    const int lo = i < l ? i : l, hi = i < l ? l : i;
                    const int pp = lo * (2 * n - lo - 1) / 2 + (hi - lo - 1);
                    const double sc = srow[l];
#pragma unroll
                    for (int v = 0; v < 5; ++v) d[v] += sc * sF[(v * n * n + line) * NP + pp];
                }
            }
            __syncthreads();
            ++sd;
        }
    }
    if constexpr (CV) {
        if (act && a.mesh.nmov) {
            // moving mesh: M du~/dt = r - V^T W (dJ/dt q), the source per unit weight at this node
            const double jd = a.mesh.nmov[((int64_t)e * nn + k) * 4];
#pragma unroll
            for (int v = 0; v < 5; ++v) d[v] -= jd * (v == 4 ? q[4] + a.phys.e_ref : q[v]);
        }
    }
    if (act) {
        if constexpr (MODAL) {
#pragma unroll
            for (int v = 0; v < 5; ++v) sdd[v * nn + k] = d[v];
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) a.Rp[off + v * nn + k] = d[v] * iJ;
        }
    }
    if constexpr (MODAL) {
        __syncthreads();
        // volume part of dU~/dt, M_D^-1 V^T W d / J (the face part adds M_D^-1 E^T of its own)
        double *Rp = a.Rp + off;
        // curved elements: V^T W d, with M_e^-1 applied once to the whole residual in the
        // surface phase
        const double *volA = cv ? tab.VtWp : tab.MVtWp;
        mfma_gemm_pk(m, KBnn, 5, [&](int i, int kb) { return volA + ((int64_t)i * KBnn + kb) * 16; },
                     [&](int kk, int c) { return sdd[c * nn + kclamp(kk, nn)]; },
                     [&](int i, int c, double v) { Rp[c * m + i] = cv ? v : v * iJ; },
                     [&](int kb) { return ksteps_of(nn, kb); });
    }
}

// ----------------------------------------------------------------------------- surface phase
template <int T, int N, int S = Dm<T, N>::SLOTS>
struct SurfLDS {
    using D = Dm<T, N>;
    static constexpr bool MODAL = T != PDG_HEX;
    // modal lift on the vector units: one row of M_D^-1 E^T per lane, the face sides shared
    // out over G groups of RW lanes whose partial sums meet in LDS
    static constexpr int RW = ((D::m + 63) / 64) * 64;
    static constexpr int G = MODAL ? D::BS / RW : 1;
    static constexpr int ops = S * 5 * D::n2;
    // modal: the element's partial residual, K and U, loaded at the start (15 m)
    static constexpr int pre = ops + S;
    static constexpr int red = pre + (MODAL ? 15 * D::m : 0);
    static constexpr int size = red + (G - 1) * 5 * D::m;
};

// EC: the entropy-conservative two-point flux at the face points instead of Lax-Friedrichs
template <int T, int N, bool NS, bool EC = false, int S = Dm<T, N>::SLOTS, bool CV = false>
__device__ __forceinline__ void surface_elem(const StageArgs &a, int e, double *sgs) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m, BS = D::BS;
    constexpr bool MODAL = T != PDG_HEX;
    const int tid = threadIdx.x;
    const int64_t off = a.mesh.off[e];
    const int s0 = a.mesh.slot_begin[e], s1 = a.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0;
    const double Jaff = a.mesh.geo[10 * (int64_t)e];
    int64_t *sops = reinterpret_cast<int64_t *>(sgs + SurfLDS<T, N, S>::ops);
    double *spre = sgs + SurfLDS<T, N, S>::pre;
    for (int t = tid; t < nsl; t += BS) sops[t] = (MODAL ? a.ops.op_poff : a.ops.op_off)[a.mesh.slot_op[s0 + t]];
    if constexpr (MODAL) {
        // issued first so that their latency overlaps the face loop
        for (int t = tid; t < 5 * m; t += BS) {
            spre[t] = a.Rp[off + t];
            if (a.mode != 0) {
                spre[5 * m + t] = a.K[off + t];
                spre[10 * m + t] = a.Uw[off + t];
            }
        }
    }
    for (int t = tid; t < nsl * n2; t += BS) {
        const int ls = t / n2, p = t % n2, sl = s0 + ls;
        const int nb = a.mesh.slot_nbr[sl];
        const double *sg = slot_geom<CV>(a.mesh, sl, p);
        double qa[5], qb[5], f[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qa[v] = a.Tq[((int64_t)sl * 5 + v) * n2 + p];
            qb[v] = a.Tq[((int64_t)nb * 5 + v) * n2 + p];
        }
        const double nv[3] = {sg[0], sg[1], sg[2]};
        if constexpr (EC) {
            ec_flux(qa, qb, nv, a.phys, f);
        } else if constexpr (CV) {
            if (a.mesh.gvn)
                lf_flux_moving(qa, qb, nv, a.mesh.gvn[(int64_t)sl * a.mesh.geo_pts + p], a.phys, f);
            else
                lf_flux(qa, qb, nv, a.phys, f);
        } else {
            lf_flux(qa, qb, nv, a.phys, f);
        }
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
        // dU~/dt = (M_D^-1 V^T W d)/J - (M_D^-1 E^T)(face terms)/J over all sides on the vector
        // units (five right-hand sides would fill five of the sixteen matrix-core columns):
        // lane i of group g sums row i of M_D^-1 E^T, read as the columns of E M_D^-1 [n2][m]
        // stored after the packed tables, over sides g, g + G, ...; the groups' partial sums
        // are added in group order, and the RK update is applied in the store
        using SL = SurfLDS<T, N, S>;
        constexpr int G = SL::G, RW = SL::RW;
        constexpr int KBm = (m + 15) / 16, KBn2 = (n2 + 15) / 16;
        constexpr int64_t em = 2 * (int64_t)n2 * KBm * 16 + 2 * (int64_t)m * KBn2 * 16;
        const int g = tid / RW, i = tid - g * RW;
        const bool lact = g < G && i < m;
        // curved elements: the plain E (E^T f), with M_e^-1 applied to the whole residual below
        constexpr bool cv = CV;
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (lact) {
            for (int ls = g; ls < nsl; ls += G) {
                const double *EMs = cv ? a.ops.data + a.ops.op_off[a.mesh.slot_op[s0 + ls]] + i
                                       : a.ops.data + sops[ls] + em + i;
                const double *fs = sgs + ls * 5 * n2;
#pragma unroll 5
                for (int p = 0; p < n2; ++p) {
                    const double c = EMs[(int64_t)p * m];
#pragma unroll
                    for (int v = 0; v < 5; ++v) acc[v] += c * fs[v * n2 + p];
                }
            }
        }
        if constexpr (G > 1) {
            double *sred = sgs + SL::red;
            if (lact && g > 0) {
#pragma unroll
                for (int v = 0; v < 5; ++v) sred[((g - 1) * 5 + v) * m + i] = acc[v];
            }
            __syncthreads();
            if (lact && g == 0) {
                for (int gg = 1; gg < G; ++gg) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) acc[v] += sred[((gg - 1) * 5 + v) * m + i];
                }
            }
        }
        if constexpr (cv) {
            // dU~/dt = M_e^-1 (V^T W d - E^T (ws f*)): the difference in place, then one product
            // with the element's mass-matrix inverse (symmetric: lane i reads its column)
            if (lact && g == 0) {
#pragma unroll
                for (int v = 0; v < 5; ++v) spre[v * m + i] -= acc[v];
            }
            __syncthreads();
            if (lact && g == 0) {
                const double *Mi = a.mesh.minv + a.mesh.minv_off[e];
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] = 0.0;
#pragma unroll 8
                for (int j = 0; j < m; ++j) {
                    const double c = Mi[(int64_t)j * m + i];
#pragma unroll
                    for (int v = 0; v < 5; ++v) acc[v] += c * spre[v * m + j];
                }
            }
        }
        if (lact && g == 0) {
            const int mode = a.mode;
            const double rk_a = a.rk_a, rk_bdt = a.rk_bdt;
            double *out = a.out + off, *Kr = a.K + off, *Uw = a.Uw + off;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const int idx = v * m + i;
                const double R = cv ? acc[v] : spre[idx] - acc[v] * iJ;
                if (mode == 0) {
                    out[idx] = R;
                } else {
                    const double Kn = (rk_a == 0.0) ? R : rk_a * spre[5 * m + idx] + R;
                    Kr[idx] = Kn;
                    Uw[idx] = spre[10 * m + idx] + rk_bdt * Kn;
                }
            }
        }
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
#pragma unroll 5
                    for (int p = 0; p < n2; ++p) {
                        const double c = I[(int64_t)p * n2 + a2];
#pragma unroll
                        for (int v = 0; v < 5; ++v) lift[v] += c * gs[v * n2 + p];
                    }
                }
            }
            // lumped mass w_k J (per node on curved hexahedra)
            const double sc = (CV ? 1.0 / a.mesh.nmet[((int64_t)e * nn + k) * 10] : iJ) / a.tab[T].w[k];
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

}  // namespace pdg
