// Device-side helpers shared by the residual and adjoint kernels (gfx950, FP64): element
// dimensions, face-plane indexing, the pointwise fluxes and the FP64 matrix-core contraction.
#pragma once

#include <cstdint>

#include "kernels.h"

namespace pdg {

// workgroup size: one lane per volume node, rounded up to whole 64-lane wavefronts
template <int N>
constexpr int kBS = (((N + 1) * (N + 1) * (N + 1) + 63) / 64) * 64;
// workgroup size of the trace work-queue kernel (the per-type trace kernels use the same)
constexpr int kTraceQBS = 128;

template <int T, int N>
struct Dm {
    static constexpr int n = N + 1, n2 = n * n, nn = n * n * n;
    static constexpr int m = T == PDG_HEX     ? nn
                             : T == PDG_PRISM ? n * n * (n + 1) / 2
                             : T == PDG_PYR   ? n * (n + 1) * (2 * n + 1) / 6
                                              : n * (n + 1) * (n + 2) / 6;
    static constexpr int BS = ((nn + 63) / 64) * 64;
    static constexpr int SLOTS = T == PDG_HEX ? 24 : T == PDG_PRISM ? 13 : T == PDG_PYR ? 8 : 6;
};

// Face sides whose data the per-type kernels hold in LDS at once.  Prisms with at most eight
// face sides run in kernels sized for eight, at four elements per CU in the Navier-Stokes volume
// phase; the few prisms with more (several mortar faces, each half in two chunks) run in kernels
// sized for Dm::SLOTS.  For the other types the larger capacity costs no occupancy (measured),
// so all their elements share one launch.
template <int T>
constexpr int kSlotsNarrow = T == PDG_PRISM ? 8 : Dm<T, 2>::SLOTS;
template <int T, int N, bool WIDE>
constexpr int kSlotCap = WIDE ? Dm<T, N>::SLOTS : kSlotsNarrow<T>;

// volume node index of plane node a2 = i_b + n*i_c on face plane (axis, side)
__device__ __forceinline__ int plane_vol(int plane, int a2, int n) {
    const int axis = plane >> 1, fi = (plane & 1) ? n - 1 : 0;
    const int ib = a2 % n, ic = a2 / n;
    if (axis == 0) return fi + n * (ib + n * ic);
    if (axis == 1) return ib + n * (fi + n * ic);
    return ib + n * (ic + n * fi);
}

// plane node index of volume node k on plane (axis, side), or -1
__device__ __forceinline__ int vol_plane(int plane, int k, int n) {
    const int i0 = k % n, i1 = (k / n) % n, i2 = k / (n * n);
    const int axis = plane >> 1, fi = (plane & 1) ? n - 1 : 0;
    if (axis == 0) return i0 == fi ? i1 + n * i2 : -1;
    if (axis == 1) return i1 == fi ? i0 + n * i2 : -1;
    return i2 == fi ? i0 + n * i1 : -1;
}

// Pointwise functions of the residual kernels take states with the energy relative to e_ref
// (Physics): q[4] = rho E - e_ref.  pm = p - p_ref then has no rounding of the mean pressure.
__device__ __forceinline__ double pressure_rel(const double q[5], double gamma) {
    return (gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// inviscid flux with the reference pressure taken out of the momentum part: (p - p_ref) I;
// energy flux (rho E + p) u = (q[4] + pm + h_ref) u
__device__ __forceinline__ void euler_flux(const double q[5], const Physics &ph, double F[3][5]) {
    const double ir = 1.0 / q[0];
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double pm = (ph.gamma - 1.0) * (q[4] - 0.5 * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
    const double H = q[4] + pm + ph.h_ref;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        F[c][0] = q[1 + c];
        F[c][1] = q[1] * u[c];
        F[c][2] = q[2] * u[c];
        F[c][3] = q[3] * u[c];
        F[c][1 + c] += pm;
        F[c][4] = H * u[c];
    }
}

// local Lax-Friedrichs flux seen from side a with outward normal nv
__device__ __forceinline__ void lf_flux(const double qa[5], const double qb[5], const double nv[3],
                                        const Physics &ph, double f[5]) {
    const double gamma = ph.gamma;
    double Fa[3][5], Fb[3][5];
    euler_flux(qa, ph, Fa);
    euler_flux(qb, ph, Fb);
    const double ira = 1.0 / qa[0], irb = 1.0 / qb[0];
    const double una = (qa[1] * nv[0] + qa[2] * nv[1] + qa[3] * nv[2]) * ira;
    const double unb = (qb[1] * nv[0] + qb[2] * nv[1] + qb[3] * nv[2]) * irb;
    const double pa = pressure_rel(qa, gamma) + ph.p_ref;
    const double pb = pressure_rel(qb, gamma) + ph.p_ref;
    const double lam = fmax(fabs(una) + sqrt(gamma * pa * ira), fabs(unb) + sqrt(gamma * pb * irb));
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double fa = Fa[0][v] * nv[0] + Fa[1][v] * nv[1] + Fa[2][v] * nv[2];
        const double fb = Fb[0][v] * nv[0] + Fb[1][v] * nv[1] + Fb[2][v] * nv[2];
        f[v] = 0.5 * (fa + fb) - 0.5 * lam * (qb[v] - qa[v]);
    }
}

// local Lax-Friedrichs flux through a face moving with normal speed vn = xdot . nv: the flux
// relative to the moving face, (F(qa) + F(qb)).nv / 2 - vn (qa + qb) / 2 - lam (qb - qa) / 2 with
// lam = max(|u.nv - vn| + c) (the grid term takes the energy absolute; bitwise antisymmetric
// under nv, vn -> -nv, -vn like lf_flux)
__device__ __forceinline__ void lf_flux_moving(const double qa[5], const double qb[5], const double nv[3],
                                               double vn, const Physics &ph, double f[5]) {
    const double gamma = ph.gamma;
    double Fa[3][5], Fb[3][5];
    euler_flux(qa, ph, Fa);
    euler_flux(qb, ph, Fb);
    const double ira = 1.0 / qa[0], irb = 1.0 / qb[0];
    const double una = (qa[1] * nv[0] + qa[2] * nv[1] + qa[3] * nv[2]) * ira;
    const double unb = (qb[1] * nv[0] + qb[2] * nv[1] + qb[3] * nv[2]) * irb;
    const double pa = pressure_rel(qa, gamma) + ph.p_ref;
    const double pb = pressure_rel(qb, gamma) + ph.p_ref;
    const double lam = fmax(fabs(una - vn) + sqrt(gamma * pa * ira), fabs(unb - vn) + sqrt(gamma * pb * irb));
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double fa = Fa[0][v] * nv[0] + Fa[1][v] * nv[1] + Fa[2][v] * nv[2];
        const double fb = Fb[0][v] * nv[0] + Fb[1][v] * nv[1] + Fb[2][v] * nv[2];
        const double qs = v == 4 ? (qa[4] + ph.e_ref) + (qb[4] + ph.e_ref) : qa[v] + qb[v];
        f[v] = 0.5 * (fa + fb) - 0.5 * vn * qs - 0.5 * lam * (qb[v] - qa[v]);
    }
}

// Two-point quantities of a state (energy relative to e_ref) for the entropy-conservative flux:
// rho, u, v, w, beta = rho / (2 p), p - p_ref (formed without the mean pressure's rounding)
__device__ __forceinline__ void ec_prim(const double q[5], const Physics &ph, double P[6]) {
    const double ir = 1.0 / q[0];
    P[0] = q[0];
    P[1] = q[1] * ir;
    P[2] = q[2] * ir;
    P[3] = q[3] * ir;
    P[5] = (ph.gamma - 1.0) * (q[4] - 0.5 * (q[1] * P[1] + q[2] * P[2] + q[3] * P[3]));
    P[4] = 0.5 * q[0] / (P[5] + ph.p_ref);
}

// Chandrashekar's entropy-conservative, kinetic-energy-preserving two-point flux in direction
// nv (any length), from ec_prim quantities; the reference pressure is taken out of the momentum
// part as in euler_flux: with p_hat = mean(rho) / (2 mean(beta)) and rho = 2 beta p,
// p_hat - p_ref = (beta_a (p_a - p_ref) + beta_b (p_b - p_ref)) / (beta_a + beta_b), a weighted
// mean without cancellation.  Logarithmic means: with s = a + b, f = (a - b)/s, u = f^2,
//   L(a, b) = s / (2 F),  F = atanh(f)/f = 1 + u/3 + u^2/5 + u^3/7 + O(u^4),
//   1/F = 1 - u/3 - 4u^2/45 - 44u^3/945 + O(u^4)
// (truncation below 1e-17 relative for u < 1e-4), else L = (a - b)/log(a/b).
__device__ __forceinline__ void ec_flux_prim(const double A[6], const double B[6], const double nv[3],
                                             double gamma, double p_ref, double f[5]) {
    const double sr = A[0] + B[0], dr = A[0] - B[0];
    const double isr = 1.0 / sr;
    const double ur = (dr * isr) * (dr * isr);
    const double rho_ln = ur < 1e-4 ? 0.5 * sr * (1.0 - ur * (1.0 / 3.0 + ur * (4.0 / 45.0 + ur * (44.0 / 945.0))))
                                    : dr / log(A[0] / B[0]);
    const double sb = A[4] + B[4], db = A[4] - B[4];
    const double isb = 1.0 / sb;
    const double ub = (db * isb) * (db * isb);
    const double ibeta_ln = ub < 1e-4 ? 2.0 * isb * (1.0 + ub * (1.0 / 3.0 + ub * (0.2 + ub * (1.0 / 7.0))))
                                      : log(A[4] / B[4]) / db;
    const double pm_hat = (A[4] * A[5] + B[4] * B[5]) * isb;  // p_hat - p_ref
    const double u[3] = {0.5 * (A[1] + B[1]), 0.5 * (A[2] + B[2]), 0.5 * (A[3] + B[3])};
    const double un = u[0] * nv[0] + u[1] * nv[1] + u[2] * nv[2];
    const double fr = rho_ln * un;
    f[0] = fr;
    f[1] = fr * u[0] + pm_hat * nv[0];
    f[2] = fr * u[1] + pm_hat * nv[1];
    f[3] = fr * u[2] + pm_hat * nv[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double ka = A[1] * A[1] + A[2] * A[2] + A[3] * A[3], kb = B[1] * B[1] + B[2] * B[2] + B[3] * B[3];
    f[4] = fr * (0.5 * ibeta_ln / (gamma - 1.0) - 0.25 * (ka + kb) + uu) + (pm_hat + p_ref) * un;
}

__device__ __forceinline__ void ec_flux(const double qa[5], const double qb[5], const double nv[3],
                                        const Physics &ph, double f[5]) {
    double A[6], B[6];
    ec_prim(qa, ph, A);
    ec_prim(qb, ph, B);
    ec_flux_prim(A, B, nv, ph.gamma, ph.p_ref, f);
}

// BR1 lifting variables (u, v, w, T); REL: the state's energy is relative to e_ref (the
// residual kernels), else absolute (the adjoint kernels)
template <bool REL = true>
__device__ __forceinline__ void lifting_vars(const double q[5], const Physics &ph, double w[4]) {
    const double ir = 1.0 / q[0];
    w[0] = q[1] * ir;
    w[1] = q[2] * ir;
    w[2] = q[3] * ir;
    const double p = (ph.gamma - 1.0) * (q[4] - 0.5 * (q[1] * w[0] + q[2] * w[1] + q[3] * w[2])) + (REL ? ph.p_ref : 0.0);
    w[3] = p * ir / ph.R;
}

// viscous flux Fv[c][v] from the state and g[s*3+c] = d(u,v,w,T)_s / dx_c
__device__ __forceinline__ void visc_flux(const double q[5], const double g[12], const Physics &ph,
                                          double Fv[3][5]) {
    const double ir = 1.0 / q[0];
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double div = g[0] + g[4] + g[8];
    const double kappa = ph.mu * ph.gamma * ph.R / ((ph.gamma - 1.0) * ph.Pr);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Fv[c][0] = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double tau = ph.mu * (g[i * 3 + c] + g[c * 3 + i]);
            if (i == c) tau -= ph.mu * (2.0 / 3.0) * div;
            Fv[c][1 + i] = tau;
        }
        Fv[c][4] = u[0] * Fv[c][1] + u[1] * Fv[c][2] + u[2] * Fv[c][3] + kappa * g[9 + c];
    }
}

// ------------------------------------------------------------------ FP64 matrix-core contraction
// C(M x NC) = A(M x K) B(K x NC) with V_MFMA_F64_16X16X4_F64 tiles, shared by the waves of the
// workgroup.  Operand lane layout (wave64): lane l holds A[l%16][l/16] and B[l/16][l%16]; the
// accumulator holds C[i][j] at lane 16*(i%4) + j, register i/4.  The store functor is called
// once per in-range output.  Every wave runs the same trip counts (full EXEC for MFMA).
typedef double v4d __attribute__((ext_vector_type(4)));

// k-steps of block kb of a K-column table
__device__ __forceinline__ int ksteps_of(int K, int kb) {
    const int r = K - 16 * kb;
    return r >= 16 ? 4 : (r + 3) >> 2;
}
// a B-operand index k < 16 KB clamped into the K valid ones (its product with A's zero padding
// is zero)
__device__ __forceinline__ int kclamp(int k, int K) { return k < K ? k : K - 1; }

// A is in the row-block layout (pack_rows): AP(i, kb) points at the 16
// values of row i, k-block kb, and the lane of k-offset l loads its four k-steps
// (k = 16 kb + 4 u + l, u = 0..3) as one 32-byte block.  No operand is masked: rows past M
// load row M - 1 and columns past NC column NC - 1, which only reach accumulator entries that
// are never stored; the k padding of A (k >= K) is zero in the packed tables, so B(k, c), called
// for every k < 16 KB, need only return a finite value there (read at a clamped k, kclamp).
// NKS(kb) (1..4) is the number of k-steps of block kb that hold any column, so k-steps that are
// padding only are not issued.  The loads of the next k-block overlap the MFMAs of the current one.
template <class AP, class BF, class CF, class KF>
__device__ __forceinline__ void mfma_gemm_pk(int M, int KB, int NC, AP A, BF B, CF C, KF NKS) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int MT = (M + 15) >> 4, NT = (NC + 15) >> 4;
    for (int t = wave; t < MT * NT; t += nw) {
        const int rt = t / NT, ct = t - rt * NT;
        const int i = rt * 16 + li, c = ct * 16 + li;
        const bool iok = i < M, cok = c < NC;
        const int ic = iok ? i : M - 1, cc = cok ? c : NC - 1;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        double av[4], bv[4], an[4], bn[4];
        auto load = [&](int kb, double *a_, double *b_) {
            const double2 *p = reinterpret_cast<const double2 *>(A(ic, kb) + 4 * lk);
            const double2 x0 = p[0], x1 = p[1];
            a_[0] = x0.x;
            a_[1] = x0.y;
            a_[2] = x1.x;
            a_[3] = x1.y;
#pragma unroll
            for (int u = 0; u < 4; ++u) b_[u] = B(16 * kb + 4 * u + lk, cc);
        };
        load(0, av, bv);
        for (int kb = 0; kb < KB; ++kb) {
            if (kb + 1 < KB) load(kb + 1, an, bn);
            const int nks = NKS(kb);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u < nks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = an[u];
                bv[u] = bn[u];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + 4 * r + lk;
            if (row < M && cok) C(row, c, acc[r]);
        }
    }
}

// BR1 lifted gradients of the lifting variables (u, v, w, T) of the element in this workgroup,
// strong form: g = grad(w_h) + M^-1 (face terms ws (w* - w_own) n), with w_h the interpolant of
// w at the volume nodes (its derivative along each node line from the 1-D D in sdm), w* =
// (w_own + w_nbr)/2 from the state traces; nodal with the lumped mass on hexahedra, modal with
// M_D on the other types (the weak form is not exact for degree-N fields on the Gauss-Radau
// lines and next to mortar faces).  On return g holds this lane's nodal gradient g[s*3+c] =
// dw_s/dx_c, sgn[f*nn + k] the nodal gradients, and for modal types sbuf[f*np + i] the
// gradients at the element's face points (np = nsl*n2).  LDS: sw 4 nn, sgn 12 nn, sbuf 12 *
// (modal: nsl, hex: 1) * n2, sgt 12 m (modal).  sops holds, per face side of a modal element,
// the offset of its packed trace operator (op_poff).  Ends synchronised.
template <int T, int N, int BS = Dm<T, N>::BS, bool REL = true, bool CV = false>
__device__ __forceinline__ void br1_gradients(const StageArgs &a, int e, int s0, int s1, const double cofT[9],
                                              double iJ, const double q[5], const int64_t *sops,
                                              const double *sdm, double *sw, double *sgn, double *sbuf,
                                              double *sgt, double g[12]) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m;
    constexpr bool MODAL = T != PDG_HEX;
    const DevType &tab = a.tab[T];
    const int tid = threadIdx.x;
    const int nsl = s1 - s0;
    const int k = tid;
    const bool act = k < nn;
    const int ii[3] = {k % n, (k / n) % n, k / (n * n)};
    const int stride[3] = {1, n, n * n};
    if (act) {
        double wv[4];
        lifting_vars<REL>(q, a.phys, wv);
#pragma unroll
        for (int s = 0; s < 4; ++s) sw[s * nn + k] = wv[s];
    }
    __syncthreads();
    // volume part: J grad(w_h) at this node, reference derivatives along the node lines, the
    // node's contravariant vectors (modal) and the element's cofactor transform
    double volc[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) volc[f] = 0.0;
    if (act) {
        double vr[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) vr[f] = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int base = k - ii[ax] * stride[ax];
            double dw[4] = {0.0, 0.0, 0.0, 0.0};
            for (int l = 0; l < n; ++l) {
                const int mm = base + l * stride[ax];
                const double dd = sdm[ax * n * n + ii[ax] * n + l];
#pragma unroll
                for (int s = 0; s < 4; ++s) dw[s] += dd * sw[s * nn + mm];
            }
            if constexpr (MODAL && !CV) {
                const double *c = tab.cmet + k * 9 + ax * 3;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    vr[s * 3 + 0] += dw[s] * c[0];
                    vr[s * 3 + 1] += dw[s] * c[1];
                    vr[s * 3 + 2] += dw[s] * c[2];
                }
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) vr[s * 3 + ax] = dw[s];
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                volc[s * 3 + c] = cofT[0 * 3 + c] * vr[s * 3 + 0] + cofT[1 * 3 + c] * vr[s * 3 + 1] +
                                  cofT[2 * 3 + c] * vr[s * 3 + 2];
        if constexpr (MODAL) {
#pragma unroll
            for (int f = 0; f < 12; ++f) sgn[f * nn + k] = volc[f];
        }
    }
    if constexpr (MODAL) {
        // face terms ws (w* - w_own) n of every side, then one GEMM for the right-hand side
        //   rhs = [V^T W | E_1^T | E_2^T | ...] [vol ; face terms]
        for (int t = tid; t < nsl * n2; t += BS) {
            const int ls = t / n2, p = t % n2, sl = s0 + ls;
            const int nb = a.mesh.slot_nbr[sl];
            const double *sg = slot_geom<CV>(a.mesh, sl, p);
            double qa[5], qb[5], wa[4], wb[4];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qa[v] = a.Tq[((int64_t)sl * 5 + v) * n2 + p];
                qb[v] = a.Tq[((int64_t)nb * 5 + v) * n2 + p];
            }
            lifting_vars<REL>(qa, a.phys, wa);
            lifting_vars<REL>(qb, a.phys, wb);
            const double ws = a.ops.Wq[a.mesh.slot_kind[sl] * n2 + p] * sg[3];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double wst = 0.5 * (wb[s] - wa[s]) * ws;
#pragma unroll
                for (int c = 0; c < 3; ++c) sbuf[(ls * 12 + s * 3 + c) * n2 + p] = wst * sg[c];
            }
        }
        __syncthreads();
        const double *data = a.ops.data;
        constexpr int KBm = (m + 15) / 16, KBnn = (nn + 15) / 16, KBn2 = (n2 + 15) / 16;
        // affine: g~ = M_D^-1 rhs / J in the same product (the tables come premultiplied by
        // M_D^-1); curved: rhs with the plain V^T W and E^T, then M_e^-1 below
        constexpr bool cv = CV;
        const double *volA = cv ? tab.VtWp : tab.MVtWp;
        const int64_t faceA = (int64_t)n2 * KBm * 16 + (cv ? 0 : (int64_t)m * KBn2 * 16);
        mfma_gemm_pk(
            m, KBnn + nsl * KBn2, 12,
            [&](int i, int kb) -> const double * {
                if (kb < KBnn) return volA + ((int64_t)i * KBnn + kb) * 16;
                const int r = kb - KBnn, ls = r / KBn2;
                return data + sops[ls] + faceA + ((int64_t)i * KBn2 + (r - ls * KBn2)) * 16;
            },
            [&](int kk, int c) {
                if (kk < KBnn * 16) return sgn[c * nn + kclamp(kk, nn)];
                const int r = kk - KBnn * 16, ls = r / (KBn2 * 16), p = r - ls * KBn2 * 16;
                return sbuf[(ls * 12 + c) * n2 + kclamp(p, n2)];
            },
            [&](int i, int c, double v) { sgt[c * m + i] = cv ? v : v * iJ; },
            [&](int kb) { return kb < KBnn ? ksteps_of(nn, kb) : ksteps_of(n2, (kb - KBnn) % KBn2); });
        __syncthreads();
        if constexpr (cv) {
            // g~ = M_e^-1 rhs (the element's own mass matrix, symmetric: lane i reads its column)
            const double *Mi = a.mesh.minv + a.mesh.minv_off[e];
            double gi[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) gi[f] = 0.0;
            if (tid < m) {
#pragma unroll 4
                for (int j = 0; j < m; ++j) {
                    const double c = Mi[(int64_t)j * m + tid];
#pragma unroll
                    for (int f = 0; f < 12; ++f) gi[f] += c * sgt[f * m + j];
                }
            }
            __syncthreads();
            if (tid < m) {
#pragma unroll
                for (int f = 0; f < 12; ++f) sgt[f * m + tid] = gi[f];
            }
            __syncthreads();
        }
        // gradients at the nodes (V g~) and at every face point (E g~)
        mfma_gemm_pk(nn, KBm, 12, [&](int i, int kb) { return tab.Vp + ((int64_t)i * KBm + kb) * 16; },
                     [&](int kk, int c) { return sgt[c * m + kclamp(kk, m)]; },
                     [&](int i, int c, double v) { sgn[c * nn + i] = v; },
                     [&](int kb) { return ksteps_of(m, kb); });
        const int np = nsl * n2;
        mfma_gemm_pk(np, KBm, 12,
                     [&](int i, int kb) { return data + sops[i / n2] + ((int64_t)(i % n2) * KBm + kb) * 16; },
                     [&](int kk, int c) { return sgt[c * m + kclamp(kk, m)]; },
                     [&](int i, int c, double v) { sbuf[c * np + i] = v; },
                     [&](int kb) { return ksteps_of(m, kb); });
        __syncthreads();
        if (act) {
#pragma unroll
            for (int f = 0; f < 12; ++f) g[f] = sgn[f * nn + k];
        }
    } else {
        // hexahedra: nodal BR1 with the lumped mass, one face side at a time
        double surf[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) surf[f] = 0.0;
        for (int sl = s0; sl < s1; ++sl) {
            __syncthreads();
            const int nb = a.mesh.slot_nbr[sl];
            const double *Wk = a.ops.Wq + a.mesh.slot_kind[sl] * n2;
            for (int p = tid; p < n2; p += BS) {
                const double *sg = slot_geom<CV>(a.mesh, sl, p);
                double qa[5], qb[5], wa[4], wb[4];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    qa[v] = a.Tq[((int64_t)sl * 5 + v) * n2 + p];
                    qb[v] = a.Tq[((int64_t)nb * 5 + v) * n2 + p];
                }
                lifting_vars<REL>(qa, a.phys, wa);
                lifting_vars<REL>(qb, a.phys, wb);
                const double ws = Wk[p] * sg[3];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double wst = 0.5 * (wb[s] - wa[s]) * ws;
#pragma unroll
                    for (int c = 0; c < 3; ++c) sbuf[(s * 3 + c) * n2 + p] = wst * sg[c];
                }
            }
            __syncthreads();
            const int op = a.mesh.slot_op[sl];
            if (act) {
                const int plane = a.ops.op_plane[op];
                const int a2 = vol_plane(plane, k, n);
                if (a2 >= 0) {
                    if (a.ops.op_perm[op]) {
                        const int p = a.ops.idata[a.ops.op_ioff[op] + n2 + a2];
#pragma unroll
                        for (int f = 0; f < 12; ++f) surf[f] += sbuf[f * n2 + p];
                    } else {
                        const double *I = a.ops.data + a.ops.op_off[op];
#pragma unroll 1
                        for (int p = 0; p < n2; ++p) {
                            const double c = I[(int64_t)p * n2 + a2];
#pragma unroll
                            for (int f = 0; f < 12; ++f) surf[f] += c * sbuf[f * n2 + p];
                        }
                    }
                }
            }
        }
        if (act) {
            const double wk = tab.w[k];
#pragma unroll
            for (int f = 0; f < 12; ++f) {
                g[f] = (surf[f] / wk + volc[f]) * iJ;
                sgn[f * nn + k] = g[f];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------- dispatch
#define PDG_DISPATCH_TN(FN, ...)                                          \
    switch (type * 16 + N) {                                              \
        case 0 * 16 + 2: FN<0, 2>(__VA_ARGS__); break;                     \
        case 0 * 16 + 3: FN<0, 3>(__VA_ARGS__); break;                     \
        case 0 * 16 + 4: FN<0, 4>(__VA_ARGS__); break;                     \
        case 0 * 16 + 5: FN<0, 5>(__VA_ARGS__); break;                     \
        case 0 * 16 + 6: FN<0, 6>(__VA_ARGS__); break;                     \
        case 1 * 16 + 2: FN<1, 2>(__VA_ARGS__); break;                     \
        case 1 * 16 + 3: FN<1, 3>(__VA_ARGS__); break;                     \
        case 1 * 16 + 4: FN<1, 4>(__VA_ARGS__); break;                     \
        case 1 * 16 + 5: FN<1, 5>(__VA_ARGS__); break;                     \
        case 1 * 16 + 6: FN<1, 6>(__VA_ARGS__); break;                     \
        case 2 * 16 + 2: FN<2, 2>(__VA_ARGS__); break;                     \
        case 2 * 16 + 3: FN<2, 3>(__VA_ARGS__); break;                     \
        case 2 * 16 + 4: FN<2, 4>(__VA_ARGS__); break;                     \
        case 2 * 16 + 5: FN<2, 5>(__VA_ARGS__); break;                     \
        case 2 * 16 + 6: FN<2, 6>(__VA_ARGS__); break;                     \
        case 3 * 16 + 2: FN<3, 2>(__VA_ARGS__); break;                     \
        case 3 * 16 + 3: FN<3, 3>(__VA_ARGS__); break;                     \
        case 3 * 16 + 4: FN<3, 4>(__VA_ARGS__); break;                     \
        case 3 * 16 + 5: FN<3, 5>(__VA_ARGS__); break;                     \
        case 3 * 16 + 6: FN<3, 6>(__VA_ARGS__); break;                     \
        default: return hipErrorInvalidValue;                             \
    }

#define PDG_DISPATCH_N(FN, ...)            \
    switch (N) {                           \
        case 2: FN<2>(__VA_ARGS__); break; \
        case 3: FN<3>(__VA_ARGS__); break; \
        case 4: FN<4>(__VA_ARGS__); break; \
        case 5: FN<5>(__VA_ARGS__); break; \
        case 6: FN<6>(__VA_ARGS__); break; \
        default: return hipErrorInvalidValue; \
    }

}  // namespace pdg
