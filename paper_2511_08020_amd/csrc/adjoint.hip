// Adjoint of the DG residual on mixed meshes (gfx950, FP64): grad = (dR/dU)^T lam.
//
// The residual is a chain of linear element operators (V, the face-point traces E, the
// sum-factorised weak derivative, the contravariant metric terms, the lifts E^T, M_D^-1 and
// 1/J) and pointwise functions (inviscid and viscous fluxes, the Lax-Friedrichs flux, the BR1
// lifting variables).  The kernels below apply each linear operator transposed and each
// pointwise function through its analytic Jacobian, in the reverse order of the residual's
// phases.  With mu = M_D^-T lam / J (hexahedra: lam / (w J)) the phases are
//   0  trace    state traces Tq = E u~ and flux cotangents Lf = -ws E mu at every face side
//   1  volume   weak-derivative and flux adjoint at the nodes; at the face points the
//               Lax-Friedrichs adjoint dLF/dq_own^T (Lf_own - Lf_nbr) (the flux is antisymmetric,
//               so the neighbour's flux contributes through the same Jacobian); Navier-Stokes
//               recomputes the BR1 gradients, runs the viscous flux adjoint, the transposed
//               gradient operator and leaves Lw = ws n . (E nu) for the face values
//   2  surface  (Navier-Stokes) BR1 face-value adjoint (Lw_nbr - Lw_own)/2 through the lifting
//               variables of the own trace, and the final lift E^T
// Every output entry is written by one thread; no atomics.
#include "phases.h"

namespace pdg {

// ------------------------------------------------------------------------ pointwise adjoints
__device__ __forceinline__ void dpressure(const double q[5], double g1, double dp[5]) {
    const double ir = 1.0 / q[0];
    const double u0 = q[1] * ir, u1 = q[2] * ir, u2 = q[3] * ir;
    dp[0] = 0.5 * g1 * (u0 * u0 + u1 * u1 + u2 * u2);
    dp[1] = -g1 * u0;
    dp[2] = -g1 * u1;
    dp[3] = -g1 * u2;
    dp[4] = g1;
}

// qb += sum_{c,v} Fb[c][v] dF[c][v]/dq of the inviscid flux (the reference pressure is constant)
__device__ __forceinline__ void euler_flux_vjp(const double q[5], const double Fb[3][5], double gamma,
                                               double qb[5]) {
    const double ir = 1.0 / q[0];
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double g1 = gamma - 1.0;
    const double p = g1 * (q[4] - 0.5 * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
    double Pc = 0.0;  // coefficient of dp
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        qb[1 + c] += Fb[c][0];
        double ac = 0.0;  // coefficient of du_c from the momentum rows m_i u_c
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            qb[1 + i] += Fb[c][1 + i] * u[c];
            ac += Fb[c][1 + i] * q[1 + i];
        }
        Pc += Fb[c][1 + c] + Fb[c][4] * u[c];
        qb[4] += Fb[c][4] * u[c];
        const double bc = ac + Fb[c][4] * (q[4] + p);
        qb[1 + c] += bc * ir;
        qb[0] -= bc * u[c] * ir;
    }
    double dp[5];
    dpressure(q, g1, dp);
#pragma unroll
    for (int v = 0; v < 5; ++v) qb[v] += Pc * dp[v];
}

// out += (d LF(qa, qb, n)/d qa)^T d; the maximum wave speed takes side a on ties and
// d|x|/dx = sign(x) with sign(0) = 0
__device__ __forceinline__ void lf_vjp(const double qa[5], const double qb[5], const double nv[3], double gamma,
                                       const double d[5], double out[5]) {
    double Fb[3][5];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 5; ++v) Fb[c][v] = 0.5 * nv[c] * d[v];
    euler_flux_vjp(qa, Fb, gamma, out);
    const double ira = 1.0 / qa[0], irb = 1.0 / qb[0];
    const double una = (qa[1] * nv[0] + qa[2] * nv[1] + qa[3] * nv[2]) * ira;
    const double unb = (qb[1] * nv[0] + qb[2] * nv[1] + qb[3] * nv[2]) * irb;
    const double pa = (gamma - 1.0) * (qa[4] - 0.5 * (qa[1] * qa[1] + qa[2] * qa[2] + qa[3] * qa[3]) * ira);
    const double pb = (gamma - 1.0) * (qb[4] - 0.5 * (qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]) * irb);
    const double ca = sqrt(gamma * pa * ira);
    const double aa = fabs(una) + ca, ab = fabs(unb) + sqrt(gamma * pb * irb);
    const double lam = fmax(aa, ab);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] += 0.5 * lam * d[v];
    if (aa >= ab) {
        double jd = 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) jd += d[v] * (qb[v] - qa[v]);
        const double coef = -0.5 * jd;
        const double sg = una > 0.0 ? 1.0 : (una < 0.0 ? -1.0 : 0.0);
        double dp[5];
        dpressure(qa, gamma - 1.0, dp);
        const double kc = gamma / (2.0 * ca) * ira;  // dc = kc (dp - p/rho e_0)
        out[0] += coef * (-sg * una * ira + kc * (dp[0] - pa * ira));
#pragma unroll
        for (int i = 0; i < 3; ++i) out[1 + i] += coef * (sg * nv[i] * ira + kc * dp[1 + i]);
        out[4] += coef * kc * dp[4];
    }
}

// qb += sum_s wb[s] dW_s/dq of the lifting variables W = (u, v, w, T), T = p / (rho R)
__device__ __forceinline__ void lifting_vjp(const double q[5], const double wb[4], const Physics &ph, double qb[5]) {
    const double ir = 1.0 / q[0];
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double g1 = ph.gamma - 1.0;
    const double p = g1 * (q[4] - 0.5 * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qb[1 + i] += wb[i] * ir;
        qb[0] -= wb[i] * u[i] * ir;
    }
    const double t = wb[3] * ir / ph.R;
    double dp[5];
    dpressure(q, g1, dp);
#pragma unroll
    for (int v = 0; v < 5; ++v) qb[v] += t * dp[v];
    qb[0] -= t * p * ir;
}

// qb += (dFv/dq)^T Fvb, gb += (dFv/dg)^T Fvb of the viscous flux (g[s*3+c] = dW_s/dx_c)
__device__ __forceinline__ void visc_vjp(const double q[5], const double g[12], const double Fvb[3][5],
                                         const Physics &ph, double qb[5], double gb[12]) {
    const double ir = 1.0 / q[0];
    const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
    const double div = g[0] + g[4] + g[8];
    const double kappa = ph.mu * ph.gamma * ph.R / ((ph.gamma - 1.0) * ph.Pr);
    double divb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double si = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double tau = ph.mu * (g[i * 3 + c] + g[c * 3 + i]);
            if (i == c) tau -= ph.mu * (2.0 / 3.0) * div;
            si += Fvb[c][4] * tau;
            const double tb = Fvb[c][1 + i] + Fvb[c][4] * u[i];
            gb[i * 3 + c] += ph.mu * tb;
            gb[c * 3 + i] += ph.mu * tb;
            if (i == c) divb -= ph.mu * (2.0 / 3.0) * tb;
        }
        qb[1 + i] += si * ir;
        qb[0] -= si * u[i] * ir;
    }
    gb[0] += divb;
    gb[4] += divb;
    gb[8] += divb;
#pragma unroll
    for (int c = 0; c < 3; ++c) gb[9 + c] += kappa * Fvb[c][4];
}

// ------------------------------------------------------------------------------ in/out helpers
__device__ __forceinline__ double lam_at(const AdjArgs &a, int64_t idx) {
    double v = a.Kb[idx];
    if (a.Ubr) v += a.c * a.Ubr[idx];
    return v;
}

__device__ __forceinline__ void store_grad(const AdjArgs &a, int64_t idx, double g) {
    if (a.mode == 0) {
        a.gout[idx] = g;
    } else {
        const double l = lam_at(a, idx);
        a.Ubar[idx] = a.Ubar[idx] + g;
        a.Kbar[idx] = a.a * l;
    }
}

__device__ __forceinline__ double face_ws(const StageArgs &s, int sl, int p, int n2) {
    return s.ops.Wq[s.mesh.slot_kind[sl] * n2 + p] * s.mesh.slot_geo[4 * (int64_t)sl + 3];
}

// hexahedra: sum over the element's face sides of I^T applied to per-point values
// src[f * np + (sl - s0) * n2 + p] at the volume node k (nf fields)
template <int NF>
__device__ __forceinline__ void hex_lift_gather(const StageArgs &s, int s0, int s1, int k, int n, int n2, int np,
                                                const double *src, double acc[NF]) {
    for (int sl = s0; sl < s1; ++sl) {
        const int op = s.mesh.slot_op[sl];
        const int a2 = vol_plane(s.ops.op_plane[op], k, n);
        if (a2 < 0) continue;
        const double *gs = src + (sl - s0) * n2;
        if (s.ops.op_perm[op]) {
            const int p = s.ops.idata[s.ops.op_ioff[op] + n2 + a2];
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] += gs[f * np + p];
        } else {
            const double *I = s.ops.data + s.ops.op_off[op];
#pragma unroll 1
            for (int p = 0; p < n2; ++p) {
                const double c = I[(int64_t)p * n2 + a2];
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] += c * gs[f * np + p];
            }
        }
    }
}

// hexahedra: value at face point p of slot sl of nodal fields src[f * nn + k] (trace operator)
template <int NF>
__device__ __forceinline__ void hex_trace_point(const StageArgs &s, int sl, int p, int n, int n2, int nn,
                                                const double *src, double out[NF]) {
    const int op = s.mesh.slot_op[sl];
    const int plane = s.ops.op_plane[op];
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] = 0.0;
    if (s.ops.op_perm[op]) {
        const int k = plane_vol(plane, s.ops.idata[s.ops.op_ioff[op] + p], n);
#pragma unroll
        for (int f = 0; f < NF; ++f) out[f] = src[f * nn + k];
    } else {
        const double *I = s.ops.data + s.ops.op_off[op] + (int64_t)p * n2;
#pragma unroll 1
        for (int a2 = 0; a2 < n2; ++a2) {
            const int k = plane_vol(plane, a2, n);
            const double c = I[a2];
#pragma unroll
            for (int f = 0; f < NF; ++f) out[f] += c * src[f * nn + k];
        }
    }
}

// --------------------------------------------------------------------------- phase 0: traces
template <int T, int N>
struct ATraceLDS {
    using D = Dm<T, N>;
    static constexpr int nd = T == PDG_HEX ? D::nn : D::m;
    static constexpr int u = 0, l = 5 * nd, mu = l + (T == PDG_HEX ? 0 : 5 * nd);
    static constexpr int ops = mu + 5 * nd;
    static constexpr int size = ops + D::SLOTS;
};

template <int T, int N>
__device__ __forceinline__ void atrace_elem(const StageArgs &s, const AdjArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    using L = ATraceLDS<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m, BS = D::BS;
    constexpr bool MODAL = T != PDG_HEX;
    double *su = smem + L::u, *sl = smem + L::l, *smu = smem + L::mu;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + L::ops);
    const int tid = threadIdx.x;
    const int64_t off = s.mesh.off[e];
    const int s0 = s.mesh.slot_begin[e], s1 = s.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0;
    const double iJ = 1.0 / s.mesh.geo[10 * (int64_t)e];
    for (int t = tid; t < nsl; t += BS) sops[t] = (MODAL ? s.ops.op_poff : s.ops.op_off)[s.mesh.slot_op[s0 + t]];
    if constexpr (MODAL) {
        for (int t = tid; t < 5 * m; t += BS) {
            su[t] = s.U[off + t];
            sl[t] = lam_at(a, off + t);
        }
        __syncthreads();
        // mu = M_D^-T lam / J
        constexpr int KBm = (m + 15) / 16;
        const double *MTp = s.tab[T].MinvTp;
        mfma_gemm_pk(m, KBm, 5, [&](int i, int kb) { return MTp + ((int64_t)i * KBm + kb) * 16; },
                     [&](int kk, int c) { return sl[c * m + kclamp(kk, m)]; },
                     [&](int i, int c, double v) { smu[c * m + i] = v * iJ; }, [&](int kb) { return ksteps_of(m, kb); });
        __syncthreads();
        // traces of u~ and mu at every face point of the element: one contraction, 10 columns
        const double *data = s.ops.data;
        double *Tq = s.Tq, *Lf = a.Lf;
        mfma_gemm_pk((s1 - s0) * n2, KBm, 10,
                  [&](int i, int kb) { return data + sops[i / n2] + ((int64_t)(i % n2) * KBm + kb) * 16; },
                  [&](int kk, int c) { const int k2 = kclamp(kk, m); return c < 5 ? su[c * m + k2] : smu[(c - 5) * m + k2]; },
                  [&](int i, int c, double v) {
                      const int slx = s0 + i / n2, p = i % n2;
                      if (c < 5)
                          Tq[((int64_t)slx * 5 + c) * n2 + p] = v;
                      else
                          Lf[((int64_t)slx * 5 + c - 5) * n2 + p] = -face_ws(s, slx, p, n2) * v;
                  },
                  [&](int kb) { return ksteps_of(m, kb); });
    } else {
        const double *w = s.tab[T].w;
        for (int t = tid; t < 5 * nn; t += BS) {
            su[t] = s.U[off + t];
            smu[t] = lam_at(a, off + t) * iJ / w[t % nn];
        }
        __syncthreads();
        for (int t = tid; t < nsl * n2; t += BS) {
            const int slx = s0 + t / n2, p = t % n2;
            double tu[5], tm[5];
            hex_trace_point<5>(s, slx, p, n, n2, nn, su, tu);
            hex_trace_point<5>(s, slx, p, n, n2, nn, smu, tm);
            const double ws = face_ws(s, slx, p, n2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                s.Tq[((int64_t)slx * 5 + v) * n2 + p] = tu[v];
                a.Lf[((int64_t)slx * 5 + v) * n2 + p] = -ws * tm[v];
            }
        }
    }
}

template <int T, int N>
__global__ __launch_bounds__(kBS<N>) void k_atrace(StageArgs s, AdjArgs a) {
    __shared__ double smem[ATraceLDS<T, N>::size];
    atrace_elem<T, N>(s, a, s.list[T][blockIdx.x], smem);
}

// --------------------------------------------------------------------------- phase 1: volume
template <int T, int N, bool NS, int S = Dm<T, N>::SLOTS>
struct AVolLDS {
    using D = Dm<T, N>;
    static constexpr bool MODAL = T != PDG_HEX;
    static constexpr int nn = D::nn, m = D::m, n2 = D::n2;
    static constexpr int dh = 0;
    static constexpr int dm = dh + 3 * D::n * D::n;            // NS: strong 1-D derivatives (BR1)
    static constexpr int ops = dm + (NS ? 3 * D::n * D::n : 0);
    static constexpr int pops = ops + S;                       // packed-operator offsets (modal)
    static constexpr int u = pops + S;                         // u~ (modal)
    static constexpr int l = u + (MODAL ? 5 * m : 0);          // lam (modal)
    static constexpr int mu = l + (MODAL ? 5 * m : 0);         // spare (modal), part of the block below
    static constexpr int d = mu + (MODAL ? 5 * m : 0);         // q, then dbar, then qbar (5 nn)
    static constexpr int tb = d + 5 * nn;                      // Tq-bar at the face points (5 S n2)
    // NS modal: the block of u~, lam and the spare (15 m) is dead once dbar is formed, so the lifting variables
    // (live only in the forward gradient recomputation) and the transposed BR1 right-hand side
    // (live only after it) reuse that block when they fit
    static constexpr bool WAL = NS && MODAL && 15 * m >= 4 * nn;
    static constexpr bool GAL = NS && MODAL;
    static constexpr int w = WAL ? u : tb + 5 * S * n2;        // NS: lifting variables (4 nn)
    static constexpr int gn = (WAL ? tb + 5 * S * n2 : w + (NS ? 4 * nn : 0));  // NS: nodal gradients / adjoints (12 nn)
    static constexpr int gf = gn + (NS ? 12 * nn : 0);         // NS: face-point gradients / adjoints (12 S n2)
    static constexpr int gm = GAL ? u : gf + (NS ? 12 * S * n2 : 0);  // NS modal: 12 m
    static constexpr int gt = GAL ? gf + 12 * S * n2 : gm + (NS && MODAL ? 12 * m : 0);  // NS modal: 12 m
    static constexpr int size = gt + (NS && MODAL ? 12 * m : 0);
    static_assert(!GAL || 12 * m <= 15 * m, "BR1 block must fit the u~, lam, mu block");
};

template <int T, int N, bool NS, int BS = Dm<T, N>::BS, int S = Dm<T, N>::SLOTS>
__device__ __forceinline__ void avol_elem(const StageArgs &s, const AdjArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    using L = AVolLDS<T, N, NS, S>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m;
    constexpr bool MODAL = T != PDG_HEX;
    double *sdh = smem + L::dh;
    double *sdm = smem + L::dm;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + L::ops);
    int64_t *spops = reinterpret_cast<int64_t *>(smem + L::pops);
    double *su = smem + L::u, *sl = smem + L::l, *sd = smem + L::d, *stb = smem + L::tb;
    double *sw = smem + L::w, *sgn = smem + L::gn, *sgf = smem + L::gf, *sgm = smem + L::gm, *sgt = smem + L::gt;

    const int tid = threadIdx.x;
    const int64_t off = s.mesh.off[e];
    const DevType &tab = s.tab[T];
    const double *geo = s.mesh.geo + 10 * (int64_t)e;
    const double iJ = 1.0 / geo[0];
    double cofT[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) cofT[i] = geo[1 + i];
    const int s0 = s.mesh.slot_begin[e], s1 = s.mesh.slot_begin[e + 1];
    const int nsl = s1 - s0, np = nsl * n2;
    const double *data = s.ops.data;
    constexpr int KBm = (m + 15) / 16, KBnn = (nn + 15) / 16, KBn2 = (n2 + 15) / 16;

    for (int t = tid; t < 3 * n * n; t += BS) sdh[t] = tab.dhat[t / (n * n)][t % (n * n)];
    if constexpr (NS)
        for (int t = tid; t < 3 * n * n; t += BS) sdm[t] = tab.dmat[t / (n * n)][t % (n * n)];
    for (int t = tid; t < nsl; t += BS) {
        sops[t] = s.ops.op_off[s.mesh.slot_op[s0 + t]];
        spops[t] = s.ops.op_poff[s.mesh.slot_op[s0 + t]];
    }
    if constexpr (MODAL) {
        for (int t = tid; t < 5 * m; t += BS) {
            su[t] = s.U[off + t];
            sl[t] = lam_at(a, off + t);
        }
        __syncthreads();
        mfma_gemm_pk(nn, KBm, 5, [&](int i, int kb) { return tab.Vp + ((int64_t)i * KBm + kb) * 16; },
                     [&](int kk, int c) { return su[c * m + kclamp(kk, m)]; },
                     [&](int i, int c, double v) { sd[c * nn + i] = v; }, [&](int kb) { return ksteps_of(m, kb); });
    }
    __syncthreads();

    const int k = tid;
    const bool act = k < nn;
    const int ii[3] = {k % n, (k / n) % n, k / (n * n)};
    const int stride[3] = {1, n, n * n};
    double q[5] = {1, 0, 0, 0, 1};
    if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = MODAL ? sd[v * nn + k] : s.U[off + v * nn + k];
    }
    __syncthreads();
    // dbar: cotangent of the weak derivative at the nodes, (M_D^-1 V^T W)^T lam / J
    if constexpr (MODAL) {
        mfma_gemm_pk(nn, KBm, 5, [&](int i, int kb) { return tab.MVtWtp + ((int64_t)i * KBm + kb) * 16; },
                     [&](int kk, int c) { return sl[c * m + kclamp(kk, m)]; },
                     [&](int i, int c, double v) { sd[c * nn + i] = v * iJ; }, [&](int kb) { return ksteps_of(m, kb); });
    } else {
        if (act) {
#pragma unroll
            for (int v = 0; v < 5; ++v) sd[v * nn + k] = lam_at(a, off + v * nn + k) * iJ;
        }
    }

    double g[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) g[f] = 0.0;
    // the lifting variables overwrite lam's block: every wave must have finished reading lam
    if constexpr (L::WAL) __syncthreads();
    if constexpr (NS) br1_gradients<T, N, BS, false>(s, e, s0, s1, cofT, iJ, q, spops, sdm, sw, sgn, sgf, sgt, g);
    else __syncthreads();

    // face points: Lax-Friedrichs adjoint (and the viscous normal flux adjoint)
    for (int t = tid; t < np; t += BS) {
        const int slx = s0 + t / n2, p = t % n2;
        const int nb = s.mesh.slot_nbr[slx];
        const double *sg = s.mesh.slot_geo + 4 * (int64_t)slx;
        const double nv[3] = {sg[0], sg[1], sg[2]};
        double qa[5], qo[5], dl[5], tbv[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qa[v] = s.Tq[((int64_t)slx * 5 + v) * n2 + p];
            qo[v] = s.Tq[((int64_t)nb * 5 + v) * n2 + p];
            dl[v] = a.Lf[((int64_t)slx * 5 + v) * n2 + p] - a.Lf[((int64_t)nb * 5 + v) * n2 + p];
        }
        lf_vjp(qa, qo, nv, s.phys.gamma, dl, tbv);
        if constexpr (NS) {
            double gp[12], gb[12];
            if constexpr (MODAL) {
#pragma unroll
                for (int f = 0; f < 12; ++f) gp[f] = sgf[f * np + t];
            } else {
                hex_trace_point<12>(s, slx, p, n, n2, nn, sgn, gp);
            }
            double Fvb[3][5];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int v = 0; v < 5; ++v) Fvb[c][v] = -0.5 * nv[c] * dl[v];
#pragma unroll
            for (int f = 0; f < 12; ++f) gb[f] = 0.0;
            visc_vjp(qa, gp, Fvb, s.phys, tbv, gb);
#pragma unroll
            for (int f = 0; f < 12; ++f) sgf[f * np + t] = gb[f];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) stb[v * np + t] = tbv[v];
    }
    __syncthreads();

    // nodes: transposed weak derivative, metric terms and flux adjoint
    double qbar[5] = {0, 0, 0, 0, 0};
    if (act) {
        double Gb[3][5];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int v = 0; v < 5; ++v) Gb[ax][v] = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const int base = k - ii[ax] * stride[ax];
            for (int i = 0; i < n; ++i) {
                const double dh = sdh[ax * n * n + i * n + ii[ax]];
                const int kk = base + i * stride[ax];
#pragma unroll
                for (int v = 0; v < 5; ++v) Gb[ax][v] += dh * sd[v * nn + kk];
            }
        }
        double Fb[3][5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double Fhb[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if constexpr (MODAL) {
                    const double *cm = tab.cmet + k * 9;
                    Fhb[b] = cm[0 * 3 + b] * Gb[0][v] + cm[1 * 3 + b] * Gb[1][v] + cm[2 * 3 + b] * Gb[2][v];
                } else {
                    Fhb[b] = Gb[b][v];
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Fb[c][v] = cofT[0 * 3 + c] * Fhb[0] + cofT[1 * 3 + c] * Fhb[1] + cofT[2 * 3 + c] * Fhb[2];
        }
        euler_flux_vjp(q, Fb, s.phys.gamma, qbar);
        if constexpr (NS) {
            double Fvb[3][5], gbn[12];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int v = 0; v < 5; ++v) Fvb[c][v] = -Fb[c][v];
#pragma unroll
            for (int f = 0; f < 12; ++f) gbn[f] = 0.0;
            visc_vjp(q, g, Fvb, s.phys, qbar, gbn);
#pragma unroll
            for (int f = 0; f < 12; ++f) sgn[f * nn + k] = gbn[f];
        }
    }

    if constexpr (NS) {
        __syncthreads();
        double vb[12];  // cotangent of the volume part of the gradient right-hand side at node k
#pragma unroll
        for (int f = 0; f < 12; ++f) vb[f] = 0.0;
        if constexpr (MODAL) {
            // g~bar = V^T gbar_nodes + sum_sides E^T gbar_faces
            mfma_gemm_pk(
                m, KBnn + nsl * KBn2, 12,
                [&](int i, int kb) -> const double * {
                    if (kb < KBnn) return tab.Vtp + ((int64_t)i * KBnn + kb) * 16;
                    const int r = kb - KBnn, ls = r / KBn2;
                    return data + spops[ls] + (int64_t)n2 * KBm * 16 + ((int64_t)i * KBn2 + (r - ls * KBn2)) * 16;
                },
                [&](int kk, int c) {
                    if (kk < KBnn * 16) return sgn[c * nn + kclamp(kk, nn)];
                    const int r = kk - KBnn * 16, ls = r / (KBn2 * 16), p = r - ls * KBn2 * 16;
                    return sgf[c * np + ls * n2 + kclamp(p, n2)];
                },
                [&](int i, int c, double v) { sgm[c * m + i] = v; },
                [&](int kb) { return kb < KBnn ? ksteps_of(nn, kb) : ksteps_of(n2, (kb - KBnn) % KBn2); });
            __syncthreads();
            // with nu = M_D^-T g~bar / J: volume part (V^T W)^T nu = (M_D^-1 V^T W)^T g~bar / J at
            // the nodes, face part E nu = (E M_D^-1) g~bar / J at the face points
            mfma_gemm_pk(nn, KBm, 12, [&](int i, int kb) { return tab.MVtWtp + ((int64_t)i * KBm + kb) * 16; },
                         [&](int kk, int c) { return sgm[c * m + kclamp(kk, m)]; },
                         [&](int i, int c, double v) { sgn[c * nn + i] = v * iJ; },
                         [&](int kb) { return ksteps_of(m, kb); });
            mfma_gemm_pk(np, KBm, 12,
                         [&](int i, int kb) {
                             return data + spops[i / n2] + (int64_t)n2 * KBm * 16 + 2 * (int64_t)m * KBn2 * 16 +
                                    ((int64_t)(i % n2) * KBm + kb) * 16;
                         },
                         [&](int kk, int c) { return sgm[c * m + kclamp(kk, m)]; },
                         [&](int i, int c, double v) { sgf[c * np + i] = v * iJ; },
                         [&](int kb) { return ksteps_of(m, kb); });
            __syncthreads();
            for (int t = tid; t < np; t += BS) {
                const int slx = s0 + t / n2, p = t % n2;
                const double *sg = s.mesh.slot_geo + 4 * (int64_t)slx;
                const double ws = face_ws(s, slx, p, n2);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    a.Lw[((int64_t)slx * 4 + r) * n2 + p] =
                        ws * (sg[0] * sgf[(r * 3 + 0) * np + t] + sg[1] * sgf[(r * 3 + 1) * np + t] +
                              sg[2] * sgf[(r * 3 + 2) * np + t]);
            }
            if (act) {
#pragma unroll
                for (int f = 0; f < 12; ++f) vb[f] = sgn[f * nn + k];
            }
        } else {
            // hexahedra: g = (surf / w + vol) / J, with the face gradients I g
            double gt[12];
            if (act) {
#pragma unroll
                for (int f = 0; f < 12; ++f) gt[f] = sgn[f * nn + k];
                hex_lift_gather<12>(s, s0, s1, k, n, n2, np, sgf, gt);
            }
            __syncthreads();
            if (act) {
                const double sc = iJ / tab.w[k];
#pragma unroll
                for (int f = 0; f < 12; ++f) {
                    sgn[f * nn + k] = gt[f] * sc;  // cotangent of the lifted face terms
                    vb[f] = gt[f] * iJ;
                }
            }
            __syncthreads();
            for (int t = tid; t < np; t += BS) {
                const int slx = s0 + t / n2, p = t % n2;
                const double *sg = s.mesh.slot_geo + 4 * (int64_t)slx;
                double sb[12];
                hex_trace_point<12>(s, slx, p, n, n2, nn, sgn, sb);
                const double ws = face_ws(s, slx, p, n2);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    a.Lw[((int64_t)slx * 4 + r) * n2 + p] =
                        ws * (sg[0] * sb[r * 3 + 0] + sg[1] * sb[r * 3 + 1] + sg[2] * sb[r * 3 + 2]);
            }
        }
        __syncthreads();
        // volume part J grad(w_h) of the gradient, transposed: first the physical-to-reference
        // transform and the node's contravariant vectors (modal) at each node, then the strong
        // derivative along each line, transposed
        if (act) {
            double vr[12];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    vr[r * 3 + b] = cofT[b * 3 + 0] * vb[r * 3 + 0] + cofT[b * 3 + 1] * vb[r * 3 + 1] +
                                    cofT[b * 3 + 2] * vb[r * 3 + 2];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double z;
                    if constexpr (MODAL) {
                        const double *cm = tab.cmet + k * 9 + ax * 3;
                        z = cm[0] * vr[r * 3 + 0] + cm[1] * vr[r * 3 + 1] + cm[2] * vr[r * 3 + 2];
                    } else {
                        z = vr[r * 3 + ax];
                    }
                    sgn[(r * 3 + ax) * nn + k] = z;
                }
            }
        }
        __syncthreads();
        if (act) {
            double wb[4] = {0, 0, 0, 0};
            for (int ax = 0; ax < 3; ++ax) {
                const int base = k - ii[ax] * stride[ax];
                for (int i = 0; i < n; ++i) {
                    const double dd = sdm[ax * n * n + i * n + ii[ax]];
                    const int kk = base + i * stride[ax];
#pragma unroll
                    for (int r = 0; r < 4; ++r) wb[r] += dd * sgn[(r * 3 + ax) * nn + kk];
                }
            }
            lifting_vjp(q, wb, s.phys, qbar);
        }
    }

    // u~bar = V^T qbar + sum_sides E^T Tq-bar (hexahedra: qbar + sum_sides I^T Tq-bar)
    __syncthreads();
    if constexpr (MODAL) {
        if (act) {
#pragma unroll
            for (int v = 0; v < 5; ++v) sd[v * nn + k] = qbar[v];
        }
        __syncthreads();
        mfma_gemm_pk(
            m, KBnn + nsl * KBn2, 5,
            [&](int i, int kb) -> const double * {
                if (kb < KBnn) return tab.Vtp + ((int64_t)i * KBnn + kb) * 16;
                const int r = kb - KBnn, ls = r / KBn2;
                return data + spops[ls] + (int64_t)n2 * KBm * 16 + ((int64_t)i * KBn2 + (r - ls * KBn2)) * 16;
            },
            [&](int kk, int c) {
                if (kk < KBnn * 16) return sd[c * nn + kclamp(kk, nn)];
                const int r = kk - KBnn * 16, ls = r / (KBn2 * 16), p = r - ls * KBn2 * 16;
                return stb[c * np + ls * n2 + kclamp(p, n2)];
            },
            [&](int i, int c, double v) {
                const int64_t idx = off + c * m + i;
                if constexpr (NS) a.Ub[idx] = v;
                else store_grad(a, idx, v);
            },
            [&](int kb) { return kb < KBnn ? ksteps_of(nn, kb) : ksteps_of(n2, (kb - KBnn) % KBn2); });
    } else {
        if (act) {
            hex_lift_gather<5>(s, s0, s1, k, n, n2, np, stb, qbar);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const int64_t idx = off + v * nn + k;
                if constexpr (NS) a.Ub[idx] = qbar[v];
                else store_grad(a, idx, qbar[v]);
            }
        }
    }
}

// WIDE: the elements with more face sides than kSlotsNarrow (list_w), else the others (list_n)
template <int T, int N, bool NS, bool WIDE>
__global__ __launch_bounds__((kVolBS<T, N>)) void k_avol(StageArgs s, AdjArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double smem[AVolLDS<T, N, NS, S>::size];
    avol_elem<T, N, NS, kVolBS<T, N>, S>(s, a, (WIDE ? s.list_w : s.list_n)[T][blockIdx.x], smem);
}

// ------------------------------------------------------------------- phase 2: BR1 face values
template <int T, int N, int S = Dm<T, N>::SLOTS>
struct ASurfLDS {
    static constexpr int tb = 0;
    static constexpr int ops = 5 * S * Dm<T, N>::n2;
    static constexpr int size = ops + S;
};

template <int T, int N, int S = Dm<T, N>::SLOTS>
__device__ __forceinline__ void asurf_elem(const StageArgs &s, const AdjArgs &a, int e, double *smem) {
    using D = Dm<T, N>;
    constexpr int n = D::n, n2 = D::n2, nn = D::nn, m = D::m, BS = D::BS;
    constexpr bool MODAL = T != PDG_HEX;
    double *stb = smem + ASurfLDS<T, N, S>::tb;
    int64_t *sops = reinterpret_cast<int64_t *>(smem + ASurfLDS<T, N, S>::ops);
    const int tid = threadIdx.x;
    const int64_t off = s.mesh.off[e];
    const int s0 = s.mesh.slot_begin[e], s1 = s.mesh.slot_begin[e + 1];
    const int np = (s1 - s0) * n2;
    for (int t = tid; t < s1 - s0; t += BS) sops[t] = (MODAL ? s.ops.op_poff : s.ops.op_off)[s.mesh.slot_op[s0 + t]];
    for (int t = tid; t < np; t += BS) {
        const int slx = s0 + t / n2, p = t % n2;
        const int nb = s.mesh.slot_nbr[slx];
        double qa[5], wb[4], tbv[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 5; ++v) qa[v] = s.Tq[((int64_t)slx * 5 + v) * n2 + p];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            wb[r] = 0.5 * (a.Lw[((int64_t)nb * 4 + r) * n2 + p] - a.Lw[((int64_t)slx * 4 + r) * n2 + p]);
        lifting_vjp(qa, wb, s.phys, tbv);
#pragma unroll
        for (int v = 0; v < 5; ++v) stb[v * np + t] = tbv[v];
    }
    __syncthreads();
    if constexpr (MODAL) {
        const double *data = s.ops.data;
        constexpr int KBm = (m + 15) / 16, KBn2 = (n2 + 15) / 16;
        mfma_gemm_pk(m, (s1 - s0) * KBn2, 5,
                     [&](int i, int kb) {
                         const int ls = kb / KBn2;
                         return data + sops[ls] + (int64_t)n2 * KBm * 16 + ((int64_t)i * KBn2 + (kb - ls * KBn2)) * 16;
                     },
                     [&](int kk, int c) {
                         const int ls = kk / (KBn2 * 16), p = kk - ls * KBn2 * 16;
                         return stb[c * np + ls * n2 + kclamp(p, n2)];
                     },
                     [&](int i, int c, double v) {
                         const int64_t idx = off + c * m + i;
                         store_grad(a, idx, a.Ub[idx] + v);
                     },
                     [&](int kb) { return ksteps_of(n2, kb % KBn2); });
    } else {
        const int k = tid;
        if (k < nn) {
            double acc[5] = {0, 0, 0, 0, 0};
            hex_lift_gather<5>(s, s0, s1, k, n, n2, np, stb, acc);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const int64_t idx = off + v * nn + k;
                store_grad(a, idx, a.Ub[idx] + acc[v]);
            }
        }
    }
}

template <int T, int N, bool WIDE>
__global__ __launch_bounds__(kBS<N>) void k_asurf(StageArgs s, AdjArgs a) {
    constexpr int S = kSlotCap<T, N, WIDE>;
    __shared__ double smem[ASurfLDS<T, N, S>::size];
    asurf_elem<T, N, S>(s, a, (WIDE ? s.list_w : s.list_n)[T][blockIdx.x], smem);
}

// ---------------------------------------------------------------------------------- launches
template <int T, int N>
static void go_atrace(const StageArgs &s, const AdjArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_atrace<T, N>), dim3(s.count[T]), dim3(Dm<T, N>::BS), 0, st, s, a);
}
// the narrow and the wide part of a type's elements, one launch each
template <int T, int N, bool NS>
static void go_avol(const StageArgs &s, const AdjArgs &a, hipStream_t st) {
    if (s.count_n[T]) hipLaunchKernelGGL((k_avol<T, N, NS, false>), dim3(s.count_n[T]), dim3(kVolBS<T, N>), 0, st, s, a);
    if (s.count_w[T]) hipLaunchKernelGGL((k_avol<T, N, NS, true>), dim3(s.count_w[T]), dim3(kVolBS<T, N>), 0, st, s, a);
}
template <int T, int N>
static void go_avol_euler(const StageArgs &s, const AdjArgs &a, hipStream_t st) {
    go_avol<T, N, false>(s, a, st);
}
// Navier-Stokes adjoint kernels exist for N <= 5, like the residual's
template <int T, int N>
static void go_avol_ns(const StageArgs &s, const AdjArgs &a, hipStream_t st) {
    if constexpr (N <= 5) go_avol<T, N, true>(s, a, st);
}
template <int T, int N>
static void go_asurf(const StageArgs &s, const AdjArgs &a, hipStream_t st) {
    if constexpr (N <= 5) {
        if (s.count_n[T]) hipLaunchKernelGGL((k_asurf<T, N, false>), dim3(s.count_n[T]), dim3(Dm<T, N>::BS), 0, st, s, a);
        if (s.count_w[T]) hipLaunchKernelGGL((k_asurf<T, N, true>), dim3(s.count_w[T]), dim3(Dm<T, N>::BS), 0, st, s, a);
    }
}

hipError_t launch_adjoint(int N, bool ns, int phase, const StageArgs &s, const AdjArgs &a, int type,
                          hipStream_t st) {
    if (s.count[type] == 0) return hipSuccess;
    if (phase == 0) {
        PDG_DISPATCH_TN(go_atrace, s, a, st);
    } else if (phase == 1) {
        if (ns) {
            PDG_DISPATCH_TN(go_avol_ns, s, a, st);
        } else {
            PDG_DISPATCH_TN(go_avol_euler, s, a, st);
        }
    } else {
        if (!ns) return hipSuccess;
        PDG_DISPATCH_TN(go_asurf, s, a, st);
    }
    return hipGetLastError();
}

__global__ void k_axpby(int64_t n, double alpha, double *y, double beta, const double *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = alpha * y[i] + beta * x[i];
}

hipError_t launch_axpby(int64_t n, double alpha, double *y, double beta, const double *x, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, alpha, y, beta, x);
    return hipGetLastError();
}

// ----------------------------------------------------------------- objective helpers (nodal)
// transpose of the nodal evaluation: Ubar = V^T qbar (hexahedra: copy); qbar [n_elems][5][nn]
template <int T, int N>
__global__ __launch_bounds__(kBS<N>) void k_nodal_adj(StageArgs s, const double *qb, double *Ub) {
    using D = Dm<T, N>;
    constexpr int nn = D::nn, m = D::m, BS = D::BS;
    const int e = s.list[T][blockIdx.x];
    const int64_t off = s.mesh.off[e];
    const double *qe = qb + (int64_t)e * 5 * nn;
    if constexpr (T == PDG_HEX) {
        for (int t = threadIdx.x; t < 5 * nn; t += BS) Ub[off + t] = qe[t];
    } else {
        __shared__ double sq[5 * nn];
        for (int t = threadIdx.x; t < 5 * nn; t += BS) sq[t] = qe[t];
        __syncthreads();
        const double *V = s.tab[T].V;
        for (int t = threadIdx.x; t < 5 * m; t += BS) {
            const int v = t / m, j = t % m;
            double acc = 0.0;
            for (int k = 0; k < nn; ++k) acc += V[(int64_t)k * m + j] * sq[v * nn + k];
            Ub[off + t] = acc;
        }
    }
}

// quadrature weights w_k J_k at the volume nodes, [n_elems][nn] in stored element order
template <int T, int N>
__global__ __launch_bounds__(kBS<N>) void k_node_weights(StageArgs s, double *wJ) {
    using D = Dm<T, N>;
    constexpr int nn = D::nn, BS = D::BS;
    const int e = s.list[T][blockIdx.x];
    const double J = s.mesh.geo[10 * (int64_t)e];
    for (int k = threadIdx.x; k < nn; k += BS) {
        // curved elements: the Jacobian at the node
        const double Jk = s.mesh.nmet ? s.mesh.nmet[((int64_t)e * nn + k) * 10] : s.tab[T].jd[k] * J;
        wJ[(int64_t)e * nn + k] = s.tab[T].w[k] * Jk;
    }
}

template <int T, int N>
static void go_nodal_adj(const StageArgs &s, const double *qb, double *Ub, hipStream_t st) {
    hipLaunchKernelGGL((k_nodal_adj<T, N>), dim3(s.count[T]), dim3(Dm<T, N>::BS), 0, st, s, qb, Ub);
}
template <int T, int N>
static void go_node_weights(const StageArgs &s, double *wJ, hipStream_t st) {
    hipLaunchKernelGGL((k_node_weights<T, N>), dim3(s.count[T]), dim3(Dm<T, N>::BS), 0, st, s, wJ);
}

hipError_t launch_nodal_adjoint(int N, const StageArgs &s, int type, const double *qb, double *Ub, hipStream_t st) {
    if (s.count[type] == 0) return hipSuccess;
    PDG_DISPATCH_TN(go_nodal_adj, s, qb, Ub, st);
    return hipGetLastError();
}

hipError_t launch_node_weights(int N, const StageArgs &s, int type, double *wJ, hipStream_t st) {
    if (s.count[type] == 0) return hipSuccess;
    PDG_DISPATCH_TN(go_node_weights, s, wJ, st);
    return hipGetLastError();
}

}  // namespace pdg
