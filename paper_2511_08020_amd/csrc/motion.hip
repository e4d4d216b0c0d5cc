// Geometry of a moving mesh at one instant (gfx950, FP64).
//
// Every element corner follows x(t) = x0 + d sin(omega t) and the element moves with the
// trilinear interpolation of its corners (collapsed for prisms, pyramids and tetrahedra, whose
// reference cubes repeat corners).  The modal projection of Alg. 1 uses M = V^T W J V, which
// cannot be precomputed once the Jacobian changes in time: before each RK stage these kernels
// rebuild, at the stage's time,
//   k_move_nodes   per volume node: J and the contravariant rows a^b = x_{b+1} x x_{b+2}, dJ/dt
//                  by Jacobi's formula (sum_b xdot_{eta_b} . a^b) and the grid velocity xdot
//   k_move_faces   per face point: outward unit normal and area factor of side 0's map
//                  (negated for side 1), and the normal speed xdot . n
//   k_move_inverse per prism, pyramid and tetrahedron: M_e = V^T W J V at the stage's s (see
//                  below), then M_e^-1 into its slot, by Gauss-Jordan elimination on register
//                  tiles (symmetric positive definite: no pivoting)
// With x = x0 + s d on every corner, dx/deta is linear in s = sin(omega t), so J at each node is
// a cubic in s and M_e(s) = M0 + s M1 + s^2 M2 + s^3 M3 exactly.  When the motion is set,
//   k_move_jcoef   per volume node: the four coefficients of J(s)
//   k_move_mass    per modal element and coefficient: M_k = V^T W diag(j_k) V (matrix cores)
// build the four matrices once; every stage then takes M_e(s) by Horner's rule.
#include <cstdint>

#include "device.h"

namespace pdg {

namespace {

// corners and corner velocities of element e into LDS (24 doubles each)
__device__ __forceinline__ void load_corners(const MoveArgs &m, int e, double *X, double *V) {
    const int t = threadIdx.x;
    if (t < 24) {
        const double x0 = m.x0[24 * (int64_t)e + t], d = m.disp[24 * (int64_t)e + t];
        X[t] = x0 + m.s * d;
        V[t] = m.c * d;
    }
}

// dx/deta_b (D[b]), dxdot/deta_b (Dv[b]) and xdot of the trilinear corner map at eta
__device__ __forceinline__ void corner_map(const double *X, const double *V, const double eta[3], double D[3][3],
                                           double Dv[3][3], double xd[3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) D[b][d] = Dv[b][d] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) xd[d] = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double sg[3], f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sg[a] = ((c >> a) & 1) ? 1.0 : -1.0;
            f[a] = 0.5 * (1.0 + sg[a] * eta[a]);
        }
        const double Nc = f[0] * f[1] * f[2];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double dN = 0.5 * sg[b] * f[(b + 1) % 3] * f[(b + 2) % 3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                D[b][d] += dN * X[3 * c + d];
                Dv[b][d] += dN * V[3 * c + d];
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) xd[d] += Nc * V[3 * c + d];
    }
}

__device__ __forceinline__ void cross(const double u[3], const double v[3], double w[3]) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

}  // namespace

template <int N>
__global__ __launch_bounds__(128) void k_move_nodes(MoveArgs m) {
    constexpr int n = N + 1, nn = n * n * n;
    const int e = blockIdx.x;
    __shared__ double X[24], V[24];
    __shared__ double smet[nn * 10], smov[nn * 4];  // the element's records, stored contiguously
    load_corners(m, e, X, V);
    __syncthreads();
    const double *ex = m.eta1d + 3 * n * (int)m.etype[e];
    bool bad = false;
    for (int k = threadIdx.x; k < nn; k += blockDim.x) {
        const double eta[3] = {ex[k % n], ex[n + (k / n) % n], ex[2 * n + k / (n * n)]};
        double D[3][3], Dv[3][3], xd[3], A[3][3];
        corner_map(X, V, eta, D, Dv, xd);
#pragma unroll
        for (int b = 0; b < 3; ++b) cross(D[(b + 1) % 3], D[(b + 2) % 3], A[b]);
        const double J = D[0][0] * A[0][0] + D[0][1] * A[0][1] + D[0][2] * A[0][2];
        double Jd = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) Jd += Dv[b][0] * A[b][0] + Dv[b][1] * A[b][1] + Dv[b][2] * A[b][2];
        double *mt = smet + k * 10;
        mt[0] = J;
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int d = 0; d < 3; ++d) mt[1 + 3 * b + d] = A[b][d];
        double *mv = smov + k * 4;
        mv[0] = Jd;
        mv[1] = xd[0];
        mv[2] = xd[1];
        mv[3] = xd[2];
        if (!(J > 0.0)) bad = true;
    }
    __syncthreads();
    double *gmet = m.nmet + (int64_t)e * nn * 10, *gmov = m.nmov + (int64_t)e * nn * 4;
    for (int t = threadIdx.x; t < nn * 10; t += blockDim.x) gmet[t] = smet[t];
    for (int t = threadIdx.x; t < nn * 4; t += blockDim.x) gmov[t] = smov[t];
    if (bad) *m.bad = 1;
}

// the coefficients of J(s) = j0 + j1 s + j2 s^2 + j3 s^3 at every volume node, into m.nmov
// ([e][node][4], overwritten by the next k_move_nodes): with a_b = dx0/deta_b and
// b_b = dd/deta_b, J = det(a + s b) expands multilinearly in the three rows
template <int N>
__global__ __launch_bounds__(128) void k_move_jcoef(MoveArgs m) {
    constexpr int n = N + 1, nn = n * n * n;
    const int e = blockIdx.x;
    __shared__ double X[24], V[24];
    if (threadIdx.x < 24) {
        X[threadIdx.x] = m.x0[24 * (int64_t)e + threadIdx.x];
        V[threadIdx.x] = m.disp[24 * (int64_t)e + threadIdx.x];
    }
    __syncthreads();
    const double *ex = m.eta1d + 3 * n * (int)m.etype[e];
    for (int k = threadIdx.x; k < nn; k += blockDim.x) {
        const double eta[3] = {ex[k % n], ex[n + (k / n) % n], ex[2 * n + k / (n * n)]};
        double A[3][3], B[3][3], xd[3], w[3];
        corner_map(X, V, eta, A, B, xd);
        double j[4];
        cross(A[1], A[2], w);
        j[0] = A[0][0] * w[0] + A[0][1] * w[1] + A[0][2] * w[2];
        j[1] = B[0][0] * w[0] + B[0][1] * w[1] + B[0][2] * w[2];
        cross(B[1], A[2], w);
        j[1] += A[0][0] * w[0] + A[0][1] * w[1] + A[0][2] * w[2];
        j[2] = B[0][0] * w[0] + B[0][1] * w[1] + B[0][2] * w[2];
        cross(A[1], B[2], w);
        j[1] += A[0][0] * w[0] + A[0][1] * w[1] + A[0][2] * w[2];
        j[2] += B[0][0] * w[0] + B[0][1] * w[1] + B[0][2] * w[2];
        cross(B[1], B[2], w);
        j[2] += A[0][0] * w[0] + A[0][1] * w[1] + A[0][2] * w[2];
        j[3] = B[0][0] * w[0] + B[0][1] * w[1] + B[0][2] * w[2];
        double *jc = m.nmov + ((int64_t)e * nn + k) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) jc[q] = j[q];
    }
}

template <int N>
__global__ __launch_bounds__(64) void k_move_faces(MoveArgs m) {
    const MoveFace F = m.faces[blockIdx.x];
    __shared__ double X[24], V[24];
    load_corners(m, F.e0, X, V);
    __syncthreads();
    const int gp = m.gp;
    const double *eta0 = m.opeta + m.opeta_off[F.op0];
    // a triangle is flat: one normal (area factor |(B - A) x (C - A)| / 8, the rule's weights
    // carry the collapse)
    double nt[3] = {0.0, 0.0, 0.0}, at = 0.0;
    if (F.kind != FACE_QUAD) {
        double u[3], v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = X[3 * F.k[1] + d] - X[3 * F.k[0] + d];
            v[d] = X[3 * F.k[2] + d] - X[3 * F.k[0] + d];
        }
        cross(u, v, nt);
        const double len = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) nt[d] = F.sgn * nt[d] / len;
        at = len / 8.0;
    }
    for (int p = threadIdx.x; p < gp; p += blockDim.x) {
        const double eta[3] = {eta0[3 * p], eta0[3 * p + 1], eta0[3 * p + 2]};
        double D[3][3], Dv[3][3], xd[3], nv[3], area;
        corner_map(X, V, eta, D, Dv, xd);
        if (F.kind == FACE_QUAD) {
            // n dS = +-a^axis of the bilinear patch at the point (the rule's measure is
            // d eta_b d eta_c)
            double a[3];
            cross(D[(F.axis + 1) % 3], D[(F.axis + 2) % 3], a);
            area = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) nv[d] = F.sgn * a[d] / area;
        } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) nv[d] = nt[d];
            area = at;
        }
        const double vn = xd[0] * nv[0] + xd[1] * nv[1] + xd[2] * nv[2];
        double *g0 = m.slot_geo + 4 * ((int64_t)F.sl0 * gp + p);
        double *g1 = m.slot_geo + 4 * ((int64_t)F.sl1 * gp + p);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g0[d] = nv[d];
            g1[d] = -nv[d];
        }
        g0[3] = area;
        g1[3] = area;
        m.gvn[(int64_t)F.sl0 * gp + p] = vn;
        m.gvn[(int64_t)F.sl1 * gp + p] = -vn;
    }
}

// (V^T W) diag(J) V on the matrix cores (the packed V^T W table, zero past nn; the operand
// diag(J) V staged in LDS sixteen columns at a time, and for each column block only the row tiles
// on and above the diagonal), its upper triangle packed by rows into the element's slot of dst;
// J at node k of element e is jsrc[(e nn + k) jstride]
template <int T, int N>
__global__ __launch_bounds__(256, 3) void k_move_mass(StageArgs a, MoveArgs m, const double *jsrc, int jstride,
                                                      double *dst) {
    using D = Dm<T, N>;
    constexpr int M = D::m, nn = D::nn;
    constexpr int KBnn = (nn + 15) / 16, NCB = (M + 15) / 16;
    __shared__ double A[M * M];
    __shared__ double sj[nn];
    __shared__ double sB[16 * KBnn * 16];
    const int e = a.list[T][blockIdx.x];
    const int tid = threadIdx.x, BS = blockDim.x;
    const DevType &tab = a.tab[T];
    for (int k = tid; k < nn; k += BS) sj[k] = jsrc[((int64_t)e * nn + k) * jstride];
    for (int cb = 0; cb < NCB; ++cb) {
        __syncthreads();
        for (int t = tid; t < 16 * KBnn * 16; t += BS) {
            const int k = t >> 4, c = 16 * cb + (t & 15);
            sB[t] = (k < nn && c < M) ? sj[k] * tab.V[(int64_t)k * M + c] : 0.0;
        }
        __syncthreads();
        const int rows = M < 16 * (cb + 1) ? M : 16 * (cb + 1);
        mfma_gemm_pk(rows, KBnn, 16, [&](int i, int kb) { return tab.VtWp + ((int64_t)i * KBnn + kb) * 16; },
                     [&](int k, int c) { return sB[k * 16 + c]; },
                     [&](int i, int c, double v) {
                         if (16 * cb + c < M) A[i * M + 16 * cb + c] = v;
                     },
                     [&](int kb) { return ksteps_of(nn, kb); });
    }
    __syncthreads();
    double *Mp = dst + m.poff[e];
    for (int t = tid; t < M * M; t += BS) {
        const int i = t / M, j = t - i * M;
        if (i <= j) Mp[i * M - i * (i - 1) / 2 + (j - i)] = A[t];
    }
}

// M_e^-1 by Gauss-Jordan elimination, with the matrix in registers: M_e(s) is first evaluated
// from the packed coefficient matrices into LDS, from which the lanes take their tiles.  One
// wave per matrix
// when m <= 64 (lane l holds tile (l / NT, l % NT) of an NT x NT grid of TB x TB tiles, no
// barrier beyond the wave), else four waves, one quadrant of the grid each.  Per pivot p the
// owners publish row p and column p (double buffered in LDS) and every lane updates each entry
// of its tile with one FMA:
//   A[i][j] -= c_i w_j,  c_i = A[i][p] (t - 1 for i = p),  w_j = A[p][j] / t (1 + 1/t for j = p),
// t = A[p][p], which is the elimination step off row and column p and gives, on them,
//   A[p][j] <- A[p][j] / t,  A[i][p] <- -A[i][p] / t,  A[p][p] <- 1 / t
// (symmetric positive definite: no pivoting).  Those two forms lose no accuracy while t <= 1:
// the matrix is first scaled by the power of two that brings its largest diagonal entry into
// [1/2, 1) (every pivot, a Schur complement's diagonal entry, is at most that entry), and the
// inverse scaled back by the same power, both exactly.  The pivot loop runs over tiles at run
// time and over the rows of a tile unrolled, so a pivot's row and column are fixed registers of
// their owners; the padding past m stays exactly zero (its row and column multipliers are zero).
template <int T, int N>
constexpr int kInvThreads = Dm<T, N>::m <= 64 ? 64 : 256;

template <int T, int N>
__global__ __launch_bounds__((kInvThreads<T, N>)) void k_move_inverse(StageArgs a, MoveArgs m) {
    constexpr int M = Dm<T, N>::m;
    constexpr int Q = M <= 64 ? 1 : 2, W = Q * Q;  // quadrants per side, one wave each
    constexpr int TB = (M + 8 * Q - 1) / (8 * Q), NT = (M + TB - 1) / TB, HB = (NT + Q - 1) / Q, MP = NT * TB;
    static_assert(HB * HB <= 64, "a quadrant of tiles per wave");
    __shared__ double buf[2][2][MP];  // [pivot parity][row, column][index]
    __shared__ double wmax[W];
    __shared__ double S[M * (M + 1) / 2];
    const int e = a.list[T][blockIdx.x];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ti = (w / Q) * HB + l / HB, tj = (w % Q) * HB + l % HB;
    const bool own = l < HB * HB && ti < NT && tj < NT;
    double *Mi = m.minv + m.minv_off[e];
    {
        // M_e(s) = ((M3 s + M2) s + M1) s + M0, upper triangle packed by rows
        const double *C = m.mcoef + m.poff[e];
        const int64_t cs = m.ptot;
        const double s = m.s;
        for (int t = tid; t < M * (M + 1) / 2; t += blockDim.x)
            S[t] = fma(fma(fma(C[t + 3 * cs], s, C[t + 2 * cs]), s, C[t + cs]), s, C[t]);
    }
    __syncthreads();
    auto at = [&](int i, int j) {
        const int r = i < j ? i : j, c = i < j ? j : i;
        return S[r * M - r * (r - 1) / 2 + (c - r)];
    };
    double dm = tid < M ? at(tid, tid) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
    if (l == 0) wmax[w] = dm;
    __syncthreads();
    dm = wmax[0];
#pragma unroll
    for (int k = 1; k < W; ++k) dm = fmax(dm, wmax[k]);
    int ex;
    frexp(dm, &ex);
    const double sc = ldexp(1.0, -ex);
    double R[TB][TB];
#pragma unroll
    for (int r = 0; r < TB; ++r)
#pragma unroll
        for (int c = 0; c < TB; ++c) {
            const int i = ti * TB + r, j = tj * TB + c;
            R[r][c] = (own && i < M && j < M) ? sc * at(i, j) : 0.0;
        }
    for (int pt = 0; pt < NT; ++pt) {
#pragma unroll
        for (int pr = 0; pr < TB; ++pr) {
            const int p = pt * TB + pr;
            if (p >= M) break;
            double *rb = buf[p & 1][0], *cb = buf[p & 1][1];
            if (own && ti == pt) {
#pragma unroll
                for (int c = 0; c < TB; ++c) rb[tj * TB + c] = R[pr][c];
            }
            if (own && tj == pt) {
#pragma unroll
                for (int r = 0; r < TB; ++r) cb[ti * TB + r] = R[r][pr];
            }
            __syncthreads();
            if (own) {
                const double t = cb[p], ip = 1.0 / t;
                double cv[TB], wr[TB];
#pragma unroll
                for (int r = 0; r < TB; ++r) cv[r] = cb[ti * TB + r];
#pragma unroll
                for (int c = 0; c < TB; ++c) wr[c] = rb[tj * TB + c] * ip;
                if (ti == pt) cv[pr] = t - 1.0;
                if (tj == pt) wr[pr] = 1.0 + ip;
#pragma unroll
                for (int r = 0; r < TB; ++r)
#pragma unroll
                    for (int c = 0; c < TB; ++c) R[r][c] -= cv[r] * wr[c];
            }
        }
    }
    if (own) {
#pragma unroll
        for (int r = 0; r < TB; ++r)
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                const int i = ti * TB + r, j = tj * TB + c;
                if (i < M && j < M) Mi[(int64_t)i * M + j] = sc * R[r][c];
            }
    }
}

template <int T, int N>
static void launch_inverse(const StageArgs &a, const MoveArgs &m, hipStream_t s) {
    hipLaunchKernelGGL((k_move_inverse<T, N>), dim3(a.count[T]), dim3(kInvThreads<T, N>), 0, s, a, m);
}

template <int N>
static void go_move(const MoveArgs &m, const StageArgs &a, hipStream_t s) {
    if (m.n_elems > 0) hipLaunchKernelGGL((k_move_nodes<N>), dim3(m.n_elems), dim3(128), 0, s, m);
    if (m.n_faces > 0) hipLaunchKernelGGL((k_move_faces<N>), dim3(m.n_faces), dim3(64), 0, s, m);
    if constexpr (N <= 5) {
        if (a.count[PDG_PRISM] > 0) launch_inverse<PDG_PRISM, N>(a, m, s);
        if (a.count[PDG_PYR] > 0) launch_inverse<PDG_PYR, N>(a, m, s);
        if (a.count[PDG_TET] > 0) launch_inverse<PDG_TET, N>(a, m, s);
    }
}

template <int N>
static void go_move_coef(const MoveArgs &m, const StageArgs &a, hipStream_t s) {
    if (m.n_elems > 0) hipLaunchKernelGGL((k_move_jcoef<N>), dim3(m.n_elems), dim3(128), 0, s, m);
    if constexpr (N <= 5) {
        for (int q = 0; q < 4; ++q) {
            const double *jsrc = m.nmov + q;
            double *dst = m.mcoef + q * m.ptot;
            if (a.count[PDG_PRISM] > 0)
                hipLaunchKernelGGL((k_move_mass<PDG_PRISM, N>), dim3(a.count[PDG_PRISM]), dim3(256), 0, s, a, m, jsrc, 4,
                                   dst);
            if (a.count[PDG_PYR] > 0)
                hipLaunchKernelGGL((k_move_mass<PDG_PYR, N>), dim3(a.count[PDG_PYR]), dim3(256), 0, s, a, m, jsrc, 4, dst);
            if (a.count[PDG_TET] > 0)
                hipLaunchKernelGGL((k_move_mass<PDG_TET, N>), dim3(a.count[PDG_TET]), dim3(256), 0, s, a, m, jsrc, 4, dst);
        }
    }
}

hipError_t launch_move_mass_coefficients(int N, const MoveArgs &m, const StageArgs &a, hipStream_t s) {
    if (N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_N(go_move_coef, m, a, s);
    return hipGetLastError();
}

hipError_t launch_move_geometry(int N, const MoveArgs &m, const StageArgs &a, hipStream_t s) {
    if (N > 5) return hipErrorInvalidValue;
    PDG_DISPATCH_N(go_move, m, a, s);
    return hipGetLastError();
}

}  // namespace pdg
