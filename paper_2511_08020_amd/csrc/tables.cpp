// Host-side operator tables: 1D rules, Lagrange operators, orthonormal collapsed bases,
// reference maps, per-(type, N) volume tables and face trace operators.
//
// Node family (Sec. 2: element-local polynomials of degree N on a tensor-product node set):
// Gauss-Lobatto in directions that do not collapse, left Gauss-Radau (contains -1, omits the
// collapsed end +1) in directions that do, so every node has a positive Jacobian.
// Modal basis (Algorithm 1, generalised Vandermonde V = phi(xi)): collapsed Jacobi products,
// orthonormal on the reference element; normalisation constants in closed form from
//   int_{-1}^{1} (1-x)^a (P_n^(a,0)(x))^2 dx = 2^(a+1) / (2n + a + 1).
// All tables are computed in extended precision (x86 long double) and rounded once to FP64:
// the residual cancels large pressure terms, so table rounding is amplified in the result.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pdg_internal.h"

namespace pdg {

using ld = long double;

static std::vector<double> to_double(const std::vector<ld> &v) { return std::vector<double>(v.begin(), v.end()); }

// ---------------------------------------------------------------------------- 1D polynomials
static void legendre_with_derivative(int n, ld x, ld &p, ld &dp, ld &pm1) {
    // P_n(x), P_n'(x), P_{n-1}(x) by the three-term recurrence
    ld p0 = 1, p1 = x, d0 = 0, d1 = 1;
    if (n == 0) { p = 1; dp = 0; pm1 = 0; return; }
    for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        ld d2 = d0 + (2 * k + 1) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    p = p1; dp = d1; pm1 = p0;
}

static ld legendre_value(int n, ld x) {
    ld p, dp, pm1;
    legendre_with_derivative(n, x, p, dp, pm1);
    return p;
}

static void rule_nodes_ld(int rule, int n, std::vector<ld> &x, std::vector<ld> &w) {
    x.assign(n, 0);
    w.assign(n, 0);
    const ld pi = 3.141592653589793238462643383279502884L;
    const ld tol = 1e-19L;
    if (rule == RULE_GL) {
        int N = n - 1;
        x[0] = -1; x[N] = 1;
        for (int i = 1; i < N; ++i) {
            ld xi = -std::cos(pi * i / N);
            for (int it = 0; it < 100; ++it) {
                // interior Lobatto nodes are the roots of P_{N+1} - P_{N-1}; its derivative is (2N+1) P_N
                ld pN1, dN1, pN;
                legendre_with_derivative(N + 1, xi, pN1, dN1, pN);
                ld dx = (pN1 - legendre_value(N - 1, xi)) / ((2 * N + 1) * pN);
                xi -= dx;
                if (std::fabs(dx) < tol) break;
            }
            x[i] = xi;
        }
        for (int i = 0; i < n; ++i) {
            ld pN = legendre_value(N, x[i]);
            w[i] = 2 / (N * (N + 1) * pN * pN);
        }
    } else if (rule == RULE_LGR) {
        x[0] = -1;
        for (int i = 1; i < n; ++i) {
            ld xi = -std::cos(2 * pi * i / (2 * n - 1));
            for (int it = 0; it < 100; ++it) {
                // nodes other than -1 are the roots of P_{n-1} + P_n
                ld pn, dpn, pnm1, q, dq, qm1;
                legendre_with_derivative(n, xi, pn, dpn, pnm1);
                legendre_with_derivative(n - 1, xi, q, dq, qm1);
                ld dx = (pn + q) / (dpn + dq);
                xi -= dx;
                if (std::fabs(dx) < tol) break;
            }
            x[i] = xi;
        }
        w[0] = (ld)2 / ((ld)n * n);
        for (int i = 1; i < n; ++i) {
            ld pm = legendre_value(n - 1, x[i]);
            w[i] = (1 - x[i]) / ((ld)n * n * pm * pm);
        }
    } else {
        for (int i = 0; i < n; ++i) {
            ld xi = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
            ld p, dp = 1, pm1;
            for (int it = 0; it < 100; ++it) {
                legendre_with_derivative(n, xi, p, dp, pm1);
                ld dx = p / dp;
                xi -= dx;
                if (std::fabs(dx) < tol) break;
            }
            legendre_with_derivative(n, xi, p, dp, pm1);
            x[i] = xi;
            w[i] = 2 / ((1 - xi * xi) * dp * dp);
        }
    }
}

void rule_nodes(int rule, int n, std::vector<double> &x, std::vector<double> &w) {
    std::vector<ld> xl, wl;
    rule_nodes_ld(rule, n, xl, wl);
    x = to_double(xl);
    w = to_double(wl);
}

static void lagrange_values_ld(const std::vector<ld> &xn, ld x, ld *out) {
    const int n = (int)xn.size();
    for (int j = 0; j < n; ++j) {
        ld v = 1;
        for (int m = 0; m < n; ++m)
            if (m != j) v *= (x - xn[m]) / (xn[j] - xn[m]);
        out[j] = v;
    }
}

void lagrange_values(const std::vector<double> &xn, double x, double *out) {
    std::vector<ld> xl(xn.begin(), xn.end()), o(xn.size());
    lagrange_values_ld(xl, x, o.data());
    for (size_t j = 0; j < xn.size(); ++j) out[j] = (double)o[j];
}

static void lagrange_derivative_matrix_ld(const std::vector<ld> &xn, std::vector<ld> &D) {
    // barycentric form: D_ij = (lam_j / lam_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij
    const int n = (int)xn.size();
    std::vector<ld> lam(n, 1);
    for (int j = 0; j < n; ++j)
        for (int m = 0; m < n; ++m)
            if (m != j) lam[j] /= (xn[j] - xn[m]);
    D.assign(n * n, 0);
    for (int i = 0; i < n; ++i) {
        ld s = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i * n + j] = (lam[j] / lam[i]) / (xn[i] - xn[j]);
            s += D[i * n + j];
        }
        D[i * n + i] = -s;
    }
}

void lagrange_derivative_matrix(const std::vector<double> &xn, std::vector<double> &D) {
    std::vector<ld> xl(xn.begin(), xn.end()), Dl;
    lagrange_derivative_matrix_ld(xl, Dl);
    D = to_double(Dl);
}

// ---------------------------------------------------------------------------- modal bases
static ld jacobi(int n, ld a, ld x) {
    // P_n^(a,0)(x) by the three-term recurrence
    if (n == 0) return 1;
    ld p0 = 1, p1 = ((a + 2) * x + a) / 2;
    for (int k = 2; k <= n; ++k) {
        ld c = 2 * k + a;
        ld a1 = 2 * k * (k + a) * (c - 2);
        ld a2 = (c - 1) * (c * (c - 2) * x + a * a);
        ld a3 = 2 * (k + a - 1) * (k - 1) * c;
        ld p2 = (a2 * p1 - a3 * p0) / a1;
        p0 = p1; p1 = p2;
    }
    return p1;
}

static ld ipow(ld x, int k) {
    ld r = 1;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

int n_modes(int type, int N) {
    int n = N + 1;
    switch (type) {
        case PDG_HEX: return n * n * n;
        case PDG_PRISM: return n * n * (n + 1) / 2;
        case PDG_PYR: return n * (n + 1) * (2 * n + 1) / 6;
        case PDG_TET: return n * (n + 1) * (n + 2) / 6;
    }
    return 0;
}

static void modal_basis_ld(int type, int N, const ld eta[3], ld *out) {
    const ld a = eta[0], b = eta[1], c = eta[2];
    const ld hb = (1 - b) / 2, hc = (1 - c) / 2;
    int j = 0;
    if (type == PDG_TET) {
        for (int p = 0; p <= N; ++p)
            for (int q = 0; q <= N - p; ++q)
                for (int r = 0; r <= N - p - q; ++r) {
                    ld nrm2 = (ld)2 / (2 * p + 1) * ((ld)1 / (p + q + 1)) * (ld)2 / (2 * (p + q + r) + 3);
                    ld v = jacobi(p, 0, a) * ipow(hb, p) * jacobi(q, 2 * p + 1, b) * ipow(hc, p + q) *
                           jacobi(r, 2 * (p + q) + 2, c);
                    out[j++] = v / std::sqrt(nrm2);
                }
    } else if (type == PDG_PRISM) {
        for (int p = 0; p <= N; ++p)
            for (int q = 0; q <= N; ++q)
                for (int r = 0; r <= N - p; ++r) {
                    ld nrm2 = (ld)2 / (2 * p + 1) * (ld)2 / (2 * q + 1) * ((ld)1 / (p + r + 1));
                    ld v = jacobi(p, 0, a) * jacobi(q, 0, b) * ipow(hc, p) * jacobi(r, 2 * p + 1, c);
                    out[j++] = v / std::sqrt(nrm2);
                }
    } else if (type == PDG_PYR) {
        for (int p = 0; p <= N; ++p)
            for (int q = 0; q <= N; ++q) {
                int mx = std::max(p, q);
                for (int r = 0; r <= N - mx; ++r) {
                    ld nrm2 = (ld)2 / (2 * p + 1) * (ld)2 / (2 * q + 1) * (ld)2 / (2 * (mx + r) + 3);
                    ld v = jacobi(p, 0, a) * jacobi(q, 0, b) * ipow(hc, mx) * jacobi(r, 2 * mx + 2, c);
                    out[j++] = v / std::sqrt(nrm2);
                }
            }
    }
}

void modal_basis(int type, int N, const double eta[3], double *out) {
    const ld e[3] = {eta[0], eta[1], eta[2]};
    std::vector<ld> o(n_modes(type, N));
    modal_basis_ld(type, N, e, o.data());
    for (size_t j = 0; j < o.size(); ++j) out[j] = (double)o[j];
}

// ---------------------------------------------------------------------------- reference maps
static const double kRef[4][8][3] = {
    // hex: the cube itself
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}, {1, 1, 1}},
    // prism (v0, v1, v3, v4, v2, v2, v5, v5)
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {-1, -1, 1}, {-1, 1, 1}, {-1, 1, 1}},
    // pyramid (b0, b1, b2, b3, apex x4)
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {-1, -1, 1}, {-1, -1, 1}, {-1, -1, 1}},
    // tet (v0, v1, v2, v2, v3 x4)
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, 1, -1}, {-1, -1, 1}, {-1, -1, 1}, {-1, -1, 1}, {-1, -1, 1}},
};

const double *ref_corner(int type, int c) { return kRef[type][c]; }

int node_rule(int type, int dir) {
    if (type == PDG_HEX) return RULE_GL;
    if (type == PDG_TET) return dir == 0 ? RULE_GL : RULE_LGR;
    return dir == 2 ? RULE_LGR : RULE_GL;  // prism, pyramid collapse in eta3
}

static void ref_map_ld(int type, const ld eta[3], ld xi[3], ld dxi[9]) {
    for (int c = 0; c < 3; ++c) xi[c] = 0;
    for (int k = 0; k < 9; ++k) dxi[k] = 0;
    for (int corner = 0; corner < 8; ++corner) {
        ld f[3], df[3];
        for (int a = 0; a < 3; ++a) {
            ld s = ((corner >> a) & 1) ? 1 : -1;
            f[a] = (1 + s * eta[a]) / 2;
            df[a] = s / 2;
        }
        ld N = f[0] * f[1] * f[2];
        ld dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
        for (int c = 0; c < 3; ++c) {
            xi[c] += N * kRef[type][corner][c];
            for (int a = 0; a < 3; ++a) dxi[c * 3 + a] += dN[a] * kRef[type][corner][c];
        }
    }
}

void ref_map(int type, const double eta[3], double xi[3], double dxi[9]) {
    const ld e[3] = {eta[0], eta[1], eta[2]};
    ld x[3], d[9];
    ref_map_ld(type, e, x, d);
    for (int c = 0; c < 3; ++c) xi[c] = (double)x[c];
    for (int k = 0; k < 9; ++k) dxi[k] = (double)d[k];
}

static bool ref_inverse_on_plane_ld(int type, int axis, int side, const ld xt[3], ld eta[3]) {
    int b = (axis + 1) % 3, c = (axis + 2) % 3;
    if (b > c) std::swap(b, c);
    eta[axis] = side ? 1 : -1;
    eta[b] = 0;
    eta[c] = 0;
    for (int it = 0; it < 200; ++it) {
        ld xi[3], J[9];
        ref_map_ld(type, eta, xi, J);
        ld r[3] = {xi[0] - xt[0], xi[1] - xt[1], xi[2] - xt[2]};
        // normal equations of the 3x2 system [dxi/deta_b, dxi/deta_c] d = r
        ld A00 = 0, A01 = 0, A11 = 0, g0 = 0, g1 = 0;
        for (int k = 0; k < 3; ++k) {
            ld jb = J[k * 3 + b], jc = J[k * 3 + c];
            A00 += jb * jb; A01 += jb * jc; A11 += jc * jc;
            g0 += jb * r[k]; g1 += jc * r[k];
        }
        ld det = A00 * A11 - A01 * A01;
        if (!(std::fabs(det) > 0)) return false;
        ld d0 = (A11 * g0 - A01 * g1) / det, d1 = (A00 * g1 - A01 * g0) / det;
        eta[b] -= d0;
        eta[c] -= d1;
        if (std::fabs(d0) + std::fabs(d1) < 1e-19L) break;
    }
    ld xi[3], J[9];
    ref_map_ld(type, eta, xi, J);
    ld err = std::fabs(xi[0] - xt[0]) + std::fabs(xi[1] - xt[1]) + std::fabs(xi[2] - xt[2]);
    return err < 1e-15L;
}

bool ref_inverse_on_plane(int type, int axis, int side, const double xt[3], double eta[3]) {
    const ld x[3] = {xt[0], xt[1], xt[2]};
    ld e[3];
    bool ok = ref_inverse_on_plane_ld(type, axis, side, x, e);
    for (int a = 0; a < 3; ++a) eta[a] = (double)e[a];
    return ok;
}

// ---------------------------------------------------------------------------- dense helpers
bool cholesky_inverse(int m, const std::vector<ld> &A, std::vector<ld> &Ainv) {
    std::vector<ld> L(m * m, 0);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j <= i; ++j) {
            ld s = A[i * m + j];
            for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
            if (i == j) {
                if (!(s > 0)) return false;
                L[i * m + i] = std::sqrt(s);
            } else {
                L[i * m + j] = s / L[j * m + j];
            }
        }
    Ainv.assign(m * m, 0);
    std::vector<ld> col(m);
    for (int e = 0; e < m; ++e) {
        // solve L y = e_e, then L^T x = y
        for (int i = 0; i < m; ++i) {
            ld s = (i == e) ? 1 : 0;
            for (int k = 0; k < i; ++k) s -= L[i * m + k] * col[k];
            col[i] = s / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            ld s = col[i];
            for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * col[k];
            col[i] = s / L[i * m + i];
        }
        for (int i = 0; i < m; ++i) Ainv[i * m + e] = col[i];
    }
    return true;
}

void build_type_tables(int type, int N, TypeTables &t) {
    t.type = type; t.N = N; t.n = N + 1;
    const int n = t.n;
    t.nn = n * n * n;
    t.m = n_modes(type, N);
    std::vector<ld> xl[3], wl[3];
    for (int a = 0; a < 3; ++a) {
        rule_nodes_ld(node_rule(type, a), n, xl[a], wl[a]);
        t.xl[a] = xl[a];
        t.x[a] = to_double(xl[a]);
        t.w1[a] = to_double(wl[a]);
        std::vector<ld> D;
        lagrange_derivative_matrix_ld(xl[a], D);
        t.dhat[a].assign(n * n, 0.0);
        t.dskew[a].assign(n * n, 0.0);
        t.dmat[a].assign(n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int l = 0; l < n; ++l) {
                t.dmat[a][i * n + l] = (double)D[i * n + l];
                t.dhat[a][i * n + l] = (double)(wl[a][l] * D[l * n + i] / wl[a][i]);
                t.dskew[a][i * n + l] = (double)((wl[a][l] * D[l * n + i] - wl[a][i] * D[i * n + l]) / wl[a][i]);
            }
    }
    std::vector<ld> w(t.nn), jd(t.nn);
    t.w.resize(t.nn);
    t.cmet.resize(t.nn * 9);
    t.jd.resize(t.nn);
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int k = i + n * (j + n * l);
                w[k] = wl[0][i] * wl[1][j] * wl[2][l];
                t.w[k] = (double)w[k];
                ld eta[3] = {xl[0][i], xl[1][j], xl[2][l]}, xi[3], J[9];
                ref_map_ld(type, eta, xi, J);
                // columns dxi/deta_a; c^a = col(a+1) x col(a+2)
                ld cm[9];
                for (int a = 0; a < 3; ++a) {
                    int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
                    ld u[3] = {J[0 * 3 + a1], J[1 * 3 + a1], J[2 * 3 + a1]};
                    ld v[3] = {J[0 * 3 + a2], J[1 * 3 + a2], J[2 * 3 + a2]};
                    cm[a * 3 + 0] = u[1] * v[2] - u[2] * v[1];
                    cm[a * 3 + 1] = u[2] * v[0] - u[0] * v[2];
                    cm[a * 3 + 2] = u[0] * v[1] - u[1] * v[0];
                }
                for (int q = 0; q < 9; ++q) t.cmet[k * 9 + q] = (double)cm[q];
                jd[k] = J[0] * cm[0] + J[3] * cm[1] + J[6] * cm[2];
                t.jd[k] = (double)jd[k];
            }
    if (type == PDG_HEX) return;
    const int m = t.m, nn = t.nn;
    std::vector<ld> V(nn * m);
    t.V.resize(nn * m);
    for (int k = 0; k < nn; ++k) {
        int i = k % n, j = (k / n) % n, l = k / (n * n);
        ld eta[3] = {xl[0][i], xl[1][j], xl[2][l]};
        modal_basis_ld(type, N, eta, &V[k * m]);
    }
    t.V = to_double(V);
    std::vector<ld> M(m * m, 0);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            ld s = 0;
            for (int k = 0; k < nn; ++k) s += V[k * m + a] * w[k] * jd[k] * V[k * m + b];
            M[a * m + b] = s;
        }
    cholesky_inverse(m, M, t.Minvl);
    t.Minv = to_double(t.Minvl);
    t.VtW.assign(m * nn, 0.0);
    for (int a = 0; a < m; ++a)
        for (int k = 0; k < nn; ++k) t.VtW[a * nn + k] = (double)(V[k * m + a] * w[k]);
    // M_D^-1 V^T W, the volume projection premultiplied by the reference mass-matrix inverse
    t.MVtW.assign(m * nn, 0.0);
    for (int a = 0; a < m; ++a)
        for (int k = 0; k < nn; ++k) {
            ld acc = 0;
            for (int b = 0; b < m; ++b) acc += t.Minvl[a * m + b] * V[k * m + b];
            t.MVtW[a * nn + k] = (double)(acc * w[k]);
        }
}

// ---------------------------------------------------------------------------- face operators
// Gauss-Legendre points (ms in s, mt in t) of a mortar half: the fewest whose collapsed product
// rule integrates total degree D = 3N (D = 3N - 1 at N = 6) exactly: s-degree D, t-degree D + 1
// with the collapse factor; ms mt <= 2 n^2 fills two chunks of n^2 points
static void mortar_rule_size(int n, int &ms, int &mt) {
    const int N = n - 1, D = N <= 5 ? 3 * N : 3 * N - 1;
    ms = (D + 2) / 2;
    mt = (D + 3) / 2;
}

static void face_points_ld(int kind, int n, std::vector<ld> &s, std::vector<ld> &t, std::vector<ld> &W) {
    std::vector<ld> x, w;
    if (kind == FACE_MORTAR0 || kind == FACE_MORTAR1) {
        int ms, mt;
        mortar_rule_size(n, ms, mt);
        std::vector<ld> xs, ws, xt, wt;
        rule_nodes_ld(RULE_LG, ms, xs, ws);
        rule_nodes_ld(RULE_LG, mt, xt, wt);
        const int n2 = n * n, c0 = (kind - FACE_MORTAR0) * n2;
        s.assign(n2, 0); t.assign(n2, 0); W.assign(n2, 0);  // padding: the half's centre, weight 0
        for (int p = 0; p < n2; ++p) {
            const int q = c0 + p;  // point q = is + ms it of the ms x mt rule
            if (q >= ms * mt) break;
            const int is = q % ms, it = q / ms;
            s[p] = xs[is]; t[p] = xt[it];
            W[p] = ws[is] * wt[it] * (1 - xt[it]);
        }
        return;
    }
    rule_nodes_ld(kind == FACE_QUAD ? RULE_GL : RULE_LG, n, x, w);
    s.resize(n * n); t.resize(n * n); W.resize(n * n);
    for (int it = 0; it < n; ++it)
        for (int is = 0; is < n; ++is) {
            int p = is + n * it;
            s[p] = x[is]; t[p] = x[it];
            W[p] = w[is] * w[it] * (kind == FACE_QUAD ? (ld)1 : (1 - x[it]));
        }
}

void face_points(int kind, int n, std::vector<double> &s, std::vector<double> &t, std::vector<double> &W) {
    std::vector<ld> sl, tl, Wl;
    face_points_ld(kind, n, sl, tl, Wl);
    s = to_double(sl); t = to_double(tl); W = to_double(Wl);
}

bool build_trace_op(const TypeTables &tt, TraceOp &op) {
    const int n = tt.n, n2 = n * n, m = tt.m;
    std::vector<ld> s, t, W;
    face_points_ld(op.kind, n, s, t, W);
    const double *XA = ref_corner(op.type, op.slots[0]);
    const double *XB = ref_corner(op.type, op.slots[1]);
    const double *XC = ref_corner(op.type, op.slots[2]);
    int b = (op.axis + 1) % 3, c = (op.axis + 2) % 3;
    if (b > c) std::swap(b, c);
    std::vector<ld> eta(n2 * 3);
    op.eta.assign(n2 * 3, 0.0);
    for (int p = 0; p < n2; ++p) {
        ld xi[3];
        for (int d = 0; d < 3; ++d) {
            if (op.kind == FACE_QUAD)
                xi[d] = XA[d] + (1 + s[p]) / 2 * (XB[d] - XA[d]) + (1 + t[p]) / 2 * (XC[d] - XA[d]);
            else
                xi[d] = (1 - s[p]) * (1 - t[p]) / 4 * XA[d] + (1 + s[p]) * (1 - t[p]) / 4 * XB[d] +
                        (1 + t[p]) / 2 * XC[d];
        }
        if (!ref_inverse_on_plane_ld(op.type, op.axis, op.side, xi, &eta[p * 3])) return false;
        for (int d = 0; d < 3; ++d) op.eta[p * 3 + d] = (double)eta[p * 3 + d];
    }
    if (op.type == PDG_HEX) {
        // plane nodes a2 = i_b + n i_c; interpolation by tensor Lagrange in (eta_b, eta_c)
        op.I.assign(n2 * n2, 0.0);
        std::vector<ld> lb(n), lc(n);
        op.perm = true;
        op.pmap.assign(n2, -1);
        op.inv.assign(n2, -1);
        for (int p = 0; p < n2; ++p) {
            lagrange_values_ld(tt.xl[b], eta[p * 3 + b], lb.data());
            lagrange_values_ld(tt.xl[c], eta[p * 3 + c], lc.data());
            for (int ic = 0; ic < n; ++ic)
                for (int ib = 0; ib < n; ++ib) op.I[p * n2 + ib + n * ic] = (double)(lb[ib] * lc[ic]);
            int hit_b = -1, hit_c = -1;
            for (int i = 0; i < n; ++i) {
                if (std::fabs(eta[p * 3 + b] - tt.xl[b][i]) < 1e-15L) hit_b = i;
                if (std::fabs(eta[p * 3 + c] - tt.xl[c][i]) < 1e-15L) hit_c = i;
            }
            if (hit_b < 0 || hit_c < 0) {
                op.perm = false;
            } else {
                op.pmap[p] = hit_b + n * hit_c;
            }
        }
        if (op.perm) {
            for (int p = 0; p < n2; ++p) {
                if (op.inv[op.pmap[p]] >= 0) { op.perm = false; break; }
                op.inv[op.pmap[p]] = p;
            }
        }
        if (!op.perm) { op.pmap.clear(); op.inv.clear(); }
        return true;
    }
    op.perm = false;
    std::vector<ld> E(n2 * m);
    for (int p = 0; p < n2; ++p) modal_basis_ld(op.type, tt.N, &eta[p * 3], &E[p * m]);
    op.E = to_double(E);
    // M_D^-1 E^T, the lift premultiplied by the reference mass-matrix inverse, and its
    // transpose E M_D^-1 (M_D is symmetric) for the adjoint
    op.MEt.assign(m * n2, 0.0);
    op.EM.assign(n2 * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int p = 0; p < n2; ++p) {
            ld acc = 0;
            for (int j = 0; j < m; ++j) acc += tt.Minvl[i * m + j] * E[p * m + j];
            op.MEt[i * n2 + p] = (double)acc;
            op.EM[p * m + i] = (double)acc;
        }
    op.Et.assign(m * n2, 0.0);
    for (int j = 0; j < m; ++j)
        for (int p = 0; p < n2; ++p) op.Et[j * n2 + p] = op.E[p * m + j];
    return true;
}

std::vector<double> pack_rows(const std::vector<double> &A, int rows, int cols) {
    const int KB = (cols + 15) / 16;
    std::vector<double> P((size_t)rows * KB * 16, 0.0);
    for (int i = 0; i < rows; ++i)
        for (int kb = 0; kb < KB; ++kb)
            for (int l = 0; l < 4; ++l)
                for (int u = 0; u < 4; ++u) {
                    const int k = 16 * kb + 4 * u + l;
                    if (k < cols) P[((size_t)i * KB + kb) * 16 + 4 * l + u] = A[(size_t)i * cols + k];
                }
    return P;
}

}  // namespace pdg
