// Internal data structures of libpolydg (host and device views).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pdg.h"

namespace pdg {

constexpr int kMaxN = 6;
constexpr int kMaxSlots = 24;  // face sides of one element (6 faces, each up to 2 mortar halves of 2 chunks)
constexpr int kNV = 5;         // conservative variables

void set_error(const std::string &msg);

// ------------------------------------------------------------------------------------------
// host-side numerics (tables.cpp)
// ------------------------------------------------------------------------------------------
enum Rule { RULE_GL = 0, RULE_LGR = 1, RULE_LG = 2 };

void rule_nodes(int rule, int n, std::vector<double> &x, std::vector<double> &w);
// 1D Lagrange basis of nodes xn at x (out[j]) and its derivative matrix D[i][j] = l_j'(x_i)
void lagrange_values(const std::vector<double> &xn, double x, double *out);
void lagrange_derivative_matrix(const std::vector<double> &xn, std::vector<double> &D);

int n_modes(int type, int N);
int node_rule(int type, int dir);  // RULE_GL / RULE_LGR per direction
// orthonormal modal basis values at reference point eta: out[m_type]
void modal_basis(int type, int N, const double eta[3], double *out);
// reference (xi-space) corners of the degenerate hexahedron of each type
const double *ref_corner(int type, int c);
// reference map xi(eta), its Jacobian dxi/deta (col-major [c][a] = dxi_c/deta_a)
void ref_map(int type, const double eta[3], double xi[3], double dxi[9]);
// eta on face plane (axis, side) with xi(eta) = xi_target (2-D Gauss-Newton)
bool ref_inverse_on_plane(int type, int axis, int side, const double xi[3], double eta[3]);

// per-(type, N) operator tables (host copies; uploaded into one device buffer)
struct TypeTables {
    int type = 0, N = 0, n = 0, nn = 0, m = 0;  // m = stored dofs (nn for hex)
    std::vector<double> x[3], w1[3];            // 1D nodes/weights per direction
    std::vector<double> dhat[3];                // [i][l] = w_l D[l][i] / w_i per direction
    std::vector<double> dskew[3];               // [i][l] = (w_l D[l][i] - w_i D[i][l]) / w_i
    std::vector<double> dmat[3];                // [i][l] = D[i][l] = l_l'(x_i), the strong derivative
    std::vector<double> w;                      // 3-D weights [nn]
    std::vector<double> cmet;                   // reference contravariant vectors [nn][a][b]
    std::vector<double> jd;                     // reference Jacobian at nodes [nn]
    std::vector<double> V;                      // [nn][m] (modal)
    std::vector<double> VtW;                    // [m][nn] = V^T diag(w) (modal)
    std::vector<double> MVtW;                   // [m][nn] = M_D^-1 V^T diag(w) (modal)
    std::vector<double> Minv;                   // [m][m] = M_D^-1, M_D = V^T W J_D V (modal)
    std::vector<long double> xl[3];             // 1D nodes in extended precision
    std::vector<long double> Minvl;             // [m][m] = M_D^-1 (modal), extended precision
};
void build_type_tables(int type, int N, TypeTables &t);

// face kinds and points: quadrilateral, triangle, and the two n^2-point chunks of a mortar
// half's rich rule (collapsed Gauss ms x mt points, exact to total degree 3N on the half; 3N - 1
// at N = 6), so that the quadrilateral side integrates its test functions times the flux
// consistently
enum FaceKind { FACE_QUAD = 0, FACE_TRI = 1, FACE_MORTAR0 = 2, FACE_MORTAR1 = 3 };
constexpr int kFaceKinds = 4;
// canonical face points (s_p, t_p) and point weights W_kind[p] (quad: w_s w_t, triangles and
// mortar chunks: w_s w_t (1-t); padding points of the last mortar chunk carry weight 0)
void face_points(int kind, int n, std::vector<double> &s, std::vector<double> &t,
                 std::vector<double> &W);

// A trace operator: maps element dofs to the n^2 face points of one face side.
struct TraceOp {
    int type, axis, side, kind;
    int slots[3];        // corner slots holding canonical vertices A, B, C (or D)
    bool perm;           // hexahedron, points coincide with face-plane nodes
    std::vector<int> pmap;      // perm: point p -> plane node a2
    std::vector<int> inv;       // perm: plane node a2 -> point p
    std::vector<double> I;      // hex dense: [p][a2] plane-node interpolation
    std::vector<double> E;      // modal: [p][j] = phi_j(eta_p)
    std::vector<double> Et;     // modal: [j][p] = E^T
    std::vector<double> MEt;    // modal: [i][p] = (M_D^-1 E^T)
    std::vector<double> EM;     // modal: [p][i] = (E M_D^-1), the transpose of MEt
    std::vector<double> eta;    // [p][3] the face points in the element's reference cube
};
// inverse of a symmetric positive definite matrix [m][m] (Cholesky); false if not definite
bool cholesky_inverse(int m, const std::vector<long double> &A, std::vector<long double> &Ainv);
bool build_trace_op(const TypeTables &tt, TraceOp &op);

// ------------------------------------------------------------------------------------------
// device-side views passed to kernels
// ------------------------------------------------------------------------------------------
struct DevType {           // pointers into the device table buffer for one (type, N)
    const double *dhat[3];  // n*n each
    const double *dskew[3]; // n*n each: (Q^T - Q) / w_i of the split form
    const double *dmat[3];  // n*n each: D[i][l], the strong derivative of the BR1 lifting
    const double *w;        // nn
    const double *cmet;     // nn*9
    const double *V;        // nn*m
    const double *VtW;      // m*nn  V^T diag(w)
    const double *Minv;     // m*m   M_D^-1
    const double *jd;       // nn reference Jacobian at the nodes
    // modal types: the constant mode's coefficient of e_ref, c0 = e_ref / psi_0, and
    // dlt = psi_0 c0 - e_ref (psi_0 the table value of the constant mode): subtracting c0 from the
    // energy's constant-mode coefficient before V u~ or E u~ and adding dlt after gives rho E - e_ref
    double c0, dlt;
    // matrix-core row-block layouts (pack_rows): V for the modal-to-nodal product;
    // M_D^-1 V^T W (the volume part of dU~/dt comes out premultiplied) and its transpose
    // W V M_D^-1 for the adjoint; V^T and (M_D^-1)^T for the adjoint's nodal transpose
    const double *Vp, *MVtWp, *MVtWtp, *Vtp, *MinvTp;
    const double *VtWp;     // V^T W in the row-block layout (curved elements: M_e^-1 applied apart)
};

// Row-block layout for FP64 MFMA A operands: row i, k-block kb (16 columns) holds
// A[i][16 kb + 4 u + l] at [(i*KB + kb)*16 + 4 l + u] (zero past the last column), so that the
// lane reading k-offset l of row i loads its four consecutive k-steps as one 32-byte block.
std::vector<double> pack_rows(const std::vector<double> &A, int rows, int cols);

struct DevOps {            // all trace operators of one N (indexed by op id)
    const int32_t *op_type;
    const int32_t *op_plane;   // 2*axis + side
    const int32_t *op_perm;    // 1 if permutation
    const int64_t *op_off;     // offset of the op's data in `data` (doubles)
    const int64_t *op_ioff;    // offset of the op's maps in `idata` (ints)
    const int64_t *op_poff;    // modal: offset of packed E (pack_rows), packed E^T, packed
                               // M_D^-1 E^T and packed E M_D^-1 follow it
    const double *data;        // hex dense I [n2*n2] | modal E [n2*m] then E^T [m*n2]
    const int32_t *idata;      // perm maps: pmap [n2] then inv [n2]
    const double *Wq;          // [2][n2] point weights per face kind
};

struct DevMesh {
    int32_t n_elems;
    const int8_t *etype;        // [n_elems]
    const int64_t *off;         // [n_elems+1] state offsets
    const double *geo;          // [n_elems][10]: J_aff, cofT[3][3] (F^_b = sum_c cofT[b][c] F_c)
    const int32_t *slot_begin;  // [n_elems+1]
    const int32_t *slot_nbr;    // [n_slots]
    const int32_t *slot_op;     // [n_slots]
    const int32_t *slot_kind;   // [n_slots]
    const double *slot_geo;     // [n_slots][geo_pts][4]: outward unit normal, area scale
    int32_t geo_pts;            // face-geometry entries per slot: 1 (flat faces) or n^2 (curved)
    const double *nmet;         // curved meshes: [n_elems][nn][10] J and contravariant rows a^b
                                // at every volume node (the affine cofactor rows composed with
                                // the collapse, per node); null if all elements are affine
    const double *minv;         // curved meshes: per modal element its M_e^-1 = (V^T W J V)^-1,
    const int64_t *minv_off;    // [m][m] row-major at minv + minv_off[e] (Alg. 1, per element)
    // moving meshes (null otherwise): per volume node dJ/dt and the grid velocity xdot
    // [n_elems][nn][4], and per face point of every slot xdot . n_out [n_slots][geo_pts]
    const double *nmov;
    const double *gvn;
};

// face geometry (outward unit normal, area factor) of slot sl at its face point p; CV: the mesh
// has curved elements (one entry per face point), else one entry per slot
template <bool CV>
__host__ __device__ inline const double *slot_geom(const DevMesh &m, int sl, int p) {
    if constexpr (CV) return m.slot_geo + 4 * ((int64_t)sl * m.geo_pts + p);
    return m.slot_geo + 4 * (int64_t)sl;
}

// The residual kernels work on states whose energy is stored relative to a reference internal
// energy: q[4] = rho E - e_ref with e_ref = p_ref / (gamma - 1) (an exact subtraction near the
// mean state), so that p - p_ref = (gamma - 1)(q[4] - rho |u|^2 / 2) is formed without the
// rounding of the large mean pressure; p_ref = (gamma - 1) e_ref, h_ref = e_ref + p_ref.
struct Physics {
    double gamma, mu, Pr, R, p_ref, e_ref, h_ref;
};

// ------------------------------------------------------------------------------------------
// adjoint with a caller-chosen workspace (api.cpp), for the no-allocation entry point
// ------------------------------------------------------------------------------------------
// doubles of each adjoint workspace buffer: flux cotangents Lf, and for Navier-Stokes the BR1
// face-value cotangents Lw and the partial gradient Ub
void adjoint_workspace(const pdg_ctx *ctx, size_t *lf, size_t *lw, size_t *ub);
int context_device(const pdg_ctx *ctx);
// looks up the current device's static workspace of pdg_vjp_static (noalloc.hip)
int static_workspace_setup();
// pdg_vjp with the given workspace instead of the context's own
int vjp_in(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U, double *Lf, double *Lw, double *Ub);

}  // namespace pdg
