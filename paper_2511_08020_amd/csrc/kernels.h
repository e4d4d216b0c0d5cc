// Launch interface of the residual kernels (kernels.hip).
#pragma once

#include "pdg_internal.h"

namespace pdg {

struct StageArgs {
    DevMesh mesh;
    DevOps ops;
    DevType tab[4];
    Physics phys;
    const int32_t *list[4];   // stored element indices per type
    int32_t count[4];
    // the same elements split by their number of face sides: at most kSlotsNarrow (narrow), or
    // more (wide); the per-type volume and surface kernels launch once for each part
    const int32_t *list_n[4], *list_w[4];
    int32_t count_n[4], count_w[4];
    const double *U;          // state (input)
    double *Tq;               // [n_slots][5][n2] state traces
    double *Fvn;              // [n_slots][5][n2] viscous normal flux traces (NS)
    double *Rp;               // partial residual (volume part), state layout
    // surface phase output: mode 0 writes dU/dt to `out`; mode 1 updates K and U in place
    int mode;
    double *out;
    double *K;
    double *Uw;
    double rk_a, rk_bdt;
    // work-queue schedule: workgroups serving each queue in the launch at hand (queue
    // q = blockIdx.x / qsub); set per phase
    int32_t qsub;
};

// phases of one residual evaluation; all launch one workgroup per element of each type
hipError_t launch_trace(int N, const StageArgs &a, int type, hipStream_t s);
hipError_t launch_volume(int N, bool ns, const StageArgs &a, int type, hipStream_t s);
hipError_t launch_surface(int N, bool ns, const StageArgs &a, int type, hipStream_t s);

// resident workgroups per CU of the work-queue kernel of a phase (0 trace, 1 volume, 2 surface;
// sizes that phase's workgroups per queue)
int queue_occupancy(int N, bool ns, int phase);

// smallest index of a non-finite entry of U[0..n) into *first (device; initialised by the caller
// to n) (check.hip)
hipError_t launch_first_nonfinite(const double *U, int64_t n, unsigned long long *first, hipStream_t s);

// volume phase in the entropy-stable split form (split.hip): per-type and work-queue launches
hipError_t launch_volume_split(int N, bool ns, const StageArgs &a, int type, hipStream_t s);
hipError_t launch_volume_split_queues(int N, bool ns, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                                      hipStream_t s);
// surface phase with the entropy-conservative two-point flux (split.hip)
hipError_t launch_surface_ec(int N, bool ns, const StageArgs &a, int type, hipStream_t s);
hipError_t launch_surface_ec_queues(int N, bool ns, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                                    hipStream_t s);

// work-queue schedule: one workgroup per queue over the elements [qb[q], qb[q+1]) of any type,
// taken type by type: qtb[4 j + t] is the index into list[t] of the first type-t element at or
// after qb[j] (j = 0..nq); phase 0 trace, 1 volume, 2 surface; each queue adds its wall-clock
// ticks to qt[q] (if not null)
hipError_t launch_queues(int N, bool ns, int phase, const StageArgs &a, const int32_t *qtb, int nq, uint64_t *qt,
                         hipStream_t s);

// Adjoint (vector-Jacobian product of the residual).  The cotangent of dU/dt is
// lam = Kb + c * Ubr (Ubr may be null).  Output mode 0 writes grad = (dR/dU)^T lam to `gout`;
// mode 1 is the reverse LSERK stage tail: Ubar += grad and Kbar = a * lam (Kbar may alias Kb
// and Ubar may alias Ubr: every entry is read and written by the same thread).
struct AdjArgs {
    const double *Kb;
    const double *Ubr;
    double c;
    double *Lf;   // [n_slots][5][n2] cotangent of each side's face flux, -ws E mu
    double *Lw;   // [n_slots][4][n2] NS: cotangent of the BR1 face values (w_own + w_nbr)/2
    double *Ub;   // NS: partial result of the volume phase (state layout)
    int mode;
    double *gout;
    double *Ubar;
    double *Kbar;
    double a;
};
// phase 0: state traces (Tq) and flux cotangents (Lf); phase 1: volume adjoint (Euler: final
// output; NS: Ub and Lw); phase 2 (NS): BR1 face-value adjoint and final output
hipError_t launch_adjoint(int N, bool ns, int phase, const StageArgs &s, const AdjArgs &a, int type,
                          hipStream_t st);
// elementwise y = alpha * y + beta * x over n doubles
hipError_t launch_axpby(int64_t n, double alpha, double *y, double beta, const double *x, hipStream_t st);

// transpose of the nodal evaluation, and the nodal quadrature weights w_k J_k
hipError_t launch_nodal_adjoint(int N, const StageArgs &s, int type, const double *qb, double *Ub, hipStream_t st);
hipError_t launch_node_weights(int N, const StageArgs &s, int type, double *wJ, hipStream_t st);

// utilities
hipError_t launch_project(int N, const StageArgs &a, int type, const double *q, double *U,
                          hipStream_t s);
hipError_t launch_nodal(int N, const StageArgs &a, int type, const double *U, double *q,
                        hipStream_t s);
hipError_t launch_sfc_keys(int n, const double *centroid, const double lo[3], double scale,
                           uint64_t *keys, hipStream_t s);
hipError_t launch_type_weights(int n, const int8_t *etype, const uint32_t wt[4], uint32_t *weight, hipStream_t s);
hipError_t launch_partition(int n, const uint32_t *w, int nq, int32_t *qb, uint64_t *scratch,
                            hipStream_t s);

// ------------------------------------------------------------------------ moving meshes
// A face of a moving mesh, seen from its side 0: the slots of both sides, side 0's stored
// element, the trace operator whose points (reference coordinates in side 0's cube) are the
// face points, the face kind, the plane's axis, the orientation sign (quadrilaterals:
// n_out = sgn a^axis / |a^axis|; triangles: n_out = sgn (B - A) x (C - A) / |...| with A, B, C
// side 0's corner slots k[0..2])
struct MoveFace {
    int32_t sl0, sl1, e0, op0;
    int32_t kind, axis;
    int32_t k[3];
    double sgn;
};

struct MoveArgs {
    int32_t n_elems, n_faces, gp;
    const double *x0, *disp;    // [n_elems][8][3] corners at t = 0 and their displacement d
    double s, c;                // sin(omega t), omega cos(omega t): x = x0 + s d, xdot = c d
    const double *eta1d;        // [4][3][n] 1-D node coordinates per type and direction
    const int8_t *etype;
    const MoveFace *faces;
    const double *opeta;        // face points of each trace operator [gp][3] ...
    const int64_t *opeta_off;   // ... at opeta + opeta_off[op]
    double *nmet, *nmov, *slot_geo, *gvn, *minv;
    const int64_t *minv_off;
    double *mcoef;              // [4][ptot]: M_e(s) = sum_q s^q M_q, each M_q's upper triangle
    const int64_t *poff;        // packed by rows (m (m + 1) / 2 entries) at poff[e] in each
    int64_t ptot;
    int32_t *bad;               // set to 1 where a Jacobian is not positive
};

// the geometry of a moving mesh at one instant: per-node metrics, dJ/dt and grid velocity,
// per-face-point normals, areas and normal speeds, and every modal element's M_e^-1
hipError_t launch_move_geometry(int N, const MoveArgs &m, const StageArgs &a, hipStream_t s);

// the coefficient matrices M_q of M_e(s) for the motion's displacements (uses nmov as scratch)
hipError_t launch_move_mass_coefficients(int N, const MoveArgs &m, const StageArgs &a, hipStream_t s);

}  // namespace pdg
