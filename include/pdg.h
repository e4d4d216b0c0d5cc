/*
 * pdg.h -- C ABI of libpolydg: the per-stage residual R(U) of modal-time-stepping DGSEM on
 * mixed hexahedral / prismatic / pyramidal / tetrahedral meshes, its LSERK4 time integration,
 * its vector-Jacobian product, and the Hilbert-curve ordering and cost-weighted partition
 * of the elements into work queues.
 *
 * Method (Kopper et al., "In-Memory Load Balancing for Discontinuous Galerkin Methods on
 * Polytopal Meshes", arXiv:2511.08020):
 *   - weak form of the compressible Euler / Navier-Stokes-Fourier equations, Sec. 2, Eq. (1);
 *   - collapsed-coordinate (Duffy) elements, Sec. 2;
 *   - modal time stepping of the non-hexahedral elements, Sec. 2, Algorithm 1;
 *   - low-storage explicit Runge-Kutta integration, Sec. 2 (method of lines);
 *   - Hilbert space-filling-curve ordering and contiguous segments, Sec. 3, Fig. 1;
 *   - loop timers attributed to elements, Sec. 3, Listing 1.
 *
 * Conventions shared by every call:
 *   - Every call returns PDG_OK (0) or a negative PDG_E* code; pdg_last_error() then holds a
 *     thread-local message.  No exception or abort crosses the ABI.
 *   - "device" pointers are HIP device memory (e.g. torch tensor data pointers); "host"
 *     pointers are ordinary CPU memory.  The caller owns every buffer it passes; the library
 *     owns its context (tables, geometry, face lists, scratch) and frees it in pdg_destroy.
 *   - Device work is enqueued asynchronously on the HIP stream given at creation, unless the
 *     call is documented as synchronous.
 *   - Floating point is IEEE binary64 throughout.
 *
 * State layout (reported by pdg_layout): elements in Hilbert-curve order; element i owns the
 * doubles [elem_offset[i], elem_offset[i+1]) of U, shaped [5][ndof] (variable-major, variables
 * rho, rho u, rho v, rho w, rho E).  Hexahedra store ndof = (N+1)^3 nodal values at the
 * Gauss-Lobatto^3 volume nodes; prisms, pyramids and tetrahedra store the ndof modal
 * coefficients of their orthonormal collapsed Jacobi basis (modes (p,q,r) with p outermost and
 * r fastest; unit norm on the reference element).  Volume nodes k = i + n*j + n*n*l, n = N+1.
 */
#ifndef PDG_H
#define PDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdg_ctx pdg_ctx;     /* opaque, library-owned */
typedef struct pdg_batch pdg_batch; /* opaque, library-owned; refers to contexts it does not own */

enum { PDG_HEX = 0, PDG_PRISM = 1, PDG_PYR = 2, PDG_TET = 3 };
enum { PDG_OK = 0, PDG_EINVAL = -1, PDG_ENOMEM = -2, PDG_EHIP = -3, PDG_EMESH = -4,
       PDG_ENOTSUP = -5, PDG_ENONFINITE = -6 };
enum { PDG_EULER = 0, PDG_NAVIER_STOKES = 1 };

/* Mesh tables (all host pointers, copied by pdg_create).  Every element is a degenerate
 * trilinear hexahedron given by 8 corners in lexicographic order c = i + 2j + 4k of [-1,1]^3;
 * collapsed corners repeat a vertex (Sec. 2, Duffy transform to the unit hexahedron):
 *   hex (c0..c7); prism (v0,v1,v3,v4,v2,v2,v5,v5); pyramid (b0,b1,b2,b3,a,a,a,a) with the base
 *   listed lexicographically; tet (v0,v1,v2,v2,v3,v3,v3,v3).
 * The mapping must be affine after the collapse (straight-sided elements) with positive
 * Jacobian.  Faces are found from shared global vertex-id sets: equal sets are conforming
 * faces; a quadrilateral face covered by two triangles is a non-conforming (mortar) face.
 * The mesh must be closed (periodic: periodic images carry the same vertex id).            */
typedef struct {
    int32_t n_elems;
    int32_t n_vertices;          /* vertex ids are in [0, n_vertices)                    */
    const int8_t *elem_type;     /* [n_elems] PDG_HEX..PDG_TET                          */
    const int32_t *elem_corner;  /* [n_elems][8] corner -> global vertex id              */
    const double *corner_xyz;    /* [n_elems][8][3] coordinates, unwrapped per element   */
    const double *centroid;      /* [n_elems][3] element centroid, used for the SFC keys */
} pdg_mesh;

typedef struct {
    int32_t N;            /* polynomial degree, 2..6 (Euler) or 2..5 (Navier-Stokes)     */
    int32_t equations;    /* PDG_EULER or PDG_NAVIER_STOKES                               */
    int32_t flux;         /* surface flux: 0 local Lax-Friedrichs (Rusanov); 1 Chandrashekar's
                             entropy-conservative two-point flux (property tests)          */
    int32_t node_family;  /* 0: Gauss-Lobatto, left Gauss-Radau in collapsing directions */
    int32_t volume_form;  /* inviscid volume term: 0 weak form (Eq. (1)); 1 entropy-stable
                             split form (Sec. 2: SBP property and Chandrashekar's two-point
                             flux): along every Gauss-Lobatto node line the weak term becomes
                             sum_m (Q^T - Q)[i][m] / w_i F#(q_i, q_m).(a_i + a_m)/2; lines on
                             Gauss-Radau nodes (collapsing directions) and viscous fluxes keep
                             the weak term.  pdg_vjp, the adjoint stages and pdg_batch_create
                             need volume_form = 0 and flux = 0 (PDG_ENOTSUP otherwise)      */
    double gamma;         /* ratio of specific heats                                     */
    double mu;            /* dynamic viscosity (Navier-Stokes)                            */
    double Pr;            /* Prandtl number (Navier-Stokes)                               */
    double R;             /* gas constant (Navier-Stokes, T = p / (rho R))                */
    double p_ref;         /* reference pressure taken out of the momentum flux, (p - p_ref)I:
                             the discrete residual of a constant flux vanishes, so R(U) is
                             unchanged in exact arithmetic while the cancellation of a large
                             mean pressure (low Mach number) is avoided; 0 disables it       */
} pdg_params;

/* Build a context: validates and copies the mesh, orders the elements along the Hilbert curve
 * of their centroids (Sec. 3, Fig. 1a; keys as pdg_sfc_keys with the centroids' bounding box),
 * builds faces, geometry and operator tables.  hip_stream: the hipStream_t all device work is
 * enqueued on (NULL = default stream).  Synchronous.
 * Curved elements (Alg. 1 takes the Jacobian at the nodes): an element's map is the trilinear
 * map of its eight corners on the reference cube (collapsed for prisms, pyramids and tetrahedra),
 * which need not be affine; quadrilateral faces are then bilinear patches.  If any element is
 * curved, the whole mesh is stepped with a Jacobian and contravariant vectors per volume node, a
 * normal and area factor per face point, and for every prism, pyramid and tetrahedron its own
 * mass-matrix inverse (V^T W J V)^-1, built at creation in extended precision.  A curved mesh
 * needs conforming faces (no quadrilateral-triangle mortars: a bilinear quadrilateral has no
 * straight diagonal); the split form averages the two nodes' contravariant vectors in each
 * two-point flux; the adjoint entry points refuse it.
 * Errors: PDG_EINVAL (bad sizes/params), PDG_EMESH (unmatched or non-manifold faces,
 * non-positive Jacobian at a node, singular mass matrix), PDG_ENOTSUP (a curved mesh with mortar
 * faces, unsupported N or options), PDG_EHIP, PDG_ENOMEM.                                    */
int pdg_create(const pdg_mesh *mesh, const pdg_params *params, void *hip_stream, pdg_ctx **out);

/* The state layout.  Outputs (host, each may be NULL): n_doubles = length of U;
 * perm[i] = input index of the element stored i-th ([n_elems]); elem_offset[i] = first double
 * of element i ([n_elems+1]); elem_type[i] = its type ([n_elems]); elem_sides[2i] = number of
 * face sides of element i (a mortar half counts as one) and elem_sides[2i+1] = how many of them
 * need interpolation to the face points (not collocated with volume nodes) ([n_elems][2]).
 * Synchronous.                                                                               */
int pdg_layout(const pdg_ctx *ctx, int64_t *n_doubles, int32_t *perm, int64_t *elem_offset,
               int8_t *elem_type, int32_t *elem_sides);

/* Physical coordinates of the volume nodes of every element (device out, [n_elems][n^3][3],
 * stored element order).  Used to set initial conditions.                                   */
int pdg_node_coords(pdg_ctx *ctx, double *xyz);

/* Modal projection of nodal values (Algorithm 1, u~ = M^-1 V^T W J q): q (device in,
 * [n_elems][5][n^3], stored element order) -> U (device out, state layout).  Hexahedra copy. */
int pdg_project(pdg_ctx *ctx, const double *q, double *U);

/* Nodal values at the volume nodes (q = V u~ for modal elements): U -> q [n_elems][5][n^3]. */
int pdg_nodal(pdg_ctx *ctx, const double *U, double *q);

/* dU/dt = R(U) (Eq. (1) with Algorithm 1's modal projection for non-hexahedra).  U, dUdt:
 * device, state layout, distinct buffers.  Asynchronous.                                    */
int pdg_residual(pdg_ctx *ctx, const double *U, double *dUdt);

/* n_steps steps of the five-stage fourth-order 2N-storage LSERK scheme (Carpenter & Kennedy
 * 1994): per stage K <- A_s K + R(U), U <- U + dt B_s K.  K is zeroed at the start of every
 * step by A_0 = 0 (its input values are ignored).  U, K: device, state layout, updated in place.
 * Asynchronous; on a moving mesh (pdg_set_motion) stage s of step i takes the geometry at the
 * time t + (i + c_s) dt from the context's time t, which advances by n_steps dt, and the call
 * is synchronous (PDG_EMESH if a Jacobian became non-positive).                             */
int pdg_rk_steps(pdg_ctx *ctx, double *U, double *K, double dt, int32_t n_steps);

/* Moving mesh (Algorithm 1: M = V^T W J V cannot be precomputed when the Jacobian changes in
 * time).  Every element corner then moves as x(t) = x0 + d sin(omega t), x0 the corner given
 * to pdg_create and d = corner_disp (host, [n_elems][8][3] in input element order, as
 * pdg_mesh.corner_xyz; equal, to 1e-12 of the largest entry, for the corners that are one
 * vertex, including periodic images, else PDG_EINVAL).
 * The residual becomes the weak form on the moving elements: the flux relative to the grid,
 * F - q xdot, in the volume term, the Lax-Friedrichs flux through the moving faces (normal
 * speed xdot . n, wave speed |u.n - xdot.n| + c), and M du~/dt = r - V^T W (dJ/dt q), so that
 * the state stays the modal coefficients (hexahedra: nodal values).  The geometry (per-node
 * metrics, dJ/dt and grid velocity, per-face-point normals and normal speeds, every modal
 * element's M_e^-1) is rebuilt on the device at the context's time (pdg_set_time) and at every
 * RK stage time (pdg_rk_steps); M_e there is evaluated from four matrices built by this call
 * (J is a cubic in sin(omega t), so M_e = M0 + s M1 + s^2 M2 + s^3 M3 exactly; device memory
 * 2 sum_e m_e (m_e + 1) doubles over the modal elements, upper triangles).  Needs conforming faces, the weak form with the LF flux and
 * N <= 5 (else PDG_ENOTSUP); the adjoint, the batch and pdg_rk_stage then refuse the context.
 * Calling it again replaces d and omega.  Synchronous; PDG_EMESH if a Jacobian is not
 * positive at the context's time.                                                           */
int pdg_set_motion(pdg_ctx *ctx, const double *corner_disp, double omega);

/* Geometry of the moving mesh at time t (becomes the context's time; pdg_residual,
 * pdg_project, pdg_node_weights and pdg_node_coords then see the mesh at t).  PDG_EINVAL
 * without a motion.  Synchronous; PDG_EMESH if a Jacobian is not positive at t.             */
int pdg_set_time(pdg_ctx *ctx, double t);

/* The context's time (0 until pdg_set_time or pdg_rk_steps on a moving mesh moves it).      */
int pdg_get_time(const pdg_ctx *ctx, double *t);

/* Vector-Jacobian product grad_U = (dR/dU)^T cot of the residual above at U (the adjoint of
 * Eq. (1) with Algorithm 1's projection; not in the paper): every linear operator of R applied
 * transposed in reverse order and every pointwise flux through its analytic Jacobian.  At the
 * flux's non-smooth points the maximum wave speed takes the element's own side on ties and
 * d|x|/dx = sign(x), sign(0) = 0.  U, cot, grad_U: device, state layout; grad_U distinct from
 * U and cot.  Asynchronous.  Scratch buffers are allocated on the first call.               */
int pdg_vjp(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U);

/* pdg_vjp for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the same result, with
 * the workspace (flux cotangents; for Navier-Stokes also the BR1 face-value cotangents and a
 * partial gradient) in a static device array of 64 MiB that every GPU the library runs on holds
 * until the process ends, instead of buffers the context allocates on its first pdg_vjp.  The
 * call allocates nothing.  Needs (slots * n^2 * 9 + n_doubles) doubles for Navier-Stokes,
 * (slots * n^2 * 5) for Euler (each rounded up to 256 bytes); larger meshes get PDG_EINVAL
 * with the sizes in pdg_last_error().  The current device must be the context's.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU race.  Asynchronous.        */
int pdg_vjp_static(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U);

/* One stage s (0..4) of the LSERK4 step above: K <- A_s K + R(U), U <- U + dt B_s K (A_0 = 0).
 * Used to recompute stage states from a checkpoint.  Device, in place.  Asynchronous.
 * PDG_ENOTSUP on a moving mesh.                                                              */
int pdg_rk_stage(pdg_ctx *ctx, double *U, double *K, double dt, int32_t stage);

/* Reverse of stage s for gradients through time: with U_s the stage's input state,
 *   Kbar <- Kbar + dt B_s Ubar;  Ubar <- Ubar + (dR/dU(U_s))^T Kbar;  Kbar <- A_s Kbar.
 * Running it for the stages of n steps in reverse order, starting from Ubar = dJ/dU_n and
 * Kbar = 0, leaves dJ/dU_0 in Ubar.  U_s, Ubar, Kbar: device, state layout, distinct buffers,
 * updated in place.  Asynchronous.                                                           */
int pdg_rk_stage_adjoint(pdg_ctx *ctx, const double *U_s, double *Ubar, double *Kbar, double dt, int32_t stage);

/* Transpose of pdg_nodal: Ubar = V^T qbar for modal elements, a copy for hexahedra.
 * qbar: device [n_elems][5][n^3] stored element order; Ubar: device, state layout.  For
 * gradients of objectives defined on the nodal values (e.g. the kinetic energy).            */
int pdg_nodal_adjoint(pdg_ctx *ctx, const double *qbar, double *Ubar);

/* Nodal quadrature weights w_k J_k (Algorithm 1's W J) of every element: device out
 * [n_elems][n^3], stored element order.  The discrete integral of a nodal field f is
 * sum(wJ * f).  Asynchronous.                                                                */
int pdg_node_weights(pdg_ctx *ctx, double *wJ);

/* Finiteness check of a state (failure detection; the paper's solver restarts from memory, Sec. 3,
 * and a blown-up state is what such a restart has to catch): PDG_OK when every entry of U (device,
 * state layout, n_doubles entries) is finite, else PDG_ENONFINITE.  first_bad (host, may be NULL)
 * receives the smallest stored index of a NaN or infinite entry, or -1.  Synchronous.          */
int pdg_check_finite(pdg_ctx *ctx, const double *U, int64_t *first_bad);

/* 63-bit Hilbert keys of the element centroids in INPUT element order (device out [n_elems]):
 * k_a = min(floor((c_a - lo_a) * scale), 2^21 - 1) with exactly one FP64 subtraction and one
 * multiplication, then J. Skilling's transpose method (AIP Conf. Proc. 707, 2004), bits
 * interleaved most significant first in axis order x, y, z.  lo: host [3].  Asynchronous.   */
int pdg_sfc_keys(pdg_ctx *ctx, const double lo[3], double scale, uint64_t *keys);

/* Cost-weighted contiguous partition of the stored (Hilbert-ordered) elements into n_queues
 * segments (Sec. 3: contiguous, non-overlapping SFC segments).  weight: device [n_elems]
 * (stored order); queue_begin: device out [n_queues+1].  With S_i the exclusive prefix sum and
 * W the total, element i goes to queue min(Q - 1, floor(Q (2 S_i + w_i) / (2W))) (the cap only
 * moves trailing zero-weight elements into the last queue); queue_begin[q] is the first element
 * of queue q and queue_begin[Q] = n_elems.  Exact integer arithmetic (128-bit products) for any
 * 32-bit weights; all-zero weights put every element in the last queue.  Asynchronous.      */
int pdg_partition(pdg_ctx *ctx, const uint32_t *weight, int32_t n_queues, int32_t *queue_begin);

/* Integer element weights from per-type costs (the device-timed costs of pdg_measure_costs,
 * Sec. 3, Listing 1): w_t = max(1, round(1024 c_t / c_hex)), with c_hex replaced by the smallest
 * positive cost when there are no hexahedra, capped at 2^24; weight[e] = w_(type of e).
 * cost_per_elem: host [4], finite and >= 0, not all 0; weight: device out [n_elems] (stored
 * order), ready for pdg_partition.  weight_type (host out [4], may be NULL) receives w_t.
 * Asynchronous.                                                                             */
int pdg_type_weights(pdg_ctx *ctx, const double cost_per_elem[4], uint32_t *weight, uint32_t weight_type[4]);

/* Install a work-queue schedule (device queue_begin [n_queues+1], copied; validated to start
 * at 0, end at n_elems and be non-decreasing): residual and RK kernels then serve each queue
 * with its own workgroups over its contiguous element segment of any types (the paper's
 * contiguous SFC segments per rank, Sec. 3), taking the segment's elements type by type, each
 * type in Hilbert order.  In each phase a queue gets as many workgroups as keep every CU at
 * that phase's queue kernel occupancy (resident workgroups / n_queues, 1..16), which share its
 * elements round-robin.  Results do not depend on the schedule.  n_queues = 0 restores the default
 * schedule (per-type launches, one workgroup per element).  Synchronous.                    */
int pdg_set_schedule(pdg_ctx *ctx, const int32_t *queue_begin, int32_t n_queues);

/* The installed schedule: *n_queues (0 = per-type launches) and, if queue_begin (host, room
 * for n_queues+1) is not NULL and a schedule is installed, its queue_begin.                  */
int pdg_get_schedule(pdg_ctx *ctx, int32_t *queue_begin, int32_t *n_queues);

/* Per-queue timers of the work-queue schedule (the paper's loop timers, Sec. 3, Listing 1,
 * taken per queue): every queue kernel adds the device wall-clock time of each workgroup to a
 * counter of its own; a queue's time is the mean over its workgroups (which share its elements).
 * queue_ms (host, may be NULL) receives the accumulated
 * milliseconds [3][n_queues] (phase 0 trace, 1 volume, 2 surface) since the timers were last
 * cleared; n_evals (may be NULL) the residual evaluations (RK stages) they cover.  reset != 0
 * clears them afterwards.  Installing a schedule clears them.  PDG_EINVAL without a schedule.
 * Synchronous.                                                                               */
int pdg_queue_times(pdg_ctx *ctx, double *queue_ms, int32_t reset, int64_t *n_evals);

/* Element weights from measured queue times (host only; no device is used).  The time of
 * queue q in phase p, queue_ms[p*n_queues + q], is shared by the queue's elements in proportion
 * to per-type costs fitted over all queues by non-negative least squares (one fit per phase):
 * the paper's attribution of loop time to the elements taking part in the loop (Sec. 3,
 * Listing 1), with the modal overhead resolved per element type.  weight[e] = max(1,
 * round(1024 c_e / mean c)) (at most 2^24) of the element's summed cost c_e.
 *   elem_type[n_elems]   types in stored (Hilbert) order (0 hex, 1 prism, 2 pyramid, 3 tet)
 *   queue_begin          [n_queues+1], 0 .. n_elems, non-decreasing
 *   type_cost[12]        (may be NULL) fitted cost per element, type t phase p at [4p + t]
 *   imbalance            (may be NULL) measured imbalance: sum over phases of the slowest queue
 *                        over sum over phases of the mean queue, minus 1
 * PDG_EINVAL on an invalid schedule, a type out of range, or negative, non-finite or all-zero
 * times.                                                                                     */
int pdg_balance_weights(int32_t n_elems, const int8_t *elem_type, int32_t n_queues, const int32_t *queue_begin,
                        const double *queue_ms, uint32_t *weight, double type_cost[12], double *imbalance);

/* Threshold-triggered rebalance of the installed work-queue schedule (Sec. 3): from the queue
 * timers accumulated since they were last cleared, the measured imbalance is compared with
 * `threshold`; above it, element weights follow from pdg_balance_weights, the elements are
 * re-partitioned into the same number of queues (pdg_partition) and the new schedule is
 * installed.  No state moves: only the queue boundaries along the Hilbert order shift, and
 * results stay bitwise identical (every element is computed the same way in any queue).  The
 * timers are cleared in both cases.
 *   info[0]  measured imbalance      info[1]  predicted imbalance of the new schedule under the
 *            attributed costs (= info[0] when not triggered)
 *   info[2]  1 if rebalanced, else 0 info[3]  residual evaluations the timers covered
 * PDG_EINVAL without a schedule or without recorded time.  Synchronous.                      */
int pdg_rebalance(pdg_ctx *ctx, double threshold, double info[4]);

/* Device-timer cost measurement (the paper's loop timers, Sec. 3, Listing 1, on the device):
 * evaluates R(U) reps + 1 times (the first warms up) with every kernel launch bracketed by HIP
 * events on the context stream, and returns
 *   cost_per_elem[4]  seconds per element per residual of hex, prism, pyramid, tet (the sum of
 *                     the element's trace, volume and surface phases over its type's count);
 *   phase_ms[12]      (may be NULL) average launch duration in ms of phase p (0 trace,
 *                     1 volume, 2 surface) for type t at phase_ms[4p + t].
 * U: device, state layout (read only).  Synchronous.                                         */
int pdg_measure_costs(pdg_ctx *ctx, const double *U, int32_t reps, double cost_per_elem[4],
                      double phase_ms[12]);

/* ---------------------------------------------------------------------------------------
 * Batched form: many independent problems (meshes of any size, any N, either equation set),
 * each an existing context, advanced together (the paper's setting of many differently sized
 * partitions, Sec. 3, gathered on one device).  Every LSERK step is one HIP graph launch that
 * holds, per stage and phase, one kernel per (element type, N, equations) group covering the
 * elements of every problem in the group; a workgroup processes a tile of `tile[type][N]`
 * consecutive elements of one problem.  Results are identical to pdg_rk_steps on each context.
 * ------------------------------------------------------------------------------------- */

/* Batch over ctxs[0..n) (distinct, alive while the batch is used; affine or curved, not moving:
 * PDG_ENOTSUP).  Tiles start at 1.  hip_stream: the stream graph launches go to.  A member set in
 * motion afterwards (pdg_set_motion) makes pdg_batch_rk_steps and pdg_batch_autotune return
 * PDG_ENOTSUP.                                                                               */
int pdg_batch_create(pdg_ctx *const *ctxs, int32_t n, void *hip_stream, pdg_batch **out);

/* n_steps LSERK4 steps of every problem i with its own U[i], K[i] (device, state layout of
 * context i, distinct) and time step dt[i] (host array).  The step graph is captured on the
 * first call and replayed; argument changes are uploaded before the launches.  Asynchronous
 * except when the arguments change (then it waits for the batch's earlier launches).         */
int pdg_batch_rk_steps(pdg_batch *b, double *const *U, double *const *K, const double *dt, int32_t n_steps);

/* Tiles (elements per workgroup) as an int32 array [4][7] indexed [type][N] (entries for
 * N < 2 ignored); each in 1..64.  Set rebuilds the work lists and drops the captured graph. */
int pdg_batch_set_tiles(pdg_batch *b, const int32_t *tiles);
int pdg_batch_get_tiles(const pdg_batch *b, int32_t *tiles);

/* Problems with at least min_elems elements run alone: per stage each such problem's three
 * phases are launched back to back through the per-type kernels of pdg_rk_steps, with the
 * stage's arguments by value (its face traces stay in the caches between the phases), before
 * the merged groups of the other problems; a change of U, K or dt then recaptures the step graph
 * on the next call.  INT32_MAX (the default) merges every problem, 0 runs every problem alone.
 * Results are the same in every arrangement.  Set rebuilds the work lists and drops the graph.  */
int pdg_batch_set_solo(pdg_batch *b, int32_t min_elems);
int pdg_batch_get_solo(const pdg_batch *b, int32_t *min_elems);

/* Autotuner: with every problem merged, for each (type, N, equations) group times the group's
 * three phases (residual mode, into library scratch: U and K are read, not modified) with tiles
 * 1, 2, 4 and 8 over reps repetitions after one warm-up and keeps the fastest (a larger tile
 * must win by 3 %); then times whole residuals with the solo threshold (pdg_batch_set_solo) at
 * INT32_MAX, 65536, 16384, 4096 and 0 elements and keeps the fastest (by 3 % over merging all).
 * Returns the tiles in tiles_out ([4][7], may be NULL).  Synchronous.                          */
int pdg_batch_autotune(pdg_batch *b, double *const *U, double *const *K, const double *dt, int32_t reps,
                       int32_t *tiles_out);

/* Release a batch (NULL is ignored); its contexts are untouched.                             */
void pdg_batch_destroy(pdg_batch *b);

/* Launch timing of the running computation: between pdg_timing_start and pdg_timing_stop every
 * per-type kernel launch of pdg_residual / pdg_rk_steps / pdg_rk_stage (not the work-queue
 * schedule) is bracketed by a HIP event pair on the context stream.  Stop waits for the stream
 * and returns, for phase p (0 trace, 1 volume, 2 surface) and type t at index 4p + t, the summed
 * launch durations total_ms and the number of launches.                                       */
int pdg_timing_start(pdg_ctx *ctx);
int pdg_timing_stop(pdg_ctx *ctx, double total_ms[12], int32_t launches[12]);

/* Message of the last failing call on this thread ("" if none).                             */
const char *pdg_last_error(void);

/* Release a context (NULL is ignored).                                                      */
void pdg_destroy(pdg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PDG_H */
