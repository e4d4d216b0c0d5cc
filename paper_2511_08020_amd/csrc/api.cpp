// C ABI of libpolydg: context creation (mesh ingest, Hilbert ordering, faces, tables) and the
// entry points declared in include/pdg.h.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>

#include "balance.h"
#include "batch.h"

using namespace pdg;

namespace pdg {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace pdg

#define PDG_TRY_HIP(call)                                                              \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(_e)); \
            return PDG_EHIP;                                                           \
        }                                                                              \
    } while (0)

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage LSERK coefficients
static const double kRKA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double kRKB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

struct pdg_ctx {
    pdg_params prm{};
    int N = 0, n = 0, nn = 0, n2 = 0;
    int device = 0;  // the GPU the context was created on
    bool ns = false;
    bool curved = false;  // some hexahedra are trilinear (per-node metrics, per-point face normals)
    bool has_mortar = false;  // quadrilateral-triangle faces
    // moving mesh (pdg_set_motion): corners x0 + d sin(omega t); geometry rebuilt per stage time
    bool moving = false;
    double time = 0.0, omega = 0.0;
    double geo_time = 0.0;             // time of the geometry on the device
    bool geo_valid = false;
    std::vector<double> disp;          // stored order [n][8][3]
    std::vector<int32_t> corner_id;    // stored order [n][8] global vertex ids
    int32_t n_vertices = 0;
    std::vector<MoveFace> mfaces;      // every face, for the per-stage face geometry
    MoveArgs mv{};
    hipStream_t stream = nullptr;
    int32_t n_elems = 0;
    std::vector<int32_t> perm;   // stored i -> input index
    std::vector<int8_t> etype;   // stored order
    std::vector<int64_t> off;    // [n_elems+1]
    int64_t n_doubles = 0;
    std::vector<int32_t> tlist[4];
    TypeTables tt[4];
    std::vector<TraceOp> ops;
    int32_t n_slots = 0;
    std::vector<void *> allocs;
    StageArgs sa{};
    double *d_Tq = nullptr, *d_Fvn = nullptr, *d_Rp = nullptr;
    double *d_Lf = nullptr, *d_Lw = nullptr, *d_Ub = nullptr;  // adjoint buffers (allocated on first use)
    double *d_centroid = nullptr;  // input order
    double *d_corners = nullptr;   // stored order [n][8][3]
    uint64_t *d_scan = nullptr;
    int32_t *d_qtb = nullptr;          // per queue boundary, per type: first index into the type list
    int32_t n_queues = 0, qb_capacity = 0;
    int64_t qt_capacity = 0;            // queue-timer slots per phase [n_queues * qmax]
    int32_t qsub[3] = {1, 1, 1};        // workgroups per queue in each phase's queue kernel
    int32_t qmax = 1;                   // the largest of them
    std::vector<int32_t> h_qb;          // host copy of the installed schedule
    uint64_t *d_qt = nullptr;           // [3][n_queues * qmax] wall-clock ticks per phase and workgroup
    int64_t qt_evals = 0;               // residual evaluations since the timers were cleared
    uint32_t *d_weight = nullptr;       // rebalance weights [n_elems]
    int32_t *d_qb_new = nullptr;        // rebalance partition [qb_capacity+1]
    double *d_scratch_out = nullptr;  // output buffer of pdg_measure_costs
    unsigned long long *d_first_bad = nullptr;  // pdg_check_finite result
    std::vector<int32_t> elem_sides;  // [n_elems][2]: face sides, sides with interpolated points
    // launch timing (pdg_timing_start/stop): event pairs around every per-type launch
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_slot;  // phase*4 + type of each recorded pair
    size_t ev_used = 0;

    ~pdg_ctx() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
    // two events for the next timed launch (grown on demand), or false on failure
    bool next_events(int slot, hipEvent_t &a, hipEvent_t &b) {
        while (ev_pool.size() < 2 * (ev_used + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            ev_pool.push_back(e);
        }
        a = ev_pool[2 * ev_used];
        b = ev_pool[2 * ev_used + 1];
        ev_slot.push_back(slot);
        ++ev_used;
        return true;
    }
    template <typename T>
    T *alloc(size_t count) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return (T *)p;
    }
    template <typename T>
    T *upload(const std::vector<T> &v) {
        T *p = alloc<T>(v.size());
        if (!p) return nullptr;
        if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return nullptr;
        return p;
    }
};

namespace {

struct FRec {
    int32_t ids[4];
    int32_t nd;
    int32_t elem;
    int32_t plane;
};

bool rec_less(const FRec &a, const FRec &b) {
    if (a.nd != b.nd) return a.nd < b.nd;
    for (int i = 0; i < 4; ++i)
        if (a.ids[i] != b.ids[i]) return a.ids[i] < b.ids[i];
    if (a.elem != b.elem) return a.elem < b.elem;
    return a.plane < b.plane;
}
bool rec_same_key(const FRec &a, const FRec &b) {
    return a.nd == b.nd && std::equal(a.ids, a.ids + 4, b.ids);
}

struct HFace {
    int kind;       // FACE_QUAD / FACE_TRI
    int32_t ids[3];  // canonical A, B, C (tri) or A, B, D (quad)
    int32_t e[2];    // stored element index, e[0] < e[1]
    int32_t plane[2];
};

void plane_slots(int plane, int slots[2][2]) {
    const int a = plane >> 1, s = plane & 1;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    if (b > c) std::swap(b, c);
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) slots[u][v] = (s << a) | (u << b) | (v << c);
}

int expected_distinct(int type) { return type == PDG_HEX ? 8 : type == PDG_PRISM ? 6 : type == PDG_PYR ? 5 : 4; }

bool collapse_ok(int type, const int32_t *c) {
    auto eq = [&](int i, int j) { return c[i] == c[j]; };
    switch (type) {
        case PDG_HEX: break;
        case PDG_PRISM: if (!(eq(4, 5) && eq(6, 7))) return false; break;
        case PDG_PYR: if (!(eq(4, 5) && eq(4, 6) && eq(4, 7))) return false; break;
        case PDG_TET: if (!(eq(2, 3) && eq(4, 5) && eq(4, 6) && eq(4, 7))) return false; break;
        default: return false;
    }
    std::vector<int32_t> d(c, c + 8);
    std::sort(d.begin(), d.end());
    return (int)(std::unique(d.begin(), d.end()) - d.begin()) == expected_distinct(type);
}

int first_slot(const int32_t *corner, int32_t vid) {
    for (int c = 0; c < 8; ++c)
        if (corner[c] == vid) return c;
    return -1;
}

}  // namespace

// Metrics of an element's trilinear corner map x(eta) on its reference cube (corner slot
// a + 2b + 4c at eta = (2a-1, 2b-1, 2c-1); the collapsed types repeat corners, so the map holds
// the collapse) at the point eta: out[0] = J, out[1 + 3b + c] = (dx/deta_{b+1} x dx/deta_{b+2})_c,
// the contravariant rows J grad eta^b (for an affine element: its cofactor rows composed with
// the reference collapse).
static void corner_map_metrics(const double *X, const double eta[3], double *out) {
    double D[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // D[b] = dx/deta_b
    for (int c = 0; c < 8; ++c) {
        double sg[3], f[3];
        for (int a = 0; a < 3; ++a) {
            sg[a] = ((c >> a) & 1) ? 1.0 : -1.0;
            f[a] = 0.5 * (1.0 + sg[a] * eta[a]);
        }
        for (int b = 0; b < 3; ++b) {
            const double dN = 0.5 * sg[b] * f[(b + 1) % 3] * f[(b + 2) % 3];
            for (int d = 0; d < 3; ++d) D[b][d] += dN * X[3 * c + d];
        }
    }
    for (int b = 0; b < 3; ++b) {
        const double *u = D[(b + 1) % 3], *v = D[(b + 2) % 3];
        out[1 + 3 * b + 0] = u[1] * v[2] - u[2] * v[1];
        out[1 + 3 * b + 1] = u[2] * v[0] - u[0] * v[2];
        out[1 + 3 * b + 2] = u[0] * v[1] - u[1] * v[0];
    }
    out[0] = D[0][0] * out[1] + D[0][1] * out[2] + D[0][2] * out[3];
}

// corner_map_metrics at every volume node of an element of type table tt: out[k][10]; false if
// J <= 0 at a node
static bool node_metrics(const double *X, const TypeTables &tt, int n, double *out) {
    const int nn = n * n * n;
    for (int k = 0; k < nn; ++k) {
        const double eta[3] = {tt.x[0][k % n], tt.x[1][(k / n) % n], tt.x[2][k / (n * n)]};
        corner_map_metrics(X, eta, out + 10 * (size_t)k);
        if (!(out[10 * (size_t)k] > 0)) return false;
    }
    return true;
}

static int build_context(pdg_ctx *ctx, const pdg_mesh *mesh) {
    const int N = ctx->N, n = ctx->n, n2 = ctx->n2;
    const int ne = mesh->n_elems;
    // ---- validate elements, affine geometry
    std::vector<double> geo_in((size_t)ne * 10);
    for (int e = 0; e < ne; ++e) {
        const int t = mesh->elem_type[e];
        if (t < 0 || t > 3) { set_error("element type out of range"); return PDG_EINVAL; }
        const int32_t *c = mesh->elem_corner + 8 * (size_t)e;
        for (int k = 0; k < 8; ++k)
            if (c[k] < 0 || c[k] >= mesh->n_vertices) { set_error("vertex id out of range"); return PDG_EINVAL; }
        if (!collapse_ok(t, c)) {
            set_error("element " + std::to_string(e) + ": corner ids do not follow the collapse pattern of its type");
            return PDG_EMESH;
        }
        const double *X = mesh->corner_xyz + 24 * (size_t)e;
        double A[3][3];  // columns a_b = (x_{slot 1,2,4} - x_0) / 2
        const int sl[3] = {1, 2, 4};
        for (int b = 0; b < 3; ++b)
            for (int d = 0; d < 3; ++d) A[b][d] = 0.5 * (X[3 * sl[b] + d] - X[d]);
        double scale = 0.0;
        for (int b = 0; b < 3; ++b)
            for (int d = 0; d < 3; ++d) scale = std::max(scale, std::fabs(A[b][d]));
        bool affine = true;
        for (int k = 0; k < 8; ++k) {
            const double *xi = ref_corner(t, k);
            for (int d = 0; d < 3; ++d) {
                double x = X[d];
                for (int b = 0; b < 3; ++b) x += A[b][d] * (xi[b] + 1.0);
                if (std::fabs(x - X[3 * k + d]) > 1e-9 * std::max(1.0, scale)) affine = false;
            }
        }
        // curved (trilinear) elements: per-node metrics and, for the modal types, a mass matrix
        // per element
        if (!affine) ctx->curved = true;
        double cof[3][3];  // row b = a_{b+1} x a_{b+2}
        for (int b = 0; b < 3; ++b) {
            const double *u = A[(b + 1) % 3], *v = A[(b + 2) % 3];
            cof[b][0] = u[1] * v[2] - u[2] * v[1];
            cof[b][1] = u[2] * v[0] - u[0] * v[2];
            cof[b][2] = u[0] * v[1] - u[1] * v[0];
        }
        const double det = A[0][0] * cof[0][0] + A[0][1] * cof[0][1] + A[0][2] * cof[0][2];
        if (!(det > 0)) {
            set_error("element " + std::to_string(e) + " has a non-positive Jacobian");
            return PDG_EMESH;
        }
        double *g = &geo_in[10 * (size_t)e];
        g[0] = det;
        for (int b = 0; b < 3; ++b)
            for (int d = 0; d < 3; ++d) g[1 + 3 * b + d] = cof[b][d];
    }

    // ---- Hilbert order of the centroids (device keys, host stable sort)
    std::vector<double> cen(mesh->centroid, mesh->centroid + 3 * (size_t)ne);
    ctx->d_centroid = ctx->upload(cen);
    if (!ctx->d_centroid) { set_error("out of device memory"); return PDG_ENOMEM; }
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        lo[d] = hi[d] = ne ? cen[d] : 0.0;
        for (int e = 1; e < ne; ++e) {
            lo[d] = std::min(lo[d], cen[3 * (size_t)e + d]);
            hi[d] = std::max(hi[d], cen[3 * (size_t)e + d]);
        }
    }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    const double scale = ext > 0 ? 2097152.0 / ext : 1.0;
    std::vector<uint64_t> keys(ne);
    {
        uint64_t *dk = ctx->alloc<uint64_t>(ne);
        if (!dk) { set_error("out of device memory"); return PDG_ENOMEM; }
        PDG_TRY_HIP(launch_sfc_keys(ne, ctx->d_centroid, lo, scale, dk, nullptr));
        PDG_TRY_HIP(hipMemcpy(keys.data(), dk, ne * sizeof(uint64_t), hipMemcpyDeviceToHost));
    }
    ctx->perm.resize(ne);
    std::iota(ctx->perm.begin(), ctx->perm.end(), 0);
    std::stable_sort(ctx->perm.begin(), ctx->perm.end(), [&](int a, int b) { return keys[a] < keys[b]; });

    // ---- stored order tables
    ctx->etype.resize(ne);
    ctx->off.assign(ne + 1, 0);
    std::vector<double> geo((size_t)ne * 10), corners((size_t)ne * 24);
    std::vector<int32_t> corner_id((size_t)ne * 8);
    for (int i = 0; i < ne; ++i) {
        const int e = ctx->perm[i];
        ctx->etype[i] = mesh->elem_type[e];
        ctx->off[i + 1] = ctx->off[i] + 5 * (int64_t)ctx->tt[ctx->etype[i]].m;
        std::copy(&geo_in[10 * (size_t)e], &geo_in[10 * (size_t)e] + 10, &geo[10 * (size_t)i]);
        std::copy(mesh->corner_xyz + 24 * (size_t)e, mesh->corner_xyz + 24 * (size_t)e + 24, &corners[24 * (size_t)i]);
        std::copy(mesh->elem_corner + 8 * (size_t)e, mesh->elem_corner + 8 * (size_t)e + 8, &corner_id[8 * (size_t)i]);
        ctx->tlist[ctx->etype[i]].push_back(i);
    }
    ctx->n_doubles = ctx->off[ne];

    // ---- faces from vertex-id sets
    std::vector<FRec> recs;
    recs.reserve((size_t)ne * 6);
    for (int i = 0; i < ne; ++i) {
        const int32_t *c = &corner_id[8 * (size_t)i];
        for (int plane = 0; plane < 6; ++plane) {
            int sl[2][2];
            plane_slots(plane, sl);
            int32_t ids[4] = {c[sl[0][0]], c[sl[0][1]], c[sl[1][0]], c[sl[1][1]]};
            std::sort(ids, ids + 4);
            int nd = (int)(std::unique(ids, ids + 4) - ids);
            if (nd < 3) continue;
            FRec r;
            for (int k = 0; k < 4; ++k) r.ids[k] = k < nd ? ids[k] : -1;
            r.nd = nd;
            r.elem = i;
            r.plane = plane;
            recs.push_back(r);
        }
    }
    std::sort(recs.begin(), recs.end(), rec_less);
    std::vector<HFace> faces;
    std::vector<size_t> left_quads;
    std::vector<char> tri_used(recs.size(), 0);
    auto quad_frame = [&](int i, int plane, const FRec &r, int32_t out[3]) {
        int sl[2][2];
        plane_slots(plane, sl);
        const int32_t *c = &corner_id[8 * (size_t)i];
        const int32_t A = r.ids[0];
        int uA = -1, vA = -1;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v)
                if (c[sl[u][v]] == A) { uA = u; vA = v; }
        int32_t n1 = c[sl[1 - uA][vA]], n2v = c[sl[uA][1 - vA]];
        out[0] = A;
        out[1] = std::min(n1, n2v);
        out[2] = std::max(n1, n2v);
    };
    for (size_t g0 = 0; g0 < recs.size();) {
        size_t g1 = g0 + 1;
        while (g1 < recs.size() && rec_same_key(recs[g0], recs[g1])) ++g1;
        const size_t cnt = g1 - g0;
        const FRec &r = recs[g0];
        if (cnt > 2) { set_error("non-manifold face"); return PDG_EMESH; }
        if (cnt == 2) {
            HFace f;
            f.kind = r.nd == 4 ? FACE_QUAD : FACE_TRI;
            f.e[0] = recs[g0].elem; f.plane[0] = recs[g0].plane;
            f.e[1] = recs[g0 + 1].elem; f.plane[1] = recs[g0 + 1].plane;
            if (f.kind == FACE_QUAD) quad_frame(f.e[0], f.plane[0], r, f.ids);
            else { f.ids[0] = r.ids[0]; f.ids[1] = r.ids[1]; f.ids[2] = r.ids[2]; }
            faces.push_back(f);
            if (r.nd == 3) tri_used[g0] = tri_used[g0 + 1] = 1;
        } else if (r.nd == 4) {
            left_quads.push_back(g0);
        }
        g0 = g1;
    }
    for (size_t qi : left_quads) {
        const FRec &q = recs[qi];
        int found = 0;
        for (int drop = 0; drop < 4; ++drop) {
            FRec key;
            int k = 0;
            for (int j = 0; j < 4; ++j)
                if (j != drop) key.ids[k++] = q.ids[j];
            key.ids[3] = -1;
            key.nd = 3;
            key.elem = -1;
            key.plane = -1;
            auto it = std::lower_bound(recs.begin(), recs.end(), key, rec_less);
            if (it == recs.end() || !rec_same_key(*it, key)) continue;
            size_t idx = it - recs.begin();
            if (idx + 1 < recs.size() && rec_same_key(recs[idx + 1], key)) continue;  // conforming elsewhere
            if (tri_used[idx]) continue;
            tri_used[idx] = 1;
            HFace f;
            f.ids[0] = key.ids[0]; f.ids[1] = key.ids[1]; f.ids[2] = key.ids[2];
            int ea = q.elem, pa = q.plane, eb = it->elem, pb = it->plane;
            if (eb < ea) { std::swap(ea, eb); std::swap(pa, pb); }
            f.e[0] = ea; f.plane[0] = pa; f.e[1] = eb; f.plane[1] = pb;
            for (int kind : {(int)FACE_MORTAR0, (int)FACE_MORTAR1}) {  // the half's two point chunks
                f.kind = kind;
                faces.push_back(f);
            }
            ++found;
        }
        if (found != 2) { set_error("quadrilateral face without a conforming or two-triangle partner"); return PDG_EMESH; }
    }
    for (size_t r = 0; r < recs.size(); ++r)
        if (recs[r].nd == 3 && !tri_used[r]) { set_error("unmatched triangular face"); return PDG_EMESH; }
    for (const HFace &f : faces)
        if (f.kind == FACE_MORTAR0 || f.kind == FACE_MORTAR1) ctx->has_mortar = true;
    if (ctx->curved) {
        for (const HFace &f : faces)
            if (f.kind == FACE_MORTAR0 || f.kind == FACE_MORTAR1) {
                set_error("curved hexahedra need conforming faces (a bilinear quadrilateral has no straight diagonal)");
                return PDG_ENOTSUP;
            }
    }

    // ---- slots, trace operators, face geometry
    std::vector<std::vector<std::pair<int, int>>> eslots(ne);  // (face, side)
    for (size_t f = 0; f < faces.size(); ++f)
        for (int s = 0; s < 2; ++s) eslots[faces[f].e[s]].push_back({(int)f, s});
    std::vector<int32_t> slot_begin(ne + 1, 0);
    // hexahedra: six faces, each up to two mortar halves of two chunks; prisms: two triangles
    // (mortar chunks) and two outer quadrilaterals (halves of chunks) plus the cut face;
    // pyramids: four triangles and the base; tetrahedra: two outer and two inner triangles
    const int maxslots[4] = {24, 13, 8, 6};
    for (int i = 0; i < ne; ++i) {
        auto &v = eslots[i];
        std::sort(v.begin(), v.end(), [&](const std::pair<int, int> &a, const std::pair<int, int> &b) {
            int pa = faces[a.first].plane[a.second], pb = faces[b.first].plane[b.second];
            if (pa != pb) return pa < pb;
            return a.first < b.first;
        });
        if ((int)v.size() > maxslots[ctx->etype[i]]) { set_error("too many face sides on one element"); return PDG_EMESH; }
        slot_begin[i + 1] = slot_begin[i] + (int)v.size();
    }
    const int ns_tot = slot_begin[ne];
    ctx->n_slots = ns_tot;
    std::vector<int32_t> face_slot(2 * faces.size(), -1);
    for (int i = 0; i < ne; ++i)
        for (size_t k = 0; k < eslots[i].size(); ++k)
            face_slot[2 * eslots[i][k].first + eslots[i][k].second] = slot_begin[i] + (int)k;
    std::vector<int32_t> slot_nbr(ns_tot), slot_op(ns_tot), slot_kind(ns_tot);
    // curved meshes: J and contravariant rows at every volume node of every element, the mass
    // matrix inverse M_e^-1 = (V^T W J V)^-1 per modal element (Alg. 1 with the Jacobian at the
    // nodes), and face geometry per face point
    const int gp = ctx->curved ? n2 : 1;
    std::vector<double> nmet, minv;
    std::vector<int64_t> minv_off;
    if (ctx->curved) {
        const int nn = ctx->nn;
        nmet.assign((size_t)ne * nn * 10, 0.0);
        minv_off.assign(ne, 0);
        int64_t tot = 0;
        for (int i = 0; i < ne; ++i) {
            const int m = ctx->tt[ctx->etype[i]].m;
            minv_off[i] = tot;
            if (ctx->etype[i] != PDG_HEX) tot += (int64_t)m * m;
        }
        minv.assign((size_t)tot, 0.0);
        // elements are independent: shared out over the host's threads (disjoint outputs)
        std::atomic<int> fail{0};
        auto work = [&](int i0, int i1) {
            std::vector<long double> M, Mi;
            for (int i = i0; i < i1 && !fail.load(std::memory_order_relaxed); ++i) {
                const TypeTables &tt = ctx->tt[ctx->etype[i]];
                double *mt = &nmet[(size_t)i * nn * 10];
                if (!node_metrics(&corners[24 * (size_t)i], tt, n, mt)) { fail = 1; return; }
                if (ctx->etype[i] == PDG_HEX) continue;
                const int m = tt.m;
                M.assign((size_t)m * m, 0.0L);
                for (int a = 0; a < m; ++a)
                    for (int b = 0; b <= a; ++b) {
                        long double acc = 0.0L;
                        for (int k = 0; k < nn; ++k)
                            acc += (long double)tt.V[(size_t)k * m + a] * tt.w[k] * mt[10 * (size_t)k] *
                                   tt.V[(size_t)k * m + b];
                        M[(size_t)a * m + b] = M[(size_t)b * m + a] = acc;
                    }
                if (!cholesky_inverse(m, M, Mi)) { fail = 2; return; }
                for (size_t q = 0; q < Mi.size(); ++q) minv[(size_t)minv_off[i] + q] = (double)Mi[q];
            }
        };
        const int nt = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        const int chunk = (ne + nt - 1) / nt;
        for (int t = 0; t < nt && t * chunk < ne; ++t) pool.emplace_back(work, t * chunk, std::min(ne, (t + 1) * chunk));
        for (auto &th : pool) th.join();
        if (fail == 1) { set_error("curved element with a non-positive Jacobian at a volume node"); return PDG_EMESH; }
        if (fail == 2) { set_error("curved element with a singular mass matrix"); return PDG_EMESH; }
    }
    std::vector<double> slot_geo(4 * (size_t)ns_tot * gp);
    std::unordered_map<uint64_t, int> op_index;
    for (size_t f = 0; f < faces.size(); ++f) {
        const HFace &F = faces[f];
        // geometry from side 0
        const int e0 = F.e[0];
        const double *X0 = &corners[24 * (size_t)e0];
        const int32_t *c0 = &corner_id[8 * (size_t)e0];
        double P[3][3];
        for (int k = 0; k < 3; ++k) {
            int s = first_slot(c0, F.ids[k]);
            for (int d = 0; d < 3; ++d) P[k][d] = X0[3 * s + d];
        }
        double u[3], v[3], nv[3];
        for (int d = 0; d < 3; ++d) { u[d] = P[1][d] - P[0][d]; v[d] = P[2][d] - P[0][d]; }
        nv[0] = u[1] * v[2] - u[2] * v[1];
        nv[1] = u[2] * v[0] - u[0] * v[2];
        nv[2] = u[0] * v[1] - u[1] * v[0];
        const double area = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        for (int d = 0; d < 3; ++d) nv[d] /= area;
        double fc[3], ec[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            fc[d] = F.kind == FACE_QUAD ? P[0][d] + 0.5 * u[d] + 0.5 * v[d] : (P[0][d] + P[1][d] + P[2][d]) / 3.0;
            for (int c = 0; c < 8; ++c) ec[d] += X0[3 * c + d] / 8.0;
        }
        const double orient = (fc[0] - ec[0]) * nv[0] + (fc[1] - ec[1]) * nv[1] + (fc[2] - ec[2]) * nv[2] < 0 ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) nv[d] *= orient;
        const double sc = F.kind == FACE_QUAD ? area / 4.0 : area / 8.0;  // |dP/ds x dP/dt| / (1 - t)
        for (int s = 0; s < 2; ++s) {
            const int i = F.e[s], t = ctx->etype[i];
            const int32_t *ci = &corner_id[8 * (size_t)i];
            TraceOp op{};
            op.type = t; op.axis = F.plane[s] >> 1; op.side = F.plane[s] & 1; op.kind = F.kind;
            for (int k = 0; k < 3; ++k) op.slots[k] = first_slot(ci, F.ids[k]);
            uint64_t key = ((((((uint64_t)t * 8 + F.plane[s]) * kFaceKinds + F.kind) * 8 + op.slots[0]) * 8 + op.slots[1]) * 8 + op.slots[2]);
            auto it = op_index.find(key);
            int id;
            if (it == op_index.end()) {
                if (!build_trace_op(ctx->tt[t], op)) { set_error("face point inversion failed"); return PDG_EMESH; }
                id = (int)ctx->ops.size();
                ctx->ops.push_back(std::move(op));
                op_index[key] = id;
            } else {
                id = it->second;
            }
            const int sl = face_slot[2 * f + s];
            slot_nbr[sl] = face_slot[2 * f + (1 - s)];
            slot_op[sl] = id;
            slot_kind[sl] = F.kind;
        }
        // geometry from side 0, negated for side 1 (bitwise antisymmetric).  A curved
        // quadrilateral face (a bilinear patch) per face point: n dS = +-a^axis of side 0's map at
        // the point (outward: + on the plane's upper side), area factor |a^axis| (the face rule's
        // reference measure is d eta_b d eta_c); triangles stay flat
        const int sl0 = face_slot[2 * f], sl1 = face_slot[2 * f + 1];
        const TraceOp &op0 = ctx->ops[slot_op[sl0]];
        const bool pointwise = ctx->curved && F.kind == FACE_QUAD;
        for (int p = 0; p < gp; ++p) {
            double g[4] = {nv[0], nv[1], nv[2], sc};
            if (pointwise) {
                double mt[10];
                corner_map_metrics(X0, &op0.eta[3 * (size_t)p], mt);
                const double *a = mt + 1 + 3 * (F.plane[0] >> 1);
                const double len = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                const double sgn = (F.plane[0] & 1) ? 1.0 : -1.0;
                for (int d = 0; d < 3; ++d) g[d] = sgn * a[d] / len;
                g[3] = len;
            }
            for (int d = 0; d < 3; ++d) {
                slot_geo[4 * ((size_t)sl0 * gp + p) + d] = g[d];
                slot_geo[4 * ((size_t)sl1 * gp + p) + d] = -g[d];
            }
            slot_geo[4 * ((size_t)sl0 * gp + p) + 3] = g[3];
            slot_geo[4 * ((size_t)sl1 * gp + p) + 3] = g[3];
        }
        // the face as a moving mesh rebuilds it: quadrilaterals from a^axis with the plane's
        // side as sign, triangles from side 0's corners with the orientation found here
        MoveFace mf{};
        mf.sl0 = sl0;
        mf.sl1 = sl1;
        mf.e0 = e0;
        mf.op0 = slot_op[sl0];
        mf.kind = F.kind;
        mf.axis = F.plane[0] >> 1;
        for (int k = 0; k < 3; ++k) mf.k[k] = first_slot(c0, F.ids[k]);
        mf.sgn = F.kind == FACE_QUAD ? ((F.plane[0] & 1) ? 1.0 : -1.0) : orient;
        ctx->mfaces.push_back(mf);
    }
    (void)N;
    ctx->elem_sides.assign(2 * (size_t)ne, 0);
    for (int i = 0; i < ne; ++i)
        for (int sl = slot_begin[i]; sl < slot_begin[i + 1]; ++sl) {
            ctx->elem_sides[2 * i] += 1;
            if (!ctx->ops[slot_op[sl]].perm) ctx->elem_sides[2 * i + 1] += 1;
        }

    // ---- upload
    auto &sa = ctx->sa;
    sa.mesh.n_elems = ne;
    sa.mesh.etype = ctx->upload(ctx->etype);
    sa.mesh.off = ctx->upload(ctx->off);
    sa.mesh.geo = ctx->upload(geo);
    sa.mesh.slot_begin = ctx->upload(slot_begin);
    sa.mesh.slot_nbr = ctx->upload(slot_nbr);
    sa.mesh.slot_op = ctx->upload(slot_op);
    sa.mesh.slot_kind = ctx->upload(slot_kind);
    sa.mesh.slot_geo = ctx->upload(slot_geo);
    sa.mesh.geo_pts = gp;
    sa.mesh.nmet = nullptr;
    sa.mesh.minv = nullptr;
    sa.mesh.minv_off = nullptr;
    sa.mesh.nmov = nullptr;
    sa.mesh.gvn = nullptr;
    if (ctx->curved) {
        sa.mesh.nmet = ctx->upload(nmet);
        sa.mesh.minv_off = ctx->upload(minv_off);
        if (!minv.empty()) sa.mesh.minv = ctx->upload(minv);
        if (!sa.mesh.nmet || !sa.mesh.minv_off || (!minv.empty() && !sa.mesh.minv)) {
            set_error("out of device memory");
            return PDG_ENOMEM;
        }
    }
    ctx->d_corners = ctx->upload(corners);
    ctx->corner_id = corner_id;
    ctx->n_vertices = mesh->n_vertices;
    // face sides above which an element needs the wide kernels (the device's kSlotsNarrow)
    const int narrow_slots[4] = {24, 8, 8, 6};
    for (int t = 0; t < 4; ++t) {
        sa.list[t] = ctx->upload(ctx->tlist[t]);
        sa.count[t] = (int32_t)ctx->tlist[t].size();
        std::vector<int32_t> ln, lw;
        for (int32_t i : ctx->tlist[t])
            (slot_begin[i + 1] - slot_begin[i] > narrow_slots[t] ? lw : ln).push_back(i);
        sa.list_n[t] = ctx->upload(ln);
        sa.list_w[t] = ctx->upload(lw);
        sa.count_n[t] = (int32_t)ln.size();
        sa.count_w[t] = (int32_t)lw.size();
        if (!sa.list[t] || !sa.list_n[t] || !sa.list_w[t]) { set_error("out of device memory"); return PDG_ENOMEM; }
        const TypeTables &tt = ctx->tt[t];
        std::vector<double> buf;
        size_t o_dh[3], o_w, o_c, o_V, o_P, o_M, o_jd;
        for (int a = 0; a < 3; ++a) { o_dh[a] = buf.size(); buf.insert(buf.end(), tt.dhat[a].begin(), tt.dhat[a].end()); }
        size_t o_ds[3];
        for (int a = 0; a < 3; ++a) { o_ds[a] = buf.size(); buf.insert(buf.end(), tt.dskew[a].begin(), tt.dskew[a].end()); }
        size_t o_dm[3];
        for (int a = 0; a < 3; ++a) { o_dm[a] = buf.size(); buf.insert(buf.end(), tt.dmat[a].begin(), tt.dmat[a].end()); }
        o_w = buf.size(); buf.insert(buf.end(), tt.w.begin(), tt.w.end());
        o_c = buf.size(); buf.insert(buf.end(), tt.cmet.begin(), tt.cmet.end());
        o_V = buf.size(); buf.insert(buf.end(), tt.V.begin(), tt.V.end());
        o_P = buf.size(); buf.insert(buf.end(), tt.VtW.begin(), tt.VtW.end());
        o_M = buf.size(); buf.insert(buf.end(), tt.Minv.begin(), tt.Minv.end());
        o_jd = buf.size(); buf.insert(buf.end(), tt.jd.begin(), tt.jd.end());
        size_t o_Vp = buf.size(), o_Vtp = buf.size(), o_MTp = buf.size(), o_MPp = buf.size(), o_MPtp = buf.size();
        size_t o_VWp = buf.size();
        if (t != PDG_HEX) {
            // packed copies start on 32-byte boundaries
            while (buf.size() % 4) buf.push_back(0.0);
            std::vector<double> Vt((size_t)tt.m * tt.nn), MPt((size_t)tt.nn * tt.m), MT((size_t)tt.m * tt.m);
            for (int k = 0; k < tt.nn; ++k)
                for (int j = 0; j < tt.m; ++j) {
                    Vt[(size_t)j * tt.nn + k] = tt.V[(size_t)k * tt.m + j];
                    MPt[(size_t)k * tt.m + j] = tt.MVtW[(size_t)j * tt.nn + k];
                }
            for (int i = 0; i < tt.m; ++i)
                for (int j = 0; j < tt.m; ++j) MT[(size_t)i * tt.m + j] = tt.Minv[(size_t)j * tt.m + i];
            const std::vector<double> MPp = pack_rows(tt.MVtW, tt.m, tt.nn), MPtp = pack_rows(MPt, tt.nn, tt.m),
                                      Vp = pack_rows(tt.V, tt.nn, tt.m), Vtp = pack_rows(Vt, tt.m, tt.nn),
                                      MTp = pack_rows(MT, tt.m, tt.m);
            o_MPp = buf.size(); buf.insert(buf.end(), MPp.begin(), MPp.end());
            o_MPtp = buf.size(); buf.insert(buf.end(), MPtp.begin(), MPtp.end());
            o_Vp = buf.size(); buf.insert(buf.end(), Vp.begin(), Vp.end());
            o_Vtp = buf.size(); buf.insert(buf.end(), Vtp.begin(), Vtp.end());
            o_MTp = buf.size(); buf.insert(buf.end(), MTp.begin(), MTp.end());
            const std::vector<double> VWp = pack_rows(tt.VtW, tt.m, tt.nn);
            o_VWp = buf.size(); buf.insert(buf.end(), VWp.begin(), VWp.end());
        }
        const double *d = ctx->upload(buf);
        if (!d) { set_error("out of device memory"); return PDG_ENOMEM; }
        DevType &dt = sa.tab[t];
        for (int a = 0; a < 3; ++a) { dt.dhat[a] = d + o_dh[a]; dt.dskew[a] = d + o_ds[a]; dt.dmat[a] = d + o_dm[a]; }
        dt.w = d + o_w; dt.cmet = d + o_c; dt.V = d + o_V; dt.VtW = d + o_P; dt.Minv = d + o_M; dt.jd = d + o_jd;
        dt.Vp = d + o_Vp; dt.Vtp = d + o_Vtp; dt.MinvTp = d + o_MTp; dt.MVtWp = d + o_MPp; dt.MVtWtp = d + o_MPtp;
        dt.VtWp = d + o_VWp;
    }
    {
        std::vector<int32_t> op_type, op_plane, op_perm, idata;
        std::vector<int64_t> op_off, op_ioff, op_poff;
        std::vector<double> data;
        for (const TraceOp &op : ctx->ops) {
            op_type.push_back(op.type);
            op_plane.push_back(2 * op.axis + op.side);
            op_perm.push_back(op.perm ? 1 : 0);
            op_off.push_back((int64_t)data.size());
            op_ioff.push_back((int64_t)idata.size());
            op_poff.push_back(0);
            if (op.type == PDG_HEX) {
                if (op.perm) {
                    idata.insert(idata.end(), op.pmap.begin(), op.pmap.end());
                    idata.insert(idata.end(), op.inv.begin(), op.inv.end());
                } else {
                    data.insert(data.end(), op.I.begin(), op.I.end());
                }
            } else {
                data.insert(data.end(), op.E.begin(), op.E.end());
                data.insert(data.end(), op.Et.begin(), op.Et.end());
                const int m = ctx->tt[op.type].m, n2 = ctx->n2;
                while (data.size() % 4) data.push_back(0.0);
                op_poff.back() = (int64_t)data.size();
                const std::vector<double> Ep = pack_rows(op.E, n2, m), Etp = pack_rows(op.Et, m, n2),
                                          MEtp = pack_rows(op.MEt, m, n2), EMp = pack_rows(op.EM, n2, m);
                data.insert(data.end(), Ep.begin(), Ep.end());
                data.insert(data.end(), Etp.begin(), Etp.end());
                data.insert(data.end(), MEtp.begin(), MEtp.end());
                data.insert(data.end(), EMp.begin(), EMp.end());
                data.insert(data.end(), op.EM.begin(), op.EM.end());  // plain, for the vector-unit lift
            }
        }
        std::vector<double> Wq;
        for (int kind = 0; kind < kFaceKinds; ++kind) {
            std::vector<double> s, t, W;
            face_points(kind, n, s, t, W);
            Wq.insert(Wq.end(), W.begin(), W.end());
        }
        sa.ops.op_type = ctx->upload(op_type);
        sa.ops.op_plane = ctx->upload(op_plane);
        sa.ops.op_perm = ctx->upload(op_perm);
        sa.ops.op_off = ctx->upload(op_off);
        sa.ops.op_ioff = ctx->upload(op_ioff);
        sa.ops.op_poff = ctx->upload(op_poff);
        sa.ops.data = ctx->upload(data);
        sa.ops.idata = ctx->upload(idata);
        sa.ops.Wq = ctx->upload(Wq);
    }
    sa.qsub = 1;
    sa.phys.gamma = ctx->prm.gamma;
    sa.phys.mu = ctx->prm.mu;
    sa.phys.Pr = ctx->prm.Pr;
    sa.phys.R = ctx->prm.R;
    {
        const double e_ref = ctx->prm.p_ref / (ctx->prm.gamma - 1.0);
        sa.phys.e_ref = e_ref;
        sa.phys.p_ref = (ctx->prm.gamma - 1.0) * e_ref;
        sa.phys.h_ref = e_ref + sa.phys.p_ref;
        for (int t = 1; t < 4; ++t) {
            const long double psi0 = ctx->tt[t].V[0];  // every entry of V's first column
            const double c0 = (double)((long double)e_ref / psi0);
            sa.tab[t].c0 = c0;
            sa.tab[t].dlt = (double)(psi0 * (long double)c0 - (long double)e_ref);
        }
        sa.tab[0].c0 = sa.tab[0].dlt = 0.0;
    }
    ctx->d_Tq = ctx->alloc<double>((size_t)ns_tot * 5 * n2);
    ctx->d_Fvn = ctx->ns ? ctx->alloc<double>((size_t)ns_tot * 5 * n2) : nullptr;
    ctx->d_Rp = ctx->alloc<double>(ctx->n_doubles);
    ctx->d_scan = ctx->alloc<uint64_t>(ne);
    sa.Tq = ctx->d_Tq;
    sa.Fvn = ctx->d_Fvn;
    sa.Rp = ctx->d_Rp;
    if (!sa.mesh.slot_geo || !ctx->d_Tq || !ctx->d_Rp || !ctx->d_scan || (ctx->ns && !ctx->d_Fvn)) {
        set_error("out of device memory");
        return PDG_ENOMEM;
    }
    return PDG_OK;
}

// the adjoint and the batched form implement the weak form with the Lax-Friedrichs flux only
static bool plain_form(const pdg_ctx *ctx) { return ctx->prm.volume_form == 0 && ctx->prm.flux == 0; }

static hipError_t launch_volume_form(pdg_ctx *ctx, const StageArgs &sa, int t) {
    return ctx->prm.volume_form ? launch_volume_split(ctx->N, ctx->ns, sa, t, ctx->stream)
                                : launch_volume(ctx->N, ctx->ns, sa, t, ctx->stream);
}
static hipError_t launch_surface_flux(pdg_ctx *ctx, const StageArgs &sa, int t) {
    return ctx->prm.flux ? launch_surface_ec(ctx->N, ctx->ns, sa, t, ctx->stream)
                         : launch_surface(ctx->N, ctx->ns, sa, t, ctx->stream);
}

static int run_stage(pdg_ctx *ctx, const double *U, int mode, double *out, double *K, double *Uw, double a,
                     double bdt) {
    StageArgs sa = ctx->sa;
    sa.U = U;
    sa.mode = mode;
    sa.out = out;
    sa.K = K;
    sa.Uw = Uw;
    sa.rk_a = a;
    sa.rk_bdt = bdt;
    if (ctx->n_queues > 0) {
        for (int ph = 0; ph < 3; ++ph) {
            sa.qsub = ctx->qsub[ph];
            uint64_t *qt = ctx->d_qt + (size_t)ph * ctx->n_queues * ctx->qmax;
            if (ph == 1 && ctx->prm.volume_form)
                PDG_TRY_HIP(launch_volume_split_queues(ctx->N, ctx->ns, sa, ctx->d_qtb, ctx->n_queues, qt, ctx->stream));
            else if (ph == 2 && ctx->prm.flux)
                PDG_TRY_HIP(launch_surface_ec_queues(ctx->N, ctx->ns, sa, ctx->d_qtb, ctx->n_queues, qt, ctx->stream));
            else
                PDG_TRY_HIP(launch_queues(ctx->N, ctx->ns, ph, sa, ctx->d_qtb, ctx->n_queues, qt, ctx->stream));
        }
        ++ctx->qt_evals;
        return PDG_OK;
    }
    for (int ph = 0; ph < 3; ++ph)
        for (int t = 0; t < 4; ++t) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool timed = ctx->timing && sa.count[t] > 0;
            if (timed) {
                if (!ctx->next_events(ph * 4 + t, e0, e1)) { set_error("hipEventCreate failed"); return PDG_EHIP; }
                PDG_TRY_HIP(hipEventRecord(e0, ctx->stream));
            }
            if (ph == 0) PDG_TRY_HIP(launch_trace(ctx->N, sa, t, ctx->stream));
            if (ph == 1) PDG_TRY_HIP(launch_volume_form(ctx, sa, t));
            if (ph == 2) PDG_TRY_HIP(launch_surface_flux(ctx, sa, t));
            if (timed) PDG_TRY_HIP(hipEventRecord(e1, ctx->stream));
        }
    return PDG_OK;
}

extern "C" {

const char *pdg_last_error(void) { return g_err.c_str(); }

int pdg_create(const pdg_mesh *mesh, const pdg_params *params, void *hip_stream, pdg_ctx **out) {
    if (!mesh || !params || !out) { set_error("null argument"); return PDG_EINVAL; }
    *out = nullptr;
    if (params->N < 2 || params->N > kMaxN) { set_error("N must be in 2..6"); return PDG_ENOTSUP; }
    if (params->equations != PDG_EULER && params->equations != PDG_NAVIER_STOKES) { set_error("unknown equations"); return PDG_EINVAL; }
    if ((params->flux != 0 && params->flux != 1) || params->node_family != 0 ||
        (params->volume_form != 0 && params->volume_form != 1)) {
        set_error("unsupported flux, node family or volume form");
        return PDG_ENOTSUP;
    }
    if (params->equations == PDG_NAVIER_STOKES && params->N > 5) {
        set_error("Navier-Stokes is available for N <= 5");
        return PDG_ENOTSUP;
    }
    if (!(params->gamma > 1.0)) { set_error("gamma must exceed 1"); return PDG_EINVAL; }
    if (!std::isfinite(params->p_ref)) { set_error("p_ref must be finite"); return PDG_EINVAL; }
    if (params->equations == PDG_NAVIER_STOKES && !(params->mu >= 0 && params->Pr > 0 && params->R > 0)) {
        set_error("invalid viscous parameters");
        return PDG_EINVAL;
    }
    if (mesh->n_elems <= 0 || mesh->n_vertices <= 0 || !mesh->elem_type || !mesh->elem_corner || !mesh->corner_xyz ||
        !mesh->centroid) {
        set_error("empty or incomplete mesh");
        return PDG_EINVAL;
    }
    pdg_ctx *ctx = new (std::nothrow) pdg_ctx();
    if (!ctx) { set_error("out of host memory"); return PDG_ENOMEM; }
    ctx->prm = *params;
    ctx->N = params->N;
    ctx->n = params->N + 1;
    ctx->nn = ctx->n * ctx->n * ctx->n;
    ctx->n2 = ctx->n * ctx->n;
    ctx->ns = params->equations == PDG_NAVIER_STOKES;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->n_elems = mesh->n_elems;
    if (hipGetDevice(&ctx->device) != hipSuccess) { set_error("hipGetDevice failed"); delete ctx; return PDG_EHIP; }
    for (int t = 0; t < 4; ++t) build_type_tables(t, ctx->N, ctx->tt[t]);
    int rc = build_context(ctx, mesh);
    if (rc == PDG_OK) rc = static_workspace_setup();
    if (rc != PDG_OK) { delete ctx; return rc; }
    if (hipDeviceSynchronize() != hipSuccess) { set_error("device synchronisation failed"); delete ctx; return PDG_EHIP; }
    *out = ctx;
    return PDG_OK;
}

void pdg_destroy(pdg_ctx *ctx) { delete ctx; }

int pdg_layout(const pdg_ctx *ctx, int64_t *n_doubles, int32_t *perm, int64_t *elem_offset, int8_t *elem_type,
               int32_t *elem_sides) {
    if (!ctx) { set_error("null context"); return PDG_EINVAL; }
    if (n_doubles) *n_doubles = ctx->n_doubles;
    if (perm) std::copy(ctx->perm.begin(), ctx->perm.end(), perm);
    if (elem_offset) std::copy(ctx->off.begin(), ctx->off.end(), elem_offset);
    if (elem_type) std::copy(ctx->etype.begin(), ctx->etype.end(), elem_type);
    if (elem_sides) std::copy(ctx->elem_sides.begin(), ctx->elem_sides.end(), elem_sides);
    return PDG_OK;
}

int pdg_residual(pdg_ctx *ctx, const double *U, double *dUdt) {
    if (!ctx || !U || !dUdt) { set_error("null argument"); return PDG_EINVAL; }
    if (U == dUdt) { set_error("U and dUdt must be distinct buffers"); return PDG_EINVAL; }
    return run_stage(ctx, U, 0, dUdt, nullptr, nullptr, 0.0, 0.0);
}

// ---- moving meshes
// stage times of Carpenter and Kennedy's five-stage fourth-order low-storage scheme
static const double kRKC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                               2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

// the moving mesh's geometry at time t, on the context's stream (nothing to do if the device
// already holds it)
static int update_geometry(pdg_ctx *ctx, double t) {
    if (ctx->geo_valid && ctx->geo_time == t) return PDG_OK;
    ctx->mv.s = std::sin(ctx->omega * t);
    ctx->mv.c = ctx->omega * std::cos(ctx->omega * t);
    ctx->geo_valid = false;
    PDG_TRY_HIP(launch_move_geometry(ctx->N, ctx->mv, ctx->sa, ctx->stream));
    ctx->geo_time = t;
    ctx->geo_valid = true;
    return PDG_OK;
}

// synchronous: PDG_EMESH if a node's Jacobian was not positive since the flag was cleared
static int check_motion(pdg_ctx *ctx) {
    int32_t bad = 0;
    PDG_TRY_HIP(hipMemcpyAsync(&bad, ctx->mv.bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (bad) {
        ctx->geo_valid = false;  // rebuilt (and checked) again on the next request
        set_error("moving mesh: non-positive Jacobian at a volume node");
        return PDG_EMESH;
    }
    return PDG_OK;
}

int pdg_set_motion(pdg_ctx *ctx, const double *corner_disp, double omega) {
    if (!ctx || !corner_disp) { set_error("null argument"); return PDG_EINVAL; }
    if (!std::isfinite(omega)) { set_error("omega must be finite"); return PDG_EINVAL; }
    if (!plain_form(ctx)) { set_error("moving meshes need the weak form and the Lax-Friedrichs flux"); return PDG_ENOTSUP; }
    if (ctx->has_mortar) {
        set_error("moving meshes need conforming faces (a bilinear quadrilateral has no straight diagonal)");
        return PDG_ENOTSUP;
    }
    if (ctx->N > 5) { set_error("moving meshes take N <= 5"); return PDG_ENOTSUP; }
    const int ne = ctx->n_elems, nn = ctx->nn, n = ctx->n, gp = ctx->n2;
    std::vector<double> disp((size_t)ne * 24);
    for (int i = 0; i < ne; ++i)
        for (int q = 0; q < 24; ++q) {
            const double v = corner_disp[24 * (size_t)ctx->perm[i] + q];
            if (!std::isfinite(v)) { set_error("corner displacement not finite"); return PDG_EINVAL; }
            disp[24 * (size_t)i + q] = v;
        }
    // one displacement per vertex: every corner holding it (periodic images included) moves alike,
    // up to the rounding of a periodic function evaluated at the images (1e-12 of the largest)
    {
        double dmax = 0.0;
        for (double v : disp) dmax = std::max(dmax, std::fabs(v));
        std::vector<int64_t> first(ctx->n_vertices, -1);
        for (size_t c = 0; c < ctx->corner_id.size(); ++c) {
            const int32_t v = ctx->corner_id[c];
            if (first[v] < 0) { first[v] = (int64_t)c; continue; }
            for (int d = 0; d < 3; ++d)
                if (std::fabs(disp[3 * c + d] - disp[3 * (size_t)first[v] + d]) > 1e-12 * dmax) {
                    set_error("corner displacements of vertex " + std::to_string(v) + " differ between its corners");
                    return PDG_EINVAL;
                }
        }
    }
    MoveArgs &m = ctx->mv;
    auto &mesh = ctx->sa.mesh;
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (!ctx->moving) {
        // every modal element's M_e (and M_e^-1) slot, and its packed upper triangle's, in
        // element order
        std::vector<int64_t> minv_off(ne, 0), poff(ne, 0);
        int64_t tot = 0, ptot = 0;
        for (int i = 0; i < ne; ++i) {
            minv_off[i] = tot;
            poff[i] = ptot;
            const int64_t me = ctx->tt[ctx->etype[i]].m;
            if (ctx->etype[i] != PDG_HEX) {
                tot += me * me;
                ptot += me * (me + 1) / 2;
            }
        }
        if (!ctx->curved) {
            // the kernels' curved path: per-node metrics, per-point face geometry, M_e^-1
            mesh.nmet = ctx->alloc<double>((size_t)ne * nn * 10);
            mesh.minv = ctx->alloc<double>((size_t)tot);
            mesh.minv_off = ctx->upload(minv_off);
            mesh.slot_geo = ctx->alloc<double>((size_t)ctx->n_slots * gp * 4);
            mesh.geo_pts = gp;
            if (!mesh.nmet || !mesh.minv || !mesh.minv_off || !mesh.slot_geo) {
                set_error("out of device memory");
                return PDG_ENOMEM;
            }
        }
        std::vector<double> eta1d((size_t)4 * 3 * n), opeta;
        for (int t = 0; t < 4; ++t)
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < n; ++i) eta1d[((size_t)t * 3 + a) * n + i] = ctx->tt[t].x[a][i];
        std::vector<int64_t> opeta_off;
        for (const TraceOp &op : ctx->ops) {
            if (op.eta.size() != 3 * (size_t)gp) { set_error("face points of a trace operator missing"); return PDG_EINVAL; }
            opeta_off.push_back((int64_t)opeta.size());
            opeta.insert(opeta.end(), op.eta.begin(), op.eta.end());
        }
        m.n_elems = ne;
        m.n_faces = (int32_t)ctx->mfaces.size();
        m.gp = gp;
        m.x0 = ctx->d_corners;
        m.disp = ctx->alloc<double>(disp.size());
        m.eta1d = ctx->upload(eta1d);
        m.etype = mesh.etype;
        m.faces = ctx->upload(ctx->mfaces);
        m.opeta = ctx->upload(opeta);
        m.opeta_off = ctx->upload(opeta_off);
        m.nmet = const_cast<double *>(mesh.nmet);
        m.nmov = ctx->alloc<double>((size_t)ne * nn * 4);
        m.slot_geo = const_cast<double *>(mesh.slot_geo);
        m.gvn = ctx->alloc<double>((size_t)ctx->n_slots * gp);
        m.minv = const_cast<double *>(mesh.minv);
        m.minv_off = mesh.minv_off;
        m.ptot = ptot;
        m.poff = ctx->upload(poff);
        m.mcoef = ptot > 0 ? ctx->alloc<double>((size_t)4 * ptot) : nullptr;
        m.bad = ctx->alloc<int32_t>(1);
        if (!m.disp || !m.eta1d || !m.faces || !m.opeta || !m.opeta_off || !m.nmov || !m.gvn || !m.bad ||
            !m.poff || (ptot > 0 && !m.mcoef)) {
            set_error("out of device memory");
            return PDG_ENOMEM;
        }
        mesh.nmov = m.nmov;
        mesh.gvn = m.gvn;
        ctx->curved = true;
        ctx->moving = true;
    }
    PDG_TRY_HIP(hipMemcpy(const_cast<double *>(m.disp), disp.data(), disp.size() * sizeof(double), hipMemcpyHostToDevice));
    // M_e(s) = sum_q s^q M_q for these displacements (J is a cubic in s = sin(omega t))
    PDG_TRY_HIP(launch_move_mass_coefficients(ctx->N, m, ctx->sa, ctx->stream));
    ctx->disp = std::move(disp);
    ctx->omega = omega;
    ctx->geo_valid = false;
    PDG_TRY_HIP(hipMemsetAsync(m.bad, 0, sizeof(int32_t), ctx->stream));
    int rc = update_geometry(ctx, ctx->time);
    return rc != PDG_OK ? rc : check_motion(ctx);
}

int pdg_set_time(pdg_ctx *ctx, double t) {
    if (!ctx) { set_error("null context"); return PDG_EINVAL; }
    if (!ctx->moving) { set_error("no mesh motion set"); return PDG_EINVAL; }
    if (!std::isfinite(t)) { set_error("time must be finite"); return PDG_EINVAL; }
    PDG_TRY_HIP(hipMemsetAsync(ctx->mv.bad, 0, sizeof(int32_t), ctx->stream));
    int rc = update_geometry(ctx, t);
    if (rc != PDG_OK) return rc;
    ctx->time = t;
    return check_motion(ctx);
}

int pdg_get_time(const pdg_ctx *ctx, double *t) {
    if (!ctx || !t) { set_error("null argument"); return PDG_EINVAL; }
    *t = ctx->time;
    return PDG_OK;
}

int pdg_rk_steps(pdg_ctx *ctx, double *U, double *K, double dt, int32_t n_steps) {
    if (!ctx || !U || !K) { set_error("null argument"); return PDG_EINVAL; }
    if (U == K) { set_error("U and K must be distinct buffers"); return PDG_EINVAL; }
    if (n_steps < 0 || !std::isfinite(dt)) { set_error("invalid step count or time step"); return PDG_EINVAL; }
    const double t0 = ctx->time;
    if (ctx->moving) PDG_TRY_HIP(hipMemsetAsync(ctx->mv.bad, 0, sizeof(int32_t), ctx->stream));
    for (int s = 0; s < n_steps; ++s)
        for (int st = 0; st < 5; ++st) {
            // a moving mesh takes each stage's geometry at the stage's time
            if (ctx->moving) {
                int rc = update_geometry(ctx, t0 + (s + kRKC[st]) * dt);
                if (rc != PDG_OK) return rc;
            }
            int rc = run_stage(ctx, U, 1, nullptr, K, U, kRKA[st], kRKB[st] * dt);
            if (rc != PDG_OK) return rc;
        }
    if (!ctx->moving) return PDG_OK;
    ctx->time = t0 + n_steps * dt;
    int rc = update_geometry(ctx, ctx->time);
    return rc != PDG_OK ? rc : check_motion(ctx);
}

static int ensure_adjoint_buffers(pdg_ctx *ctx) {
    if (ctx->d_Lf) return PDG_OK;
    const size_t pts = (size_t)ctx->n_slots * ctx->n2;
    ctx->d_Lf = ctx->alloc<double>(pts * 5);
    if (ctx->ns) {
        ctx->d_Lw = ctx->alloc<double>(pts * 4);
        ctx->d_Ub = ctx->alloc<double>(ctx->n_doubles);
    }
    if (!ctx->d_Lf || (ctx->ns && (!ctx->d_Lw || !ctx->d_Ub))) {
        set_error("out of device memory");
        return PDG_ENOMEM;
    }
    return PDG_OK;
}

// the adjoint phases with the given workspace (Lf: slots*n2*5; NS also Lw: slots*n2*4, Ub: state)
static int run_adjoint_in(pdg_ctx *ctx, const double *U, const AdjArgs &base, double *Lf, double *Lw, double *Ub) {
    StageArgs sa = ctx->sa;
    sa.U = U;
    AdjArgs aa = base;
    aa.Lf = Lf;
    aa.Lw = Lw;
    aa.Ub = Ub;
    for (int ph = 0; ph < (ctx->ns ? 3 : 2); ++ph)
        for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_adjoint(ctx->N, ctx->ns, ph, sa, aa, t, ctx->stream));
    return PDG_OK;
}

static int run_adjoint(pdg_ctx *ctx, const double *U, const AdjArgs &base) {
    int rc = ensure_adjoint_buffers(ctx);
    if (rc != PDG_OK) return rc;
    return run_adjoint_in(ctx, U, base, ctx->d_Lf, ctx->d_Lw, ctx->d_Ub);
}

static int vjp_check(const pdg_ctx *ctx, const double *U, const double *cot, const double *grad_U) {
    if (!ctx || !U || !cot || !grad_U) { set_error("null argument"); return PDG_EINVAL; }
    if (grad_U == U || grad_U == cot) { set_error("grad_U must not alias U or cot"); return PDG_EINVAL; }
    if (!plain_form(ctx)) { set_error("the adjoint needs the weak form and the Lax-Friedrichs flux"); return PDG_ENOTSUP; }
    if (ctx->curved) { set_error("the adjoint takes affine elements only"); return PDG_ENOTSUP; }
    return PDG_OK;
}

static AdjArgs vjp_args(const double *cot, double *grad_U) {
    AdjArgs a{};
    a.Kb = cot;
    a.mode = 0;
    a.gout = grad_U;
    return a;
}

extern "C++" {
namespace pdg {
void adjoint_workspace(const pdg_ctx *ctx, size_t *lf, size_t *lw, size_t *ub) {
    const size_t pts = (size_t)ctx->n_slots * ctx->n2;
    *lf = pts * 5;
    *lw = ctx->ns ? pts * 4 : 0;
    *ub = ctx->ns ? (size_t)ctx->n_doubles : 0;
}

int context_device(const pdg_ctx *ctx) { return ctx->device; }

int vjp_in(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U, double *Lf, double *Lw, double *Ub) {
    int rc = vjp_check(ctx, U, cot, grad_U);
    if (rc != PDG_OK) return rc;
    return run_adjoint_in(ctx, U, vjp_args(cot, grad_U), Lf, Lw, Ub);
}
}  // namespace pdg
}

int pdg_vjp(pdg_ctx *ctx, const double *U, const double *cot, double *grad_U) {
    int rc = vjp_check(ctx, U, cot, grad_U);
    if (rc != PDG_OK) return rc;
    return run_adjoint(ctx, U, vjp_args(cot, grad_U));
}

int pdg_rk_stage(pdg_ctx *ctx, double *U, double *K, double dt, int32_t stage) {
    if (!ctx || !U || !K) { set_error("null argument"); return PDG_EINVAL; }
    if (U == K) { set_error("U and K must be distinct buffers"); return PDG_EINVAL; }
    if (stage < 0 || stage > 4 || !std::isfinite(dt)) { set_error("invalid stage or time step"); return PDG_EINVAL; }
    if (ctx->moving) { set_error("a moving mesh steps with pdg_rk_steps"); return PDG_ENOTSUP; }
    return run_stage(ctx, U, 1, nullptr, K, U, kRKA[stage], kRKB[stage] * dt);
}

int pdg_rk_stage_adjoint(pdg_ctx *ctx, const double *U_s, double *Ubar, double *Kbar, double dt, int32_t stage) {
    if (!ctx || !U_s || !Ubar || !Kbar) { set_error("null argument"); return PDG_EINVAL; }
    if (Ubar == Kbar || U_s == Ubar || U_s == Kbar) { set_error("U_s, Ubar and Kbar must be distinct buffers"); return PDG_EINVAL; }
    if (stage < 0 || stage > 4 || !std::isfinite(dt)) { set_error("invalid stage or time step"); return PDG_EINVAL; }
    if (!plain_form(ctx)) { set_error("the adjoint needs the weak form and the Lax-Friedrichs flux"); return PDG_ENOTSUP; }
    if (ctx->curved) { set_error("the adjoint takes affine elements only"); return PDG_ENOTSUP; }
    AdjArgs a{};
    a.Kb = Kbar;
    a.Ubr = Ubar;
    a.c = kRKB[stage] * dt;
    a.mode = 1;
    a.Ubar = Ubar;
    a.Kbar = Kbar;
    a.a = kRKA[stage];
    return run_adjoint(ctx, U_s, a);
}

int pdg_nodal_adjoint(pdg_ctx *ctx, const double *qbar, double *Ubar) {
    if (!ctx || !qbar || !Ubar) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_nodal_adjoint(ctx->N, ctx->sa, t, qbar, Ubar, ctx->stream));
    return PDG_OK;
}

int pdg_check_finite(pdg_ctx *ctx, const double *U, int64_t *first_bad) {
    if (!ctx || !U) { set_error("null argument"); return PDG_EINVAL; }
    if (first_bad) *first_bad = -1;
    if (!ctx->d_first_bad) {
        ctx->d_first_bad = ctx->alloc<unsigned long long>(1);
        if (!ctx->d_first_bad) { set_error("out of device memory"); return PDG_ENOMEM; }
    }
    unsigned long long v = (unsigned long long)ctx->n_doubles;
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    PDG_TRY_HIP(hipMemcpy(ctx->d_first_bad, &v, sizeof(v), hipMemcpyHostToDevice));
    PDG_TRY_HIP(launch_first_nonfinite(U, ctx->n_doubles, ctx->d_first_bad, ctx->stream));
    PDG_TRY_HIP(hipMemcpyAsync(&v, ctx->d_first_bad, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (v >= (unsigned long long)ctx->n_doubles) return PDG_OK;
    if (first_bad) *first_bad = (int64_t)v;
    set_error("non-finite state entry at stored index " + std::to_string(v));
    return PDG_ENONFINITE;
}

int pdg_node_weights(pdg_ctx *ctx, double *wJ) {
    if (!ctx || !wJ) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_node_weights(ctx->N, ctx->sa, t, wJ, ctx->stream));
    return PDG_OK;
}

int pdg_project(pdg_ctx *ctx, const double *q, double *U) {
    if (!ctx || !q || !U) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_project(ctx->N, ctx->sa, t, q, U, ctx->stream));
    return PDG_OK;
}

int pdg_nodal(pdg_ctx *ctx, const double *U, double *q) {
    if (!ctx || !q || !U) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_nodal(ctx->N, ctx->sa, t, U, q, ctx->stream));
    return PDG_OK;
}

int pdg_node_coords(pdg_ctx *ctx, double *xyz) {
    if (!ctx || !xyz) { set_error("null argument"); return PDG_EINVAL; }
    // host evaluation of the element map at the volume nodes (set-up path, not per stage)
    const int n = ctx->n, nn = ctx->nn, ne = ctx->n_elems;
    std::vector<double> corners((size_t)ne * 24);
    PDG_TRY_HIP(hipMemcpy(corners.data(), ctx->d_corners, corners.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (ctx->moving) {  // the corners at the context's time
        const double sn = std::sin(ctx->omega * ctx->time);
        for (size_t q = 0; q < corners.size(); ++q) corners[q] += sn * ctx->disp[q];
    }
    std::vector<double> out((size_t)ne * nn * 3);
    for (int i = 0; i < ne; ++i) {
        const TypeTables &tt = ctx->tt[ctx->etype[i]];
        const double *X = &corners[24 * (size_t)i];
        for (int k = 0; k < nn; ++k) {
            const double eta[3] = {tt.x[0][k % n], tt.x[1][(k / n) % n], tt.x[2][k / (n * n)]};
            double x[3] = {0, 0, 0};
            for (int c = 0; c < 8; ++c) {
                double Nc = 1.0;
                for (int a = 0; a < 3; ++a) Nc *= 0.5 * (1.0 + (((c >> a) & 1) ? 1.0 : -1.0) * eta[a]);
                for (int d = 0; d < 3; ++d) x[d] += Nc * X[3 * c + d];
            }
            for (int d = 0; d < 3; ++d) out[((size_t)i * nn + k) * 3 + d] = x[d];
        }
    }
    PDG_TRY_HIP(hipMemcpyAsync(xyz, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    return PDG_OK;
}

int pdg_sfc_keys(pdg_ctx *ctx, const double lo[3], double scale, uint64_t *keys) {
    if (!ctx || !lo || !keys) { set_error("null argument"); return PDG_EINVAL; }
    PDG_TRY_HIP(launch_sfc_keys(ctx->n_elems, ctx->d_centroid, lo, scale, keys, ctx->stream));
    return PDG_OK;
}

int pdg_partition(pdg_ctx *ctx, const uint32_t *weight, int32_t n_queues, int32_t *queue_begin) {
    if (!ctx || !weight || !queue_begin) { set_error("null argument"); return PDG_EINVAL; }
    if (n_queues <= 0) { set_error("n_queues must be positive"); return PDG_EINVAL; }
    PDG_TRY_HIP(launch_partition(ctx->n_elems, weight, n_queues, queue_begin, ctx->d_scan, ctx->stream));
    return PDG_OK;
}

int pdg_type_weights(pdg_ctx *ctx, const double cost_per_elem[4], uint32_t *weight, uint32_t weight_type[4]) {
    if (!ctx || !cost_per_elem || !weight) { set_error("null argument"); return PDG_EINVAL; }
    double ref = 0.0;
    for (int t = 0; t < 4; ++t) {
        const double c = cost_per_elem[t];
        if (!std::isfinite(c) || c < 0.0) { set_error("costs must be finite and non-negative"); return PDG_EINVAL; }
        if (c > 0.0 && (ref == 0.0 || c < ref)) ref = c;
    }
    if (ref == 0.0) { set_error("all costs are zero"); return PDG_EINVAL; }
    if (cost_per_elem[0] > 0.0) ref = cost_per_elem[0];
    uint32_t wt[4];
    for (int t = 0; t < 4; ++t)
        wt[t] = (uint32_t)std::min(16777216.0, std::max(1.0, std::nearbyint(1024.0 * cost_per_elem[t] / ref)));
    if (weight_type)
        for (int t = 0; t < 4; ++t) weight_type[t] = wt[t];
    PDG_TRY_HIP(launch_type_weights(ctx->n_elems, ctx->sa.mesh.etype, wt, weight, ctx->stream));
    return PDG_OK;
}

// clears the per-queue timers of the installed schedule (synchronous)
static int clear_queue_timers(pdg_ctx *ctx) {
    ctx->qt_evals = 0;
    if (ctx->n_queues <= 0) return PDG_OK;
    std::vector<uint64_t> z((size_t)3 * ctx->n_queues * ctx->qmax, 0);
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    PDG_TRY_HIP(hipMemcpy(ctx->d_qt, z.data(), z.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    return PDG_OK;
}

// installs a validated host schedule
static int install_schedule(pdg_ctx *ctx, const std::vector<int32_t> &qb) {
    const int32_t nq = (int32_t)qb.size() - 1;
    // workgroups per queue, per phase: as many as keep every CU at that phase's queue kernel
    // occupancy, all resident at once (a queue then has several elements in flight, like the
    // threads of one rank), at most 16
    int cus = 0, dev = 0;
    PDG_TRY_HIP(hipGetDevice(&dev));
    PDG_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int32_t qs[3], qsub = 1;
    for (int ph = 0; ph < 3; ++ph) {
        const int64_t resident = (int64_t)std::max(cus, 1) * queue_occupancy(ctx->N, ctx->ns, ph);
        qs[ph] = (int32_t)std::min<int64_t>(16, std::max<int64_t>(1, resident / std::max(nq, 1)));
        qsub = std::max(qsub, qs[ph]);
    }
    if (nq > ctx->qb_capacity) {
        ctx->d_qtb = ctx->alloc<int32_t>((size_t)4 * (nq + 1));
        ctx->d_qb_new = ctx->alloc<int32_t>(nq + 1);
        if (!ctx->d_qtb || !ctx->d_qb_new) { set_error("out of device memory"); return PDG_ENOMEM; }
        ctx->qb_capacity = nq;
    }
    if ((int64_t)nq * qsub > ctx->qt_capacity) {
        ctx->d_qt = ctx->alloc<uint64_t>((size_t)3 * nq * qsub);
        if (!ctx->d_qt) { set_error("out of device memory"); return PDG_ENOMEM; }
        ctx->qt_capacity = (int64_t)nq * qsub;
    }
    std::copy(qs, qs + 3, ctx->qsub);
    ctx->qmax = qsub;
    // the queue kernels take each segment type by type: the type-t elements of [qb[j], qb[j+1])
    // are tlist[t][qtb[4 j + t] .. qtb[4 (j + 1) + t]) (the type lists are in element order)
    std::vector<int32_t> qtb((size_t)4 * (nq + 1));
    for (int32_t j = 0; j <= nq; ++j)
        for (int t = 0; t < 4; ++t)
            qtb[(size_t)4 * j + t] = (int32_t)(std::lower_bound(ctx->tlist[t].begin(), ctx->tlist[t].end(), qb[j]) -
                                               ctx->tlist[t].begin());
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    PDG_TRY_HIP(hipMemcpy(ctx->d_qtb, qtb.data(), qtb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    ctx->h_qb = qb;
    ctx->n_queues = nq;
    return clear_queue_timers(ctx);
}

int pdg_set_schedule(pdg_ctx *ctx, const int32_t *queue_begin, int32_t n_queues) {
    if (!ctx) { set_error("null context"); return PDG_EINVAL; }
    if (n_queues == 0) { ctx->n_queues = 0; ctx->h_qb.clear(); ctx->qt_evals = 0; return PDG_OK; }
    if (n_queues < 0 || !queue_begin) { set_error("invalid queue schedule"); return PDG_EINVAL; }
    std::vector<int32_t> qb(n_queues + 1);
    PDG_TRY_HIP(hipMemcpyAsync(qb.data(), queue_begin, qb.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    const std::string err = check_schedule(ctx->n_elems, n_queues, qb.data());
    if (!err.empty()) { set_error(err); return PDG_EINVAL; }
    return install_schedule(ctx, qb);
}

int pdg_get_schedule(pdg_ctx *ctx, int32_t *queue_begin, int32_t *n_queues) {
    if (!ctx || !n_queues) { set_error("null argument"); return PDG_EINVAL; }
    *n_queues = ctx->n_queues;
    if (queue_begin && ctx->n_queues > 0) std::copy(ctx->h_qb.begin(), ctx->h_qb.end(), queue_begin);
    return PDG_OK;
}

// per-phase, per-queue milliseconds accumulated by the queue kernels: the mean over each
// queue's workgroups (they share its elements round-robin), proportional to the queue's work
static int read_queue_ms(pdg_ctx *ctx, std::vector<double> &ms) {
    const size_t nq = (size_t)ctx->n_queues, qmax = (size_t)ctx->qmax;
    std::vector<uint64_t> ticks(3 * nq * qmax);
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    PDG_TRY_HIP(hipMemcpy(ticks.data(), ctx->d_qt, ticks.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    PDG_TRY_HIP(hipGetDevice(&dev));
    PDG_TRY_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) { set_error("device wall-clock rate unavailable"); return PDG_EHIP; }
    ms.assign(3 * nq, 0.0);
    for (size_t ph = 0; ph < 3; ++ph)
        for (size_t q = 0; q < nq; ++q) {
            uint64_t sum = 0;
            const size_t qsub = (size_t)ctx->qsub[ph];
            for (size_t s = 0; s < qsub; ++s) sum += ticks[ph * nq * qmax + q * qsub + s];
            ms[ph * nq + q] = (double)sum / qsub / khz;
        }
    return PDG_OK;
}

int pdg_queue_times(pdg_ctx *ctx, double *queue_ms, int32_t reset, int64_t *n_evals) {
    if (!ctx) { set_error("null context"); return PDG_EINVAL; }
    if (ctx->n_queues <= 0) { set_error("no work-queue schedule installed"); return PDG_EINVAL; }
    if (n_evals) *n_evals = ctx->qt_evals;
    if (queue_ms) {
        std::vector<double> ms;
        const int rc = read_queue_ms(ctx, ms);
        if (rc != PDG_OK) return rc;
        std::copy(ms.begin(), ms.end(), queue_ms);
    }
    return reset ? clear_queue_timers(ctx) : PDG_OK;
}

int pdg_balance_weights(int32_t n_elems, const int8_t *elem_type, int32_t n_queues, const int32_t *queue_begin,
                        const double *queue_ms, uint32_t *weight, double type_cost[12], double *imbalance) {
    if (!elem_type || !queue_begin || !queue_ms || !weight) { set_error("null argument"); return PDG_EINVAL; }
    if (n_elems <= 0) { set_error("n_elems must be positive"); return PDG_EINVAL; }
    const std::string err = check_schedule(n_elems, n_queues, queue_begin);
    if (!err.empty()) { set_error(err); return PDG_EINVAL; }
    for (int32_t e = 0; e < n_elems; ++e)
        if (elem_type[e] < 0 || elem_type[e] > 3) { set_error("element type out of range"); return PDG_EINVAL; }
    double tot = 0.0;
    for (size_t i = 0; i < (size_t)3 * n_queues; ++i) {
        if (!(queue_ms[i] >= 0.0) || !std::isfinite(queue_ms[i])) {
            set_error("queue times must be finite and non-negative");
            return PDG_EINVAL;
        }
        tot += queue_ms[i];
    }
    if (!(tot > 0.0)) { set_error("no queue time recorded"); return PDG_EINVAL; }
    std::vector<double> cost;
    double tc[12];
    attribute_costs(n_elems, elem_type, n_queues, queue_begin, queue_ms, cost, tc);
    cost_weights(n_elems, cost, weight);
    if (type_cost) std::copy(tc, tc + 12, type_cost);
    if (imbalance) *imbalance = queue_imbalance(std::vector<double>(queue_ms, queue_ms + 3 * (size_t)n_queues),
                                                n_queues);
    return PDG_OK;
}

int pdg_rebalance(pdg_ctx *ctx, double threshold, double info[4]) {
    if (!ctx || !info) { set_error("null argument"); return PDG_EINVAL; }
    if (ctx->n_queues <= 0) { set_error("no work-queue schedule installed"); return PDG_EINVAL; }
    if (!(threshold >= 0.0)) { set_error("threshold must be non-negative"); return PDG_EINVAL; }
    const int32_t n = ctx->n_elems, nq = ctx->n_queues;
    std::vector<double> ms;
    int rc = read_queue_ms(ctx, ms);
    if (rc != PDG_OK) return rc;
    double tot = 0.0;
    for (double v : ms) tot += v;
    if (!(tot > 0.0) || ctx->qt_evals == 0) { set_error("no queue time recorded since the last reset"); return PDG_EINVAL; }
    const double before = queue_imbalance(ms, nq);
    info[0] = before;
    info[1] = before;
    info[2] = 0.0;
    info[3] = (double)ctx->qt_evals;
    if (before <= threshold) return clear_queue_timers(ctx);
    std::vector<double> cost;
    double tc[12];
    attribute_costs(n, ctx->etype.data(), nq, ctx->h_qb.data(), ms.data(), cost, tc);
    std::vector<uint32_t> w(n);
    cost_weights(n, cost, w.data());
    if (!ctx->d_weight) {
        ctx->d_weight = ctx->alloc<uint32_t>(n);
        if (!ctx->d_weight) { set_error("out of device memory"); return PDG_ENOMEM; }
    }
    PDG_TRY_HIP(hipMemcpyAsync(ctx->d_weight, w.data(), (size_t)n * sizeof(uint32_t), hipMemcpyHostToDevice,
                               ctx->stream));
    PDG_TRY_HIP(launch_partition(n, ctx->d_weight, nq, ctx->d_qb_new, ctx->d_scan, ctx->stream));
    std::vector<int32_t> qb(nq + 1);
    PDG_TRY_HIP(hipMemcpyAsync(qb.data(), ctx->d_qb_new, qb.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    const std::string err = check_schedule(n, nq, qb.data());
    if (!err.empty()) { set_error("rebalance partition invalid: " + err); return PDG_EHIP; }
    info[1] = queue_imbalance(queue_loads(n, cost, nq, qb.data()), nq);
    info[2] = 1.0;
    return install_schedule(ctx, qb);
}

int pdg_measure_costs(pdg_ctx *ctx, const double *U, int32_t reps, double cost_per_elem[4], double phase_ms[12]) {
    if (!ctx || !U || !cost_per_elem || reps <= 0) { set_error("invalid argument"); return PDG_EINVAL; }
    if (!ctx->d_scratch_out) {
        ctx->d_scratch_out = ctx->alloc<double>(ctx->n_doubles);
        if (!ctx->d_scratch_out) { set_error("out of device memory"); return PDG_ENOMEM; }
    }
    StageArgs sa = ctx->sa;
    sa.U = U; sa.mode = 0; sa.out = ctx->d_scratch_out;
    // one event pair per (phase, type); every launch is bracketed on the context stream
    struct Events {
        hipEvent_t e[3][4][2];
        bool ok = true;
        Events() {
            for (auto &a : e) for (auto &b : a) for (auto &c : b) ok = ok && hipEventCreate(&c) == hipSuccess;
        }
        ~Events() {
            for (auto &a : e) for (auto &b : a) for (auto &c : b) (void)hipEventDestroy(c);
        }
    } ev;
    if (!ev.ok) { set_error("hipEventCreate failed"); return PDG_EHIP; }
    double acc[3][4] = {};
    for (int r = 0; r <= reps; ++r) {  // r = 0 warms up
        for (int ph = 0; ph < 3; ++ph)
            for (int t = 0; t < 4; ++t) {
                PDG_TRY_HIP(hipEventRecord(ev.e[ph][t][0], ctx->stream));
                if (ph == 0) PDG_TRY_HIP(launch_trace(ctx->N, sa, t, ctx->stream));
                if (ph == 1) PDG_TRY_HIP(launch_volume_form(ctx, sa, t));
                if (ph == 2) PDG_TRY_HIP(launch_surface_flux(ctx, sa, t));
                PDG_TRY_HIP(hipEventRecord(ev.e[ph][t][1], ctx->stream));
            }
        PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
        if (r == 0) continue;
        for (int ph = 0; ph < 3; ++ph)
            for (int t = 0; t < 4; ++t) {
                float ms = 0;
                PDG_TRY_HIP(hipEventElapsedTime(&ms, ev.e[ph][t][0], ev.e[ph][t][1]));
                acc[ph][t] += ms;
            }
    }
    for (int t = 0; t < 4; ++t) {
        double tot = 0.0;
        for (int ph = 0; ph < 3; ++ph) tot += acc[ph][t] / reps;
        cost_per_elem[t] = ctx->sa.count[t] ? 1e-3 * tot / ctx->sa.count[t] : 0.0;
    }
    if (phase_ms)
        for (int ph = 0; ph < 3; ++ph)
            for (int t = 0; t < 4; ++t) phase_ms[ph * 4 + t] = acc[ph][t] / reps;
    return PDG_OK;
}

int pdg_timing_start(pdg_ctx *ctx) {
    if (!ctx) { set_error("null context"); return PDG_EINVAL; }
    ctx->timing = true;
    ctx->ev_used = 0;
    ctx->ev_slot.clear();
    return PDG_OK;
}

int pdg_timing_stop(pdg_ctx *ctx, double total_ms[12], int32_t launches[12]) {
    if (!ctx || !total_ms || !launches) { set_error("null argument"); return PDG_EINVAL; }
    ctx->timing = false;
    for (int i = 0; i < 12; ++i) { total_ms[i] = 0.0; launches[i] = 0; }
    PDG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < ctx->ev_used; ++i) {
        float ms = 0.0f;
        PDG_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev_pool[2 * i], ctx->ev_pool[2 * i + 1]));
        total_ms[ctx->ev_slot[i]] += ms;
        launches[ctx->ev_slot[i]] += 1;
    }
    ctx->ev_used = 0;
    ctx->ev_slot.clear();
    return PDG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Batched form: many independent contexts advanced with one graph launch per LSERK step
// ------------------------------------------------------------------------------------------
struct pdg_batch {
    struct Group {
        int type = 0, N = 0;
        bool ns = false;
        bool cv = false;              // the problems have curved elements
        int mesh = -1;                // -1: every merged problem of this (type, N, equations, cv)
        std::vector<BatchItem> items;
        BatchItem *d_items = nullptr;
    };
    std::vector<pdg_ctx *> ctx;
    hipStream_t stream = nullptr;     // caller's stream (graph launches)
    hipStream_t cap = nullptr;        // library stream used for capture
    int32_t tile[4][kMaxN + 1] = {};  // elements per workgroup for each (type, N)
    // problems with at least solo_min elements run their three phases back to back on their own
    // (one element per workgroup), the others are merged per (type, N, equations)
    int32_t solo_min = INT32_MAX;
    std::vector<Group> groups;
    StageArgs *d_args = nullptr;      // [6][n]: stages 0..4 of an LSERK step, then a residual
    std::vector<StageArgs> h_args;
    std::vector<const void *> cur;    // U, K of the arguments in d_args
    std::vector<double> cur_dt;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> allocs;

    ~pdg_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (void *p : allocs) (void)hipFree(p);
    }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

static bool batch_solo(const pdg_batch *b, int32_t i) { return b->ctx[i]->n_elems >= b->solo_min; }

// the launch groups: one per (type, N, equations, curved) over the merged problems, and one per
// type of every solo problem
static void batch_make_groups(pdg_batch *b) {
    for (auto &g : b->groups)
        if (g.d_items) {
            (void)hipFree(g.d_items);
            b->allocs.erase(std::find(b->allocs.begin(), b->allocs.end(), (void *)g.d_items));
        }
    b->groups.clear();
    for (int32_t i = 0; i < (int32_t)b->ctx.size(); ++i) {
        if (!batch_solo(b, i)) continue;
        for (int t = 0; t < 4; ++t)
            if (b->ctx[i]->sa.count[t] > 0) {
                pdg_batch::Group g;
                g.type = t;
                g.N = b->ctx[i]->N;
                g.ns = b->ctx[i]->ns;
                g.cv = b->ctx[i]->curved;
                g.mesh = i;
                b->groups.push_back(g);
            }
    }
    for (int t = 0; t < 4; ++t)
        for (int N = 2; N <= kMaxN; ++N)
            for (int ns = 0; ns < 2; ++ns)
                for (int cv = 0; cv < 2; ++cv) {
                    bool any = false;
                    for (int32_t i = 0; i < (int32_t)b->ctx.size(); ++i) {
                        const pdg_ctx *c = b->ctx[i];
                        any |= !batch_solo(b, i) && c->N == N && (int)c->ns == ns && (int)c->curved == cv &&
                               c->sa.count[t] > 0;
                    }
                    if (any) {
                        pdg_batch::Group g;
                        g.type = t;
                        g.N = N;
                        g.ns = ns;
                        g.cv = cv;
                        b->groups.push_back(g);
                    }
                }
}

static int batch_build_items(pdg_batch *b) {
    batch_make_groups(b);
    for (auto &g : b->groups) {
        g.items.clear();
        const int L = g.mesh >= 0 ? 1 : std::max(1, b->tile[g.type][g.N]);
        for (int32_t i = 0; i < (int32_t)b->ctx.size(); ++i) {
            const pdg_ctx *c = b->ctx[i];
            if (c->N != g.N || c->ns != g.ns || c->curved != g.cv) continue;
            if (g.mesh >= 0 ? i != g.mesh : batch_solo(b, i)) continue;
            const int32_t cnt = c->sa.count[g.type];
            for (int32_t f = 0; f < cnt; f += L) g.items.push_back({i, f, std::min<int32_t>(L, cnt - f)});
        }
        if (g.d_items) {
            (void)hipFree(g.d_items);
            b->allocs.erase(std::find(b->allocs.begin(), b->allocs.end(), (void *)g.d_items));
            g.d_items = nullptr;
        }
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(1, g.items.size()) * sizeof(BatchItem)) != hipSuccess) {
            set_error("out of device memory");
            return PDG_ENOMEM;
        }
        b->allocs.push_back(p);
        g.d_items = (BatchItem *)p;
        if (!g.items.empty())
            PDG_TRY_HIP(hipMemcpy(g.d_items, g.items.data(), g.items.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
    }
    b->drop_graph();
    return PDG_OK;
}

// arguments of every mesh for the five stages (mode 1) and for a plain residual into each
// context's scratch output (slot 5, used by the autotuner)
static int batch_set_args(pdg_batch *b, double *const *U, double *const *K, const double *dt) {
    const size_t n = b->ctx.size();
    bool same = b->cur.size() == 2 * n;
    for (size_t i = 0; same && i < n; ++i)
        same = b->cur[2 * i] == U[i] && b->cur[2 * i + 1] == K[i] && b->cur_dt[i] == dt[i];
    if (same) return PDG_OK;
    b->h_args.assign(6 * n, StageArgs{});
    for (size_t i = 0; i < n; ++i) {
        pdg_ctx *c = b->ctx[i];
        if (!c->d_scratch_out) {
            c->d_scratch_out = c->alloc<double>(c->n_doubles);
            if (!c->d_scratch_out) { set_error("out of device memory"); return PDG_ENOMEM; }
        }
        for (int s = 0; s < 6; ++s) {
            StageArgs a = c->sa;
            a.U = U[i];
            if (s < 5) {
                a.mode = 1;
                a.out = nullptr;
                a.K = K[i];
                a.Uw = U[i];
                a.rk_a = kRKA[s];
                a.rk_bdt = kRKB[s] * dt[i];
            } else {
                a.mode = 0;
                a.out = c->d_scratch_out;
            }
            b->h_args[s * n + i] = a;
        }
    }
    // the previous graph launches may still read the argument array
    PDG_TRY_HIP(hipStreamSynchronize(b->stream));
    PDG_TRY_HIP(hipMemcpy(b->d_args, b->h_args.data(), b->h_args.size() * sizeof(StageArgs), hipMemcpyHostToDevice));
    // solo problems take their arguments by value: the captured graph holds the old ones
    for (size_t i = 0; i < n; ++i)
        if (batch_solo(b, (int32_t)i)) { b->drop_graph(); break; }
    b->cur.resize(2 * n);
    b->cur_dt.assign(dt, dt + n);
    for (size_t i = 0; i < n; ++i) {
        b->cur[2 * i] = U[i];
        b->cur[2 * i + 1] = K[i];
    }
    return PDG_OK;
}

// one stage: every solo problem's three phases back to back through the per-type kernels of
// the plain stepping, with the stage's arguments by value (its traces stay in cache between the
// phases), then the merged groups phase by phase
static int batch_launch_stage(pdg_batch *b, int slot, hipStream_t s) {
    const size_t n = b->ctx.size();
    size_t gi = 0;
    while (gi < b->groups.size() && b->groups[gi].mesh >= 0) {
        const int i = b->groups[gi].mesh;
        const pdg_ctx *c = b->ctx[i];
        const StageArgs &sa = b->h_args[slot * n + i];
        for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_trace(c->N, sa, t, s));
        for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_volume(c->N, c->ns, sa, t, s));
        for (int t = 0; t < 4; ++t) PDG_TRY_HIP(launch_surface(c->N, c->ns, sa, t, s));
        while (gi < b->groups.size() && b->groups[gi].mesh == i) ++gi;
    }
    for (int ph = 0; ph < 3; ++ph)
        for (size_t k = gi; k < b->groups.size(); ++k) {
            const auto &g = b->groups[k];
            PDG_TRY_HIP(launch_batch_phase(g.type, g.N, g.ns, g.cv, ph, b->d_args + slot * n, g.d_items,
                                           (int)g.items.size(), s));
        }
    return PDG_OK;
}

extern "C" {

int pdg_batch_create(pdg_ctx *const *ctxs, int32_t n, void *hip_stream, pdg_batch **out) {
    if (!ctxs || n <= 0 || !out) { set_error("invalid batch arguments"); return PDG_EINVAL; }
    *out = nullptr;
    pdg_batch *b = new (std::nothrow) pdg_batch();
    if (!b) { set_error("out of host memory"); return PDG_ENOMEM; }
    b->stream = (hipStream_t)hip_stream;
    for (int32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) { delete b; set_error("null context in batch"); return PDG_EINVAL; }
        if (!plain_form(ctxs[i])) {
            delete b;
            set_error("the batched form needs the weak form and the Lax-Friedrichs flux");
            return PDG_ENOTSUP;
        }
        if (ctxs[i]->moving) {
            delete b;
            set_error("the batched form takes fixed meshes only (each stage of a moving mesh needs its own geometry)");
            return PDG_ENOTSUP;
        }
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) { delete b; set_error("a context appears twice in the batch"); return PDG_EINVAL; }
        b->ctx.push_back(ctxs[i]);
    }
    for (int t = 0; t < 4; ++t)
        for (int N = 0; N <= kMaxN; ++N) b->tile[t][N] = 1;
    void *p = nullptr;
    if (hipMalloc(&p, 6 * (size_t)n * sizeof(StageArgs)) != hipSuccess) { delete b; set_error("out of device memory"); return PDG_ENOMEM; }
    b->allocs.push_back(p);
    b->d_args = (StageArgs *)p;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) { delete b; set_error("stream creation failed"); return PDG_EHIP; }
    int rc = batch_build_items(b);
    if (rc != PDG_OK) { delete b; return rc; }
    *out = b;
    return PDG_OK;
}

void pdg_batch_destroy(pdg_batch *b) { delete b; }

int pdg_batch_set_tiles(pdg_batch *b, const int32_t *tiles) {
    if (!b || !tiles) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t)
        for (int N = 2; N <= kMaxN; ++N)
            if (tiles[t * (kMaxN + 1) + N] < 1 || tiles[t * (kMaxN + 1) + N] > 64) { set_error("tile sizes must be in 1..64"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t)
        for (int N = 0; N <= kMaxN; ++N) b->tile[t][N] = std::max(1, tiles[t * (kMaxN + 1) + N]);
    return batch_build_items(b);
}

int pdg_batch_set_solo(pdg_batch *b, int32_t min_elems) {
    if (!b) { set_error("null argument"); return PDG_EINVAL; }
    if (min_elems < 0) { set_error("min_elems must be non-negative"); return PDG_EINVAL; }
    b->solo_min = min_elems;
    return batch_build_items(b);
}

int pdg_batch_get_solo(const pdg_batch *b, int32_t *min_elems) {
    if (!b || !min_elems) { set_error("null argument"); return PDG_EINVAL; }
    *min_elems = b->solo_min;
    return PDG_OK;
}

int pdg_batch_get_tiles(const pdg_batch *b, int32_t *tiles) {
    if (!b || !tiles) { set_error("null argument"); return PDG_EINVAL; }
    for (int t = 0; t < 4; ++t)
        for (int N = 0; N <= kMaxN; ++N) tiles[t * (kMaxN + 1) + N] = b->tile[t][N];
    return PDG_OK;
}

int pdg_batch_rk_steps(pdg_batch *b, double *const *U, double *const *K, const double *dt, int32_t n_steps) {
    if (!b || !U || !K || !dt) { set_error("null argument"); return PDG_EINVAL; }
    if (n_steps < 0) { set_error("negative step count"); return PDG_EINVAL; }
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        if (!U[i] || !K[i] || U[i] == K[i] || !std::isfinite(dt[i])) { set_error("invalid state buffers or time step"); return PDG_EINVAL; }
        if (b->ctx[i]->moving) { set_error("a context of the batch was set in motion after the batch was made"); return PDG_ENOTSUP; }
    }
    if (n_steps == 0) return PDG_OK;
    int rc = batch_set_args(b, U, K, dt);
    if (rc != PDG_OK) return rc;
    if (!b->exec) {
        PDG_TRY_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        for (int s = 0; s < 5; ++s) {
            rc = batch_launch_stage(b, s, b->cap);
            if (rc != PDG_OK) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->cap, &g);
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
        }
        PDG_TRY_HIP(hipStreamEndCapture(b->cap, &b->graph));
        PDG_TRY_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    for (int32_t s = 0; s < n_steps; ++s) PDG_TRY_HIP(hipGraphLaunch(b->exec, b->stream));
    return PDG_OK;
}

int pdg_batch_autotune(pdg_batch *b, double *const *U, double *const *K, const double *dt, int32_t reps,
                       int32_t *tiles_out) {
    if (!b || !U || !K || !dt) { set_error("null argument"); return PDG_EINVAL; }
    for (pdg_ctx *c : b->ctx)
        if (c->moving) { set_error("a context of the batch was set in motion after the batch was made"); return PDG_ENOTSUP; }
    int rc = batch_set_args(b, U, K, dt);
    if (rc != PDG_OK) return rc;
    reps = std::max(1, reps);
    const size_t n = b->ctx.size();
    hipEvent_t e0, e1;
    PDG_TRY_HIP(hipEventCreate(&e0));
    PDG_TRY_HIP(hipEventCreate(&e1));
    // one full residual so that every trace buffer holds valid values
    rc = batch_launch_stage(b, 5, b->stream);
    // tiles of the merged groups, with every problem merged
    b->solo_min = INT32_MAX;
    rc = batch_build_items(b);
    static const int cand[] = {1, 2, 4, 8};
    for (size_t gi = 0; rc == PDG_OK && gi < b->groups.size(); ++gi) {
        if (b->groups[gi].mesh >= 0) continue;
        const int gt = b->groups[gi].type, gN = b->groups[gi].N;
        float best = 0.0f;
        int best_L = 1;
        for (int L : cand) {
            b->tile[gt][gN] = L;
            rc = batch_build_items(b);  // rebuilds the groups in the same order
            if (rc != PDG_OK) break;
            const auto &g = b->groups[gi];
            float ms = 0.0f;
            for (int r = 0; r <= reps && rc == PDG_OK; ++r) {  // r = 0 warms up
                if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = PDG_EHIP; break; }
                for (int ph = 0; ph < 3; ++ph)
                    if (launch_batch_phase(g.type, g.N, g.ns, g.cv, ph, b->d_args + 5 * n, g.d_items, (int)g.items.size(),
                                           b->stream) != hipSuccess) { rc = PDG_EHIP; break; }
                if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = PDG_EHIP; break; }
                float t = 0.0f;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (r > 0) ms += t;
            }
            if (rc != PDG_OK) break;
            if (L == 1 || ms < 0.97f * best) { best = ms; best_L = L; }  // a larger tile must win clearly
        }
        b->tile[gt][gN] = best_L;
    }
    // which problems run alone: every problem with at least solo_min elements, timed over whole
    // residuals for a few thresholds (all merged first; a threshold must win by 3 %)
    static const int32_t solo_cand[] = {INT32_MAX, 65536, 16384, 4096, 0};
    float best_solo = 0.0f;
    int32_t best_min = INT32_MAX;
    for (int32_t sm : solo_cand) {
        if (rc != PDG_OK) break;
        b->solo_min = sm;
        rc = batch_build_items(b);
        if (rc != PDG_OK) break;
        float ms = 0.0f;
        for (int r = 0; r <= reps && rc == PDG_OK; ++r) {
            if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = PDG_EHIP; break; }
            if (batch_launch_stage(b, 5, b->stream) != PDG_OK) { rc = PDG_EHIP; break; }
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = PDG_EHIP; break; }
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (r > 0) ms += t;
        }
        if (rc != PDG_OK) break;
        if (sm == INT32_MAX || ms < 0.97f * best_solo) { best_solo = ms; best_min = sm; }
    }
    b->solo_min = best_min;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PDG_OK) { if (rc == PDG_EHIP) set_error("HIP error during autotuning"); return rc; }
    rc = batch_build_items(b);
    if (rc != PDG_OK) return rc;
    if (tiles_out) return pdg_batch_get_tiles(b, tiles_out);
    return PDG_OK;
}

}  // extern "C"
