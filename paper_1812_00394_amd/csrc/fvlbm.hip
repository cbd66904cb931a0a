// C ABI of the FVLBM library: state layout in the caller's workspace, the step driver and the
// import / export / reduction entry points.  See include/fvlbm.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "adjoint.h"
#include "kernels.h"
#include "pair.h"

namespace fvlbm {

fvlbm_mesh *build_mesh(int64_t n_nodes, const double *xy, int64_t n_cells, const int64_t *cell_ptr,
                       const int64_t *cell_nodes, int64_t n_bf, const int64_t *bf_nodes, const int32_t *bf_group,
                       int32_t n_groups, const int32_t *group_kind, const double *pshift, int32_t order);

namespace {
thread_local std::string g_last_error;

void check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw Error(FVLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kBlock = 256;
constexpr int kRedBlocks = 512;   // fixed reduction grid (deterministic sums)
constexpr int kMaxSstSweeps = 1000;
// the adjoint reverses the implicit SST variant for at most this many sweeps (it keeps every
// sweep's increments)
constexpr int kMaxAdjSstSweeps = 16;

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// Carves the caller's workspace: every array 256-byte aligned.
struct Carver {
    size_t off = 0;
    char *base = nullptr;
    template <typename P>
    P *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        P *p = base ? reinterpret_cast<P *>(base + off) : nullptr;
        off += count * sizeof(P);
        return p;
    }
};

}  // namespace

void set_last_error(const std::string &msg) { g_last_error = msg; }

}  // namespace fvlbm


using namespace fvlbm;

// ---- the reduction buffer of fvlbm_totals_noalloc: device memory the library holds itself ----
// One per GPU the library runs on, for the whole process: 16 KiB, of which the per-block partial
// sums of the fixed reduction grid (kRedBlocks blocks x 3 sums) use 12 KiB.  In host code the array's name is a host-side
// stand-in, not a device address: its device address is looked up once per device (when a state is
// created on it) and kept in g_scratch_dev; host code uses only that address.
namespace {
constexpr size_t kNoAllocScratchDoubles = 2048;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on `dev` (which must be the current device), looked up once.
double *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw Error(FVLBM_EDEVICE, "device index out of range for the reduction buffer");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_dev[dev];
}
}  // namespace

struct fvlbm_state {
    const fvlbm_mesh *mesh = nullptr;
    int precision = FVLBM_FP64;
    int sst = 0;
    fvlbm_params par{};
    hipStream_t stream = nullptr;
    Geo<double> geo64{};
    Geo<float> geo32{};
    int32_t n_cells = 0;
    int device = 0;              // the HIP device current when the state was created
    double *noalloc = nullptr;   // that device's reduction buffer of fvlbm_totals_noalloc
    int32_t *bzg = nullptr;
    void *F = nullptr, *X = nullptr, *Y = nullptr, *A = nullptr, *G = nullptr;
    void *M[2] = {nullptr, nullptr};
    void *K[2] = {nullptr, nullptr}, *W[2] = {nullptr, nullptr};
    void *tau = nullptr, *nut = nullptr, *aux = nullptr;
    void *tau3 = nullptr;        // the third stage's relaxation time (per-stage SST)
    void *aux2 = nullptr;        // while a recorded step runs with the per-stage SST: its second solve's aux planes
    int sst_stages = 0;          // the SST is solved before every stage (params.sst = 2)
    int cur_m = 0, cur_kw = 0;
    // tiles of the fused stage kernels: ring (extended halo lists), tiled (ring 1 only, with or
    // without the stage values in LDS) or the two-kernel split path
    bool ring = true, tiled = true, tile_vals = true;
    bool face = false;           // the edge loop with atomics (FVLBM_SWEEP=face)
    bool pair = false;           // the ring-tiled stage sweeps with two threads per cell (k_stage_pair)
    bool fp64_geometry = false;  // FP32 state whose ring sweeps form the edge data from FP64 geometry
    int32_t n_faces = 0;         // interior edges, each once
    int32_t *faces = nullptr;    // [n_faces] face codes 4 c + s
    void *acc = nullptr;         // [8][n] outflow sums of the edge loop
    int ring_s = 4, ring_wv = 0, ring_wg = 0;
    size_t sst_lds_bytes = 0;
    bool want_aux = false;       // the SST launch also stores the aux planes (adjoint recompute)
    void *F_out = nullptr;       // where a step writes f^{n+1} (nullptr: over f^n)
    uint64_t *clip = nullptr;    // while a recorded step runs with the r32 limiter: its clip states [3][n]
    int held_segs = 0;           // trailing segments of the recorded run whose tapes the segment buffers hold
    int32_t *hptr = nullptr, *hcell = nullptr;
    int32_t *xptr = nullptr, *xn1 = nullptr, *xcell = nullptr;
    int16_t *xlnb = nullptr;
    int16_t *lnb = nullptr;
    int8_t *rev = nullptr;
    void *scr1 = nullptr;        // one n-array of T for diagnostics
    int tile_w = 0;
    size_t lds_bytes = 0;
    double *scratch = nullptr;   // 9 n doubles (staging of user-order FP64 arrays)
    double *partial = nullptr;   // kRedBlocks * 4
    double *result = nullptr;    // 4
    int64_t steps_done = 0;
    // record / adjoint (fvlbm_record, fvlbm_adjoint_step)
    char *adj_ws = nullptr;
    size_t adj_bytes = 0;
    int32_t rec_steps = 0, rec_ckpt = 0;
    // the reverse recomputes the next segment on a second stream while it reverses the current one
    hipStream_t side = nullptr;
    hipEvent_t ev_rev = nullptr, ev_rec = nullptr;
    bool adj_two_sets = false;   // the recorded workspace holds the second set of segment buffers
    // per-kernel event timing (fvlbm_timing)
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
    size_t pool_used = 0;
    double t_ms[FVLBM_K_COUNT] = {};
    int64_t t_count[FVLBM_K_COUNT] = {};
    ~fvlbm_state() {
        for (auto &e : event_pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (ev_rev) (void)hipEventDestroy(ev_rev);
        if (ev_rec) (void)hipEventDestroy(ev_rec);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace {

template <typename T>
Geo<T> &geo_of(fvlbm_state *st);
template <>
Geo<double> &geo_of<double>(fvlbm_state *st) { return st->geo64; }
template <>
Geo<float> &geo_of<float>(fvlbm_state *st) { return st->geo32; }

// Interior edges, each once, in cell order: slot s of cell c with neighbour c' > c (face code
// 4 c + s).  A periodic edge joining a cell to itself does not occur (it would need a period of one
// cell).
std::vector<int32_t> face_list(const fvlbm_mesh *m) {
    std::vector<int32_t> f;
    const int64_t n = m->n;
    f.reserve((size_t)(2 * n));
    for (int64_t c = 0; c < n; ++c)
        for (int s = 0; s < kSlots; ++s) {
            const int32_t nb = m->nbr[(size_t)s * n + c];
            if (nb > c) f.push_back((int32_t)(4 * c + s));
        }
    return f;
}

// Layout of the workspace.  Geometry arrays are written by fvlbm_init; the rest is state.
template <typename T>
void carve(Carver &cv, const fvlbm_mesh *m, int sst, fvlbm_state *st, bool geo64 = false) {
    const size_t n = (size_t)m->n, nb = m->b_cell.size(), S = kSlots * n;
    Geo<T> &g = geo_of<T>(st);
    st->n_cells = (int32_t)n;
    g.n = (int32_t)n;
    g.nb = (int32_t)nb;
    g.nbr = cv.take<int32_t>(S);
    g.nlx = cv.take<T>(S);
    g.nly = cv.take<T>(S);
    g.rfx = cv.take<T>(S);
    g.rfy = cv.take<T>(S);
    g.qx = cv.take<T>(S);
    g.qy = cv.take<T>(S);
    g.cx = cv.take<T>(S);
    g.cy = cv.take<T>(S);
    g.area = cv.take<double>(n);
    g.inv_area = cv.take<T>(n);
    g.mi = cv.take<T>(3 * n);
    g.tp = cv.take<T>(6 * n);
    g.bfirst = cv.take<int32_t>(n);
    g.wdist = cv.take<double>(n);
    g.perm = cv.take<int32_t>(n);
    g.b_kind = cv.take<int32_t>(nb);
    g.b_cell = cv.take<int32_t>(nb);
    g.b_group = cv.take<int32_t>(nb);
    st->bzg = cv.take<int32_t>(nb);
    g.b_nx = cv.take<double>(nb);
    g.b_ny = cv.take<double>(nb);
    g.b_l = cv.take<double>(nb);
    g.b_dperp = cv.take<double>(nb);
    g.b_xfx = cv.take<double>(nb);
    g.b_ux = cv.take<double>(nb);
    g.b_uy = cv.take<double>(nb);
    g.b_rho = cv.take<double>(nb);
    g.b_drho = cv.take<double>(nb);
    g.b_k = cv.take<double>(nb);
    g.b_w = cv.take<double>(nb);
    st->F = cv.take<T>(9 * n);
    st->X = cv.take<T>(9 * n);
    st->Y = cv.take<T>(9 * n);
    st->A = cv.take<T>(9 * n);
    st->G = cv.take<T>(16 * n);
    st->M[0] = cv.take<T>(3 * n);
    st->M[1] = cv.take<T>(3 * n);
    st->tau = cv.take<T>(n);
    st->nut = cv.take<T>(n);
    if (sst) {
        st->K[0] = cv.take<T>(n);
        st->K[1] = cv.take<T>(n);
        st->W[0] = cv.take<T>(n);
        st->W[1] = cv.take<T>(n);
        st->aux = cv.take<T>(15 * n);
        st->tau3 = cv.take<T>(n);
    }
    st->lnb = cv.take<int16_t>(S);
    st->rev = cv.take<int8_t>(S);
    st->scr1 = cv.take<T>(n);
    st->hptr = cv.take<int32_t>((size_t)m->n_tiles + 1);
    st->hcell = cv.take<int32_t>(std::max<size_t>(1, m->halo_cell.size()));
    st->xptr = cv.take<int32_t>((size_t)m->n_tiles + 1);
    st->xn1 = cv.take<int32_t>((size_t)m->n_tiles);
    st->xcell = cv.take<int32_t>(std::max<size_t>(1, m->ext_cell.size()));
    st->xlnb = cv.take<int16_t>(kSlots * std::max<size_t>(1, m->ext_cell.size()));
    st->scratch = cv.take<double>(9 * n);
    st->partial = cv.take<double>((size_t)kRedBlocks * 4);
    st->result = cv.take<double>(4);
    st->n_faces = (int32_t)m->n_interior_edges;
    st->faces = cv.take<int32_t>(std::max<size_t>(1, (size_t)m->n_interior_edges));
    st->acc = cv.take<T>(8 * n);
    if (geo64) {
        GeoF64 &d = g.g64;
        d.n = (int32_t)n;
        d.nlx = cv.take<double>(S);
        d.nly = cv.take<double>(S);
        d.rfx = cv.take<double>(S);
        d.rfy = cv.take<double>(S);
        d.qx = cv.take<double>(S);
        d.qy = cv.take<double>(S);
        d.cx = cv.take<double>(S);
        d.cy = cv.take<double>(S);
        d.inv_area = cv.take<double>(n);
        d.mi = cv.take<double>(3 * n);
        d.tp = cv.take<double>(6 * n);
        d.bfirst = g.bfirst;
    }
}

size_t layout_bytes(const fvlbm_mesh *m, int precision, int sst) {
    Carver cv;
    fvlbm_state tmp;
    if (precision == FVLBM_FP64)
        carve<double>(cv, m, sst, &tmp);
    else
        carve<float>(cv, m, sst, &tmp, precision == FVLBM_FP32_DEV_GEO64);
    return cv.off + 256;
}

template <typename T>
StepPar<T> step_par(const fvlbm_params &p) {
    StepPar<T> s;
    s.rho0 = T(p.rho0);
    s.dt = T(p.dt);
    s.nu = T(p.nu);
    s.a1 = T(p.a1);
    s.bstar = T(p.beta_star);
    s.sk1 = T(p.sigma_k1);
    s.sk2 = T(p.sigma_k2);
    s.sw1 = T(p.sigma_w1);
    s.sw2 = T(p.sigma_w2);
    s.b1 = T(p.beta1);
    s.b2 = T(p.beta2);
    s.kappa = T(p.kappa);
    s.limiter = p.limiter;
    // Ga1 recovered from f^(2) when the stage solve's a = dt / (4 tau) stays <= 4 for every cell
    // (tau >= tau0 = 3 nu): its rounding amplification 1 + a is then at most 5
    s.recover = p.dt <= 16.0 * 3.0 * p.nu ? 1 : 0;
    return s;
}

template <typename P>
void h2d(P *dst, const std::vector<P> &src, hipStream_t s) {
    if (!src.empty()) check(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(P), hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
}

void upload_scratch(fvlbm_state *st, const double *host, size_t count) {
    check(hipMemcpyAsync(st->scratch, host, count * sizeof(double), hipMemcpyHostToDevice, st->stream), "hipMemcpyAsync H2D");
}

// Boundary values from the parameters: velocity rotated by theta for inlets / far field, zero on
// resting walls; k = 0 and omega = 60 nu / (beta1 d_perp^2) on walls; zero-gradient flag on outlets
// and far-field outflow edges.
void boundary_values(const fvlbm_mesh *m, const fvlbm_params &p, std::vector<double> v[6], std::vector<int32_t> &zg) {
    const size_t nb = m->b_cell.size();
    for (int i = 0; i < 6; ++i) v[i].assign(nb, 0.0);
    zg.assign(nb, 0);
    const double c = std::cos(p.theta), s = std::sin(p.theta);
    for (size_t b = 0; b < nb; ++b) {
        const int g = m->b_group[b], kind = m->b_kind[b];
        double ux = p.group_u[g][0], uy = p.group_u[g][1], rho = p.group_rho[g], k = p.group_k[g], w = p.group_w[g];
        if (p.bface_vals) {
            const double *q = p.bface_vals + 5 * m->b_user[b];
            ux = q[0];
            uy = q[1];
            rho = q[2];
            k = q[3];
            w = q[4];
        }
        if (kind == FVLBM_INLET || kind == FVLBM_FARFIELD) {
            const double rx = c * ux - s * uy, ry = s * ux + c * uy;
            ux = rx;
            uy = ry;
        }
        if (kind == FVLBM_WALL) ux = uy = 0.0;
        if (kind == FVLBM_WALL || kind == FVLBM_MOVING_WALL) {
            k = 0.0;
            const double dp = m->b_dperp[b];
            w = 60.0 * p.nu / (p.beta1 * dp * dp);
        }
        if (kind == FVLBM_OUTLET) zg[b] = 1;
        if (kind == FVLBM_FARFIELD && !(ux * m->b_nx[b] + uy * m->b_ny[b] < 0)) zg[b] = 1;
        v[0][b] = ux;
        v[1][b] = uy;
        v[2][b] = rho;
        v[3][b] = rho - p.rho0;
        v[4][b] = k;
        v[5][b] = w;
    }
}

template <typename T>
void upload_geometry(fvlbm_state *st) {
    const fvlbm_mesh *m = st->mesh;
    hipStream_t s = st->stream;
    Geo<T> &g = geo_of<T>(st);
    // per-edge working copies in the state's arithmetic type, converted from the FP64 masters
    auto as_t = [](const std::vector<double> &v) { return std::vector<T>(v.begin(), v.end()); };
    std::vector<double> qx(m->rfx.size()), qy(m->rfy.size()), ia(m->n);
    for (size_t i = 0; i < qx.size(); ++i) {
        qx[i] = m->rfx[i] - m->dx[i];
        qy[i] = m->rfy[i] - m->dy[i];
    }
    for (int64_t i = 0; i < m->n; ++i) ia[i] = 1.0 / m->area[i];
    std::vector<T> mi(3 * (size_t)m->n);
    for (int64_t i = 0; i < m->n; ++i) {
        mi[i] = (T)m->mi00[i];
        mi[m->n + i] = (T)m->mi01[i];
        mi[2 * m->n + i] = (T)m->mi11[i];
    }
    std::vector<std::vector<T>> conv = {as_t(m->nlx), as_t(m->nly), as_t(m->rfx), as_t(m->rfy), as_t(qx),
                                        as_t(qy),      as_t(m->cx),  as_t(m->cy),  as_t(ia)};
    h2d(const_cast<int32_t *>(g.nbr), m->nbr, s);
    h2d(const_cast<T *>(g.nlx), conv[0], s);
    h2d(const_cast<T *>(g.nly), conv[1], s);
    h2d(const_cast<T *>(g.rfx), conv[2], s);
    h2d(const_cast<T *>(g.rfy), conv[3], s);
    h2d(const_cast<T *>(g.qx), conv[4], s);
    h2d(const_cast<T *>(g.qy), conv[5], s);
    h2d(const_cast<T *>(g.cx), conv[6], s);
    h2d(const_cast<T *>(g.cy), conv[7], s);
    h2d(const_cast<T *>(g.inv_area), conv[8], s);
    h2d(const_cast<T *>(g.mi), mi, s);
    const std::vector<T> tp = as_t(m->tri_p);
    h2d(const_cast<T *>(g.tp), tp, s);
    std::vector<double> mi64;
    if (st->fp64_geometry) {
        // the FP64 masters themselves
        const GeoF64 &d = g.g64;
        mi64.resize(3 * (size_t)m->n);
        for (int64_t i = 0; i < m->n; ++i) {
            mi64[i] = m->mi00[i];
            mi64[m->n + i] = m->mi01[i];
            mi64[2 * m->n + i] = m->mi11[i];
        }
        h2d(const_cast<double *>(d.nlx), m->nlx, s);
        h2d(const_cast<double *>(d.nly), m->nly, s);
        h2d(const_cast<double *>(d.rfx), m->rfx, s);
        h2d(const_cast<double *>(d.rfy), m->rfy, s);
        h2d(const_cast<double *>(d.qx), qx, s);
        h2d(const_cast<double *>(d.qy), qy, s);
        h2d(const_cast<double *>(d.cx), m->cx, s);
        h2d(const_cast<double *>(d.cy), m->cy, s);
        h2d(const_cast<double *>(d.inv_area), ia, s);
        h2d(const_cast<double *>(d.mi), mi64, s);
        h2d(const_cast<double *>(d.tp), m->tri_p, s);
    }
    h2d(const_cast<int32_t *>(g.bfirst), m->bfirst, s);
    h2d(const_cast<double *>(g.area), m->area, s);
    h2d(const_cast<double *>(g.wdist), m->wdist, s);
    std::vector<int32_t> perm(m->n);
    for (int64_t i = 0; i < m->n; ++i) perm[i] = (int32_t)m->perm[i];
    h2d(const_cast<int32_t *>(g.perm), perm, s);
    if (st->face) {
        const std::vector<int32_t> faces = face_list(m);
        // a periodic cell that is its own neighbour across an edge: the two half-edges carry opposite
        // normals and the same upwind value, so their fluxes cancel and the edge list leaves them out
        int64_t self_pairs = 0;
        for (size_t s = 0; s < m->nbr.size(); ++s)
            if (m->nbr[s] == (int32_t)(s % (size_t)m->n)) ++self_pairs;
        if (self_pairs % 2 || (int64_t)faces.size() + self_pairs / 2 != m->n_interior_edges)
            throw Error(FVLBM_EMESH, "init: the edge list does not cover the interior edges");
        if (!faces.empty()) h2d(st->faces, faces, s);
    }
    h2d(const_cast<int32_t *>(g.b_kind), m->b_kind, s);
    h2d(const_cast<int32_t *>(g.b_cell), m->b_cell, s);
    h2d(const_cast<int32_t *>(g.b_group), m->b_group, s);
    h2d(const_cast<double *>(g.b_nx), m->b_nx, s);
    h2d(const_cast<double *>(g.b_ny), m->b_ny, s);
    h2d(const_cast<double *>(g.b_l), m->b_l, s);
    h2d(const_cast<double *>(g.b_dperp), m->b_dperp, s);
    h2d(const_cast<double *>(g.b_xfx), m->b_xfx, s);
    h2d(st->lnb, m->lnb, s);
    h2d(st->rev, m->rev, s);
    h2d(st->hptr, m->halo_ptr, s);
    h2d(st->hcell, m->halo_cell, s);
    h2d(st->xptr, m->ext_ptr, s);
    h2d(st->xn1, m->ext_n1, s);
    h2d(st->xcell, m->ext_cell, s);
    h2d(st->xlnb, m->ext_lnb, s);
    std::vector<double> bv[6];
    std::vector<int32_t> zg;
    boundary_values(m, st->par, bv, zg);
    h2d(const_cast<double *>(g.b_ux), bv[0], s);
    h2d(const_cast<double *>(g.b_uy), bv[1], s);
    h2d(const_cast<double *>(g.b_rho), bv[2], s);
    h2d(const_cast<double *>(g.b_drho), bv[3], s);
    h2d(const_cast<double *>(g.b_k), bv[4], s);
    h2d(const_cast<double *>(g.b_w), bv[5], s);
    h2d(st->bzg, zg, s);
    // host staging vectors must stay alive until the copies ran
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// Brackets a launch with events when timing is on.
struct Timed {
    fvlbm_state *st;
    int id;
    std::pair<hipEvent_t, hipEvent_t> ev{};
    Timed(fvlbm_state *s, int k) : st(s), id(k) {
        if (!st->timing) return;
        if (st->pool_used == st->event_pool.size()) {
            std::pair<hipEvent_t, hipEvent_t> e;
            check(hipEventCreate(&e.first), "hipEventCreate");
            check(hipEventCreate(&e.second), "hipEventCreate");
            st->event_pool.push_back(e);
        }
        ev = st->event_pool[st->pool_used++];
        check(hipEventRecord(ev.first, st->stream), "hipEventRecord");
    }
    ~Timed() {
        if (!st->timing) return;
        (void)hipEventRecord(ev.second, st->stream);
        st->events.push_back({id, ev});
    }
};

// Folds recorded events into the per-kernel sums (synchronises) and recycles them.
void drain_events(fvlbm_state *st) {
    if (st->events.empty()) return;
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
    for (auto &e : st->events) {
        float ms = 0;
        check(hipEventElapsedTime(&ms, e.second.first, e.second.second), "hipEventElapsedTime");
        st->t_ms[e.first] += ms;
        st->t_count[e.first] += 1;
    }
    st->events.clear();
    st->pool_used = 0;
}

// One ring-tiled stage sweep (stage J; J = 0 the explicit scheme) over all tiles; edges per cell
// and the face-value limiter are template switches of the kernel.
template <typename T, int J, int S, int LIM>
void stage_ring_launch(fvlbm_state *st, const Geo<T> &g, const RingTiles &rt, const StageBufs<T> &b,
                       const StepPar<T> &p, hipStream_t s) {
    const int nt = st->mesh->n_tiles, wv = st->ring_wv, wg = st->ring_wg;
    const size_t lds = st->lds_bytes;
    if constexpr (std::is_same_v<T, float>) {
        if (st->fp64_geometry) {
            k_stage_ring<T, J, S, LIM, true><<<nt, kTileCells, lds, s>>>(g, rt, st->lnb, wv, wg, b, p);
            return;
        }
    }
    if (st->pair)
        k_stage_pair<T, J, S, LIM><<<nt, 2 * kTileCells, lds, s>>>(g, rt, st->lnb, wv, wg, b, p);
    else
        k_stage_ring<T, J, S, LIM><<<nt, kTileCells, lds, s>>>(g, rt, st->lnb, wv, wg, b, p);
}

// One ring-tiled stage sweep (stage J; J = 0 the explicit scheme) over all tiles; edges per cell
// and the face-value limiter are template switches of the kernel.
template <typename T, int J>
void stage_ring(fvlbm_state *st, const Geo<T> &g, const RingTiles &rt, const StageBufs<T> &b, const StepPar<T> &p,
                hipStream_t s) {
    // LIM: 0 none, 1 the face-value clip of r32, 2 the gradient limiter of r35, 3 the clip of r32
    // with its states recorded for the adjoint
    if (st->ring_s == 3) {
        if (p.limiter == 1 && b.clip)
            stage_ring_launch<T, J, 3, 3>(st, g, rt, b, p, s);
        else if (p.limiter == 1)
            stage_ring_launch<T, J, 3, 1>(st, g, rt, b, p, s);
        else if (p.limiter == 2)
            stage_ring_launch<T, J, 3, 2>(st, g, rt, b, p, s);
        else
            stage_ring_launch<T, J, 3, 0>(st, g, rt, b, p, s);
    } else {
        if (p.limiter == 1 && b.clip)
            stage_ring_launch<T, J, 4, 3>(st, g, rt, b, p, s);
        else if (p.limiter == 1)
            stage_ring_launch<T, J, 4, 1>(st, g, rt, b, p, s);
        else if (p.limiter == 2)
            stage_ring_launch<T, J, 4, 2>(st, g, rt, b, p, s);
        else
            stage_ring_launch<T, J, 4, 0>(st, g, rt, b, p, s);
    }
}

// The SST update (Step 1) from the macro variables M and k, omega = K0, W0 into K1, W1, the
// relaxation time tau_out and nu_t: one ring launch, or the two split kernels.  With
// params.sst_sweeps = m > 0 (the implicit variant) that launch writes the increments' linear system
// into the G buffer instead (free at both points a step solves the SST), and m Jacobi sweeps follow.
template <typename T, int S>
void launch_sst_jacobi(fvlbm_state *st, const T *K0, const T *W0, T *K1, T *W1, T *tau_out, const StepPar<T> &p) {
    const Geo<T> &g = geo_of<T>(st);
    hipStream_t s = st->stream;
    T *J = (T *)st->G, *nut = (T *)st->nut;
    const size_t n = (size_t)g.n;
    const int nbk = blocks_for(g.n);
    const int m = st->par.sst_sweeps;
    Timed t(st, FVLBM_K_SST_JACOBI);
    // the launches alternate their block order, the first descending after the ascending system launch
    if (m == 1) {
        k_sst_jacobi<T, S, false, true, false><<<nbk, kBlock, 0, s>>>(g, J, J + 8 * n, nullptr, K0, W0, K1, W1, tau_out, nut, p);
        return;
    }
    // sweep 1 gave R' (planes 8, 9); sweeps 2 .. m alternate between planes 10-11 and 12-13
    const T *din = J + 8 * n;
    for (int i = 2; i < m; ++i) {
        T *dout = J + (i % 2 ? 12 : 10) * n;
        if (i % 2 == 0)
            k_sst_jacobi<T, S, true, false, false><<<nbk, kBlock, 0, s>>>(g, J, din, dout, K0, W0, K1, W1, tau_out, nut, p);
        else
            k_sst_jacobi<T, S, true, false, true><<<nbk, kBlock, 0, s>>>(g, J, din, dout, K0, W0, K1, W1, tau_out, nut, p);
        din = dout;
    }
    if (m % 2 == 0)
        k_sst_jacobi<T, S, true, true, false><<<nbk, kBlock, 0, s>>>(g, J, din, nullptr, K0, W0, K1, W1, tau_out, nut, p);
    else
        k_sst_jacobi<T, S, true, true, true><<<nbk, kBlock, 0, s>>>(g, J, din, nullptr, K0, W0, K1, W1, tau_out, nut, p);
}

// One ring launch of the SST kernel; FP32 states with FP64 geometry take the kernel that forms the
// edge data from the FP64 copies.
template <typename T, int S, bool AUX, bool IMPL, typename Args>
void sst_ring_launch(const fvlbm_state *st, int nt, size_t lds, hipStream_t s, const Args &a) {
    std::apply(
        [&](auto &&...x) {
            if constexpr (std::is_same_v<T, float>) {
                if (st->fp64_geometry) {
                    k_sst_ring<T, S, AUX, IMPL, true><<<nt, kTileCells, lds, s>>>(x...);
                    return;
                }
            }
            k_sst_ring<T, S, AUX, IMPL><<<nt, kTileCells, lds, s>>>(x...);
        },
        a);
}

template <typename T>
void launch_sst(fvlbm_state *st, const T *M, const T *K0, const T *W0, T *K1, T *W1, T *tau_out, const StepPar<T> &p) {
    const Geo<T> &g = geo_of<T>(st);
    hipStream_t s = st->stream;
    T *aux = (T *)st->aux, *nut = (T *)st->nut;
    const bool impl = st->par.sst_sweeps > 0;
    T *J = (T *)st->G;
    if (st->ring) {
        const RingTiles rt{st->xptr, st->xn1, st->xcell, st->xlnb, (int32_t)std::max<size_t>(1, st->mesh->ext_cell.size())};
        const int nt = st->mesh->n_tiles, wv = st->ring_wv, wg = st->ring_wg;
        const size_t lds = st->sst_lds_bytes;
        Timed t(st, FVLBM_K_SST);
        const auto args = std::make_tuple(g, rt, st->lnb, wv, wg, st->bzg, M, K0, W0, aux, K1, W1, tau_out, nut, J, p);
        if (st->ring_s == 3) {
            if (impl && st->want_aux)
                sst_ring_launch<T, 3, true, true>(st, nt, lds, s, args);
            else if (impl)
                sst_ring_launch<T, 3, false, true>(st, nt, lds, s, args);
            else if (st->want_aux)
                sst_ring_launch<T, 3, true, false>(st, nt, lds, s, args);
            else
                sst_ring_launch<T, 3, false, false>(st, nt, lds, s, args);
        } else {
            if (impl && st->want_aux)
                sst_ring_launch<T, 4, true, true>(st, nt, lds, s, args);
            else if (impl)
                sst_ring_launch<T, 4, false, true>(st, nt, lds, s, args);
            else if (st->want_aux)
                sst_ring_launch<T, 4, true, false>(st, nt, lds, s, args);
            else
                sst_ring_launch<T, 4, false, false>(st, nt, lds, s, args);
        }
    } else {
        const int nbk = blocks_for(g.n);
        { Timed t(st, FVLBM_K_SST_A); k_sst_a<T><<<nbk, kBlock, 0, s>>>(g, st->bzg, M, K0, W0, aux, p); }
        Timed t(st, FVLBM_K_SST_B);
        if (impl)
            k_sst_b<T, true><<<nbk, kBlock, 0, s>>>(g, st->bzg, M, K0, W0, aux, K1, W1, tau_out, nut, J, p);
        else
            k_sst_b<T, false><<<nbk, kBlock, 0, s>>>(g, st->bzg, M, K0, W0, aux, K1, W1, tau_out, nut, J, p);
    }
    if (impl) {
        if (st->ring_s == 3)
            launch_sst_jacobi<T, 3>(st, K0, W0, K1, W1, tau_out, p);
        else
            launch_sst_jacobi<T, 4>(st, K0, W0, K1, W1, tau_out, p);
    }
}

// One stage sweep of the edge loop: the LSQ gradient planes of the stage field, the interior
// edges' fluxes summed per cell with atomics, then per cell the boundary edges and the stage
// epilogue.
template <typename T, int J>
void face_stage(fvlbm_state *st, const Geo<T> &g, const StageBufs<T> &b, const StepPar<T> &p) {
    hipStream_t s = st->stream;
    const int n = g.n, nbk = blocks_for(n);
    T *G = (T *)st->G, *acc = (T *)st->acc;
    {
        Timed t(st, FVLBM_K_GRAD);
        k_grad<T><<<nbk, kBlock, 0, s>>>(g, b.src, G, p.rho0);
        if (p.limiter == 2) k_bj<T><<<nbk, kBlock, 0, s>>>(g, b.src, G, p.rho0);
    }
    {
        Timed t(st, FVLBM_K_FACE);
        k_fill<T><<<blocks_for(8 * (size_t)n), kBlock, 0, s>>>(8 * n, acc, T(0));
        const int nf = st->n_faces;
        if (nf > 0) {
            if (p.limiter == 1)
                k_face_flux<T, true><<<blocks_for(nf), kBlock, 0, s>>>(g, st->faces, nf, b.src, G, acc);
            else
                k_face_flux<T, false><<<blocks_for(nf), kBlock, 0, s>>>(g, st->faces, nf, b.src, G, acc);
        }
    }
    constexpr int kid = J == 1 ? FVLBM_K_SWEEP1 : (J == 2 ? FVLBM_K_SWEEP2 : FVLBM_K_SWEEP3);
    Timed t(st, kid);
    k_face_epilogue<T, J><<<nbk, kBlock, 0, s>>>(g, G, acc, b, p);
}

template <typename T>
void launch_step(fvlbm_state *st) {
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n;
    const int nbk = blocks_for(n);
    hipStream_t s = st->stream;
    StepPar<T> p = step_par<T>(st->par);
    T *F = (T *)st->F, *X = (T *)st->X, *Y = (T *)st->Y, *A = (T *)st->A, *G = (T *)st->G;
    T *Mcur = (T *)st->M[st->cur_m], *Mnew = (T *)st->M[st->cur_m ^ 1];
    T *tau = (T *)st->tau;
    const RingTiles rt{st->xptr, st->xn1, st->xcell, st->xlnb, (int32_t)std::max<size_t>(1, st->mesh->ext_cell.size())};
    T *K0 = nullptr, *W0 = nullptr, *K1 = nullptr, *W1 = nullptr;
    if (st->sst) {
        K0 = (T *)st->K[st->cur_kw];
        W0 = (T *)st->W[st->cur_kw];
        K1 = (T *)st->K[st->cur_kw ^ 1];
        W1 = (T *)st->W[st->cur_kw ^ 1];
        launch_sst<T>(st, Mcur, K0, W0, K1, W1, tau, p);
        st->cur_kw ^= 1;
    }
    // per-stage SST (reading of Step 5): stage 1 also writes the stage-2 macro variables (into the
    // buffer stage 3 fills at the end), from which the SST is solved again, from k^n, omega^n, for
    // the third stage's relaxation time; the step keeps that solve's k, omega, nu_t.  The second
    // stage's SST inputs are the first's (the first stage's solve keeps rho and u).
    const bool per_stage = st->sst && st->sst_stages;
    T *tau3 = (T *)st->tau3;
    const size_t nn = (size_t)n;
    uint64_t *clip = st->clip;
    const StageBufs<T> b1{X, F, tau, A, Y, nullptr, per_stage ? Mnew : nullptr, nullptr, clip};
    const StageBufs<T> b2{Y, F, tau, A, X, nullptr, nullptr, per_stage ? tau3 : nullptr, clip ? clip + nn : nullptr};
    const StageBufs<T> b3{X, nullptr, nullptr, A, nullptr, st->F_out ? (T *)st->F_out : F, Mnew, nullptr,
                          clip ? clip + 2 * nn : nullptr};
    auto sst_stage3 = [&] {
        if (!per_stage) return;
        // a recorded step keeps the second solve's aux planes apart from the first's
        void *aux1 = st->aux;
        if (st->want_aux && st->aux2) st->aux = st->aux2;
        launch_sst<T>(st, Mnew, K0, W0, K1, W1, tau3, p);
        st->aux = aux1;
    };
    if (st->ring) {
        // stage 1 takes f^(1) from f^n on the fly: no separate collision launch
        { Timed t(st, FVLBM_K_SWEEP1); stage_ring<T, 1>(st, g, rt, b1, p, s); }
        sst_stage3();
        { Timed t(st, FVLBM_K_SWEEP2); stage_ring<T, 2>(st, g, rt, b2, p, s); }
        { Timed t(st, FVLBM_K_SWEEP3); stage_ring<T, 3>(st, g, rt, b3, p, s); }
        st->cur_m ^= 1;
        check(hipGetLastError(), "kernel launch");
        return;
    }
    { Timed t(st, FVLBM_K_COLLIDE1); k_collide1<T><<<nbk, kBlock, 0, s>>>(n, F, tau, X, p); }
    if (st->face) {
        face_stage<T, 1>(st, g, b1, p);
        sst_stage3();
        face_stage<T, 2>(st, g, b2, p);
        face_stage<T, 3>(st, g, b3, p);
    } else if (st->tiled) {
        const int nt = st->mesh->n_tiles;
        const size_t lds = st->lds_bytes;
        const int nth = kTileCells + kHaloThreads;
        if (st->tile_vals) {
            { Timed t(st, FVLBM_K_SWEEP1); k_stage_tiled<T, 1, true><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b1, p); }
            sst_stage3();
            { Timed t(st, FVLBM_K_SWEEP2); k_stage_tiled<T, 2, true><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b2, p); }
            { Timed t(st, FVLBM_K_SWEEP3); k_stage_tiled<T, 3, true><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b3, p); }
        } else {
            { Timed t(st, FVLBM_K_SWEEP1); k_stage_tiled<T, 1, false><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b1, p); }
            sst_stage3();
            { Timed t(st, FVLBM_K_SWEEP2); k_stage_tiled<T, 2, false><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b2, p); }
            { Timed t(st, FVLBM_K_SWEEP3); k_stage_tiled<T, 3, false><<<nt, nth, lds, s>>>(g, st->hptr, st->hcell, st->lnb, st->tile_w, b3, p); }
        }
    } else {
        // gradient planes of a stage field, limited by reading r35 when asked
        auto grads = [&](const T *src) {
            Timed t(st, FVLBM_K_GRAD);
            k_grad<T><<<nbk, kBlock, 0, s>>>(g, src, G, p.rho0);
            if (p.limiter == 2) k_bj<T><<<nbk, kBlock, 0, s>>>(g, src, G, p.rho0);
        };
        grads(X);
        { Timed t(st, FVLBM_K_SWEEP1); k_sweep<T, 1><<<nbk, kBlock, 0, s>>>(g, G, b1, p); }
        sst_stage3();
        grads(Y);
        { Timed t(st, FVLBM_K_SWEEP2); k_sweep<T, 2><<<nbk, kBlock, 0, s>>>(g, G, b2, p); }
        grads(X);
        { Timed t(st, FVLBM_K_SWEEP3); k_sweep<T, 3><<<nbk, kBlock, 0, s>>>(g, G, b3, p); }
    }
    st->cur_m ^= 1;
    check(hipGetLastError(), "kernel launch");
}

// One step of the explicit scheme (the SST first, as in launch_step), ring path only: f^{n+1} goes
// to the X buffer, which then becomes F.
template <typename T>
void launch_explicit(fvlbm_state *st) {
    if (!st->ring) throw Error(FVLBM_ESTATE, "explicit step: needs the ring-tiled sweep (FVLBM_SWEEP unset or ring)");
    const Geo<T> &g = geo_of<T>(st);
    hipStream_t s = st->stream;
    StepPar<T> p = step_par<T>(st->par);
    T *F = (T *)st->F, *X = (T *)st->X, *tau = (T *)st->tau;
    T *Mcur = (T *)st->M[st->cur_m], *Mnew = (T *)st->M[st->cur_m ^ 1];
    const RingTiles rt{st->xptr, st->xn1, st->xcell, st->xlnb, (int32_t)std::max<size_t>(1, st->mesh->ext_cell.size())};
    if (st->sst) {
        launch_sst<T>(st, Mcur, (const T *)st->K[st->cur_kw], (const T *)st->W[st->cur_kw], (T *)st->K[st->cur_kw ^ 1],
                      (T *)st->W[st->cur_kw ^ 1], tau, p);
        st->cur_kw ^= 1;
    }
    const StageBufs<T> b0{F, nullptr, tau, nullptr, nullptr, X, Mnew};
    {
        Timed t(st, FVLBM_K_EXPLICIT);
        stage_ring<T, 0>(st, g, rt, b0, p, s);
    }
    std::swap(st->F, st->X);
    st->cur_m ^= 1;
    check(hipGetLastError(), "kernel launch");
}

template <typename T>
double residual(fvlbm_state *st) {
    const int n = st->n_cells;
    k_residual<T><<<kRedBlocks, kBlock, 0, st->stream>>>(n, (T *)st->M[st->cur_m], (T *)st->M[st->cur_m ^ 1], st->partial);
    k_finish<2><<<1, kBlock, 0, st->stream>>>(st->partial, kRedBlocks, st->result);
    double r[2];
    check(hipMemcpyAsync(r, st->result, sizeof(r), hipMemcpyDeviceToHost, st->stream), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
    // relative L2 change of the velocity; a flow at rest (zero denominator) gives the absolute norm
    return r[1] > 0 ? std::sqrt(r[0] / r[1]) : std::sqrt(r[0]);
}

template <typename T>
void import_state(fvlbm_state *st, const double *f, const double *k, const double *w) {
    const Geo<T> &g = geo_of<T>(st);
    const int nbk = blocks_for(g.n);
    if (f) {
        upload_scratch(st, f, 9 * (size_t)g.n);
        k_import_f<T><<<nbk, kBlock, 0, st->stream>>>(g, st->scratch, (T *)st->F, st->par.rho0);
    }
    k_macro<T><<<nbk, kBlock, 0, st->stream>>>(g.n, (T *)st->F, (T *)st->M[st->cur_m], T(st->par.rho0));
    if (st->sst) {
        if (k) {
            check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
            upload_scratch(st, k, g.n);
            k_import_scalar<T><<<nbk, kBlock, 0, st->stream>>>(g, st->scratch, (T *)st->K[st->cur_kw]);
        }
        if (w) {
            check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
            upload_scratch(st, w, g.n);
            k_import_scalar<T><<<nbk, kBlock, 0, st->stream>>>(g, st->scratch, (T *)st->W[st->cur_kw]);
        }
    }
    check(hipGetLastError(), "kernel launch");
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
}

// Chooses the sweep variant: the ring-tiled kernels when every tile's extended halo fits one
// thread per ext cell and their LDS fits; else the ring-1 tiled kernels unless their LDS would not
// fit; else the two-kernel path.  The environment variable FVLBM_SWEEP (ring, tiled, tiled-grads,
// split, face; pair: the ring-tiled stage sweeps with two threads per cell) restricts the choice.
// LDS of the ring-tiled transposed convection: values, gradient adjoints and, on triangle meshes,
// the inverse LSQ matrices of tile and ring-1 cells.
template <typename T>
size_t adj_t_lds(const fvlbm_state *st) {
    return ((size_t)8 * st->ring_wv + (size_t)(st->ring_s == 3 ? 19 : 16) * st->ring_wg) * sizeof(T);
}
// LDS of the ring-tiled SST reverse: cell values, net-inflow and gradient adjoints, and on
// triangle meshes the inverse LSQ matrices.
template <typename T>
size_t adj_sst_lds(const fvlbm_state *st) {
    return ((size_t)14 * st->ring_wv + (size_t)(st->ring_s == 3 ? 11 : 8) * st->ring_wg) * sizeof(T);
}

template <typename T>
void choose_sweep(fvlbm_state *st) {
    static_assert(kTileCells == kTile, "tile size of the kernels and of the mesh preprocessing differ");
    st->tile_w = kTile + st->mesh->halo_max;
    int dev = 0, max_lds = 0;
    check(hipGetDevice(&dev), "hipGetDevice");
    check(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    const char *env = std::getenv("FVLBM_SWEEP");
    const std::string mode = env ? env : "";
    st->ring_s = st->mesh->max_faces <= 3 ? 3 : 4;
    st->ring_wv = kTile + st->mesh->ext_max;
    st->ring_wg = kTile + st->mesh->halo_max;
    if (mode == "face" && st->fp64_geometry) throw Error(FVLBM_EINVAL, "init: FP32 storage with FP64 geometry needs the ring-tiled sweep");
    if (mode == "face") {
        // the edge loop with atomics: gradients in HBM, then one thread per interior edge
        st->face = true;
        st->ring = false;
        st->tiled = false;
        st->lds_bytes = 0;
        return;
    }
    const size_t ring_lds = ((size_t)8 * st->ring_wv + (size_t)16 * st->ring_wg) * sizeof(T);
    // the adjoint's ring kernels must fit as well: transposed convection and the SST reverse
    const size_t adj_lds = std::max(adj_t_lds<T>(st), adj_sst_lds<T>(st));
    // one thread per ring-1 cell; ring-2 cells beyond one per thread are looped over
    st->ring = (mode.empty() || mode == "ring" || mode == "pair") && st->mesh->halo_max <= kTileCells &&
               std::max(ring_lds, adj_lds) <= (size_t)max_lds;
    if (st->fp64_geometry && !st->ring)
        throw Error(FVLBM_EINVAL, "init: FP32 storage with FP64 geometry needs the ring-tiled sweep");
    if (st->ring) {
        // the stage sweeps with two threads per cell (pair) or one (ring)
        st->pair = mode == "pair" && !st->fp64_geometry;
        st->lds_bytes = ring_lds;
        st->sst_lds_bytes = ((size_t)8 * st->ring_wv + (size_t)6 * st->ring_wg) * sizeof(T);
        st->tiled = false;
        return;
    }
    // values staged in LDS as well when 24 planes fit in a third of a CU's LDS (occupancy), else
    // gradients only; the two-kernel path when not even those fit
    const size_t with_vals = (size_t)24 * st->tile_w * sizeof(T), grads = (size_t)16 * st->tile_w * sizeof(T);
    st->tile_vals = mode != "tiled-grads" && with_vals <= (size_t)std::min(max_lds, 160 * 1024 / 3);
    st->lds_bytes = st->tile_vals ? with_vals : grads;
    // the tiled kernels form gradients in LDS without the limiter of r35: with it, the two-kernel path
    st->tiled = st->lds_bytes <= (size_t)max_lds && mode != "split" && st->par.limiter != 2;
}

template <typename T>
void do_init(fvlbm_state *st, const double *rho, const double *u, const double *k, const double *w) {
    choose_sweep<T>(st);
    upload_geometry<T>(st);
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    // rho and u staged in the scratch area: rho [n] then u [n][2]
    check(hipMemcpyAsync(st->scratch, rho, n * sizeof(double), hipMemcpyHostToDevice, st->stream), "hipMemcpyAsync H2D");
    check(hipMemcpyAsync(st->scratch + n, u, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, st->stream), "hipMemcpyAsync H2D");
    k_init_feq<T><<<nbk, kBlock, 0, st->stream>>>(g, st->scratch, st->scratch + n, (T *)st->F, st->par.rho0);
    k_fill<T><<<nbk, kBlock, 0, st->stream>>>(n, (T *)st->tau, T(3.0 * st->par.nu));
    k_fill<T><<<nbk, kBlock, 0, st->stream>>>(n, (T *)st->nut, T(0));
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
    import_state<T>(st, nullptr, k, w);
    // the residual of a first step compares with the initial velocity
    check(hipMemcpyAsync(st->M[st->cur_m ^ 1], st->M[st->cur_m], 3 * (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
}

template <typename T>
void export_moments(fvlbm_state *st, int on_device, double *rho, double *u, double *k, double *w, double *nut) {
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    const T *M = (const T *)st->M[st->cur_m];
    auto run = [&](double *dst, size_t count, auto launch) {
        if (!dst) return;
        double *target = on_device ? dst : st->scratch;
        launch(target);
        if (!on_device) {
            check(hipMemcpyAsync(dst, st->scratch, count * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
            check(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
    };
    run(rho, n, [&](double *t) { k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, M, st->par.rho0, t); });
    run(u, 2 * (size_t)n, [&](double *t) { k_export_vel<T><<<nbk, kBlock, 0, s>>>(g, M, t); });
    run(k, n, [&](double *t) { k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->K[st->cur_kw], 0.0, t); });
    run(w, n, [&](double *t) { k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->W[st->cur_kw], 0.0, t); });
    run(nut, n, [&](double *t) { k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->nut, 0.0, t); });
    check(hipGetLastError(), "kernel launch");
}

template <typename T>
void totals(fvlbm_state *st, double out[3]) {
    k_totals<T><<<kRedBlocks, kBlock, 0, st->stream>>>(geo_of<T>(st), (const T *)st->M[st->cur_m], st->par.rho0, st->partial);
    k_finish<3><<<1, kBlock, 0, st->stream>>>(st->partial, kRedBlocks, st->result);
    check(hipMemcpyAsync(out, st->result, 3 * sizeof(double), hipMemcpyDeviceToHost, st->stream), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
}

// The totals of fvlbm_moments into a caller device buffer, asynchronously, with the partial sums in
// the library's own reduction buffer instead of the workspace (same kernels, same summation order).
template <typename T>
void totals_noalloc(fvlbm_state *st, double *out_dev) {
    static_assert((size_t)kRedBlocks * 3 <= kNoAllocScratchDoubles, "the reduction buffer is too small");
    k_totals<T><<<kRedBlocks, kBlock, 0, st->stream>>>(geo_of<T>(st), (const T *)st->M[st->cur_m], st->par.rho0, st->noalloc);
    k_finish<3><<<1, kBlock, 0, st->stream>>>(st->noalloc, kRedBlocks, out_dev);
    check(hipGetLastError(), "kernel launch");
}

template <typename T>
void forces(fvlbm_state *st, uint64_t mask, double out[3]) {
    k_forces<T><<<kRedBlocks, kBlock, 0, st->stream>>>(geo_of<T>(st), (const T *)st->M[st->cur_m], st->par.rho0, st->par.nu,
                                                         (unsigned long long)mask, st->par.jr_group, st->par.jr_xmin,
                                                         st->par.eps_tau, st->partial);
    k_finish<3><<<1, kBlock, 0, st->stream>>>(st->partial, kRedBlocks, st->result);
    check(hipMemcpyAsync(out, st->result, 3 * sizeof(double), hipMemcpyDeviceToHost, st->stream), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
}

template <typename T>
void apply_advection(fvlbm_state *st, const double *gin, double *out) {
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    upload_scratch(st, gin, 9 * (size_t)n);
    k_import_f<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, (T *)st->X, st->par.rho0);
    k_grad<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->X, (T *)st->G, T(st->par.rho0));
    if (st->par.limiter == 2) k_bj<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->X, (T *)st->G, T(st->par.rho0));
    k_advect<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->X, (const T *)st->G, (T *)st->Y, T(st->par.rho0), st->par.limiter);
    // Gamma^a is exported without the w_a rho0 shift
    k_export_f<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->Y, st->scratch, 0.0);
    check(hipGetLastError(), "kernel launch");
    check(hipMemcpyAsync(out, st->scratch, 9 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

template <typename T, int S, bool ACC, int EPI>
void launch_T_ring(fvlbm_state *st, const T *f, const T *tau1, T a_dt, const T *lam, T lscale, T *out, double *dth,
                   const AdjBufs<T> &ab, const StepPar<T> &p, const uint64_t *clip) {
    const Geo<T> &g = geo_of<T>(st);
    const RingTiles rt{st->xptr, st->xn1, st->xcell, st->xlnb, (int32_t)std::max<size_t>(1, st->mesh->ext_cell.size())};
    if constexpr (EPI != 0) {
        // the stage reverses of a step limited by r32: the edges' recorded clip states
        if (clip) {
            k_adv_T_ring<T, S, ACC, EPI, true><<<st->mesh->n_tiles, kTileCells, adj_t_lds<T>(st), st->stream>>>(
                g, rt, st->lnb, st->rev, st->ring_wv, st->ring_wg, lam, lscale, out, f, tau1, a_dt, dth, T(st->par.rho0),
                ab, p, clip);
            return;
        }
    }
    if (clip) throw Error(FVLBM_ESTATE, "adv_transpose: clip states only in a stage reverse");
    k_adv_T_ring<T, S, ACC, EPI><<<st->mesh->n_tiles, kTileCells, adj_t_lds<T>(st), st->stream>>>(
        g, rt, st->lnb, st->rev, st->ring_wv, st->ring_wg, lam, lscale, out, f, tau1, a_dt, dth, T(st->par.rho0), ab, p);
}

// Transposed convection at field f (with tau1: at the stage solve of f with a = dt / (4 tau1))
// applied to lscale lam, accumulated into out (acc) or stored there; the theta part per cell is
// added to dth.  epi = J: the stage-J reverse follows, taking the complete adjoint of the stage
// field (the ring path then leaves out undefined for cells without boundary edges).
// Uses st->G for the gradient adjoints.
template <typename T>
void adv_transpose(fvlbm_state *st, const T *f, const T *tau1, const T *lam, T lscale, T *out, double *dth, bool acc,
                   int epi = 0, const AdjBufs<T> &ab = AdjBufs<T>{}, const StepPar<T> &p = StepPar<T>{},
                   const uint64_t *clip = nullptr) {
    const T a_dt = T(st->par.dt / 4.0);
    const Geo<T> &g = geo_of<T>(st);
    const int nbk = blocks_for(g.n);
    hipStream_t s = st->stream;
    // stage 3 stores the transpose (its f^(3) adjoint starts from it), stages 2 and 1 add to theirs
    if ((acc && epi == 3) || (!acc && (epi == 1 || epi == 2)))
        throw Error(FVLBM_EINVAL, "adv_transpose: stage epilogue and accumulation do not match");
    // the ring kernel hands its input values to the stage-3 / 2 reverse, which read the same arrays
    if ((epi == 3 && lam != ab.lnext) || (epi == 2 && lam != ab.lam))
        throw Error(FVLBM_EINVAL, "adv_transpose: the transposed input is not the stage reverse's");
    // the gradient limiter of r35 reverses on the two-kernel transposes, whatever sweep ran forward
    // (they read the global geometry and gradient planes, which every state holds)
    if (st->ring && p.limiter != 2) {
        // one launch: the boundary cells' ghost parts are fused into the ring kernel
        const bool s3 = st->ring_s == 3;
#define FVLBM_T_RING(S_, ACC_, EPI_) launch_T_ring<T, S_, ACC_, EPI_>(st, f, tau1, a_dt, lam, lscale, out, dth, ab, p, clip)
        if (!acc && epi == 3)
            s3 ? FVLBM_T_RING(3, false, 3) : FVLBM_T_RING(4, false, 3);
        else if (!acc)
            s3 ? FVLBM_T_RING(3, false, 0) : FVLBM_T_RING(4, false, 0);
        else if (epi == 0)
            s3 ? FVLBM_T_RING(3, true, 0) : FVLBM_T_RING(4, true, 0);
        else if (epi == 2)
            s3 ? FVLBM_T_RING(3, true, 2) : FVLBM_T_RING(4, true, 2);
        else
            s3 ? FVLBM_T_RING(3, true, 1) : FVLBM_T_RING(4, true, 1);
#undef FVLBM_T_RING
        return;
    }
    if (!acc) k_fill<T><<<blocks_for(9 * (size_t)g.n), kBlock, 0, s>>>(9 * g.n, out, T(0));
    T *Gb = ab.Gb ? ab.Gb : (T *)st->G;
    // the face-value limiter of r32: its clip states formed again from the stage field and its
    // gradient planes (the two-kernel sweeps record none); the planes go to the state's own gradient
    // buffer, free here (these states recompute on the caller's stream only)
    const bool lim1 = p.limiter == 1;
    if (lim1) {
        if (!(ab.sf && ab.clipr && Gb != (T *)st->G))
            throw Error(FVLBM_ESTATE, "adv_transpose: the face-value limiter's reverse has no buffers");
        const T *sf = f;
        if (tau1) {
            k_collide1<T><<<nbk, kBlock, 0, s>>>(g.n, f, tau1, ab.sf, p);
            sf = ab.sf;
        }
        k_grad<T><<<nbk, kBlock, 0, s>>>(g, sf, (T *)st->G, T(st->par.rho0));
        k_clip_states<T><<<nbk, kBlock, 0, s>>>(g, sf, (const T *)st->G, ab.clipr);
    }
    // the gradient limiter of r35: its reverse between the edge part and the LSQ transposes
    const bool bj = p.limiter == 2;
    if (bj && !(ab.lD && ab.bjc)) throw Error(FVLBM_ESTATE, "adv_transpose: the gradient limiter's reverse has no buffers");
    if (bj) {
        k_adv_T1<T, false><<<nbk, kBlock, 0, s>>>(g, lam, lscale, out, Gb);
        k_adv_T_bj<T><<<nbk, kBlock, 0, s>>>(g, f, tau1, a_dt, T(st->par.rho0), Gb, out, ab.lD, ab.bjc, dth);
    } else if (lim1) {
        k_adv_T1<T, true, true><<<nbk, kBlock, 0, s>>>(g, lam, lscale, out, Gb, ab.clipr);
    } else {
        k_adv_T1<T><<<nbk, kBlock, 0, s>>>(g, lam, lscale, out, Gb);
    }
    if (g.nb > 0)
        k_adv_T1b<T, 0><<<blocks_for(g.nb), kBlock, 0, s>>>(g, f, tau1, a_dt, lam, lscale, out, (const T *)Gb, dth,
                                                            T(st->par.rho0), ab, p);
    if (bj)
        k_adv_T2<T, true><<<nbk, kBlock, 0, s>>>(g, st->rev, (const T *)Gb, out, ab.lD, ab.bjc);
    else
        k_adv_T2<T><<<nbk, kBlock, 0, s>>>(g, st->rev, (const T *)Gb, out);
    if (epi == 3)
        k_adj_stage<T, 3><<<nbk, kBlock, 0, s>>>(g.n, ab, p, out);
    else if (epi == 2)
        k_adj_stage<T, 2><<<nbk, kBlock, 0, s>>>(g.n, ab, p, out);
    else if (epi == 1)
        k_adj_stage<T, 1><<<nbk, kBlock, 0, s>>>(g.n, ab, p, out);
}

// Diagnostic: gbar = Gamma^a(g)^T lam and d(lam . Gamma^a(g))/d theta.
template <typename T>
void apply_advection_adjoint(fvlbm_state *st, const double *gin, const double *lam, double *out, double *dtheta) {
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    upload_scratch(st, gin, 9 * (size_t)n);
    k_import_f<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, (T *)st->X, st->par.rho0);
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    upload_scratch(st, lam, 9 * (size_t)n);
    k_import_f<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, (T *)st->Y, 0.0);
    k_fill<T><<<blocks_for(9 * (size_t)n), kBlock, 0, s>>>(9 * n, (T *)st->A, T(0));
    double *dth = st->scratch + 8 * (size_t)n;   // last plane of the staging area (free after import)
    k_fill<double><<<nbk, kBlock, 0, s>>>(n, dth, 0.0);
    adv_transpose<T>(st, (const T *)st->X, (const T *)nullptr, (const T *)st->Y, T(1), (T *)st->A, dth, true);
    k_sum<double><<<kRedBlocks, kBlock, 0, s>>>(n, dth, st->partial);
    k_export_f<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->A, st->scratch, 0.0);
    k_finish<1><<<1, kBlock, 0, s>>>(st->partial, kRedBlocks, st->result);
    check(hipGetLastError(), "kernel launch");
    check(hipMemcpyAsync(out, st->scratch, 9 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check(hipMemcpyAsync(dtheta, st->result, sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// ---------------------------------------------------------------------------------------------
// Record and adjoint.  Layout of the caller's adjoint workspace (all T unless noted):
//   checkpoints: (ceil(N/C) + 1) states of f [9n], k [n], omega [n] (the last one: the final state)
//   segment:     C + 1 states of the same form (the inputs of a segment's steps and its output)
//   stage data:  C slots of f^(2), f^(3), Q [9n each], tau [n], aux [15n]
//   adjoint:     lF, lF2 [9n], lK, lW, lK2, lW2 [n], lf1, lf2, lf3, lam, lg1 [9n each], ltau [n],
//                lx [11n], lnet [2n], lown [4n], lgrad [8n], pbar [5n] (FP64)
// ---------------------------------------------------------------------------------------------
template <typename T>
struct AdjLayout {
    T *ckpt, *seg, *stg, *lF, *lF2, *lK, *lW, *lK2, *lW2, *lf1, *lf2, *lf3, *lam, *lg1, *ltau, *lx, *lnet, *lown, *lgrad;
    T *ltau3, *lK3, *lW3, *zero2;   // per-stage SST: the adjoints of tau3 and of the second solve's k^n, omega^n; [2][n] zeros
    // the implicit SST variant's reverse: its system again (planes 0-9 of J), the increments of
    // sweeps 2 .. m [kMaxAdjSstSweeps - 1][2][n], the adjoints of R' [2][n], of the couplings [8][n],
    // of the increments (two [2][n] buffers), and the neighbours' parts of the rows' reverse [16][n]
    T *Jr, *dlt, *lR, *lC, *ld0, *ld1, *lslot;
    T *lD;              // the gradient limiter's reverse (reading r35): bound parts [8][n] and their codes
    int8_t *bjc;
    T *Gb;              // gradient-plane adjoints of the two-kernel transposes [16][n]
    T *sf;              // the face-value limiter on the two-kernel transposes: a stage field [9][n] and
    uint64_t *clipr;    // its clip states [n]
    T *seg2, *stg2;     // a second set of segment buffers when the run has more than one segment
    uint64_t *clip, *clip2;   // per step of a segment: the r32 clip states of its three sweeps [3][n]
    double *pbar;
    size_t state_len;
    size_t stage_len;   // per step of a segment: f^(2), f^(3), Q [9][n] each, tau [n], aux [15][n], and for the
                        // per-stage SST tau3 [n] and the second solve's aux [15][n]
};

// The layout with segment set k (0 or 1) as its segment buffers: segment sg of a run lives in set
// sg % 2, so that one segment can be recomputed while the next is reversed; without a second set
// every segment uses the first.
template <typename T>
AdjLayout<T> segment_set(const AdjLayout<T> &L, int k) {
    AdjLayout<T> r = L;
    if ((k & 1) && L.seg2) {
        r.seg = L.seg2;
        r.stg = L.stg2;
        r.clip = L.clip2;
    }
    return r;
}

// The adjoint recomputes the next segment concurrently with the reverse of the current one only on
// meshes of at most this many tiles: a launch there leaves most of the GPU idle, while on larger
// meshes each launch fills it and the two streams only compete (measured: backstep, 481 tiles,
// adjoint / forward 3.05 -> 2.29; 4.0M cells, 15,608 tiles, 2.91 -> 3.02).
constexpr int32_t kOverlapMaxTiles = 1024;

// Whether the adjoint workspace holds a second set of segment buffers (runs of more than one
// segment): the record pass then keeps the tapes of the last two segments, and on small meshes the
// reverse overlaps.  FVLBM_ADJ_OVERLAP=0 in the environment keeps one set.
inline bool adjoint_two_sets(const fvlbm_mesh *) {
    const char *e = std::getenv("FVLBM_ADJ_OVERLAP");
    return !(e && std::string(e) == "0");
}

template <typename T>
size_t adj_carve(Carver &cv, int64_t n, int32_t n_steps, int32_t ckpt, bool overlap, AdjLayout<T> &L) {
    const size_t sl = 11 * (size_t)n;
    const size_t nck = (size_t)((n_steps + ckpt - 1) / ckpt) + 1;
    L.state_len = sl;
    L.ckpt = cv.take<T>(nck * sl);
    L.seg = cv.take<T>((size_t)(ckpt + 1) * sl);
    L.stage_len = 59 * (size_t)n;
    L.stg = cv.take<T>((size_t)ckpt * L.stage_len);
    L.clip = cv.take<uint64_t>((size_t)ckpt * 3 * n);
    L.seg2 = L.stg2 = nullptr;
    L.clip2 = nullptr;
    if (overlap && nck > 2) {
        L.seg2 = cv.take<T>((size_t)(ckpt + 1) * sl);
        L.stg2 = cv.take<T>((size_t)ckpt * L.stage_len);
        L.clip2 = cv.take<uint64_t>((size_t)ckpt * 3 * n);
    }
    L.lF = cv.take<T>(9 * (size_t)n);
    L.lF2 = cv.take<T>(9 * (size_t)n);
    L.lK = cv.take<T>(n);
    L.lW = cv.take<T>(n);
    L.lK2 = cv.take<T>(n);
    L.lW2 = cv.take<T>(n);
    L.lf1 = cv.take<T>(9 * (size_t)n);
    L.lf2 = cv.take<T>(9 * (size_t)n);
    L.lf3 = cv.take<T>(9 * (size_t)n);
    L.lam = cv.take<T>(9 * (size_t)n);
    L.lg1 = cv.take<T>(9 * (size_t)n);
    L.ltau = cv.take<T>(n);
    L.lx = cv.take<T>(11 * (size_t)n);
    L.lnet = cv.take<T>(2 * (size_t)n);
    L.lown = cv.take<T>(4 * (size_t)n);
    L.lgrad = cv.take<T>(8 * (size_t)n);
    L.ltau3 = cv.take<T>(n);
    L.lK3 = cv.take<T>(n);
    L.lW3 = cv.take<T>(n);
    L.zero2 = cv.take<T>(2 * (size_t)n);
    L.Jr = cv.take<T>(10 * (size_t)n);
    L.dlt = cv.take<T>((size_t)(kMaxAdjSstSweeps - 1) * 2 * n);
    L.lR = cv.take<T>(2 * (size_t)n);
    L.lC = cv.take<T>(8 * (size_t)n);
    L.ld0 = cv.take<T>(2 * (size_t)n);
    L.ld1 = cv.take<T>(2 * (size_t)n);
    L.lslot = cv.take<T>(16 * (size_t)n);
    L.lD = cv.take<T>(8 * (size_t)n);
    L.bjc = cv.take<int8_t>(8 * (size_t)n);
    L.Gb = cv.take<T>(16 * (size_t)n);
    L.sf = cv.take<T>(9 * (size_t)n);
    L.clipr = cv.take<uint64_t>(n);
    L.pbar = cv.take<double>(5 * (size_t)n);
    return cv.off + 256;
}

template <typename T>
AdjLayout<T> adj_layout(fvlbm_state *st) {
    Carver cv;
    cv.base = st->adj_ws;
    AdjLayout<T> L;
    adj_carve<T>(cv, st->n_cells, st->rec_steps, st->rec_ckpt, st->adj_two_sets, L);
    return L;
}

// copy the current state (f, k, omega) into / out of a slot of 11 n values
template <typename T>
void save_state(fvlbm_state *st, T *slot) {
    const size_t n = st->n_cells;
    check(hipMemcpyAsync(slot, st->F, 9 * n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    if (st->sst) {
        check(hipMemcpyAsync(slot + 9 * n, st->K[st->cur_kw], n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
        check(hipMemcpyAsync(slot + 10 * n, st->W[st->cur_kw], n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    }
}

template <typename T>
void load_state(fvlbm_state *st, const T *slot) {
    const size_t n = st->n_cells;
    check(hipMemcpyAsync(st->F, slot, 9 * n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    if (st->sst) {
        check(hipMemcpyAsync(st->K[st->cur_kw], slot + 9 * n, n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
        check(hipMemcpyAsync(st->W[st->cur_kw], slot + 10 * n, n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    }
    k_macro<T><<<blocks_for(n), kBlock, 0, st->stream>>>((int)n, (const T *)st->F, (T *)st->M[st->cur_m], T(st->par.rho0));
}

// Stage data of one step of a segment, kept from the segment's forward pass for its reverse.
template <typename T>
struct StageSlot {
    T *Y, *X, *A, *tau, *aux;
    uint64_t *clip;   // [3][n]: the clip states of sweeps 1, 2, 3 (face-value limiter of r32)
    T *tau3, *aux2;   // per-stage SST: the third stage's relaxation time, the second solve's aux planes
};

template <typename T>
StageSlot<T> stage_slot(const fvlbm_state *st, const AdjLayout<T> &L, int i) {
    const size_t n = st->n_cells;
    T *b = L.stg + (size_t)i * L.stage_len;
    return StageSlot<T>{b, b + 9 * n, b + 18 * n, st->sst ? b + 27 * n : (T *)st->tau, b + 28 * n,
                        L.clip + (size_t)i * 3 * n, b + 43 * n, b + 44 * n};
}

// Step j of a segment, in place in the segment buffers: reads the state in segment slot j, writes
// the next one into slot j + 1, and its stage data (f^(2), f^(3), Q and with the SST tau and the
// aux planes) into stage slot j, so that its reverse needs no recomputation.
template <typename T>
void step_seg(fvlbm_state *st, const AdjLayout<T> &L, int j) {
    const size_t n = st->n_cells;
    T *in = L.seg + (size_t)j * L.state_len, *out = in + L.state_len;
    const StageSlot<T> ss = stage_slot<T>(st, L, j);
    void *F = st->F, *X = st->X, *Y = st->Y, *A = st->A, *tau = st->tau, *aux = st->aux, *tau3 = st->tau3;
    void *K0 = st->K[0], *K1 = st->K[1], *W0 = st->W[0], *W1 = st->W[1];
    st->F = in;
    st->F_out = out;
    st->X = ss.X;
    st->Y = ss.Y;
    st->A = ss.A;
    st->clip = st->par.limiter == 1 ? ss.clip : nullptr;
    if (st->sst) {
        st->K[st->cur_kw] = in + 9 * n;
        st->K[st->cur_kw ^ 1] = out + 9 * n;
        st->W[st->cur_kw] = in + 10 * n;
        st->W[st->cur_kw ^ 1] = out + 10 * n;
        st->tau = ss.tau;
        st->aux = ss.aux;
        st->want_aux = true;
        if (st->sst_stages) {
            st->tau3 = ss.tau3;
            st->aux2 = ss.aux2;
        }
    }
    launch_step<T>(st);
    st->F = F;
    st->F_out = nullptr;
    st->clip = nullptr;
    st->X = X;
    st->Y = Y;
    st->A = A;
    st->tau = tau;
    st->aux = aux;
    st->tau3 = tau3;
    st->aux2 = nullptr;
    st->K[0] = K0;
    st->K[1] = K1;
    st->W[0] = W0;
    st->W[1] = W1;
    st->want_aux = false;
}

// Segments of a recorded run of N steps with at most C steps each, placed from the end: segment sg
// (of nseg = ceil(N / C)) covers steps [first, last); only the first may be shorter than C.
inline void segment_bounds(int N, int C, int sg, int &first, int &last) {
    const int nseg = (N + C - 1) / C;
    last = N - (nseg - 1 - sg) * C;
    first = std::max(0, last - C);
}

// Advances the recorded run, storing a checkpoint at the start of every segment and the final
// state.  The last segment, and with two sets of segment buffers the one before it too, is run
// through its set of segment buffers, so that the reverse starts without recomputing them.
template <typename T>
void record(fvlbm_state *st) {
    AdjLayout<T> L = adj_layout<T>(st);
    const int N = st->rec_steps, C = st->rec_ckpt;
    const int nseg = (N + C - 1) / C;
    const int held = (L.seg2 && nseg > 1) ? 2 : 1;
    for (int sg = 0; sg < nseg - held; ++sg) {
        int first, last;
        segment_bounds(N, C, sg, first, last);
        save_state<T>(st, L.ckpt + (size_t)sg * L.state_len);
        for (int i = first; i < last; ++i) launch_step<T>(st);
    }
    for (int sg = nseg - held; sg < nseg; ++sg) {
        int first, last;
        segment_bounds(N, C, sg, first, last);
        save_state<T>(st, L.ckpt + (size_t)sg * L.state_len);
        const AdjLayout<T> Ls = segment_set(L, sg % 2);
        save_state<T>(st, Ls.seg);
        for (int i = first; i < last; ++i) step_seg<T>(st, Ls, i - first);
        load_state<T>(st, Ls.seg + (size_t)(last - first) * L.state_len);
    }
    save_state<T>(st, L.ckpt + (size_t)nseg * L.state_len);
    st->held_segs = held;
    st->steps_done += N;
    check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
}

// Reverse of one step whose input state is in `slot` and whose stage data is in `ss`: from the
// adjoint of the step's output (f: L.lF; k, omega: L.lK, L.lW) to that of its input (f: L.lF2;
// k, omega: L.lK2, L.lW2).
template <typename T>
void reverse_step(fvlbm_state *st, const AdjLayout<T> &L, const T *slot, const StageSlot<T> &ss) {
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    StepPar<T> p = step_par<T>(st->par);
    // the step's input: f, its macro variables (kept by the SST), k, omega
    const T *fn = slot;
    const T *Mn = st->sst ? ss.aux + 12 * (size_t)n : nullptr;
    const T *Kn = st->sst ? slot + 9 * (size_t)n : nullptr, *Wn = st->sst ? slot + 10 * (size_t)n : nullptr;
    // per-stage SST (reading r33): the third stage's tau3 comes from a second SST solve on the
    // stage-2 macro variables, which gives the step's k, omega; the first solve gives tau only
    const bool per_stage = st->sst && st->sst_stages;
    AdjBufs<T> b{fn, ss.Y, ss.X, ss.A, ss.tau, L.lF, L.lF2, L.lf1, L.lf2, L.lf3, L.lam, L.lg1, L.ltau};
    if (per_stage) {
        b.tau3 = ss.tau3;
        b.ltau3 = L.ltau3;
    }
    b.lD = L.lD;
    b.bjc = L.bjc;
    b.Gb = L.Gb;
    b.sf = L.sf;
    b.clipr = L.clipr;
    // the SST reverse of one solve: from the adjoints of its outputs (k, omega: lk, lw; tau: lt) to
    // those of its inputs (the macro variables M, added onto lf through the moments of the field they
    // came from; k^n, omega^n into lk_out, lw_out)
    auto sst_reverse = [&](const T *M, const T *aux, const T *lk, const T *lw, const T *lt, T *lf, T *lk_out,
                           T *lw_out) {
        SstAdj sa{st->bzg, L.pbar};
        const int m = st->par.sst_sweeps;
        if (m > 0) {
            // the implicit variant (reading r34): its system again, the increments of sweeps 2 .. m,
            // the reverse of the floor and nu_t, the transposed sweeps, the rows' reverse; then the
            // face, closure and gradient reverses as for the point-implicit update
            const size_t nn = (size_t)n;
            auto delta = [&](int i) { return i == 1 ? L.Jr + 8 * nn : L.dlt + (size_t)(i - 2) * 2 * nn; };
            k_adj_impl_sys<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, aux, L.Jr, p);
            for (int i = 2; i <= m; ++i)
                k_sst_jacobi<T, 4, true, false><<<nbk, kBlock, 0, s>>>(g, L.Jr, delta(i - 1), delta(i), nullptr, nullptr,
                                                                    nullptr, nullptr, nullptr, nullptr, p);
            k_fill<T><<<blocks_for(11 * nn), kBlock, 0, s>>>(11 * n, L.lx, T(0));
            k_fill<T><<<blocks_for(2 * nn), kBlock, 0, s>>>(2 * n, L.lR, T(0));
            k_fill<T><<<blocks_for(8 * nn), kBlock, 0, s>>>(8 * n, L.lC, T(0));
            T *lin = L.ld0, *lout = L.ld1;
            k_adj_impl_fin<T><<<nbk, kBlock, 0, s>>>(g, sa, aux, delta(m), Kn, Wn, lk, lw, lt, lin, L.lx, L.lown, p);
            for (int i = m; i >= 2; --i) {
                k_adj_impl_sweep<T><<<nbk, kBlock, 0, s>>>(g, st->rev, L.Jr, lin, delta(i - 1), L.lR, L.lC, lout);
                std::swap(lin, lout);
            }
            k_add<T><<<blocks_for(2 * nn), kBlock, 0, s>>>(2 * n, lin, L.lR);
            k_adj_impl_rows<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, aux, L.lR, L.lC, L.lx, L.lnet, L.lown, L.lslot, p);
            k_adj_impl_gather<T><<<nbk, kBlock, 0, s>>>(g, st->rev, M, L.lslot, L.lx, p.rho0);
            k_adj_sst_faces<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, aux, L.lnet, L.lx, p);
            k_adj_sst_local<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, L.lown, L.lx, L.lgrad, p);
            k_adj_sst_grad<T><<<nbk, kBlock, 0, s>>>(g, sa, st->rev, M, L.lgrad, L.lx, lf, lk_out, lw_out, p.rho0);
        } else if (st->ring && !(sizeof(T) == 8 && st->ring_s == 4)) {
            // (FP64 on meshes with quads takes the split kernels: the ring kernel spills 81 VGPRs
            // there, and the airfoil's lift adjoint ran 9 % slower with it)
            const RingTiles rt{st->xptr, st->xn1, st->xcell, st->xlnb, (int32_t)std::max<size_t>(1, st->mesh->ext_cell.size())};
            const int nt = st->mesh->n_tiles, wv = st->ring_wv, wg = st->ring_wg;
            const size_t lds = adj_sst_lds<T>(st);
            if (st->ring_s == 3)
                k_adj_sst_ring<T, 3><<<nt, kTileCells, lds, s>>>(g, rt, st->lnb, st->rev, wv, wg, sa, M, Kn, Wn, aux, lk, lw,
                                                              lt, lf, lk_out, lw_out, p);
            else if constexpr (sizeof(T) == 4)
                k_adj_sst_ring<T, 4><<<nt, kTileCells, lds, s>>>(g, rt, st->lnb, st->rev, wv, wg, sa, M, Kn, Wn, aux, lk, lw,
                                                              lt, lf, lk_out, lw_out, p);
        } else {
            k_fill<T><<<blocks_for(11 * (size_t)n), kBlock, 0, s>>>(11 * n, L.lx, T(0));
            k_adj_sst_update<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, aux, lk, lw, lt, L.lx, L.lnet, L.lown, p);
            k_adj_sst_faces<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, aux, L.lnet, L.lx, p);
            k_adj_sst_local<T><<<nbk, kBlock, 0, s>>>(g, sa, M, Kn, Wn, L.lown, L.lx, L.lgrad, p);
            k_adj_sst_grad<T><<<nbk, kBlock, 0, s>>>(g, sa, st->rev, M, L.lgrad, L.lx, lf, lk_out, lw_out, p.rho0);
        }
    };
    // stage 3: Ga3 enters f^{n+1} with weight dt/3, its transpose is applied to dt/3 lF; then the
    // reverse of the combination and of the third stage
    // with the face-value limiter of r32: the clip states the forward sweeps recorded
    const bool lim = st->par.limiter == 1;
    adv_transpose<T>(st, ss.X, nullptr, L.lF, p.dt / T(3), L.lf3, L.pbar, false, 3, b, p, lim ? ss.clip + 2 * (size_t)n : nullptr);
    // per-stage SST: the second solve's reverse adds its part to the f^(2) adjoint before the second
    // stage's reverse consumes it
    if (per_stage)
        sst_reverse(ss.aux2 + 12 * (size_t)n, ss.aux2, L.lK, L.lW, L.ltau3, L.lf2, L.lK3, L.lW3);
    // stage 2: transpose at f^(2), then its stage reverse (the Ga1 adjoint goes to lg1)
    adv_transpose<T>(st, ss.Y, nullptr, L.lam, T(1), L.lf2, L.pbar, true, 2, b, p, lim ? ss.clip + (size_t)n : nullptr);
    // stage 1: transpose at f^(1), formed from f^n, then its stage reverse
    adv_transpose<T>(st, fn, ss.tau, L.lg1, T(1), L.lf1, L.pbar, true, 1, b, p, lim ? ss.clip : nullptr);
    if (per_stage) {
        // the first solve's k, omega are overwritten by the second's: only its tau has an adjoint
        k_fill<T><<<blocks_for(2 * (size_t)n), kBlock, 0, s>>>(2 * n, L.zero2, T(0));
        sst_reverse(Mn, ss.aux, L.zero2, L.zero2 + n, L.ltau, L.lF2, L.lK2, L.lW2);
        k_add<T><<<nbk, kBlock, 0, s>>>(n, L.lK3, L.lK2);
        k_add<T><<<nbk, kBlock, 0, s>>>(n, L.lW3, L.lW2);
    } else if (st->sst) {
        sst_reverse(Mn, ss.aux, L.lK, L.lW, L.ltau, L.lF2, L.lK2, L.lW2);
    }
    check(hipGetLastError(), "kernel launch");
}

// Reverse of the whole recorded run (L.lF / lK / lW seeded with the adjoint of the final state).
// Each segment is recomputed once from its checkpoint in its set of segment buffers, keeping every
// step's input state and stage data (the last one or two segments come from the record pass while
// their buffers still hold them); then its steps are reversed from the last.  On the ring path and
// small meshes the recompute of segment sg - 1 runs on a second stream while segment sg is
// reversed: the two touch disjoint
// buffers (the recompute: its segment set, the macro buffers and nu_t; the reverse: the other set
// and the adjoint fields), and each waits only for the work on the set it is about to reuse.
template <typename T>
void reverse_run(fvlbm_state *st, const AdjLayout<T> &L0) {
    AdjLayout<T> L = L0;         // lF / lF2 (and lK, lW / lK2, lW2) alternate between steps
    const int N = st->rec_steps, C = st->rec_ckpt;
    const int nseg = (N + C - 1) / C;
    const size_t n = st->n_cells;
    const bool overlap = st->ring && nseg > 1 && L.seg2 && st->mesh->n_tiles <= kOverlapMaxTiles;
    const int held = st->held_segs;   // trailing segments whose tapes the record pass left
    auto is_held = [&](int sg) { return sg >= nseg - held; };
    if (overlap && !st->side) {
        // non-blocking: no implicit ordering with a legacy default stream; the events order the two
        check(hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
        check(hipEventCreateWithFlags(&st->ev_rev, hipEventDisableTiming), "hipEventCreate");
        check(hipEventCreateWithFlags(&st->ev_rec, hipEventDisableTiming), "hipEventCreate");
    }
    hipStream_t main_stream = st->stream;
    struct Restore {
        fvlbm_state *st;
        hipStream_t s;
        ~Restore() { st->stream = s; }
    } restore{st, main_stream};
    auto recompute = [&](int sg, hipStream_t s) {
        const AdjLayout<T> Ls = segment_set(L, sg % 2);
        int first, last;
        segment_bounds(N, C, sg, first, last);
        st->stream = s;
        check(hipMemcpyAsync(Ls.seg, L.ckpt + (size_t)sg * L.state_len, L.state_len * sizeof(T), hipMemcpyDeviceToDevice, s),
              "hipMemcpyAsync D2D");
        k_macro<T><<<blocks_for(n), kBlock, 0, s>>>((int)n, Ls.seg, (T *)st->M[st->cur_m], T(st->par.rho0));
        for (int i = first; i < last; ++i) step_seg<T>(st, Ls, i - first);
        st->stream = main_stream;
    };
    if (!is_held(nseg - 1)) recompute(nseg - 1, main_stream);
    st->held_segs = 0;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        int first, last;
        segment_bounds(N, C, sg, first, last);
        if (overlap && sg > 0 && !is_held(sg - 1)) {
            // set (sg - 1) % 2 was last read by the reverse of segment sg + 1, all of it queued
            check(hipEventRecord(st->ev_rev, main_stream), "hipEventRecord");
            check(hipStreamWaitEvent(st->side, st->ev_rev, 0), "hipStreamWaitEvent");
            recompute(sg - 1, st->side);
            check(hipEventRecord(st->ev_rec, st->side), "hipEventRecord");
        }
        const AdjLayout<T> Ls = segment_set(L, sg % 2);
        for (int i = last - 1; i >= first; --i) {
            reverse_step<T>(st, L, Ls.seg + (size_t)(i - first) * L.state_len, stage_slot<T>(st, Ls, i - first));
            std::swap(L.lF, L.lF2);
            if (st->sst) {
                std::swap(L.lK, L.lK2);
                std::swap(L.lW, L.lW2);
            }
        }
        if (sg > 0 && !is_held(sg - 1)) {
            if (overlap)
                check(hipStreamWaitEvent(main_stream, st->ev_rec, 0), "hipStreamWaitEvent");
            else
                recompute(sg - 1, main_stream);
        }
    }
    if (L.lF != L0.lF)
        check(hipMemcpyAsync(L0.lF, L.lF, 9 * n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    if (L.lK != L0.lK) {
        check(hipMemcpyAsync(L0.lK, L.lK, n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
        check(hipMemcpyAsync(L0.lW, L.lW, n * sizeof(T), hipMemcpyDeviceToDevice, st->stream), "hipMemcpyAsync D2D");
    }
    // restore the final state
    load_state<T>(st, L.ckpt + (size_t)nseg * L.state_len);
    // macro buffers for a residual of a later step: both hold the final macro variables
    check(hipMemcpyAsync(st->M[st->cur_m ^ 1], st->M[st->cur_m], 3 * n * sizeof(T), hipMemcpyDeviceToDevice, st->stream),
          "hipMemcpyAsync D2D");
}

template <typename T>
void reduce_pbar(fvlbm_state *st, const AdjLayout<T> &L, double out[5]) {
    const int n = st->n_cells;
    for (int i = 0; i < 5; ++i) {
        k_sum<double><<<kRedBlocks, kBlock, 0, st->stream>>>(n, L.pbar + (size_t)i * n, st->partial);
        k_finish<1><<<1, kBlock, 0, st->stream>>>(st->partial, kRedBlocks, st->result + i % 4);
        check(hipMemcpyAsync(out + i, st->result + i % 4, sizeof(double), hipMemcpyDeviceToHost, st->stream), "hipMemcpyAsync D2H");
        check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
    }
}

template <typename T>
void adjoint_forces(fvlbm_state *st, uint64_t mask, const double seed[3], double dparams[5]) {
    AdjLayout<T> L = adj_layout<T>(st);
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    k_fill<T><<<blocks_for(9 * (size_t)n), kBlock, 0, s>>>(9 * n, L.lF, T(0));
    k_fill<T><<<nbk, kBlock, 0, s>>>(n, L.lK, T(0));
    k_fill<T><<<nbk, kBlock, 0, s>>>(n, L.lW, T(0));
    k_fill<double><<<blocks_for(5 * (size_t)n), kBlock, 0, s>>>(5 * n, L.pbar, 0.0);
    k_adj_forces<T><<<nbk, kBlock, 0, s>>>(g, (const T *)st->F, (unsigned long long)mask, st->par.jr_group, st->par.jr_xmin,
                                          st->par.eps_tau, st->par.nu, seed[0], seed[1], seed[2], T(st->par.rho0), L.lF);
    reverse_run<T>(st, L);
    reduce_pbar<T>(st, L, dparams);
}

template <typename T>
void adjoint_state(fvlbm_state *st, const double *lf, const double *lk, const double *lw, double *lf0, double *lk0,
                   double *lw0, double dparams[5]) {
    AdjLayout<T> L = adj_layout<T>(st);
    const Geo<T> &g = geo_of<T>(st);
    const int n = g.n, nbk = blocks_for(n);
    hipStream_t s = st->stream;
    upload_scratch(st, lf, 9 * (size_t)n);
    k_import_f<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, L.lF, 0.0);
    k_fill<T><<<nbk, kBlock, 0, s>>>(n, L.lK, T(0));
    k_fill<T><<<nbk, kBlock, 0, s>>>(n, L.lW, T(0));
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st->sst && lk) {
        upload_scratch(st, lk, n);
        k_import_scalar<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, L.lK);
        check(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    if (st->sst && lw) {
        upload_scratch(st, lw, n);
        k_import_scalar<T><<<nbk, kBlock, 0, s>>>(g, st->scratch, L.lW);
        check(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    k_fill<double><<<blocks_for(5 * (size_t)n), kBlock, 0, s>>>(5 * n, L.pbar, 0.0);
    reverse_run<T>(st, L);
    k_export_f<T><<<nbk, kBlock, 0, s>>>(g, L.lF, st->scratch, 0.0);
    check(hipMemcpyAsync(lf0, st->scratch, 9 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st->sst && lk0) {
        k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, L.lK, 0.0, st->scratch);
        check(hipMemcpyAsync(lk0, st->scratch, n * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
        check(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    if (st->sst && lw0) {
        k_export_scalar<T><<<nbk, kBlock, 0, s>>>(g, L.lW, 0.0, st->scratch);
        check(hipMemcpyAsync(lw0, st->scratch, n * sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
        check(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    reduce_pbar<T>(st, L, dparams);
}

// A state-changing call (step, set_state) after fvlbm_record: the tape no longer ends at the current
// state, so the recording is dropped and a later adjoint call returns FVLBM_ESTATE.
void drop_recording(fvlbm_state *st) {
    st->adj_ws = nullptr;
    st->adj_bytes = 0;
    st->held_segs = 0;
}

template <typename F>
fvlbm_status guarded(F &&fn) {
    try {
        fn();
        return FVLBM_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FVLBM_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FVLBM_EINVAL;
    }
}

}  // namespace

extern "C" {

fvlbm_status fvlbm_mesh_create(int64_t n_nodes, const double *node_xy, int64_t n_cells, const int64_t *cell_ptr,
                               const int64_t *cell_nodes, int64_t n_bfaces, const int64_t *bface_nodes,
                               const int32_t *bface_group, int32_t n_groups, const int32_t *group_kind,
                               const double *periodic_shift, int32_t order, fvlbm_mesh **out) {
    return guarded([&] {
        if (!out) throw Error(FVLBM_EINVAL, "mesh_create: out is NULL");
        *out = nullptr;
        *out = build_mesh(n_nodes, node_xy, n_cells, cell_ptr, cell_nodes, n_bfaces, bface_nodes, bface_group,
                          n_groups, group_kind, periodic_shift, order);
    });
}

void fvlbm_mesh_destroy(fvlbm_mesh *mesh) { delete mesh; }

fvlbm_status fvlbm_mesh_counts(const fvlbm_mesh *m, int64_t counts[4]) {
    return guarded([&] {
        if (!m || !counts) throw Error(FVLBM_EINVAL, "mesh_counts: NULL argument");
        counts[0] = m->n;
        counts[1] = m->n_interior_edges;
        counts[2] = m->n_boundary_edges;
        counts[3] = m->max_faces;
    });
}

fvlbm_status fvlbm_mesh_geometry(const fvlbm_mesh *m, double *area, double *centroid, double *wall_dist) {
    return guarded([&] {
        if (!m) throw Error(FVLBM_EINVAL, "mesh_geometry: NULL mesh");
        for (int64_t i = 0; i < m->n; ++i) {
            const int64_t u = m->perm[i];
            if (area) area[u] = m->area[i];
            if (centroid) {
                centroid[2 * u] = m->xc[i];
                centroid[2 * u + 1] = m->yc[i];
            }
            if (wall_dist) wall_dist[u] = m->wdist[i];
        }
    });
}

fvlbm_status fvlbm_mesh_permutation(const fvlbm_mesh *m, int64_t *perm) {
    return guarded([&] {
        if (!m || !perm) throw Error(FVLBM_EINVAL, "mesh_permutation: NULL argument");
        std::memcpy(perm, m->perm.data(), m->n * sizeof(int64_t));
    });
}

fvlbm_status fvlbm_state_bytes(const fvlbm_mesh *m, int32_t precision, int32_t sst, size_t *bytes) {
    return guarded([&] {
        if (!m || !bytes) throw Error(FVLBM_EINVAL, "state_bytes: NULL argument");
        if (precision != FVLBM_FP64 && precision != FVLBM_FP32_DEV && precision != FVLBM_FP32_DEV_GEO64) throw Error(FVLBM_EINVAL, "state_bytes: bad precision");
        *bytes = layout_bytes(m, precision, sst ? 1 : 0);
    });
}

fvlbm_status fvlbm_init(const fvlbm_mesh *m, const fvlbm_params *p, int32_t precision, const double *rho,
                        const double *u, const double *k, const double *omega, void *workspace, size_t ws_bytes,
                        void *hip_stream, fvlbm_state **out) {
    return guarded([&] {
        if (!out) throw Error(FVLBM_EINVAL, "init: out is NULL");
        *out = nullptr;
        if (!m || !p || !rho || !u || !workspace) throw Error(FVLBM_EINVAL, "init: NULL argument");
        if (precision != FVLBM_FP64 && precision != FVLBM_FP32_DEV && precision != FVLBM_FP32_DEV_GEO64) throw Error(FVLBM_EINVAL, "init: bad precision");
        if (p->n_groups != m->n_groups) throw Error(FVLBM_EINVAL, "init: params.n_groups differs from the mesh");
        if (!(p->nu > 0) || !(p->dt > 0) || !(p->rho0 > 0)) throw Error(FVLBM_EINVAL, "init: nu, dt and rho0 must be > 0 (tau = 3 nu)");
        if (p->sst < 0 || p->sst > 2) throw Error(FVLBM_EINVAL, "init: sst must be 0, 1 or 2");
        if (p->sst && (!k || !omega)) throw Error(FVLBM_EINVAL, "init: SST needs k and omega");
        if (p->limiter < 0 || p->limiter > 2) throw Error(FVLBM_EINVAL, "init: limiter must be 0, 1 or 2");
        if (p->sst_sweeps < 0 || p->sst_sweeps > kMaxSstSweeps) throw Error(FVLBM_EINVAL, "init: sst_sweeps must be in [0, " + std::to_string(kMaxSstSweeps) + "]");
        if (reinterpret_cast<uintptr_t>(workspace) % 256) throw Error(FVLBM_EINVAL, "init: workspace must be 256-byte aligned");
        const size_t need = layout_bytes(m, precision, p->sst ? 1 : 0);
        if (ws_bytes < need) throw Error(FVLBM_EINVAL, "init: workspace too small (" + std::to_string(ws_bytes) + " < " + std::to_string(need) + ")");
        auto st = std::make_unique<fvlbm_state>();
        st->mesh = m;
        st->precision = precision;
        st->sst = p->sst ? 1 : 0;
        st->sst_stages = p->sst == 2 ? 1 : 0;
        st->par = *p;
        st->par.bface_vals = nullptr;   // only used here, the caller's array is not kept
        st->stream = reinterpret_cast<hipStream_t>(hip_stream);
        check(hipGetDevice(&st->device), "hipGetDevice");
        st->noalloc = scratch_on(st->device);
        Carver cv;
        cv.base = reinterpret_cast<char *>(workspace);
        fvlbm_params pv = *p;
        if (precision == FVLBM_FP64) {
            carve<double>(cv, m, st->sst, st.get());
            st->par = pv;
            do_init<double>(st.get(), rho, u, k, omega);
        } else {
            st->fp64_geometry = precision == FVLBM_FP32_DEV_GEO64;
            carve<float>(cv, m, st->sst, st.get(), st->fp64_geometry);
            st->par = pv;
            do_init<float>(st.get(), rho, u, k, omega);
        }
        st->par.bface_vals = nullptr;
        *out = st.release();
    });
}

fvlbm_status fvlbm_set_state(fvlbm_state *st, const double *f, const double *k, const double *omega) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "set_state: NULL state");
        drop_recording(st);
        if ((k || omega) && !st->sst) throw Error(FVLBM_ESTATE, "set_state: k / omega given to a laminar state");
        if (st->precision == FVLBM_FP64)
            import_state<double>(st, f, k, omega);
        else
            import_state<float>(st, f, k, omega);
    });
}

fvlbm_status fvlbm_step(fvlbm_state *st, int32_t n_steps, double *res) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "step: NULL state");
        if (n_steps < 0) throw Error(FVLBM_EINVAL, "step: n_steps < 0");
        drop_recording(st);
        for (int32_t i = 0; i < n_steps; ++i) {
            if (st->precision == FVLBM_FP64)
                launch_step<double>(st);
            else
                launch_step<float>(st);
            if (st->timing && st->events.size() > 4096) drain_events(st);
        }
        st->steps_done += n_steps;
        if (res) {
            const double r = st->precision == FVLBM_FP64 ? residual<double>(st) : residual<float>(st);
            *res = r;
            if (!std::isfinite(r)) throw Error(FVLBM_EDIVERGED, "step: non-finite velocity residual");
        }
    });
}

fvlbm_status fvlbm_run_to_residual(fvlbm_state *st, int64_t max_steps, int32_t check_every, double tol,
                                   int64_t *steps_out, double *residual_out) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "run_to_residual: NULL state");
        if (max_steps < 1 || check_every < 1 || !(tol >= 0))
            throw Error(FVLBM_EINVAL, "run_to_residual: needs max_steps >= 1, check_every >= 1, tol >= 0");
        drop_recording(st);
        int64_t done = 0;
        double r = 0;
        if (steps_out) *steps_out = 0;
        while (done < max_steps) {
            const int32_t blk = (int32_t)std::min<int64_t>(check_every, max_steps - done);
            for (int32_t i = 0; i < blk; ++i) {
                if (st->precision == FVLBM_FP64)
                    launch_step<double>(st);
                else
                    launch_step<float>(st);
                if (st->timing && st->events.size() > 4096) drain_events(st);
            }
            done += blk;
            st->steps_done += blk;
            r = st->precision == FVLBM_FP64 ? residual<double>(st) : residual<float>(st);
            if (steps_out) *steps_out = done;
            if (residual_out) *residual_out = r;
            if (!std::isfinite(r)) throw Error(FVLBM_EDIVERGED, "run_to_residual: non-finite velocity residual");
            if (r < tol) break;
        }
    });
}

fvlbm_status fvlbm_step_explicit(fvlbm_state *st, int32_t n_steps, double *res) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "step_explicit: NULL state");
        if (n_steps < 0) throw Error(FVLBM_EINVAL, "step_explicit: n_steps < 0");
        drop_recording(st);
        for (int32_t i = 0; i < n_steps; ++i) {
            if (st->precision == FVLBM_FP64)
                launch_explicit<double>(st);
            else
                launch_explicit<float>(st);
            if (st->timing && st->events.size() > 4096) drain_events(st);
        }
        st->steps_done += n_steps;
        if (res) {
            const double r = st->precision == FVLBM_FP64 ? residual<double>(st) : residual<float>(st);
            *res = r;
            if (!std::isfinite(r)) throw Error(FVLBM_EDIVERGED, "step_explicit: non-finite velocity residual");
        }
    });
}

fvlbm_status fvlbm_moments(fvlbm_state *st, int32_t on_device, double *rho, double *u, double *k, double *omega,
                           double *nu_t, double tot[3]) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "moments: NULL state");
        if ((k || omega || nu_t) && !st->sst) throw Error(FVLBM_ESTATE, "moments: k / omega / nu_t of a laminar state");
        if (st->precision == FVLBM_FP64)
            export_moments<double>(st, on_device, rho, u, k, omega, nu_t);
        else
            export_moments<float>(st, on_device, rho, u, k, omega, nu_t);
        if (tot) {
            if (st->precision == FVLBM_FP64)
                totals<double>(st, tot);
            else
                totals<float>(st, tot);
            for (int i = 0; i < 3; ++i)
                if (!std::isfinite(tot[i])) throw Error(FVLBM_EDIVERGED, "moments: non-finite totals");
        }
    });
}

fvlbm_status fvlbm_totals_noalloc(fvlbm_state *st, double *totals_dev) {
    return guarded([&] {
        if (!st || !totals_dev) throw Error(FVLBM_EINVAL, "totals_noalloc: NULL argument");
        if (st->n_cells < 1) throw Error(FVLBM_EINVAL, "totals_noalloc: empty state");
        if (st->precision == FVLBM_FP64)
            totals_noalloc<double>(st, totals_dev);
        else
            totals_noalloc<float>(st, totals_dev);
    });
}

fvlbm_status fvlbm_get_f(fvlbm_state *st, int32_t on_device, double *f) {
    return guarded([&] {
        if (!st || !f) throw Error(FVLBM_EINVAL, "get_f: NULL argument");
        const int nbk = blocks_for(st->n_cells);
        double *target = on_device ? f : st->scratch;
        if (st->precision == FVLBM_FP64)
            k_export_f<double><<<nbk, kBlock, 0, st->stream>>>(st->geo64, (const double *)st->F, target, st->par.rho0);
        else
            k_export_f<float><<<nbk, kBlock, 0, st->stream>>>(st->geo32, (const float *)st->F, target, st->par.rho0);
        check(hipGetLastError(), "kernel launch");
        if (!on_device) {
            check(hipMemcpyAsync(f, st->scratch, 9 * (size_t)st->n_cells * sizeof(double), hipMemcpyDeviceToHost, st->stream), "hipMemcpyAsync D2H");
            check(hipStreamSynchronize(st->stream), "hipStreamSynchronize");
        }
    });
}

fvlbm_status fvlbm_forces(fvlbm_state *st, uint64_t mask, double force[2], double *j_r) {
    return guarded([&] {
        if (!st || !force) throw Error(FVLBM_EINVAL, "forces: NULL argument");
        double r[3];
        if (st->precision == FVLBM_FP64)
            forces<double>(st, mask, r);
        else
            forces<float>(st, mask, r);
        force[0] = r[0];
        force[1] = r[1];
        if (j_r) *j_r = r[2];
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(r[i])) throw Error(FVLBM_EDIVERGED, "forces: non-finite result");
    });
}

fvlbm_status fvlbm_lift_drag(fvlbm_state *st, uint64_t mask, double u_ref, double chord, double coeffs[2]) {
    return guarded([&] {
        if (!st || !coeffs) throw Error(FVLBM_EINVAL, "lift_drag: NULL argument");
        if (!(u_ref > 0) || !(chord > 0)) throw Error(FVLBM_EINVAL, "lift_drag: u_ref and chord must be positive");
        double r[3];
        if (st->precision == FVLBM_FP64)
            forces<double>(st, mask, r);
        else
            forces<float>(st, mask, r);
        if (!std::isfinite(r[0]) || !std::isfinite(r[1])) throw Error(FVLBM_EDIVERGED, "lift_drag: non-finite force");
        const double c = std::cos(st->par.theta), s = std::sin(st->par.theta);
        const double q = 0.5 * st->par.rho0 * u_ref * u_ref * chord;
        coeffs[0] = (-s * r[0] + c * r[1]) / q;
        coeffs[1] = (c * r[0] + s * r[1]) / q;
    });
}

fvlbm_status fvlbm_apply_advection(fvlbm_state *st, const double *g_in, double *out) {
    return guarded([&] {
        if (!st || !g_in || !out) throw Error(FVLBM_EINVAL, "apply_advection: NULL argument");
        if (st->precision == FVLBM_FP64)
            apply_advection<double>(st, g_in, out);
        else
            apply_advection<float>(st, g_in, out);
    });
}

fvlbm_status fvlbm_timing(fvlbm_state *st, int32_t enable) {
    return guarded([&] {
        if (!st) throw Error(FVLBM_EINVAL, "timing: NULL state");
        drain_events(st);
        if (enable) {
            for (int i = 0; i < FVLBM_K_COUNT; ++i) {
                st->t_ms[i] = 0;
                st->t_count[i] = 0;
            }
        }
        st->timing = enable != 0;
    });
}

fvlbm_status fvlbm_timing_read(fvlbm_state *st, double ms[FVLBM_K_COUNT], int64_t launches[FVLBM_K_COUNT]) {
    return guarded([&] {
        if (!st || !ms || !launches) throw Error(FVLBM_EINVAL, "timing_read: NULL argument");
        drain_events(st);
        for (int i = 0; i < FVLBM_K_COUNT; ++i) {
            ms[i] = st->t_ms[i];
            launches[i] = st->t_count[i];
        }
    });
}

fvlbm_status fvlbm_mesh_max_dt(const fvlbm_mesh *m, double *dt) {
    return guarded([&] {
        if (!m || !dt) throw Error(FVLBM_EINVAL, "mesh_max_dt: NULL argument");
        double worst = 0;
        const int64_t n = m->n;
        for (int64_t c = 0; c < n; ++c) {
            for (int a = 1; a < 9; ++a) {
                double out = 0;
                for (int s = 0; s < kSlots; ++s) {
                    const int64_t si = s * n + c;
                    if (m->nbr[si] == -1) continue;
                    out += std::max(0.0, ex(a) * m->nlx[si] + ey(a) * m->nly[si]);
                }
                worst = std::max(worst, out / m->area[c]);
            }
        }
        *dt = 1.0 / worst;
    });
}

fvlbm_status fvlbm_apply_advection_adjoint(fvlbm_state *st, const double *g_in, const double *lam, double *g_bar,
                                           double *d_theta) {
    return guarded([&] {
        if (!st || !g_in || !lam || !g_bar || !d_theta) throw Error(FVLBM_EINVAL, "apply_advection_adjoint: NULL argument");
        if (st->par.limiter) throw Error(FVLBM_ESTATE, "apply_advection_adjoint: the limited convection has no adjoint here");
        if (st->precision == FVLBM_FP64)
            apply_advection_adjoint<double>(st, g_in, lam, g_bar, d_theta);
        else
            apply_advection_adjoint<float>(st, g_in, lam, g_bar, d_theta);
    });
}

fvlbm_status fvlbm_adjoint_bytes(const fvlbm_mesh *m, int32_t precision, int32_t n_steps, int32_t ckpt_every,
                                 size_t *bytes) {
    return guarded([&] {
        if (!m || !bytes) throw Error(FVLBM_EINVAL, "adjoint_bytes: NULL argument");
        if (n_steps < 1 || ckpt_every < 1) throw Error(FVLBM_EINVAL, "adjoint_bytes: n_steps and ckpt_every must be >= 1");
        if (precision != FVLBM_FP64 && precision != FVLBM_FP32_DEV && precision != FVLBM_FP32_DEV_GEO64)
            throw Error(FVLBM_EINVAL, "adjoint_bytes: bad precision");
        Carver cv;
        if (precision == FVLBM_FP64) {
            AdjLayout<double> L;
            *bytes = adj_carve<double>(cv, m->n, n_steps, std::min(ckpt_every, n_steps), adjoint_two_sets(m), L);
        } else {
            AdjLayout<float> L;
            *bytes = adj_carve<float>(cv, m->n, n_steps, std::min(ckpt_every, n_steps), adjoint_two_sets(m), L);
        }
    });
}

fvlbm_status fvlbm_record(fvlbm_state *st, int32_t n_steps, int32_t ckpt_every, void *workspace, size_t ws_bytes) {
    return guarded([&] {
        if (!st || !workspace) throw Error(FVLBM_EINVAL, "record: NULL argument");
        if (n_steps < 1 || ckpt_every < 1) throw Error(FVLBM_EINVAL, "record: n_steps and ckpt_every must be >= 1");
        if (st->sst && st->par.sst_sweeps > kMaxAdjSstSweeps)
            throw Error(FVLBM_ESTATE, "record: the implicit SST variant's adjoint takes at most " + std::to_string(kMaxAdjSstSweeps) + " sweeps");
        if (reinterpret_cast<uintptr_t>(workspace) % 256) throw Error(FVLBM_EINVAL, "record: workspace must be 256-byte aligned");
        // the layout (as fvlbm_adjoint_bytes sizes it), fixed here for the adjoint calls that follow
        st->adj_two_sets = adjoint_two_sets(st->mesh);
        Carver cv;
        const int32_t ck = std::min(ckpt_every, n_steps);
        size_t need = 0;
        if (st->precision == FVLBM_FP64) {
            AdjLayout<double> L;
            need = adj_carve<double>(cv, st->n_cells, n_steps, ck, st->adj_two_sets, L);
        } else {
            AdjLayout<float> L;
            need = adj_carve<float>(cv, st->n_cells, n_steps, ck, st->adj_two_sets, L);
        }
        if (ws_bytes < need) throw Error(FVLBM_EINVAL, "record: workspace too small (" + std::to_string(ws_bytes) + " < " + std::to_string(need) + ")");
        st->adj_ws = reinterpret_cast<char *>(workspace);
        st->adj_bytes = ws_bytes;
        st->rec_steps = n_steps;
        st->rec_ckpt = std::min(ckpt_every, n_steps);
        if (st->precision == FVLBM_FP64)
            record<double>(st);
        else
            record<float>(st);
    });
}

fvlbm_status fvlbm_adjoint_step(fvlbm_state *st, uint64_t wall_group_mask, const double seed[3], double dparams[5]) {
    return guarded([&] {
        if (!st || !seed || !dparams) throw Error(FVLBM_EINVAL, "adjoint_step: NULL argument");
        if (!st->adj_ws) throw Error(FVLBM_ESTATE, "adjoint_step: no recorded run (call fvlbm_record first; a step or set_state since then drops it)");
        if (st->precision == FVLBM_FP64)
            adjoint_forces<double>(st, wall_group_mask, seed, dparams);
        else
            adjoint_forces<float>(st, wall_group_mask, seed, dparams);
        for (int i = 0; i < 5; ++i)
            if (!std::isfinite(dparams[i])) throw Error(FVLBM_EDIVERGED, "adjoint_step: non-finite gradient");
    });
}

fvlbm_status fvlbm_adjoint_lift_drag(fvlbm_state *st, uint64_t wall_group_mask, double u_ref, double chord,
                                     const double seed[2], double coeffs[2], double dparams[5]) {
    return guarded([&] {
        if (!st || !seed || !dparams) throw Error(FVLBM_EINVAL, "adjoint_lift_drag: NULL argument");
        if (!(u_ref > 0) || !(chord > 0)) throw Error(FVLBM_EINVAL, "adjoint_lift_drag: u_ref and chord must be positive");
        if (!st->adj_ws) throw Error(FVLBM_ESTATE, "adjoint_lift_drag: no recorded run (call fvlbm_record first; a step or set_state since then drops it)");
        // the force of the final (current) state
        double r[3];
        if (st->precision == FVLBM_FP64)
            forces<double>(st, wall_group_mask, r);
        else
            forces<float>(st, wall_group_mask, r);
        if (!std::isfinite(r[0]) || !std::isfinite(r[1])) throw Error(FVLBM_EDIVERGED, "adjoint_lift_drag: non-finite force");
        // C_l = F . (-sin, cos) / q, C_d = F . (cos, sin) / q with q = rho0 u_ref^2 chord / 2
        const double c = std::cos(st->par.theta), sn = std::sin(st->par.theta);
        const double q = 0.5 * st->par.rho0 * u_ref * u_ref * chord;
        const double cl = (-sn * r[0] + c * r[1]) / q, cd = (c * r[0] + sn * r[1]) / q;
        if (coeffs) {
            coeffs[0] = cl;
            coeffs[1] = cd;
        }
        // J = seed . (C_l, C_d): the adjoint of the force, then the explicit turn of the lift and drag
        // directions with theta, dC_l/dtheta = -C_d and dC_d/dtheta = C_l at fixed force
        const double sf[3] = {(-seed[0] * sn + seed[1] * c) / q, (seed[0] * c + seed[1] * sn) / q, 0.0};
        if (st->precision == FVLBM_FP64)
            adjoint_forces<double>(st, wall_group_mask, sf, dparams);
        else
            adjoint_forces<float>(st, wall_group_mask, sf, dparams);
        dparams[0] += -seed[0] * cd + seed[1] * cl;
        for (int i = 0; i < 5; ++i)
            if (!std::isfinite(dparams[i])) throw Error(FVLBM_EDIVERGED, "adjoint_lift_drag: non-finite gradient");
    });
}

fvlbm_status fvlbm_adjoint_state(fvlbm_state *st, const double *lam_f, const double *lam_k, const double *lam_w,
                                 double *lam_f0, double *lam_k0, double *lam_w0, double dparams[5]) {
    return guarded([&] {
        if (!st || !lam_f || !lam_f0 || !dparams) throw Error(FVLBM_EINVAL, "adjoint_state: NULL argument");
        if (!st->adj_ws) throw Error(FVLBM_ESTATE, "adjoint_state: no recorded run (call fvlbm_record first; a step or set_state since then drops it)");
        if (st->precision == FVLBM_FP64)
            adjoint_state<double>(st, lam_f, lam_k, lam_w, lam_f0, lam_k0, lam_w0, dparams);
        else
            adjoint_state<float>(st, lam_f, lam_k, lam_w, lam_f0, lam_k0, lam_w0, dparams);
    });
}

void fvlbm_state_destroy(fvlbm_state *st) { delete st; }

const char *fvlbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
