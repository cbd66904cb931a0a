// Host preprocessing of an unstructured 2D mesh (FP64): validation, edge matching, periodic
// pairing, cell geometry, least-squares coefficients, wall distance and cell renumbering.
//
// Geometry follows the finite-volume notation of the convection term, Eq. (advection) of
// arXiv 1812.00394: A = cell area, n = outward unit normal, dl = edge length, the face value taken
// at the edge midpoint.  The gradient of a cell field is the weighted least-squares fit over the
// edge neighbours (weights 1/|d|^2), with boundary edges contributing their midpoint.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>
#include <utility>

#include "internal.h"

namespace fvlbm {
namespace {

struct Seg {
    double ax, ay, bx, by;
};

double point_segment_dist2(double px, double py, const Seg &s) {
    double ex = s.bx - s.ax, ey = s.by - s.ay;
    double len2 = ex * ex + ey * ey;
    double t = len2 > 0 ? ((px - s.ax) * ex + (py - s.ay) * ey) / len2 : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    double qx = s.ax + t * ex - px, qy = s.ay + t * ey - py;
    return qx * qx + qy * qy;
}

// Bounding-volume hierarchy over wall segments for the exact nearest-wall query.
struct Bvh {
    struct Node {
        double lo[2], hi[2];
        int32_t left, right;   // children (internal node) or -1
        int32_t first, count;  // segment range (leaf)
    };
    std::vector<Seg> segs;
    std::vector<Node> nodes;

    int32_t build(int32_t first, int32_t count) {
        Node nd;
        nd.lo[0] = nd.lo[1] = std::numeric_limits<double>::infinity();
        nd.hi[0] = nd.hi[1] = -std::numeric_limits<double>::infinity();
        for (int32_t i = first; i < first + count; ++i) {
            const Seg &s = segs[i];
            nd.lo[0] = std::min({nd.lo[0], s.ax, s.bx});
            nd.lo[1] = std::min({nd.lo[1], s.ay, s.by});
            nd.hi[0] = std::max({nd.hi[0], s.ax, s.bx});
            nd.hi[1] = std::max({nd.hi[1], s.ay, s.by});
        }
        nd.left = nd.right = -1;
        nd.first = first;
        nd.count = count;
        int32_t id = (int32_t)nodes.size();
        nodes.push_back(nd);
        if (count > 4) {
            int axis = (nd.hi[0] - nd.lo[0]) >= (nd.hi[1] - nd.lo[1]) ? 0 : 1;
            int32_t mid = first + count / 2;
            std::nth_element(segs.begin() + first, segs.begin() + mid, segs.begin() + first + count,
                             [axis](const Seg &a, const Seg &b) {
                                 double ma = axis == 0 ? a.ax + a.bx : a.ay + a.by;
                                 double mb = axis == 0 ? b.ax + b.bx : b.ay + b.by;
                                 return ma < mb;
                             });
            int32_t l = build(first, mid - first);
            int32_t r = build(mid, first + count - mid);
            nodes[id].left = l;
            nodes[id].right = r;
        }
        return id;
    }

    static double box_dist2(const Node &n, double px, double py) {
        double dx = std::max({n.lo[0] - px, 0.0, px - n.hi[0]});
        double dy = std::max({n.lo[1] - py, 0.0, py - n.hi[1]});
        return dx * dx + dy * dy;
    }

    double query(double px, double py) const {
        double best = std::numeric_limits<double>::infinity();
        int32_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const Node &nd = nodes[stack[--sp]];
            if (box_dist2(nd, px, py) >= best) continue;
            if (nd.left < 0) {
                for (int32_t i = nd.first; i < nd.first + nd.count; ++i)
                    best = std::min(best, point_segment_dist2(px, py, segs[i]));
            } else {
                double dl = box_dist2(nodes[nd.left], px, py);
                double dr = box_dist2(nodes[nd.right], px, py);
                // push the farther child first so the nearer one is visited first
                if (dl < dr) {
                    stack[sp++] = nd.right;
                    stack[sp++] = nd.left;
                } else {
                    stack[sp++] = nd.left;
                    stack[sp++] = nd.right;
                }
            }
        }
        return std::sqrt(best);
    }
};

template <typename F>
void parallel_for(int64_t n, F &&fn) {
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 20000 || hw == 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + hw - 1) / hw;
    for (unsigned t = 0; t < hw; ++t) {
        int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([&fn, lo, hi] { fn(lo, hi); });
    }
    for (auto &t : th) t.join();
}

uint64_t spread_bits(uint64_t v) {  // 21 bits -> every other bit of 42
    v &= 0x1fffff;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

}  // namespace

// Builds the mesh; throws fvlbm::Error on invalid input.
// Tile-local slot code of a slot with no interior neighbour: -1 unused; the k-th boundary edge of
// the cell (in slot order) -2 - k, counting k in nbnd.
inline int16_t slot_code(int32_t nb, int &nbnd) {
    if (nb == -1) return -1;
    return (int16_t)(-2 - nbnd++);
}

fvlbm_mesh *build_mesh(int64_t n_nodes, const double *xy, int64_t n_cells, const int64_t *cell_ptr,
                       const int64_t *cell_nodes, int64_t n_bf, const int64_t *bf_nodes, const int32_t *bf_group,
                       int32_t n_groups, const int32_t *group_kind, const double *pshift, int32_t order) {
    if (n_nodes <= 0 || n_cells <= 0 || !xy || !cell_ptr || !cell_nodes)
        throw Error(FVLBM_EINVAL, "mesh_create: empty mesh or NULL array");
    if (n_cells > (int64_t)std::numeric_limits<int32_t>::max() / 8)
        throw Error(FVLBM_EINVAL, "mesh_create: too many cells for 32-bit indexing");
    if (n_bf < 0 || (n_bf > 0 && (!bf_nodes || !bf_group)))
        throw Error(FVLBM_EINVAL, "mesh_create: boundary arrays missing");
    if (n_groups < 0 || n_groups > FVLBM_MAX_GROUPS || (n_groups > 0 && !group_kind))
        throw Error(FVLBM_EINVAL, "mesh_create: n_groups must be in [0, 16]");
    if (order < FVLBM_ORDER_NONE || order > FVLBM_ORDER_TILES) throw Error(FVLBM_EINVAL, "mesh_create: bad order");
    auto m = std::make_unique<fvlbm_mesh>();
    m->n = n_cells;
    m->n_nodes = n_nodes;
    m->n_groups = n_groups;
    m->n_bfaces_user = n_bf;
    double shift[FVLBM_MAX_GROUPS][2] = {};
    for (int g = 0; g < n_groups; ++g) {
        if (group_kind[g] < FVLBM_WALL || group_kind[g] > FVLBM_PERIODIC)
            throw Error(FVLBM_EINVAL, "mesh_create: group kind out of range");
        m->kinds[g] = group_kind[g];
        if (pshift) {
            shift[g][0] = pshift[2 * g];
            shift[g][1] = pshift[2 * g + 1];
        }
    }
    if (cell_ptr[0] != 0) throw Error(FVLBM_EINVAL, "mesh_create: cell_ptr[0] must be 0");
    for (int64_t c = 0; c < n_cells; ++c) {
        int64_t nv = cell_ptr[c + 1] - cell_ptr[c];
        if (nv < 3 || nv > kSlots) throw Error(FVLBM_EMESH, "mesh_create: cells must have 3 or 4 nodes");
        m->max_faces = std::max<int32_t>(m->max_faces, (int32_t)nv);
    }
    const int64_t H = cell_ptr[n_cells];
    for (int64_t i = 0; i < H; ++i)
        if (cell_nodes[i] < 0 || cell_nodes[i] >= n_nodes) throw Error(FVLBM_EMESH, "mesh_create: node id out of range");
    for (int64_t i = 0; i < 2 * n_bf; ++i)
        if (bf_nodes[i] < 0 || bf_nodes[i] >= n_nodes) throw Error(FVLBM_EMESH, "mesh_create: boundary node id out of range");
    for (int64_t i = 0; i < n_bf; ++i)
        if (bf_group[i] < 0 || bf_group[i] >= n_groups) throw Error(FVLBM_EMESH, "mesh_create: boundary edge group out of range");

    // ---- cell area (shoelace) and centroid, user order ----
    std::vector<double> area(n_cells), cxu(n_cells), cyu(n_cells);
    std::vector<int64_t> hcell(H);
    for (int64_t c = 0; c < n_cells; ++c) {
        int64_t p0 = cell_ptr[c], nv = cell_ptr[c + 1] - p0;
        double a2 = 0, sx = 0, sy = 0;
        for (int64_t k = 0; k < nv; ++k) {
            int64_t i = cell_nodes[p0 + k], j = cell_nodes[p0 + (k + 1) % nv];
            double x0 = xy[2 * i], y0 = xy[2 * i + 1], x1 = xy[2 * j], y1 = xy[2 * j + 1];
            double cr = x0 * y1 - x1 * y0;
            a2 += cr;
            sx += (x0 + x1) * cr;
            sy += (y0 + y1) * cr;
            hcell[p0 + k] = c;
        }
        if (!(a2 > 0)) throw Error(FVLBM_EMESH, "mesh_create: non-positive area of cell " + std::to_string(c));
        area[c] = 0.5 * a2;
        cxu[c] = sx / (3.0 * a2);
        cyu[c] = sy / (3.0 * a2);
    }

    // ---- edge matching: sort the (node pair) keys of all half-edges ----
    auto hnodes = [&](int64_t h, int64_t &a, int64_t &b) {
        int64_t c = hcell[h], p0 = cell_ptr[c], nv = cell_ptr[c + 1] - p0, k = h - p0;
        a = cell_nodes[h];
        b = cell_nodes[p0 + (k + 1) % nv];
    };
    auto key_of = [&](int64_t a, int64_t b) { return std::min(a, b) * n_nodes + std::max(a, b); };
    std::vector<std::pair<int64_t, int64_t>> keys(H);
    for (int64_t h = 0; h < H; ++h) {
        int64_t a, b;
        hnodes(h, a, b);
        if (a == b) throw Error(FVLBM_EMESH, "mesh_create: degenerate edge");
        keys[h] = {key_of(a, b), h};
    }
    std::sort(keys.begin(), keys.end());
    std::vector<int64_t> partner(H, -1);   // user half-edge across an interior edge
    std::vector<int64_t> single;
    for (int64_t i = 0; i < H;) {
        int64_t j = i;
        while (j < H && keys[j].first == keys[i].first) ++j;
        if (j - i > 2) throw Error(FVLBM_EMESH, "mesh_create: an edge is shared by more than two cells");
        if (j - i == 2) {
            partner[keys[i].second] = keys[i + 1].second;
            partner[keys[i + 1].second] = keys[i].second;
            m->n_interior_edges++;
        } else {
            single.push_back(keys[i].second);
        }
        i = j;
    }
    // boundary edges given by the caller must match the unpaired half-edges one to one
    std::vector<std::pair<int64_t, int64_t>> bkeys(n_bf);
    for (int64_t i = 0; i < n_bf; ++i) bkeys[i] = {key_of(bf_nodes[2 * i], bf_nodes[2 * i + 1]), i};
    std::sort(bkeys.begin(), bkeys.end());
    for (int64_t i = 1; i < n_bf; ++i)
        if (bkeys[i].first == bkeys[i - 1].first) throw Error(FVLBM_EMESH, "mesh_create: duplicate boundary edge");
    if ((int64_t)single.size() != n_bf)
        throw Error(FVLBM_EMESH, "mesh_create: " + std::to_string(single.size()) + " unpaired edges but " +
                                     std::to_string(n_bf) + " boundary edges given");
    std::vector<int64_t> hbface(H, -1);
    for (int64_t h : single) {
        int64_t a, b;
        hnodes(h, a, b);
        int64_t k = key_of(a, b);
        auto it = std::lower_bound(bkeys.begin(), bkeys.end(), std::make_pair(k, (int64_t)-1));
        if (it == bkeys.end() || it->first != k)
            throw Error(FVLBM_EMESH, "mesh_create: a mesh boundary edge has no boundary group");
        hbface[h] = it->second;
    }
    // ---- periodic pairing: partner edge midpoint = midpoint + shift of the group ----
    std::vector<double> pshift_x(H, 0.0), pshift_y(H, 0.0);  // image offset of the neighbour
    {
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
        for (int64_t i = 0; i < n_nodes; ++i) {
            xmin = std::min(xmin, xy[2 * i]);
            xmax = std::max(xmax, xy[2 * i]);
            ymin = std::min(ymin, xy[2 * i + 1]);
            ymax = std::max(ymax, xy[2 * i + 1]);
        }
        double tol = 1e-9 * std::max(xmax - xmin, ymax - ymin);
        struct PE {
            int64_t qx, qy, h;
        };
        std::vector<PE> pes;
        for (int64_t h : single) {
            int32_t g = bf_group[hbface[h]];
            if (group_kind[g] != FVLBM_PERIODIC) continue;
            int64_t a, b;
            hnodes(h, a, b);
            double mx = 0.5 * (xy[2 * a] + xy[2 * b]), my = 0.5 * (xy[2 * a + 1] + xy[2 * b + 1]);
            pes.push_back({(int64_t)std::llround(mx / tol), (int64_t)std::llround(my / tol), h});
        }
        auto cmp = [](const PE &p, const PE &q) { return p.qx != q.qx ? p.qx < q.qx : p.qy < q.qy; };
        std::vector<PE> sorted = pes;
        std::sort(sorted.begin(), sorted.end(), cmp);
        for (const PE &p : pes) {
            int32_t g = bf_group[hbface[p.h]];
            int64_t a, b;
            hnodes(p.h, a, b);
            double tx = 0.5 * (xy[2 * a] + xy[2 * b]) + shift[g][0];
            double ty = 0.5 * (xy[2 * a + 1] + xy[2 * b + 1]) + shift[g][1];
            int64_t qx = std::llround(tx / tol), qy = std::llround(ty / tol);
            int64_t found = -1;
            for (int64_t ox = -1; ox <= 1 && found < 0; ++ox)
                for (int64_t oy = -1; oy <= 1 && found < 0; ++oy) {
                    PE key{qx + ox, qy + oy, 0};
                    auto it = std::lower_bound(sorted.begin(), sorted.end(), key, cmp);
                    if (it != sorted.end() && it->qx == key.qx && it->qy == key.qy) found = it->h;
                }
            if (found < 0) throw Error(FVLBM_EMESH, "mesh_create: periodic edge without a partner");
            partner[p.h] = found;
            pshift_x[p.h] = -shift[g][0];
            pshift_y[p.h] = -shift[g][1];
            hbface[p.h] = -2;   // periodic: treated as interior
        }
        for (const PE &p : pes)
            if (partner[partner[p.h]] != p.h) throw Error(FVLBM_EMESH, "mesh_create: periodic pairing is not mutual");
        m->n_interior_edges += (int64_t)pes.size() / 2;
    }
    m->n_boundary_edges = 0;
    for (int64_t h : single)
        if (hbface[h] >= 0) m->n_boundary_edges++;

    // ---- renumbering ----
    std::vector<int64_t> perm(n_cells);
    std::iota(perm.begin(), perm.end(), 0);
    if (order == FVLBM_ORDER_MORTON || order == FVLBM_ORDER_TILES) {
        double xmin = *std::min_element(cxu.begin(), cxu.end()), xmax = *std::max_element(cxu.begin(), cxu.end());
        double ymin = *std::min_element(cyu.begin(), cyu.end()), ymax = *std::max_element(cyu.begin(), cyu.end());
        double span = std::max(xmax - xmin, ymax - ymin);
        if (!(span > 0)) span = 1;
        std::vector<uint64_t> code(n_cells);
        const double q = (double)((1u << 21) - 1);
        for (int64_t c = 0; c < n_cells; ++c) {
            uint64_t ix = (uint64_t)((cxu[c] - xmin) / span * q);
            uint64_t iy = (uint64_t)((cyu[c] - ymin) / span * q);
            code[c] = spread_bits(ix) | (spread_bits(iy) << 1);
        }
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
        if (order == FVLBM_ORDER_TILES) {
            // Tiles of kTile cells grown breadth-first on the cell graph, each from the first cell
            // (in Morton order) not yet placed; a region that runs out of unplaced neighbours
            // continues from the next such cell.  The tiles keep the Morton order of their seeds and
            // the cells inside a tile their Morton order.  On anisotropic meshes a Morton tile of thin
            // cells is a long strip with a large halo; a graph-grown tile stays compact.
            std::vector<int64_t> rank(n_cells);
            for (int64_t i = 0; i < n_cells; ++i) rank[perm[i]] = i;
            std::vector<char> placed(n_cells, 0);
            std::vector<int64_t> out, queue;
            out.reserve(n_cells);
            int64_t next = 0;
            while ((int64_t)out.size() < n_cells) {
                const size_t start = out.size(), limit = std::min<size_t>(n_cells, start + kTile);
                queue.clear();
                size_t head = 0;
                while (out.size() < limit) {
                    if (head == queue.size()) {
                        while (next < n_cells && placed[perm[next]]) ++next;
                        if (next == n_cells) break;
                        queue.push_back(perm[next]);
                        placed[perm[next]] = 1;
                    }
                    const int64_t c = queue[head++];
                    out.push_back(c);
                    for (int64_t h = cell_ptr[c]; h < cell_ptr[c + 1]; ++h) {
                        if (partner[h] < 0) continue;
                        const int64_t v = hcell[partner[h]];
                        if (!placed[v]) {
                            placed[v] = 1;
                            queue.push_back(v);
                        }
                    }
                }
                for (size_t i = head; i < queue.size(); ++i) placed[queue[i]] = 0;   // queued, not taken
                std::sort(out.begin() + start, out.end(), [&](int64_t a, int64_t b) { return rank[a] < rank[b]; });
            }
            perm = out;
        }
    } else if (order == FVLBM_ORDER_RCM) {
        std::vector<int32_t> deg(n_cells, 0);
        for (int64_t h = 0; h < H; ++h)
            if (partner[h] >= 0) deg[hcell[h]]++;
        std::vector<char> seen(n_cells, 0);
        std::vector<int64_t> out;
        out.reserve(n_cells);
        std::vector<int64_t> byDeg(n_cells);
        std::iota(byDeg.begin(), byDeg.end(), 0);
        std::stable_sort(byDeg.begin(), byDeg.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
        for (int64_t s : byDeg) {
            if (seen[s]) continue;
            size_t head = out.size();
            out.push_back(s);
            seen[s] = 1;
            while (head < out.size()) {
                int64_t c = out[head++];
                std::vector<int64_t> nb;
                for (int64_t h = cell_ptr[c]; h < cell_ptr[c + 1]; ++h)
                    if (partner[h] >= 0 && !seen[hcell[partner[h]]]) nb.push_back(hcell[partner[h]]);
                std::stable_sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
                for (int64_t v : nb)
                    if (!seen[v]) {
                        seen[v] = 1;
                        out.push_back(v);
                    }
            }
        }
        std::reverse(out.begin(), out.end());
        perm = out;
    }
    m->perm = perm;
    m->iperm.assign(n_cells, 0);
    for (int64_t i = 0; i < n_cells; ++i) m->iperm[perm[i]] = i;

    // ---- per-cell and per-slot arrays in internal order ----
    const int64_t N = n_cells;
    m->area.resize(N);
    m->xc.resize(N);
    m->yc.resize(N);
    for (int64_t i = 0; i < N; ++i) {
        m->area[i] = area[perm[i]];
        m->xc[i] = cxu[perm[i]];
        m->yc[i] = cyu[perm[i]];
    }
    // vertex offsets from the centroid of triangle cells (exact differences of nearby values)
    m->tri_p.assign(6 * N, 0.0);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t u = perm[i], p0 = cell_ptr[u];
        if (cell_ptr[u + 1] - p0 != 3) continue;
        for (int k = 0; k < 3; ++k) {
            const int64_t v = cell_nodes[p0 + k];
            m->tri_p[(2 * k) * N + i] = xy[2 * v] - cxu[u];
            m->tri_p[(2 * k + 1) * N + i] = xy[2 * v + 1] - cyu[u];
        }
    }
    m->nbr.assign(kSlots * N, -1);
    m->rev.assign(kSlots * N, 0);
    for (auto *v : {&m->nlx, &m->nly, &m->rfx, &m->rfy, &m->dx, &m->dy, &m->cx, &m->cy}) v->assign(kSlots * N, 0.0);
    for (auto *v : {&m->mi00, &m->mi01, &m->mi11}) v->assign(N, 0.0);
    for (int64_t i = 0; i < N; ++i) {
        int64_t u = perm[i], p0 = cell_ptr[u], nv = cell_ptr[u + 1] - p0;
        double M00 = 0, M01 = 0, M11 = 0;
        for (int64_t k = 0; k < nv; ++k) {
            int64_t h = p0 + k, a, b;
            hnodes(h, a, b);
            double ax = xy[2 * a], ay = xy[2 * a + 1], bx = xy[2 * b], by = xy[2 * b + 1];
            int64_t s = k * N + i;
            m->nlx[s] = by - ay;
            m->nly[s] = -(bx - ax);
            double fx = 0.5 * (ax + bx), fy = 0.5 * (ay + by);
            m->rfx[s] = fx - cxu[u];
            m->rfy[s] = fy - cyu[u];
            if (partner[h] >= 0) {
                int64_t nb = hcell[partner[h]];
                m->nbr[s] = (int32_t)m->iperm[nb];
                m->rev[s] = (int8_t)(partner[h] - cell_ptr[nb]);
                m->dx[s] = cxu[nb] + pshift_x[h] - cxu[u];
                m->dy[s] = cyu[nb] + pshift_y[h] - cyu[u];
            } else {
                int64_t bi = (int64_t)m->b_cell.size();
                m->nbr[s] = (int32_t)(-2 - bi);
                m->dx[s] = m->rfx[s];
                m->dy[s] = m->rfy[s];
                int64_t ub = hbface[h];
                int32_t g = bf_group[ub];
                double l = std::sqrt(m->nlx[s] * m->nlx[s] + m->nly[s] * m->nly[s]);
                m->b_cell.push_back((int32_t)i);
                m->b_group.push_back(g);
                m->b_kind.push_back(group_kind[g]);
                m->b_user.push_back(ub);
                m->b_l.push_back(l);
                m->b_nx.push_back(m->nlx[s] / l);
                m->b_ny.push_back(m->nly[s] / l);
                m->b_dperp.push_back((m->rfx[s] * m->nlx[s] + m->rfy[s] * m->nly[s]) / l);
                m->b_xfx.push_back(fx);
                m->b_xfy.push_back(fy);
            }
            double w = 1.0 / (m->dx[s] * m->dx[s] + m->dy[s] * m->dy[s]);
            M00 += w * m->dx[s] * m->dx[s];
            M01 += w * m->dx[s] * m->dy[s];
            M11 += w * m->dy[s] * m->dy[s];
        }
        double det = M00 * M11 - M01 * M01;
        if (!(det > 1e-14 * (M00 * M11))) throw Error(FVLBM_EMESH, "mesh_create: degenerate least-squares stencil");
        double i00 = M11 / det, i01 = -M01 / det, i11 = M00 / det;
        m->mi00[i] = i00;
        m->mi01[i] = i01;
        m->mi11[i] = i11;
        for (int64_t k = 0; k < nv; ++k) {
            int64_t s = k * N + i;
            double w = 1.0 / (m->dx[s] * m->dx[s] + m->dy[s] * m->dy[s]);
            m->cx[s] = w * (i00 * m->dx[s] + i01 * m->dy[s]);
            m->cy[s] = w * (i01 * m->dx[s] + i11 * m->dy[s]);
        }
    }

    // first boundary edge of each cell (its boundary edges are consecutive, in slot order)
    m->bfirst.assign(N, -1);
    for (size_t b = m->b_cell.size(); b-- > 0;) m->bfirst[m->b_cell[b]] = (int32_t)b;

    // ---- tiles and halos for the fused stage kernels ----
    m->n_tiles = (int32_t)((N + kTile - 1) / kTile);
    m->halo_ptr.assign(m->n_tiles + 1, 0);
    m->ext_ptr.assign(m->n_tiles + 1, 0);
    m->ext_n1.assign(m->n_tiles, 0);
    m->lnb.assign(kSlots * N, 0);
    std::vector<int16_t> ext_lnb_rows;
    for (int32_t t = 0; t < m->n_tiles; ++t) {
        const int64_t lo = (int64_t)t * kTile, hi = std::min<int64_t>(N, lo + kTile);
        std::vector<int32_t> halo;
        for (int64_t c = lo; c < hi; ++c)
            for (int s = 0; s < kSlots; ++s) {
                const int32_t nb = m->nbr[s * N + c];
                if (nb >= 0 && (nb < lo || nb >= hi)) halo.push_back(nb);
            }
        std::sort(halo.begin(), halo.end());
        halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
        for (int64_t c = lo; c < hi; ++c) {
            int nbnd = 0;
            for (int s = 0; s < kSlots; ++s) {
                const int32_t nb = m->nbr[s * N + c];
                if (nb < 0) {
                    m->lnb[s * N + c] = slot_code(nb, nbnd);
                    continue;
                }
                int64_t local;
                if (nb >= lo && nb < hi)
                    local = nb - lo;
                else
                    local = kTile + (std::lower_bound(halo.begin(), halo.end(), nb) - halo.begin());
                if (local > 32767) throw Error(FVLBM_EMESH, "mesh_create: tile halo too large");
                m->lnb[s * N + c] = (int16_t)local;
            }
        }
        m->halo_ptr[t + 1] = m->halo_ptr[t] + (int32_t)halo.size();
        m->halo_max = std::max<int32_t>(m->halo_max, (int32_t)halo.size());
        m->halo_cell.insert(m->halo_cell.end(), halo.begin(), halo.end());
        // second ring: interior neighbours of ring-1 cells outside the tile and ring 1
        std::vector<int32_t> ring2;
        for (int32_t h : halo)
            for (int s = 0; s < kSlots; ++s) {
                const int32_t nb = m->nbr[s * N + h];
                if (nb < 0 || (nb >= lo && nb < hi) || std::binary_search(halo.begin(), halo.end(), nb)) continue;
                ring2.push_back(nb);
            }
        std::sort(ring2.begin(), ring2.end());
        ring2.erase(std::unique(ring2.begin(), ring2.end()), ring2.end());
        const size_t e0 = m->ext_cell.size();
        m->ext_cell.insert(m->ext_cell.end(), halo.begin(), halo.end());
        m->ext_cell.insert(m->ext_cell.end(), ring2.begin(), ring2.end());
        m->ext_ptr[t + 1] = (int32_t)m->ext_cell.size();
        m->ext_n1[t] = (int32_t)halo.size();
        m->ext_max = std::max<int32_t>(m->ext_max, (int32_t)(halo.size() + ring2.size()));
        // tile-local column of each ring-1 cell's neighbours: tile cells c - lo, ext entry j kTile + j
        ext_lnb_rows.resize(m->ext_cell.size() * kSlots, 0);
        for (size_t j = 0; j < halo.size(); ++j) {
            int nbnd = 0;
            for (int s = 0; s < kSlots; ++s) {
                const int32_t nb = m->nbr[s * N + halo[j]];
                if (nb < 0) {
                    ext_lnb_rows[(e0 + j) * kSlots + s] = slot_code(nb, nbnd);
                    continue;
                }
                int64_t local;
                if (nb >= lo && nb < hi)
                    local = nb - lo;
                else if (std::binary_search(halo.begin(), halo.end(), nb))
                    local = kTile + (std::lower_bound(halo.begin(), halo.end(), nb) - halo.begin());
                else
                    local = kTile + (int64_t)halo.size() + (std::lower_bound(ring2.begin(), ring2.end(), nb) - ring2.begin());
                if (local > 32767) throw Error(FVLBM_EMESH, "mesh_create: tile halo too large");
                ext_lnb_rows[(e0 + j) * kSlots + s] = (int16_t)local;
            }
        }
    }
    // ring-1 neighbour columns as [kSlots][n_ext]
    {
        const size_t ne = m->ext_cell.size();
        m->ext_lnb.assign(kSlots * std::max<size_t>(ne, 1), 0);
        for (size_t e = 0; e < ne; ++e)
            for (int s = 0; s < kSlots; ++s) m->ext_lnb[s * ne + e] = ext_lnb_rows[e * kSlots + s];
    }

    // ---- wall distance: exact nearest point over WALL / MOVING_WALL edges ----
    m->wdist.assign(N, kNoWallDistance);
    Bvh bvh;
    for (int64_t i = 0; i < n_bf; ++i) {
        int32_t k = group_kind[bf_group[i]];
        if (k != FVLBM_WALL && k != FVLBM_MOVING_WALL) continue;
        int64_t a = bf_nodes[2 * i], b = bf_nodes[2 * i + 1];
        bvh.segs.push_back({xy[2 * a], xy[2 * a + 1], xy[2 * b], xy[2 * b + 1]});
    }
    if (!bvh.segs.empty()) {
        bvh.build(0, (int32_t)bvh.segs.size());
        parallel_for(N, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) m->wdist[i] = bvh.query(m->xc[i], m->yc[i]);
        });
    }
    return m.release();
}

}  // namespace fvlbm
