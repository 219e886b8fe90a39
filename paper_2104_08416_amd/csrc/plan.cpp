// plan.cpp -- host setup: GLL basis, global numbering, geometry, element/node reordering,
// workgroup tiling. Built with -ffp-contract=off so the centroid and cell arithmetic of
// the curve ordering is evaluated exactly as written (no fused multiply-add).
#include "plan.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>

#include "../../include/sem.h"

namespace sem {
namespace {

// ------------------------------------------------------------------ GLL basis on [-1, 1]
// Legendre P_p, P_p' and P_p'' at x from the recurrences
//   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},  P'_{k+1} = P'_{k-1} + (2k+1) P_k,
//   P''_{k+1} = P''_{k-1} + (2k+1) P'_k.
void legendre_all(int p, double x, double& P, double& dP, double& d2P) {
    double p0 = 1.0, p1 = x;          // P_{k-1}, P_k
    double d0 = 0.0, d1 = 1.0;        // P'_{k-1}, P'_k
    double s0 = 0.0, s1 = 0.0;        // P''_{k-1}, P''_k
    if (p == 0) { P = 1.0; dP = 0.0; d2P = 0.0; return; }
    for (int k = 1; k < p; ++k) {
        const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        const double d2 = d0 + (2 * k + 1) * p1;
        const double s2 = s0 + (2 * k + 1) * d1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2; s0 = s1; s1 = s2;
    }
    P = p1; dP = d1; d2P = s1;
}

// Interior GLL nodes are the roots of P_p'; Newton's method from Chebyshev extrema.
void gll_basis(int p, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D) {
    const int n = p + 1;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP, d2P;
            legendre_all(p, t, P, dP, d2P);
            const double step = dP / d2P;
            t -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < n / 2; ++i) {            // exact symmetry
        const double s = 0.5 * (x[p - i] - x[i]);
        x[i] = -s;
        x[p - i] = s;
    }
    if (p % 2 == 0) x[p / 2] = 0.0;
    for (int i = 0; i < n; ++i) {
        double P, dP, d2P;
        legendre_all(p, x[i], P, dP, d2P);
        w[i] = 2.0 / (p * (p + 1) * P * P);
    }
    // derivative matrix from barycentric weights: D_ij = (b_j / b_i) / (x_i - x_j)
    std::vector<double> b(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) b[j] /= (x[j] - x[k]);
    D.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i * n + j] = (b[j] / b[i]) / (x[i] - x[j]);
            s += D[i * n + j];
        }
        D[i * n + i] = -s;
    }
}

// --------------------------------------------------------------- original numbering
inline int lidx(int a, int b, int p) { return a + (p + 1) * b; }

// local (a, b) of step t along local edge k (corner k -> corner k+1)
inline void edge_ab(int k, int t, int p, int& a, int& b) {
    switch (k) {
        case 0: a = t; b = 0; break;
        case 1: a = p; b = t; break;
        case 2: a = p - t; b = p; break;
        default: a = 0; b = p - t; break;
    }
}

std::string number_nodes(const MeshIn& m, int p, std::vector<int32_t>& conn, int64_t& nn) {
    const int n = p + 1, nq = n * n;
    const int64_t ne = m.ne, nv = m.nv;
    std::vector<uint8_t> used(nv, 0);
    for (int64_t i = 0; i < ne * 4; ++i) {
        const int32_t v = m.quad[i];
        if (v < 0 || v >= nv) return "vertex id out of range";
        used[v] = 1;
    }
    for (int64_t v = 0; v < nv; ++v)
        if (!used[v]) return "vertex " + std::to_string(v) + " is not used by any element";
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* q = m.quad + 4 * e;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                if (q[i] == q[j]) return "element " + std::to_string(e) + " repeats a vertex";
    }
    // every (element, local edge) with its unordered vertex pair; rank edges by first use
    struct EdgeUse { int64_t key; int64_t pos; };
    std::vector<EdgeUse> uses(ne * 4);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 4; ++k) {
            const int64_t s = m.quad[4 * e + k], f = m.quad[4 * e + (k + 1) % 4];
            uses[4 * e + k] = {std::min(s, f) * nv + std::max(s, f), 4 * e + k};
        }
    std::vector<EdgeUse> sorted = uses;
    std::sort(sorted.begin(), sorted.end(), [](const EdgeUse& a, const EdgeUse& b) {
        return a.key != b.key ? a.key < b.key : a.pos < b.pos;
    });
    std::vector<int64_t> first_pos;      // per distinct edge, in key order
    std::vector<int64_t> edge_of_use(ne * 4);
    for (size_t i = 0; i < sorted.size();) {
        size_t j = i;
        while (j < sorted.size() && sorted[j].key == sorted[i].key) ++j;
        if (j - i > 2) return "an edge is shared by more than two elements";
        if (j - i == 2) {
            const int64_t pa = sorted[i].pos, pb = sorted[i + 1].pos;
            if (m.quad[pa] == m.quad[pb])
                return "elements " + std::to_string(pa / 4) + " and " + std::to_string(pb / 4) +
                       " traverse their shared edge in the same direction (orientation)";
        }
        for (size_t k = i; k < j; ++k) edge_of_use[sorted[k].pos] = (int64_t)first_pos.size();
        first_pos.push_back(sorted[i].pos);
        i = j;
    }
    const int64_t nedge = (int64_t)first_pos.size();
    std::vector<int64_t> by_first(nedge);
    std::iota(by_first.begin(), by_first.end(), 0);
    std::sort(by_first.begin(), by_first.end(),
              [&](int64_t a, int64_t b) { return first_pos[a] < first_pos[b]; });
    std::vector<int64_t> rank(nedge);
    for (int64_t r = 0; r < nedge; ++r) rank[by_first[r]] = r;

    const int pe = p - 1;
    const int64_t base_int = nv + nedge * pe;
    nn = base_int + ne * (int64_t)pe * pe;
    if (nn > INT32_MAX) return "mesh too large for 32-bit node ids";
    conn.assign(ne * nq, -1);
    static const int cab[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int64_t e = 0; e < ne; ++e) {
        int32_t* c = conn.data() + e * nq;
        const int32_t* q = m.quad + 4 * e;
        for (int k = 0; k < 4; ++k) c[lidx(cab[k][0] * p, cab[k][1] * p, p)] = q[k];
        for (int k = 0; k < 4; ++k) {
            const int32_t s = q[k], f = q[(k + 1) % 4];
            const int64_t r = rank[edge_of_use[4 * e + k]];
            for (int t = 1; t < p; ++t) {
                int a, b;
                edge_ab(k, t, p, a, b);
                const int off = s < f ? t - 1 : p - 1 - t;
                c[lidx(a, b, p)] = (int32_t)(nv + r * pe + off);
            }
        }
        for (int b = 1; b < p; ++b)
            for (int a = 1; a < p; ++a)
                c[lidx(a, b, p)] = (int32_t)(base_int + e * pe * pe + (a - 1) + pe * (b - 1));
    }
    return "";
}

// ------------------------------------------------------------------------- geometry
struct Corners { double x[4], y[4]; };

inline Corners corners(const MeshIn& m, int64_t e) {
    Corners c;
    for (int k = 0; k < 4; ++k) {
        const int32_t v = m.quad[4 * e + k];
        c.x[k] = m.vxy[2 * v];
        c.y[k] = m.vxy[2 * v + 1];
    }
    return c;
}

inline void map_point(const Corners& c, double s, double t, double& x, double& y) {
    const double n0 = 0.25 * (1 - s) * (1 - t), n1 = 0.25 * (1 + s) * (1 - t);
    const double n2 = 0.25 * (1 + s) * (1 + t), n3 = 0.25 * (1 - s) * (1 + t);
    x = n0 * c.x[0] + n1 * c.x[1] + n2 * c.x[2] + n3 * c.x[3];
    y = n0 * c.y[0] + n1 * c.y[1] + n2 * c.y[2] + n3 * c.y[3];
}

// Jacobian columns of the bilinear map at (s, t)
inline void jac(const Corners& c, double s, double t, double& xs, double& xt, double& ys,
                double& yt) {
    xs = 0.25 * ((1 - t) * (c.x[1] - c.x[0]) + (1 + t) * (c.x[2] - c.x[3]));
    ys = 0.25 * ((1 - t) * (c.y[1] - c.y[0]) + (1 + t) * (c.y[2] - c.y[3]));
    xt = 0.25 * ((1 - s) * (c.x[3] - c.x[0]) + (1 + s) * (c.x[2] - c.x[1]));
    yt = 0.25 * ((1 - s) * (c.y[3] - c.y[0]) + (1 + s) * (c.y[2] - c.y[1]));
}

// ------------------------------------------------------------------------- orders
uint64_t splitmix64(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// spread the low 32 bits of v to the even bit positions
inline uint64_t spread_bits(uint64_t v) {
    v &= 0xFFFFFFFFull;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// Descend the generalized Hilbert construction (a region = origin, major axis A of w
// cells, minor axis B of h cells; entered at the origin, left at the far end of its
// first row along A) into the one sub-region holding the cell, adding the cell counts
// of the sub-regions the curve visits before it.
int64_t hilbert_index(int64_t W, int64_t H, int64_t cx, int64_t cy) {
    int64_t x = 0, y = 0, ax, ay, bx, by;
    if (W >= H) { ax = W; ay = 0; bx = 0; by = H; }
    else { ax = 0; ay = H; bx = W; by = 0; }
    int64_t index = 0;
    auto sgn = [](int64_t v) -> int64_t { return (v > 0) - (v < 0); };
    for (;;) {
        const int64_t w = std::llabs(ax + ay), h = std::llabs(bx + by);
        const int64_t dax = sgn(ax), day = sgn(ay), dbx = sgn(bx), dby = sgn(by);
        // coordinates of the cell in this region's frame
        const int64_t i = (cx - x) * dax + (cy - y) * day;   // along A
        const int64_t j = (cx - x) * dbx + (cy - y) * dby;   // along B
        if (h == 1) return index + i;
        if (w == 1) return index + j;
        int64_t w2 = w / 2, h2 = h / 2;
        if (2 * w > 3 * h) {
            if ((w2 & 1) && w > 2) ++w2;
            if (i < w2) {
                ax = w2 * dax; ay = w2 * day;
            } else {
                index += w2 * h;
                x += w2 * dax; y += w2 * day;
                ax -= w2 * dax; ay -= w2 * day;
            }
        } else {
            if ((h2 & 1) && h > 2) ++h2;
            const int64_t bx2 = h2 * dbx, by2 = h2 * dby, ax2 = w2 * dax, ay2 = w2 * day;
            if (j >= h2) {                       // upper rows, original axes
                index += w2 * h2;
                x += bx2; y += by2;
                bx -= bx2; by -= by2;
            } else if (i < w2) {                 // near part of the first rows, swapped
                const int64_t nax = bx2, nay = by2;
                bx = ax2; by = ay2;
                ax = nax; ay = nay;
            } else {                             // far part, swapped and reversed
                index += w2 * h2 + w * (h - h2);
                const int64_t nx = x + (ax - dax) + (bx2 - dbx);
                const int64_t ny = y + (ay - day) + (by2 - dby);
                const int64_t nbx = -(ax - ax2), nby = -(ay - ay2);
                x = nx; y = ny;
                ax = -bx2; ay = -by2;
                bx = nbx; by = nby;
            }
        }
    }
}

void nearest_nodes(const Plan& plan, int64_t n, const double* xy, int32_t* out) {
    if (n <= 0) return;
    const int64_t nn = plan.nn;
    const double* nxy = plan.node_xy.data();
    // nodes bucketed on a uniform grid of about two nodes per cell over their bounding box
    double x0 = nxy[0], x1 = nxy[0], y0 = nxy[1], y1 = nxy[1];
    for (int64_t i = 1; i < nn; ++i) {
        x0 = std::min(x0, nxy[2 * i]); x1 = std::max(x1, nxy[2 * i]);
        y0 = std::min(y0, nxy[2 * i + 1]); y1 = std::max(y1, nxy[2 * i + 1]);
    }
    const double w = std::max(x1 - x0, 1e-300), hgt = std::max(y1 - y0, 1e-300);
    const double h = std::max(std::sqrt(2.0 * w * hgt / (double)nn), std::max(w, hgt) / 65536.0);
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(65536, (int64_t)(w / h) + 1));
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(65536, (int64_t)(hgt / h) + 1));
    auto cell_x = [&](double x) { return std::min<int64_t>(gx - 1, std::max<int64_t>(0, (int64_t)std::floor((x - x0) / h))); };
    auto cell_y = [&](double y) { return std::min<int64_t>(gy - 1, std::max<int64_t>(0, (int64_t)std::floor((y - y0) / h))); };
    std::vector<int64_t> start(gx * gy + 1, 0);
    std::vector<int32_t> ids(nn);
    for (int64_t i = 0; i < nn; ++i) start[cell_y(nxy[2 * i + 1]) * gx + cell_x(nxy[2 * i]) + 1]++;
    for (int64_t c = 0; c < gx * gy; ++c) start[c + 1] += start[c];
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < nn; ++i) ids[fill[cell_y(nxy[2 * i + 1]) * gx + cell_x(nxy[2 * i])]++] = (int32_t)i;
    }
    for (int64_t k = 0; k < n; ++k) {
        const double px = xy[2 * k], py = xy[2 * k + 1];
        const int64_t cx = cell_x(px), cy = cell_y(py);
        int32_t best = -1;
        double bd = INFINITY;
        // rings of cells at Chebyshev distance r around the point's (clamped) cell; every node
        // outside the (2r+1)^2 block lies at least `gap` from the point
        for (int64_t r = 0;; ++r) {
            for (int64_t yy = cy - r; yy <= cy + r; ++yy) {
                if (yy < 0 || yy >= gy) continue;
                const bool edge_row = yy == cy - r || yy == cy + r;
                for (int64_t xx = cx - r; xx <= cx + r; xx += (edge_row || r == 0) ? 1 : 2 * r) {
                    if (xx < 0 || xx >= gx) continue;
                    const int64_t c = yy * gx + xx;
                    for (int64_t t = start[c]; t < start[c + 1]; ++t) {
                        const int32_t i = ids[t];
                        const double dx = nxy[2 * i] - px, dy = nxy[2 * i + 1] - py;
                        const double d = dx * dx + dy * dy;
                        if (d < bd || (d == bd && i < best)) { bd = d; best = i; }
                    }
                }
            }
            if (cx - r <= 0 && cy - r <= 0 && cx + r >= gx - 1 && cy + r >= gy - 1) break;   // all cells seen
            const double bx0 = x0 + (double)(cx - r) * h, bx1 = x0 + (double)(cx + r + 1) * h;
            const double by0 = y0 + (double)(cy - r) * h, by1 = y0 + (double)(cy + r + 1) * h;
            const double gap = std::min(std::min(px - bx0, bx1 - px), std::min(py - by0, by1 - py));
            // stop once nothing outside the block can be as close (a relative margin covers the
            // rounding of the block edges; equal distances must still be compared by id)
            if (best >= 0 && gap > 0.0 && gap * gap > bd * (1.0 + 1e-9)) break;
        }
        out[k] = best;
    }
}

// Element order of the benchmark section's node-walk strategies (Sec. 5): a breadth-first
// (Cuthill-McKee) walk over the mesh vertices, two vertices being neighbours when they
// share an element. The walk starts at the vertex of least priority (restarting there
// among unvisited vertices for further components) and queues each visited vertex's
// unvisited neighbours in ascending (priority, id); every visited vertex lists its
// not-yet-listed elements in ascending id. Priority: the vertex degree (distinct
// neighbours) or, with by_distance, the squared distance to (min x, min y).
static std::vector<int32_t> vertex_walk(const MeshIn& m, bool by_distance) {
    const int64_t nv = m.nv, ne = m.ne;
    const int K = m.nvpe;
    // elements of every vertex, ascending (corners of a valid element are distinct)
    std::vector<int32_t> v2e_b(nv + 1, 0), v2e((size_t)ne * K);
    for (int64_t i = 0; i < ne * K; ++i) v2e_b[m.quad[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) v2e_b[v + 1] += v2e_b[v];
    {
        std::vector<int32_t> fill(v2e_b.begin(), v2e_b.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < K; ++k) v2e[fill[m.quad[K * e + k]]++] = (int32_t)e;
    }
    std::vector<int32_t> stamp(nv, -1), nbr;
    auto neighbours = [&](int32_t v) {
        nbr.clear();
        stamp[v] = v;
        for (int32_t i = v2e_b[v]; i < v2e_b[v + 1]; ++i)
            for (int k = 0; k < K; ++k) {
                const int32_t w = m.quad[K * (int64_t)v2e[i] + k];
                if (stamp[w] != v) { stamp[w] = v; nbr.push_back(w); }
            }
    };
    std::vector<double> prio(nv);
    if (by_distance) {
        double x0 = INFINITY, y0 = INFINITY;
        for (int64_t v = 0; v < nv; ++v) {
            x0 = std::min(x0, m.vxy[2 * v]);
            y0 = std::min(y0, m.vxy[2 * v + 1]);
        }
        for (int64_t v = 0; v < nv; ++v) {
            const double dx = m.vxy[2 * v] - x0, dy = m.vxy[2 * v + 1] - y0;
            prio[v] = dx * dx + dy * dy;
        }
    } else {
        for (int64_t v = 0; v < nv; ++v) {
            neighbours((int32_t)v);
            prio[v] = (double)nbr.size();
        }
        std::fill(stamp.begin(), stamp.end(), -1);
    }
    auto before = [&](int32_t a, int32_t b) { return prio[a] < prio[b] || (prio[a] == prio[b] && a < b); };
    std::vector<int32_t> starts(nv);
    std::iota(starts.begin(), starts.end(), 0);
    std::sort(starts.begin(), starts.end(), before);
    std::vector<uint8_t> visited(nv, 0), listed(ne, 0);
    std::vector<int32_t> queue, order;
    queue.reserve(nv);
    order.reserve(ne);
    for (int32_t s : starts) {
        if (visited[s]) continue;
        visited[s] = 1;
        queue.clear();
        queue.push_back(s);
        for (size_t head = 0; head < queue.size(); ++head) {
            const int32_t v = queue[head];
            for (int32_t i = v2e_b[v]; i < v2e_b[v + 1]; ++i)
                if (!listed[v2e[i]]) { listed[v2e[i]] = 1; order.push_back(v2e[i]); }
            neighbours(v);
            size_t k0 = queue.size();
            for (int32_t w : nbr)
                if (!visited[w]) { visited[w] = 1; queue.push_back(w); }
            std::sort(queue.begin() + k0, queue.end(), before);
        }
    }
    return order;
}

void build_tiles(Plan& P, int tile_elems, int tile_items, int max_owned, bool split_single) {
    const int64_t ne = P.ne, nq = P.nq;
    // node -> incident elements (new numbering)
    std::vector<int32_t> n2e_b(P.nn + 1, 0), n2e((size_t)ne * nq);
    for (int64_t i = 0; i < ne * nq; ++i) n2e_b[P.conn_soa[i] + 1]++;
    for (int64_t i = 0; i < P.nn; ++i) n2e_b[i + 1] += n2e_b[i];
    {
        std::vector<int32_t> fill(n2e_b.begin(), n2e_b.end() - 1);
        for (int64_t q = 0; q < nq; ++q)
            for (int64_t e = 0; e < ne; ++e) n2e[fill[P.conn_soa[q * ne + e]]++] = (int32_t)e;
    }
    auto node_of = [&](int64_t e, int64_t q) { return P.conn_soa[q * ne + e]; };
    // accum[v]: the node takes an accumulator slot. With split_single only the nodes on an
    // element's edge do (those of two or more elements and those on the domain boundary);
    // the element-interior nodes of a quadrilateral are finished by their element alone.
    std::vector<uint8_t> accum(P.nn, split_single && P.nvpe != 3 ? 0 : 1);
    if (split_single && P.nvpe != 3)
        for (int64_t q = 0; q < nq; ++q) {
            const int64_t a = q % P.n, b = q / P.n;
            if (a == 0 || a == P.p || b == 0 || b == P.p)
                for (int64_t e2 = 0; e2 < ne; ++e2) accum[node_of(e2, q)] = 1;
        }
    // counted[v] = number of nodes below v that occupy an accumulator slot
    std::vector<int64_t> counted(P.nn + 1, 0);
    for (int64_t v = 0; v < P.nn; ++v) counted[v + 1] = counted[v] + accum[v];
    P.tile_elems = tile_elems > 0 ? tile_elems : 0;
    P.tile_items = tile_elems > 0 ? 0 : tile_items;
    P.tile_eb.assign(1, 0);
    P.tile_nb.assign(1, 0);
    P.halo_b.assign(1, 0);
    P.halo.clear();
    // With first-touch numbering the nodes first touched by element e are exactly its ids
    // >= node_hi (1 + largest id touched so far), so a tile's owned range is contiguous.
    // Halo elements of a tile touch one of its owned nodes and lie later in the order.
    std::vector<int32_t> mark(ne, -1), cand, fresh_halo;
    int64_t e = 0;
    int32_t node_hi = 0;
    int32_t t = 0;
    while (e < ne) {
        const int64_t e0 = e;
        const int32_t nb = node_hi;
        int64_t halo_count = 0;
        cand.clear();
        while (e < ne) {
            int32_t new_hi = node_hi;
            for (int64_t q = 0; q < nq; ++q) new_hi = std::max(new_hi, node_of(e, q) + 1);
            fresh_halo.clear();
            for (int64_t q = 0; q < nq; ++q) {
                const int32_t v = node_of(e, q);
                if (v < node_hi) continue;
                for (int32_t k = n2e_b[v]; k < n2e_b[v + 1]; ++k) {
                    const int32_t f = n2e[k];
                    if (f != e && mark[f] != t) { mark[f] = t; fresh_halo.push_back(f); }
                }
            }
            const bool was_halo = mark[e] == t && std::find(fresh_halo.begin(), fresh_halo.end(), (int32_t)e) == fresh_halo.end();
            const int64_t own_after = e - e0 + 1;
            const int64_t halo_after = halo_count - (was_halo ? 1 : 0) + (int64_t)fresh_halo.size();
            bool stop;
            if (tile_elems > 0) stop = own_after > tile_elems;
            else stop = e > e0 && (own_after + halo_after > tile_items || counted[new_hi] - counted[nb] > max_owned);
            if (stop) {
                for (int32_t f : fresh_halo) mark[f] = -1;     // undo the tentative marks
                break;
            }
            for (int32_t f : fresh_halo) cand.push_back(f);
            if (was_halo) mark[e] = -1;                        // it is an own element now
            halo_count = halo_after;
            node_hi = new_hi;
            ++e;
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t f : cand)
            if (f >= e && mark[f] == t) P.halo.push_back(f);
        P.tile_eb.push_back((int32_t)e);
        P.tile_nb.push_back(node_hi);
        P.halo_b.push_back((int32_t)P.halo.size());
        ++t;
    }
    P.max_owned = 0;
    for (size_t k = 0; k + 1 < P.tile_nb.size(); ++k)
        P.max_owned = std::max<int32_t>(P.max_owned, P.tile_nb[k + 1] - P.tile_nb[k]);
    P.tile_ns.clear();
    P.max_shared = P.max_owned;
    if (!split_single) return;
    // stable partition of every owned range: edge nodes, then element-interior nodes
    const int64_t nt = (int64_t)P.tile_nb.size() - 1;
    std::vector<int32_t> perm(P.nn);
    P.tile_ns.resize(nt);
    P.max_shared = 0;
    for (int64_t k = 0; k < nt; ++k) {
        const int32_t b = P.tile_nb[k], f = P.tile_nb[k + 1];
        int32_t next = b;
        for (int32_t v = b; v < f; ++v)
            if (accum[v]) perm[v] = next++;
        P.tile_ns[k] = next - b;
        P.max_shared = std::max<int32_t>(P.max_shared, next - b);
        for (int32_t v = b; v < f; ++v)
            if (!accum[v]) perm[v] = next++;
    }
    for (auto& v : P.conn_soa) v = perm[v];
    std::vector<int32_t> n2o(P.nn);
    std::vector<double> minv(P.nn);
    for (int64_t v = 0; v < P.nn; ++v) {
        n2o[perm[v]] = P.node_new2old[v];
        minv[perm[v]] = P.minv[v];
    }
    P.node_new2old.swap(n2o);
    P.minv.swap(minv);
    for (int64_t v = 0; v < P.nn; ++v) P.node_old2new[P.node_new2old[v]] = (int32_t)v;
}

void element_geometry(const Plan& P, const MeshIn& m, int64_t e, double* g11, double* g12,
                      double* g22, double* det) {
    const Corners c = corners(m, e);
    const int n = P.n;
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            double xs, xt, ys, yt;
            jac(c, P.xi[a], P.xi[b], xs, xt, ys, yt);
            const double d = xs * yt - xt * ys;
            const double ww = P.w[a] * P.w[b];
            const int q = a + n * b;
            det[q] = d;
            g11[q] = ww * (xt * xt + yt * yt) / d;
            g12[q] = -ww * (xs * xt + ys * yt) / d;
            g22[q] = ww * (xs * xs + ys * ys) / d;
        }
}

std::string build_plan(const MeshIn& m, const PlanOptions& opt, Plan& P, int& code) {
    code = SEM_ERR_INVALID_ARG;
    if (opt.p < 1 || opt.p > 7) return "p must be in 1..7";
    if (m.nvpe != 3 && m.nvpe != 4) return "elements must have 3 or 4 vertices";
    if (m.ne < 1 || m.nv < m.nvpe || !m.vxy || !m.quad || !m.c2) return "empty or null mesh";
    if (m.nvpe == 3 && opt.p % 2 == 0)
        return "triangles use odd p (the nodal quadrature weights are not all positive at even p)";
    if (opt.elem_order < 0 || opt.elem_order > 5) return "unknown element order";
    if (opt.node_order < 0 || opt.node_order > 1) return "unknown node order";
    if (opt.tile_elems < 0 || (opt.tile_elems == 0 && opt.tile_items < 1)) return "bad tile size";
    for (int64_t e = 0; e < m.ne; ++e)
        if (!(m.c2[e] > 0.0) || !std::isfinite(m.c2[e])) return "c2 must be positive and finite";
    for (int64_t i = 0; i < 2 * m.nv; ++i)
        if (!std::isfinite(m.vxy[i])) return "vertex coordinates must be finite";
    P = Plan();
    P.p = opt.p;
    P.n = opt.p + 1;
    P.nvpe = m.nvpe;
    P.nq = m.nvpe == 3 ? tri_nq(opt.p) : P.n * P.n;
    P.ne = m.ne;
    P.nv = m.nv;
    gll_basis(P.p, P.xi, P.w, P.D);

    code = SEM_ERR_BAD_MESH;
    std::string err = m.nvpe == 3 ? tri_number_nodes(m, P.p, P.conn0, P.nn) : number_nodes(m, P.p, P.conn0, P.nn);
    if (!err.empty()) return err;
    const int n = P.n, nq = P.nq;
    const int64_t ne = P.ne, nn = P.nn;

    // geometry: Jacobians at every GLL point, mass, node coordinates, CFL dt
    std::vector<double> G0((size_t)3 * nq * ne), mass(nn, 0.0);
    P.node_xy.assign(2 * nn, 0.0);
    std::vector<uint8_t> placed(nn, 0);
    double dt_cfl = INFINITY;
    if (m.nvpe == 3) {
        // affine triangles: one Jacobian per element; nodes at the mapped reference nodes;
        // dt_cfl from the smallest distance between two local nodes (a provisional dt, see
        // dt_from_stability)
        G0.assign((size_t)3 * ne, 0.0);
        err = tri_reference(P.p, P.xi, P.tri_xy, P.tri_w, P.tri_S);
        if (!err.empty()) return err;
        err = tri_symmetry(P.p, P.tri_S);
        if (!err.empty()) return err;
        std::vector<double> px(nq), py(nq);
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t* t = m.quad + 3 * e;
            const double x0 = m.vxy[2 * t[0]], y0 = m.vxy[2 * t[0] + 1];
            const double a = m.vxy[2 * t[1]] - x0, c = m.vxy[2 * t[1] + 1] - y0;   // column X1 - X0
            const double b = m.vxy[2 * t[2]] - x0, d = m.vxy[2 * t[2] + 1] - y0;   // column X2 - X0
            const double det = a * d - b * c;
            if (!(det > 0.0)) return "non-positive Jacobian (clockwise or degenerate triangle) in element " +
                                     std::to_string(e);
            // det J^-1 J^-T = (1 / det) [[b^2 + d^2, -(a b + c d)], [., a^2 + c^2]]
            G0[0 * (size_t)ne + e] = (b * b + d * d) / det;
            G0[1 * (size_t)ne + e] = -(a * b + c * d) / det;
            G0[2 * (size_t)ne + e] = (a * a + c * c) / det;
            for (int q = 0; q < nq; ++q) {
                px[q] = x0 + P.tri_xy[2 * q] * a + P.tri_xy[2 * q + 1] * b;
                py[q] = y0 + P.tri_xy[2 * q] * c + P.tri_xy[2 * q + 1] * d;
                const int32_t v = P.conn0[e * nq + q];
                mass[v] += det * P.tri_w[q];
                if (!placed[v]) {
                    placed[v] = 1;
                    P.node_xy[2 * v] = px[q];
                    P.node_xy[2 * v + 1] = py[q];
                }
            }
            double dmin = INFINITY;
            for (int q = 0; q < nq; ++q)
                for (int r = q + 1; r < nq; ++r) {
                    const double dx = px[r] - px[q], dy = py[r] - py[q];
                    dmin = std::min(dmin, std::sqrt(dx * dx + dy * dy));
                }
            dt_cfl = std::min(dt_cfl, dmin / std::sqrt(m.c2[e]));
        }
        P.dt_from_stability = !(opt.dt > 0.0);
    } else {
        std::vector<double> g11(nq), g12(nq), g22(nq), det(nq), px(nq), py(nq);
        for (int64_t e = 0; e < ne; ++e) {
            element_geometry(P, m, e, g11.data(), g12.data(), g22.data(), det.data());
            for (int q = 0; q < nq; ++q) {
                if (!(det[q] > 0.0))
                    return "non-positive Jacobian in element " + std::to_string(e);
                G0[(0 * (size_t)nq + q) * ne + e] = g11[q];
                G0[(1 * (size_t)nq + q) * ne + e] = g12[q];
                G0[(2 * (size_t)nq + q) * ne + e] = g22[q];
                mass[P.conn0[e * nq + q]] += P.w[q % n] * P.w[q / n] * det[q];
            }
            const Corners c = corners(m, e);
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) map_point(c, P.xi[a], P.xi[b], px[a + n * b], py[a + n * b]);
            for (int q = 0; q < nq; ++q) {
                const int32_t v = P.conn0[e * nq + q];
                if (!placed[v]) {
                    placed[v] = 1;
                    P.node_xy[2 * v] = px[q];
                    P.node_xy[2 * v + 1] = py[q];
                }
            }
            double dmin = INFINITY;
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    const int q = a + n * b;
                    if (a + 1 < n) {
                        const double dx = px[q + 1] - px[q], dy = py[q + 1] - py[q];
                        dmin = std::min(dmin, std::sqrt(dx * dx + dy * dy));
                    }
                    if (b + 1 < n) {
                        const double dx = px[q + n] - px[q], dy = py[q + n] - py[q];
                        dmin = std::min(dmin, std::sqrt(dx * dx + dy * dy));
                    }
                }
            dt_cfl = std::min(dt_cfl, dmin / std::sqrt(m.c2[e]));
        }
    }
    for (int64_t v = 0; v < m.nv; ++v) {       // vertex nodes sit exactly on the vertices
        P.node_xy[2 * v] = m.vxy[2 * v];
        P.node_xy[2 * v + 1] = m.vxy[2 * v + 1];
    }
    const double cfl = opt.cfl > 0.0 ? opt.cfl : 0.3;
    P.dt = opt.dt > 0.0 ? opt.dt : cfl * dt_cfl;
    code = SEM_ERR_INVALID_ARG;
    if (!(P.dt > 0.0) || !std::isfinite(P.dt)) return "dt must be positive";

    // ---------------------------------------------------------------- element order
    const auto t_reorder = std::chrono::steady_clock::now();
    std::vector<uint64_t> key(ne);
    if (opt.elem_order == SEM_ORDER_HILBERT || opt.elem_order == SEM_ORDER_MORTON) {
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int64_t v = 0; v < m.nv; ++v) {
            xmin = std::min(xmin, m.vxy[2 * v]);
            xmax = std::max(xmax, m.vxy[2 * v]);
            ymin = std::min(ymin, m.vxy[2 * v + 1]);
            ymax = std::max(ymax, m.vxy[2 * v + 1]);
        }
        const double wm = xmax - xmin, hm = ymax - ymin;
        const double r = wm / hm;
        const double s = std::sqrt((double)ne);
        const int64_t W = std::max<int64_t>(1, (int64_t)std::ceil(s));
        const int64_t H = std::max<int64_t>(1, (int64_t)std::ceil(s / r));
        const double sx = (double)W / wm, sy = (double)H / hm;
        for (int64_t e = 0; e < ne; ++e) {
            double cxm, cym;
            if (m.nvpe == 3) {
                const int32_t* t = m.quad + 3 * e;
                cxm = ((m.vxy[2 * t[0]] + m.vxy[2 * t[1]]) + m.vxy[2 * t[2]]) / 3.0;
                cym = ((m.vxy[2 * t[0] + 1] + m.vxy[2 * t[1] + 1]) + m.vxy[2 * t[2] + 1]) / 3.0;
            } else {
                const Corners c = corners(m, e);
                cxm = ((c.x[0] + c.x[1]) + (c.x[2] + c.x[3])) * 0.25;
                cym = ((c.y[0] + c.y[1]) + (c.y[2] + c.y[3])) * 0.25;
            }
            int64_t cx = (int64_t)std::floor((cxm - xmin) * sx);
            int64_t cy = (int64_t)std::floor((cym - ymin) * sy);
            cx = std::min<int64_t>(std::max<int64_t>(cx, 0), W - 1);
            cy = std::min<int64_t>(std::max<int64_t>(cy, 0), H - 1);
            key[e] = opt.elem_order == SEM_ORDER_HILBERT
                         ? (uint64_t)hilbert_index(W, H, cx, cy)
                         : (spread_bits((uint64_t)cx) | (spread_bits((uint64_t)cy) << 1));
        }
    } else if (opt.elem_order == SEM_ORDER_RANDOM) {
        for (int64_t e = 0; e < ne; ++e) key[e] = splitmix64(opt.seed ^ (uint64_t)e);
    } else if (opt.elem_order == SEM_ORDER_CONNECTIVITY || opt.elem_order == SEM_ORDER_DISTANCE) {
        const std::vector<int32_t> walk = vertex_walk(m, opt.elem_order == SEM_ORDER_DISTANCE);
        for (int64_t k = 0; k < ne; ++k) key[walk[k]] = (uint64_t)k;
    } else {
        for (int64_t e = 0; e < ne; ++e) key[e] = (uint64_t)e;
    }
    P.elem_new2old.resize(ne);
    std::iota(P.elem_new2old.begin(), P.elem_new2old.end(), 0);
    std::stable_sort(P.elem_new2old.begin(), P.elem_new2old.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    P.elem_old2new.resize(ne);
    for (int64_t k = 0; k < ne; ++k) P.elem_old2new[P.elem_new2old[k]] = (int32_t)k;

    // ---------------------------------------------------------------- node order
    P.node_new2old.resize(nn);
    if (opt.node_order == SEM_NODES_ORIGINAL) {
        std::iota(P.node_new2old.begin(), P.node_new2old.end(), 0);
    } else {
        // degree = distinct other nodes sharing an element (stamp per node)
        std::vector<int32_t> n2e_b(nn + 1, 0), n2e(ne * nq);
        for (int64_t i = 0; i < ne * nq; ++i) n2e_b[P.conn0[i] + 1]++;
        for (int64_t i = 0; i < nn; ++i) n2e_b[i + 1] += n2e_b[i];
        {
            std::vector<int32_t> fill(n2e_b.begin(), n2e_b.end() - 1);
            for (int64_t e = 0; e < ne; ++e)
                for (int q = 0; q < nq; ++q) n2e[fill[P.conn0[e * nq + q]]++] = (int32_t)e;
        }
        std::vector<int32_t> degree(nn, 0), stamp(nn, -1);
        for (int64_t v = 0; v < nn; ++v) {
            int32_t cnt = 0;
            for (int32_t k = n2e_b[v]; k < n2e_b[v + 1]; ++k) {
                const int32_t* c = P.conn0.data() + (int64_t)n2e[k] * nq;
                for (int q = 0; q < nq; ++q)
                    if (stamp[c[q]] != (int32_t)v) { stamp[c[q]] = (int32_t)v; ++cnt; }
            }
            degree[v] = cnt - 1;
        }
        std::vector<uint8_t> seen(nn, 0);
        int64_t next = 0;
        std::vector<std::pair<int32_t, int32_t>> fresh;   // (degree, local index)
        for (int64_t k = 0; k < ne; ++k) {
            const int32_t* c = P.conn0.data() + (int64_t)P.elem_new2old[k] * nq;
            fresh.clear();
            for (int q = 0; q < nq; ++q)
                if (!seen[c[q]]) { seen[c[q]] = 1; fresh.emplace_back(degree[c[q]], q); }
            std::stable_sort(fresh.begin(), fresh.end(),
                             [](const std::pair<int32_t, int32_t>& a,
                                const std::pair<int32_t, int32_t>& b) { return a.first < b.first; });
            for (auto& f : fresh) P.node_new2old[next++] = c[f.second];
        }
    }
    P.node_old2new.resize(nn);
    for (int64_t i = 0; i < nn; ++i) P.node_old2new[P.node_new2old[i]] = (int32_t)i;
    P.reorder_seconds = seconds_since(t_reorder);

    // ---------------------------------------------------------------- new-order arrays
    P.conn_soa.resize((size_t)nq * ne);
    P.c2.resize(ne);
    if (m.nvpe == 3) {
        P.tri_G.resize((size_t)3 * ne);
        for (int64_t k = 0; k < ne; ++k) {
            const int64_t e = P.elem_new2old[k];
            P.c2[k] = m.c2[e];
            for (int c = 0; c < 3; ++c) P.tri_G[(size_t)c * ne + k] = G0[(size_t)c * ne + e];
            for (int q = 0; q < nq; ++q) P.conn_soa[(size_t)q * ne + k] = P.node_old2new[P.conn0[e * nq + q]];
        }
    }
    if (m.nvpe == 4) {
    P.G_soa.resize((size_t)3 * nq * ne);
    P.bilin.resize((size_t)6 * ne);
    for (int64_t k = 0; k < ne; ++k) {
        const int64_t e = P.elem_new2old[k];
        P.c2[k] = m.c2[e];
        const Corners cc = corners(m, e);
        P.bilin[0 * ne + k] = ((cc.x[1] - cc.x[0]) + (cc.x[2] - cc.x[3])) * 0.25;
        P.bilin[1 * ne + k] = ((cc.x[3] - cc.x[0]) + (cc.x[2] - cc.x[1])) * 0.25;
        P.bilin[2 * ne + k] = ((cc.x[0] - cc.x[1]) + (cc.x[2] - cc.x[3])) * 0.25;
        P.bilin[3 * ne + k] = ((cc.y[1] - cc.y[0]) + (cc.y[2] - cc.y[3])) * 0.25;
        P.bilin[4 * ne + k] = ((cc.y[3] - cc.y[0]) + (cc.y[2] - cc.y[1])) * 0.25;
        P.bilin[5 * ne + k] = ((cc.y[0] - cc.y[1]) + (cc.y[2] - cc.y[3])) * 0.25;
        for (int q = 0; q < nq; ++q) {
            P.conn_soa[(size_t)q * ne + k] = P.node_old2new[P.conn0[e * nq + q]];
            for (int c = 0; c < 3; ++c)
                P.G_soa[((size_t)c * nq + q) * ne + k] = G0[((size_t)c * nq + q) * ne + e];
        }
    }
    }
    P.minv.resize(nn);
    for (int64_t i = 0; i < nn; ++i) P.minv[i] = 1.0 / mass[P.node_new2old[i]];
    if (!colour_elements(P)) {
        code = SEM_ERR_BAD_MESH;
        return "greedy element colouring needs more than 64 colours";
    }
    if (opt.node_order == SEM_NODES_FIRST_TOUCH) {
        build_tiles(P, opt.tile_elems, opt.tile_items, opt.max_owned, opt.split_single);
        if (opt.border && opt.split_single) split_border(P);
    }
    code = SEM_OK;
    return "";
}

void split_border(Plan& P) {
    const int64_t ne = P.ne, nq = P.nq, nt = (int64_t)P.tile_eb.size() - 1;
    std::vector<int32_t> tile_of_elem(ne);
    for (int64_t t = 0; t < nt; ++t)
        for (int32_t e = P.tile_eb[t]; e < P.tile_eb[t + 1]; ++e) tile_of_elem[e] = (int32_t)t;
    // tiles touching each node: the first one seen and whether another one touches it too
    std::vector<int32_t> first_tile(P.nn, -1);
    std::vector<uint8_t> border(P.nn, 0);
    for (int64_t q = 0; q < nq; ++q)
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t v = P.conn_soa[q * ne + e], t = tile_of_elem[e];
            if (first_tile[v] < 0) first_tile[v] = t;
            else if (first_tile[v] != t) border[v] = 1;
        }
    std::vector<int32_t> perm(P.nn);
    P.tile_nbd.assign(nt, 0);
    P.border_nodes.clear();
    P.max_shared = 0;
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t b = P.tile_nb[t], ns = P.tile_ns[t], f = P.tile_nb[t + 1];
        int32_t next = b;
        for (int32_t v = b; v < b + ns; ++v)
            if (!border[v]) perm[v] = next++;
        const int32_t n_internal = next - b;
        for (int32_t v = b; v < b + ns; ++v)
            if (border[v]) { perm[v] = next; P.border_nodes.push_back(next); ++next; }
        P.tile_nbd[t] = next - b - n_internal;
        P.tile_ns[t] = n_internal;
        P.max_shared = std::max(P.max_shared, n_internal);
        for (int32_t v = b + ns; v < f; ++v) perm[v] = v;      // element-interior nodes stay
    }
    for (auto& v : P.conn_soa) v = perm[v];
    std::vector<int32_t> n2o(P.nn);
    std::vector<double> minv(P.nn);
    for (int64_t v = 0; v < P.nn; ++v) {
        n2o[perm[v]] = P.node_new2old[v];
        minv[perm[v]] = P.minv[v];
    }
    P.node_new2old.swap(n2o);
    P.minv.swap(minv);
    for (int64_t v = 0; v < P.nn; ++v) P.node_old2new[P.node_new2old[v]] = (int32_t)v;
    P.halo.clear();
    P.halo_b.assign(nt + 1, 0);
}

bool colour_elements(Plan& P) {
    // used[v]: colours of the already-coloured elements around global node v; the colours
    // an element must avoid are the union over its nodes
    const int64_t ne = P.ne, nq = P.nq;
    std::vector<uint64_t> used(P.nn, 0);
    P.colour.assign(ne, 0);
    int32_t nc = 0;
    for (int64_t k = 0; k < ne; ++k) {
        uint64_t taken = 0;
        for (int64_t q = 0; q < nq; ++q) taken |= used[P.conn_soa[q * ne + k]];
        if (taken == ~0ull) return false;
        const int c = __builtin_ctzll(~taken);
        P.colour[k] = c;
        nc = std::max(nc, c + 1);
        for (int64_t q = 0; q < nq; ++q) used[P.conn_soa[q * ne + k]] |= 1ull << c;
    }
    P.n_colours = nc;
    return true;
}

}  // namespace sem
