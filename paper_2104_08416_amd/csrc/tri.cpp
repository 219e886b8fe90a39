// tri.cpp -- host setup of the paper's own element type (Sec. 4.2): affine triangles whose
// local nodes are the Lobatto grid of Blyth and Pozrikidis and double as quadrature points.
//
// Reference triangle (0, 0), (1, 0), (0, 1). Local node (i, j), i + j <= p, k = p - i - j, at
//   x = (1 + 2 v_i - v_j - v_k) / 3,  y = (1 + 2 v_j - v_i - v_k) / 3,
// v the GLL nodes on [0, 1]; local index q runs over j (outer) and i (inner). The nodal basis
// dual to these nodes is formed here through the Proriol-Koornwinder-Dubiner polynomials,
// an orthogonal basis of the polynomials of degree <= p on the triangle (the Vandermonde
// matrix on these nodes is well conditioned): N = psi V^-1 with V[q][m] = psi_m(x_q). The
// weights are the integrals of the N_q; psi_0 is the only basis polynomial with a nonzero
// integral, so omega_q = (V^-1)[0][q] psi_0 / 2.
//
// A step needs, per element, K_e = c^2 (g11 Sxx + g12 Sxy + g22 Syy) with the reference
// matrices Sxx = Dx^T W Dx, Sxy = Dx^T W Dy + Dy^T W Dx, Syy = Dy^T W Dy (D the nodal
// derivative matrices, W the weights) and the element factors G = det J J^-1 J^-T.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "plan.h"

namespace sem {
namespace {

// Jacobi P_n^(a,b)(x), n = 0..N, by the three-term recurrence
void jacobi_all(int N, double a, double b, double x, std::vector<double>& P) {
    P.assign(N + 1, 0.0);
    P[0] = 1.0;
    if (N == 0) return;
    P[1] = 0.5 * ((a + b + 2.0) * x + (a - b));
    for (int n = 2; n <= N; ++n) {
        const double c = 2.0 * n + a + b;
        const double a1 = 2.0 * n * (n + a + b) * (c - 2.0);
        const double a2 = (c - 1.0) * (c * (c - 2.0) * x + a * a - b * b);
        const double a3 = 2.0 * (n + a - 1.0) * (n + b - 1.0) * c;
        P[n] = (a2 * P[n - 1] - a3 * P[n - 2]) / a1;
    }
}

double jacobi(int n, double a, double b, double x) {
    std::vector<double> P;
    jacobi_all(n, a, b, x, P);
    return P[n];
}

// d/dx P_n^(a,b) = (n + a + b + 1) / 2 P_{n-1}^(a+1,b+1)
double jacobi_d(int n, double a, double b, double x) {
    return n == 0 ? 0.0 : 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

// psi_{ij}(r, s) = P_i(a) P_j^(2i+1,0)(b) ((1 - b) / 2)^i on the triangle (-1,-1), (1,-1),
// (-1, 1) with the collapsed coordinates a = 2 (1 + r) / (1 - s) - 1, b = s (a = -1 at the
// top vertex, where the expressions below stay polynomial), and its r- and s-derivatives.
void pkd(int i, int j, double r, double s, double& psi, double& dr, double& ds) {
    const double a = s < 1.0 - 1e-14 ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    const double b = s;
    const double f = jacobi(i, 0.0, 0.0, a), df = jacobi_d(i, 0.0, 0.0, a);
    const double g = jacobi(j, 2.0 * i + 1.0, 0.0, b), dg = jacobi_d(j, 2.0 * i + 1.0, 0.0, b);
    const double h = 0.5 * (1.0 - b);
    const double hi = std::pow(h, i), him1 = i > 0 ? std::pow(h, i - 1) : 0.0;
    psi = f * g * hi;
    dr = i > 0 ? df * g * him1 : 0.0;
    ds = (i > 0 ? df * g * 0.5 * (1.0 + a) * him1 : 0.0) + f * (dg * hi - (i > 0 ? 0.5 * i * g * him1 : 0.0));
}

// inverse of an n x n matrix (row-major) by Gauss-Jordan with partial pivoting
bool invert(std::vector<double> A, int n, std::vector<double>& inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
        if (!(std::fabs(A[(size_t)piv * n + c]) > 0.0)) return false;
        for (int k = 0; k < n; ++k) {
            std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
            std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
        }
        const double d = A[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            A[(size_t)c * n + k] /= d;
            inv[(size_t)c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return true;
}

}  // namespace

int tri_nq(int p) { return (p + 1) * (p + 2) / 2; }

int tri_lidx(int i, int j, int p) { return j * (p + 1) - j * (j - 1) / 2 + i; }

std::string tri_reference(int p, const std::vector<double>& gll_x, std::vector<double>& xy,
                          std::vector<double>& w, std::vector<double>& S) {
    const int nq = tri_nq(p);
    xy.assign(2 * nq, 0.0);
    std::vector<double> v(p + 1);
    for (int t = 0; t <= p; ++t) v[t] = 0.5 * (gll_x[t] + 1.0);
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i + j <= p; ++i) {
            const int k = p - i - j, q = tri_lidx(i, j, p);
            xy[2 * q] = (1.0 + 2.0 * v[i] - v[j] - v[k]) / 3.0;
            xy[2 * q + 1] = (1.0 + 2.0 * v[j] - v[i] - v[k]) / 3.0;
        }
    // Vandermonde and its derivatives in (x, y): d/dx = 2 d/dr, d/dy = 2 d/ds
    std::vector<double> V((size_t)nq * nq), Vx((size_t)nq * nq), Vy((size_t)nq * nq);
    for (int q = 0; q < nq; ++q) {
        const double r = 2.0 * xy[2 * q] - 1.0, s = 2.0 * xy[2 * q + 1] - 1.0;
        int m = 0;
        for (int i = 0; i <= p; ++i)
            for (int j = 0; i + j <= p; ++j, ++m) {
                double psi, dr, ds;
                pkd(i, j, r, s, psi, dr, ds);
                V[(size_t)q * nq + m] = psi;
                Vx[(size_t)q * nq + m] = 2.0 * dr;
                Vy[(size_t)q * nq + m] = 2.0 * ds;
            }
    }
    std::vector<double> Vi;
    if (!invert(V, nq, Vi)) return "singular Vandermonde matrix of the triangle nodes";
    // D[q][m] = dN_m/dx (x_q) = sum_k Vx[q][k] Vi[k][m]
    std::vector<double> Dx((size_t)nq * nq, 0.0), Dy((size_t)nq * nq, 0.0);
    for (int q = 0; q < nq; ++q)
        for (int m = 0; m < nq; ++m) {
            double sx = 0.0, sy = 0.0;
            for (int k = 0; k < nq; ++k) {
                sx += Vx[(size_t)q * nq + k] * Vi[(size_t)k * nq + m];
                sy += Vy[(size_t)q * nq + k] * Vi[(size_t)k * nq + m];
            }
            Dx[(size_t)q * nq + m] = sx;
            Dy[(size_t)q * nq + m] = sy;
        }
    // psi_0 = 1; the reference triangle has area 1/2
    w.assign(nq, 0.0);
    for (int q = 0; q < nq; ++q) w[q] = 0.5 * Vi[q];
    for (int q = 0; q < nq; ++q)
        if (!(w[q] > 0.0)) return "non-positive quadrature weight on the triangle nodes (use odd p)";
    S.assign((size_t)3 * nq * nq, 0.0);
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) {
            double sxx = 0.0, sxy = 0.0, syy = 0.0;
            for (int q = 0; q < nq; ++q) {
                const double xa = Dx[(size_t)q * nq + a], ya = Dy[(size_t)q * nq + a];
                const double xb = Dx[(size_t)q * nq + b], yb = Dy[(size_t)q * nq + b];
                sxx += w[q] * xa * xb;
                sxy += w[q] * (xa * yb + ya * xb);
                syy += w[q] * ya * yb;
            }
            S[(size_t)a * nq + b] = sxx;
            S[(size_t)(nq + a) * nq + b] = sxy;
            S[(size_t)(2 * nq + a) * nq + b] = syy;
        }
    return "";
}

std::string tri_symmetry(int p, const std::vector<double>& S) {
    // On an affine triangle, with n_i the gradients of the barycentric coordinates on the
    // reference triangle (n_1 = (-1, -1), n_2 = (1, 0), n_3 = (0, 1)) and c_ij = -n_i.G n_j,
    //   g11 Sxx + g12 Sxy + g22 Syy = c_12 E_12 + c_23 E_23 + c_13 E_13,
    //   E_12 = Sxx, E_13 = Syy, E_23 = Sxx + Syy - Sxy,  c_12 = g11 + g12, c_23 = -g12,
    //   c_13 = g12 + g22.
    // The node set is invariant under the rotations of the vertices, and E_23, E_13 are Sxx
    // seen from rotated vertices: E[q][m] = Sxx[s(q)][s(m)] with s_23 taking node (i, j, k) to
    // node (j, k, i) and s_13 = s_23^-1 taking it to (k, i, j). The triangle kernel relies on
    // exactly these two maps; checked here entry by entry.
    const int nq = tri_nq(p);
    auto sxx = [&](int a, int b) { return S[(size_t)a * nq + b]; };
    auto sxy = [&](int a, int b) { return S[(size_t)(nq + a) * nq + b]; };
    auto syy = [&](int a, int b) { return S[(size_t)(2 * nq + a) * nq + b]; };
    std::vector<int> s23(nq), s13(nq);
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i + j <= p; ++i) {
            const int k = p - i - j, q = tri_lidx(i, j, p);
            s23[q] = tri_lidx(j, k, p);
            s13[q] = tri_lidx(k, i, p);
        }
    double scale = 0.0, err = 0.0;
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) {
            scale = std::max(scale, std::fabs(sxx(a, b)));
            err = std::max(err, std::fabs(sxx(a, b) + syy(a, b) - sxy(a, b) - sxx(s23[a], s23[b])));
            err = std::max(err, std::fabs(syy(a, b) - sxx(s13[a], s13[b])));
        }
    if (!(err <= 1e-12 * scale)) return "the triangle's reference matrices lack the vertex symmetry of the nodes";
    return "";
}

std::string tri_number_nodes(const MeshIn& m, int p, std::vector<int32_t>& conn, int64_t& nn) {
    const int nq = tri_nq(p);
    const int64_t ne = m.ne, nv = m.nv;
    std::vector<uint8_t> used(nv, 0);
    for (int64_t i = 0; i < ne * 3; ++i) {
        const int32_t v = m.quad[i];
        if (v < 0 || v >= nv) return "vertex id out of range";
        used[v] = 1;
    }
    for (int64_t v = 0; v < nv; ++v)
        if (!used[v]) return "vertex " + std::to_string(v) + " is not used by any element";
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* t = m.quad + 3 * e;
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2])
            return "element " + std::to_string(e) + " repeats a vertex";
    }
    // distinct edges ranked by first use over (element, local edge)
    struct Use { int64_t key, pos; };
    std::vector<Use> uses((size_t)ne * 3);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            const int64_t s = m.quad[3 * e + k], f = m.quad[3 * e + (k + 1) % 3];
            uses[3 * e + k] = {std::min(s, f) * nv + std::max(s, f), 3 * e + k};
        }
    std::vector<Use> sorted = uses;
    std::sort(sorted.begin(), sorted.end(),
              [](const Use& a, const Use& b) { return a.key != b.key ? a.key < b.key : a.pos < b.pos; });
    std::vector<int64_t> first_pos, edge_of_use((size_t)ne * 3);
    for (size_t i = 0; i < sorted.size();) {
        size_t j = i;
        while (j < sorted.size() && sorted[j].key == sorted[i].key) ++j;
        if (j - i > 2) return "an edge is shared by more than two elements";
        if (j - i == 2 && m.quad[sorted[i].pos] == m.quad[sorted[i + 1].pos])
            return "two triangles traverse their shared edge in the same direction (orientation)";
        for (size_t k = i; k < j; ++k) edge_of_use[sorted[k].pos] = (int64_t)first_pos.size();
        first_pos.push_back(sorted[i].pos);
        i = j;
    }
    const int64_t nedge = (int64_t)first_pos.size();
    std::vector<int64_t> by_first(nedge), rank(nedge);
    std::iota(by_first.begin(), by_first.end(), 0);
    std::sort(by_first.begin(), by_first.end(), [&](int64_t a, int64_t b) { return first_pos[a] < first_pos[b]; });
    for (int64_t r = 0; r < nedge; ++r) rank[by_first[r]] = r;
    const int pe = p - 1, ni = (p - 1) * (p - 2) / 2;
    const int64_t base_int = nv + nedge * pe;
    nn = base_int + ne * (int64_t)ni;
    if (nn > INT32_MAX) return "mesh too large for 32-bit node ids";
    conn.assign((size_t)ne * nq, -1);
    for (int64_t e = 0; e < ne; ++e) {
        int32_t* c = conn.data() + e * nq;
        const int32_t* t = m.quad + 3 * e;
        c[tri_lidx(0, 0, p)] = t[0];
        c[tri_lidx(p, 0, p)] = t[1];
        c[tri_lidx(0, p, p)] = t[2];
        for (int k = 0; k < 3; ++k) {
            const int32_t s = t[k], f = t[(k + 1) % 3];
            const int64_t r = rank[edge_of_use[3 * e + k]];
            for (int st = 1; st < p; ++st) {
                // step st from the start vertex of local edge k
                const int i = k == 0 ? st : (k == 1 ? p - st : 0);
                const int j = k == 0 ? 0 : (k == 1 ? st : p - st);
                const int off = s < f ? st - 1 : p - 1 - st;
                c[tri_lidx(i, j, p)] = (int32_t)(nv + r * pe + off);
            }
        }
        int next = 0;
        for (int j = 1; j < p; ++j)
            for (int i = 1; i + j < p; ++i) c[tri_lidx(i, j, p)] = (int32_t)(base_int + e * (int64_t)ni + next++);
    }
    return "";
}

}  // namespace sem
