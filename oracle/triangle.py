"""The paper's own element type (Sec. 4.2): affine triangles whose local nodes are the
Lobatto grid of Blyth and Pozrikidis and double as quadrature points, with the nodal basis
dual to those nodes (FP64). Test infrastructure only (see the package header).

Sec. 4.2 maps a reference triangle to each element by x = x^(e) + J^(e) x-hat, so the
Jacobian and its inverse K^(e) are constant per element. The local basis and the local
nodes form a dual system (N_p(x_q) = delta_pq, Eq. dual_sys); integrals over an element
are det J^(e) times a weighted sum over its local nodes (Eq. numerical_integ); the lumped
mass at a global node sums det J omega_q over the element nodes meeting there (Eq. A-bar);
derivatives are K^(e) applied to reference derivatives (Eq. deriv_u).

Readings:
  * reference triangle (0, 0), (1, 0), (0, 1); elements list their three vertices
    counter-clockwise; J has the columns X1 - X0 and X2 - X0;
  * local node (i, j), i, j >= 0, i + j <= p, k = p - i - j, sits at
        x = (1 + 2 v_i - v_j - v_k) / 3,   y = (1 + 2 v_j - v_i - v_k) / 3,
    where v are the Gauss-Lobatto-Legendre nodes moved to [0, 1] (the Blyth-Pozrikidis
    grid; every edge carries exactly the 1D GLL nodes, so neighbours conform); local index
    q runs over j (outer) and i (inner);
  * the basis is the Lagrange basis of the polynomials of degree <= p dual to the nodes,
    which is unique. The paper writes it through Appell polynomials; here it is the
    inverse of the monomial Vandermonde matrix, computed exactly in rational arithmetic
    from the FP64 node coordinates and rounded once, so the representation leaves no
    trace in the result;
  * omega_q is the integral of N_q over the reference triangle (the interpolatory rule on
    the nodes, exact for degree <= p). These weights are all positive for p = 1, 3, 5, 7
    and are not for even p (p = 2 gives zero weight at the vertices, p = 4 and 6 negative
    ones), so only odd p are used: a lumped mass needs positive weights;
  * second-order form as for the quadrilaterals: element matrix
        K_e[a, b] = c_e^2 det J sum_q omega_q (J^-T grad N_a)(x_q) . (J^-T grad N_b)(x_q)
    and the unweighted lumped mass; natural (free) boundaries;
  * time step: 0.6 times the leapfrog limit 2 / sqrt(lambda_max(M^-1 K)) (``dt_default``),
    since a CFL number on the node spacing does not bound this element's spectrum.

Original global numbering: vertex nodes first (node id = vertex id), then the p - 1 interior
nodes of every edge in order of first appearance over (element, local edge 0..2), each
edge's nodes counted from its lower-id vertex, then the (p - 1)(p - 2) / 2 interior nodes
of each element in element order and local order. Local edge 0 runs from vertex 0 to
vertex 1 (nodes (t, 0)), edge 1 from vertex 1 to vertex 2 (nodes (p - t, t)), edge 2 from
vertex 2 to vertex 0 (nodes (0, p - t)), t the step from the start vertex.
"""
from __future__ import annotations

import functools
from fractions import Fraction
from math import factorial

import numpy as np

from . import gll as _gll
from . import solver as _solver


def local_nodes(p: int):
    """[(i, j)] in local order (j outer, i inner)."""
    return [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]


def local_index(i: int, j: int, p: int) -> int:
    return sum(p + 1 - jj for jj in range(j)) + i


def reference_nodes(p: int) -> np.ndarray:
    """Blyth-Pozrikidis nodes on the reference triangle, [nq, 2]."""
    xi, _ = _gll.gll(p)
    v = 0.5 * (xi + 1.0)
    pts = []
    for i, j in local_nodes(p):
        k = p - i - j
        pts.append(((1.0 + 2.0 * v[i] - v[j] - v[k]) / 3.0, (1.0 + 2.0 * v[j] - v[i] - v[k]) / 3.0))
    return np.array(pts)


def _monomials(p: int):
    return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]


def _inverse_exact(A):
    """Inverse of a square matrix of Fractions by Gauss-Jordan elimination (exact)."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        piv = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


@functools.lru_cache(maxsize=None)
def _exact_coefficients(p: int):
    """C as Fractions: N_m = sum_k C[k][m] x^a_k y^b_k (inverse of the monomial Vandermonde
    at the FP64 node coordinates, taken as exact rationals)."""
    pts = [(Fraction(float(x)), Fraction(float(y))) for x, y in reference_nodes(p)]
    V = [[x ** a * y ** b for (a, b) in _monomials(p)] for x, y in pts]
    return _inverse_exact(V)


@functools.lru_cache(maxsize=None)
def _exact_operators(p: int):
    """(Dx, Dy, omega) as Fractions: Dx[q][m] = dN_m/dx (x_q), omega[m] = integral of N_m."""
    pts = [(Fraction(float(x)), Fraction(float(y))) for x, y in reference_nodes(p)]
    mons = _monomials(p)
    C = _exact_coefficients(p)
    n = len(pts)

    def dmono(x, y, a, b, axis):
        if axis == 0:
            return a * x ** (a - 1) * y ** b if a > 0 else Fraction(0)
        return b * x ** a * y ** (b - 1) if b > 0 else Fraction(0)

    D = []
    for axis in (0, 1):
        Vd = [[dmono(x, y, a, b, axis) for (a, b) in mons] for x, y in pts]
        D.append([[sum(Vd[q][k] * C[k][m] for k in range(n)) for m in range(n)] for q in range(n)])
    integ = [Fraction(factorial(a) * factorial(b), factorial(a + b + 2)) for (a, b) in mons]
    omega = [sum(integ[k] * C[k][m] for k in range(n)) for m in range(n)]
    return D[0], D[1], omega


def reference_operators(p: int):
    """(Dx [nq, nq], Dy [nq, nq], omega [nq]) in FP64: D[q, m] is the derivative of N_m at
    local node q along the reference axis, omega the quadrature weights."""
    Dx, Dy, om = _exact_operators(p)
    f = np.vectorize(float)
    return f(np.array(Dx, dtype=object)), f(np.array(Dy, dtype=object)), f(np.array(om, dtype=object))


def basis_values(p: int, pts) -> np.ndarray:
    """N_m(x) at points ``pts`` [k, 2] -> [k, nq], in FP64 from the exact coefficients rounded
    once (the monomial sums lose about cond(Vandermonde) ulps: ~1e-12 at p = 7)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    C = np.vectorize(float)(np.array(_exact_coefficients(p), dtype=object))
    V = np.stack([pts[:, 0] ** a * pts[:, 1] ** b for (a, b) in _monomials(p)], axis=1)
    return V @ C


def check_p(p: int):
    if p < 1 or p > 7 or p % 2 == 0:
        raise ValueError("triangles use odd p in 1..7 (positive quadrature weights)")


def global_numbering(tris: np.ndarray, n_vertices: int, p: int):
    """Return (conn [E, nq] int64, n_nodes) in the original numbering (module header)."""
    tris = np.asarray(tris, dtype=np.int64)
    E = tris.shape[0]
    nq = (p + 1) * (p + 2) // 2
    if np.unique(tris).size != n_vertices or tris.min() < 0 or tris.max() >= n_vertices:
        raise ValueError("every vertex must be used by at least one element")
    conn = np.full((E, nq), -1, np.int64)
    for c, (i, j) in enumerate(((0, 0), (p, 0), (0, p))):
        conn[:, local_index(i, j, p)] = tris[:, c]
    edge_ids = {}
    next_id = n_vertices
    edge_steps = (lambda t: (t, 0), lambda t: (p - t, t), lambda t: (0, p - t))
    for e in range(E):
        for k in range(3):
            a, b = int(tris[e, k]), int(tris[e, (k + 1) % 3])
            key = (min(a, b), max(a, b))
            if key not in edge_ids:
                edge_ids[key] = next_id
                next_id += p - 1
            base = edge_ids[key]
            for t in range(1, p):
                m = t - 1 if a < b else p - 1 - t          # counted from the lower-id vertex
                conn[e, local_index(*edge_steps[k](t), p)] = base + m
    inner = [local_index(i, j, p) for i, j in local_nodes(p) if i > 0 and j > 0 and p - i - j > 0]
    for e in range(E):
        for q in inner:
            conn[e, q] = next_id
            next_id += 1
    return conn, next_id


def jacobians(vxy, tris):
    """(J [E, 2, 2], detJ [E]) of the affine maps."""
    X = np.asarray(vxy, dtype=np.float64)[np.asarray(tris, dtype=np.int64)]     # [E, 3, 2]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]], axis=2)              # columns
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    return J, det


def check_geometry(vxy, tris):
    _, det = jacobians(vxy, tris)
    if not np.all(det > 0):
        raise ValueError("non-positive Jacobian (clockwise or degenerate triangle)")


def element_stiffness(vxy, tris, p: int, c2=None, elements=None):
    """K_e [E, nq, nq] from the definition (module header); c2 None -> c^2-free."""
    Dx, Dy, om = reference_operators(p)
    J, det = jacobians(vxy, tris if elements is None else np.asarray(tris)[elements])
    Kinv = np.linalg.inv(J)                                  # K^(e), [E, 2, 2]
    # physical gradients at the nodes: grad N_m(x_q) = K^T (dN/dx-hat, dN/dy-hat)
    gx = Kinv[:, 0, 0][:, None, None] * Dx + Kinv[:, 1, 0][:, None, None] * Dy   # [E, q, m]
    gy = Kinv[:, 0, 1][:, None, None] * Dx + Kinv[:, 1, 1][:, None, None] * Dy
    w = det[:, None] * om[None, :]                           # [E, q]
    Ke = np.einsum("eq,eqa,eqb->eab", w, gx, gx) + np.einsum("eq,eqa,eqb->eab", w, gy, gy)
    if c2 is not None:
        c2 = np.asarray(c2, dtype=np.float64)
        Ke = Ke * (c2 if elements is None else c2[elements])[:, None, None]
    return Ke


def lumped_mass(vxy, tris, conn, p: int):
    _, _, om = reference_operators(p)
    _, det = jacobians(vxy, tris)
    M = np.zeros(int(conn.max()) + 1)
    np.add.at(M, conn.ravel(), (det[:, None] * om[None, :]).ravel())
    return M


def node_coordinates(vxy, tris, conn, p: int):
    ref = reference_nodes(p)
    X = np.asarray(vxy, dtype=np.float64)[np.asarray(tris, dtype=np.int64)]
    xy = X[:, None, 0, :] + ref[None, :, 0:1] * (X[:, None, 1, :] - X[:, None, 0, :]) + \
        ref[None, :, 1:2] * (X[:, None, 2, :] - X[:, None, 0, :])
    out = np.zeros((int(conn.max()) + 1, 2))
    out[conn.ravel()] = xy.reshape(-1, 2)
    return out


def cfl_dt(vxy, tris, c2, p: int, cfl: float = 0.3) -> float:
    """cfl * min_e(dx_min,e / c_e), dx_min,e the smallest distance between two local nodes of
    element e (the reading of the quadrilaterals' rule for an unstructured node set)."""
    ref = reference_nodes(p)
    X = np.asarray(vxy, dtype=np.float64)[np.asarray(tris, dtype=np.int64)]
    pts = X[:, None, 0, :] + ref[None, :, 0:1] * (X[:, None, 1, :] - X[:, None, 0, :]) + \
        ref[None, :, 1:2] * (X[:, None, 2, :] - X[:, None, 0, :])          # [E, nq, 2]
    d = np.sqrt(((pts[:, :, None, :] - pts[:, None, :, :]) ** 2).sum(-1))
    nq = ref.shape[0]
    d[:, np.arange(nq), np.arange(nq)] = np.inf
    return float(cfl * np.min(d.min(axis=(1, 2)) / np.sqrt(np.asarray(c2, dtype=np.float64))))


class TriSEM(_solver.SEM):
    """Assembled FP64 operator of a triangle mesh (original numbering); the leapfrog run,
    energy and power iteration of ``solver.SEM`` apply unchanged."""

    def __init__(self, vxy, tris, c2, p: int, chunk: int = 8192):
        check_p(p)
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.quads = np.asarray(tris, dtype=np.int64)          # element vertex lists
        self.p = p
        self.c2 = np.asarray(c2, dtype=np.float64).copy()
        check_geometry(self.vxy, self.quads)
        self.conn, self.n_nodes = global_numbering(self.quads, self.vxy.shape[0], p)
        self.mass = lumped_mass(self.vxy, self.quads, self.conn, p)
        self.minv = 1.0 / self.mass
        self.node_xy = node_coordinates(self.vxy, self.quads, self.conn, p)
        self._chunk = chunk
        self.K = self._assemble(self.c2)

    def _assemble(self, c2):
        import scipy.sparse as sp
        E, nq = self.conn.shape
        rows, cols, vals = [], [], []
        for lo in range(0, E, self._chunk):
            el = np.arange(lo, min(E, lo + self._chunk))
            Ke = element_stiffness(self.vxy, self.quads, self.p, c2, elements=el)
            c = self.conn[el]
            rows.append(np.repeat(c, nq, axis=1).ravel())
            cols.append(np.tile(c, (1, nq)).ravel())
            vals.append(Ke.ravel())
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n_nodes, self.n_nodes))
        return K.tocsr()

    def element_K_hat(self, elements):
        return element_stiffness(self.vxy, self.quads, self.p, None, elements=elements)

    def dt_cfl(self, cfl: float = 0.3) -> float:
        return cfl_dt(self.vxy, self.quads, self.c2, self.p, cfl)

    def dt_default(self, frac: float = 0.6) -> float:
        """frac times the leapfrog stability limit 2 / sqrt(lambda_max(M^-1 K)). The node-
        spacing rule of the quadrilaterals does not bound the spectrum of this element: at
        p = 7 the largest stable CFL number on the smallest node distance is about 0.12."""
        return frac * 2.0 / np.sqrt(self.lambda_max())


def sampled_rows(vxy, tris, c2, p, conn, nodes, u):
    """(K u)[nodes] and the lumped mass M[nodes], one node at a time from the element
    matrices of the triangles around each node (Eqs. R and A-bar restricted to the rows of
    the sampled nodes); ``u`` is [n_nodes]. For meshes too large to assemble."""
    _, _, om = reference_operators(p)
    start, elem, slot = _solver.node_incidence(conn, int(conn.max()) + 1)
    nodes = np.asarray(nodes, dtype=np.int64)
    ks = [np.arange(start[v], start[v + 1]) for v in nodes]
    els = np.unique(np.concatenate([elem[k] for k in ks]))
    Ke = element_stiffness(vxy, tris, p, c2, elements=els)
    _, det = jacobians(vxy, np.asarray(tris)[els])
    pos = {int(e): i for i, e in enumerate(els)}
    u = np.asarray(u, dtype=np.float64)
    r = np.zeros(nodes.size)
    M = np.zeros(nodes.size)
    for i, k in enumerate(ks):
        for e, q in zip(elem[k], slot[k]):
            j = pos[int(e)]
            r[i] += Ke[j, q] @ u[conn[e]]
            M[i] += om[q] * det[j]
    return r, M
