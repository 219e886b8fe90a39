"""Local-to-global node map, element geometry, stiffness and lumped mass (FP64).

Sec. 4.2 of the paper represents u by its values U_mu at global SEM nodes, with mu(p, e)
mapping local node p of element e to its global node; the gradient of u inside an
element is a sum of reference-basis derivatives mapped by the inverse Jacobian (Eq.
deriv_u); the mass is the quadrature-weighted Jacobian summed over the element nodes
that meet at a global node (Eq. A-bar); and the assembled term R collects, at every
global node, the quadrature of flux times test-function derivative (Eq. R).

Readings for the tensor-product quadrilateral used here (the paper uses affine
triangles with a constant Jacobian):
  * the element map is the bilinear map of the four CCW corners, so the Jacobian is
    evaluated at every GLL point;
  * second-order form: with M = 1 and flux c^2 grad u the assembled R becomes
    -K u with K_e[p, q] = c_e^2 sum_k w_k detJ_k grad N_p(x_k) . grad N_q(x_k);
  * local node index q = a + (p+1) b, a along the first reference axis (corner 0 to
    corner 1), b along the second (corner 0 to corner 3).

Original global numbering (the "unordered" numbering every result is reported in):
vertex nodes first (node id = vertex id), then the p-1 interior nodes of every edge in
order of first appearance over (element, local edge 0..3), each edge's nodes counted
from its lower-id vertex, then the (p-1)^2 interior nodes of each element in element
order with the first reference axis fastest.
"""
from __future__ import annotations

import numpy as np

from . import gll as _gll


def local_index(a, b, p):
    return a + (p + 1) * b


def _edge_local(k: int, t: int, p: int):
    """Local (a, b) of the point at step t (0..p) along local edge k, walked from its
    start corner k to corner (k+1) % 4."""
    if k == 0:
        return t, 0
    if k == 1:
        return p, t
    if k == 2:
        return p - t, p
    return 0, p - t


_CORNER_AB = ((0, 0), (1, 0), (1, 1), (0, 1))   # in units of p


def global_numbering(quads: np.ndarray, n_vertices: int, p: int):
    """Return (conn [E, (p+1)^2] int64, n_nodes) in the original numbering.

    Raises ValueError for a non-conforming input: unused vertices, an edge shared by
    more than two elements, or two elements traversing a shared edge in the same
    direction (inconsistent orientation).
    """
    quads = np.asarray(quads, dtype=np.int64)
    E = quads.shape[0]
    n = p + 1
    if np.unique(quads).size != n_vertices or quads.min() < 0 or quads.max() >= n_vertices:
        raise ValueError("every vertex must be used by at least one element")
    start = quads                                  # [E, 4] start vertex of local edge k
    end = np.roll(quads, -1, axis=1)               # [E, 4] end vertex
    lo = np.minimum(start, end).ravel()
    hi = np.maximum(start, end).ravel()
    key = lo * n_vertices + hi
    uniq, first, inv, counts = np.unique(key, return_index=True, return_inverse=True,
                                         return_counts=True)
    if counts.max() > 2:
        raise ValueError("an edge is shared by more than two elements")
    # edges that appear twice must be walked in opposite directions
    st = start.ravel()
    order = np.argsort(inv, kind="stable")
    pairs = counts[inv[order]] == 2
    occ = order[pairs].reshape(-1, 2)
    if occ.size and np.any(st[occ[:, 0]] == st[occ[:, 1]]):
        raise ValueError("inconsistent element orientation across a shared edge")
    # rank edges by first appearance over (element, local edge)
    rank_of_uniq = np.empty(uniq.size, np.int64)
    rank_of_uniq[np.argsort(first, kind="stable")] = np.arange(uniq.size)
    edge_rank = rank_of_uniq[inv].reshape(E, 4)
    n_edges = uniq.size
    pe = p - 1
    base_int = n_vertices + n_edges * pe
    conn = np.empty((E, n * n), np.int64)
    for k in range(4):
        a, b = _CORNER_AB[k]
        conn[:, local_index(a * p, b * p, p)] = quads[:, k]
    for k in range(4):
        s = start[:, k]
        f = end[:, k]
        for t in range(1, p):
            a, b = _edge_local(k, t, p)
            off = np.where(s < f, t - 1, p - 1 - t)
            conn[:, local_index(a, b, p)] = n_vertices + edge_rank[:, k] * pe + off
    for b in range(1, p):
        for a in range(1, p):
            conn[:, local_index(a, b, p)] = base_int + np.arange(E) * pe * pe + (a - 1) + pe * (b - 1)
    return conn, base_int + E * pe * pe


def bilinear(vxy: np.ndarray, quads: np.ndarray, xi, eta):
    """Physical coordinates of reference points (xi, eta) in every element -> [E, P, 2]."""
    X = vxy[quads]                                 # [E, 4, 2]
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    N = 0.25 * np.stack([(1 - xi) * (1 - eta), (1 + xi) * (1 - eta),
                         (1 + xi) * (1 + eta), (1 - xi) * (1 + eta)], axis=1)  # [P, 4]
    return np.einsum("pk,ekd->epd", N, X)


def reference_points(p: int):
    """Reference coordinates of the (p+1)^2 local nodes in local order q = a + (p+1) b."""
    x, _ = _gll.gll(p)
    n = p + 1
    a = np.tile(np.arange(n), n)
    b = np.repeat(np.arange(n), n)
    return x[a], x[b]


def node_coordinates(vxy, quads, conn, p):
    """Coordinates of every global node: vertex nodes take the vertex coordinates; the
    others are mapped from the first element (original order) that contains them."""
    n_nodes = int(conn.max()) + 1
    xi, eta = reference_points(p)
    E = quads.shape[0]
    first = np.full(n_nodes, E, np.int64)
    np.minimum.at(first, conn.ravel(), np.repeat(np.arange(E), conn.shape[1]))
    xy = np.empty((n_nodes, 2))
    # local slot of each node inside its first element
    slot = np.empty(n_nodes, np.int64)
    ee = np.repeat(np.arange(E), conn.shape[1])
    qq = np.tile(np.arange(conn.shape[1]), E)
    mask = ee == first[conn.ravel()]
    slot[conn.ravel()[mask]] = qq[mask]
    X = vxy[quads[first]]                            # [N, 4, 2]
    s, t = xi[slot], eta[slot]
    N4 = 0.25 * np.stack([(1 - s) * (1 - t), (1 + s) * (1 - t),
                          (1 + s) * (1 + t), (1 - s) * (1 + t)], axis=1)
    xy[:] = np.einsum("nk,nkd->nd", N4, X)
    nv = vxy.shape[0]
    xy[:nv] = vxy
    return xy


def jacobians(vxy, quads, p):
    """Per element and local node: (x_xi, x_eta, y_xi, y_eta, detJ), each [E, (p+1)^2]."""
    X = vxy[quads]                                   # [E, 4, 2]
    xi, eta = reference_points(p)
    xi = xi[None, :]
    eta = eta[None, :]
    x0, x1, x2, x3 = (X[:, k, 0][:, None] for k in range(4))
    y0, y1, y2, y3 = (X[:, k, 1][:, None] for k in range(4))
    x_xi = 0.25 * ((1 - eta) * (x1 - x0) + (1 + eta) * (x2 - x3))
    x_eta = 0.25 * ((1 - xi) * (x3 - x0) + (1 + xi) * (x2 - x1))
    y_xi = 0.25 * ((1 - eta) * (y1 - y0) + (1 + eta) * (y2 - y3))
    y_eta = 0.25 * ((1 - xi) * (y3 - y0) + (1 + xi) * (y2 - y1))
    det = x_xi * y_eta - x_eta * y_xi
    return x_xi, x_eta, y_xi, y_eta, det


def reference_gradients(p: int):
    """dxi[k, q], deta[k, q]: reference derivatives of basis function q at local node k.

    With N_q(xi, eta) = l_a(xi) l_b(eta) for q = (a, b) and node k = (i, j):
    dN_q/dxi (k) = D[i, a] delta(j, b),  dN_q/deta (k) = delta(i, a) D[j, b].
    """
    D = _gll.derivative_matrix(p)
    n = p + 1
    dxi = np.zeros((n * n, n * n))
    deta = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            k = local_index(i, j, p)
            for b in range(n):
                for a in range(n):
                    q = local_index(a, b, p)
                    if j == b:
                        dxi[k, q] = D[i, a]
                    if i == a:
                        deta[k, q] = D[j, b]
    return dxi, deta


def quadrature_weights(p: int):
    """w_k = w_i w_j for local node k = (i, j)."""
    _, w = _gll.gll(p)
    n = p + 1
    return np.outer(w, w).ravel()        # index j*n + i == local_index(i, j)


def check_geometry(vxy, quads, p):
    """Raise ValueError if any Jacobian determinant at a GLL point is not positive."""
    det = jacobians(vxy, quads, p)[4]
    if not np.all(det > 0.0):
        bad = np.unique(np.nonzero(det <= 0.0)[0])
        raise ValueError(f"non-positive Jacobian in {bad.size} element(s), first {bad[0]}")


def element_stiffness(vxy, quads, p, c2=None, elements=None):
    """Dense element matrices K_e [E, n^2, n^2] (c^2-free if ``c2`` is None).

    K_e[p, q] = c_e^2 sum_k w_k detJ_k grad N_p(x_k) . grad N_q(x_k), with
    grad N = J^{-T} (dN/dxi, dN/deta):
      dN/dx = ( y_eta dN/dxi - y_xi dN/deta) / detJ,
      dN/dy = (-x_eta dN/dxi + x_xi dN/deta) / detJ.
    """
    if elements is not None:
        quads = quads[elements]
        if c2 is not None:
            c2 = np.asarray(c2)[elements]
    x_xi, x_eta, y_xi, y_eta, det = jacobians(vxy, quads, p)
    dxi, deta = reference_gradients(p)
    wq = quadrature_weights(p)
    gx = (y_eta[:, :, None] * dxi[None] - y_xi[:, :, None] * deta[None]) / det[:, :, None]
    gy = (-x_eta[:, :, None] * dxi[None] + x_xi[:, :, None] * deta[None]) / det[:, :, None]
    s = wq[None, :] * det                                    # [E, n^2]
    K = np.einsum("ek,ekp,ekq->epq", s, gx, gx) + np.einsum("ek,ekp,ekq->epq", s, gy, gy)
    if c2 is not None:
        K *= np.asarray(c2, dtype=np.float64)[:, None, None]
    return K


def lumped_mass(vxy, quads, conn, p):
    """M_nu = sum over (e, k) with mu(k, e) = nu of w_k detJ_k (no density weight)."""
    det = jacobians(vxy, quads, p)[4]
    wq = quadrature_weights(p)
    n_nodes = int(conn.max()) + 1
    return np.bincount(conn.ravel(), weights=(wq[None, :] * det).ravel(), minlength=n_nodes)
