"""Explicit leapfrog stepping of the assembled SEM system (FP64).

The paper advances dU/dt = M^-1 (R + D U + y(t)) (Sec. 4.2, Eq. u_change) with sources
added at the global node a source point maps to (Alg. 3). Here the acoustic equation is
taken in its second-order form u_tt = div(c^2 grad u) + s with an unweighted lumped mass
and natural (homogeneous Neumann, "free") boundaries, and advanced with leapfrog in
increment form (replacing the paper's Heun scheme):

    a^n       = M^-1 (f^n - K u^n)
    v^{n+1/2} = v^{n-1/2} + dt a^n
    u^{n+1}   = u^n + dt v^{n+1/2}

starting from u^0 = v^{-1/2} = 0 and t_n = n dt. The point source is a Ricker wavelet
of peak frequency f0 delayed by t0 = 1/f0 (the paper names the wavelet without its
parameters). Receivers record u^{n+1} after step n. The time step follows a CFL number
of 0.3 on the smallest distance between neighbouring GLL nodes of an element:
dt = cfl * min_e(dx_min,e / c_e).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import gll as _gll
from . import mesh as _mesh


def ricker(t, f0: float, t0: float):
    a = (np.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def cfl_dt(vxy, quads, c2, p: int, cfl: float = 0.3) -> float:
    xi, eta = _mesh.reference_points(p)
    pts = _mesh.bilinear(vxy, quads, xi, eta)            # [E, n^2, 2]
    n = p + 1
    P = pts.reshape(-1, n, n, 2)                         # [E, b, a, 2]
    dx_a = np.sqrt(np.sum((P[:, :, 1:] - P[:, :, :-1]) ** 2, axis=-1))
    dx_b = np.sqrt(np.sum((P[:, 1:, :] - P[:, :-1, :]) ** 2, axis=-1))
    dmin = np.minimum(dx_a.reshape(len(P), -1).min(axis=1), dx_b.reshape(len(P), -1).min(axis=1))
    return float(cfl * np.min(dmin / np.sqrt(np.asarray(c2, dtype=np.float64))))


def snap_to_nodes(points, node_xy):
    """Nearest global node of each point; equal distances go to the lowest node id."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    out = np.empty(points.shape[0], np.int64)
    for i, (x, y) in enumerate(points):
        d = (node_xy[:, 0] - x) ** 2 + (node_xy[:, 1] - y) ** 2
        out[i] = int(np.argmin(d))                       # first minimum = lowest id
    return out


class SEM:
    """Assembled FP64 SEM operator on a conforming quad mesh (original numbering).

    Holds K = sum_e P_e^T K_e P_e (scipy CSR, summed from the dense element matrices of
    ``mesh.element_stiffness``) and the lumped mass. Suitable for meshes up to a few
    hundred thousand nodes.
    """

    def __init__(self, vxy, quads, c2, p: int, chunk: int = 8192):
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.quads = np.asarray(quads, dtype=np.int64)
        self.p = p
        self.c2 = np.asarray(c2, dtype=np.float64).copy()
        _mesh.check_geometry(self.vxy, self.quads, p)
        self.conn, self.n_nodes = _mesh.global_numbering(self.quads, self.vxy.shape[0], p)
        self.mass = _mesh.lumped_mass(self.vxy, self.quads, self.conn, p)
        self.minv = 1.0 / self.mass
        self.node_xy = _mesh.node_coordinates(self.vxy, self.quads, self.conn, p)
        self._chunk = chunk
        self.K = self._assemble(self.c2)

    def _assemble(self, c2):
        E, nq = self.conn.shape
        rows, cols, vals = [], [], []
        for lo in range(0, E, self._chunk):
            el = np.arange(lo, min(E, lo + self._chunk))
            Ke = _mesh.element_stiffness(self.vxy, self.quads, self.p, c2, elements=el)
            c = self.conn[el]
            rows.append(np.repeat(c, nq, axis=1).ravel())
            cols.append(np.tile(c, (1, nq)).ravel())
            vals.append(Ke.ravel())
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n_nodes, self.n_nodes))
        return K.tocsr()

    def set_c2(self, c2):
        self.c2 = np.asarray(c2, dtype=np.float64).copy()
        self.K = self._assemble(self.c2)

    def apply_K(self, u):
        return self.K @ u

    def element_K_hat(self, elements):
        """c^2-free element matrices of the given elements."""
        return _mesh.element_stiffness(self.vxy, self.quads, self.p, None, elements=elements)

    def dt_cfl(self, cfl: float = 0.3) -> float:
        return cfl_dt(self.vxy, self.quads, self.c2, self.p, cfl)

    def lambda_max(self, iters: int | None = None, seed: int = 11, tol: float = 1e-14,
                   max_iters: int = 100000) -> float:
        """Largest eigenvalue of M^-1 K by power iteration (M^-1 K is similar to the
        symmetric M^-1/2 K M^-1/2, so its spectrum is real and non-negative).

        With ``iters`` the iteration runs that many times. Otherwise it runs until the
        estimate has changed by at most ``tol`` (relative) for 20 iterations in a row:
        the error falls like (lambda_2 / lambda_1)^k, and that ratio is close to 1 on
        graded meshes."""
        rng = np.random.default_rng(seed)
        x = rng.standard_normal(self.n_nodes)
        lam = 0.0
        calm = 0
        for k in range(iters if iters is not None else max_iters):
            y = self.minv * (self.K @ x)
            new = float(np.linalg.norm(y) / np.linalg.norm(x))
            calm = calm + 1 if abs(new - lam) <= tol * new else 0
            lam = new
            x = y / np.linalg.norm(y)
            if iters is None and calm >= 20:
                break
        return lam

    def energy(self, u_next, u, v_half):
        """E^{n+1/2} = 1/2 v^{n+1/2}' M v^{n+1/2} + 1/2 u^{n+1}' K u^n."""
        return 0.5 * float(v_half @ (self.mass * v_half)) + 0.5 * float(u_next @ (self.K @ u))

    def run(self, nsteps: int, dt: float, src_nodes=(), src_shot=(), f0: float = 10.0,
            t0: float | None = None, rec_nodes=(), n_shots: int = 1, u0=None, v0=None,
            src_amp=None, record_every=None, callback=None):
        """Leapfrog for ``nsteps`` steps; all shots advance together.

        ``src_amp`` (optional [n_src, nsteps]) replaces the Ricker amplitudes of the
        sources step by step. Returns (traces [S, R, nsteps], u [N, S], v [N, S]).
        """
        t0 = 1.0 / f0 if t0 is None else t0
        N, S = self.n_nodes, n_shots
        u = np.zeros((N, S)) if u0 is None else np.array(u0, dtype=np.float64).reshape(N, S)
        v = np.zeros((N, S)) if v0 is None else np.array(v0, dtype=np.float64).reshape(N, S)
        src_nodes = np.asarray(src_nodes, dtype=np.int64)
        src_shot = np.asarray(src_shot, dtype=np.int64)
        rec_nodes = np.asarray(rec_nodes, dtype=np.int64)
        traces = np.zeros((S, rec_nodes.size, nsteps))
        minv = self.minv[:, None]
        for n in range(nsteps):
            f = np.zeros((N, S))
            if src_nodes.size:
                amp = ricker(n * dt, f0, t0) * np.ones(src_nodes.size) if src_amp is None \
                    else src_amp[:, n]
                np.add.at(f, (src_nodes, src_shot), amp)
            a = minv * (f - self.K @ u)
            v = v + dt * a
            u_new = u + dt * v
            if callback is not None:
                callback(n, u, u_new, v)
            u = u_new
            if rec_nodes.size:
                traces[:, :, n] = u[rec_nodes, :].T
        return traces, u, v


def standing_mode(node_xy, L: float, m: int, n: int):
    """phi = cos(m pi x / L) cos(n pi y / L), a Neumann eigenmode of the square."""
    return np.cos(m * np.pi * node_xy[:, 0] / L) * np.cos(n * np.pi * node_xy[:, 1] / L)


def node_incidence(conn, n_nodes):
    """CSR of the elements around every node: (start [N+1], elements [E*nq], local slot)."""
    E, nq = conn.shape
    flat = conn.ravel()
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=n_nodes)
    start = np.concatenate([[0], np.cumsum(counts)])
    return start, order // nq, order % nq


def sampled_rows(vxy, quads, c2, p, conn, nodes, u):
    """(K u)[nodes] and the lumped mass M[nodes], one node at a time, from the element
    matrices of the elements around each node (Eqs. R and A-bar restricted to the rows of
    the sampled nodes). ``u`` is [n_nodes] or [n_nodes, S]; returns (r [k(,S)], M [k])."""
    start, elem, slot = node_incidence(conn, int(conn.max()) + 1)
    nodes = np.asarray(nodes, dtype=np.int64)
    ks = [np.arange(start[v], start[v + 1]) for v in nodes]
    els = np.unique(np.concatenate([elem[k] for k in ks]))
    Ke = _mesh.element_stiffness(vxy, quads, p, c2, elements=els)
    det = _mesh.jacobians(vxy, quads[els], p)[4]
    wq = _mesh.quadrature_weights(p)
    pos = {int(e): i for i, e in enumerate(els)}
    u = np.asarray(u, dtype=np.float64)
    r = np.zeros((nodes.size,) + u.shape[1:])
    M = np.zeros(nodes.size)
    for i, k in enumerate(ks):
        for e, q in zip(elem[k], slot[k]):
            j = pos[int(e)]
            r[i] += Ke[j, q] @ u[conn[e]]
            M[i] += wq[q] * det[j, q]
    return r, M
