"""The paper's own formulation: the first-order u-v system with the Heun scheme (FP64).

Test infrastructure only (see the package header).

Sec. 4.1 restates the acoustic wave equation as a first-order system with a continuous
scalar u and a discontinuous vector v (Eqs. def_v_1, def_u_1), cast in the general form
M u_t = -(B v)_{,k} + D u + sources, v_t = E v + F grad u (Eqs. def_u_2, def_v_2) with
M = 1/K, B = -I, F = I/rho and D = E = 0. Sec. 4.2 discretises it: v lives on the local
nodes of every element (V^(e)_kp, Eq. v_change), u on the global nodes with the lumped
mass M-bar and the assembled term R (Eqs. u_change, u_change_r_effic); Sec. 4.2.1 advances
both with Heun's predictor-corrector.

Readings (the paper works on triangles with an Appell basis; here quads with GLL nodes,
as for the rest of this oracle):
  * rho = 1 and K = c^2 per element, so M-bar_nu = sum over (e, q -> nu) of
    w_q detJ_q / c_e^2, and F = I;
  * grad N at a node is J^{-T} (dN/dxi, dN/deta) at that node (the paper's K^(e) J^-1);
  * R_nu = sum over (e, p -> nu) of -sum_q w_q detJ_q V^(e)_q . grad N_p(x_q);
  * the point source y(t) enters Eq. u_change at its node; the corrector evaluates the
    rates at t_{n+1} = (n+1) h, the predictor at t_n;
  * Ricker, t0 and node snapping as in ``solver``; receivers record U after each step.
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from .solver import ricker


class FirstOrderSEM:
    """Element gradient operators, weights and the weighted lumped mass of one mesh."""

    def __init__(self, vxy, quads, c2, p: int):
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.quads = np.asarray(quads, dtype=np.int64)
        self.c2 = np.asarray(c2, dtype=np.float64)
        self.p = p
        _mesh.check_geometry(self.vxy, self.quads, p)
        self.conn, self.n_nodes = _mesh.global_numbering(self.quads, self.vxy.shape[0], p)
        x_xi, x_eta, y_xi, y_eta, det = _mesh.jacobians(self.vxy, self.quads, p)
        dxi, deta = _mesh.reference_gradients(p)
        # gx[e, k, q]: d N_q / dx at local node k of element e (J^{-T} applied)
        self.gx = (y_eta[:, :, None] * dxi[None] - y_xi[:, :, None] * deta[None]) / det[:, :, None]
        self.gy = (-x_eta[:, :, None] * dxi[None] + x_xi[:, :, None] * deta[None]) / det[:, :, None]
        self.wdet = _mesh.quadrature_weights(p)[None, :] * det            # [E, nq]
        self.mass = np.bincount(self.conn.ravel(), weights=(self.wdet / self.c2[:, None]).ravel(),
                                minlength=self.n_nodes)
        self.node_xy = _mesh.node_coordinates(self.vxy, self.quads, self.conn, p)

    def v_rate(self, U):
        """Eq. v_change with E = 0, F = I: V-dot at every local node, [E, 2, nq, S]."""
        Ue = U[self.conn]                                                  # [E, nq, S]
        return np.stack([np.einsum("ekq,eqs->eks", self.gx, Ue),
                         np.einsum("ekq,eqs->eks", self.gy, Ue)], axis=1)

    def assemble_R(self, V):
        """Eq. u_change_r_effic with B = -I: R_nu, [N, S]."""
        Re = -(np.einsum("eq,eqp,eqs->eps", self.wdet, self.gx, V[:, 0])
               + np.einsum("eq,eqp,eqs->eps", self.wdet, self.gy, V[:, 1]))
        R = np.zeros((self.n_nodes, V.shape[-1]))
        np.add.at(R, self.conn.ravel(), Re.reshape(-1, V.shape[-1]))
        return R

    def u_rate(self, V, f):
        """Eq. u_change with D = 0: U-dot = M-bar^{-1} (R + y)."""
        return (self.assemble_R(V) + f) / self.mass[:, None]

    def run(self, nsteps: int, h: float, src_nodes=(), src_shot=(), f0: float = 10.0,
            t0: float | None = None, rec_nodes=(), n_shots: int = 1, u0=None, v0=None):
        """Heun steps from (u0, v0) (default 0, Eq. initial_cond). Returns (traces
        [S, R, nsteps], U [N, S], V [E, 2, nq, S])."""
        t0 = 1.0 / f0 if t0 is None else t0
        N, S = self.n_nodes, n_shots
        E, nq = self.conn.shape
        U = np.zeros((N, S)) if u0 is None else np.array(u0, dtype=np.float64).reshape(N, S)
        V = np.zeros((E, 2, nq, S)) if v0 is None else np.array(v0, dtype=np.float64).reshape(E, 2, nq, S)
        src_nodes = np.asarray(src_nodes, dtype=np.int64)
        src_shot = np.asarray(src_shot, dtype=np.int64)
        rec_nodes = np.asarray(rec_nodes, dtype=np.int64)
        traces = np.zeros((S, rec_nodes.size, nsteps))

        def force(t):
            f = np.zeros((N, S))
            if src_nodes.size:
                np.add.at(f, (src_nodes, src_shot), ricker(t, f0, t0))
            return f

        for n in range(nsteps):
            dU0 = self.u_rate(V, force(n * h))
            dV0 = self.v_rate(U)
            Up = U + h * dU0                                               # predictor
            Vp = V + h * dV0
            dU1 = self.u_rate(Vp, force((n + 1) * h))
            dV1 = self.v_rate(Up)
            U = U + 0.5 * h * (dU0 + dU1)                                  # corrector
            V = V + 0.5 * h * (dV0 + dV1)
            if rec_nodes.size:
                traces[:, :, n] = U[rec_nodes, :].T
        return traces, U, V
