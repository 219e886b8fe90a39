"""Discrete adjoint of the leapfrog recurrence and the gradient w.r.t. element c^2 (FP64).

Not in the paper; derived from the discrete forward of ``solver`` (discretize, then
differentiate). Eliminating v, the forward is

    u^{n+1} = (2I - A) u^n - u^{n-1} + dt^2 M^-1 f^n,   A = dt^2 M^-1 K(m),
    K(m) = sum_e m_e Khat_e,  m_e = c_e^2,  u^0 = u^{-1} = 0,

with receiver samples d^n = R u^{n+1} (n = 0..N-1) and a loss L(d). Writing
g^k = R^T dL/dd^{k-1} (k = 1..N), the multipliers mu^k = M^-1 lambda^k obey

    mu^k = M^-1 g^k + (2I - A) mu^{k+1} - mu^{k+2},   mu^{N+1} = mu^{N+2} = 0,

which is the forward recurrence run backwards in time with sources M^-1 g^k at the
receiver nodes, and

    dL/dm_e = -dt^2 sum_{n=0}^{N-1} (mu^{n+1})^T Khat_e u^n.

With w^j the state after j steps of the forward stepper driven by the sources
f^j = g^{N-j} / dt^2, mu^{N-j} = w^{j+1}, so the sum pairs u^n with w^{N-n}.
"""
from __future__ import annotations

import numpy as np

from .solver import SEM, ricker


def misfit(traces, observed):
    r = np.asarray(traces, dtype=np.float64) - np.asarray(observed, dtype=np.float64)
    return 0.5 * float(np.sum(r * r))


def forward_history(sem: SEM, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots):
    """Forward run keeping every state u^0..u^N -> (traces, hist [N+1, nodes, S])."""
    hist = np.zeros((nsteps + 1, sem.n_nodes, n_shots))

    def keep(n, u, u_new, v):
        hist[n + 1] = u_new

    traces, _, _ = sem.run(nsteps, dt, src_nodes, src_shot, f0, rec_nodes=rec_nodes,
                           n_shots=n_shots, callback=keep)
    return traces, hist


def adjoint_states(sem: SEM, nsteps, dt, rec_nodes, dL_dd, n_shots):
    """w^0..w^N of the adjoint recurrence for trace gradients dL_dd [S, R, N]."""
    R = len(rec_nodes)
    src_nodes = np.tile(np.asarray(rec_nodes, dtype=np.int64), n_shots)
    src_shot = np.repeat(np.arange(n_shots), R)
    # amplitude of receiver r of shot s at adjoint step j: dL/dd[s, r, N-1-j] / dt^2
    amp = (np.asarray(dL_dd, dtype=np.float64)[:, :, ::-1] / (dt * dt)).reshape(n_shots * R, nsteps)
    hist = np.zeros((nsteps + 1, sem.n_nodes, n_shots))

    def keep(n, u, u_new, v):
        hist[n + 1] = u_new

    sem.run(nsteps, dt, src_nodes, src_shot, rec_nodes=(), n_shots=n_shots, src_amp=amp,
            callback=keep)
    return hist


def gradient_c2(sem: SEM, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots, dL_dd,
                u_hist=None):
    """dL/dc^2_e for every element, given dL/d(traces)."""
    if u_hist is None:
        _, u_hist = forward_history(sem, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots)
    w_hist = adjoint_states(sem, nsteps, dt, rec_nodes, dL_dd, n_shots)
    E = sem.conn.shape[0]
    g = np.zeros(E)
    chunk = 4096
    for lo in range(0, E, chunk):
        el = np.arange(lo, min(E, lo + chunk))
        Kh = sem.element_K_hat(el)                         # [e, nq, nq]
        c = sem.conn[el]
        for n in range(1, nsteps):                         # u^0 = 0 contributes nothing
            ue = u_hist[n][c]                              # [e, nq, S]
            we = w_hist[nsteps - n][c]
            g[el] += np.einsum("eps,epq,eqs->e", we, Kh, ue)
    return -dt * dt * g


def misfit_and_gradient(sem: SEM, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots,
                        observed):
    traces, u_hist = forward_history(sem, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots)
    J = misfit(traces, observed)
    g = gradient_c2(sem, nsteps, dt, src_nodes, src_shot, f0, rec_nodes, n_shots,
                    traces - observed, u_hist=u_hist)
    return J, g
