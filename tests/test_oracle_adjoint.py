"""Pins of the oracle's discrete adjoint: its gradient w.r.t. element c^2 must equal
central finite differences of the oracle's own forward misfit (the definition of the
gradient), and the adjoint map must be linear in the trace gradient."""
import numpy as np
import pytest

import workloads
from oracle import adjoint, solver


def _tiny(nsteps=80, p=3, n=6, shots=2):
    vxy, quads, xc, yc = workloads.grid_mesh(n, n, 600.0, 600.0, jitter=0.2, seed=9)
    c = workloads.layered_c(yc, 600.0, c_top=1500.0, c_step=300.0)
    rng = np.random.default_rng(21)
    c2_true = (c * (1 + 0.1 * rng.uniform(-1, 1, c.size))) ** 2
    c2 = c * c
    sem = solver.SEM(vxy, quads, c2_true, p)
    dt = sem.dt_cfl()
    src = solver.snap_to_nodes([[150.0, 450.0], [420.0, 300.0]][:shots], sem.node_xy)
    rec = solver.snap_to_nodes(np.stack([np.linspace(50, 550, 7), np.full(7, 600.0)], 1), sem.node_xy)
    f0 = 40.0
    obs, _, _ = sem.run(nsteps, dt, src, np.arange(shots), f0, rec_nodes=rec, n_shots=shots)
    sem.set_c2(c2)
    return sem, dt, src, rec, f0, obs, shots, nsteps


def _J(sem, c2, dt, src, rec, f0, obs, shots, nsteps):
    sem.set_c2(c2)
    tr, _, _ = sem.run(nsteps, dt, src, np.arange(shots), f0, rec_nodes=rec, n_shots=shots)
    return adjoint.misfit(tr, obs)


def test_gradient_matches_central_differences():
    sem, dt, src, rec, f0, obs, shots, nsteps = _tiny()
    c2 = sem.c2.copy()
    J, g = adjoint.misfit_and_gradient(sem, nsteps, dt, src, np.arange(shots), f0, rec, shots, obs)
    assert J > 0
    rng = np.random.default_rng(4)
    els = rng.choice(c2.size, 10, replace=False)
    fd = []
    for e in els:
        h = 1e-4 * c2[e]
        cp = c2.copy(); cp[e] += h
        cm = c2.copy(); cm[e] -= h
        fd.append((_J(sem, cp, dt, src, rec, f0, obs, shots, nsteps) -
                   _J(sem, cm, dt, src, rec, f0, obs, shots, nsteps)) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(g[els] - fd) / np.linalg.norm(fd) < 1e-6


def test_directional_derivative():
    sem, dt, src, rec, f0, obs, shots, nsteps = _tiny(nsteps=60)
    c2 = sem.c2.copy()
    J, g = adjoint.misfit_and_gradient(sem, nsteps, dt, src, np.arange(shots), f0, rec, shots, obs)
    d = np.random.default_rng(8).uniform(-1, 1, c2.size) * c2
    eps = 1e-5
    fd = (_J(sem, c2 + eps * d, dt, src, rec, f0, obs, shots, nsteps) -
          _J(sem, c2 - eps * d, dt, src, rec, f0, obs, shots, nsteps)) / (2 * eps)
    assert g @ d == pytest.approx(fd, rel=1e-7)


def test_gradient_linear_in_trace_gradient():
    sem, dt, src, rec, f0, obs, shots, nsteps = _tiny(nsteps=40)
    rng = np.random.default_rng(2)
    a = rng.standard_normal(obs.shape)
    b = rng.standard_normal(obs.shape)
    args = (sem, nsteps, dt, src, np.arange(shots), f0, rec, shots)
    ga = adjoint.gradient_c2(*args, a)
    gb = adjoint.gradient_c2(*args, b)
    gab = adjoint.gradient_c2(*args, 2.0 * a - 3.0 * b)
    np.testing.assert_allclose(gab, 2.0 * ga - 3.0 * gb, atol=1e-12 * np.abs(gab).max())
