"""Pins of the oracle's time stepping: discrete energy, a closed-form standing mode with
spectral convergence in p, source and receiver conventions, permutation invariance.

The paper advances Eq. u_change explicitly (Sec. 4.2.1) with sources added per Alg. 3;
the leapfrog increment form here is the build's reading of that step.
"""
import numpy as np
import pytest

import workloads
from oracle import reorder, solver


def test_energy_conserved_source_free():
    wl = workloads.workload("layered1024", n=8)
    sem = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = sem.dt_cfl()
    rng = np.random.default_rng(5)
    u0 = np.exp(-((sem.node_xy[:, 0] - 4000) ** 2 + (sem.node_xy[:, 1] - 6000) ** 2) / 1e6)
    u0 = u0 + 1e-3 * rng.standard_normal(sem.n_nodes)
    v0 = 1e-2 * rng.standard_normal(sem.n_nodes)
    energies = []

    def cb(n, u, u_new, v):
        energies.append(sem.energy(u_new[:, 0], u[:, 0], v[:, 0]))

    sem.run(1000, dt, u0=u0, v0=v0, callback=cb)
    e = np.array(energies)
    assert e[0] > 0
    assert np.abs(e / e[0] - 1.0).max() < 1e-12


def _standing_error(p, nel=4, m=3, n=2, cfl=0.3):
    L = 1.0
    vxy, quads, _, _ = workloads.grid_mesh(nel, nel, L, L)
    sem = solver.SEM(vxy, quads, np.ones(quads.shape[0]), p)
    dt = sem.dt_cfl(cfl)
    omega = np.pi * np.sqrt(m * m + n * n) / L
    theta = np.arccos(1.0 - (omega * dt) ** 2 / 2.0)
    nsteps = int(round(2.0 * np.pi / theta))            # about one period
    phi = solver.standing_mode(sem.node_xy, L, m, n)
    v0 = phi * (1.0 - np.cos(theta)) / dt
    _, u, _ = sem.run(nsteps, dt, u0=phi, v0=v0)
    exact = phi * np.cos(nsteps * theta)
    return float(np.abs(u[:, 0] - exact).max())


def test_standing_mode_spectral_convergence():
    """u^0 = phi, v^{-1/2} = phi (1 - cos theta)/dt with cos theta = 1 - (omega dt)^2/2 makes
    leapfrog exact for the continuous mode, so what is left is the spatial error, which
    must fall exponentially in p."""
    errs = {p: _standing_error(p) for p in range(2, 11)}
    ps = sorted(errs)
    for a, b in zip(ps, ps[1:]):
        assert errs[b] < errs[a], errs
    assert errs[10] < 1e-8
    # exponential: log-error roughly linear in p with a clearly negative slope
    slope = np.polyfit(ps, np.log10([errs[p] for p in ps]), 1)[0]
    assert slope < -0.8, (slope, errs)


def test_ricker_closed_form_points():
    f0 = 15.0
    t0 = 1.0 / f0
    assert solver.ricker(t0, f0, t0) == 1.0
    # zero crossings at t0 +- 1/(pi f0 sqrt 2)
    tz = t0 + 1.0 / (np.pi * f0 * np.sqrt(2.0))
    assert abs(solver.ricker(tz, f0, t0)) < 1e-15
    assert abs(solver.ricker(0.0, f0, t0) - (1 - 2 * np.pi ** 2) * np.exp(-np.pi ** 2)) < 1e-14 * 1e-3


def test_single_step_source_response():
    """From rest, one step puts u^1 = dt^2 M^-1 ricker(0) at the source node only."""
    wl = workloads.workload("homog64", n=6)
    sem = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = sem.dt_cfl()
    s = solver.snap_to_nodes(wl.src_xy, sem.node_xy)
    tr, u, v = sem.run(1, dt, s, [0], wl.f0, rec_nodes=s)
    expect = dt * dt * sem.minv[s[0]] * solver.ricker(0.0, wl.f0, 1 / wl.f0)
    assert u[s[0], 0] == pytest.approx(expect, rel=1e-14)
    assert np.count_nonzero(u[:, 0]) == 1
    assert tr[0, 0, 0] == u[s[0], 0]


def test_snap_ties_go_to_lowest_id():
    xy = np.array([[0.0, 0.0], [2.0, 0.0], [1.0, 5.0]])
    assert solver.snap_to_nodes([[1.0, 0.0]], xy)[0] == 0


@pytest.mark.parametrize("kind", ["hilbert", "morton", "random", "connectivity", "distance"])
def test_relabelling_leaves_traces_unchanged(kind):
    """The reordering is a relabelling (Sec. 4.3): running the SEM on the reordered
    element list and mapping back gives the unordered result to rounding."""
    wl = workloads.workload("layered1024", n=10, nsteps=150)
    sem = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = sem.dt_cfl()
    src = solver.snap_to_nodes(wl.src_xy, sem.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, sem.node_xy)
    tr0, u0, _ = sem.run(wl.nsteps, dt, src, [0], wl.f0, rec_nodes=rec)
    perm, _ = reorder.reorder(kind, wl.vxy, wl.quads, sem.conn)
    sem2 = solver.SEM(wl.vxy, wl.quads[perm], wl.c2[perm], wl.p)
    # node correspondence through the local slots of the same physical element
    m = np.empty(sem.n_nodes, np.int64)
    m[sem.conn[perm].ravel()] = sem2.conn.ravel()
    tr1, u1, _ = sem2.run(wl.nsteps, dt, m[src], [0], wl.f0, rec_nodes=m[rec])
    err = np.linalg.norm(u1[m] - u0) / np.linalg.norm(u0)
    assert err < 1e-12
    np.testing.assert_allclose(tr1, tr0, atol=1e-12 * np.abs(tr0).max())
