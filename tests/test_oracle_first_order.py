"""Pins of the first-order u-v system with Heun (Sec. 4.1, 4.2, 4.2.1) in the oracle."""
import numpy as np
import pytest
from scipy.linalg import expm

import workloads
from oracle import first_order, mesh, solver


def _mesh(n=3, p=2, jitter=0.2):
    vxy, quads, xc, yc = workloads.grid_mesh(n, n, 300.0, 300.0, jitter=jitter, seed=7)
    c = workloads.layered_c(yc, 300.0, c_top=1500.0, c_step=400.0)
    return vxy, quads, c * c, p


def test_weighted_mass_sums_to_area_over_c2():
    """M-bar = sum w detJ / c^2 sums to sum_e area_e / c_e^2 (shoelace areas)."""
    vxy, quads, c2, p = _mesh(4, 3)
    fo = first_order.FirstOrderSEM(vxy, quads, c2, p)
    X = vxy[quads]
    area = 0.5 * np.abs(np.sum(X[:, :, 0] * np.roll(X[:, :, 1], -1, axis=1)
                               - np.roll(X[:, :, 0], -1, axis=1) * X[:, :, 1], axis=1))
    assert fo.mass.sum() == pytest.approx(np.sum(area / c2), rel=1e-13)


def test_R_of_grad_is_minus_stiffness():
    """With V = grad U (Eq. v_change, F = I), Eq. u_change_r_effic gives R = -K-hat U, the
    c^2-free stiffness of the second-order oracle."""
    vxy, quads, c2, p = _mesh(3, 3)
    fo = first_order.FirstOrderSEM(vxy, quads, c2, p)
    sem = solver.SEM(vxy, quads, np.ones_like(c2), p)
    U = np.random.default_rng(1).standard_normal((fo.n_nodes, 2))
    R = fo.assemble_R(fo.v_rate(U))
    np.testing.assert_allclose(R, -(sem.K @ U), atol=1e-12 * np.abs(sem.K @ U).max())


def _dense_operator(fo):
    """A of the linear system d/dt [U; V] = A [U; V] (no source), column by column."""
    N, (E, nq) = fo.n_nodes, fo.conn.shape
    nv = E * 2 * nq
    A = np.zeros((N + nv, N + nv))
    for k in range(N + nv):
        x = np.zeros(N + nv)
        x[k] = 1.0
        U, V = x[:N, None], x[N:].reshape(E, 2, nq, 1)
        A[:N, k] = fo.u_rate(V, np.zeros((N, 1)))[:, 0]
        A[N:, k] = fo.v_rate(U).ravel()
    return A


def test_heun_step_is_second_order_taylor_polynomial():
    """For a linear system Heun's predictor-corrector is y + h A y + h^2/2 A^2 y."""
    vxy, quads, c2, p = _mesh(2, 2)
    fo = first_order.FirstOrderSEM(vxy, quads, c2, p)
    A = _dense_operator(fo)
    N, (E, nq) = fo.n_nodes, fo.conn.shape
    x = np.random.default_rng(2).standard_normal(A.shape[0])
    h = 2e-3
    _, U, V = fo.run(1, h, u0=x[:N], v0=x[N:])
    expect = x + h * (A @ x) + 0.5 * h * h * (A @ (A @ x))
    got = np.concatenate([U[:, 0], V.ravel()])
    np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_heun_is_second_order_in_time():
    """Against the exact flow exp(T A) of the semi-discrete system, halving h divides the
    error at a fixed time by about 4."""
    vxy, quads, c2, p = _mesh(2, 3)
    fo = first_order.FirstOrderSEM(vxy, quads, c2, p)
    A = _dense_operator(fo)
    N = fo.n_nodes
    x = np.zeros(A.shape[0])
    x[:N] = np.exp(-((fo.node_xy[:, 0] - 150) ** 2 + (fo.node_xy[:, 1] - 150) ** 2) / 5000.0)
    T = 0.02
    errs = []
    for steps in (40, 80, 160):
        _, U, V = fo.run(steps, T / steps, u0=x[:N], v0=x[N:])
        exact = expm(T * A) @ x
        errs.append(np.linalg.norm(np.concatenate([U[:, 0], V.ravel()]) - exact) / np.linalg.norm(exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_single_step_point_source():
    """From rest with one source at node s: V-tilde = 0, so U^1 = h/2 (y(0) + y(h)) / M-bar_s
    at s and 0 elsewhere, and V^1 = h/2 grad(U-tilde)."""
    vxy, quads, c2, p = _mesh(3, 2)
    fo = first_order.FirstOrderSEM(vxy, quads, c2, p)
    s = int(solver.snap_to_nodes([[150.0, 150.0]], fo.node_xy)[0])
    h, f0 = 1e-4, 25.0
    tr, U, V = fo.run(1, h, [s], [0], f0, rec_nodes=[s])
    y0, y1 = solver.ricker(0.0, f0, 1 / f0), solver.ricker(h, f0, 1 / f0)
    assert U[s, 0] == pytest.approx(0.5 * h * (y0 + y1) / fo.mass[s], rel=1e-14)
    assert np.count_nonzero(U[:, 0]) == 1
    Ut = np.zeros((fo.n_nodes, 1))
    Ut[s, 0] = h * y0 / fo.mass[s]
    np.testing.assert_allclose(V, 0.5 * h * fo.v_rate(Ut), rtol=1e-14, atol=1e-30)
    assert tr[0, 0, 0] == U[s, 0]
