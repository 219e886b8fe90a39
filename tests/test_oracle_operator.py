"""Pins of the oracle's assembled operator: numbering, mass, stiffness.

Mass = sum of quadrature-weighted Jacobians (Sec. 4.2, Eq. A-bar); stiffness from the
mapped basis gradients (Eqs. deriv_u and R).
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import gll, mesh, reorder, solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_numbering_and_first_touch():
    g = json.load(open(os.path.join(GOLDEN, "first_touch_2x1_p2.json")))
    vxy = np.array(g["vxy"], dtype=np.float64)
    quads = np.array(g["quads"], dtype=np.int64)
    conn, n = mesh.global_numbering(quads, vxy.shape[0], g["p"])
    assert n == 15
    np.testing.assert_array_equal(conn, g["conn"])
    deg = reorder.node_degree(conn, n)
    np.testing.assert_array_equal(deg, g["degree"])
    elem = reorder.element_order("hilbert", vxy, quads)
    np.testing.assert_array_equal(elem, g["elem_new2old_hilbert"])
    np.testing.assert_array_equal(reorder.first_touch_nodes(conn, elem, deg), g["node_new2old"])


@pytest.mark.parametrize("p", [1, 2, 4, 5])
def test_structured_node_count_and_coincidence(p):
    wl = workloads.workload("layered1024", n=6, p=p)
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], p)
    assert n == wl.n_nodes
    # nodes shared between elements are geometrically the same point in each element
    xi, eta = mesh.reference_points(p)
    pts = mesh.bilinear(wl.vxy, wl.quads, xi, eta).reshape(-1, 2)
    xy = mesh.node_coordinates(wl.vxy, wl.quads, conn, p)
    np.testing.assert_allclose(pts, xy[conn.ravel()], atol=1e-9)


def test_numbering_rejects_bad_meshes():
    vxy = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1], [2, 1]], dtype=np.float64)
    with pytest.raises(ValueError):      # second element clockwise: shared edge walked the same way
        mesh.global_numbering(np.array([[0, 1, 4, 3], [1, 4, 5, 2]]), 6, 3)
    with pytest.raises(ValueError):      # vertex 5 unused
        mesh.global_numbering(np.array([[0, 1, 4, 3]]), 6, 3)
    with pytest.raises(ValueError):      # inverted element -> negative Jacobian
        mesh.check_geometry(vxy, np.array([[0, 3, 4, 1]]), 3)


@pytest.mark.parametrize("name,kw", [("homog64", dict(n=8)), ("layered1024", dict(n=12)),
                                     ("graded1414", dict(n=10, p=5))])
def test_mass_sums_to_area(name, kw):
    wl = workloads.workload(name, **kw)
    conn, _ = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    M = mesh.lumped_mass(wl.vxy, wl.quads, conn, wl.p)
    assert np.all(M > 0)
    assert abs(M.sum() - wl.Lx * wl.Ly) < 1e-13 * wl.Lx * wl.Ly


@pytest.fixture(scope="module")
def jittered():
    wl = workloads.workload("layered1024", n=10)
    return wl, solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)


def test_stiffness_symmetric_psd_and_kills_constants(jittered):
    wl, sem = jittered
    K = sem.K
    rng = np.random.default_rng(0)
    x = rng.standard_normal(sem.n_nodes)
    y = rng.standard_normal(sem.n_nodes)
    knorm = abs(K).sum(axis=1).max()
    assert abs(x @ (K @ y) - y @ (K @ x)) < 1e-13 * knorm * np.linalg.norm(x) * np.linalg.norm(y)
    assert np.abs(K @ np.ones(sem.n_nodes)).max() < 1e-13 * knorm
    assert x @ (K @ x) > 0


def test_stiffness_of_linear_field(jittered):
    """grad of a linear field is exact on bilinear elements and the GLL rule integrates
    grad N . const exactly, so (K u)_nu = c^2 * boundary flux: zero at interior nodes
    and c^2 a (edge length / 2) w_j on the non-corner nodes of the right edge."""
    wl, _ = jittered
    c2 = np.full(wl.n_elements, 4.0)
    sem = solver.SEM(wl.vxy, wl.quads, c2, wl.p)
    a, b = 0.7, -1.3
    u = a * sem.node_xy[:, 0] + b * sem.node_xy[:, 1] + 5.0
    r = sem.K @ u
    L = wl.Lx
    xy = sem.node_xy
    on_bnd = (np.abs(xy[:, 0]) < 1e-9) | (np.abs(xy[:, 0] - L) < 1e-9) | \
             (np.abs(xy[:, 1]) < 1e-9) | (np.abs(xy[:, 1] - L) < 1e-9)
    scale = 4.0 * (abs(a) + abs(b)) * L / wl.nx
    assert np.abs(r[~on_bnd]).max() < 1e-11 * scale
    # right edge, excluding corners and element vertices: a GLL node at reference t_j
    _, w = gll.gll(wl.p)
    h = L / wl.ny
    right = (np.abs(xy[:, 0] - L) < 1e-9) & (xy[:, 1] > 1e-9) & (xy[:, 1] < L - 1e-9)
    yy = xy[right, 1]
    frac = (yy / h) - np.floor(yy / h)
    inner = (frac > 1e-9) & (frac < 1 - 1e-9)
    x, _ = gll.gll(wl.p)
    tloc = 2.0 * frac[inner] - 1.0
    j = np.array([int(np.argmin(np.abs(x - t))) for t in tloc])
    np.testing.assert_allclose(r[right][inner], 4.0 * a * (h / 2.0) * w[j], rtol=1e-10)


@pytest.mark.parametrize("hx,hy", [(2.0, 0.5), (1.0, 3.0)])
def test_rectangle_tensor_product_identity(hx, hy):
    """Axis-aligned h_x x h_y rectangle: K_e = c^2 [(h_y/h_x) W (x) S + (h_x/h_y) S (x) W]
    with S = D^T W D the 1D stiffness and W the 1D weights (q = a + n b ordering)."""
    p = 4
    vxy = np.array([[0, 0], [hx, 0], [hx, hy], [0, hy]], dtype=np.float64) + [3.0, -1.0]
    quads = np.array([[0, 1, 2, 3]])
    Ke = mesh.element_stiffness(vxy, quads, p, np.array([2.5]))[0]
    x, w = gll.gll(p)
    D = gll.derivative_matrix(p)
    S = D.T @ np.diag(w) @ D
    W = np.diag(w)
    expect = 2.5 * ((hy / hx) * np.kron(W, S) + (hx / hy) * np.kron(S, W))
    np.testing.assert_allclose(Ke, expect, atol=1e-13 * np.abs(expect).max())


def test_stiffness_rotation_invariant():
    p = 5
    rng = np.random.default_rng(3)
    base = np.array([[0, 0], [1.2, 0.1], [1.0, 0.9], [-0.1, 1.1]])
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    K0 = mesh.element_stiffness(base, np.array([[0, 1, 2, 3]]), p)[0]
    K1 = mesh.element_stiffness(base @ R.T + rng.standard_normal(2), np.array([[0, 1, 2, 3]]), p)[0]
    np.testing.assert_allclose(K0, K1, atol=1e-12 * np.abs(K0).max())


def test_cfl_dt_homogeneous_closed_form():
    """Uniform h x h elements: the smallest GLL spacing is h (xi_1 - xi_0) / 2."""
    wl = workloads.workload("homog64")
    x, _ = gll.gll(4)
    h = wl.Lx / wl.nx
    expect = 0.3 * (h * (x[1] - x[0]) / 2.0) / 1500.0
    dt = solver.cfl_dt(wl.vxy, wl.quads, wl.c2, wl.p)
    assert abs(dt - expect) < 1e-12 * expect
    assert abs(dt - 5.40e-4) < 0.01e-4          # 1 km / 64, p=4, c=1500


def test_stability_bound_above_cfl_dt(jittered):
    wl, sem = jittered
    lam = sem.lambda_max(iters=300)
    assert sem.dt_cfl() < 2.0 / np.sqrt(lam)
