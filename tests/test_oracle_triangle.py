"""Pins of the oracle's triangle element (Sec. 4.2; Blyth-Pozrikidis nodes, nodal basis,
interpolatory weights): a hand-worked numbering fixture, the textbook linear-triangle
(cotangent) stiffness at p = 1, node placement facts, duality and exactness of the
derivatives on polynomials, weights against an independent collapsed Gauss quadrature,
operator properties on jittered meshes, energy conservation and spectral convergence of a
standing mode."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import gll, triangle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ODD = (1, 3, 5, 7)


def test_numbering_hand_worked():
    g = json.load(open(os.path.join(GOLDEN, "tri_numbering_2el_p3.json")))
    conn, n = triangle.global_numbering(np.array(g["tris"]), len(g["vxy"]), g["p"])
    np.testing.assert_array_equal(conn, g["conn"])
    assert n == g["n_nodes"]


@pytest.mark.parametrize("p", ODD)
def test_node_count_and_placement(p):
    """(p+1)(p+2)/2 nodes (21 at p = 5, Sec. 5); vertices at the corners; each edge carries
    the 1D GLL nodes on [0, 1]; the set is invariant under the six symmetries of the
    triangle (permutations of the barycentric coordinates)."""
    X = triangle.reference_nodes(p)
    assert X.shape == ((p + 1) * (p + 2) // 2, 2)
    if p == 5:
        assert X.shape[0] == 21
    for (i, j), c in zip(((0, 0), (p, 0), (0, p)), ((0, 0), (1, 0), (0, 1))):
        np.testing.assert_allclose(X[triangle.local_index(i, j, p)], c, atol=1e-15)
    v = 0.5 * (gll.gll(p)[0] + 1.0)
    for t in range(p + 1):
        np.testing.assert_allclose(X[triangle.local_index(t, 0, p)], (v[t], 0.0), atol=1e-15)
        np.testing.assert_allclose(X[triangle.local_index(0, t, p)], (0.0, v[t]), atol=1e-15)
        np.testing.assert_allclose(X[triangle.local_index(t, p - t, p)], (v[t], 1.0 - v[t]), atol=1e-15)
    lam = np.stack([1.0 - X[:, 0] - X[:, 1], X[:, 0], X[:, 1]], axis=1)
    key = lambda L: sorted(map(tuple, np.round(L, 12)))
    import itertools
    for perm in itertools.permutations(range(3)):
        assert key(lam[:, perm]) == key(lam)


@pytest.mark.parametrize("p", ODD)
def test_duality_and_derivative_exactness(p):
    X = triangle.reference_nodes(p)
    np.testing.assert_allclose(triangle.basis_values(p, X), np.eye(X.shape[0]), atol=1e-11)
    Dx, Dy, _ = triangle.reference_operators(p)
    x, y = X[:, 0], X[:, 1]
    for a in range(p + 1):
        for b in range(p + 1 - a):
            f = x ** a * y ** b
            fx = a * x ** max(a - 1, 0) * y ** b if a else 0 * x
            fy = b * x ** a * y ** max(b - 1, 0) if b else 0 * x
            np.testing.assert_allclose(Dx @ f, fx, atol=1e-11 * max(1, p * p))
            np.testing.assert_allclose(Dy @ f, fy, atol=1e-11 * max(1, p * p))
    # one degree more is not reproduced (the basis spans degree <= p only)
    f = x ** (p + 1)
    assert np.abs(Dx @ f - (p + 1) * x ** p).max() > 1e-6


def _collapsed_gauss(f, n=12):
    """Integral over the reference triangle by Gauss-Legendre on the square mapped with
    x = u (1 - v), y = v (Jacobian 1 - v): independent of the nodal rule."""
    t, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    U, V = np.meshgrid(t, t, indexing="ij")
    W = np.outer(w, w)
    return float(np.sum(W * (1.0 - V) * f(U * (1.0 - V), V)))


@pytest.mark.parametrize("p", ODD)
def test_weights_integrate_exactly_to_degree_p(p):
    _, _, om = triangle.reference_operators(p)
    X = triangle.reference_nodes(p)
    assert om.sum() == pytest.approx(0.5, abs=1e-14)
    assert om.min() > 0
    for a in range(p + 1):
        for b in range(p + 1 - a):
            f = lambda x, y: x ** a * y ** b
            assert om @ f(X[:, 0], X[:, 1]) == pytest.approx(_collapsed_gauss(f), abs=1e-14)
    # each weight is the integral of its basis function
    for m in (0, X.shape[0] // 2, X.shape[0] - 1):
        g = lambda x, y: triangle.basis_values(p, np.stack([x.ravel(), y.ravel()], 1))[:, m].reshape(x.shape)
        assert om[m] == pytest.approx(_collapsed_gauss(g), abs=1e-11)


@pytest.mark.parametrize("p", (2, 4, 6))
def test_even_orders_have_non_positive_weights(p):
    """Why only odd p are used: the interpolatory weights of even p are not all positive."""
    import fractions  # noqa: F401  (exact path of the oracle)
    Dx, Dy, om = (np.vectorize(float)(np.array(a, dtype=object)) for a in triangle._exact_operators(p))
    assert om.min() <= 1e-15
    with pytest.raises(ValueError):
        triangle.check_p(p)


def test_p1_is_the_linear_triangle_cotangent_stiffness():
    """p = 1: vertices, weights 1/6, and K_e[a, b] = -(c^2 / 2) cot(angle opposite edge ab),
    K_e[a, a] = -sum of the row (the classical linear-element stiffness)."""
    vxy = np.array([[0.0, 0.0], [3.0, 0.4], [1.1, 2.0]])
    tris = np.array([[0, 1, 2]])
    _, _, om = triangle.reference_operators(1)
    np.testing.assert_allclose(om, [1 / 6] * 3, atol=1e-16)
    Ke = triangle.element_stiffness(vxy, tris, 1, np.array([2.5]))[0]
    want = np.zeros((3, 3))
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        u, w = vxy[a] - vxy[c], vxy[b] - vxy[c]
        cot = (u @ w) / abs(u[0] * w[1] - u[1] * w[0])
        want[a, b] = want[b, a] = -0.5 * 2.5 * cot
    want[np.arange(3), np.arange(3)] = -want.sum(axis=1)
    np.testing.assert_allclose(Ke, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("p", (3, 5))
def test_operator_properties_on_a_jittered_mesh(p):
    vxy, tris, _, _ = workloads.tri_mesh(5, 4, 700.0, 400.0, jitter=0.2, seed=5)
    rng = np.random.default_rng(1)
    c2 = rng.uniform(1.0, 4.0, tris.shape[0]) * 1500.0 ** 2
    sem = triangle.TriSEM(vxy, tris, c2, p)
    K = sem.K.toarray()
    nrm = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-13 * nrm
    assert np.abs(K @ np.ones(sem.n_nodes)).max() <= 1e-12 * nrm
    assert np.linalg.eigvalsh(K).min() >= -1e-11 * nrm
    assert sem.mass.sum() == pytest.approx(700.0 * 400.0, rel=1e-13)
    assert sem.mass.min() > 0
    # patch test (constant c): a linear field gives zero at nodes away from the boundary
    sem = triangle.TriSEM(vxy, tris, np.full(tris.shape[0], 1500.0 ** 2), p)
    K = sem.K.toarray()
    nrm = np.abs(K).max()
    xy = sem.node_xy
    u = 0.3 * xy[:, 0] - 1.7 * xy[:, 1] + 5.0
    r = K @ u
    inner = (xy[:, 0] > 1e-9) & (xy[:, 0] < 700 - 1e-9) & (xy[:, 1] > 1e-9) & (xy[:, 1] < 400 - 1e-9)
    assert np.abs(r[inner]).max() <= 1e-12 * nrm * np.abs(u).max()
    assert np.abs(r[~inner]).max() > 1e-3 * nrm
    # every element maps a shared node to the same coordinates
    ref = triangle.reference_nodes(p)
    X = vxy[tris]
    pts = X[:, None, 0] + ref[None, :, 0:1] * (X[:, None, 1] - X[:, None, 0]) + ref[None, :, 1:2] * (X[:, None, 2] - X[:, None, 0])
    np.testing.assert_allclose(xy[sem.conn], pts, atol=1e-9)


def test_energy_conserved():
    vxy, tris, _, _ = workloads.tri_mesh(6, 6, 600.0, 600.0, jitter=0.2, seed=3)
    sem = triangle.TriSEM(vxy, tris, np.full(tris.shape[0], 1500.0 ** 2), 5)
    dt = sem.dt_default()
    xy = sem.node_xy
    u0 = np.exp(-((xy[:, 0] - 300) ** 2 + (xy[:, 1] - 250) ** 2) / 2e3)
    es = []
    sem.run(500, dt, u0=u0, callback=lambda n, u, un, v: es.append(sem.energy(un[:, 0], u[:, 0], v[:, 0])))
    es = np.array(es)
    assert np.abs(es / es[0] - 1.0).max() < 1e-12


def _standing_error(p, n):
    """Max error after about one period of the Neumann mode cos(3 pi x) cos(2 pi y) on an
    n x n triangulated unit square, leapfrog with the time factor that is exact for the
    continuous mode (so the error left is the spatial one, mostly a phase error)."""
    vxy, tris, _, _ = workloads.tri_mesh(n, n, 1.0, 1.0)
    sem = triangle.TriSEM(vxy, tris, np.ones(tris.shape[0]), p)
    dt = sem.dt_default(0.5)
    om = np.pi * np.sqrt(13.0)
    th = np.arccos(1.0 - (om * dt) ** 2 / 2.0)
    nst = int(round(2 * np.pi / th))
    phi = np.cos(3 * np.pi * sem.node_xy[:, 0]) * np.cos(2 * np.pi * sem.node_xy[:, 1])
    _, u, _ = sem.run(nst, dt, u0=phi, v0=phi * (1 - np.cos(th)) / dt)
    return float(np.abs(u[:, 0] - phi * np.cos(nst * th)).max())


def test_standing_mode_converges():
    """The error falls with p at fixed h and with h at fixed p. The rate in h is algebraic
    (about h^3 to h^4 at p = 3 and 5): the nodal rule is exact only to degree p, so mass
    lumping and stiffness quadrature limit the order, unlike the GLL quadrilaterals."""
    errs = {p: _standing_error(p, 4) for p in ODD}
    assert errs[1] > errs[3] > errs[5] > errs[7], errs
    assert errs[7] < 0.05, errs
    eh = [_standing_error(5, n) for n in (4, 8, 16)]
    assert eh[0] > 4 * eh[1] > 16 * eh[2], eh
    assert eh[2] < 1e-3, eh


def test_node_spacing_cfl_does_not_bound_the_spectrum():
    """Why the triangle time step comes from lambda_max: at p = 7 the CFL-0.3 rule on the
    smallest node distance exceeds the leapfrog limit."""
    vxy, tris, _, _ = workloads.tri_mesh(4, 4, 1.0, 1.0)
    sem = triangle.TriSEM(vxy, tris, np.ones(tris.shape[0]), 7)
    assert sem.dt_cfl(0.3) > 2.0 / np.sqrt(sem.lambda_max())
    assert sem.dt_default() < 2.0 / np.sqrt(sem.lambda_max())


def test_sampled_rows_match_assembly():
    """The per-node checker of the full-size GPU tests equals rows of the assembled K and
    the lumped mass (corner, edge, interior and vertex nodes, jittered mesh, variable c)."""
    vxy, tris, _, _ = workloads.tri_mesh(7, 5, 700.0, 500.0, jitter=0.2, seed=8)
    c2 = np.random.default_rng(2).uniform(1.0, 3.0, tris.shape[0]) * 1e6
    sem = triangle.TriSEM(vxy, tris, c2, 5)
    u = np.random.default_rng(3).standard_normal(sem.n_nodes)
    nodes = np.unique(np.r_[0, 7, 40, sem.n_nodes - 1, np.random.default_rng(4).choice(sem.n_nodes, 40, replace=False)])
    r, M = triangle.sampled_rows(vxy, tris, c2, 5, sem.conn, nodes, u)
    np.testing.assert_allclose(r, (sem.K @ u)[nodes], rtol=1e-13, atol=1e-13 * np.abs(sem.K @ u).max())
    np.testing.assert_allclose(M, sem.mass[nodes], rtol=1e-13)


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_stiffness_is_cotangent_weighted_rotations_of_one_matrix(p):
    """On an affine triangle the element stiffness is a sum over the three vertex pairs,
    K_e = sum c_ij E_ij with c_ij = -det J grad(lambda_i).grad(lambda_j) (the cotangent
    weights), and the three E_ij are one matrix seen from rotated vertices: E[q][m] =
    E_12[s(q)][s(m)] for the node rotations (i, j, k) -> (j, k, i) and (k, i, j), since the
    Blyth-Pozrikidis node set is invariant under them (Sec. 4.2). Checked with the oracle's
    exact basis: the matrices to 1e-12 and K_e of random triangles to 1e-12."""
    Dx, Dy, om = triangle.reference_operators(p)
    Sxx, Syy = (Dx.T * om) @ Dx, (Dy.T * om) @ Dy
    Sxy = (Dx.T * om) @ Dy + (Dy.T * om) @ Dx
    nodes = triangle.local_nodes(p)
    s23 = np.array([triangle.local_index(j, p - i - j, p) for i, j in nodes])
    s13 = np.array([triangle.local_index(p - i - j, i, p) for i, j in nodes])
    E12, E23, E13 = Sxx, Sxx + Syy - Sxy, Syy
    scale = np.abs(Sxx).max()
    assert np.abs(E23 - Sxx[np.ix_(s23, s23)]).max() <= 1e-12 * scale
    assert np.abs(E13 - Sxx[np.ix_(s13, s13)]).max() <= 1e-12 * scale
    # the rotations are not trivial: Sxx itself is not invariant under them
    assert np.abs(Sxx - Sxx[np.ix_(s23, s23)]).max() > 1e-3 * scale
    rng = np.random.default_rng(31)
    vxy = rng.uniform(-1.0, 1.0, size=(30, 2))
    tris = np.arange(30).reshape(10, 3)
    J, det = triangle.jacobians(vxy, tris)
    flip = det < 0
    tris[flip] = tris[flip][:, ::-1]
    J, det = triangle.jacobians(vxy, tris)
    Ke = triangle.element_stiffness(vxy, tris, p)
    n = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])      # reference barycentric gradients
    for e in range(len(tris)):
        g = np.linalg.solve(J[e].T, n.T).T                    # physical gradients, [3, 2]
        c = lambda a, b: -det[e] * (g[a] @ g[b])
        K2 = c(0, 1) * E12 + c(1, 2) * E23 + c(0, 2) * E13
        assert np.abs(K2 - Ke[e]).max() <= 1e-12 * np.abs(Ke[e]).max()
