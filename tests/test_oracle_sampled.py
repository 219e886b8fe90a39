"""Pins of the oracle helpers that check the GPU at full size, where the assembled
operator does not fit: ``node_incidence`` and ``sampled_rows`` must give exactly the rows
of the assembled K u and the lumped mass (Sec. 4.2, Eqs. R and A-bar), and
``lambda_max`` the largest eigenvalue of M^-1/2 K M^-1/2 from a dense eigensolver."""
import numpy as np
import pytest

import workloads
from oracle import mesh, solver


def _sample_nodes(wl, conn, n_nodes):
    """Domain corners, a vertex on the boundary and one inside, edge-interior nodes on
    and off the boundary, element-interior nodes."""
    nx, ny = wl.nx, wl.ny
    nv = wl.vxy.shape[0]
    corners = [0, nx, (nx + 1) * ny, (nx + 1) * (ny + 1) - 1]
    vert = [nx // 2, (nx + 1) * (ny // 2) + nx // 2]
    p = wl.p
    q_edge = [1, (p + 1) * 1 + p]                    # (a=1, b=0) and (a=p, b=1)
    q_int = [(p + 1) * 1 + 1, (p + 1) * (p // 2) + p // 2]
    e_mid = (ny // 2) * nx + nx // 2
    edge = [int(conn[0, q]) for q in q_edge] + [int(conn[e_mid, q]) for q in q_edge]
    inner = [int(conn[e_mid, q]) for q in q_int] + [int(conn[nx * ny - 1, q_int[0]])]
    nodes = np.array(corners + vert + edge + inner, dtype=np.int64)
    assert np.all(nodes < n_nodes) and np.all(nodes[:6] < nv)
    assert np.all(nodes[-3:] >= n_nodes - wl.quads.shape[0] * (p - 1) ** 2)
    return nodes


@pytest.mark.parametrize("name,n,shots", [("layered1024", 12, 1), ("layered1024", 12, 3),
                                          ("graded1414", 10, 1), ("graded1414", 10, 3)])
def test_sampled_rows_equal_assembled(name, n, shots):
    wl = workloads.workload(name, n=n)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    nodes = _sample_nodes(wl, o.conn, o.n_nodes)
    u = workloads.random_field(o.n_nodes, shots, seed=17).T
    if shots == 1:
        u = u[:, 0]
    r, M = solver.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, o.conn, nodes, u)
    r_full = o.K @ u
    scale = np.abs(r_full).max()
    assert np.abs(r - r_full[nodes]).max() <= 1e-13 * scale
    np.testing.assert_allclose(M, o.mass[nodes], rtol=1e-13, atol=0)


def test_node_incidence_lists_every_slot_once():
    wl = workloads.workload("graded1414", n=7)
    conn, n_nodes = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    start, elem, slot = solver.node_incidence(conn, n_nodes)
    assert start[0] == 0 and start[-1] == conn.size
    seen = set()
    for v in range(n_nodes):
        for e, q in zip(elem[start[v]:start[v + 1]], slot[start[v]:start[v + 1]]):
            assert conn[e, q] == v
            seen.add((int(e), int(q)))
    assert len(seen) == conn.size
    # a vertex inside the mesh belongs to 4 elements, an edge node to 2, an interior one to 1
    counts = np.diff(start)
    nv = wl.vxy.shape[0]
    assert counts[(wl.nx + 1) * 3 + 3] == 4
    assert counts[nv] == 1 or counts[nv] == 2
    assert np.all(counts[n_nodes - wl.quads.shape[0] * (wl.p - 1) ** 2:] == 1)


@pytest.mark.parametrize("name", ["layered1024", "graded1414"])
def test_lambda_max_against_dense_eigensolver(name):
    wl = workloads.workload(name, n=6)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = 1.0 / np.sqrt(o.mass)
    A = o.K.toarray() * s[:, None] * s[None, :]
    lam = np.linalg.eigvalsh(A)[-1]
    assert abs(o.lambda_max() / lam - 1.0) <= 1e-8
