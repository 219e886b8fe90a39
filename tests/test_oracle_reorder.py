"""Pins of the oracle's reordering (Sec. 4.3) against brute force and closed forms.

The paper states that the generalized Hilbert curve equals the standard one when the
sides are powers of two (Sec. 3); the standard curve is produced here by an independent
textbook bit-manipulation conversion, not by the oracle's recursive splitter.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import mesh, reorder

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def standard_hilbert_d2xy(order: int, d: int):
    """Classic iterative distance -> (x, y) conversion for a 2^order square."""
    n = 1 << order
    x = y = 0
    t = d
    s = 1
    while s < n:
        rx = 1 & (t // 2)
        ry = 1 & (t ^ rx)
        if ry == 0:
            if rx == 1:
                x = s - 1 - x
                y = s - 1 - y
            x, y = y, x
        x += s * rx
        y += s * ry
        t //= 4
        s *= 2
    return x, y


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 6])
def test_generalized_curve_equals_standard_on_powers_of_two(order):
    n = 1 << order
    xs, ys = reorder.gilbert_cells(n, n)
    ref = [standard_hilbert_d2xy(order, d) for d in range(n * n)]
    assert list(zip(xs.tolist(), ys.tolist())) == ref
    # start at (0, 0), end at (2^a - 1, 0); second cell (0,1) for odd orders, (1,0) for even
    assert (xs[0], ys[0]) == (0, 0)
    assert (xs[-1], ys[-1]) == (n - 1, 0)
    assert (xs[1], ys[1]) == ((0, 1) if order % 2 else (1, 0))


def test_generalized_curve_power_of_two_large():
    """Order 10 (the 1024 x 1024 grid of the layered workload), sampled."""
    xs, ys = reorder.gilbert_cells(1024, 1024)
    rng = np.random.default_rng(0)
    for d in rng.integers(0, 1024 * 1024, 2000).tolist():
        assert (xs[d], ys[d]) == standard_hilbert_d2xy(10, d)


def test_generalized_curve_properties_small_rectangles():
    for W in range(1, 25):
        for H in range(1, 25):
            xs, ys = reorder.gilbert_cells(W, H)
            cells = set(zip(xs.tolist(), ys.tolist()))
            assert len(cells) == W * H and min(xs) == 0 and max(xs) == W - 1
            assert min(ys) == 0 and max(ys) == H - 1
            assert (xs[0], ys[0]) == (0, 0)
            step = np.abs(np.diff(xs)) + np.abs(np.diff(ys))
            diag = (np.abs(np.diff(xs)) == 1) & (np.abs(np.diff(ys)) == 1)
            # every move is to a side neighbour, except a single diagonal move that
            # appears exactly when the longer side is odd and the shorter side even
            assert np.all((step == 1) | diag)
            big, small = max(W, H), min(W, H)
            expect_diag = 1 if (big % 2 == 1 and small % 2 == 0 and small > 2) else 0
            assert int(diag.sum()) == expect_diag, (W, H)


def test_hilbert_order_one_element_per_cell_matches_standard_curve():
    """64 x 64 uniform grid: one element per cell, so list L is the standard curve of
    order 6 over the element (i, j) grid."""
    wl = workloads.workload("homog64")
    L = reorder.hilbert_order(wl.vxy, wl.quads)
    ref = [standard_hilbert_d2xy(6, d) for d in range(64 * 64)]
    np.testing.assert_array_equal(L, [x + 64 * y for x, y in ref])


def test_hilbert_order_jittered_still_one_per_cell():
    wl = workloads.workload("layered1024", n=32)
    cx, cy, W, H = reorder.centroid_cells(wl.vxy, wl.quads)
    e = np.arange(wl.n_elements)
    np.testing.assert_array_equal(cx, e % 32)
    np.testing.assert_array_equal(cy, e // 32)
    assert (W, H) == (32, 32)


def test_hilbert_order_graded_many_per_cell():
    """Graded mesh: many elements share a cell near the fine corner, cells at the coarse
    corner are empty; L still lists each element once, cells in curve order, ids
    ascending inside a cell."""
    wl = workloads.workload("graded1414", n=40)
    L = reorder.hilbert_order(wl.vxy, wl.quads)
    assert sorted(L.tolist()) == list(range(wl.n_elements))
    cx, cy, W, H = reorder.centroid_cells(wl.vxy, wl.quads)
    idx = reorder.hilbert_index_grid(W, H)
    key = idx[cy, cx]
    counts = np.bincount(cy * W + cx, minlength=W * H)
    assert counts.max() > 4 and (counts == 0).sum() > 0
    k = key[L]
    assert np.all(np.diff(k) >= 0)
    same = np.diff(k) == 0
    assert np.all(np.diff(L)[same] > 0)


def test_morton_brute_force():
    rng = np.random.default_rng(1)
    cx = rng.integers(0, 1 << 20, 500)
    cy = rng.integers(0, 1 << 20, 500)
    key = reorder.morton_key(cx, cy)
    for a, b, k in zip(cx.tolist(), cy.tolist(), key.tolist()):
        s = 0
        for bit in range(21):
            s |= ((a >> bit) & 1) << (2 * bit)
            s |= ((b >> bit) & 1) << (2 * bit + 1)
        assert s == k


def test_splitmix64_reference_value():
    # SplitMix64 seeded with 0: first output of the reference generator
    assert int(reorder.splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF


def test_random_order_is_permutation_and_seeded():
    a = reorder.random_order(1000, 3)
    b = reorder.random_order(1000, 3)
    c = reorder.random_order(1000, 4)
    assert sorted(a.tolist()) == list(range(1000))
    np.testing.assert_array_equal(a, b)
    assert np.any(a != c)


def _brute_degree(conn, n_nodes):
    nb = [set() for _ in range(n_nodes)]
    for row in conn.tolist():
        for a in row:
            nb[a].update(row)
    return np.array([len(s) - 1 for s in nb])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_degree_brute_force(p):
    wl = workloads.workload("layered1024", n=5, p=p)
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], p)
    np.testing.assert_array_equal(reorder.node_degree(conn, n, chunk=64), _brute_degree(conn, n))


def test_first_touch_properties():
    wl = workloads.workload("layered1024", n=12)
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    elem, node = reorder.reorder("hilbert", wl.vxy, wl.quads, conn)
    assert sorted(node.tolist()) == list(range(n))
    new_id = np.empty(n, np.int64)
    new_id[node] = np.arange(n)
    deg = reorder.node_degree(conn, n)
    seen = -1
    for e in elem.tolist():
        ids = new_id[conn[e]]
        fresh = ids[ids > seen]
        # fresh nodes of an element get the next consecutive ids...
        np.testing.assert_array_equal(np.sort(fresh), np.arange(seen + 1, seen + 1 + fresh.size))
        # ...ordered by ascending degree
        assert np.all(np.diff(deg[node[np.sort(fresh)]]) >= 0)
        seen = max(seen, ids.max())


# ------------------------------------------------------ the paper's node-walk strategies
def test_walk_orders_hand_worked_fixture():
    """Node Connectivity and Node Distance strategies (Sec. 5) on a scrambled 3x1 strip,
    against orders worked by hand (tests/golden/walk_orders_strip3.json)."""
    g = json.load(open(os.path.join(GOLDEN, "walk_orders_strip3.json")))
    vxy, quads = np.array(g["vxy"], float), np.array(g["quads"])
    nv = vxy.shape[0]
    np.testing.assert_array_equal(reorder.vertex_degree(quads, nv), g["degree"])
    for kind, prio in (("connectivity", reorder.vertex_degree(quads, nv)),
                       ("distance", reorder.distance_priority(vxy))):
        el, vt = reorder.walk_order(quads, nv, prio)
        np.testing.assert_array_equal(el, g[kind]["elements"], err_msg=kind)
        np.testing.assert_array_equal(vt, g[kind]["vertices"], err_msg=kind)
        np.testing.assert_array_equal(reorder.element_order(kind, vxy, quads), g[kind]["elements"])


@pytest.mark.parametrize("kind", ["connectivity", "distance"])
def test_walk_orders_are_breadth_first(kind):
    """On a jittered 13x9 grid: the vertex visit order is a breadth-first order from the
    start vertex (hop counts never decrease, checked against scipy's shortest paths); the
    start has the least priority; every element is listed when its first vertex is
    visited, elements of one vertex in ascending id."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    vxy, quads, _, _ = workloads.grid_mesh(13, 9, 1300.0, 900.0, jitter=0.2, seed=5)
    nv = vxy.shape[0]
    prio = reorder.vertex_degree(quads, nv) if kind == "connectivity" else reorder.distance_priority(vxy)
    el, vt = reorder.walk_order(quads, nv, prio)
    assert sorted(el.tolist()) == list(range(quads.shape[0]))
    assert sorted(vt.tolist()) == list(range(nv))
    best = min(range(nv), key=lambda v: (prio[v], v))
    assert vt[0] == best
    rows, cols = [], []
    for q in quads.tolist():
        for a in q:
            for b in q:
                if a != b:
                    rows.append(a)
                    cols.append(b)
    A = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(nv, nv)).tocsr()
    hops = shortest_path(A, unweighted=True, indices=[vt[0]])[0]
    assert np.all(np.diff(hops[vt]) >= 0)
    pos = np.empty(nv, np.int64)
    pos[vt] = np.arange(nv)
    first = np.array([pos[q].min() for q in quads[el]])
    assert np.all(np.diff(first) >= 0)
    same = np.diff(first) == 0
    assert np.all(np.diff(el)[same] > 0)
