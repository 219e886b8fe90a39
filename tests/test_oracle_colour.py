"""Pins of the oracle's greedy element colouring (Sec. 5, the colouring paragraph after
Alg. 2): a hand-worked fixture, validity and the first-fit property by brute force, and
the colour count of a structured grid, whose interior vertices make 4-cliques."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import colour, mesh, reorder

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [1, 3])
def test_hand_worked_grid(p):
    g = json.load(open(os.path.join(GOLDEN, "colour_grid3x2.json")))
    quads = np.array(g["quads"], dtype=np.int64)
    conn, _ = mesh.global_numbering(quads, len(g["vxy"]), p)
    for order, want in zip(g["orders"], g["colours"]):
        np.testing.assert_array_equal(colour.greedy_colours(conn, order), want)


def _brute_force_check(conn, order, col):
    """Joined elements differ; every colour below an element's own is taken by an
    earlier-visited neighbour (first fit)."""
    E = conn.shape[0]
    sets = [set(r.tolist()) for r in conn]
    pos = np.empty(E, np.int64)
    pos[np.asarray(order)] = np.arange(E)
    for e in range(E):
        joined = [f for f in range(E) if f != e and sets[e] & sets[f]]
        assert all(col[f] != col[e] for f in joined)
        earlier = {int(col[f]) for f in joined if pos[f] < pos[e]}
        assert set(range(int(col[e]))) <= earlier


@pytest.mark.parametrize("kind", ["hilbert", "lex", "random", "morton"])
def test_valid_and_first_fit(kind):
    wl = workloads.workload("layered1024", n=9, p=2)
    conn, _ = mesh.global_numbering(wl.quads, wl.vxy.shape[0], 2)
    order = reorder.element_order(kind, wl.vxy, wl.quads, seed=3)
    col = colour.greedy_colours(conn, order)
    _brute_force_check(conn, order, col)
    # an interior vertex is shared by 4 elements, which are pairwise joined
    assert col.max() + 1 >= 4


@pytest.mark.parametrize("nx,ny", [(2, 2), (5, 3), (8, 8)])
def test_lexicographic_grid_needs_four(nx, ny):
    """Row-major first fit on a structured grid alternates 0,1 on even rows and 2,3 on
    odd rows: exactly the clique number 4."""
    vxy, quads, _, _ = workloads.grid_mesh(nx, ny, 1.0, 1.0)
    conn, _ = mesh.global_numbering(quads, vxy.shape[0], 2)
    col = colour.greedy_colours(conn)
    i = np.arange(nx * ny) % nx
    j = np.arange(nx * ny) // nx
    np.testing.assert_array_equal(col, (i % 2) + 2 * (j % 2))


def test_strip_needs_two():
    vxy, quads, _, _ = workloads.grid_mesh(7, 1, 7.0, 1.0)
    conn, _ = mesh.global_numbering(quads, vxy.shape[0], 3)
    np.testing.assert_array_equal(colour.greedy_colours(conn), np.arange(7) % 2)


def test_colour_classes_partition_in_order():
    wl = workloads.workload("layered1024", n=6)
    conn, _ = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    order = reorder.element_order("hilbert", wl.vxy, wl.quads)
    col = colour.greedy_colours(conn, order)
    cls = colour.colour_classes(col, order)
    assert sorted(np.concatenate(cls).tolist()) == list(range(conn.shape[0]))
    pos = np.empty(conn.shape[0], np.int64)
    pos[order] = np.arange(conn.shape[0])
    for c, members in enumerate(cls):
        assert np.all(col[members] == c)
        assert np.all(np.diff(pos[members]) > 0)
