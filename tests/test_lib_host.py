"""CPU tests of the C-ABI library: exported symbols, host-only setup bit-exact against the
oracle's independent reorder (Sec. 4.3), the Hilbert key function against the oracle's
curve enumeration, node snapping, dt, and error paths forced from the host."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import workloads
from oracle import mesh, reorder, solver

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported(semlib):
    hdr = open(os.path.join(ROOT, "include", "sem.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sem_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 19
    lib = ctypes.CDLL(semlib.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(semlib.EXPORTS)


def _oracle_perm(wl, kind, seed=3):
    conn, _ = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    return reorder.reorder(kind, wl.vxy, wl.quads, conn, seed=seed)


CASES = [("homog64", dict(), ("hilbert", "lex", "random", "connectivity", "distance")),
         ("layered1024", dict(n=30), ("hilbert", "morton", "lex", "random", "connectivity", "distance")),
         ("graded1414", dict(n=40, p=5), ("hilbert", "morton", "random", "connectivity", "distance")),
         ("batch512", dict(n=48), ("hilbert", "random", "connectivity", "distance"))]


@pytest.mark.parametrize("name,kw,orders", CASES)
def test_permutations_bit_exact(semlib, name, kw, orders):
    wl = workloads.workload(name, **kw)
    for kind in orders:
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, order=kind, device=-1, seed=3)
        e, n = s.permutations()
        oe, on = _oracle_perm(wl, kind)
        np.testing.assert_array_equal(e, oe, err_msg=kind)
        np.testing.assert_array_equal(n, on, err_msg=kind)
        s.close()


@pytest.mark.parametrize("name,kw", [("batch512", dict(n=48)), ("graded1414", dict(n=30, p=5))])
def test_64_shot_lanes_regroup_owned_nodes(semlib, name, kw):
    """With 64 shot lanes every tile's owned range lists its nodes on an element edge first
    (nodes of two or more elements and nodes on the domain boundary), then its
    element-interior nodes, each group in first-touch order; the element order is unchanged
    and the accumulator slots fit the LDS budget."""
    wl = workloads.workload(name, **kw)
    conn, n_nodes = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    start, _, _ = solver.node_incidence(conn, n_nodes)
    n = wl.p + 1
    a_loc, b_loc = np.arange(n * n) % n, np.arange(n * n) // n
    edge_q = (a_loc == 0) | (a_loc == wl.p) | (b_loc == 0) | (b_loc == wl.p)
    edge = np.zeros(n_nodes, bool)
    edge[conn[:, edge_q].ravel()] = True
    assert edge[np.diff(start) > 1].all()           # every shared node lies on an edge
    oe, on = _oracle_perm(wl, "hilbert")
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, n_shots=64, lds_bytes=16384)
    inf = s.info()
    assert inf["shot_lanes"] == 64
    assert 0 < inf["max_accum_nodes"] <= 16384 // (64 * 8) < inf["max_owned_nodes"]
    e, n = s.permutations()
    s.close()
    np.testing.assert_array_equal(e, oe)
    assert np.array_equal(np.sort(n), np.arange(n_nodes)) and not np.array_equal(n, on)
    pos = np.empty(n_nodes, np.int64)
    pos[on] = np.arange(n_nodes)              # first-touch position of every node
    p_lib = pos[n]
    ends = np.flatnonzero(np.maximum.accumulate(p_lib) == np.arange(n_nodes)) + 1
    assert len(ends) >= inf["n_tiles"]
    b = 0
    for t in ends:
        blk = n[b:t]
        shared = edge[blk]
        k = int(shared.sum())
        assert shared[:k].all() and not shared[k:].any()
        assert np.all(np.diff(pos[blk[:k]]) > 0) and np.all(np.diff(pos[blk[k:]]) > 0)
        b = t


@pytest.mark.slow
def test_permutations_bit_exact_256():
    """65,536 elements, 1,050,625 nodes: a size that spans many tiles."""
    from paper_2104_08416_amd import sem as semlib
    wl = workloads.workload("layered1024", n=256)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, order="hilbert", device=-1)
    e, n = s.permutations()
    oe, on = _oracle_perm(wl, "hilbert")
    np.testing.assert_array_equal(e, oe)
    np.testing.assert_array_equal(n, on)


def test_hilbert_index_matches_curve_enumeration(semlib):
    for W in range(1, 25):
        for H in range(1, 25):
            xs, ys = reorder.gilbert_cells(W, H)
            idx = semlib.hilbert_index(W, H, xs, ys)
            np.testing.assert_array_equal(idx, np.arange(W * H), err_msg=f"{W}x{H}")


@pytest.mark.parametrize("W,H", [(1414, 1414), (1024, 1024), (1000, 37), (37, 1000), (513, 511)])
def test_hilbert_index_large_grids(semlib, W, H):
    xs, ys = reorder.gilbert_cells(W, H)
    idx = semlib.hilbert_index(W, H, xs, ys)
    np.testing.assert_array_equal(idx, np.arange(W * H))


def test_dt_nodes_and_snapping_match_oracle(semlib):
    wl = workloads.workload("batch512", n=24, n_shots=5)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, n_shots=5)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    assert s.n_nodes == o.n_nodes
    assert abs(s.dt - o.dt_cfl()) <= 1e-15 * o.dt_cfl()
    np.testing.assert_array_equal(s.node_coords(), o.node_xy)
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    np.testing.assert_array_equal(src, solver.snap_to_nodes(wl.src_xy, o.node_xy))
    rec = s.set_receivers(wl.rec_xy)
    np.testing.assert_array_equal(rec, solver.snap_to_nodes(wl.rec_xy, o.node_xy))
    assert s.info()["n_receivers"] == wl.rec_xy.shape[0]


@pytest.mark.parametrize("name,kw", [("layered1024", dict(n=30)), ("tri2000", dict(n=24, p=5)),
                                     ("graded1414", dict(n=12, p=5))])
def test_snapping_is_the_nearest_node_everywhere(semlib, name, kw):
    """Point snapping (a bucket-grid search in the library) returns the node a scan of all
    nodes returns: random points inside and far outside the mesh, points on nodes, and
    midpoints of node pairs (equal distances go to the lowest id)."""
    wl = workloads.workload(name, **kw)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1)
    xy = s.node_coords()
    lo, hi = xy.min(0), xy.max(0)
    rng = np.random.default_rng(5)
    pts = [rng.uniform(lo, hi, size=(600, 2)),
           rng.uniform(lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo), size=(200, 2)),
           xy[rng.choice(len(xy), 100, replace=False)]]
    a, b = rng.choice(len(xy), 100), rng.choice(len(xy), 100)
    pts.append(0.5 * (xy[a] + xy[b]))
    near = rng.choice(len(xy), 100)
    pts.append(0.5 * (xy[near] + xy[np.argsort(np.abs(xy[:, 0] - xy[near[0], 0]))[1]]))
    pts = np.concatenate(pts)
    np.testing.assert_array_equal(s.set_receivers(pts), solver.snap_to_nodes(pts, xy))
    np.testing.assert_array_equal(s.set_sources(pts[:300], np.zeros(300, np.int32), 10.0),
                                  solver.snap_to_nodes(pts[:300], xy))
    s.close()


def test_tiling_covers_every_node_once(semlib):
    wl = workloads.workload("layered1024", n=40)
    for te in (16, 50, 128):
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, tile_elems=te)
        inf = s.info()
        assert inf["n_tiles"] == -(-wl.n_elements // te)
        assert inf["max_owned_nodes"] >= wl.n_nodes / inf["n_tiles"]


def test_original_node_order_is_identity(semlib):
    wl = workloads.workload("homog64", n=8)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, node_order="original")
    _, n = s.permutations()
    np.testing.assert_array_equal(n, np.arange(s.n_nodes))


def _err(semlib, fn):
    with pytest.raises(semlib.SemError) as ei:
        fn()
    return ei.value.status


def test_error_paths(semlib):
    vxy = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1], [2, 1]], dtype=np.float64)
    good = np.array([[0, 1, 4, 3], [1, 2, 5, 4]])
    c2 = np.ones(2)
    S = semlib.Simulator
    assert _err(semlib, lambda: S(vxy, np.array([[0, 1, 4, 3], [1, 4, 5, 2]]), c2, 2, device=-1)) == "BAD_MESH"
    assert _err(semlib, lambda: S(vxy, np.array([[0, 3, 4, 1], [1, 2, 5, 4]]), c2, 2, device=-1)) == "BAD_MESH"
    assert _err(semlib, lambda: S(vxy, good[:1], c2[:1], 2, device=-1)) == "BAD_MESH"
    assert _err(semlib, lambda: S(vxy, np.array([[0, 1, 4, 9], [1, 2, 5, 4]]), c2, 2, device=-1)) == "BAD_MESH"
    assert _err(semlib, lambda: S(vxy, good, c2, 0, device=-1)) == "INVALID_ARG"
    assert _err(semlib, lambda: S(vxy, good, c2, 9, device=-1)) == "INVALID_ARG"
    assert _err(semlib, lambda: S(vxy, good, np.array([1.0, -1.0]), 2, device=-1)) == "INVALID_ARG"
    assert _err(semlib, lambda: S(vxy, good, c2, 2, device=-1, n_shots=0)) == "INVALID_ARG"
    assert _err(semlib, lambda: S(vxy, good, c2, 2, device=-1, n_shots=6, shot_lanes=4)) == "INVALID_ARG"
    assert _err(semlib, lambda: S(vxy, good, c2, 2, device=0, node_order="original", stream=0)) == "INVALID_ARG"
    s = S(vxy, good, c2, 2, device=-1)
    assert _err(semlib, lambda: s.step()) == "NO_DEVICE"
    assert _err(semlib, lambda: s.reset()) == "NO_DEVICE"
    assert _err(semlib, lambda: s.set_sources([[0.5, 0.5]], [1], 10.0)) == "INVALID_ARG"
    assert _err(semlib, lambda: s.set_sources([[0.5, 0.5]], [0], -1.0)) == "INVALID_ARG"
    with pytest.raises(semlib.SemError):
        semlib.hilbert_index(4, 4, [4], [0])


def test_autotune_needs_device(semlib):
    wl = workloads.workload("homog64", n=8)
    with pytest.raises(semlib.SemError) as ei:
        semlib.autotune(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, stream=0)
    assert ei.value.status == "NO_DEVICE"


@pytest.mark.parametrize("kind", ["connectivity", "distance"])
def test_walk_orders_on_hand_worked_strip(semlib, kind):
    """The library's node-walk element orders on the scrambled 3x1 strip worked by hand."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "walk_orders_strip3.json")))
    vxy, quads = np.array(g["vxy"], float), np.array(g["quads"], np.int32)
    s = semlib.Simulator(vxy, quads, np.full(3, 1.0), 2, order=kind, device=-1)
    e, _ = s.permutations()
    s.close()
    np.testing.assert_array_equal(e, g[kind]["elements"])



@pytest.mark.parametrize("prec,w", [("f32", 4), ("f64", 8)])
def test_algorithmic_bytes_model(semlib, prec, w):
    """The roofline numerator, from mesh counts alone: leapfrog per element nq int32 ids,
    3 nq factors and c2, per node dt/M and u, v read and written per shot; the fused Heun
    step per element ids, the 8-word record, V^n read and V^{n+1} written, per node 5 words."""
    wl = workloads.workload("layered1024", n=12)
    nq = (wl.p + 1) ** 2
    for shots in (1, 64):
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, precision=prec, n_shots=shots)
        inf = s.info()
        E, N = inf["n_elements"], inf["n_nodes"]
        assert inf["alg_bytes_per_step"] == E * (4 * nq + (3 * nq + 1) * w) + N * w * (1 + 4 * shots)
        s.close()
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, precision=prec, formulation="heun")
    inf = s.info()
    E, N = inf["n_elements"], inf["n_nodes"]
    assert inf["alg_bytes_per_step"] == E * (4 * nq + 8 * w + 4 * nq * w) + N * 5 * w
    s.close()


@pytest.mark.parametrize("name,kw,orders", [
    ("layered1024", dict(n=20), ("hilbert", "morton", "lex", "random", "connectivity")),
    ("graded1414", dict(n=16, p=5), ("hilbert", "random")),
    ("homog64", dict(n=12, p=2), ("hilbert", "distance"))])
def test_colours_bit_exact(semlib, name, kw, orders):
    """The library's greedy element colouring (Sec. 5) equals the oracle's first-fit
    colouring visited in the same element order, element by element."""
    from oracle import colour
    wl = workloads.workload(name, **kw)
    conn, _ = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    for kind in orders:
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, order=kind, device=-1, seed=3)
        e, _ = s.permutations()
        want = colour.greedy_colours(conn, e)
        got = s.colours()
        np.testing.assert_array_equal(got, want, err_msg=kind)
        assert s.info()["n_colours"] == int(want.max()) + 1
        s.close()


def test_scatter_options(semlib):
    """The scatter option: AUTO resolves to the owner-tile LDS scatter; COLOUR is single-shot
    leapfrog only, ATOMIC single shot or 64-shot lanes; unknown values are refused."""
    wl = workloads.workload("layered1024", n=12)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1)
    assert s.info()["scatter"] == semlib.SCATTERS["lds_atomic"]
    s.close()
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, scatter="colour")
    assert s.info()["scatter"] == semlib.SCATTERS["colour"]
    s.close()
    for kw in (dict(scatter="colour", n_shots=2), dict(scatter="atomic", formulation="heun"),
               dict(scatter="colour", n_shots=64), dict(scatter="atomic", n_shots=8)):
        with pytest.raises(semlib.SemError) as ei:
            semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, **kw)
        assert ei.value.status == "INVALID_ARG"
    semlib.SCATTERS["bogus"] = 7
    try:
        with pytest.raises(semlib.SemError):
            semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, device=-1, scatter="bogus")
    finally:
        del semlib.SCATTERS["bogus"]


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_triangle_setup_matches_oracle(semlib, p):
    """Triangles (the paper's element, Sec. 4.2): node count, original numbering through the
    node coordinates, and the element and node permutations of every order bit-exact against
    the oracle; the colours are the oracle's first-fit colours."""
    from oracle import colour, triangle
    wl = workloads.workload("tri2000", n=14, p=p)
    conn, nn = triangle.global_numbering(wl.quads, wl.vxy.shape[0], p)
    xy_o = triangle.node_coordinates(wl.vxy, wl.quads, conn, p)
    for kind in ("hilbert", "morton", "lex", "random", "connectivity", "distance"):
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, p, order=kind, device=-1, seed=3)
        assert s.n_nodes == nn
        assert s.info()["vertices_per_element"] == 3
        np.testing.assert_allclose(s.node_coords(), xy_o, rtol=0, atol=1e-12)
        e, n = s.permutations()
        oe, on = reorder.reorder(kind, wl.vxy, wl.quads, conn, seed=3)
        np.testing.assert_array_equal(e, oe, err_msg=kind)
        np.testing.assert_array_equal(n, on, err_msg=kind)
        np.testing.assert_array_equal(s.colours(), colour.greedy_colours(conn, e), err_msg=kind)
        s.close()


@pytest.mark.parametrize("prec,threads,cap", [("f32", 512, 3968), ("f64", 512, 2368), ("f32", 256, 1536),
                                              ("f64", 256, 1152)])
def test_triangle_tiles_fit_the_lds_of_resident_workgroups(semlib, prec, threads, cap):
    """Default triangle tiles: about 240 own + halo elements in whole workgroup passes, and
    no tile owns more nodes than lets the workgroups the registers allow on a CU share its
    160 KB of LDS (stage of the element values, FP64 accumulator and three prefetch arrays
    per owned node)."""
    wl = workloads.workload("tri2000", n=120, p=5)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, 5, precision=prec, block_threads=threads, device=-1)
    inf = s.info()
    epb = (64 // 21) * (threads // 64)
    assert inf["tile_items"] == max(1, (240 + epb // 2) // epb) * epb
    assert 0 < inf["max_owned_nodes"] <= cap
    word = 8 if prec == "f64" else 4
    per_cu = max(1, (16 if prec == "f64" else 20) // (threads // 64))
    lds = epb * 24 * word + ((inf["max_owned_nodes"] + 63) // 64 * 64) * (8 + 3 * word)
    assert lds * per_cu <= 160 * 1024
    s.close()


def test_triangle_options_refused(semlib):
    wl = workloads.workload("tri2000", n=6)
    for kw in (dict(p=4), dict(p=5, formulation="heun"), dict(p=5, scatter="colour")):
        p = kw.pop("p")
        with pytest.raises(semlib.SemError) as ei:
            semlib.Simulator(wl.vxy, wl.quads, wl.c2, p, device=-1, **kw)
        assert ei.value.status in ("INVALID_ARG", "BAD_MESH"), kw
    cw = wl.quads[:, ::-1].copy()                       # clockwise triangles
    with pytest.raises(semlib.SemError) as ei:
        semlib.Simulator(wl.vxy, cw, wl.c2, 5, device=-1)
    assert ei.value.status == "BAD_MESH"


def test_border_split_of_64_shot_tiles(semlib):
    """64 shot lanes with the atomic scatter: no halos; each tile's owned range lists the
    nodes of two or more of its own elements, then its border nodes (touched by another
    tile), then single-element nodes; the border nodes are exactly the nodes whose incident
    elements lie in two or more tiles."""
    wl = workloads.workload("batch512", n=20, n_shots=64)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, n_shots=64, scatter="atomic", device=-1,
                         lds_bytes=16384)
    inf = s.info()
    assert inf["halo_elements"] == 0 and inf["n_tiles"] > 4
    e, n = s.permutations()
    oe, on = _oracle_perm(wl, "hilbert")
    np.testing.assert_array_equal(e, oe)                  # element order unchanged
    assert sorted(n.tolist()) == list(range(s.n_nodes))
    s.close()
