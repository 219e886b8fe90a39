"""GPU parity of the paper's triangle element (Sec. 4.2: Blyth-Pozrikidis nodes, nodal basis,
nodes as quadrature points) through the C ABI against the FP64 triangle oracle.

Tolerances: FP64 rel L2 <= 1e-12; FP32 after 1000 steps <= 1e-5; gradient FP64 <= 1e-10
against the oracle's discrete adjoint. At full size (the 250k-triangle, p = 5 workload of
the paper's single-layer benchmark shape) the oracle computes sampled rows of K u one node
at a time.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import adjoint, solver, triangle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _small(n=12, p=5, nsteps=300):
    wl = workloads.workload("tri2000", n=n, p=p, nsteps=nsteps)
    wl.src_xy = np.array([[900.0, 800.0]])
    return wl


def _run_both(semlib, wl, precision, order, **kw):
    o = triangle.TriSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = o.dt_default()
    src = solver.snap_to_nodes(wl.src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    tr_o, u_o, v_o = o.run(wl.nsteps, dt, src, wl.src_shot, wl.f0, rec_nodes=rec)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=precision, order=order, dt=dt, **kw)
    assert s.info()["vertices_per_element"] == 3
    np.testing.assert_array_equal(s.set_sources(wl.src_xy, wl.src_shot, wl.f0), src)
    np.testing.assert_array_equal(s.set_receivers(wl.rec_xy), rec)
    tr = s.run(wl.nsteps).double().cpu().numpy()
    u = s.get_field(semlib.FIELD_U).double().cpu().numpy()[0]
    v = s.get_field(semlib.FIELD_V).double().cpu().numpy()[0]
    s.close()
    return (tr, u, v), (tr_o, u_o[:, 0], v_o[:, 0])


@pytest.mark.parametrize("p", [1, 3, 5, 7])
@pytest.mark.parametrize("order", ["hilbert", "random"])
def test_fp64_triangles(semlib, gpu_ok, p, order):
    """Jittered 12 x 6 cells (144 triangles), tiles of 20 elements (ragged, halos), source,
    receivers, 300 steps, FP64: wavefield, velocity and traces <= 1e-12."""
    say("case triangles fp64", p, order)
    wl = _small(p=p)
    (tr, u, v), (tr_o, u_o, v_o) = _run_both(semlib, wl, "f64", order, tile_elems=20)
    assert np.abs(u_o).max() > 0
    say(f"triangles p={p} {order}: u {rel(u, u_o):.3e} v {rel(v, v_o):.3e} traces {rel(tr, tr_o):.3e}")
    assert rel(u, u_o) <= 1e-12 and rel(v, v_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12


def test_fp32_triangles_1000_steps(semlib, gpu_ok):
    """p = 5 (21 nodes), 64 x 32 cells (4096 triangles), FP32, 1000 steps, default tiles."""
    say("case triangles fp32 1000 steps")
    wl = _small(n=64, p=5, nsteps=1000)
    (tr, u, v), (tr_o, u_o, v_o) = _run_both(semlib, wl, "f32", "hilbert")
    eu, ev = rel(u, u_o), rel(v, v_o)
    say(f"triangles p=5 fp32 1000 steps: u {eu:.3e} v {ev:.3e} traces {rel(tr, tr_o):.3e}")
    assert eu <= 1e-5 and ev <= 1e-5


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_apply_stiffness_triangles(semlib, gpu_ok, prec, tol):
    import torch
    wl = _small(n=20, p=5)
    o = triangle.TriSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec, n_shots=2)
    x = workloads.random_field(o.n_nodes, 2, seed=6)
    r = s.apply_stiffness(torch.tensor(x, dtype=s.torch_dtype, device="cuda")).double().cpu().numpy()
    assert rel(r, (o.K @ x.T).T) <= tol
    s.close()


def test_default_dt_and_stability(semlib, gpu_ok):
    """The default triangle time step is 0.6 of the estimated leapfrog limit, close to the
    oracle's converged estimate."""
    wl = _small(n=16, p=5)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64")
    inf = s.info()
    assert inf["dt"] == pytest.approx(0.6 * inf["dt_stable"], rel=1e-12)
    o = triangle.TriSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    assert inf["lambda_max"] == pytest.approx(o.lambda_max(), rel=3e-2)
    s.close()


def test_adjoint_gradient_triangles(semlib, gpu_ok):
    """Gradient of the receiver misfit with respect to c^2 per triangle (2 shots, p = 3)
    against the oracle's discrete adjoint: <= 1e-10."""
    import torch
    say("case adjoint triangles")
    vxy, tris, _, yc = workloads.tri_mesh(8, 8, 800.0, 800.0, jitter=0.2, seed=9)
    c = workloads.layered_c(yc, 800.0, c_top=1500.0, c_step=300.0)
    rng = np.random.default_rng(21)
    c2_true = (c * (1 + 0.1 * rng.uniform(-1, 1, c.size))) ** 2
    p, nsteps, f0 = 3, 120, 30.0
    o = triangle.TriSEM(vxy, tris, c2_true, p)
    dt = o.dt_default()
    src_xy = np.array([[200.0, 600.0], [560.0, 400.0]])
    rec_xy = np.stack([np.linspace(50, 750, 9), np.full(9, 800.0)], 1)
    src = solver.snap_to_nodes(src_xy, o.node_xy)
    rec = solver.snap_to_nodes(rec_xy, o.node_xy)
    obs, _, _ = o.run(nsteps, dt, src, np.arange(2), f0, rec_nodes=rec, n_shots=2)
    o.set_c2(c * c)
    J, g_o = adjoint.misfit_and_gradient(o, nsteps, dt, src, np.arange(2), f0, rec, 2, obs)
    s = semlib.Simulator(vxy, tris, c * c, p, precision="f64", n_shots=2, dt=dt, tile_elems=24)
    s.set_sources(src_xy, np.arange(2), f0)
    s.set_receivers(rec_xy)
    tr = s.run(nsteps)
    res = (tr - torch.tensor(obs, device="cuda")).contiguous()
    assert 0.5 * float((res ** 2).sum()) == pytest.approx(J, rel=1e-11)
    g = s.adjoint_gradient(res, nsteps, 30).cpu().numpy()
    s.close()
    assert rel(g, g_o) <= 1e-10


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 3e-6)])
def test_tri2000_full_size_sampled(semlib, gpu_ok, prec, tol):
    """The full single-layer triangle workload (500 x 250 cells, 250k triangles, p = 5,
    3.1 M nodes) in the launch configuration of the benchmark: K u at 2000 sampled nodes
    against the oracle's per-node rows, and K 1 = 0 everywhere."""
    import torch
    say("case tri2000 full size", prec)
    wl = workloads.workload("tri2000")
    conn, n = triangle.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec)
    assert s.n_nodes == n and s.n_elements == 250000
    x = workloads.random_field(n, 1, seed=3)[0]
    r = s.apply_stiffness(torch.tensor(x[None, :], dtype=s.torch_dtype, device="cuda")).double().cpu().numpy()[0]
    nodes = np.unique(np.r_[0, n - 1, np.random.default_rng(17).choice(n, 2000, replace=False)])
    r_o, _ = triangle.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, conn, nodes, x)
    assert rel(r[nodes], r_o) <= tol
    r1 = s.apply_stiffness(torch.ones((1, n), dtype=s.torch_dtype, device="cuda")).double().cpu().numpy()[0]
    assert np.abs(r1).max() <= 20 * tol * np.abs(r).max()
    s.close()
