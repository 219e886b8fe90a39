"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle cannot step these meshes, so it computes sampled outputs one node at a time
(the rows of K and M around each sampled node, Eqs. R and A-bar) and the tests also check
properties that hold at any size (K 1 = 0, discrete energy of source-free leapfrog).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import mesh, solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sample_nodes(n_nodes, k=3000, seed=17):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(n_nodes, k, replace=False), [0, n_nodes - 1]]))


@pytest.fixture(scope="module")
def layered_full():
    wl = workloads.workload("layered1024")
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    return wl, conn, n


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 3e-6)])
def test_layered1024_apply_and_step_sampled(semlib, gpu_ok, layered_full, prec, tol):
    """1024 x 1024 jittered layered quads, p=4 (16.8 M nodes): stiffness apply and one
    leapfrog step at 3000 sampled nodes, against the oracle's per-node rows."""
    import torch
    wl, conn, n = layered_full
    say("case layered1024 full size", prec)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec)
    assert s.n_nodes == n == 16785409
    nodes = sample_nodes(n)
    x = workloads.random_field(n, 1, seed=3)[0]
    y = workloads.random_field(n, 1, seed=4)[0]
    dt_ = s.torch_dtype
    r = s.apply_stiffness(torch.tensor(x[None, :], dtype=dt_, device="cuda")).cpu().numpy()[0]
    r_o, M_o = solver.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, conn, nodes, x)
    assert rel(r[nodes], r_o) <= tol
    # K 1 = 0 at every node
    r1 = s.apply_stiffness(torch.ones((1, n), dtype=dt_, device="cuda")).cpu().numpy()[0]
    assert np.abs(r1).max() <= 20 * tol * np.abs(r).max()
    # one source-free step from (u, v) = (x, y)
    s.set_field(semlib.FIELD_U, torch.tensor(x[None, :], dtype=dt_, device="cuda"))
    s.set_field(semlib.FIELD_V, torch.tensor(y[None, :], dtype=dt_, device="cuda"))
    s.run(1, record=False)
    u1 = s.get_field(semlib.FIELD_U).cpu().numpy()[0]
    v1 = s.get_field(semlib.FIELD_V).cpu().numpy()[0]
    v_o = y[nodes] - s.dt * r_o / M_o
    u_o = x[nodes] + s.dt * v_o
    assert rel(v1[nodes], v_o) <= tol
    assert rel(u1[nodes], u_o) <= tol
    # sources and receivers snap to the oracle's nearest nodes at this size
    node_xy = mesh.node_coordinates(wl.vxy, wl.quads, conn, wl.p)
    np.testing.assert_array_equal(s.set_sources(wl.src_xy, wl.src_shot, wl.f0),
                                  solver.snap_to_nodes(wl.src_xy, node_xy))
    np.testing.assert_array_equal(s.set_receivers(wl.rec_xy[:8]), solver.snap_to_nodes(wl.rec_xy[:8], node_xy))
    s.close()


def test_layered1024_energy_conserved_fp64(semlib, gpu_ok, layered_full):
    """Source-free leapfrog conserves E = 1/2 v'Mv + 1/2 u^{n+1}'K u^n (K symmetric) at full
    size: 200 FP64 steps from a smooth bump."""
    import torch
    wl, conn, n = layered_full
    say("case layered1024 energy")
    xy = mesh.node_coordinates(wl.vxy, wl.quads, conn, wl.p)
    M = mesh.lumped_mass(wl.vxy, wl.quads, conn, wl.p)
    u0 = np.exp(-((xy[:, 0] - 4000.0) ** 2 + (xy[:, 1] - 6000.0) ** 2) / (2 * 300.0 ** 2))
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64")
    s.set_field(semlib.FIELD_U, torch.tensor(u0[None, :], device="cuda"))

    def energy(u_prev):
        u = s.get_field(semlib.FIELD_U)
        v = s.get_field(semlib.FIELD_V).cpu().numpy()[0]
        ku = s.apply_stiffness(u_prev).cpu().numpy()[0]
        return 0.5 * float(v @ (M * v)) + 0.5 * float(u.cpu().numpy()[0] @ ku)

    up = s.get_field(semlib.FIELD_U)
    s.run(1, record=False)
    e0 = energy(up)
    s.run(198, record=False)
    up = s.get_field(semlib.FIELD_U)
    s.run(1, record=False)
    e1 = energy(up)
    say("energy", e0, e1)
    assert e0 > 0
    assert abs(e1 / e0 - 1.0) <= 1e-11
    s.close()


def test_graded1414_p5_apply_sampled(semlib, gpu_ok):
    """About 2 M graded quads (1:8), p=5 (50 M nodes), FP32: sampled stiffness apply."""
    import torch
    say("case graded1414 full size")
    wl = workloads.workload("graded1414")
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32")
    assert s.n_nodes == n
    nodes = sample_nodes(n, 2000)
    x = workloads.random_field(n, 1, seed=6)[0]
    r = s.apply_stiffness(torch.tensor(x[None, :], dtype=torch.float32, device="cuda")).cpu().numpy()[0]
    r_o, _ = solver.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, conn, nodes, x)
    assert rel(r[nodes], r_o) <= 3e-6
    s.close()


def test_batch512_64_shots_apply_sampled(semlib, gpu_ok):
    """512 x 512 jittered quads, p=4, 64 shots (the batched kernel): sampled apply per shot."""
    import torch
    say("case batch512 full size")
    wl = workloads.workload("batch512")
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=64)
    nodes = sample_nodes(n, 1500)
    x = workloads.random_field(n, 64, seed=8)
    r = s.apply_stiffness(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    r_o, _ = solver.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, conn, nodes, x.T)
    assert rel(r[:, nodes].T, r_o) <= 3e-6
    s.close()


def test_batch512_64_shots_step_sampled(semlib, gpu_ok):
    """512 x 512 jittered quads, p=4, 64 shots, FP32, one leapfrog step with the 64 point
    sources active: sampled nodes and every source node, against the oracle's rows. The
    fields are scaled so that the source term is comparable to the stiffness term."""
    import torch
    say("case batch512 64-shot step")
    wl = workloads.workload("batch512")
    conn, n = mesh.global_numbering(wl.quads, wl.vxy.shape[0], wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=64)
    assert s.info()["shot_lanes"] == 64
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    x = 1e-12 * workloads.random_field(n, 64, seed=10)
    y = 1e-12 * workloads.random_field(n, 64, seed=11)
    s.set_field(semlib.FIELD_U, torch.tensor(x, dtype=torch.float32, device="cuda"))
    s.set_field(semlib.FIELD_V, torch.tensor(y, dtype=torch.float32, device="cuda"))
    s.run(1, record=False)
    u1 = s.get_field(semlib.FIELD_U).cpu().numpy()
    v1 = s.get_field(semlib.FIELD_V).cpu().numpy()
    nodes = np.unique(np.concatenate([sample_nodes(n, 1500), src]))
    r_o, M_o = solver.sampled_rows(wl.vxy, wl.quads, wl.c2, wl.p, conn, nodes, x.T)
    f = np.zeros((nodes.size, 64))
    amp = solver.ricker(0.0, wl.f0, 1.0 / wl.f0)
    for k, sh in zip(src, wl.src_shot):
        f[np.searchsorted(nodes, k), sh] += amp
    v_o = y.T[nodes] + s.dt * (f - r_o) / M_o[:, None]
    u_o = x.T[nodes] + s.dt * v_o
    assert rel(v1[:, nodes].T, v_o) <= 3e-6
    assert rel(u1[:, nodes].T, u_o) <= 3e-6
    # the source nodes alone, where the source term is of the size of the stiffness term
    at = np.searchsorted(nodes, src)
    dv_src = s.dt * amp / M_o[at]
    assert np.max(np.abs(dv_src)) > 0.5 * np.max(np.abs(v_o[at, wl.src_shot] - y.T[src, wl.src_shot]))
    assert rel(v1[wl.src_shot, src], v_o[at, wl.src_shot]) <= 3e-6
    s.close()
