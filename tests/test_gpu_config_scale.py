"""Multi-step parity at the scale of the benchmark workloads, the differentiable forward, and
the inversion workload's gradient at full size.

The FP64 oracle steps meshes of up to about a million nodes in seconds per hundred steps,
so the multi-step comparisons run on reduced versions of the workloads that keep their
structure (jitter, layers, grading, p, shot batch) and their launch configuration (tile
sizes and kernels do not depend on the mesh size):
  * layered jittered 256^2, p=4, FP32, 1000 steps, four element orders;
  * graded 1:8 128^2, p=5, FP32, 1000 steps, three element orders;
  * 64-shot batch 256^2, p=4, FP32, 1000 steps, three of the shots against the oracle;
  * the first-order system with Heun, FP32, 1000 steps.
Tolerance: rel L2 <= 1e-5 after 1000 steps (FP32 state and arithmetic, FP64 LDS sums).

The inversion workload (512^2, 8 shots, 1500 steps, checkpoints every 40) is too large for
the oracle's finite differences; there the FP32 adjoint gradient is compared with central
differences of the FP64 GPU forward, whose parity with the oracle is established by the
FP64 tests (<= 1e-12), on 16 seeded elements: rel L2 <= 1e-4.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import adjoint, first_order, solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_run(wl, nsteps, shots=None):
    """Oracle run of a workload; ``shots`` picks a subset of the sources' shots (renumbered
    0..k-1 in the given order)."""
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = o.dt_cfl()
    src_xy, src_shot, S = wl.src_xy, wl.src_shot, wl.n_shots
    if shots is not None:
        pick = [int(np.flatnonzero(wl.src_shot == s)[0]) for s in shots]
        src_xy, src_shot, S = wl.src_xy[pick], np.arange(len(shots)), len(shots)
    src = solver.snap_to_nodes(src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    tr, u, v = o.run(nsteps, dt, src, src_shot, wl.f0, rec_nodes=rec, n_shots=S)
    return dict(dt=dt, src=src, rec=rec, tr=tr, u=u, v=v)


def _gpu_run(semlib, wl, nsteps, dt, precision, order, **kw):
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=precision, order=order,
                         n_shots=wl.n_shots, dt=dt, **kw)
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    rec = s.set_receivers(wl.rec_xy)
    tr = s.run(nsteps)
    u = s.get_field(semlib.FIELD_U)
    v = s.get_field(semlib.FIELD_V)
    s.synchronize()
    out = dict(src=src, rec=rec, tr=tr.double().cpu().numpy(), u=u.double().cpu().numpy().T,
               v=v.double().cpu().numpy().T, info=s.info())
    s.close()
    return out


@pytest.fixture(scope="module")
def layered256():
    # source 200 m below the top so that the receivers see the wave within 1000 steps
    wl = workloads.workload("layered1024", n=256, nsteps=1000)
    wl.src_xy = np.array([[5000.0, 9800.0]])
    return wl, _oracle_run(wl, wl.nsteps)


@pytest.mark.parametrize("order", ["hilbert", "morton", "lex", "random"])
def test_layered256_fp32_1000_steps(semlib, gpu_ok, layered256, order):
    """Layered jittered mesh (256^2, p=4, 1.05 M nodes), FP32, 1000 steps, each element
    order against the one oracle run (the reorder is a relabelling)."""
    wl, o = layered256
    say("case layered256 fp32 1000 steps", order)
    g = _gpu_run(semlib, wl, wl.nsteps, o["dt"], "f32", order)
    np.testing.assert_array_equal(g["src"], o["src"])
    np.testing.assert_array_equal(g["rec"], o["rec"])
    assert np.abs(o["tr"]).max() > 1e-3 * np.abs(o["u"]).max()     # the wave reached them
    eu, ev, et = rel(g["u"], o["u"]), rel(g["v"], o["v"]), rel(g["tr"], o["tr"])
    say(f"layered256 fp32 {order}: u {eu:.3e} v {ev:.3e} traces {et:.3e}")
    assert eu <= 1e-5 and ev <= 1e-5 and et <= 1e-5


@pytest.fixture(scope="module")
def graded128():
    wl = workloads.workload("graded1414", n=128, nsteps=1000)
    return wl, _oracle_run(wl, wl.nsteps)


@pytest.mark.parametrize("order", ["hilbert", "morton", "random"])
def test_graded128_p5_fp32_1000_steps(semlib, gpu_ok, graded128, order):
    """Graded 1:8 mesh (128^2, p=5, smooth random c), FP32, 1000 steps."""
    wl, o = graded128
    say("case graded128 p5 fp32 1000 steps", order)
    g = _gpu_run(semlib, wl, wl.nsteps, o["dt"], "f32", order)
    assert np.abs(o["u"]).max() > 0
    eu, ev = rel(g["u"], o["u"]), rel(g["v"], o["v"])
    say(f"graded128 p5 fp32 {order}: u {eu:.3e} v {ev:.3e}")
    assert eu <= 1e-5 and ev <= 1e-5


@pytest.fixture(scope="module")
def batch256():
    wl = workloads.workload("batch512", n=256, n_shots=64, nsteps=1000)
    pick = [0, 1, 63]
    return wl, pick, _oracle_run(wl, wl.nsteps, shots=pick)


@pytest.mark.parametrize("scatter", ["auto", "atomic"])
def test_batch256_64_shots_fp32_1000_steps(semlib, gpu_ok, batch256, scatter):
    """64-shot batch (256^2, p=4, one wave per element and one shot per lane), FP32, 1000
    steps, LDS scatter and atomic border scatter; shots 0, 1 and 63 against an oracle run of
    those three sources."""
    say("case batch256 64 shots fp32 1000 steps", scatter)
    wl, pick, o = batch256
    g = _gpu_run(semlib, wl, wl.nsteps, o["dt"], "f32", "hilbert", scatter=scatter)
    assert g["info"]["shot_lanes"] == 64
    for k, s in enumerate(pick):
        assert np.abs(o["u"][:, k]).max() > 0
        eu, ev = rel(g["u"][:, s], o["u"][:, k]), rel(g["v"][:, s], o["v"][:, k])
        et = rel(g["tr"][s], o["tr"][k])
        say(f"batch256 fp32 {scatter} shot {s}: u {eu:.3e} v {ev:.3e} traces {et:.3e}")
        assert eu <= 1e-5 and ev <= 1e-5
        if np.abs(o["tr"][k]).max() > 1e-3 * np.abs(o["u"][:, k]).max():
            assert et <= 1e-5


def test_heun_fp32_1000_steps(semlib, gpu_ok):
    """The first-order system with Heun (Sec. 4.2.1), FP32, 1000 steps on a 48^2 layered
    mesh against the FP64 oracle; the per-step growth factor the library reports stays
    small enough that rounding noise cannot grow to the tolerance within the run."""
    say("case heun fp32 1000 steps")
    wl = workloads.workload("layered1024", n=48)
    wl.src_xy = np.array([[5000.0, 9000.0]])
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", formulation="heun")
    inf = s.info()
    say("heun growth per step", inf["growth_per_step"], "dt/dt_stable", inf["dt"] / inf["dt_stable"])
    assert inf["growth_per_step"] > 1.0
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    rec = s.set_receivers(wl.rec_xy)
    fo = first_order.FirstOrderSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    tr_o, u_o, _ = fo.run(1000, s.dt, src, wl.src_shot, wl.f0, rec_nodes=rec)
    tr = s.run(1000).double().cpu().numpy()
    u = s.get_field(semlib.FIELD_U).double().cpu().numpy()
    s.close()
    err = rel(u, u_o.T)
    say(f"heun fp32 1000 steps: u {err:.3e} traces {rel(tr, tr_o):.3e}")
    assert err <= 1e-5
    assert rel(tr, tr_o) <= 1e-5


def _small_inversion(shots=2, nsteps=80):
    vxy, quads, xc, yc = workloads.grid_mesh(8, 8, 800.0, 800.0, jitter=0.2, seed=9)
    c = workloads.layered_c(yc, 800.0, c_top=1500.0, c_step=300.0)
    rng = np.random.default_rng(21)
    c2_true = (c * (1 + 0.1 * rng.uniform(-1, 1, c.size))) ** 2
    src_xy = np.array([[200.0, 600.0], [560.0, 400.0]])[:shots]
    rec_xy = np.stack([np.linspace(50, 750, 9), np.full(9, 800.0)], 1)
    return vxy, quads, c * c, c2_true, src_xy, rec_xy, 30.0, nsteps


@pytest.mark.parametrize("where", ["cuda", "cpu"])
def test_sem_forward_autograd(semlib, gpu_ok, where):
    """sem_forward (torch.autograd.Function): loss.backward() gives the oracle's adjoint
    gradient, on the device and in the dtype of c2; a second forward on the same
    simulator before backward does not change the first graph's gradient."""
    import torch
    say("case sem_forward", where)
    vxy, quads, c2, c2_true, src_xy, rec_xy, f0, nsteps = _small_inversion()
    p = 3
    o = solver.SEM(vxy, quads, c2_true, p)
    dt = o.dt_cfl()
    src = solver.snap_to_nodes(src_xy, o.node_xy)
    rec = solver.snap_to_nodes(rec_xy, o.node_xy)
    obs, _, _ = o.run(nsteps, dt, src, np.arange(2), f0, rec_nodes=rec, n_shots=2)
    o.set_c2(c2)
    _, g_o = adjoint.misfit_and_gradient(o, nsteps, dt, src, np.arange(2), f0, rec, 2, obs)
    s = semlib.Simulator(vxy, quads, c2, p, precision="f64", n_shots=2, dt=dt, tile_elems=16)
    s.set_sources(src_xy, np.arange(2), f0)
    s.set_receivers(rec_xy)
    m = torch.tensor(c2, dtype=torch.float64, device=where, requires_grad=True)
    tr = semlib.sem_forward(m, s, nsteps, 30)
    obs_t = torch.tensor(obs, device=tr.device)
    loss = 0.5 * ((tr - obs_t) ** 2).sum()
    # another model on the same simulator before the first backward
    m2 = torch.tensor(c2_true, dtype=torch.float64, device=where, requires_grad=True)
    tr2 = semlib.sem_forward(m2, s, nsteps, 30)
    assert rel(tr2.detach().cpu().numpy(), obs) <= 1e-12
    loss.backward()
    assert m.grad is not None and m.grad.device.type == where and m.grad.dtype == torch.float64
    err = rel(m.grad.cpu().numpy(), g_o)
    say(f"sem_forward gradient vs oracle adjoint ({where}): {err:.3e}")
    assert err <= 1e-10
    # and the same value as the C ABI's gradient call
    s.set_c2(c2)
    res = (s.run(nsteps) - obs_t).contiguous()
    g = s.adjoint_gradient(res, nsteps, 30).cpu().numpy()
    assert rel(m.grad.cpu().numpy(), g) <= 1e-12
    # changed receivers between forward and backward are refused
    tr3 = semlib.sem_forward(m, s, nsteps, 30)
    s.set_receivers(rec_xy)
    with pytest.raises(RuntimeError):
        tr3.sum().backward()
    s.close()


def test_inversion512_fp32_gradient_vs_fd(semlib, gpu_ok):
    """Inversion workload at full size: 512^2 jittered layered mesh, p=4, 8 shots x 128
    receivers, 1500 steps, checkpoints every 40. The FP32 adjoint gradient of the misfit at
    the starting model against central differences (relative step 1e-4 of c^2_e) of the
    FP64 GPU forward on 16 seeded elements."""
    import torch
    say("case inversion512 fp32 gradient vs FD")
    wl = workloads.workload("adjoint512")
    N, C = wl.nsteps, wl.ckpt_every
    f64 = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", n_shots=wl.n_shots)
    dt = f64.dt
    f64.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    f64.set_receivers(wl.rec_xy)
    obs = f64.run(N).clone()                      # observed traces: the true model
    f64.set_c2(wl.c2_init)
    s32 = semlib.Simulator(wl.vxy, wl.quads, wl.c2_init, wl.p, precision="f32", n_shots=wl.n_shots,
                           dt=dt)
    s32.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    s32.set_receivers(wl.rec_xy)
    res = (s32.run(N).double() - obs).float().contiguous()
    rnorm = float(res.double().norm() / obs.norm())
    say(f"inversion512 relative residual of the starting model: {rnorm:.3e}")
    assert rnorm > 1e-3                           # the data see the anomaly
    g = s32.adjoint_gradient(res, N, C).cpu().numpy()
    s32.close()
    assert np.isfinite(g).all()
    # 16 seeded elements among those within 300 m of the anomaly (the region the data see)
    cen = wl.vxy[wl.quads].mean(axis=1)
    near = np.flatnonzero(np.linalg.norm(cen - wl.anomaly_xy, axis=1) <= 300.0)
    rng = np.random.default_rng(workloads.SEEDS["fd_elements"])
    els = rng.choice(near, 16, replace=False)
    fd = []
    for e in els:
        h = 1e-4 * wl.c2_init[e]
        tr = []
        for sgn in (1.0, -1.0):
            cp = wl.c2_init.copy()
            cp[e] += sgn * h
            f64.set_c2(cp)
            tr.append(f64.run(N))
        # J+ - J- = 1/2 sum (d+ - d-) (d+ + d- - 2 obs), without forming J
        dJ = 0.5 * float(((tr[0] - tr[1]) * (tr[0] + tr[1] - 2.0 * obs)).sum())
        fd.append(dJ / (2.0 * h))
    f64.close()
    fd = np.array(fd)
    err = rel(g[els], fd)
    say(f"inversion512 fp32 gradient vs FD on 16 elements: rel L2 {err:.3e}, |fd| max {np.abs(fd).max():.3e}")
    assert np.abs(fd).max() > 0
    assert err <= 1e-4
