"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 paths rel L2 <= 1e-12 (rounding order only); FP32 after 1000 steps
rel L2 <= 1e-5; gradients vs central finite differences <= 1e-4.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import adjoint, mesh, solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_both(semlib, wl, nsteps, precision="f64", order="hilbert", **kw):
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = o.dt_cfl()
    src = solver.snap_to_nodes(wl.src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    tr_o, u_o, v_o = o.run(nsteps, dt, src, wl.src_shot, wl.f0, rec_nodes=rec, n_shots=wl.n_shots)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=precision, order=order,
                         n_shots=wl.n_shots, dt=dt, **kw)
    gsrc = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    grec = s.set_receivers(wl.rec_xy)
    np.testing.assert_array_equal(gsrc, src)
    np.testing.assert_array_equal(grec, rec)
    tr = s.run(nsteps)
    u = s.get_field(semlib.FIELD_U)
    v = s.get_field(semlib.FIELD_V)
    s.synchronize()
    out = (tr.cpu().numpy(), u.cpu().numpy().T, v.cpu().numpy().T)
    s.close()
    return out, (tr_o, u_o, v_o)


@pytest.mark.parametrize("order", ["hilbert", "lex", "random"])
def test_fp64_homog64_full_size(semlib, gpu_ok, order):
    """64 x 64 uniform quads, p=4, c=1500, Ricker 10 Hz at the centre, 200 steps, FP64."""
    say("case homog64 fp64", order)
    wl = workloads.workload("homog64")
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", order)
    assert np.abs(u_o).max() > 0
    assert rel(u, u_o) <= 1e-12
    assert rel(v, v_o) <= 1e-12
    assert np.abs(tr - tr_o).max() <= 1e-12 * np.abs(u_o).max()


@pytest.mark.parametrize("order", ["hilbert", "morton", "lex", "random", "connectivity", "distance"])
def test_fp64_layered_ragged_tiles(semlib, gpu_ok, order):
    """30 x 30 jittered layered mesh with 64-element tiles: 15 tiles, a ragged last tile,
    halos across tile borders; source close enough that receivers see the wave."""
    say("case layered30 fp64", order)
    wl = workloads.workload("layered1024", n=30, nsteps=400)
    wl.src_xy = np.array([[5000.0, 8000.0]])
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", order, tile_elems=64)
    assert rel(u, u_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12


@pytest.mark.parametrize("lanes", [1, 2, 8])
def test_fp64_batched_shots(semlib, gpu_ok, lanes):
    """8 shots at seeded positions advanced together, shots-per-element lanes 1/2/8."""
    say("case batch fp64 lanes", lanes)
    wl = workloads.workload("batch512", n=24, n_shots=8, nsteps=300)
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", "hilbert",
                                            shot_lanes=lanes, tile_elems=48)
    assert rel(u, u_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12


@pytest.mark.parametrize("shots,block,lds", [(64, 0, 0), (64, 256, 32768), (128, 1024, 49152)])
def test_fp64_64_shot_lanes(semlib, gpu_ok, shots, block, lds):
    """One wave per element with one shot per lane: 64 or 128 shots at seeded positions,
    FP64, default and small LDS budgets (many tiles, ragged last tile, halos)."""
    say("case 64-lane shots fp64", shots, block, lds)
    wl = workloads.workload("batch512", n=24, n_shots=shots, nsteps=300)
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", "hilbert",
                                            block_threads=block, lds_bytes=lds)
    assert rel(u, u_o) <= 1e-12
    assert rel(v, v_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12


@pytest.mark.parametrize("shots,block,lds", [(64, 0, 0), (64, 256, 32768), (128, 1024, 49152)])
def test_fp64_64_shot_lanes_atomic_border(semlib, gpu_ok, shots, block, lds):
    """64 shot lanes with the atomic scatter: tiles process their own elements only, border
    nodes sum through global atomics on their 64-shot rows of v and take u in a border pass.
    FP64 against the oracle, sources and receivers (some on border nodes)."""
    say("case 64-lane shots fp64 atomic border", shots, block, lds)
    wl = workloads.workload("batch512", n=24, n_shots=shots, nsteps=300)
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", "hilbert",
                                            block_threads=block, lds_bytes=lds, scatter="atomic")
    assert rel(u, u_o) <= 1e-12
    assert rel(v, v_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", n_shots=shots, scatter="atomic",
                         block_threads=block, lds_bytes=lds)
    inf = s.info()
    assert inf["scatter"] == semlib.SCATTERS["atomic"] and inf["halo_elements"] == 0
    s.close()


def test_apply_stiffness_fp32_64_shots_atomic_border(semlib, gpu_ok):
    import torch
    wl = workloads.workload("layered1024", n=40)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=64, scatter="atomic")
    x = workloads.random_field(o.n_nodes, 64, seed=9)
    r = s.apply_stiffness(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert rel(r, (o.K @ x.T).T) <= 2e-6
    s.close()


def test_64_shot_lanes_selected(semlib, gpu_ok):
    wl = workloads.workload("batch512", n=16, n_shots=64)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=64)
    inf = s.info()
    assert inf["shot_lanes"] == 64 and inf["block_threads"] == 512
    assert inf["max_accum_nodes"] * 64 * 8 <= 64 * 1024 < inf["max_owned_nodes"] * 64 * 8
    s.close()


def test_apply_stiffness_fp32_64_shots(semlib, gpu_ok):
    import torch
    say("case apply fp32 64 shots")
    wl = workloads.workload("layered1024", n=40)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=64)
    x = workloads.random_field(o.n_nodes, 64, seed=9)
    r = s.apply_stiffness(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    r_o = (o.K @ x.T).T
    assert rel(r, r_o) <= 2e-6


@pytest.mark.parametrize("scatter", ["auto", "colour", "atomic"])
def test_fp32_1000_steps(semlib, gpu_ok, scatter):
    """FP32 state and arithmetic against the FP64 oracle after 1000 steps, with each way of
    summing the element contributions (owner-tile LDS, colour passes, global atomics)."""
    say("case layered64 fp32 1000 steps", scatter)
    wl = workloads.workload("layered1024", n=64, nsteps=1000)
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f32", "hilbert", scatter=scatter)
    err = rel(u, u_o)
    say("fp32 rel L2 after 1000 steps", scatter, err)
    assert err <= 1e-5


@pytest.mark.parametrize("scatter", ["colour", "atomic"])
@pytest.mark.parametrize("order", ["hilbert", "random", "lex"])
def test_fp64_global_scatter(semlib, gpu_ok, scatter, order):
    """The paper's colour passes (Sec. 5, Alg. 2) and the global-atomic scatter, FP64, 30 x 30
    jittered layered mesh, source and receivers, 400 steps: <= 1e-12 against the oracle."""
    say("case layered30 fp64 scatter", scatter, order)
    wl = workloads.workload("layered1024", n=30, nsteps=400)
    wl.src_xy = np.array([[5000.0, 8000.0]])
    (tr, u, v), (tr_o, u_o, v_o) = run_both(semlib, wl, wl.nsteps, "f64", order, scatter=scatter)
    assert rel(u, u_o) <= 1e-12
    assert rel(v, v_o) <= 1e-12
    assert rel(tr, tr_o) <= 1e-12
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", order=order, scatter=scatter)
    inf = s.info()
    assert inf["scatter"] == semlib.SCATTERS[scatter] and inf["n_colours"] >= 4
    s.close()


@pytest.mark.parametrize("scatter", ["colour", "atomic"])
def test_apply_stiffness_fp64_global_scatter(semlib, gpu_ok, scatter):
    import torch
    say("case apply fp64", scatter)
    wl = workloads.workload("layered1024", n=40)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", scatter=scatter)
    x = workloads.random_field(o.n_nodes, 1, seed=3)
    r = s.apply_stiffness(torch.tensor(x, device="cuda")).cpu().numpy()
    assert rel(r, (o.K @ x.T).T) <= 1e-13
    s.close()


def test_apply_stiffness_fp64(semlib, gpu_ok):
    import torch
    say("case apply fp64")
    wl = workloads.workload("layered1024", n=40)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", n_shots=2, tile_elems=100)
    x = workloads.random_field(o.n_nodes, 2, seed=3)
    r = s.apply_stiffness(torch.tensor(x, device="cuda")).cpu().numpy()
    r_o = (o.K @ x.T).T
    assert rel(r, r_o) <= 1e-13


def test_apply_stiffness_fp32(semlib, gpu_ok):
    """FP32 stiffness apply against the FP64 oracle: rounding-level agreement."""
    import torch
    say("case apply fp32")
    wl = workloads.workload("layered1024", n=48)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32")
    x = workloads.random_field(o.n_nodes, 1, seed=5)
    r = s.apply_stiffness(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    r_o = (o.K @ x.T).T
    assert rel(r, r_o) <= 2e-6


def test_resume_from_saved_fields(semlib, gpu_ok):
    """run(200) == run(100) + save (u, v) + restore into a fresh context + run(100)."""
    import torch
    say("case resume")
    wl = workloads.workload("layered1024", n=20)
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    u0 = np.exp(-((o.node_xy[:, 0] - 4000) ** 2 + (o.node_xy[:, 1] - 6000) ** 2) / 2e6)[None, :]
    a = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64")
    a.set_field(semlib.FIELD_U, torch.tensor(u0, device="cuda"))
    a.run(100, record=False)
    su, sv = a.get_field(semlib.FIELD_U), a.get_field(semlib.FIELD_V)
    a.run(100, record=False)
    ua = a.get_field(semlib.FIELD_U).cpu().numpy()
    b = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64")
    b.set_field(semlib.FIELD_U, su)
    b.set_field(semlib.FIELD_V, sv)
    b.run(100, record=False)
    ub = b.get_field(semlib.FIELD_U).cpu().numpy()
    assert rel(ub, ua) <= 1e-14
    _, u_o, _ = o.run(200, a.dt, u0=u0.T)
    assert rel(ua, u_o.T) <= 1e-12


def _tiny_inversion(semlib, precision, shots=2, nsteps=80, n=8, p=3, **kw):
    vxy, quads, xc, yc = workloads.grid_mesh(n, n, 800.0, 800.0, jitter=0.2, seed=9)
    c = workloads.layered_c(yc, 800.0, c_top=1500.0, c_step=300.0)
    rng = np.random.default_rng(21)
    c2_true = (c * (1 + 0.1 * rng.uniform(-1, 1, c.size))) ** 2
    c2 = c * c
    o = solver.SEM(vxy, quads, c2_true, p)
    dt = o.dt_cfl()
    src_xy = np.array([[200.0, 600.0], [560.0, 400.0]])[:shots] if shots <= 2 else \
        np.random.default_rng(22).uniform(0.0, 800.0, size=(shots, 2))
    rec_xy = np.stack([np.linspace(50, 750, 9), np.full(9, 800.0)], 1)
    src = solver.snap_to_nodes(src_xy, o.node_xy)
    rec = solver.snap_to_nodes(rec_xy, o.node_xy)
    f0 = 30.0
    obs, _, _ = o.run(nsteps, dt, src, np.arange(shots), f0, rec_nodes=rec, n_shots=shots)
    o.set_c2(c2)
    J, g_o = adjoint.misfit_and_gradient(o, nsteps, dt, src, np.arange(shots), f0, rec, shots, obs)
    kw = kw or dict(tile_elems=16)
    s = semlib.Simulator(vxy, quads, c2, p, precision=precision, n_shots=shots, dt=dt, **kw)
    s.set_sources(src_xy, np.arange(shots), f0)
    s.set_receivers(rec_xy)
    return o, s, dict(dt=dt, src=src, rec=rec, f0=f0, obs=obs, J=J, g=g_o, c2=c2, nsteps=nsteps,
                      shots=shots)


@pytest.mark.parametrize("ckpt", [7, 80, 200])
def test_adjoint_gradient_fp64_matches_oracle(semlib, gpu_ok, ckpt):
    import torch
    say("case adjoint fp64 ckpt", ckpt)
    o, s, d = _tiny_inversion(semlib, "f64")
    tr = s.run(d["nsteps"])
    res = tr - torch.tensor(d["obs"], device="cuda")
    J = 0.5 * float((res.double() ** 2).sum())
    assert J == pytest.approx(d["J"], rel=1e-11)
    g = s.adjoint_gradient(res.contiguous(), d["nsteps"], ckpt).cpu().numpy()
    assert rel(g, d["g"]) <= 1e-10


@pytest.mark.parametrize("scatter", ["colour", "atomic"])
def test_adjoint_gradient_fp64_global_scatter(semlib, gpu_ok, scatter):
    """Gradient pairing inside the element launches of the colour and atomic scatters."""
    import torch
    say("case adjoint fp64", scatter)
    o, s, d = _tiny_inversion(semlib, "f64", shots=1, scatter=scatter)
    tr = s.run(d["nsteps"])
    res = tr - torch.tensor(d["obs"], device="cuda")
    g = s.adjoint_gradient(res.contiguous(), d["nsteps"], 30).cpu().numpy()
    assert rel(g, d["g"]) <= 1e-10


def test_colour_scatter_is_bitwise_reproducible(semlib, gpu_ok):
    """The paper's colour passes add each node's contributions one colour class after another,
    at most one per class, so a rerun (and the adjoint's recomputation of the forward from its
    checkpoints) reproduces every bit: FP64, 80 steps, traces, wavefield and the gradient
    equal to the last bit on a second run."""
    import torch
    say("case colour bitwise")
    o, s, d = _tiny_inversion(semlib, "f64", shots=1, scatter="colour")
    runs = []
    for _ in range(2):
        s.reset()
        tr = s.run(d["nsteps"])
        u = s.get_field(semlib.FIELD_U).cpu().numpy()
        res = (tr - torch.tensor(d["obs"], device="cuda")).contiguous()
        g = s.adjoint_gradient(res, d["nsteps"], 30).cpu().numpy()
        runs.append((tr.cpu().numpy(), u, g))
    s.close()
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert rel(runs[0][2], d["g"]) <= 1e-10


@pytest.mark.parametrize("scatter", ["auto", "atomic"])
def test_adjoint_gradient_fp64_64_shot_lanes(semlib, gpu_ok, scatter):
    """Gradient pairing of the one-wave-per-element kernel: 64 shots, small tiles, with the
    LDS scatter and with the atomic border scatter."""
    import torch
    say("case adjoint fp64 64 shots", scatter)
    o, s, d = _tiny_inversion(semlib, "f64", shots=64, lds_bytes=16384, scatter=scatter)
    assert s.info()["shot_lanes"] == 64
    tr = s.run(d["nsteps"])
    res = tr - torch.tensor(d["obs"], device="cuda")
    g = s.adjoint_gradient(res.contiguous(), d["nsteps"], 30).cpu().numpy()
    assert rel(g, d["g"]) <= 1e-10


def test_adjoint_gradient_fp32_vs_finite_differences(semlib, gpu_ok):
    import torch
    say("case adjoint fp32 vs FD")
    o, s, d = _tiny_inversion(semlib, "f32", nsteps=120)
    tr = s.run(d["nsteps"])
    res = (tr.double() - torch.tensor(d["obs"], device="cuda")).float().contiguous()
    g = s.adjoint_gradient(res, d["nsteps"], 40).cpu().numpy()
    rng = np.random.default_rng(4)
    els = rng.choice(d["c2"].size, 16, replace=False)
    fd = []
    for e in els:
        h = 1e-4 * d["c2"][e]
        Js = []
        for sgn in (1, -1):
            cp = d["c2"].copy()
            cp[e] += sgn * h
            o.set_c2(cp)
            t, _, _ = o.run(d["nsteps"], d["dt"], d["src"], np.arange(d["shots"]), d["f0"],
                            rec_nodes=d["rec"], n_shots=d["shots"])
            Js.append(adjoint.misfit(t, d["obs"]))
        fd.append((Js[0] - Js[1]) / (2 * h))
    err = rel(g[els], fd)
    say("fp32 gradient vs FD rel", err)
    assert err <= 1e-4


def test_unstable_dt_rejected(semlib, gpu_ok):
    wl = workloads.workload("homog64", n=8)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64")
    inf = s.info()
    assert 0 < inf["dt"] < inf["dt_stable"]
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    assert inf["lambda_max"] == pytest.approx(o.lambda_max(400), rel=2e-2)
    with pytest.raises(semlib.SemError) as ei:
        semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", dt=1.5 * inf["dt_stable"])
    assert ei.value.status == "UNSTABLE_DT"


@pytest.mark.parametrize("shots", [1, 64, "tri"])
def test_autotune_picks_a_timed_candidate(semlib, gpu_ok, shots):
    """The autotuner times every candidate, returns the fastest, and a context built with
    its options reproduces the default context's wavefield to rounding."""
    import torch
    say("case autotune", shots)
    if shots == "tri":
        wl = workloads.workload("tri2000", n=40, p=5, nsteps=60)
        wl.src_xy = np.array([[900.0, 800.0]])
        shots = 1
    else:
        wl = workloads.workload("batch512", n=32, n_shots=shots, nsteps=60)
    tri = wl.quads.shape[1] == 3
    best, rows = semlib.autotune(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=shots, steps=10)
    assert len(rows) == (9 if tri else 6 if shots == 1 else 8)
    assert all(r["us_per_step"] > 0 for r in rows)
    assert best["us_per_step"] == min(r["us_per_step"] for r in rows)
    if tri:
        assert {r["tile_items"] for r in rows} == {k * 3 * t // 64 for k in (8, 14, 20) for t in (256, 512, 1024)}
    elif shots == 1:
        assert len({r["tile_items"] for r in rows}) == 4      # 2 tile sizes x 3 workgroup sizes
    kw = {k: best[k] for k in ("block_threads", "lds_bytes", "tile_items")}
    out = []
    for opts in (kw, {}):
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f32", n_shots=shots, **opts)
        s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
        s.run(wl.nsteps, record=False)
        out.append(s.get_field(semlib.FIELD_U).double().cpu().numpy())
        s.close()
    assert np.abs(out[0]).max() > 0
    assert rel(out[0], out[1]) <= 1e-5


@pytest.mark.parametrize("prec,tol,nsteps", [("f64", 1e-12, 200), ("f32", 1e-5, 300)])
def test_heun_first_order_matches_oracle(semlib, gpu_ok, prec, tol, nsteps):
    """The paper's first-order u-v system with Heun (Sec. 4.2.1) against the FP64 oracle:
    layered jittered 20x20 mesh, p=4, 40-element tiles (ragged, halos), source and
    receivers, wavefield and traces."""
    from oracle import first_order
    say("case heun", prec)
    wl = workloads.workload("layered1024", n=20)
    wl.src_xy = np.array([[5000.0, 8000.0]])
    fo = first_order.FirstOrderSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec, formulation="heun",
                         tile_elems=40)
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    rec = s.set_receivers(wl.rec_xy)
    tr_o, u_o, _ = fo.run(nsteps, s.dt, src, wl.src_shot, wl.f0, rec_nodes=rec)
    tr = s.run(nsteps).double().cpu().numpy()
    u = s.get_field(semlib.FIELD_U).double().cpu().numpy()
    with pytest.raises(semlib.SemError):
        s.get_field(semlib.FIELD_V)
    s.close()
    assert np.abs(u_o).max() > 0
    err = rel(u, u_o.T)
    say("heun", prec, "rel L2", err)
    assert err <= tol
    assert rel(tr, tr_o) <= tol


def test_heun_state_changes(semlib, gpu_ok):
    """The Heun path keeps the next step's predicted U between calls; runs split over calls,
    reset, and a field written between runs (which must discard that prediction) all match
    the FP64 oracle."""
    from oracle import first_order
    say("case heun state changes")
    wl = workloads.workload("layered1024", n=12)
    fo = first_order.FirstOrderSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", formulation="heun")
    xy = fo.node_xy                              # original node numbering, as the fields
    u0 = np.exp(-((xy[:, 0] - 5000.0) ** 2 + (xy[:, 1] - 4000.0) ** 2) / (2 * 800.0 ** 2))
    import torch
    dev = torch.device("cuda")
    s.set_field(semlib.FIELD_U, torch.tensor(u0[None, :], dtype=torch.float64, device=dev))
    s.run(20, record=False)
    s.run(30, record=False)                      # split: 50 steps over two calls
    u50 = s.get_field(semlib.FIELD_U).double().cpu().numpy()[0]
    _, u50_o, v50_o = fo.run(50, s.dt, u0=u0)
    assert rel(u50, u50_o[:, 0]) <= 1e-12
    u_new = 2.0 * u50                            # a new field with V kept
    s.set_field(semlib.FIELD_U, torch.tensor(u_new[None, :], dtype=torch.float64, device=dev))
    s.run(40, record=False)
    u90 = s.get_field(semlib.FIELD_U).double().cpu().numpy()[0]
    _, u90_o, _ = fo.run(40, s.dt, u0=u_new, v0=v50_o)
    assert rel(u90, u90_o[:, 0]) <= 1e-12
    s.reset()                                    # zero state, then the same 50 steps again
    s.set_field(semlib.FIELD_U, torch.tensor(u0[None, :], dtype=torch.float64, device=dev))
    s.run(50, record=False)
    assert rel(s.get_field(semlib.FIELD_U).double().cpu().numpy()[0], u50_o[:, 0]) <= 1e-12
    s.close()
