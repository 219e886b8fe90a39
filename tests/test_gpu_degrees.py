"""GPU parity at every polynomial degree the kernels are built for (p = 1..7), against the
FP64 CPU oracle: the single-shot row kernel, the 64-shot kernel (one wave per element)
and the Heun kernels of the first-order system (predictor, fused corrector). The p = 4
cases are covered at larger sizes elsewhere; here each degree runs on a small mesh in random
element order, so that every tile has a large halo, with a source, receivers and the
default tiles.

Tolerances: FP64 rel L2 <= 1e-12 (rounding order only); FP32 rel L2 <= 1e-5; traces: the
largest error over the largest wavefield value, same bounds.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import first_order, solver

pytestmark = pytest.mark.gpu

DEGREES = [1, 2, 3, 5, 6, 7]
TOL = {"f64": 1e-12, "f32": 1e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _small(name, p, **kw):
    wl = workloads.workload(name, n=8, p=p, **kw)
    if name == "layered1024":
        wl.src_xy = np.array([[5000.0, 8000.0]])      # close to the receivers near the top
    return wl


def _trace_err(tr, tr_o, u_o):
    """Largest trace error on the scale of the wavefield (early traces are near zero)."""
    return float(np.abs(np.asarray(tr) - tr_o).max() / np.abs(u_o).max())


def _leapfrog(semlib, wl, prec, nsteps):
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    dt = o.dt_cfl()
    src = solver.snap_to_nodes(wl.src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    tr_o, u_o, v_o = o.run(nsteps, dt, src, wl.src_shot, wl.f0, rec_nodes=rec, n_shots=wl.n_shots)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec, order="random",
                         n_shots=wl.n_shots, dt=dt)
    s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    s.set_receivers(wl.rec_xy)
    lanes = s.info()["shot_lanes"]
    tr = s.run(nsteps).double().cpu().numpy()
    u = s.get_field(semlib.FIELD_U).double().cpu().numpy().T
    v = s.get_field(semlib.FIELD_V).double().cpu().numpy().T
    s.close()
    assert np.abs(u_o).max() > 0
    return lanes, (rel(u, u_o), rel(v, v_o), _trace_err(tr, tr_o, u_o))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("p", DEGREES)
def test_single_shot_every_degree(semlib, gpu_ok, p, prec):
    say("case single shot degree", p, prec)
    wl = _small("layered1024", p)
    lanes, errs = _leapfrog(semlib, wl, prec, 60)
    say("single shot", p, prec, "rel L2 u, v, traces", errs)
    assert lanes == 1
    assert max(errs) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("p", DEGREES)
def test_64_shots_every_degree(semlib, gpu_ok, p, prec):
    say("case 64 shots degree", p, prec)
    wl = _small("batch512", p, n_shots=64)
    lanes, errs = _leapfrog(semlib, wl, prec, 40)
    say("64 shots", p, prec, "rel L2 u, v, traces", errs)
    assert lanes == 64
    assert max(errs) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("p", DEGREES)
def test_heun_every_degree(semlib, gpu_ok, p, prec):
    say("case heun degree", p, prec)
    wl = _small("layered1024", p)
    fo = first_order.FirstOrderSEM(wl.vxy, wl.quads, wl.c2, wl.p)
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=prec, order="random",
                         formulation="heun")
    src = s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    rec = s.set_receivers(wl.rec_xy)
    tr_o, u_o, _ = fo.run(60, s.dt, src, wl.src_shot, wl.f0, rec_nodes=rec)
    tr = s.run(60).double().cpu().numpy()
    u = s.get_field(semlib.FIELD_U).double().cpu().numpy()
    s.close()
    assert np.abs(u_o).max() > 0
    errs = (rel(u, u_o.T), _trace_err(tr, tr_o, u_o))
    say("heun", p, prec, "rel L2 u, traces", errs)
    assert max(errs) <= TOL[prec]
