"""The allocation-free stiffness apply (static per-device scratch) against sem_apply_stiffness
through the C ABI: two calls in a row, the second on a smaller mesh, each <= 1e-13 (FP64)
against the allocating entry point and against the oracle's assembled K; sizes beyond the
scratch are refused."""
import sys

import numpy as np
import pytest

import workloads
from oracle import solver

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_noalloc_apply_matches_allocating_apply(semlib, gpu_ok):
    import torch
    for n, shots in ((40, 2), (12, 1)):            # the second call with a smaller input
        print("case noalloc apply", n, shots, flush=True)
        sys.stdout.flush()
        wl = workloads.workload("layered1024", n=n)
        o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
        s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", n_shots=shots, tile_elems=64)
        x = torch.tensor(workloads.random_field(o.n_nodes, shots, seed=n), device="cuda")
        r_alloc = s.apply_stiffness(x).cpu().numpy()
        r = torch.full_like(x, float("nan"))
        s.apply_stiffness_noalloc(x, r)
        s.synchronize()
        r = r.cpu().numpy()
        assert np.isfinite(r).all()
        assert rel(r, r_alloc) <= 1e-13
        assert rel(r, (o.K @ x.cpu().numpy().T).T) <= 1e-13
        s.close()


def test_noalloc_apply_refuses_oversized(semlib, gpu_ok):
    """FP64 and 2^22 node-shots and more exceed half of the 64 MiB scratch."""
    import torch
    wl = workloads.workload("batch512", n=256, n_shots=4)       # 1.05 M nodes x 4 shots x 8 B
    s = semlib.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision="f64", n_shots=4)
    x = torch.zeros((4, s.n_nodes), dtype=torch.float64, device="cuda")
    with pytest.raises(semlib.SemError) as ei:
        s.apply_stiffness_noalloc(x, torch.empty_like(x))
    assert ei.value.status == "INVALID_ARG"
    s.close()
