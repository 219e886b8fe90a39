"""ctypes binding of the C ABI in ``include/sem.h`` (argument marshalling only).

Every step of the time step runs in the HIP library ``libsem_hip.so``; this module only
converts NumPy/PyTorch arguments to pointers and sizes. PyTorch supplies device memory
(tensor ``data_ptr()``) and the stream (``torch.cuda.current_stream()``). If the built
library is missing, importing this module raises ``ImportError``: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem_hip.so")

F32, F64 = 0, 1
ORDERS = {"hilbert": 0, "morton": 1, "lex": 2, "random": 3, "connectivity": 4, "distance": 5}
NODE_ORDERS = {"first_touch": 0, "original": 1}
FORMULATIONS = {"leapfrog": 0, "heun": 1}
SCATTERS = {"auto": 0, "lds_atomic": 1, "colour": 2, "atomic": 3}
FIELD_U, FIELD_V = 0, 1
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BAD_MESH", -3: "UNSTABLE_DT", -4: "HIP_ERROR",
          -5: "OOM", -6: "NO_DEVICE"}


class SemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("vxy", ctypes.c_void_p),
                ("n_elements", ctypes.c_int64), ("quad", ctypes.c_void_p), ("c2", ctypes.c_void_p),
                ("vertices_per_element", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("precision", ctypes.c_int32), ("elem_order", ctypes.c_int32),
                ("node_order", ctypes.c_int32), ("seed", ctypes.c_uint64), ("n_shots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("tile_elems", ctypes.c_int32), ("shot_lanes", ctypes.c_int32),
                ("tile_items", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("formulation", ctypes.c_int32),
                ("scatter", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("p", ctypes.c_int32),
                ("n_shots", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_sources", ctypes.c_int32),
                ("n_receivers", ctypes.c_int32), ("tile_elems", ctypes.c_int32),
                ("shot_lanes", ctypes.c_int32), ("max_owned_nodes", ctypes.c_int32),
                ("tile_items", ctypes.c_int32), ("geometry_on_the_fly", ctypes.c_int32),
                ("block_threads", ctypes.c_int32),
                ("n_tiles", ctypes.c_int64), ("halo_elements", ctypes.c_int64), ("step", ctypes.c_int64),
                ("dt", ctypes.c_double), ("dt_stable", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("alg_bytes_per_step", ctypes.c_double), ("alg_flops_per_step", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("reorder_seconds", ctypes.c_double),
                ("max_accum_nodes", ctypes.c_int32), ("kernel_bytes_per_step", ctypes.c_double),
                ("n_colours", ctypes.c_int32), ("scatter", ctypes.c_int32),
                ("vertices_per_element", ctypes.c_int32), ("growth_per_step", ctypes.c_double)]


EXPORTS = ("sem_create", "sem_create_error", "sem_get_info", "sem_get_permutations",
           "sem_get_node_coords", "sem_set_sources", "sem_set_receivers", "sem_set_c2", "sem_reset",
           "sem_run", "sem_step", "sem_get_field", "sem_set_field", "sem_apply_stiffness",
           "sem_adjoint_gradient", "sem_synchronize", "sem_hilbert_index", "sem_last_error",
           "sem_destroy", "sem_autotune", "sem_get_colours", "sem_apply_stiffness_noalloc")


def _load():
    # PyTorch-ROCm ships its own HIP runtime with the same soname as the system one; load it
    # first so that the library binds to the runtime that owns torch's memory and streams
    # (two HIP runtimes in one process cannot share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2104_08416_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, VP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.sem_create.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Options), ctypes.POINTER(P)]
    lib.sem_create_error.restype = ctypes.c_char_p
    lib.sem_get_info.argtypes = [P, ctypes.POINTER(_Info)]
    lib.sem_get_permutations.argtypes = [P, VP, VP]
    lib.sem_get_node_coords.argtypes = [P, VP]
    lib.sem_get_colours.argtypes = [P, VP]
    lib.sem_set_sources.argtypes = [P, I32, VP, VP, D, D, VP]
    lib.sem_set_receivers.argtypes = [P, I32, VP, VP]
    lib.sem_set_c2.argtypes = [P, VP, I32]
    lib.sem_reset.argtypes = [P]
    lib.sem_run.argtypes = [P, I64, VP]
    lib.sem_step.argtypes = [P]
    lib.sem_get_field.argtypes = [P, I32, VP]
    lib.sem_set_field.argtypes = [P, I32, VP]
    lib.sem_apply_stiffness.argtypes = [P, VP, VP]
    lib.sem_apply_stiffness_noalloc.argtypes = [P, VP, VP]
    lib.sem_adjoint_gradient.argtypes = [P, VP, I64, I32, VP]
    lib.sem_synchronize.argtypes = [P]
    lib.sem_hilbert_index.argtypes = [I64, I64, I64, VP, VP, VP]
    lib.sem_last_error.argtypes = [P]
    lib.sem_last_error.restype = ctypes.c_char_p
    lib.sem_destroy.argtypes = [P]
    lib.sem_destroy.restype = None
    lib.sem_autotune.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Options), I32, I32,
                                 ctypes.POINTER(_Options), ctypes.POINTER(D), VP, I32,
                                 ctypes.POINTER(I32)]
    return lib


_lib = _load()


def library():
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def hilbert_index(W: int, H: int, cx, cy) -> np.ndarray:
    cx = np.ascontiguousarray(cx, dtype=np.int64)
    cy = np.ascontiguousarray(cy, dtype=np.int64)
    out = np.empty(cx.size, np.int64)
    rc = _lib.sem_hilbert_index(W, H, cx.size, _ptr(cx), _ptr(cy), _ptr(out))
    if rc:
        raise SemError(rc, "sem_hilbert_index")
    return out


class Simulator:
    """One SEM context (mesh, reorder, geometry, device state).

    ``quads`` is [E, 4] (quadrilaterals) or [E, 3] (the paper's triangles, odd p).
    ``device=-1`` builds a host-only context (setup, permutations, snapping; no compute).
    """

    def __init__(self, vxy, quads, c2, p: int, precision: str = "f32", order: str = "hilbert",
                 n_shots: int = 1, dt: float = 0.0, cfl: float = 0.3, device: int = 0,
                 seed: int = 3, node_order: str = "first_touch", tile_elems: int = 0,
                 shot_lanes: int = 0, tile_items: int = 0, block_threads: int = 0,
                 lds_bytes: int = 0, formulation: str = "leapfrog", scatter: str = "auto",
                 stream=None):
        self._vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        self._quads = np.ascontiguousarray(quads, dtype=np.int32)
        self._c2 = np.ascontiguousarray(c2, dtype=np.float64)
        self.precision = precision
        self.device = device
        m = _Mesh(self._vxy.shape[0], _ptr(self._vxy), self._quads.shape[0], _ptr(self._quads),
                  _ptr(self._c2), self._quads.shape[1])
        if device >= 0:
            import torch
            if stream is None:
                with torch.cuda.device(device):
                    stream = torch.cuda.current_stream(device).cuda_stream
            self._torch_device = torch.device("cuda", device)
        o = _Options(p, F64 if precision == "f64" else F32, ORDERS[order], NODE_ORDERS[node_order],
                     seed, n_shots, device, dt, cfl, stream or 0, tile_elems, shot_lanes, tile_items,
                     block_threads, lds_bytes, FORMULATIONS[formulation], SCATTERS[scatter])
        h = ctypes.c_void_p()
        rc = _lib.sem_create(ctypes.byref(m), ctypes.byref(o), ctypes.byref(h))
        if rc:
            raise SemError(rc, _lib.sem_create_error().decode())
        self._h = h
        self.n_shots = n_shots
        inf = self.info()
        self.n_elements = inf["n_elements"]
        self.n_nodes = inf["n_nodes"]
        self.p = p
        self.dt = inf["dt"]
        self.n_receivers = 0
        # bumped by every change of the sources or receivers (checked by sem_forward), and
        # the model that sem_forward set last (None after any other set_c2)
        self.io_version = 0
        self._forward_model = None

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc: int, what: str):
        if rc:
            raise SemError(rc, f"{what}: {_lib.sem_last_error(self._h).decode()}")

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def close(self):
        if getattr(self, "_h", None):
            _lib.sem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ host queries
    def info(self) -> dict:
        inf = _Info()
        self._check(_lib.sem_get_info(self._h, ctypes.byref(inf)), "sem_get_info")
        return {name: getattr(inf, name) for name, _ in _Info._fields_}

    def permutations(self):
        e = np.empty(self.n_elements, np.int32)
        n = np.empty(self.n_nodes, np.int32)
        self._check(_lib.sem_get_permutations(self._h, _ptr(e), _ptr(n)), "sem_get_permutations")
        return e, n

    def colours(self) -> np.ndarray:
        c = np.empty(self.n_elements, np.int32)
        self._check(_lib.sem_get_colours(self._h, _ptr(c)), "sem_get_colours")
        return c

    def node_coords(self) -> np.ndarray:
        xy = np.empty((self.n_nodes, 2), np.float64)
        self._check(_lib.sem_get_node_coords(self._h, _ptr(xy)), "sem_get_node_coords")
        return xy

    def set_sources(self, xy, shot=None, f0: float = 10.0, t0: Optional[float] = None) -> np.ndarray:
        xy = np.ascontiguousarray(np.atleast_2d(xy), dtype=np.float64)
        n = xy.shape[0]
        shot = np.zeros(n, np.int32) if shot is None else np.ascontiguousarray(shot, dtype=np.int32)
        t0 = 1.0 / f0 if t0 is None else t0
        nodes = np.empty(n, np.int32)
        self._check(_lib.sem_set_sources(self._h, n, _ptr(xy), _ptr(shot), f0, t0, _ptr(nodes)),
                    "sem_set_sources")
        self.io_version += 1
        return nodes

    def set_receivers(self, xy) -> np.ndarray:
        xy = np.ascontiguousarray(np.atleast_2d(xy), dtype=np.float64)
        nodes = np.empty(xy.shape[0], np.int32)
        self._check(_lib.sem_set_receivers(self._h, xy.shape[0], _ptr(xy), _ptr(nodes)),
                    "sem_set_receivers")
        self.n_receivers = xy.shape[0]
        self.io_version += 1
        return nodes

    def set_c2(self, c2):
        """New model c^2 [n_elements] in original element order: a NumPy array, a CPU
        tensor, or a float64 tensor on this simulator's GPU (read in stream order)."""
        if hasattr(c2, "is_cuda") and c2.is_cuda:
            assert c2.dtype.is_floating_point and c2.numel() == self.n_elements
            c2 = c2.detach().to(dtype=__import__("torch").float64).contiguous()
            assert c2.device == self._torch_device, "c2 lives on another GPU than the simulator"
            self._check(_lib.sem_set_c2(self._h, c2.data_ptr(), 1), "sem_set_c2")
        else:
            if hasattr(c2, "detach"):
                c2 = c2.detach().cpu().numpy()
            c2 = np.ascontiguousarray(c2, dtype=np.float64)
            assert c2.size == self.n_elements
            self._check(_lib.sem_set_c2(self._h, _ptr(c2), 0), "sem_set_c2")
        self._forward_model = None

    # ------------------------------------------------------------------ device calls
    def reset(self):
        self._check(_lib.sem_reset(self._h), "sem_reset")

    def step(self):
        self._check(_lib.sem_step(self._h), "sem_step")

    def run(self, nsteps: int, traces=None, record: bool = True):
        """Advance ``nsteps``; returns the traces tensor [S, R, nsteps] (allocated if needed)."""
        import torch
        if traces is None and record and self.n_receivers > 0:
            traces = torch.empty((self.n_shots, self.n_receivers, nsteps), dtype=self.torch_dtype,
                                 device=self._torch_device)
        ptr = traces.data_ptr() if traces is not None else None
        if traces is not None:
            assert traces.is_contiguous() and traces.dtype == self.torch_dtype
            assert tuple(traces.shape) == (self.n_shots, self.n_receivers, nsteps)
        self._check(_lib.sem_run(self._h, nsteps, ptr), "sem_run")
        return traces

    def get_field(self, which: int = FIELD_U):
        import torch
        out = torch.empty((self.n_shots, self.n_nodes), dtype=self.torch_dtype, device=self._torch_device)
        self._check(_lib.sem_get_field(self._h, which, out.data_ptr()), "sem_get_field")
        return out

    def set_field(self, which: int, x):
        assert x.is_contiguous() and x.dtype == self.torch_dtype
        assert tuple(x.shape) == (self.n_shots, self.n_nodes)
        self._check(_lib.sem_set_field(self._h, which, x.data_ptr()), "sem_set_field")

    def apply_stiffness(self, u):
        import torch
        assert u.is_contiguous() and u.dtype == self.torch_dtype
        r = torch.empty_like(u)
        self._check(_lib.sem_apply_stiffness(self._h, u.data_ptr(), r.data_ptr()), "sem_apply_stiffness")
        return r

    def apply_stiffness_noalloc(self, u, r):
        """r = K u into the caller's tensor r without any device allocation (static scratch;
        asynchronous on the simulator's stream)."""
        assert u.is_contiguous() and u.dtype == self.torch_dtype
        assert r.is_contiguous() and r.dtype == self.torch_dtype and r.shape == u.shape
        self._check(_lib.sem_apply_stiffness_noalloc(self._h, u.data_ptr(), r.data_ptr()),
                    "sem_apply_stiffness_noalloc")
        return r

    def adjoint_gradient(self, dL_dtraces, nsteps: int, ckpt_every: int = 40):
        import torch
        assert dL_dtraces.is_contiguous() and dL_dtraces.dtype == self.torch_dtype
        assert tuple(dL_dtraces.shape) == (self.n_shots, self.n_receivers, nsteps)
        g = torch.empty(self.n_elements, dtype=torch.float64, device=self._torch_device)
        self._check(_lib.sem_adjoint_gradient(self._h, dL_dtraces.data_ptr(), nsteps, ckpt_every,
                                              g.data_ptr()), "sem_adjoint_gradient")
        return g

    def synchronize(self):
        self._check(_lib.sem_synchronize(self._h), "sem_synchronize")


def _make_forward():
    import torch

    class SemForward(torch.autograd.Function):
        """traces = SemForward.apply(c2, sim, nsteps, ckpt_every): forward run from rest with
        the model ``c2`` (float64 tensor on the CPU or on the simulator's GPU, original
        element order); backward returns dL/dc2 from the checkpointed discrete adjoint, on
        the device and in the dtype of ``c2``.

        The model is saved with the graph: if the simulator's model was changed after this
        forward (another forward on the same simulator, or set_c2), backward sets it back.
        Sources and receivers are not saved; backward refuses to run when they changed."""

        @staticmethod
        def forward(ctx, c2, sim: Simulator, nsteps: int, ckpt_every: int = 40):
            model = c2.detach().to(sim._torch_device, torch.float64).clone()
            sim.set_c2(model)
            sim._forward_model = model
            sim.reset()
            tr = sim.run(nsteps)
            ctx.sim = sim
            ctx.nsteps = nsteps
            ctx.ckpt_every = ckpt_every
            ctx.model = model
            ctx.io_version = sim.io_version
            ctx.c2_device, ctx.c2_dtype = c2.device, c2.dtype
            return tr

        @staticmethod
        def backward(ctx, grad_traces):
            sim = ctx.sim
            if sim.io_version != ctx.io_version:
                raise RuntimeError("sources or receivers changed between forward and backward")
            if sim._forward_model is not ctx.model:
                # the simulator holds another model now: restore this forward's model
                sim.set_c2(ctx.model)
                sim._forward_model = ctx.model
            g = sim.adjoint_gradient(grad_traces.contiguous().to(sim.torch_dtype), ctx.nsteps,
                                     ctx.ckpt_every)
            return g.to(device=ctx.c2_device, dtype=ctx.c2_dtype), None, None, None

    return SemForward


_SemForward = None


def autotune(vxy, quads, c2, p: int, precision: str = "f32", order: str = "hilbert", n_shots: int = 1,
             device: int = 0, warmup: int = 3, steps: int = 20, stream=None, **fixed):
    """Time the step kernel over the library's candidate launch configurations (see
    sem_autotune) and return (best, table): ``best`` holds the Simulator keyword arguments
    of the fastest (block_threads, shot_lanes, lds_bytes, tile_items, us_per_step); ``table``
    one dict per candidate. Keyword arguments in ``fixed`` (block_threads, shot_lanes, lds_bytes,
    tile_items, tile_elems, dt, cfl, seed) are held fixed."""
    import torch
    vxy = np.ascontiguousarray(vxy, dtype=np.float64)
    quads = np.ascontiguousarray(quads, dtype=np.int32)
    c2 = np.ascontiguousarray(c2, dtype=np.float64)
    if stream is None:
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
    m = _Mesh(vxy.shape[0], _ptr(vxy), quads.shape[0], _ptr(quads), _ptr(c2), quads.shape[1])
    f = dict(fixed)
    o = _Options(p, F64 if precision == "f64" else F32, ORDERS[order], NODE_ORDERS["first_touch"],
                 f.pop("seed", 3), n_shots, device, f.pop("dt", 0.0), f.pop("cfl", 0.3), stream or 0,
                 f.pop("tile_elems", 0), f.pop("shot_lanes", 0), f.pop("tile_items", 0),
                 f.pop("block_threads", 0), f.pop("lds_bytes", 0))
    if f:
        raise TypeError(f"unknown fixed options {sorted(f)}")
    best = _Options()
    best_us = ctypes.c_double()
    table = np.zeros((64, 5), np.float64)
    n = ctypes.c_int32()
    rc = _lib.sem_autotune(ctypes.byref(m), ctypes.byref(o), warmup, steps, ctypes.byref(best),
                           ctypes.byref(best_us), _ptr(table), table.shape[0], ctypes.byref(n))
    if rc:
        raise SemError(rc, _lib.sem_create_error().decode())
    rows = [dict(block_threads=int(r[0]), shot_lanes=int(r[1]), lds_bytes=int(r[2]), tile_items=int(r[3]),
                 us_per_step=float(r[4])) for r in table[:min(n.value, table.shape[0])]]
    return (dict(block_threads=best.block_threads, shot_lanes=best.shot_lanes, lds_bytes=best.lds_bytes,
                 tile_items=best.tile_items, us_per_step=best_us.value), rows)


def sem_forward(c2, sim: Simulator, nsteps: int, ckpt_every: int = 40):
    """Differentiable forward: receiver traces as a function of per-element c^2."""
    global _SemForward
    if _SemForward is None:
        _SemForward = _make_forward()
    return _SemForward.apply(c2, sim, nsteps, ckpt_every)
