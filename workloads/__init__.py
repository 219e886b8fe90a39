"""Seeded synthetic workloads for the Hilbert-ordered spectral-element time step.

This package only *draws inputs*: quadrilateral meshes (vertex coordinates and CCW
connectivity in generator order), per-element squared wave speeds, source and
receiver positions, Ricker frequencies and run lengths. It holds none of the
method's arithmetic (no basis, geometry, reordering or time stepping), so both the
CPU oracle and the HIP path may import it.

Conventions
-----------
* Domain origin at the bottom-left, y up.
* Vertex (I, J) has id ``I + (nx + 1) * J``; element (i, j) has id ``i + nx * j``
  (this generator order is the "lexicographic" element order).
* Element corners are listed counter-clockwise: (I, J), (I+1, J), (I+1, J+1), (I, J+1).
* Wave-speed models are sampled at the *unjittered* element centre, so the
  generator never evaluates the method's centroid.

The paper's benchmark meshes (Gmsh triangle meshes of a 2000 x 1000 domain, a
single-layer and a six-layer model) are not available; the named workloads below
stand in for them (near-uniform jittered quads for the single-layer benchmark, a
geometrically graded mesh for the high size-variation benchmark).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "grid_mesh",
    "tri_mesh",
    "layered_c",
    "workload",
    "WORKLOADS",
    "SEEDS",
]

# One seed per random draw, recorded so every run is reproducible.
SEEDS = {"mesh": 0, "c_noise": 1, "sources": 2, "random_order": 3, "fd_elements": 4}


@dataclasses.dataclass
class Workload:
    name: str
    p: int
    nx: int
    ny: int
    Lx: float
    Ly: float
    vxy: np.ndarray          # [Nv, 2] float64
    quads: np.ndarray        # [E, 4] int32, CCW
    c2: np.ndarray           # [E] float64, squared wave speed per element
    src_xy: np.ndarray       # [Ns, 2] float64
    src_shot: np.ndarray     # [Ns] int32, shot index of each source
    n_shots: int
    rec_xy: np.ndarray       # [R, 2] float64
    f0: float                # Ricker peak frequency [Hz]
    nsteps: int
    cfl: float = 0.3
    precision: str = "f32"
    orders: tuple = ("hilbert",)
    ckpt_every: int = 0
    c2_init: Optional[np.ndarray] = None   # starting model of the inversion workload
    anomaly_xy: Optional[np.ndarray] = None  # centre of the inversion workload's anomaly

    @property
    def n_elements(self) -> int:
        return int(self.quads.shape[0])

    @property
    def n_nodes(self) -> int:
        """Global GLL node count of a structured nx x ny quad grid of order p."""
        return (self.nx * self.p + 1) * (self.ny * self.p + 1)

    @property
    def t0(self) -> float:
        return 1.0 / self.f0


def _axis(n: int, L: float, grade_ratio: float) -> np.ndarray:
    """Vertex coordinates along one axis; geometric grading makes the last element
    ``grade_ratio`` times the first (smallest elements at the origin)."""
    if grade_ratio == 1.0:
        return np.arange(n + 1, dtype=np.float64) * (L / n)
    q = grade_ratio ** (1.0 / (n - 1))
    x = L * (q ** np.arange(n + 1, dtype=np.float64) - 1.0) / (q ** n - 1.0)
    x[0], x[-1] = 0.0, L
    return x


def grid_mesh(nx: int, ny: int, Lx: float, Ly: float, jitter: float = 0.0,
              grade_ratio: float = 1.0, seed: int = SEEDS["mesh"]):
    """Structured quad grid; interior vertices optionally jittered uniformly by
    +-``jitter`` of the local spacing per axis (boundary vertices stay put).

    Returns ``(vxy [Nv,2] f64, quads [E,4] i32, xc [E] f64, yc [E] f64)`` where
    (xc, yc) is the unjittered element centre used to sample wave-speed models.
    """
    xs = _axis(nx, Lx, grade_ratio)
    ys = _axis(ny, Ly, grade_ratio)
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # [ny+1, nx+1]
    vxy = np.stack([X.ravel(), Y.ravel()], axis=1).copy()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=vxy.shape)
        hx = np.diff(xs)
        hy = np.diff(ys)
        # local spacing at an interior vertex: the smaller adjacent element size
        hxv = np.minimum(np.r_[hx[0], hx], np.r_[hx, hx[-1]])
        hyv = np.minimum(np.r_[hy[0], hy], np.r_[hy, hy[-1]])
        Hx, Hy = np.meshgrid(hxv, hyv, indexing="xy")
        d[:, 0] *= Hx.ravel()
        d[:, 1] *= Hy.ravel()
        I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
        interior = ((I > 0) & (I < nx) & (J > 0) & (J < ny)).ravel()
        vxy[interior] += d[interior]
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v0 = i + (nx + 1) * j
    quads = np.stack([v0, v0 + 1, v0 + (nx + 1) + 1, v0 + (nx + 1)], axis=1).astype(np.int32)
    xc = 0.5 * (xs[i] + xs[i + 1])
    yc = 0.5 * (ys[j] + ys[j + 1])
    return vxy, quads, xc, yc


def tri_mesh(nx: int, ny: int, Lx: float, Ly: float, jitter: float = 0.0, seed: int = SEEDS["mesh"]):
    """Triangle mesh: the jittered quad lattice of ``grid_mesh`` with every cell cut into two
    CCW triangles along the diagonal that alternates with (i + j) parity, cell by cell.

    Returns ``(vxy [Nv,2] f64, tris [2E,3] i32, xc, yc)``; (xc, yc) is the unjittered centre
    of each triangle's cell, used to sample wave-speed models."""
    vxy, quads, xc, yc = grid_mesh(nx, ny, Lx, Ly, jitter=jitter, seed=seed)
    i = np.arange(quads.shape[0]) % nx
    j = np.arange(quads.shape[0]) // nx
    a = (i + j) % 2 == 0                      # diagonal v0-v2, else v1-v3
    v0, v1, v2, v3 = quads.T
    t1 = np.where(a[:, None], np.stack([v0, v1, v2], 1), np.stack([v0, v1, v3], 1))
    t2 = np.where(a[:, None], np.stack([v0, v2, v3], 1), np.stack([v1, v2, v3], 1))
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return vxy, tris, np.repeat(xc, 2), np.repeat(yc, 2)


def layered_c(yc: np.ndarray, Ly: float, n_layers: int = 6, c_top: float = 1500.0,
              c_step: float = 600.0) -> np.ndarray:
    """Horizontal layers of equal thickness; layer 0 at the top."""
    k = np.minimum(n_layers - 1, np.floor((Ly - yc) / (Ly / n_layers))).astype(np.int64)
    k = np.maximum(k, 0)
    return c_top + c_step * k


def _top_receivers(Lx: float, Ly: float, n: int = 128) -> np.ndarray:
    x = (np.arange(n, dtype=np.float64) + 0.5) * (Lx / n)
    return np.stack([x, np.full(n, Ly)], axis=1)


def _smooth_random_c(xc, yc, Lx, Ly, lo=1500.0, hi=4000.0, grid=1024, sigma=8.0,
                     seed=SEEDS["c_noise"]):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = gaussian_filter(rng.standard_normal((grid, grid)), sigma=sigma, mode="wrap")
    ix = np.clip((xc / Lx * grid).astype(np.int64), 0, grid - 1)
    iy = np.clip((yc / Ly * grid).astype(np.int64), 0, grid - 1)
    s = g[iy, ix]
    s = (s - s.min()) / (s.max() - s.min())
    return lo + (hi - lo) * s


def workload(name: str, n: Optional[int] = None, nsteps: Optional[int] = None,
             p: Optional[int] = None, n_shots: Optional[int] = None) -> Workload:
    """Build a named workload. ``n`` overrides the elements per side (reduced-size
    variants for tests), ``nsteps``/``p``/``n_shots`` override run length, order and
    shot count."""
    if name == "homog64":
        # 1 km x 1 km, 64 x 64 uniform quads, p=4, c=1500, Ricker 10 Hz at the centre, 200 steps, FP64.
        nx = n or 64
        L = 1000.0
        vxy, quads, xc, yc = grid_mesh(nx, nx, L, L)
        c = np.full(quads.shape[0], 1500.0)
        return Workload(name, p or 4, nx, nx, L, L, vxy, quads, c * c,
                        np.array([[L / 2, L / 2]]), np.zeros(1, np.int32), 1,
                        _top_receivers(L, L), 10.0, nsteps or 200, precision="f64",
                        orders=("hilbert", "lex", "random"))
    if name == "layered1024":
        # 10 km x 10 km, 1024^2 quads jittered +-20%, p=4, six layers 1500..4500 +-5% noise, 15 Hz, 2000 steps.
        nx = n or 1024
        L = 10000.0
        vxy, quads, xc, yc = grid_mesh(nx, nx, L, L, jitter=0.2)
        rng = np.random.default_rng(SEEDS["c_noise"])
        c = layered_c(yc, L) * (1.0 + rng.uniform(-0.05, 0.05, size=quads.shape[0]))
        return Workload(name, p or 4, nx, nx, L, L, vxy, quads, c * c,
                        np.array([[L / 2, L / 2]]), np.zeros(1, np.int32), 1,
                        _top_receivers(L, L), 15.0, nsteps or 2000, precision="f32",
                        orders=("hilbert", "morton", "lex", "random"))
    if name == "graded1414":
        # 10 km x 10 km, 1414^2 quads graded 1:8 toward (0,0), p=5, smooth random c 1500..4000, 1000 steps.
        nx = n or 1414
        L = 10000.0
        vxy, quads, xc, yc = grid_mesh(nx, nx, L, L, grade_ratio=8.0)
        c = _smooth_random_c(xc, yc, L, L)
        return Workload(name, p or 5, nx, nx, L, L, vxy, quads, c * c,
                        np.array([[L / 2, L / 2]]), np.zeros(1, np.int32), 1,
                        _top_receivers(L, L), 15.0, nsteps or 1000, precision="f32",
                        orders=("hilbert", "morton", "random"))
    if name == "batch512":
        # 512^2 jittered quads, p=4, six layers (no noise), 64 shots at seeded uniform positions, 1500 steps.
        nx = n or 512
        L = 10000.0
        S = n_shots or 64
        vxy, quads, xc, yc = grid_mesh(nx, nx, L, L, jitter=0.2)
        c = layered_c(yc, L)
        rng = np.random.default_rng(SEEDS["sources"])
        src = rng.uniform(0.0, L, size=(S, 2))
        return Workload(name, p or 4, nx, nx, L, L, vxy, quads, c * c,
                        src, np.arange(S, dtype=np.int32), S, _top_receivers(L, L),
                        15.0, nsteps or 1500, precision="f32", orders=("hilbert", "random"))
    if name == "adjoint512":
        # 512^2 jittered quads, p=4; true model = layers x (1 + 10% Gaussian anomaly), initial = layers;
        # 8 shots x 128 receivers, 1500 steps, checkpoints every 40 steps.
        # In 1500 steps at the CFL-0.3 time step a wave travels about 200 m in the 1500 m/s top
        # layer (~10 elements), so the shots, the anomaly and the receivers they illuminate sit
        # within that reach: the anomaly 150 m below the top edge (sigma = L/64), the shots on
        # a line 100 m below the top, 125 m apart, centred over it.
        nx = n or 512
        L = 10000.0
        S = n_shots or 8
        vxy, quads, xc, yc = grid_mesh(nx, nx, L, L, jitter=0.2)
        c0 = layered_c(yc, L)
        sig = L / 64.0
        anomaly = np.array([L / 2, L - 150.0])
        bump = np.exp(-((xc - anomaly[0]) ** 2 + (yc - anomaly[1]) ** 2) / (2.0 * sig * sig))
        c_true = c0 * (1.0 + 0.1 * bump)
        src = np.stack([L / 2 + (np.arange(S) - (S - 1) / 2.0) * (L / 80.0), np.full(S, L - L / 100.0)],
                       axis=1)
        wl = Workload(name, p or 4, nx, nx, L, L, vxy, quads, c_true * c_true,
                      src, np.arange(S, dtype=np.int32), S, _top_receivers(L, L),
                      15.0, nsteps or 1500, precision="f32", orders=("hilbert",),
                      ckpt_every=40, c2_init=c0 * c0)
        wl.anomaly_xy = anomaly
        return wl
    if name == "tri2000":
        # The paper's single-layer benchmark shape (Sec. 5): a 2000 x 1000 domain of near-uniform
        # unstructured triangles, p=5 (21 local nodes), constant wave speed; 500 x 250 jittered
        # cells cut into 250k triangles, c = 1500, Ricker 15 Hz at the centre, 128 receivers.
        nx = n or 500
        Lx, Ly = 2000.0, 1000.0
        vxy, tris, xc, yc = tri_mesh(nx, max(1, nx // 2), Lx, Ly, jitter=0.2)
        c = np.full(tris.shape[0], 1500.0)
        return Workload(name, p or 5, nx, max(1, nx // 2), Lx, Ly, vxy, tris, c * c,
                        np.array([[Lx / 2, Ly / 2]]), np.zeros(1, np.int32), 1,
                        _top_receivers(Lx, Ly), 15.0, nsteps or 1000, precision="f32",
                        orders=("hilbert", "morton", "lex", "random"))
    raise KeyError(f"unknown workload {name!r}")


WORKLOADS = ("homog64", "layered1024", "graded1414", "batch512", "adjoint512", "tri2000")


def random_field(n_nodes: int, n_shots: int = 1, seed: int = 7) -> np.ndarray:
    """Seeded nodal test field ``[n_shots, n_nodes]`` (float64), uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n_shots, n_nodes))
