"""Seeded synthetic inputs for the natural-convection state solve.

This module produces the *inputs* of the method and nothing else: grid sizes,
the design field gamma (one value per element), the element heat source s, the
Dirichlet DOF mask, random states and random directions, and the arrival trace
of the serving workload.  It holds none of the method's arithmetic (no material
interpolation, no stabilisation, no element integrals), so the CPU oracle and
the HIP path can both be fed from it without sharing any computation.

Conventions (shared by every consumer):

* Structured grid of ``nx*ny*nz`` cubic elements of edge ``h``.  Element
  ``e = i + nx*(j + ny*k)``; node ``n = i + (nx+1)*(j + (ny+1)*k)``.
* Node-major interleaved state ``x[n*5 + f]`` with f = 0,1,2,3,4 = u,v,w,p,T
  (five unknowns per node, trilinear equal-order elements, Sec. "Finite element
  formulation").
* ``mask[n*5 + f] = 1`` marks a DOF whose value in ``x`` is prescribed.  Walls
  carry no-slip and T = 0 (u, v, w, T masked on every boundary node); for solves
  the pressure of node 0 is pinned as well, since the closed cavity fixes the
  pressure only up to a constant.
* The heat source occupies the elements whose centres lie in the central
  quarter of every extent; the design there is forced to solid (gamma = 0),
  since the source sits inside the solid subdomain (Sec. "Governing equations",
  heat source definition).

Random numbers come from numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

NF = 5  # unknowns per node: u, v, w, p, T


@dataclasses.dataclass
class Problem:
    """One state-solve instance: grid, physical parameters and element fields."""

    name: str
    nx: int
    ny: int
    nz: int
    h: float
    Pr: float
    Gr: float
    Ck: float
    qf: float
    alpha_max: float
    q_alpha: float
    eg: tuple
    gamma: np.ndarray  # [n_el] float64
    s: np.ndarray  # [n_el] float64
    mask_walls: np.ndarray  # [n_dof] uint8, walls only
    mask_solve: np.ndarray  # [n_dof] uint8, walls + pinned pressure at node 0
    design: Optional[np.ndarray] = None  # [n_el] bool, design domain (None: every element)

    @property
    def n_el(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_dof(self) -> int:
        return NF * self.n_nodes

    def phys(self) -> np.ndarray:
        """Physical parameters in the flat order the oracle and the binding use."""
        return np.array([self.Pr, self.Gr, self.Ck, self.qf, self.alpha_max,
                         self.q_alpha, *self.eg], dtype=np.float64)


def n_dof(nx: int, ny: int, nz: int) -> int:
    return NF * (nx + 1) * (ny + 1) * (nz + 1)


def wall_mask(nx: int, ny: int, nz: int, pin_pressure: bool = False) -> np.ndarray:
    """DOF mask: u, v, w, T prescribed on every boundary node; optional p pin at node 0."""
    I = np.arange(nx + 1)
    J = np.arange(ny + 1)
    K = np.arange(nz + 1)
    bk = (K == 0) | (K == nz)
    bj = (J == 0) | (J == ny)
    bi = (I == 0) | (I == nx)
    bnd = bk[:, None, None] | bj[None, :, None] | bi[None, None, :]
    m = np.zeros((nz + 1, ny + 1, nx + 1, NF), dtype=np.uint8)
    for f in (0, 1, 2, 4):
        m[..., f] = bnd
    m = m.reshape(-1)
    if pin_pressure:
        m[3] = 1
    return m


def source_region(nx: int, ny: int, nz: int) -> np.ndarray:
    """Boolean [n_el]: element centre inside the central quarter of every extent.

    Element i of an extent with n elements has centre (i + 1/2)/n; it is in the
    region when 3/8 <= (i + 1/2)/n <= 5/8, tested in exact integers.
    """
    def ax(n):
        i = np.arange(n)
        c = 16 * i + 8
        return (c >= 6 * n) & (c <= 10 * n)

    w = ax(nz)[:, None, None] & ax(ny)[None, :, None] & ax(nx)[None, None, :]
    return w.reshape(-1)


def box_mean(f: np.ndarray) -> np.ndarray:
    """3x3x3 box mean over the neighbours that exist (truncated at the grid edge).

    ``f`` has shape (nz, ny, nx).  The sum and the neighbour count are both
    separable, so the mean is a product of three 1-D three-point passes.
    """
    def pass1(a, axis):
        pad = [(0, 0)] * a.ndim
        pad[axis] = (1, 1)
        b = np.pad(a, pad)
        n = a.shape[axis]
        sl = lambda s, e: tuple(slice(s, e) if d == axis else slice(None) for d in range(a.ndim))
        return b[sl(0, n)] + b[sl(1, n + 1)] + b[sl(2, n + 2)]

    s = f
    c = np.ones_like(f)
    for axis in range(3):
        s = pass1(s, axis)
        c = pass1(c, axis)
    return s / c


def gamma_uniform_smoothed(nx, ny, nz, seed) -> np.ndarray:
    """U[0,1) per element, one box-mean pass."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.random((nz, ny, nx))
    return box_mean(f).reshape(-1)


def gamma_thresholded(nx, ny, nz, seed, solid_frac, passes=4, extra_passes=0) -> np.ndarray:
    """Smoothed Gaussian random field thresholded to ``solid_frac`` solid.

    i.i.d. N(0,1) per element, ``passes`` box-mean passes, threshold at the
    ``100*solid_frac`` percentile (solid, gamma = 0, below; fluid, gamma = 1,
    at or above), then ``extra_passes`` box-mean passes that give intermediate
    values at the fluid/solid interfaces.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.standard_normal((nz, ny, nx))
    for _ in range(passes):
        f = box_mean(f)
    thr = np.percentile(f, 100.0 * solid_frac)
    g = (f >= thr).astype(np.float64)
    for _ in range(extra_passes):
        g = box_mean(g)
    return g.reshape(-1)


def make_problem(name, nx, ny, nz, h, Gr, gamma, *, Pr=1.0, Ck=0.1, qf=0.881,
                 alpha_max=1.0e4, q_alpha=1.0, eg=(0.0, 0.0, -1.0), s0=1.0) -> Problem:
    omega = source_region(nx, ny, nz)
    gamma = np.array(gamma, dtype=np.float64, copy=True)
    gamma[omega] = 0.0
    s = np.where(omega, s0, 0.0).astype(np.float64)
    return Problem(name=name, nx=nx, ny=ny, nz=nz, h=h, Pr=Pr, Gr=Gr, Ck=Ck, qf=qf,
                   alpha_max=alpha_max, q_alpha=q_alpha, eg=tuple(float(c) for c in eg),
                   gamma=gamma, s=s, mask_walls=wall_mask(nx, ny, nz),
                   mask_solve=wall_mask(nx, ny, nz, pin_pressure=True))


# The five workloads.  C1 is the small case, C2 the bench workload, C3 the
# paper-scale single-GPU share (160x320x160 elements of the paper with the long,
# vertical axis along z), C4 the adjoint case and C5 the serving trace.

def config(idx: int, n: Optional[int] = None, seed: Optional[int] = None) -> Problem:
    if idx == 1:
        n = 8
        g = gamma_uniform_smoothed(n, n, n, 1001)
        return make_problem("C1 8x8x8 Gr=1e3", n, n, n, 1.0 / n, 1.0e3, g)
    if idx == 2:
        n = 64
        g = gamma_thresholded(n, n, n, 1002, 0.40)
        return make_problem("C2 64x64x64 Gr=1e4", n, n, n, 1.0 / n, 1.0e4, g)
    if idx == 3:
        nx, ny, nz = 160, 160, 320
        g = gamma_thresholded(nx, ny, nz, 1003, 0.30)
        return make_problem("C3 160x160x320 Gr=1e6", nx, ny, nz, 1.0 / 320, 1.0e6, g)
    if idx == 4:
        n = 96
        g = gamma_thresholded(n, n, n, 1004, 0.40, extra_passes=1)
        return make_problem("C4 96x96x96 Gr=1e5", n, n, n, 1.0 / n, 1.0e5, g)
    raise ValueError("config index must be 1..4 (C5 is a request trace, see serving_trace)")


def scaled_config(nx, ny, nz, Gr, seed, solid_frac=0.40, extra_passes=0, h=None, name=None) -> Problem:
    """A C2-style problem at any size (parity cases, ragged tiles, serving requests)."""
    g = gamma_thresholded(nx, ny, nz, seed, solid_frac, extra_passes=extra_passes)
    if h is None:
        h = 1.0 / max(nx, ny, nz)
    return make_problem(name or f"{nx}x{ny}x{nz} Gr={Gr:g}", nx, ny, nz, h, Gr, g)


@dataclasses.dataclass
class Request:
    idx: int
    arrival_s: float
    n: int
    Gr: float
    seed: int


def serving_trace(n_requests=256, rate_per_s=20.0, seed=4000,
                  sizes=(16, 24, 32, 48), log_gr=(3.0, 5.0)) -> List[Request]:
    """Poisson arrivals, grid size uniform over ``sizes``, log10 Gr uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=n_requests)
    grs = 10.0 ** rng.uniform(log_gr[0], log_gr[1], size=n_requests)
    return [Request(i, float(t[i]), int(ns[i]), float(grs[i]), 5000 + i) for i in range(n_requests)]


def request_problem(r: Request) -> Problem:
    return scaled_config(r.n, r.n, r.n, r.Gr, r.seed, name=f"req{r.idx} n={r.n} Gr={r.Gr:.3g}")


def random_state(p: Problem, seed: int = 2001, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Free DOFs ~ U[-1, 1], prescribed DOFs at 0 (their wall value)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1.0, 1.0, size=p.n_dof)
    m = p.mask_walls if mask is None else mask
    x[m.astype(bool)] = 0.0
    return x


def random_direction(p: Problem, seed: int, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """N(0,1) direction with the prescribed entries set to 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(p.n_dof)
    m = p.mask_walls if mask is None else mask
    v[m.astype(bool)] = 0.0
    return v


def random_gamma_direction(p: Problem, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(p.n_el)


def tiny_problem(nx, ny, nz, Gr=1.0e3, seed=7, h=None, **kw) -> Problem:
    """Small problem with gamma ~ U[0,1) per element (no smoothing, no source forcing)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.random(nx * ny * nz)
    if h is None:
        h = 1.0 / max(nx, ny, nz)
    return make_problem(f"tiny {nx}x{ny}x{nz}", nx, ny, nz, h, Gr, g, **kw)


# ---------------------------------------------------------------------------
# The paper's own test problem (Sec. "Numerical examples", heat sink in a
# closed cubic cavity): unit cube, heat-generating solid block at the middle of
# the bottom, design box of edge 0.75 resting on it, T = 0 and no-slip on the
# vertical walls and the top, insulated no-slip bottom, volume fraction 5 %.
# Vertical axis z (gravity -z).  The quarter domain [0, 1/2]^2 x [0, 1] uses
# the planes x = 1/2 and y = 1/2 as symmetry planes (normal velocity 0, every
# other field free there).  Figure 1 with the exact placement is not part of
# the text, so the block and the design box are centred in x and y, the block
# (0.1 x 0.1 in plan, 0.05 high) sits on the bottom and the design box starts
# on the block's top face.

CAVITY_SOURCE = ((0.45, 0.55), (0.45, 0.55), (0.0, 0.05))
CAVITY_DESIGN = ((0.125, 0.875), (0.125, 0.875), (0.05, 0.80))


def _centre_in(n_el: int, lo: float, hi: float, n_per_unit: int) -> np.ndarray:
    """Elements whose centre (i + 1/2) / n_per_unit lies in [lo, hi] (bounds
    given in 1/1000 so that the test is exact in integers)."""
    i = np.arange(n_el)
    c = 2000 * i + 1000  # 2000 * (i + 1/2)
    return (c >= round(2000 * lo * 1000) * n_per_unit // 1000) & \
           (c <= round(2000 * hi * 1000) * n_per_unit // 1000)


def cavity_mask(nx: int, ny: int, nz: int, quarter: bool, pin_pressure: bool) -> np.ndarray:
    """Dirichlet DOFs of the cavity: no-slip on x = 0, y = 0, z = 0, z = top
    (and x = 1, y = 1 for the full cube); T = 0 on those walls except the
    bottom; for the quarter domain the normal velocity on x = nx (u) and
    y = ny (v)."""
    I = np.arange(nx + 1)[None, None, :]
    J = np.arange(ny + 1)[None, :, None]
    K = np.arange(nz + 1)[:, None, None]
    full = (nz + 1, ny + 1, nx + 1)
    side_lo = (I == 0) | (J == 0)
    side_hi = np.zeros(full, dtype=bool) if quarter else ((I == nx) | (J == ny))
    cold = np.broadcast_to(side_lo | side_hi | (K == nz), full)
    wall = cold | np.broadcast_to(K == 0, full)
    m = np.zeros(full + (NF,), dtype=np.uint8)
    for f in (0, 1, 2):
        m[..., f] = wall
    m[..., 4] = cold
    if quarter:
        m[..., 0] |= np.broadcast_to(I == nx, full)
        m[..., 1] |= np.broadcast_to(J == ny, full)
    m = m.reshape(-1)
    if pin_pressure:
        m[3] = 1
    return m


def cavity_problem(N: int, Gr: float, *, quarter: bool = True, vf: float = 0.05, s0: float = 1.0e4,
                   Ck: float = 1.0e-2, Pr: float = 1.0, qf: float = 0.881, q_alpha: float = 8.0,
                   alpha_max: float = 1.0e5, design: Optional[np.ndarray] = None) -> Problem:
    """The cavity at N elements per unit length (N even, N >= 20 so that the
    0.05-high block spans an element).  ``design``: gamma on the design box
    (default: the uniform initial design 1 - vf); gamma = 1 (fluid) elsewhere
    and 0 on the block.  Default parameters: Ck, s0, Pr of the paper's examples
    and the first continuation step (qf, q_alpha, alpha_max)."""
    if N % 2 or N < 20:
        raise ValueError("cavity_problem: N must be even and >= 20")
    nx = ny = N // 2 if quarter else N
    nz = N
    h = 1.0 / N
    ax = lambda n, b: _centre_in(n, b[0], b[1], N)
    def region(box):
        return (ax(nz, box[2])[:, None, None] & ax(ny, box[1])[None, :, None]
                & ax(nx, box[0])[None, None, :]).reshape(-1)
    omega = region(CAVITY_SOURCE)
    dom = region(CAVITY_DESIGN) & ~omega
    gamma = np.ones(nx * ny * nz)
    if design is None:
        gamma[dom] = 1.0 - vf
    else:
        gamma[dom] = np.asarray(design, dtype=np.float64)
    gamma[omega] = 0.0
    s = np.where(omega, s0, 0.0).astype(np.float64)
    name = f"cavity {'quarter' if quarter else 'full'} N={N} Gr={Gr:g}"
    return Problem(name=name, nx=nx, ny=ny, nz=nz, h=h, Pr=Pr, Gr=Gr, Ck=Ck, qf=qf,
                   alpha_max=alpha_max, q_alpha=q_alpha, eg=(0.0, 0.0, -1.0), gamma=gamma, s=s,
                   mask_walls=cavity_mask(nx, ny, nz, quarter, False),
                   mask_solve=cavity_mask(nx, ny, nz, quarter, True), design=dom)
