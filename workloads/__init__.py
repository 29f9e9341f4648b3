"""Seeded synthetic inputs for the grey radiative-transfer lattice-Boltzmann step.

This module is shared by the tests, the benchmark and the FP64 oracle.  It
holds no arithmetic of the method itself (no streaming weights, no moments,
no collision): only quadrature tables taken from a library routine, grid
geometry, and seeded random coefficient fields and initial states.

Workload shapes follow the paper's tests (Sec. 4 and Sec. 5):

* ``sphere``     homogeneous radiating sphere (Sec. 4.2.2),
* ``diffusion``  Gaussian pulse in a scattering medium (Sec. 4.2.3),
* ``beams``      crossing beams plus an opaque obstacle (Sec. 4.1.1, 4.2.1),
* ``batch``      many independent small domains of uneven size and opacity,
* ``moving``     a relativistic shear flow with a log-normal absorption field
                 (mixed-frame equation of App. B),
* ``free_wave``  a spherical wave in vacuum (Sec. 4.1.2), on a Lebedev or a
                 Gauss-Legendre product rule (Sec. 3.2.1).

Conventions: dx = 1, cell centres at (i + 1/2), arrays are indexed
``[z, y, x]`` with x fastest, populations ``[dir, z, y, x]`` and are
weight-absorbed (I_i = w_i I(n_i), Sec. 3.2 discrete moments).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Face indices, in the order used by the C ABI and the oracle.
FACE_MX, FACE_PX, FACE_MY, FACE_PY, FACE_MZ, FACE_PZ = range(6)
# Boundary kinds.
BC_OUTFLOW, BC_PERIODIC, BC_INFLOW = 0, 1, 2
# Collision kinds.
COLL_IMPLICIT, COLL_EXPLICIT, COLL_LAMBDA = 0, 1, 2

LEBEDEV_ORDERS = {6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 74: 13, 86: 15,
                  110: 17, 146: 19, 170: 21, 194: 23}


def lebedev(npoints: int) -> Tuple[np.ndarray, np.ndarray]:
    """Lebedev rule with ``npoints`` nodes (Sec. 3.2.1, Lebedev quadrature).

    Returns unit directions ``(N, 3)`` and weights ``(N,)`` normalised to
    sum to 1 (the discrete moments of Sec. 3.2 carry the 1/(4 pi) of the
    continuous definitions).  Nodes come from ``scipy.integrate.lebedev_rule``.
    """
    from scipy.integrate import lebedev_rule
    order = LEBEDEV_ORDERS[npoints]
    x, w = lebedev_rule(order)
    dirs = np.ascontiguousarray(x.T, dtype=np.float64)
    # Renormalise each node to unit length (they are, to the last bit or two).
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    weights = np.asarray(w, dtype=np.float64) / (4.0 * np.pi)
    return dirs, weights


def lebedev_degree(npoints: int) -> int:
    return LEBEDEV_ORDERS[npoints]


def gauss_legendre_product(n_theta: int, n_phi: int) -> Tuple[np.ndarray, np.ndarray]:
    """Product rule on the sphere (Sec. 3.2.1, Gauss-Legendre quadrature):
    ``n_theta`` Gauss-Legendre nodes in mu = cos(theta) (numpy's leggauss)
    times ``n_phi`` equally spaced azimuths phi_j = 2 pi (j + 1/2) / n_phi
    (the trapezoidal rule), weights a_k / (2 n_phi) so that they sum to 1.
    Integrates the spherical harmonics of degree below
    min(2 n_theta, n_phi) exactly; with n_phi even the node set is centrally
    symmetric.  Returns unit directions ``(N, 3)`` and weights ``(N,)``."""
    mu, a = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    st = np.sqrt(1.0 - mu ** 2)
    dirs = np.stack([np.outer(st, np.cos(phi)).ravel(), np.outer(st, np.sin(phi)).ravel(),
                     np.repeat(mu, n_phi)], axis=1)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    w = np.repeat(a / (2.0 * n_phi), n_phi)
    return np.ascontiguousarray(dirs), w


def gauss_legendre_degree(n_theta: int, n_phi: int) -> int:
    return min(2 * n_theta - 1, n_phi - 1)


def quadrature(rule) -> Tuple[np.ndarray, np.ndarray]:
    """``("lebedev", npoints)`` or ``("gl", n_theta, n_phi)``."""
    if rule[0] == "lebedev":
        return lebedev(rule[1])
    if rule[0] == "gl":
        return gauss_legendre_product(rule[1], rule[2])
    raise ValueError(f"unknown rule {rule!r}")


def nearest_direction(dirs: np.ndarray, target: Sequence[float]) -> int:
    t = np.asarray(target, dtype=np.float64)
    t = t / np.linalg.norm(t)
    return int(np.argmax(dirs @ t))


@dataclasses.dataclass
class InflowPlane:
    """Prescribed ghost values for one (face, direction) pair.

    ``values`` is float32 in the face's own layout: x faces ``[z, y]``,
    y faces ``[z, x]``, z faces ``[y, x]``.
    """
    face: int
    direction: int
    values: np.ndarray


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    dt: float
    dirs: np.ndarray
    weights: np.ndarray
    bc: Tuple[int, int, int, int, int, int]
    kappa_a: np.ndarray              # float32 [z, y, x]
    kappa_s: np.ndarray              # float32 [z, y, x]
    eta: np.ndarray                  # float32 [z, y, x]
    I0: np.ndarray                   # float64 [dir, z, y, x]
    steps: int
    dx: float = 1.0
    vel: Optional[np.ndarray] = None  # float32 [3, z, y, x] (vx, vy, vz)
    inflow: List[InflowPlane] = dataclasses.field(default_factory=list)
    collision: int = COLL_IMPLICIT
    lambda_iters: int = 5
    lam: float = 0.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def ndir(self) -> int:
        return int(self.dirs.shape[0])

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)


def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) + 0.5


def _zero_state(ndir: int, nz: int, ny: int, nx: int, alloc: bool = True) -> np.ndarray:
    if not alloc:
        return np.zeros((0,), dtype=np.float64)
    return np.zeros((ndir, nz, ny, nx), dtype=np.float64)


# ---------------------------------------------------------------------------
# Homogeneous radiating sphere (Sec. 4.2.2).
# ---------------------------------------------------------------------------
def sphere(n: int = 32, npoints: int = 50, radius: float = 8.0,
           kappa: float = 10.0, dt: float = 0.5, steps: int = 100) -> Problem:
    """kappa_a = eta = ``kappa`` inside a centred sphere, 0 outside; kappa_s = 0;
    zero initial populations; outflow on all faces.  A cell is inside when its
    centre is closer than ``radius`` to the box centre."""
    dirs, w = lebedev(npoints)
    c = _centres(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    inside = r < radius
    ka = np.where(inside, kappa, 0.0).astype(np.float32)
    return Problem(
        name=f"sphere{n}", nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w,
        bc=(BC_OUTFLOW,) * 6, kappa_a=ka, kappa_s=np.zeros_like(ka), eta=ka.copy(),
        I0=_zero_state(len(w), n, n, n), steps=steps,
        meta={"radius": radius, "kappa": kappa, "centre": n / 2},
    )


# ---------------------------------------------------------------------------
# Spherical wave in the free-streaming regime (Sec. 4.1.2).
# ---------------------------------------------------------------------------
def free_wave(n: int = 200, rule=("lebedev", 194), radius: float = 16.0, dt: float = 0.2,
              steps: int = 200, alloc_state: bool = True) -> Problem:
    """Vacuum (no absorption, emission or scattering), outflow faces, an
    isotropic unit intensity inside a centred sphere of ``radius`` cells:
    I_i = w_i (E = 1) where the cell centre is inside, 0 elsewhere."""
    dirs, w = quadrature(rule)
    c = _centres(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = ((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2) < radius ** 2
    I0 = (w[:, None, None, None] * inside[None]) if alloc_state else np.zeros((0,))
    zeros = np.zeros((n, n, n), dtype=np.float32)
    name = "wave%d_%s" % (n, "_".join(str(v) for v in rule))
    return Problem(
        name=name, nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w, bc=(BC_OUTFLOW,) * 6,
        kappa_a=zeros, kappa_s=zeros.copy(), eta=zeros.copy(), I0=I0, steps=steps,
        meta={"radius": radius, "centre": n / 2, "rule": tuple(rule)},
    )


# ---------------------------------------------------------------------------
# Gaussian pulse in a scattering medium (Sec. 4.2.3).
# ---------------------------------------------------------------------------
def diffusion(n: int = 128, npoints: int = 50, kappa_s: float = 1e3,
              jitter: float = 0.05, sigma: float = 6.0, amplitude: float = 1.0,
              dt: float = 0.5, steps: int = 1000, seed: int = 2,
              alloc_state: bool = True) -> Problem:
    """Pure scattering, kappa_s = ``kappa_s`` (1 + jitter U(-1, 1)) per cell,
    isotropic Gaussian energy pulse I_i = w_i E0(r) at the box centre,
    periodic boundaries."""
    dirs, w = lebedev(npoints)
    rng = np.random.default_rng(seed)
    ks = (kappa_s * (1.0 + jitter * rng.uniform(-1.0, 1.0, size=(n, n, n)))).astype(np.float32)
    c = _centres(n)
    r2 = ((c[:, None, None] - n / 2) ** 2 + (c[None, :, None] - n / 2) ** 2
          + (c[None, None, :] - n / 2) ** 2)
    E0 = amplitude * np.exp(-r2 / (2.0 * sigma ** 2))
    I0 = (w[:, None, None, None] * E0[None]) if alloc_state else np.zeros((0,))
    zeros = np.zeros((n, n, n), dtype=np.float32)
    return Problem(
        name=f"diffusion{n}", nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w,
        bc=(BC_PERIODIC,) * 6, kappa_a=zeros, kappa_s=ks, eta=zeros.copy(),
        I0=I0, steps=steps,
        meta={"sigma": sigma, "amplitude": amplitude, "E0": E0},
    )


# ---------------------------------------------------------------------------
# Crossing beams plus opaque sphere (Sec. 4.1.1 crossing beams, Sec. 4.2.1 shadow).
# ---------------------------------------------------------------------------
def beams(n: int = 256, npoints: int = 110, dt: float = 0.5, steps: int = 500,
          seed: int = 3, beam_a: bool = True, beam_b: bool = True,
          obstacle: bool = True, alloc_state: bool = True) -> Problem:
    """Beam A along +x injected through the x = 0 face, beam B along the
    stencil direction nearest (1, 1, 0)/sqrt(2) injected through the y = 0
    face, both with unit ghost populations inside a disk; an opaque sphere
    (kappa_a = 1e4) sits in beam A's path; background kappa_a is
    log-uniform in [1e-3, 1e1] per 16^3 block (per (n/16)^3 block when the
    box is scaled down).  Geometry scales with n / 256."""
    dirs, w = lebedev(npoints)
    s = n / 256.0
    rng = np.random.default_rng(seed)
    nb = max(1, n // 16)
    blk = int(np.ceil(n / nb))
    block_vals = 10.0 ** rng.uniform(-3.0, 1.0, size=(nb, nb, nb))
    idx = np.minimum(np.arange(n) // blk, nb - 1)
    ka = block_vals[idx[:, None, None], idx[None, :, None], idx[None, None, :]]
    c = _centres(n)
    if obstacle:
        ctr = (200 * s, 96 * s, 128 * s)          # (x, y, z)
        r2 = ((c[None, None, :] - ctr[0]) ** 2 + (c[None, :, None] - ctr[1]) ** 2
              + (c[:, None, None] - ctr[2]) ** 2)
        ka = np.where(r2 < (20 * s) ** 2, 1e4, ka)
    ka = ka.astype(np.float32)
    zeros = np.zeros((n, n, n), dtype=np.float32)
    inflow = []
    ia = nearest_direction(dirs, (1, 0, 0))
    ib = nearest_direction(dirs, (1, 1, 0))
    rad = 12 * s
    if beam_a:   # face -x, plane layout [z, y]
        disk = ((c[:, None] - 128 * s) ** 2 + (c[None, :] - 96 * s) ** 2) < rad ** 2
        inflow.append(InflowPlane(FACE_MX, ia, disk.astype(np.float32)))
    if beam_b:   # face -y, plane layout [z, x]
        disk = ((c[:, None] - 98 * s) ** 2 + (c[None, :] - 32 * s) ** 2) < rad ** 2
        inflow.append(InflowPlane(FACE_MY, ib, disk.astype(np.float32)))
    bc = [BC_OUTFLOW] * 6
    bc[FACE_MX] = BC_INFLOW
    bc[FACE_MY] = BC_INFLOW
    return Problem(
        name=f"beams{n}", nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w,
        bc=tuple(bc), kappa_a=ka, kappa_s=zeros, eta=zeros.copy(),
        I0=_zero_state(len(w), n, n, n, alloc_state), steps=steps, inflow=inflow,
        meta={"beam_a_dir": ia, "beam_b_dir": ib,
              "obstacle_centre": (200 * s, 96 * s, 128 * s), "obstacle_radius": 20 * s},
    )


def beams_costs(n: int = 256, npoints: int = 110, dt: float = 0.5, steps: int = 20,
                seed: int = 3, kappa_s: float = 0.5, kappa_a_max: float = 1.0,
                alloc_state: bool = True) -> Problem:
    """The crossing-beams geometry for comparing the cost of the collision
    kinds (Sec. 6 compares the explicit and the iterated implicit stepper):
    the same beams and obstacle, with absorption capped at ``kappa_a_max``
    and uniform scattering ``kappa_s`` so that the explicit step is stable
    (dt (kappa_a + kappa_s) < 1), and emission eta = kappa_a / 10."""
    p = beams(n=n, npoints=npoints, dt=dt, steps=steps, seed=seed, alloc_state=alloc_state)
    ka = np.minimum(p.kappa_a, np.float32(kappa_a_max)).astype(np.float32)
    p.kappa_a = ka
    p.kappa_s = np.full(p.shape, kappa_s, dtype=np.float32)
    p.eta = (ka * np.float32(0.1)).astype(np.float32)
    p.name = f"beams_costs{n}"
    return p


# ---------------------------------------------------------------------------
# Batched opacity sweep: many independent domains.
# ---------------------------------------------------------------------------
BATCH_EDGES = (24, 32, 48, 64, 96)


def batch_domain(d: int, seed: int = 4, npoints: int = 50, dt: float = 0.5,
                 edges: Sequence[int] = BATCH_EDGES, steps_range=(50, 400)) -> Problem:
    """Domain ``d`` of the sweep: cubic edge drawn from ``edges``; one scalar
    kappa_a and kappa_s, each log-uniform in [1e-2, 1e3]; eta = kappa_a * B
    with B = 1; a step count uniform in ``steps_range``; zero initial
    populations; outflow boundaries.  Draws come from ``default_rng([seed, d])``."""
    dirs, w = lebedev(npoints)
    rng = np.random.default_rng([seed, d])
    n = int(rng.choice(np.asarray(edges)))
    ka = float(10.0 ** rng.uniform(-2.0, 3.0))
    ks = float(10.0 ** rng.uniform(-2.0, 3.0))
    steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
    full = lambda v: np.full((n, n, n), v, dtype=np.float32)
    return Problem(
        name=f"batch{d}", nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w,
        bc=(BC_OUTFLOW,) * 6, kappa_a=full(ka), kappa_s=full(ks), eta=full(ka),
        I0=np.zeros((0,)), steps=steps, meta={"kappa_a": ka, "kappa_s": ks},
    )


# ---------------------------------------------------------------------------
# Moving fluid: relativistic shear flow (App. B mixed-frame equation).
# ---------------------------------------------------------------------------
def gaussian_random_field(n: int, corr_len: float, seed: int) -> np.ndarray:
    """Unit-variance Gaussian random field on an n^3 periodic grid with
    covariance exp(-r^2 / (2 corr_len^2)): white noise filtered in Fourier
    space by the square root of that covariance's spectrum."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    filt = np.exp(-0.25 * k2 * corr_len ** 2)
    g = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    g -= g.mean()
    g /= g.std()
    return g


def moving(n: int = 192, npoints: int = 146, dt: float = 0.5, steps: int = 64,
           vmax: float = 0.5, shear_width: float = 8.0, corr_len: float = 10.0,
           sigma_ln: float = 1.0, kappa_s: float = 0.5, seed: int = 5,
           alloc_state: bool = True) -> Problem:
    """Fluid-frame kappa_a log-normal (mean 1), fluid-frame kappa_s constant,
    fluid-frame eta = kappa_a * B with B = 1, shear flow
    v_x = vmax tanh((y - n/2) / shear_width); zero initial populations;
    outflow boundaries.  Geometry scales with n / 192."""
    dirs, w = lebedev(npoints)
    s = n / 192.0
    g = gaussian_random_field(n, corr_len * s, seed)
    ka = np.exp(sigma_ln * g - 0.5 * sigma_ln ** 2).astype(np.float32)
    c = _centres(n)
    vx = vmax * np.tanh((c - n / 2) / (shear_width * s))
    vel = np.zeros((3, n, n, n), dtype=np.float32)
    vel[0] = vx[None, :, None].astype(np.float32)
    return Problem(
        name=f"moving{n}", nx=n, ny=n, nz=n, dt=dt, dirs=dirs, weights=w,
        bc=(BC_OUTFLOW,) * 6, kappa_a=ka, kappa_s=np.full((n, n, n), kappa_s, np.float32),
        eta=ka.copy(), I0=_zero_state(len(w), n, n, n, alloc_state), steps=steps,
        vel=vel, meta={"detector_face": FACE_PX},
    )


# ---------------------------------------------------------------------------
# Generic seeded problems for parity tests.
# ---------------------------------------------------------------------------
def random_problem(seed: int, shape: Tuple[int, int, int] = (11, 13, 37),
                   npoints: int = 26, dt: float = 0.5,
                   bc: Sequence[int] = (BC_OUTFLOW,) * 6, steps: int = 3,
                   kappa_range=(-2.0, 2.0), moving_fluid: bool = False,
                   vmax: float = 0.6, inflow_planes: int = 0,
                   collision: int = COLL_IMPLICIT, lam: float = 0.0,
                   lambda_iters: int = 5) -> Problem:
    """Random state and random log-uniform coefficient fields on a ragged
    box ``shape = (nz, ny, nx)``.  With ``moving_fluid`` a random velocity
    field with |v| < vmax is added.  ``inflow_planes`` random ghost planes
    are attached to the inflow faces listed in ``bc``."""
    nz, ny, nx = shape
    dirs, w = lebedev(npoints)
    rng = np.random.default_rng(seed)
    lo, hi = kappa_range
    ka = (10.0 ** rng.uniform(lo, hi, size=shape)).astype(np.float32)
    ks = (10.0 ** rng.uniform(lo, hi, size=shape)).astype(np.float32)
    eta = (10.0 ** rng.uniform(lo, hi, size=shape)).astype(np.float32)
    I0 = rng.uniform(0.0, 1.0, size=(len(w), nz, ny, nx)) * w[:, None, None, None]
    vel = None
    if moving_fluid:
        v = rng.standard_normal((3, nz, ny, nx))
        v /= np.linalg.norm(v, axis=0, keepdims=True)
        v *= rng.uniform(0.0, vmax, size=(1, nz, ny, nx))
        vel = v.astype(np.float32)
    inflow = []
    faces = [f for f in range(6) if bc[f] == BC_INFLOW]
    sizes = {0: (nz, ny), 1: (nz, ny), 2: (nz, nx), 3: (nz, nx), 4: (ny, nx), 5: (ny, nx)}
    for k in range(inflow_planes):
        if not faces:
            break
        f = faces[k % len(faces)]
        axis, side = f // 2, f % 2
        # Only directions that enter the box through this face.
        comp = dirs[:, axis]
        cand = np.nonzero(comp > 1e-12)[0] if side == 0 else np.nonzero(comp < -1e-12)[0]
        dsel = int(rng.choice(cand))
        vals = rng.uniform(0.0, 1.0, size=sizes[f]).astype(np.float32)
        inflow.append(InflowPlane(f, dsel, vals))
    return Problem(
        name=f"random{seed}", nx=nx, ny=ny, nz=nz, dt=dt, dirs=dirs, weights=w,
        bc=tuple(bc), kappa_a=ka, kappa_s=ks, eta=eta, I0=I0, steps=steps,
        vel=vel, inflow=inflow, collision=collision, lam=lam,
        lambda_iters=lambda_iters,
    )
