"""FP64 CPU oracle for the grey radiative-transfer lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module; the HIP library never
does, and this module imports nothing from it.  It is deliberately plain
and slow: numpy in float64, loops over directions and stencil taps in the
order the paper writes them, no fusion, no blocking.

What one step computes (Weih et al. 2020, Sec. 3.3 "Numerical procedure"):

1. stream: every population is pulled from the point r - n_i dt by the
   trilinear interpolation of eq. (interp), with the per-axis shift vectors
   x^, y^, z^ that point along sgn(n_i^a);
2. moments of the streamed populations, E* = sum_i I*_i and
   F* = sum_i n_i I*_i (eq. moments_discrete);
3. collision, one of
   * implicit (eq. rte_implicit): the exact solution of the per-cell linear
     system, with equilibrium and sources taken at the new time level;
   * explicit (eq. collision-step);
   * Lambda iteration with a fixed number of cycles (Sec. 3.3, list 1.-4.);
   * moving fluid: the implicit mixed-frame equation of App. B, with the
     fluid-frame energy density J from eq. (J).

The adjoint part (``stream_transpose``, ``collide_moving_vjp``,
``detected_energy_gradient``) differentiates this same forward run in reverse
mode; it is pinned by the transpose identity and by finite differences of
the forward run.

Conventions: populations are weight-absorbed (I_i = w_i I(n_i)); kappa_s in
the inputs is the paper's kappa_0 and ``lam`` is lambda = 3 kappa_1 / kappa_0
(eq. rte_gray_bgkform); arrays are ``[dir, z, y, x]``.

Readings of the paper that this oracle fixes (the paper is silent there):
* the state is post-collision; a step streams first, then collides;
* boundaries: a source point outside the box is wrapped on periodic axes;
  if it is then outside along exactly one axis whose face is an inflow face
  with a prescribed ghost plane for that direction, it takes that ghost
  value; otherwise it is vacuum (0) — this covers outflow faces and
  edge/corner ghosts;
* the Lambda iteration starts from the moments of the streamed populations;
* the sources of the coupling list use k_s = k_0 - k_1 / 3 as that list
  defines it (eq. rte_gray's momentum sink would be k_0 - k_1; the two agree
  for isotropic scattering, lam = 0), and H_0 is the time component of H
  orthogonal to the fluid four-velocity, H_0 = v^j H_j, the sign with which
  S_0 equals the energy the collision takes from the radiation.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

FACE_MX, FACE_PX, FACE_MY, FACE_PY, FACE_MZ, FACE_PZ = range(6)
BC_OUTFLOW, BC_PERIODIC, BC_INFLOW = 0, 1, 2
COLL_IMPLICIT, COLL_EXPLICIT, COLL_LAMBDA = 0, 1, 2

# array axis (0 = z, 1 = y, 2 = x) -> (low face, high face)
_AXIS_FACES = {0: (FACE_MZ, FACE_PZ), 1: (FACE_MY, FACE_PY), 2: (FACE_MX, FACE_PX)}


# ---------------------------------------------------------------------------
# Streaming (Sec. 3.3, eqs. rte-stream-collide and interp)
# ---------------------------------------------------------------------------
def shift_signs(n: np.ndarray) -> np.ndarray:
    """sgn(n^a) for the shift vectors x^, y^, z^ below eq. (interp).

    sgn(0) is taken as +1: the tap it selects carries weight
    dt |n^a| = 0, and zero-weight taps are skipped."""
    return np.where(np.asarray(n) < 0.0, -1, 1).astype(np.int64)


def tap_weight(n: np.ndarray, dt: float, dx: float, bx: int, by: int, bz: int) -> float:
    """Weight of the tap r - bx x^ - by y^ - bz z^ in eq. (interp).

    Per axis the factor is dt |n^a| when the tap is shifted along that
    axis and (dx - dt |n^a|) when it is not; the product is divided by
    dx dy dz (a uniform grid, dx = dy = dz)."""
    f = 1.0
    for b, comp in ((bx, n[0]), (by, n[1]), (bz, n[2])):
        f *= dt * abs(comp) if b else (dx - dt * abs(comp))
    return f / (dx * dx * dx)


def _wrap_and_flag(prob, cz, cy, cx):
    sizes = (prob.nz, prob.ny, prob.nx)
    coords = [np.asarray(cz), np.asarray(cy), np.asarray(cx)]
    outs = []
    for a in range(3):
        lo_face, _ = _AXIS_FACES[a]
        if prob.bc[lo_face] == BC_PERIODIC:
            coords[a] = np.mod(coords[a], sizes[a])
        outs.append((coords[a] < 0) | (coords[a] >= sizes[a]))
    coords = np.broadcast_arrays(*coords)
    outs = np.broadcast_arrays(*outs)
    return coords, outs


def source_value(I_i: np.ndarray, i: int, prob, cz, cy, cx, ghosts: bool = True) -> np.ndarray:
    """Population ``i`` at integer cell coordinates that may lie outside the box.

    Periodic axes wrap.  A point still outside along exactly one axis takes
    the prescribed inflow ghost value of that face for direction ``i`` if
    one exists (and ``ghosts`` is true), else 0; a point outside along two
    or three axes is 0."""
    (cz, cy, cx), (oz, oy, ox) = _wrap_and_flag(prob, cz, cy, cx)
    nout = oz.astype(np.int64) + oy.astype(np.int64) + ox.astype(np.int64)
    vals = I_i[np.clip(cz, 0, prob.nz - 1), np.clip(cy, 0, prob.ny - 1),
               np.clip(cx, 0, prob.nx - 1)].astype(np.float64)
    vals = np.where(nout == 0, vals, 0.0)
    if not ghosts:
        return vals
    for plane in prob.inflow:
        if plane.direction != i or prob.bc[plane.face] != BC_INFLOW:
            continue
        axis = {FACE_MX: 2, FACE_PX: 2, FACE_MY: 1, FACE_PY: 1, FACE_MZ: 0, FACE_PZ: 0}[plane.face]
        size = (prob.nz, prob.ny, prob.nx)[axis]
        coord = (cz, cy, cx)[axis]
        at_face = (coord == -1) if plane.face % 2 == 0 else (coord == size)
        mask = (nout == 1) & at_face
        if not np.any(mask):
            continue
        pv = np.asarray(plane.values, dtype=np.float64)
        if axis == 2:
            g = pv[np.clip(cz, 0, prob.nz - 1), np.clip(cy, 0, prob.ny - 1)]
        elif axis == 1:
            g = pv[np.clip(cz, 0, prob.nz - 1), np.clip(cx, 0, prob.nx - 1)]
        else:
            g = pv[np.clip(cy, 0, prob.ny - 1), np.clip(cx, 0, prob.nx - 1)]
        vals = np.where(mask, g, vals)
    return vals


def _taps(n_i: np.ndarray, dt: float, dx: float):
    """The eight (bx, by, bz, weight) taps of eq. (interp), zero weights dropped."""
    out = []
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                wgt = tap_weight(n_i, dt, dx, bx, by, bz)
                if wgt != 0.0:
                    out.append((bx, by, bz, wgt))
    return out


def stream_direction(I_i: np.ndarray, i: int, prob, ghosts: bool = True) -> np.ndarray:
    """I*_i(r) = I_i(r - n_i dt) by eq. (interp) on the whole box."""
    n_i = prob.dirs[i]
    s = shift_signs(n_i)        # (sx, sy, sz)
    z = np.arange(-1, prob.nz + 1)[:, None, None]
    y = np.arange(-1, prob.ny + 1)[None, :, None]
    x = np.arange(-1, prob.nx + 1)[None, None, :]
    padded = source_value(I_i, i, prob, z, y, x, ghosts=ghosts)
    out = np.zeros((prob.nz, prob.ny, prob.nx), dtype=np.float64)
    for bx, by, bz, wgt in _taps(n_i, prob.dt, prob.dx):
        oz, oy, ox = 1 - bz * s[2], 1 - by * s[1], 1 - bx * s[0]
        out += wgt * padded[oz:oz + prob.nz, oy:oy + prob.ny, ox:ox + prob.nx]
    return out


def stream(I: np.ndarray, prob) -> np.ndarray:
    out = np.empty((prob.ndir, prob.nz, prob.ny, prob.nx), dtype=np.float64)
    for i in range(prob.ndir):
        out[i] = stream_direction(I[i], i, prob)
    return out


def stream_cells(I: np.ndarray, prob, cells: np.ndarray) -> np.ndarray:
    """I* at a list of cells ``cells[k] = (z, y, x)`` only: ``[dir, k]``."""
    cells = np.asarray(cells, dtype=np.int64)
    out = np.zeros((prob.ndir, len(cells)), dtype=np.float64)
    for i in range(prob.ndir):
        n_i = prob.dirs[i]
        s = shift_signs(n_i)
        for bx, by, bz, wgt in _taps(n_i, prob.dt, prob.dx):
            v = source_value(I[i], i, prob, cells[:, 0] - bz * s[2],
                             cells[:, 1] - by * s[1], cells[:, 2] - bx * s[0])
            out[i] += wgt * v
    return out


def boundary_fluxes(I: np.ndarray, prob) -> Tuple[np.ndarray, float]:
    """Energy that one streaming step carries out of and into the box.

    Outflux: the pull of eq. (interp), evaluated at destination points just
    outside the box with in-box sources only, summed per face; a destination
    outside along several axes is booked on the first of them in the order
    x, y, z.  Influx: the part of the in-box streamed populations that came
    from inflow ghost values.  Intended for small boxes."""
    out = np.zeros(6, dtype=np.float64)
    influx = 0.0
    sizes = (prob.nz, prob.ny, prob.nx)
    periodic = [prob.bc[_AXIS_FACES[a][0]] == BC_PERIODIC for a in range(3)]
    ranges = [np.arange(0, sizes[a]) if periodic[a] else np.arange(-1, sizes[a] + 1)
              for a in range(3)]
    dz, dy, dxx = np.meshgrid(*ranges, indexing="ij")
    outside = [(c < 0) | (c >= sizes[a]) for a, c in enumerate((dz, dy, dxx))]
    for i in range(prob.ndir):
        n_i = prob.dirs[i]
        s = shift_signs(n_i)
        D = np.zeros(dz.shape)
        for bx, by, bz, wgt in _taps(n_i, prob.dt, prob.dx):
            D += wgt * source_value(I[i], i, prob, dz - bz * s[2], dy - by * s[1],
                                    dxx - bx * s[0], ghosts=False)
        booked = np.zeros(dz.shape, dtype=bool)
        for a in (2, 1, 0):                       # x, then y, then z
            c = (dz, dy, dxx)[a]
            lo, hi = _AXIS_FACES[a]
            m_lo = outside[a] & (c < 0) & ~booked
            m_hi = outside[a] & (c >= sizes[a]) & ~booked
            out[lo] += D[m_lo].sum()
            out[hi] += D[m_hi].sum()
            booked |= outside[a]
        if any(p.direction == i for p in prob.inflow):
            full = stream_direction(I[i], i, prob, ghosts=True)
            none = stream_direction(I[i], i, prob, ghosts=False)
            influx += float((full - none).sum())
    return out, influx


# ---------------------------------------------------------------------------
# Moments (Sec. 3.2, eqs. moments_discrete and higher_moments)
# ---------------------------------------------------------------------------
def moments(I: np.ndarray, dirs: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    E = np.zeros(I.shape[1:], dtype=np.float64)
    F = np.zeros((3,) + I.shape[1:], dtype=np.float64)
    for i in range(I.shape[0]):
        E += I[i]
        for a in range(3):
            F[a] += dirs[i, a] * I[i]
    return E, F


def second_moment(I: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    P = np.zeros((3, 3) + I.shape[1:], dtype=np.float64)
    for i in range(I.shape[0]):
        for a in range(3):
            for b in range(3):
                P[a, b] += dirs[i, a] * dirs[i, b] * I[i]
    return P


def total_energy(I: np.ndarray) -> float:
    return float(np.sum(I, dtype=np.float64))


# ---------------------------------------------------------------------------
# Collisions (Sec. 3.3 and App. B)
# ---------------------------------------------------------------------------
def _f64(a):
    return np.asarray(a, dtype=np.float64)


def collide_implicit(Istar, dirs, w, kappa_a, kappa_0, eta, dt, lam=0.0):
    """Exact solution of eq. (rte_implicit) in every cell.

    With E, F the new-time moments, each population obeys
        I_i (1 + dt (k0 + ka)) = I*_i + dt w_i (k0 (E + lam n_i.F) + eta),
    so every I_i is affine in the four unknowns (E, F).  Taking the
    moments of these N equations gives a 4x4 linear system for (E, F),
    whose coefficients are the quadrature sums sum w_i, sum w_i n_i and
    sum w_i n_i n_i (no isotropy of the rule is assumed).  The system is
    solved per cell with a library solver and the populations follow."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    c = 1.0 / (1.0 + dt * (k0 + ka))
    S0 = 0.0
    S1 = np.zeros(3)
    S2 = np.zeros((3, 3))
    for i in range(len(w)):
        S0 += w[i]
        S1 += w[i] * dirs[i]
        S2 += w[i] * np.outer(dirs[i], dirs[i])
    M = np.zeros((4, 4))
    M[0, 0] = S0
    M[0, 1:] = lam * S1
    M[1:, 0] = S1
    M[1:, 1:] = lam * S2
    Estar, Fstar = moments(Istar, dirs)
    shp = Estar.shape
    # Multiplied through by 1 + dt (k0 + ka), the moment equations read
    #   [(1 + dt ka) I4 + dt k0 (I4 - M)] (E, F) = (E* + dt eta S0, F* + dt eta S1);
    # forming I4 - M once keeps large dt k0 from cancelling against 1.
    IM = np.eye(4) - M
    A = ((1.0 + dt * ka).reshape(-1)[:, None, None] * np.eye(4)[None]
         + (dt * k0).reshape(-1)[:, None, None] * IM[None])
    rhs = np.empty((Estar.size, 4))
    rhs[:, 0] = (Estar + dt * et * S0).reshape(-1)
    for a in range(3):
        rhs[:, 1 + a] = (Fstar[a] + dt * et * S1[a]).reshape(-1)
    sol = np.linalg.solve(A, rhs[..., None])[..., 0]
    E = sol[:, 0].reshape(shp)
    F = sol[:, 1:].T.reshape((3,) + shp)
    out = np.empty_like(Istar)
    for i in range(len(w)):
        ndotF = dirs[i, 0] * F[0] + dirs[i, 1] * F[1] + dirs[i, 2] * F[2]
        out[i] = c * (Istar[i] + dt * w[i] * (k0 * (E + lam * ndotF) + et))
    return out


def collide_explicit(Istar, dirs, w, kappa_a, kappa_0, eta, dt, lam=0.0):
    """Eq. (collision-step) with I^eq and S from eq. (source-and-equil),
    all evaluated on the streamed populations."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    Estar, Fstar = moments(Istar, dirs)
    out = np.empty_like(Istar)
    for i in range(len(w)):
        ndotF = dirs[i, 0] * Fstar[0] + dirs[i, 1] * Fstar[1] + dirs[i, 2] * Fstar[2]
        Ieq = w[i] * (Estar + lam * ndotF)
        S = w[i] * et - ka * Istar[i]
        out[i] = Istar[i] - k0 * dt * (Istar[i] - Ieq) + dt * S
    return out


def collide_lambda(Istar, dirs, w, kappa_a, kappa_0, eta, dt, lam=0.0, cycles=5,
                   return_moments=False):
    """Lambda iteration (Sec. 3.3, list 1.-4.) run for a fixed number of cycles.

    1. guess (E, F) = moments of the streamed populations;
    2. solve each decoupled equation of eq. (rte_implicit) for I_i with
       (E, F) held fixed;
    3. recompute (E, F) from these I_i;
    4. repeat."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    c = 1.0 / (1.0 + dt * (k0 + ka))
    E, F = moments(Istar, dirs)
    out = np.empty_like(Istar)
    for _ in range(cycles):
        for i in range(len(w)):
            ndotF = dirs[i, 0] * F[0] + dirs[i, 1] * F[1] + dirs[i, 2] * F[2]
            out[i] = c * (Istar[i] + dt * w[i] * (k0 * (E + lam * ndotF) + et))
        E, F = moments(out, dirs)
    if return_moments:
        return out, E, F
    return out


def fluid_frame_J(E, F, P, v):
    """Eq. (J): J = W^2 (E - 2 F^i v_i + P^ij v_i v_j)."""
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    W2 = 1.0 / (1.0 - v2)
    Fv = F[0] * v[0] + F[1] * v[1] + F[2] * v[2]
    Pvv = np.zeros_like(E)
    for a in range(3):
        for b in range(3):
            Pvv += P[a, b] * v[a] * v[b]
    return W2 * (E - 2.0 * Fv + Pvv)


def fluid_frame_H(E, F, P, v):
    """Eq. (J), second line:
        H_j = W^3 (F^i v_i - E) v_j + W h_ji F^i - W h_ji v_k P^ik,
        h_ij = W^2 v_i v_j + delta_ij  (projector orthogonal to the fluid),
    and the time component from the orthogonality of H to the fluid
    four-velocity (coupling list, item 4), taken as the contravariant one:
    H^mu u_mu = 0 with u_mu = W (-1, v) (flat metric, signature - + + +,
    c = 1) gives H_0 = v^j H_j.  With it S_0 of ``four_force`` is the rate at
    which the collision takes energy from the radiation (the covariant
    component, -v^j H_j, would flip the sign of the flux term).
    Returns (H_0, H_x, H_y, H_z) stacked on a leading axis of 4."""
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    W = 1.0 / np.sqrt(1.0 - v2)
    Fv = F[0] * v[0] + F[1] * v[1] + F[2] * v[2]
    H = np.zeros((4,) + np.shape(E), dtype=np.float64)
    for j in range(3):
        Hj = W ** 3 * (Fv - E) * v[j]
        for i in range(3):
            h_ji = W ** 2 * v[j] * v[i] + (1.0 if i == j else 0.0)
            Hj = Hj + W * h_ji * F[i]
            for k in range(3):
                Hj = Hj - W * h_ji * v[k] * P[i, k]
        H[1 + j] = Hj
    H[0] = v[0] * H[1] + v[1] * H[2] + v[2] * H[3]
    return H


def four_force(J, H, v, kappa_a, kappa_0, eta, lam=0.0):
    """The radiative sources of the coupling list (Sec. 5, item 4):
        S_0 = W (ka J - eta) + k H_0,   S_j = W (ka J - eta) v_j + k H_j,
    fluid-frame ka, eta, with k = ka + k_s and k_s = k_0 - k_1 / 3 as the
    list defines it; k_1 = lam k_0 / 3 (lam = 3 k_1 / k_0, eq. rte_gray_bgkform),
    so k = ka + k_0 (1 - lam / 9).  Returns (S_0, S_x, S_y, S_z)."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    W = 1.0 / np.sqrt(1.0 - v2)
    k = ka + (k0 - (lam * k0 / 3.0) / 3.0)
    G = W * (ka * J - et)
    S = np.zeros((4,) + np.shape(J), dtype=np.float64)
    S[0] = G + k * H[0]
    for j in range(3):
        S[1 + j] = G * v[j] + k * H[1 + j]
    return S


def coupling(I, dirs, vel=None, kappa_a=None, kappa_0=None, eta=None, lam=0.0):
    """What the coupling loop of Sec. 5 takes from a state (items 3 and 4):
    the lab-frame moments E, F^i, P^ij (eqs. moments_discrete and
    higher_moments), the fluid-frame J and H_mu (eq. J), and the sources
    S_0, S_j.  vel None is a fluid at rest.  The sources need the
    fluid-frame kappa_a, kappa_0 (= kappa_s) and eta; without them S is None.
    P is returned as its six components xx, xy, xz, yy, yz, zz."""
    E, F = moments(I, dirs)
    P = second_moment(I, dirs)
    v = np.zeros((3,) + E.shape) if vel is None else _f64(vel)
    J = fluid_frame_J(E, F, P, v)
    H = fluid_frame_H(E, F, P, v)
    S = None
    if kappa_a is not None:
        S = four_force(J, H, v, kappa_a, kappa_0, eta, lam)
    P6 = np.stack([P[0, 0], P[0, 1], P[0, 2], P[1, 1], P[1, 2], P[2, 2]])
    return {"E": E, "F": F, "P": P6, "J": J, "H": H, "S": S}


def collide_moving(Istar, dirs, w, kappa_a, kappa_0, eta, vel, dt):
    """Implicit step of the mixed-frame equation at the end of App. B.

    Fluid-frame kappa_a, kappa_0 and eta; lab-frame populations.  With
    D_i = 1 - v.n_i and W the Lorentz factor, each population obeys
        I_i (1 + dt W D_i (ka + k0)) = I*_i + dt w_i (eta + k0 J) / (W^3 D_i^3),
    J being the fluid-frame energy density of the new populations, eq. (J).
    Every I_i is affine in J, I_i = p_i + q_i J; J of these is affine in J
    too, J = X + Y J, which is solved for J."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    v = _f64(vel)
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    W = 1.0 / np.sqrt(1.0 - v2)
    p = np.empty_like(Istar)
    q = np.empty_like(Istar)
    for i in range(len(w)):
        D = 1.0 - (v[0] * dirs[i, 0] + v[1] * dirs[i, 1] + v[2] * dirs[i, 2])
        a = 1.0 / (1.0 + dt * W * D * (ka + k0))
        p[i] = a * (Istar[i] + dt * w[i] * et / (W ** 3 * D ** 3))
        q[i] = a * dt * w[i] * k0 / (W ** 3 * D ** 3)
    Ep, Fp = moments(p, dirs)
    Pp = second_moment(p, dirs)
    Eq, Fq = moments(q, dirs)
    Pq = second_moment(q, dirs)
    X = fluid_frame_J(Ep, Fp, Pp, v)
    Y = fluid_frame_J(Eq, Fq, Pq, v)
    J = X / (1.0 - Y)
    return p + q * J[None]


# ---------------------------------------------------------------------------
# One step and a run
# ---------------------------------------------------------------------------
def collide(Istar, prob, collision=None):
    coll = prob.collision if collision is None else collision
    if prob.vel is not None:
        return collide_moving(Istar, prob.dirs, prob.weights, prob.kappa_a,
                              prob.kappa_s, prob.eta, prob.vel, prob.dt)
    args = (Istar, prob.dirs, prob.weights, prob.kappa_a, prob.kappa_s, prob.eta, prob.dt)
    if coll == COLL_IMPLICIT:
        return collide_implicit(*args, lam=prob.lam)
    if coll == COLL_EXPLICIT:
        return collide_explicit(*args, lam=prob.lam)
    if coll == COLL_LAMBDA:
        return collide_lambda(*args, lam=prob.lam, cycles=prob.lambda_iters)
    raise ValueError(f"unknown collision {coll}")


def step(I: np.ndarray, prob, collision=None) -> np.ndarray:
    """One stream-then-collide step (Sec. 3.3): returns I at t + dt."""
    return collide(stream(I, prob), prob, collision)


def run(prob, steps: Optional[int] = None, I0: Optional[np.ndarray] = None,
        collision=None, callback=None) -> np.ndarray:
    I = np.array(prob.I0 if I0 is None else I0, dtype=np.float64, copy=True)
    nsteps = prob.steps if steps is None else steps
    for k in range(nsteps):
        if callback is not None:
            callback(k, I)
        I = step(I, prob, collision)
    return I


def step_cells(I: np.ndarray, prob, cells: np.ndarray, collision=None) -> np.ndarray:
    """I at t + dt at selected cells only (for boxes too large for a full step).

    The collision is local, so streaming the selected cells and colliding
    them with their own coefficients gives the same values as a full step."""
    cells = np.asarray(cells, dtype=np.int64)
    Istar = stream_cells(I, prob, cells)[:, :, None, None]    # [dir, k, 1, 1]
    sel = lambda f: np.asarray(f)[cells[:, 0], cells[:, 1], cells[:, 2]][:, None, None]

    class _Local:
        pass
    loc = _Local()
    loc.dirs, loc.weights, loc.dt, loc.lam = prob.dirs, prob.weights, prob.dt, prob.lam
    loc.collision, loc.lambda_iters = prob.collision, prob.lambda_iters
    loc.kappa_a, loc.kappa_s, loc.eta = sel(prob.kappa_a), sel(prob.kappa_s), sel(prob.eta)
    loc.vel = None
    if prob.vel is not None:
        loc.vel = np.stack([sel(prob.vel[a]) for a in range(3)])
    return collide(Istar, loc, collision)[:, :, 0, 0]


# ---------------------------------------------------------------------------
# Adjoint of a run (gradient of a detected energy)
# ---------------------------------------------------------------------------
def detector_weights(prob, face: int = FACE_PX) -> np.ndarray:
    """Weights d with L(I) = sum d * I for the energy that one streaming step
    carries out through ``face`` (the face entry of ``boundary_fluxes``).

    By eq. (interp) a population on a face cell sends the fraction
    dt |n_i^a| / dx across the face of axis a it points out of.  A corner or
    edge cell can send energy out along several axes; such energy is booked
    on the first of them in the order x, y, z (the reading used for the face
    fluxes).  So the weight on face axis a is dt |n_i^a| / dx times
    (1 - dt |n_i^b| / dx) for every earlier axis b whose face the cell also
    leaves through (non-periodic b), and 0 off the face or for directions
    that do not leave through it."""
    axis = {FACE_MX: 2, FACE_PX: 2, FACE_MY: 1, FACE_PY: 1, FACE_MZ: 0, FACE_PZ: 0}[face]
    sizes = (prob.nz, prob.ny, prob.nx)
    comp_of_axis = {2: 0, 1: 1, 0: 2}          # array axis -> component of n
    d = np.zeros((prob.ndir, prob.nz, prob.ny, prob.nx))
    if prob.bc[face] == BC_PERIODIC:
        return d
    coords = np.meshgrid(np.arange(prob.nz), np.arange(prob.ny), np.arange(prob.nx),
                         indexing="ij")
    for i in range(prob.ndir):
        n_i = prob.dirs[i]
        nc = n_i[comp_of_axis[axis]]
        leaving = nc < 0 if face % 2 == 0 else nc > 0
        if not leaving:
            continue
        on_face = coords[axis] == (0 if face % 2 == 0 else sizes[axis] - 1)
        wgt = np.where(on_face, prob.dt * abs(nc) / prob.dx, 0.0)
        for b in (2, 1, 0):                    # earlier axes in the order x, y, z
            if b == axis:
                break
            lo, hi = _AXIS_FACES[b]
            if prob.bc[lo] == BC_PERIODIC:
                continue
            nb = n_i[comp_of_axis[b]]
            if nb == 0.0:
                continue
            out_b = coords[b] == (sizes[b] - 1 if nb > 0 else 0)
            wgt = np.where(out_b, wgt * (1.0 - prob.dt * abs(nb) / prob.dx), wgt)
        d[i] = wgt
    return d


def stream_transpose(nu: np.ndarray, prob) -> np.ndarray:
    """Transpose of the streaming map I -> I* with vacuum ghosts.

    The pull of eq. (interp) writes I*_i(r) = sum_b w_b I_i(r - b.s_i), so its
    transpose scatters each streamed value back to the cells it was pulled
    from: out_i(r - b.s_i) += w_b nu_i(r).  Sources outside the box are ghost
    values, not state, and receive nothing (periodic axes wrap).  Written as
    that scatter, tap by tap, so it is checked against ``stream`` by the
    identity <A x, y> = <x, A^T y>."""
    out = np.zeros_like(nu, dtype=np.float64)
    zz, yy, xx = np.meshgrid(np.arange(prob.nz), np.arange(prob.ny), np.arange(prob.nx),
                             indexing="ij")
    for i in range(prob.ndir):
        s = shift_signs(prob.dirs[i])
        for bx, by, bz, wgt in _taps(prob.dirs[i], prob.dt, prob.dx):
            (cz, cy, cx), (oz, oy, ox) = _wrap_and_flag(prob, zz - bz * s[2], yy - by * s[1],
                                                        xx - bx * s[0])
            inside = ~(oz | oy | ox)
            # one tap maps distinct cells to distinct sources (a shift, wrapped
            # on periodic axes), so a plain indexed add accumulates exactly
            out[i][cz[inside], cy[inside], cx[inside]] += wgt * nu[i][inside]
    return out


def _moving_terms(dirs, w, ka, k0, et, v, dt, Istar):
    """The affine form of the moving-fluid collision used by ``collide_moving``:
    I_i = p_i + q_i J with J = X / (1 - Y); returns its pieces."""
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    W = 1.0 / np.sqrt(1.0 - v2)
    n = len(w)
    D = np.stack([1.0 - (v[0] * dirs[i, 0] + v[1] * dirs[i, 1] + v[2] * dirs[i, 2])
                  for i in range(n)])
    a = 1.0 / (1.0 + dt * W * D * (ka + k0))
    c = np.stack([dt * w[i] / (W ** 3 * D[i] ** 3) for i in range(n)])
    p = a * (Istar + c * et)
    q = a * c * k0
    X = W ** 2 * np.sum(D ** 2 * p, axis=0)
    Y = W ** 2 * np.sum(D ** 2 * q, axis=0)
    return W, D, a, c, p, q, X, Y


def collide_moving_vjp(Istar, mu, dirs, w, kappa_a, kappa_0, eta, vel, dt):
    """Vector-Jacobian product of ``collide_moving`` at the streamed state
    Istar with the cotangent mu (both [dir, ...]).

    The collision is I_i = p_i + q_i J, J = X / (1 - Y), with
    a_i = 1 / (1 + dt W D_i (ka + k0)), p_i = a_i (I*_i + c_i eta),
    q_i = a_i c_i k0, c_i = dt w_i / (W^3 D_i^3), X = W^2 sum D_i^2 p_i and
    Y = W^2 sum D_i^2 q_i (the sums are eq. (J) written with D_i = 1 - v.n_i).
    Returns (nu = (dI/dI*)^T mu, and the cotangents of kappa_a, kappa_0, eta),
    by the chain rule through exactly these expressions."""
    ka, k0, et = _f64(kappa_a), _f64(kappa_0), _f64(eta)
    v = _f64(vel)
    W, D, a, c, p, q, X, Y = _moving_terms(dirs, w, ka, k0, et, v, dt, Istar)
    J = X / (1.0 - Y)
    # cotangents of J and of each p_i, q_i
    gJ = np.sum(mu * q, axis=0)
    gp = mu.copy()
    gq = mu * J
    # J = X / (1 - Y)
    gX = gJ / (1.0 - Y)
    gY = gJ * X / (1.0 - Y) ** 2
    gp = gp + gX * W ** 2 * D ** 2
    gq = gq + gY * W ** 2 * D ** 2
    # p_i = a_i (I*_i + c_i eta), q_i = a_i c_i k0
    nu = gp * a
    g_eta = np.sum(gp * a * c, axis=0)
    g_k0 = np.sum(gq * a * c, axis=0)
    ga = gp * (Istar + c * et) + gq * c * k0
    # a_i = 1 / (1 + dt W D_i (ka + k0)): da/dk = -a^2 dt W D_i for ka and k0
    dadk = -a ** 2 * dt * W * D
    g_ka = np.sum(ga * dadk, axis=0)
    g_k0 = g_k0 + g_ka
    return nu, g_ka, g_k0, g_eta


def detected_energy(prob, steps: int, face: int = FACE_PX, I0=None) -> float:
    """L = sum over the states I^0 .. I^(steps-1) entering each step of the
    energy that streams out through ``face`` (the detector of
    ``detector_weights``)."""
    d = detector_weights(prob, face)
    I = np.array(prob.I0 if I0 is None else I0, dtype=np.float64, copy=True)
    L = 0.0
    for _ in range(steps):
        L += float(np.sum(d * I))
        I = step(I, prob)
    return L


def detected_energy_gradient(prob, steps: int, face: int = FACE_PX, I0=None):
    """L of ``detected_energy`` and its gradient with respect to the per-cell
    kappa_a, kappa_s (= kappa_0) and eta, by reverse-mode differentiation of
    the run: lambda^n = d + S^T (dC/dI*)^T lambda^(n+1), lambda^steps = 0, where
    S is the streaming map and C the moving-fluid collision (a static fluid is
    the case v = 0).  Stores every state (small boxes only)."""
    vel = prob.vel if prob.vel is not None else np.zeros((3,) + prob.shape)
    d = detector_weights(prob, face)
    I = np.array(prob.I0 if I0 is None else I0, dtype=np.float64, copy=True)
    states = []
    L = 0.0
    for _ in range(steps):
        states.append(I)
        L += float(np.sum(d * I))
        I = collide_moving(stream(I, prob), prob.dirs, prob.weights, prob.kappa_a,
                           prob.kappa_s, prob.eta, vel, prob.dt)
    lam = np.zeros_like(I)
    g_ka = np.zeros(prob.shape)
    g_ks = np.zeros(prob.shape)
    g_eta = np.zeros(prob.shape)
    for n in range(steps - 1, -1, -1):
        Istar = stream(states[n], prob)
        nu, a1, a2, a3 = collide_moving_vjp(Istar, lam, prob.dirs, prob.weights, prob.kappa_a,
                                            prob.kappa_s, prob.eta, vel, prob.dt)
        g_ka += a1
        g_ks += a2
        g_eta += a3
        lam = d + stream_transpose(nu, prob)
    return L, g_ka, g_ks, g_eta
