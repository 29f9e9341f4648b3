"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None compares the oracle with itself:
each one checks it against a closed form, a brute-force solve, a library
routine (scipy's binomial law and Lebedev tables), an exact identity of the
discrete scheme, or a symmetry.
"""
import itertools
import os

import numpy as np
import pytest

import workloads as wl
from oracle import analytic
from oracle import lbrt_oracle as orc


def _problem(shape=(6, 7, 8), npoints=14, dt=0.5, bc=(wl.BC_OUTFLOW,) * 6, seed=0, **kw):
    p = wl.random_problem(seed, shape=shape, npoints=npoints, dt=dt, bc=bc, **kw)
    return p


# ---------------------------------------------------------------------------
# Quadrature (Sec. 3.2.1: eqs. iso-tensors, isotropy-cond, sph-quad-cond)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_theta,n_phi", [(2, 4), (6, 8), (8, 14), (10, 20)])
def test_gauss_legendre_product_exactness(n_theta, n_phi):
    """The product rule (Sec. 3.2.1) integrates every monomial of degree up
    to min(2 n_theta - 1, n_phi - 1) exactly (against the closed-form sphere
    averages), fails some monomial one degree higher, has positive weights
    summing to 1, and is centrally symmetric for even n_phi."""
    dirs, w = wl.gauss_legendre_product(n_theta, n_phi)
    p = wl.gauss_legendre_degree(n_theta, n_phi)
    assert len(w) == n_theta * n_phi and np.all(w > 0) and abs(w.sum() - 1.0) < 1e-14
    err = {}
    for a in range(p + 2):
        for b in range(p + 2 - a):
            for c in range(p + 2 - a - b):
                q = np.sum(w * dirs[:, 0] ** a * dirs[:, 1] ** b * dirs[:, 2] ** c)
                err[(a, b, c)] = abs(q - analytic.monomial_average(a, b, c))
    assert max(e for k, e in err.items() if sum(k) <= p) < 1e-14
    assert max(e for k, e in err.items() if sum(k) == p + 1) > 1e-6
    # central symmetry: -n_i is a node with the same weight
    for i in range(len(w)):
        j = int(np.argmin(np.linalg.norm(dirs + dirs[i], axis=1)))
        assert np.linalg.norm(dirs[j] + dirs[i]) < 1e-14 and w[j] == w[i]


@pytest.mark.parametrize("npoints", [6, 14, 26, 38, 50, 74, 86, 110, 146])
def test_lebedev_monomial_exactness(npoints):
    dirs, w = wl.lebedev(npoints)
    p = wl.lebedev_degree(npoints)
    assert abs(w.sum() - 1.0) < 1e-14
    worst = 0.0
    for a in range(p + 1):
        for b in range(p + 1 - a):
            for c in range(p + 1 - a - b):
                q = np.sum(w * dirs[:, 0] ** a * dirs[:, 1] ** b * dirs[:, 2] ** c)
                worst = max(worst, abs(q - analytic.monomial_average(a, b, c)))
    assert worst < 2e-15
    # the degree is tight: some monomial of degree p + 1 is not integrated exactly
    fails = [abs(np.sum(w * dirs[:, 0] ** a * dirs[:, 1] ** b * dirs[:, 2] ** c)
                 - analytic.monomial_average(a, b, c))
             for a in range(p + 2) for b in range(p + 2 - a) for c in [p + 1 - a - b]]
    assert max(fails) > 1e-9


@pytest.mark.parametrize("npoints", [14, 50, 110, 146])
def test_isotropy_tensors_low_rank(npoints):
    dirs, w = wl.lebedev(npoints)
    assert abs(np.sum(w) - 1) < 1e-14
    assert np.max(np.abs(w @ dirs)) < 1e-15
    T2 = np.einsum("i,ia,ib->ab", w, dirs, dirs)
    assert np.max(np.abs(T2 - np.eye(3) / 3.0)) < 1e-15
    T3 = np.einsum("i,ia,ib,ic->abc", w, dirs, dirs, dirs)
    assert np.max(np.abs(T3)) < 1e-15


# ---------------------------------------------------------------------------
# Streaming (Sec. 3.3, eq. interp)
# ---------------------------------------------------------------------------
def test_tap_weights_partition_of_unity():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        dt = rng.uniform(0.0, 1.0)
        taps = orc._taps(n, dt, 1.0)
        assert abs(sum(t[3] for t in taps) - 1.0) < 1e-15
        for t in taps:
            assert t[3] > 0.0


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1, -1])
def test_exact_shift_at_unit_cfl(axis, sign):
    """dt = dx and an axis direction: the pull is an exact one-cell shift
    (Sec. 4.1.1, reduced streaming formula)."""
    p = _problem(shape=(5, 6, 7), npoints=6, dt=1.0, bc=(wl.BC_PERIODIC,) * 6)
    target = np.zeros(3)
    target[axis] = sign
    i = wl.nearest_direction(p.dirs, target)
    out = orc.stream_direction(p.I0[i], i, p)
    arr_axis = 2 - axis
    assert np.array_equal(out, np.roll(p.I0[i], sign, axis=arr_axis))


@pytest.mark.parametrize("dt", [0.5, 0.3, 1.0])
@pytest.mark.parametrize("npoints,target", [(26, (1, 1, 1)), (26, (1, -1, 0)),
                                            (110, (1, 1, 0)), (50, (-1, 0, 0)),
                                            (146, (0.3, -0.5, 0.8))])
def test_pure_streaming_is_binomial_product(dt, npoints, target):
    dirs, w = wl.lebedev(npoints)
    i = wl.nearest_direction(dirs, target)
    nsteps = 7
    shape = (17, 17, 17)
    origin = (8, 8, 8)
    p = wl.random_problem(0, shape=shape, npoints=npoints, dt=dt)
    p.kappa_a[:] = 0
    p.kappa_s[:] = 0
    p.eta[:] = 0
    I = np.zeros_like(p.I0)
    I[i][origin] = 1.0
    for _ in range(nsteps):
        I = orc.step(I, p)
    ref = analytic.binomial_green(nsteps, dirs[i], dt, 1.0, shape, origin)
    assert np.max(np.abs(I[i] - ref)) < 1e-15
    others = np.delete(I, i, axis=0)
    assert np.max(np.abs(others)) == 0.0


def test_periodic_streaming_conserves_each_direction():
    p = _problem(shape=(9, 10, 11), npoints=50, dt=0.7, bc=(wl.BC_PERIODIC,) * 6)
    out = orc.stream(p.I0, p)
    s0 = p.I0.reshape(p.ndir, -1).sum(axis=1)
    s1 = out.reshape(p.ndir, -1).sum(axis=1)
    assert np.max(np.abs(s1 - s0) / s0) < 1e-14


@pytest.mark.parametrize("bc", [
    (wl.BC_OUTFLOW,) * 6,
    (wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC),
    (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW),
])
def test_streaming_energy_budget(bc):
    """sum I* = sum I - outflux + influx, exactly (partition of unity)."""
    p = _problem(shape=(5, 6, 7), npoints=26, dt=0.6, bc=bc, inflow_planes=5)
    out, influx = orc.boundary_fluxes(p.I0, p)
    Istar = orc.stream(p.I0, p)
    lhs = Istar.sum()
    rhs = p.I0.sum() - out.sum() + influx
    assert abs(lhs - rhs) < 1e-13 * p.I0.sum()
    if wl.BC_INFLOW in bc:
        assert influx > 0
    if all(b == wl.BC_PERIODIC for b in bc):
        assert out.sum() == 0


def test_outflux_corner_worked_example():
    """A unit population on the far corner moving along (+,+,+): the
    definition books dt|n^x| on +x, (1 - dt|n^x|) dt|n^y| on +y and
    (1 - dt|n^x|)(1 - dt|n^y|) dt|n^z| on +z."""
    p = _problem(shape=(4, 4, 4), npoints=26, dt=0.5)
    i = wl.nearest_direction(p.dirs, (1, 1, 1))
    n = p.dirs[i]
    I = np.zeros_like(p.I0)
    I[i, 3, 3, 3] = 1.0
    out, influx = orc.boundary_fluxes(I, p)
    dx_, dy_, dz_ = 0.5 * abs(n[0]), 0.5 * abs(n[1]), 0.5 * abs(n[2])
    assert abs(out[wl.FACE_PX] - dx_) < 1e-16
    assert abs(out[wl.FACE_PY] - (1 - dx_) * dy_) < 1e-16
    assert abs(out[wl.FACE_PZ] - (1 - dx_) * (1 - dy_) * dz_) < 1e-16
    assert out[wl.FACE_MX] == out[wl.FACE_MY] == out[wl.FACE_MZ] == 0.0
    assert influx == 0.0


@pytest.mark.parametrize("bc", [
    (wl.BC_OUTFLOW,) * 6,
    (wl.BC_PERIODIC, wl.BC_PERIODIC) + (wl.BC_OUTFLOW,) * 4,
    (wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC),
])
def test_detector_weights_give_the_face_outflux(bc):
    """The adjoint's detector weights d (one linear functional per face)
    reproduce the face entries of boundary_fluxes, which evaluates the pull
    at destinations outside the box: sum d * I equals the booked outflux on
    every face, including edge and corner cells (first of x, y, z)."""
    p = _problem(shape=(5, 6, 7), npoints=26, dt=0.7, bc=bc)
    out, _ = orc.boundary_fluxes(p.I0, p)
    for face in range(6):
        d = orc.detector_weights(p, face)
        got = float(np.sum(d * p.I0))
        assert abs(got - out[face]) < 1e-14 * p.I0.sum(), (face, got, out[face])
        if bc[face] == wl.BC_PERIODIC:
            assert not d.any()


def test_inflow_ghost_enters_by_its_weight():
    """Sec. 4.1.1 beam injection: a unit ghost value on face -x for direction
    +x reaches the first layer with weight dt |n^x| / dx and nothing else."""
    p = _problem(shape=(3, 4, 5), npoints=14, dt=0.4,
                 bc=(wl.BC_INFLOW,) + (wl.BC_OUTFLOW,) * 5)
    i = wl.nearest_direction(p.dirs, (1, 0, 0))
    vals = np.zeros((3, 4), dtype=np.float32)
    vals[1, 2] = 1.0
    p.inflow = [wl.InflowPlane(wl.FACE_MX, i, vals)]
    I = np.zeros_like(p.I0)
    out = orc.stream(I, p)
    ref = np.zeros_like(out)
    ref[i, 1, 2, 0] = 0.4
    assert np.array_equal(out, ref)


# ---------------------------------------------------------------------------
# Moments (Sec. 3.2, eq. moments_discrete)
# ---------------------------------------------------------------------------
def test_moments_of_polynomial_fields():
    """I_i = w_i (a + b.n_i + n_i.C.n_i) has E = a + tr(C)/3 and F = b/3."""
    dirs, w = wl.lebedev(50)
    rng = np.random.default_rng(3)
    a = rng.uniform(1, 2, size=(2, 3, 4))
    b = rng.standard_normal((3, 2, 3, 4))
    C = rng.standard_normal((3, 3))
    I = np.empty((50, 2, 3, 4))
    for i in range(50):
        I[i] = w[i] * (a + np.tensordot(dirs[i], b, axes=(0, 0)) + dirs[i] @ C @ dirs[i])
    E, F = orc.moments(I, dirs)
    assert np.max(np.abs(E - (a + np.trace(C) / 3))) < 1e-14
    assert np.max(np.abs(F - b / 3)) < 1e-14


# ---------------------------------------------------------------------------
# Collisions (Sec. 3.3, App. B)
# ---------------------------------------------------------------------------
def _random_collision_inputs(npoints=26, shape=(2, 2, 3), seed=7, kmax=3.0):
    dirs, w = wl.lebedev(npoints)
    rng = np.random.default_rng(seed)
    Istar = rng.uniform(0, 1, size=(npoints,) + shape) * w[:, None, None, None]
    ka = 10 ** rng.uniform(-2, kmax, size=shape)
    k0 = 10 ** rng.uniform(-2, kmax, size=shape)
    eta = 10 ** rng.uniform(-2, kmax, size=shape)
    return dirs, w, Istar, ka, k0, eta


@pytest.mark.parametrize("lam", [0.0, 0.5, -0.25])
@pytest.mark.parametrize("npoints", [14, 26, 50])
def test_implicit_matches_dense_solve(lam, npoints):
    """The N x N system of eq. (rte_implicit), built and solved densely."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(npoints)
    dt = 0.5
    got = orc.collide_implicit(Istar, dirs, w, ka, k0, eta, dt, lam)
    N = npoints
    for idx in np.ndindex(ka.shape):
        A = np.eye(N) * (1 + dt * (k0[idx] + ka[idx]))
        A -= dt * k0[idx] * np.outer(w, np.ones(N)) * (1 + lam * dirs @ dirs.T)
        rhs = Istar[(slice(None),) + idx] + dt * w * eta[idx]
        ref = np.linalg.solve(A, rhs)
        sl = (slice(None),) + idx
        assert np.max(np.abs(got[sl] - ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("lam", [0.0, 0.5, -0.25])
def test_implicit_moments_closed_form(lam):
    """With a rule exact to degree 2, the moments of eq. (rte_implicit) solve to
    E = (E* + dt eta)/(1 + dt ka) and F = F*/(1 + dt(k0 + ka) - dt k0 lam/3)."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(50, shape=(3, 3, 3), kmax=5)
    dt = 0.5
    out = orc.collide_implicit(Istar, dirs, w, ka, k0, eta, dt, lam)
    Es, Fs = orc.moments(Istar, dirs)
    E, F = orc.moments(out, dirs)
    # The oracle solves the system with the rule's actual sum w_i = 1 + O(1e-16);
    # that rounding is amplified by dt k0 / (1 + dt ka) in E.
    tol = 1e-14 + 1e-15 * (1 + dt * k0) / (1 + dt * ka)
    assert np.all(np.abs(E / ((Es + dt * eta) / (1 + dt * ka)) - 1) < tol)
    Fref = Fs / (1 + dt * (k0 + ka) - dt * k0 * lam / 3)
    # F = sum n_i I_i cancels terms of size E: rounding is relative to E.
    assert np.all(np.abs(F - Fref) < 1e-14 * (np.abs(E) + np.abs(Fs)))


def test_lambda_iteration_converges_to_implicit():
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(26, kmax=0.5)
    dt = 0.5
    ref = orc.collide_implicit(Istar, dirs, w, ka, k0, eta, dt, 0.3)
    got = orc.collide_lambda(Istar, dirs, w, ka, k0, eta, dt, 0.3, cycles=200)
    assert np.max(np.abs(got - ref) / ref) < 1e-12


def test_lambda_absorption_only_converges_in_one_cycle():
    """Sec. 4.2.1 reports convergence within three cycles in the shadow test
    (absorption only): with kappa_0 = 0 the first cycle is already exact."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(26, kmax=7)
    k0 = np.zeros_like(k0)
    ka = np.full_like(ka, 1e7)
    dt = 0.2
    ref = orc.collide_implicit(Istar, dirs, w, ka, k0, eta, dt)
    got = orc.collide_lambda(Istar, dirs, w, ka, k0, eta, dt, cycles=1)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-14


def test_lambda_moments_follow_geometric_recursion():
    """Each cycle maps E -> c (E* + dt (k0 E + eta)) (rule exact to degree 1),
    so E_K = E_inf + (E* - E_inf) (c dt k0)^K."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(50, kmax=1)
    dt = 0.5
    for K in (1, 2, 5):
        _, E, _ = orc.collide_lambda(Istar, dirs, w, ka, k0, eta, dt, cycles=K,
                                     return_moments=True)
        Es, _ = orc.moments(Istar, dirs)
        c = 1 / (1 + dt * (k0 + ka))
        Einf = (Es + dt * eta) / (1 + dt * ka)
        ref = Einf + (Es - Einf) * (c * dt * k0) ** K
        assert np.max(np.abs(E / ref - 1)) < 1e-13


@pytest.mark.parametrize("lam", [0.5, -0.9])
def test_lambda_flux_follows_geometric_recursion(lam):
    """With lambda != 0 each cycle maps F -> c (F* + dt k0 lam F / 3) (the
    rule integrates n n^T to I / 3 and n to 0), so at a finite cycle count
    F_K = F_inf + (F* - F_inf) a^K with a = c dt k0 lam / 3 and
    F_inf = c F* / (1 - a); E follows the lambda = 0 recursion unchanged."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(50, kmax=1)
    dt = 0.5
    Es, Fs = orc.moments(Istar, dirs)
    c = 1 / (1 + dt * (k0 + ka))
    a = c * dt * k0 * lam / 3
    Finf = c * Fs / (1 - a)
    Einf = (Es + dt * eta) / (1 + dt * ka)
    for K in (1, 2, 3, 5):
        _, E, F = orc.collide_lambda(Istar, dirs, w, ka, k0, eta, dt, lam, cycles=K,
                                     return_moments=True)
        Fref = Finf + (Fs - Finf) * a ** K
        assert np.all(np.abs(F - Fref) < 1e-13 * (np.abs(Es) + np.abs(Fs)))
        Eref = Einf + (Es - Einf) * (c * dt * k0) ** K
        assert np.max(np.abs(E / Eref - 1)) < 1e-13


def test_explicit_properties():
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(50, kmax=0)
    dt = 0.3
    lam = 0.4
    Es, Fs = orc.moments(Istar, dirs)
    # pure scattering conserves E; F relaxes by (1 - dt k0 (1 - lam/3))
    out = orc.collide_explicit(Istar, dirs, w, 0 * ka, k0, 0 * eta, dt, lam)
    E, F = orc.moments(out, dirs)
    assert np.max(np.abs(E / Es - 1)) < 1e-14
    assert np.max(np.abs(F - Fs * (1 - dt * k0 + dt * k0 * lam / 3))) < 1e-14
    # pure absorption decays every population by (1 - dt ka); emission adds dt w eta
    out = orc.collide_explicit(Istar, dirs, w, ka, 0 * k0, eta, dt, lam)
    ref = Istar * (1 - dt * ka) + dt * w[:, None, None, None] * eta
    assert np.max(np.abs(out - ref)) < 1e-15


@pytest.mark.parametrize("coll", [orc.COLL_IMPLICIT, orc.COLL_EXPLICIT, orc.COLL_LAMBDA])
def test_isotropic_equilibrium_is_fixed_point(coll):
    """I_i = w_i B with eta = kappa_a B is unchanged by a full step on a
    periodic box, for any kappa_0 and lambda (Sec. 3.2, eq. source-and-equil)."""
    p = _problem(shape=(4, 5, 6), npoints=50, dt=0.5, bc=(wl.BC_PERIODIC,) * 6)
    B = 2.5
    p.eta = (p.kappa_a.astype(np.float64) * B)
    p.lam = 0.3
    I = np.broadcast_to(p.weights[:, None, None, None] * B, p.I0.shape).copy()
    out = orc.step(I, p, collision=coll)
    assert np.max(np.abs(out / I - 1)) < 1e-13


def test_moving_at_rest_equals_static():
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(50)
    dt = 0.5
    vel = np.zeros((3,) + ka.shape)
    a = orc.collide_moving(Istar, dirs, w, ka, k0, eta, vel, dt)
    b = orc.collide_implicit(Istar, dirs, w, ka, k0, eta, dt)
    assert np.max(np.abs(a - b) / b) < 1e-13


@pytest.mark.parametrize("npoints", [26, 50])
def test_moving_matches_dense_solve(npoints):
    """Dense N x N solve of the mixed-frame implicit equation (App. B) with
    J written as W^2 sum_j (1 - v.n_j)^2 I_j."""
    dirs, w, Istar, ka, k0, eta = _random_collision_inputs(npoints)
    rng = np.random.default_rng(11)
    v = rng.standard_normal((3,) + ka.shape)
    v *= rng.uniform(0, 0.7, size=ka.shape) / np.linalg.norm(v, axis=0)
    dt = 0.5
    got = orc.collide_moving(Istar, dirs, w, ka, k0, eta, v, dt)
    for idx in np.ndindex(ka.shape):
        vv = v[(slice(None),) + idx]
        W = 1 / np.sqrt(1 - vv @ vv)
        D = 1 - dirs @ vv
        A = np.diag(1 + dt * W * D * (ka[idx] + k0[idx]))
        A -= np.outer(dt * w * k0[idx] / (W ** 3 * D ** 3), W ** 2 * D ** 2)
        rhs = Istar[(slice(None),) + idx] + dt * w * eta[idx] / (W ** 3 * D ** 3)
        ref = np.linalg.solve(A, rhs)
        assert np.max(np.abs(got[(slice(None),) + idx] - ref) / ref) < 1e-12


@pytest.mark.parametrize("npoints,tol", [(110, 5e-6), (146, 1e-8)])
def test_moving_boosted_equilibrium_is_fixed_point(npoints, tol):
    """I_i = w_i B / (W^4 (1 - v.n_i)^4) with eta = kappa_a B has J = B in the
    continuum and is then a fixed point of the mixed-frame collision; on a
    rule of finite degree only up to its error on <(1 - v.n)^-2> = W^2."""
    dirs, w = wl.lebedev(npoints)
    shape = (1, 1, 4)
    B = 1.7
    vel = np.zeros((3,) + shape)
    vel[0, 0, 0, :] = [0.0, 0.2, 0.5, -0.4]
    vel[1, 0, 0, :] = [0.0, 0.1, 0.0, 0.2]
    ka = np.full(shape, 3.0)
    k0 = np.full(shape, 0.5)
    eta = ka * B
    W = 1 / np.sqrt(1 - (vel ** 2).sum(axis=0))
    I = np.empty((npoints,) + shape)
    for i in range(npoints):
        D = 1 - (dirs[i][:, None, None, None] * vel).sum(axis=0)
        I[i] = w[i] * B / (W ** 4 * D ** 4)
    out = orc.collide_moving(I, dirs, w, ka, k0, eta, vel, 0.5)
    assert np.max(np.abs(out / I - 1)) < tol


# ---------------------------------------------------------------------------
# Coupling moments and sources (Sec. 3.2 eq. higher_moments; Sec. 5 eq. J and
# coupling item 4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("npoints", [14, 50, 110])
def test_second_moment_identities(npoints):
    """P is symmetric with trace E (unit directions); an isotropic state
    I_i = w_i E0 has P = E0 / 3 delta (the rule's isotropy, eq. iso-tensors);
    a state in one direction has P = n n^T I."""
    dirs, w = wl.lebedev(npoints)
    rng = np.random.default_rng(npoints)
    I = rng.random((npoints, 3, 4, 5))
    P = orc.second_moment(I, dirs)
    E, _ = orc.moments(I, dirs)
    assert np.array_equal(P, P.transpose(1, 0, 2, 3, 4))
    assert np.max(np.abs(P[0, 0] + P[1, 1] + P[2, 2] - E)) < 1e-13 * E.max()
    E0 = rng.random((3, 4, 5))
    Piso = orc.second_moment(w[:, None, None, None] * E0[None], dirs)
    for a in range(3):
        for b in range(3):
            assert np.max(np.abs(Piso[a, b] - (E0 / 3 if a == b else 0.0))) < 1e-14
    k = npoints // 3
    one = np.zeros((npoints, 1, 1, 1))
    one[k] = 2.5
    np.testing.assert_allclose(orc.second_moment(one, dirs)[:, :, 0, 0, 0],
                               2.5 * np.outer(dirs[k], dirs[k]), rtol=0, atol=1e-15)


def _random_lab_moments(rng, n, vmax):
    E = rng.random(n) + 1.0
    F = rng.normal(size=(3, n)) * 0.3
    A = rng.normal(size=(3, 3, n)) * 0.2
    P = 0.5 * (A + A.transpose(1, 0, 2)) + np.eye(3)[:, :, None] * (E / 3)
    v = rng.normal(size=(3, n))
    v *= rng.uniform(0.0, vmax, n) / np.linalg.norm(v, axis=0)
    return E, F, P, v


def _covariant_JH(E, F, P, v):
    """J = T^mn u_m u_n and H^m = -h^m_a T^ab u_b, h^m_a = delta + u^m u_a,
    from the stress tensor T^00 = E, T^0i = F^i, T^ij = P^ij with the
    Minkowski metric diag(-1, 1, 1, 1)."""
    n = E.shape[0]
    T = np.zeros((4, 4, n))
    T[0, 0] = E
    T[0, 1:] = F
    T[1:, 0] = F
    T[1:, 1:] = P
    W = 1.0 / np.sqrt(1.0 - (v ** 2).sum(axis=0))
    u_up = np.concatenate([W[None], W * v])
    u_dn = u_up * np.array([-1.0, 1.0, 1.0, 1.0])[:, None]
    J = np.einsum("mnk,mk,nk->k", T, u_dn, u_dn)
    Tu = np.einsum("abk,bk->ak", T, u_dn)
    H_up = -(Tu + u_up * np.einsum("ak,ak->k", u_dn, Tu))
    return J, H_up, u_dn


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fluid_frame_moments_are_the_covariant_projection(seed):
    """Eq. (J) written out in E, F, P and v against the tensor projection of
    the radiation stress tensor onto the fluid four-velocity and its
    orthogonal complement; H_0 is the contravariant time component."""
    rng = np.random.default_rng(seed)
    E, F, P, v = _random_lab_moments(rng, 64, 0.95)
    J_ref, H_ref, u_dn = _covariant_JH(E, F, P, v)
    J = orc.fluid_frame_J(E, F, P, v)
    H = orc.fluid_frame_H(E, F, P, v)
    scale = np.abs(J_ref).max() + np.abs(H_ref).max()
    assert np.max(np.abs(J - J_ref)) < 1e-12 * scale
    assert np.max(np.abs(H - H_ref)) < 1e-12 * scale
    assert np.max(np.abs(np.einsum("ak,ak->k", H, u_dn))) < 1e-12 * scale


def test_boosted_isotropic_radiation():
    """T^mn = (4/3) J0 u^m u^n + (J0 / 3) g^mn, isotropic radiation of energy
    density J0 in the fluid frame seen from the lab: eq. (J) gives J = J0 and
    H = 0, and with eta = kappa_a J0 (radiative equilibrium) both sources
    vanish for any scattering opacity and lambda."""
    rng = np.random.default_rng(11)
    n = 32
    v = rng.normal(size=(3, n))
    v *= rng.uniform(0.0, 0.9, n) / np.linalg.norm(v, axis=0)
    W2 = 1.0 / (1.0 - (v ** 2).sum(axis=0))
    J0 = rng.uniform(0.5, 2.0, n)
    E = 4.0 / 3.0 * J0 * W2 - J0 / 3.0
    F = 4.0 / 3.0 * J0 * W2 * v
    P = 4.0 / 3.0 * J0 * W2 * v[:, None] * v[None, :] + np.eye(3)[:, :, None] * (J0 / 3.0)
    J = orc.fluid_frame_J(E, F, P, v)
    H = orc.fluid_frame_H(E, F, P, v)
    assert np.max(np.abs(J / J0 - 1.0)) < 1e-12
    assert np.max(np.abs(H)) < 1e-12 * np.max(J0 * W2)
    ka = rng.uniform(0.1, 5.0, n)
    for k0, lam in ((0.0, 0.0), (3.0, 0.0), (2.0, 0.5)):
        S = orc.four_force(J, H, v, ka, np.full(n, k0), ka * J0, lam)
        assert np.max(np.abs(S)) < 1e-11 * np.max(ka * J0 * W2)


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_sources_at_rest(lam):
    """v = 0: J = E, H_j = F_j, H_0 = 0, S_0 = kappa_a E - eta and
    S_j = (kappa_a + kappa_0 - kappa_1 / 3) F_j with kappa_1 = lam kappa_0 / 3."""
    p = _problem(npoints=26, seed=5, lam=lam)
    rng = np.random.default_rng(3)
    I = rng.random((p.ndir,) + p.shape)
    out = orc.coupling(I, p.dirs, None, p.kappa_a, p.kappa_s, p.eta, lam)
    E, F = out["E"], out["F"]
    assert np.array_equal(out["J"], E)
    assert np.max(np.abs(out["H"][1:] - F)) < 1e-15 * E.max()
    assert np.array_equal(out["H"][0], np.zeros_like(E))
    ka, k0 = p.kappa_a.astype(np.float64), p.kappa_s.astype(np.float64)
    np.testing.assert_allclose(out["S"][0], ka * E - p.eta, rtol=1e-14, atol=1e-14 * E.max())
    k = ka + k0 * (1.0 - lam / 9.0)
    for j in range(3):
        np.testing.assert_allclose(out["S"][1 + j], k * F[j], rtol=1e-13,
                                   atol=1e-14 * E.max() * k.max())


def test_sources_are_the_static_collision_exchange():
    """The implicit collision (eq. rte_implicit, lambda = 0, fluid at rest)
    evaluates its sink at the new time level, so what it takes from the
    radiation in one step is dt times the sources of the new state:
    E - E* = -dt S_0 and F - F* = -dt S_j."""
    p = _problem(shape=(4, 5, 6), npoints=50, seed=9)
    rng = np.random.default_rng(4)
    Istar = rng.random((p.ndir,) + p.shape) * p.weights[:, None, None, None]
    out = orc.collide_implicit(Istar, p.dirs, p.weights, p.kappa_a, p.kappa_s, p.eta, p.dt)
    Es, Fs = orc.moments(Istar, p.dirs)
    c = orc.coupling(out, p.dirs, None, p.kappa_a, p.kappa_s, p.eta)
    scale = np.abs(c["E"]).max() + p.dt * np.abs(c["S"]).max()
    assert np.max(np.abs(c["E"] - Es + p.dt * c["S"][0])) < 1e-13 * scale
    assert np.max(np.abs(c["F"] - Fs + p.dt * c["S"][1:])) < 1e-13 * scale


@pytest.mark.parametrize("npoints", [50, 146])
def test_sources_are_the_moving_collision_exchange(npoints):
    """The mixed-frame collision of App. B takes from the radiation, in one
    step, dt times the sources of the new state (the lab-frame four-force),
    except for the quadrature's error on the fluid-frame emission's lab
    energy and momentum, <(1 - v.n)^-3> = W^4 and <n (1 - v.n)^-3> = W^4 v:
        E - E* = -dt S_0 + dt (eta + k0 J) (Q / W^3 - W),
        F - F* = -dt S_j + dt (eta + k0 J) (Q_j / W^3 - W v_j),
    Q = sum_i w_i / D_i^3, Q_j = sum_i w_i n_ij / D_i^3 — an identity of the
    discrete scheme for any rule, which fixes the sign of H_0."""
    dirs, w = wl.lebedev(npoints)
    rng = np.random.default_rng(npoints)
    shape = (2, 3, 4)
    vel = rng.normal(size=(3,) + shape)
    vel *= rng.uniform(0.0, 0.6, shape) / np.linalg.norm(vel, axis=0)
    ka = rng.uniform(0.1, 3.0, shape)
    k0 = rng.uniform(0.0, 2.0, shape)
    eta = rng.uniform(0.0, 2.0, shape)
    dt = 0.5
    Istar = rng.random((npoints,) + shape) * w[:, None, None, None]
    out = orc.collide_moving(Istar, dirs, w, ka, k0, eta, vel, dt)
    Es, Fs = orc.moments(Istar, dirs)
    c = orc.coupling(out, dirs, vel, ka, k0, eta)
    W = 1.0 / np.sqrt(1.0 - (vel ** 2).sum(axis=0))
    Q = np.zeros(shape)
    Qj = np.zeros((3,) + shape)
    for i in range(npoints):
        D = 1.0 - (dirs[i][:, None, None, None] * vel).sum(axis=0)
        Q += w[i] / D ** 3
        Qj += w[i] * dirs[i][:, None, None, None] / D ** 3
    src = dt * (eta + k0 * c["J"])
    scale = np.abs(c["E"]).max() + dt * np.abs(c["S"]).max() + np.abs(src).max()
    assert np.max(np.abs(c["E"] - Es + dt * c["S"][0] - src * (Q / W ** 3 - W))) < 1e-13 * scale
    assert np.max(np.abs(c["F"] - Fs + dt * c["S"][1:] - src * (Qj / W ** 3 - W * vel))) \
        < 1e-13 * scale


# ---------------------------------------------------------------------------
# Whole steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rule", [("lebedev", 26), ("gl", 4, 6)])
def test_free_wave_moves_each_direction_at_unit_speed(rule):
    """The spherical wave of Sec. 4.1.2 on a small box, before its front
    reaches a face (its support, not only its front): the total energy is
    conserved, and each direction's
    distribution keeps its mass and moves its centroid by n_i dt per step
    (the pull's weights sum to 1 and their first moment along each axis is
    dt n^a: the interpolation is exact for linear fields)."""
    # the pull widens the support by at most one cell per step and axis:
    # radius + steps + 1 < 16 keeps it off the faces
    p = wl.free_wave(n=32, rule=rule, radius=4.0, dt=0.2, steps=10)
    I = orc.run(p)
    z, y, x = np.meshgrid(*(np.arange(32.0),) * 3, indexing="ij")
    pos = np.stack([x, y, z])
    t = p.steps * p.dt
    assert abs(orc.total_energy(I) / orc.total_energy(p.I0) - 1.0) < 1e-13
    for i in range(p.ndir):
        m0, m1 = p.I0[i].sum(), I[i].sum()
        assert abs(m1 / m0 - 1.0) < 1e-13
        c0 = (pos * p.I0[i]).reshape(3, -1).sum(axis=1) / m0
        c1 = (pos * I[i]).reshape(3, -1).sum(axis=1) / m1
        assert np.max(np.abs(c1 - c0 - t * p.dirs[i])) < 1e-12
def test_diffusion_moments_follow_exact_recursion():
    """Pure isotropic scattering: the total energy and its x-moments after
    each step equal the exact per-direction moment recursion."""
    # no mass can travel more than one cell per step, so nothing reaches the
    # box edge and the periodic box behaves as the unbounded lattice
    n = 44
    p = wl.diffusion(n=n, npoints=26, kappa_s=50.0, jitter=0.0, sigma=1.5, steps=8)
    x = np.arange(n) + 0.5 - n / 2
    E0 = p.meta["E0"]
    T = E0.sum()
    X1 = (E0 * x[None, None, :]).sum()
    X2 = (E0 * x[None, None, :] ** 2).sum()
    ref = analytic.diffusion_x_moments(p.steps, p.dirs, p.weights, p.dt, 1.0, 50.0, T, X1, X2)
    I = p.I0.copy()
    for k in range(p.steps):
        I = orc.step(I, p)
        E = I.sum(axis=0)
        got = (E.sum(), (E * x[None, None, :]).sum(), (E * x[None, None, :] ** 2).sum())
        assert abs(got[0] / ref[k + 1, 0] - 1) < 1e-13
        assert abs(got[1] - ref[k + 1, 1]) < 1e-12 * T
        assert abs(got[2] / ref[k + 1, 2] - 1) < 1e-12


@pytest.mark.slow
def test_sphere_reaches_analytic_profile():
    """Homogeneous sphere (Sec. 4.2.2) at kappa R = 80 on 32^3: deep inside
    E = B = 1; the shell-averaged E of each radial band follows the analytic
    solution, and the far field falls off like it.  The comparison is
    discretisation-limited (a staircase sphere of radius 8 cells, a 50-point
    rule, the pull's diffusion), so each band's tolerance is 1.5x the error
    of this same run recorded by tests/golden/make_sphere_convergence.py,
    which also records that every error shrinks at 64^3 (R = 16): the
    recorded convergence is checked here too."""
    import json
    conv = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "sphere_convergence.json")))
    run32, run64 = conv["runs"]
    assert run32["n"] == 32 and run64["n"] == 64
    for e32, e64 in zip(run32["band_rel_err"], run64["band_rel_err"]):
        assert e64 < e32
    assert run64["falloff_rel_err"] < run32["falloff_rel_err"]
    p = wl.sphere(n=32, steps=100)
    I = orc.run(p)
    E = I.sum(axis=0)
    c = np.arange(32) + 0.5 - 16
    r = np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)
    assert abs(E[15, 15, 15] - 1.0) < 1e-7
    # analytic E at every distinct cell radius (the grid has few of them)
    r2 = np.round(r ** 2, 6)
    uniq, inv = np.unique(r2, return_inverse=True)
    Ea = np.array([analytic.sphere_moments(np.sqrt(u), 8.0, 10.0)[0] for u in uniq])
    Ea = Ea[inv].reshape(r.shape)
    for (lo, hi), e32 in zip(conv["bands_in_R"], run32["band_rel_err"]):
        m = (r >= lo * 8.0) & (r < hi * 8.0)
        assert abs(E[m].mean() / Ea[m].mean() - 1) < 1.5 * e32, (lo, hi)
    # the far field falls off like the analytic solution: ratio between shells
    m1 = (r >= 10) & (r < 11)
    m2 = (r >= 15) & (r < 16)
    fall = abs((E[m2].mean() / E[m1].mean()) / (Ea[m2].mean() / Ea[m1].mean()) - 1)
    assert fall < 1.5 * run32["falloff_rel_err"]


def test_octahedral_symmetry_of_centred_sphere():
    """Lebedev rules are invariant under the octahedral group (Sec. 3.2.1);
    a centred sphere must give E invariant under axis swaps and reflections."""
    p = wl.sphere(n=16, radius=5.0, kappa=2.0, steps=12)
    I = orc.run(p)
    E = I.sum(axis=0)
    scale = np.max(np.abs(E))
    for perm in itertools.permutations(range(3)):
        assert np.max(np.abs(E - np.transpose(E, perm))) < 1e-13 * scale
    for ax in range(3):
        assert np.max(np.abs(E - np.flip(E, axis=ax))) < 1e-13 * scale


def test_crossing_beams_superpose():
    """With eta = 0 and fixed coefficients the scheme is linear: the two
    beams of the crossing test (Sec. 4.1.1) do not interact."""
    kw = dict(n=32, steps=6)
    pa = wl.beams(beam_b=False, **kw)
    pb = wl.beams(beam_a=False, **kw)
    pab = wl.beams(**kw)
    Ia, Ib, Iab = orc.run(pa), orc.run(pb), orc.run(pab)
    assert np.max(np.abs(Iab - (Ia + Ib))) < 1e-15
    assert Ia.sum() > 0 and Ib.sum() > 0


# ---------------------------------------------------------------------------
# Adjoint of a run (gradient of the energy detected on a face)
# ---------------------------------------------------------------------------
def _f64_fields(p):
    """Coefficient fields in float64, so that finite-difference steps are exact."""
    p.kappa_a = np.asarray(p.kappa_a, dtype=np.float64)
    p.kappa_s = np.asarray(p.kappa_s, dtype=np.float64)
    p.eta = np.asarray(p.eta, dtype=np.float64)
    if p.vel is not None:
        p.vel = np.asarray(p.vel, dtype=np.float64)
    return p


@pytest.mark.parametrize("bc", [(wl.BC_OUTFLOW,) * 6, (wl.BC_PERIODIC,) * 6,
                                (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC,
                                 wl.BC_OUTFLOW, wl.BC_INFLOW)])
def test_stream_transpose_is_the_transpose(bc):
    """<S x, y> = <x, S^T y> for the pull of eq. (interp) with vacuum ghosts."""
    p = _problem(shape=(5, 6, 7), npoints=26, bc=bc, seed=8, inflow_planes=2)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((p.ndir,) + p.shape)
    y = rng.standard_normal((p.ndir,) + p.shape)
    Sx = np.stack([orc.stream_direction(x[i], i, p, ghosts=False) for i in range(p.ndir)])
    lhs = float(np.sum(Sx * y))
    rhs = float(np.sum(x * orc.stream_transpose(y, p)))
    assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(Sx * y))


@pytest.mark.parametrize("vmag", [0.0, 0.45])
def test_collision_vjp_matches_finite_differences(vmag):
    """The vector-Jacobian product of the moving collision (and of the static
    one at v = 0) against central differences of the forward collision."""
    dirs, w = wl.lebedev(26)
    rng = np.random.default_rng(2)
    Is = rng.uniform(0.1, 1.0, (26, 3)) * w[:, None]
    mu = rng.standard_normal((26, 3))
    ka = np.array([0.7, 30.0, 0.01])
    k0 = np.array([0.4, 0.02, 50.0])
    et = np.array([0.3, 5.0, 0.0])
    v = rng.standard_normal((3, 3))
    v *= vmag / np.linalg.norm(v, axis=0, keepdims=True)
    dt = 0.5
    nu, gka, gk0, geta = orc.collide_moving_vjp(Is, mu, dirs, w, ka, k0, et, v, dt)
    f = lambda Is, ka, k0, et: np.sum(mu * orc.collide_moving(Is, dirs, w, ka, k0, et, v, dt),
                                      axis=0)
    for c in range(3):
        for name, g, arr in (("ka", gka, ka), ("k0", gk0, k0), ("eta", geta, et)):
            h = 1e-5 * max(1.0, abs(arr[c]))
            up, dn = arr.copy(), arr.copy()
            up[c] += h
            dn[c] -= h
            args_up = {"ka": (Is, up, k0, et), "k0": (Is, ka, up, et), "eta": (Is, ka, k0, up)}[name]
            args_dn = {"ka": (Is, dn, k0, et), "k0": (Is, ka, dn, et), "eta": (Is, ka, k0, dn)}[name]
            fd = (f(*args_up)[c] - f(*args_dn)[c]) / (2 * h)
            assert abs(fd - g[c]) < 1e-7 * max(1.0, abs(fd)), (name, c, fd, g[c])
        for i in (0, 7, 25):
            e = np.zeros_like(Is)
            e[i, c] = 1e-6
            fd = (f(Is + e, ka, k0, et)[c] - f(Is - e, ka, k0, et)[c]) / 2e-6
            assert abs(fd - nu[i, c]) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("moving,bc,planes", [
    (False, (wl.BC_OUTFLOW,) * 6, 0),
    (True, (wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW,
            wl.BC_INFLOW), 2),
])
def test_detected_energy_gradient_matches_finite_differences(moving, bc, planes):
    """Reverse-mode gradient of the energy leaving through +x over a 3-step run
    against central differences of the forward run (FP64, float64 fields)."""
    p = _f64_fields(wl.random_problem(3, shape=(5, 6, 7), npoints=14, steps=3,
                                      moving_fluid=moving, vmax=0.5, bc=bc,
                                      inflow_planes=planes))
    L, gka, gks, geta = orc.detected_energy_gradient(p, 3)
    assert abs(L - orc.detected_energy(p, 3)) < 1e-13 * abs(L)
    gmax = max(np.abs(gka).max(), np.abs(gks).max(), np.abs(geta).max())
    for cell in [(2, 3, 6), (4, 5, 5), (1, 2, 5), (3, 0, 6)]:
        for fld, g in ((p.kappa_a, gka), (p.kappa_s, gks), (p.eta, geta)):
            base = fld[cell]
            h = 1e-4 * max(1.0, abs(base))
            fld[cell] = base + h
            Lp = orc.detected_energy(p, 3)
            fld[cell] = base - h
            Lm = orc.detected_energy(p, 3)
            fld[cell] = base
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[cell]) < 1e-6 * gmax + 1e-6 * abs(fd), (cell, fd, g[cell])


@pytest.mark.parametrize("moving,bc,planes,coll", [
    (False, (wl.BC_OUTFLOW,) * 6, 0, wl.COLL_IMPLICIT),
    (False, (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC,
             wl.BC_PERIODIC), 4, wl.COLL_EXPLICIT),
    (True, (wl.BC_PERIODIC,) * 2 + (wl.BC_OUTFLOW,) * 2 + (wl.BC_INFLOW,) * 2, 3,
     wl.COLL_IMPLICIT),
])
def test_step_cells_equals_the_full_step(moving, bc, planes, coll):
    """The sampled-cell step (used where a full oracle step is too large)
    gives, at every cell including faces, edges and corners, the values of
    the pinned full step: streaming is a pull, and the collision is local."""
    p = wl.random_problem(17, shape=(5, 6, 7), npoints=26, bc=bc, inflow_planes=planes,
                          moving_fluid=moving, collision=coll, steps=1)
    full = orc.step(np.asarray(p.I0, dtype=np.float64), p)
    cells = np.array(list(itertools.product(range(5), range(6), range(7))))
    got = orc.step_cells(np.asarray(p.I0, dtype=np.float64), p, cells)
    ref = full[:, cells[:, 0], cells[:, 1], cells[:, 2]]
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-300)
