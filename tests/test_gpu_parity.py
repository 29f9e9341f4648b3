"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Boxes are ragged and large enough that several tiles take the boundary-free
path and several take the checked path.  Tolerances: FP64 storage 1e-12
relative; FP32 1e-5 relative (global relative L2 on populations, E and F);
BF16/FP16 storage 2e-3 relative on E and F.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def L():
    return gh.lib()


SHAPE = (10, 12, 150)   # (nz, ny, nx): interior and boundary tiles, ragged in x


def oracle_run(prob, I0_eff, steps, collision=None):
    I = I0_eff.copy()
    fluxes = []
    for _ in range(steps):
        fluxes.append(orc.boundary_fluxes(I, prob) if prob.ncell <= 40000 else None)
        I = orc.step(I, prob, collision)
    E, F = orc.moments(I, prob.dirs)
    return I, E, F, fluxes


def check(res, I, E, F, tol, tol_ef=None):
    tol_ef = tol if tol_ef is None else tol_ef
    eI = gh.rel_l2(res["I"], I)
    eE = gh.rel_l2(res["E"], E)
    eF = gh.rel_l2(res["F"], F)
    print(f"rel L2: I {eI:.3e}  E {eE:.3e}  F {eF:.3e}", flush=True)
    assert eE < tol_ef and eF < tol_ef
    if tol is not None:
        assert eI < tol


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("coll,lam", [(wl.COLL_IMPLICIT, 0.0), (wl.COLL_IMPLICIT, 0.4),
                                      (wl.COLL_EXPLICIT, 0.0), (wl.COLL_EXPLICIT, -0.25),
                                      (wl.COLL_LAMBDA, 0.0), (wl.COLL_LAMBDA, 0.5)])
def test_static_collisions(storage, tol, coll, lam):
    st = {"fp64": L().LBRT_FP64, "fp32": L().LBRT_FP32}[storage]
    kr = (-2.0, 2.0) if coll == wl.COLL_IMPLICIT else (-2.0, 0.0)   # explicit: dt k < 1
    p = wl.random_problem(101, shape=SHAPE, npoints=26, kappa_range=kr, collision=coll,
                          lam=lam, lambda_iters=3, steps=3)
    res = gh.run_problem(p, storage=st)
    I, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
    check(res, I, E, F, tol)


@pytest.mark.parametrize("npoints", [6, 14, 26, 38, 50, 74, 86, 110, 146])
def test_every_bucket_fp32(npoints):
    p = wl.random_problem(7 + npoints, shape=(6, 9, 70), npoints=npoints, steps=2)
    res = gh.run_problem(p, storage=L().LBRT_FP32)
    I, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
    check(res, I, E, F, 1e-5)


@pytest.mark.parametrize("bc", [
    (wl.BC_PERIODIC,) * 6,
    (wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_OUTFLOW),
    (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC),
])
def test_boundaries_and_diagnostics_fp64(bc):
    p = wl.random_problem(5, shape=(7, 9, 13), npoints=26, bc=bc, inflow_planes=4, steps=2)
    res = gh.run_problem(p, storage=L().LBRT_FP64)
    I, E, F, fluxes = oracle_run(p, res["I0_eff"], p.steps)
    check(res, I, E, F, 1e-12)
    diag = res["diag"]
    out = sum(f[0] for f in fluxes)
    infl = sum(f[1] for f in fluxes)
    scale = res["I0_eff"].sum()
    assert np.max(np.abs(diag[1:7] - out)) < 1e-12 * scale
    assert abs(diag[7] - infl) < 1e-12 * scale
    assert abs(diag[0] - E.sum()) < 1e-12 * scale


def test_budget_identity_fp32_large():
    """sum E* = sum E - outflux + influx for one step (exact for the pull)."""
    p = wl.random_problem(9, shape=(20, 24, 150), npoints=50,
                          bc=(wl.BC_INFLOW,) + (wl.BC_OUTFLOW,) * 5, inflow_planes=3, steps=1)
    res = gh.run_problem(p, storage=L().LBRT_FP32)
    d = res["diag"]
    E0 = res["I0_eff"].sum()
    lhs = d[8]
    rhs = E0 - d[1:7].sum() + d[7]
    assert abs(lhs - rhs) < 1e-6 * E0


def test_moving_fluid():
    for st, tol in ((L().LBRT_FP64, 1e-12), (L().LBRT_FP32, 1e-5)):
        p = wl.random_problem(21, shape=SHAPE, npoints=50, moving_fluid=True, vmax=0.6, steps=2)
        res = gh.run_problem(p, storage=st)
        I, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
        check(res, I, E, F, tol)


@pytest.mark.parametrize("storage", ["bf16", "fp16"])
def test_reduced_storage(storage):
    st = {"bf16": L().LBRT_BF16, "fp16": L().LBRT_FP16}[storage]
    p = wl.random_problem(33, shape=SHAPE, npoints=50, steps=3, kappa_range=(-2, 1))
    res = gh.run_problem(p, storage=st)
    I, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
    check(res, I, E, F, None, tol_ef=2e-3)


def test_exact_shift_is_bit_exact():
    """dt = dx: axis directions shift by one cell exactly (Sec. 4.1.1)."""
    p = wl.random_problem(3, shape=(8, 10, 70), npoints=6, dt=1.0, bc=(wl.BC_PERIODIC,) * 6,
                          steps=1)
    p.kappa_a[:] = 0
    p.kappa_s[:] = 0
    p.eta[:] = 0
    res = gh.run_problem(p, storage=L().LBRT_FP32)
    I0 = res["I0_eff"]
    for i in range(6):
        n = p.dirs[i]
        a = int(np.argmax(np.abs(n)))
        ref = np.roll(I0[i], int(np.sign(n[a])), axis=2 - a)
        assert np.array_equal(res["I"][i], ref)


@pytest.mark.parametrize("bc,planes", [
    ((wl.BC_PERIODIC, wl.BC_PERIODIC) + (wl.BC_OUTFLOW,) * 4, 0),
    ((wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC), 6),
])
def test_tile_shapes_are_bit_identical(bc, planes):
    """Tile shape and z-range lengths change which cells take which kernel
    (main or general) and where the z-march starts; results must not move."""
    p = wl.random_problem(41, shape=(12, 16, 140), npoints=50, steps=2, bc=bc,
                          inflow_planes=planes)
    ref = gh.run_problem(p, storage=L().LBRT_FP32, tile="64x1")
    for tile, zlen, zg in (("32x2", None, None), ("16x4", None, None), ("8x8", None, None),
                           ("64x1", 1, 1), ("64x1", 5, 3), ("64x1", 12, 12), ("32x2", 7, 2)):
        got = gh.run_problem(p, storage=L().LBRT_FP32, tile=tile, zlen=zlen, zlen_general=zg)
        assert np.array_equal(got["I"], ref["I"]), (tile, zlen, zg)
        assert np.array_equal(got["E"], ref["E"]), (tile, zlen, zg)


def test_repeat_runs_are_bit_identical():
    p = wl.random_problem(43, shape=SHAPE, npoints=110, steps=2)
    a = gh.run_problem(p, storage=L().LBRT_FP32)
    b = gh.run_problem(p, storage=L().LBRT_FP32)
    assert np.array_equal(a["I"], b["I"])
    assert np.array_equal(a["diag"], b["diag"])


def test_sphere_fp64_full_length():
    """Homogeneous sphere, 32^3 x 50 directions, 100 steps, FP64: 1e-12."""
    p = wl.sphere(n=32, steps=100)
    res = gh.run_problem(p, storage=L().LBRT_FP64)
    I = orc.run(p)
    E, F = orc.moments(I, p.dirs)
    check(res, I, E, F, 1e-12)
