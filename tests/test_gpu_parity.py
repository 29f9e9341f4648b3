"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Boxes are ragged and large enough that several tiles take the boundary-free
path and several take the checked path.  Every comparison is made twice:
as a global relative L2 error and element by element.

* FP64 storage: 1e-12, both as relative L2 and as max |got - ref| / max |ref|
  per field (populations, E, each F component).
* FP32 storage: 1e-5, the same two ways.
* BF16/FP16 storage (E and F only, from the FP32 collision): 2e-3 relative
  L2, and element by element |dE|, |dF| <= 2 k u max E after k steps, u the
  unit roundoff of the 16-bit format (2^-8 BF16, 2^-11 FP16): each step
  rounds every stored population once, stochastically, to one of its two
  neighbouring 16-bit values (relative error below one unit in the last
  place, 2u), and the pull and the implicit collision are averages with
  nonnegative weights, so a cell's accumulated error stays below 2 k u times
  the energy scale (the FP32 arithmetic around it adds far less).
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


def max_rel(got, ref):
    """max |got - ref| / max |ref| over one field."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def check(res, I, E, F, tol, tol_ef=None, steps=None, unit_roundoff=None):
    """tol: relative L2 and element-wise bound for I, E and F (None: the
    populations are not compared).  tol_ef: the relative L2 bound of E and F
    when it differs.  With unit_roundoff (16-bit storage), E and F are
    bounded element by element by 2 steps u max E (see the module doc)."""
    tol_ef = tol if tol_ef is None else tol_ef
    eI = gh.rel_l2(res["I"], I)
    eE = gh.rel_l2(res["E"], E)
    eF = gh.rel_l2(res["F"], F)
    mI = max_rel(res["I"], I)
    mE = max_rel(res["E"], E)
    mF = max(max_rel(res["F"][a], F[a]) for a in range(3))
    print(f"rel L2: I {eI:.3e}  E {eE:.3e}  F {eF:.3e} | max/max: I {mI:.3e}  E {mE:.3e}  "
          f"F {mF:.3e}", flush=True)
    assert eE < tol_ef and eF < tol_ef
    if unit_roundoff is None:
        assert mE < tol_ef and mF < tol_ef
    else:
        bound = 2.0 * steps * unit_roundoff * np.max(np.abs(E))
        dE = np.max(np.abs(res["E"] - E))
        dF = np.max(np.abs(res["F"] - F))
        print(f"element-wise |dE| {dE:.3e} |dF| {dF:.3e} bound {bound:.3e}", flush=True)
        assert dE <= bound and dF <= bound
    if tol is not None:
        assert eI < tol and mI < tol


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
    (wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_INFLOW, wl.BC_INFLOW),
    (wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW),
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


@pytest.mark.parametrize("bc", [
    (wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_INFLOW),
    (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_INFLOW),
])
def test_z_face_inflow_fp32(bc):
    """Inflow ghost planes on z faces: the z ranges next to such a face run
    on the checked path (a tile plan of their own), and the z-face influx is
    booked by the z-face kernel (diag[7]); both against the oracle on a box
    where interior tiles exist too."""
    p = wl.random_problem(55, shape=(40, 12, 150), npoints=50, bc=bc, inflow_planes=6, steps=2)
    res = gh.run_problem(p, storage=L().LBRT_FP32)
    I = res["I0_eff"].copy()
    influx = 0.0
    out = np.zeros(6)
    for _ in range(p.steps):
        o, infl = orc.boundary_fluxes(I, p)
        out += o
        influx += infl
        I = orc.step(I, p)
    E, F = orc.moments(I, p.dirs)
    check(res, I, E, F, 1e-5)
    scale = res["I0_eff"].sum()
    d = res["diag"]
    print(f"influx {d[7]:.9e} vs {influx:.9e}; outflux max diff "
          f"{np.max(np.abs(d[1:7] - out)) / scale:.2e}", flush=True)
    assert influx > 0 and abs(d[7] - influx) < 1e-6 * scale
    assert np.max(np.abs(d[1:7] - out)) < 1e-6 * scale


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("shape,bc,planes", [
    ((2, 2, 2), (wl.BC_PERIODIC,) * 6, 0),
    ((2, 2, 2), (wl.BC_OUTFLOW,) * 6, 0),
    ((2, 3, 2), (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_INFLOW,
                 wl.BC_OUTFLOW), 4),
    ((3, 2, 67), (wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_PERIODIC,
                  wl.BC_PERIODIC), 3),
])
def test_smallest_boxes(shape, bc, planes, storage, tol):
    """Boxes at the smallest edge the library takes (2 cells): every tile is
    ragged and every tap is next to a face, so a periodic wrap lands on the
    cell's own row and every x-shifted tap of a vacuum face is a ghost.
    Populations, E, F and the face fluxes against the oracle.  F sums
    populations of size E with both signs, and on these boxes it nearly
    cancels (a periodic 2^3 box relaxes to isotropy), so its rounding is
    bounded relative to max E rather than to F's own norm."""
    st = {"fp64": L().LBRT_FP64, "fp32": L().LBRT_FP32}[storage]
    p = wl.random_problem(61, shape=shape, npoints=50, bc=bc, inflow_planes=planes, steps=3)
    print(f"smallest box {shape} {storage}", flush=True)
    res = gh.run_problem(p, storage=st)
    I, E, F, fluxes = oracle_run(p, res["I0_eff"], p.steps)
    eI, mI, mE = gh.rel_l2(res["I"], I), max_rel(res["I"], I), max_rel(res["E"], E)
    dF = float(np.max(np.abs(res["F"] - F)) / np.max(np.abs(E)))
    print(f"I rel L2 {eI:.3e} max/max {mI:.3e}; E max/max {mE:.3e}; "
          f"max |dF| / max E {dF:.3e}", flush=True)
    assert eI < tol and mI < tol and mE < tol and dF < tol
    d = res["diag"]
    scale = res["I0_eff"].sum()
    ftol = 1e-12 if storage == "fp64" else 1e-6
    assert np.max(np.abs(d[1:7] - sum(f[0] for f in fluxes))) < ftol * scale
    assert abs(d[7] - sum(f[1] for f in fluxes)) < ftol * scale


@pytest.mark.parametrize("storage", ["bf16", "fp16", "bf16s", "fp16s"])
@pytest.mark.parametrize("shape,bc,planes", [
    ((2, 2, 2), (wl.BC_PERIODIC,) * 6, 0),
    ((2, 3, 2), (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_INFLOW,
                 wl.BC_OUTFLOW), 4),
])
def test_smallest_boxes_16bit(shape, bc, planes, storage):
    """The 16-bit storage forms (plain and equilibrium-shifted) on the
    smallest boxes: E and F element by element within 2 k u max E after k
    steps (the module doc's bound)."""
    st = {"bf16": L().LBRT_BF16, "fp16": L().LBRT_FP16, "bf16s": L().LBRT_BF16_SHIFTED,
          "fp16s": L().LBRT_FP16_SHIFTED}[storage]
    u = 2.0 ** -8 if storage.startswith("bf16") else 2.0 ** -11
    p = wl.random_problem(61, shape=shape, npoints=50, bc=bc, inflow_planes=planes, steps=3)
    print(f"smallest box {shape} {storage}", flush=True)
    res = gh.run_problem(p, storage=st)
    _, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
    bound = 2.0 * p.steps * u * np.max(np.abs(E))
    dE = float(np.max(np.abs(res["E"] - E)))
    dF = float(np.max(np.abs(res["F"] - F)))
    print(f"|dE| {dE:.3e} |dF| {dF:.3e} bound {bound:.3e}", flush=True)
    assert dE <= bound and dF <= bound


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_zero_steps_gives_the_moments_of_the_input(storage):
    """nsteps = 0 leaves the state untouched and writes E and F of I_a."""
    st = {"fp64": L().LBRT_FP64, "fp32": L().LBRT_FP32}[storage]
    p = wl.random_problem(63, shape=(5, 7, 70), npoints=26, steps=0)
    res = gh.run_problem(p, storage=st)
    assert np.array_equal(res["I"], res["I0_eff"].reshape(res["I"].shape))
    E, F = orc.moments(res["I0_eff"], p.dirs)
    tol = 1e-13 if storage == "fp64" else 1e-6
    assert max_rel(res["E"], E) < tol
    assert max(max_rel(res["F"][a], F[a]) for a in range(3)) < tol
    assert np.all(res["diag"] == 0.0)


def test_step_with_inflow_graph_replays_match_eager():
    """lbrt_step with inflow planes enqueues kernels only (its ghost table is
    written by a kernel), so it can be captured: replays of the captured
    steps equal the eager result, with eager work on the same context
    between the replays."""
    torch = gh.torch_mod()
    Lb = L()
    p = wl.random_problem(57, shape=(12, 16, 140), npoints=50, steps=2,
                          bc=(wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW,
                              wl.BC_INFLOW, wl.BC_OUTFLOW), inflow_planes=4)
    ctx = Lb.lbrt_init(Lb.Desc.from_problem(p))
    ka, ks, eta, _, inflow = gh.upload_fields(p)
    I0 = torch.from_numpy(np.asarray(p.I0, dtype=np.float32)).reshape(-1).cuda()
    Ia, Ib = I0.clone(), torch.empty_like(I0)
    E = torch.empty(p.ncell, device="cuda")
    diag = torch.zeros(Lb.LBRT_DIAG_LEN, dtype=torch.float64, device="cuda")

    def run(stream=None):
        Lb.lbrt_step(ctx, Ia, Ib, ka, ks, eta, inflow=inflow, nsteps=p.steps, E=E, diag=diag,
                     stream=stream)

    run()
    torch.cuda.synchronize()
    ref_I, ref_E, ref_d = Ia.clone(), E.clone(), diag.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    Ia.copy_(I0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        run(stream=s.cuda_stream)
    for rep in range(3):
        # eager work on the same context between replays: a call without
        # inflow planes rewrites the ghost table
        Xa, Xb = I0.clone(), torch.empty_like(I0)
        Lb.lbrt_step(ctx, Xa, Xb, ka, ks, eta, nsteps=1)
        Ia.copy_(I0)
        E.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ia, ref_I), rep
        assert torch.equal(E, ref_E), rep
        assert torch.equal(diag, ref_d), rep
    ctx.close()


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
    u = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}[storage]
    check(res, I, E, F, None, tol_ef=2e-3, steps=p.steps, unit_roundoff=u)


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


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("bc,planes", [
    ((wl.BC_PERIODIC, wl.BC_PERIODIC) + (wl.BC_OUTFLOW,) * 4, 0),
    ((wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC), 6),
])
def test_tile_shapes_are_bit_identical(bc, planes, storage):
    """Tile shape and z-range lengths change which cells take which kernel
    (main, pair or general) and where the z-march starts; results must not
    move.  BF16 runs the interior on the pair kernel, with the same
    stochastic rounding bits for a cell whichever kernel stores it."""
    st = {"fp32": L().LBRT_FP32, "bf16": L().LBRT_BF16}[storage]
    p = wl.random_problem(41, shape=(12, 16, 140), npoints=50, steps=2, bc=bc,
                          inflow_planes=planes)
    ref = gh.run_problem(p, storage=st, tile="64x1")
    for tile, zlen, zg in (("32x2", None, None), ("16x4", None, None), ("8x8", None, None),
                           ("64x1", 1, 1), ("64x1", 5, 3), ("64x1", 12, 12), ("32x2", 7, 2)):
        got = gh.run_problem(p, storage=st, tile=tile, zlen=zlen, zlen_general=zg)
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


@pytest.mark.parametrize("storage,npoints,shape,bc,planes,coll,lam", [
    ("fp16", 110, (12, 16, 140), (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW,
                                  wl.BC_INFLOW, wl.BC_OUTFLOW), 6, wl.COLL_IMPLICIT, 0.0),
    ("bf16", 50, (9, 11, 70), (wl.BC_PERIODIC,) * 6, 0, wl.COLL_IMPLICIT, 0.3),
    ("fp16", 110, (7, 9, 266), (wl.BC_OUTFLOW,) * 6, 0, wl.COLL_EXPLICIT, -0.25),
    ("bf16", 50, (8, 10, 136), (wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_INFLOW,
                                wl.BC_PERIODIC, wl.BC_PERIODIC), 3, wl.COLL_LAMBDA, 0.5),
    ("bf16", 110, (12, 16, 140), (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW,
                                  wl.BC_OUTFLOW, wl.BC_OUTFLOW), 4, wl.COLL_IMPLICIT, 0.0),
    ("fp16", 50, (9, 11, 70), (wl.BC_PERIODIC,) * 6, 0, wl.COLL_IMPLICIT, 0.0),
    ("bf16", 50, (10, 12, 134), (wl.BC_OUTFLOW,) * 6, 0, wl.COLL_IMPLICIT, 0.4),
    ("bf16s", 110, (12, 16, 140), (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW,
                                   wl.BC_INFLOW, wl.BC_OUTFLOW), 6, wl.COLL_IMPLICIT, 0.0),
    ("fp16s", 50, (9, 11, 70), (wl.BC_PERIODIC,) * 6, 0, wl.COLL_IMPLICIT, 0.3),
    ("bf16s", 50, (8, 10, 136), (wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_INFLOW,
                                 wl.BC_PERIODIC, wl.BC_PERIODIC), 3, wl.COLL_LAMBDA, 0.5),
    ("fp16s", 110, (7, 9, 266), (wl.BC_OUTFLOW,) * 6, 0, wl.COLL_EXPLICIT, -0.25),
])
def test_pair_kernel_equals_main_kernel(storage, npoints, shape, bc, planes, coll, lam):
    """The interior on the two-cells-per-lane kernel (x in [2, nx - 2), the
    face columns on the checked path) against the one-cell-per-lane main
    kernel: the same populations, E and F bit for bit (with the same
    stochastic rounding bits), for plain and equilibrium-shifted 16-bit
    storage (the shifted state's E array included).  The diagnostics are
    sums in a
    different grouping: the energy sums (FP64 per lane) to 1e-12, the face
    fluxes (FP32 per lane over a block's z range, then FP64) to 1e-6."""
    st = {"bf16": L().LBRT_BF16, "fp16": L().LBRT_FP16, "bf16s": L().LBRT_BF16_SHIFTED,
          "fp16s": L().LBRT_FP16_SHIFTED}[storage]
    p = wl.random_problem(91, shape=shape, npoints=npoints, bc=bc, inflow_planes=planes,
                          collision=coll, lam=lam, steps=3,
                          kappa_range=(-2.0, 2.0) if coll == wl.COLL_IMPLICIT else (-2.0, 0.0))
    print(f"pair vs main: {storage} {shape} x {npoints}", flush=True)
    a = gh.run_problem(p, storage=st, pair=True)
    b = gh.run_problem(p, storage=st, pair=False)
    torch = gh.torch_mod()
    torch.cuda.synchronize()
    assert torch.equal(a["raw"], b["raw"])
    assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["F"], b["F"])
    scale = a["I0_eff"].sum()
    d = np.abs(a["diag"] - b["diag"])
    assert max(d[0], d[8]) <= 1e-12 * scale
    assert np.max(d[1:8]) <= 1e-6 * scale


def test_pair_kernel_against_oracle_ragged():
    """The pair kernel (FP16) on a box whose interior is not a whole number
    of 128-cell tiles, against the FP64 oracle with the 16-bit bounds of the
    module doc."""
    p = wl.random_problem(93, shape=(9, 10, 174), npoints=110, steps=2,
                          bc=(wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW,
                              wl.BC_OUTFLOW, wl.BC_OUTFLOW), inflow_planes=3)
    res = gh.run_problem(p, storage=L().LBRT_FP16, pair=True)
    I, E, F, _ = oracle_run(p, res["I0_eff"], p.steps)
    check(res, I, E, F, None, tol_ef=2e-3, steps=p.steps, unit_roundoff=2.0 ** -11)


@pytest.mark.parametrize("storage", ["bf16", "fp16"])
def test_stochastic_rounding_follows_slow_decay(storage):
    """A uniform isotropic field in a periodic box with weak absorption
    (dt kappa_a = 1e-4, below half a unit in the last place of both formats
    at the stored values, 1.0): each step multiplies every population by
    c = 1 / (1 + dt kappa_a).  With round-to-nearest the stored values never
    change; with stochastic rounding the mean over cells follows c^n, within
    a few standard errors of the per-element rounding noise."""
    Lb = L()
    st = {"bf16": Lb.LBRT_BF16, "fp16": Lb.LBRT_FP16}[storage]
    u = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}[storage]
    p = wl.random_problem(95, shape=(16, 16, 64), npoints=26, steps=200,
                          bc=(wl.BC_PERIODIC,) * 6)
    p.kappa_a[:] = 2e-4
    p.kappa_s[:] = 0.0
    p.eta[:] = 0.0
    p.I0 = np.broadcast_to(p.weights[:, None, None, None], (p.ndir,) + p.shape).copy()
    c = 1.0 / (1.0 + p.dt * np.float64(np.float32(2e-4)))
    exact = c ** p.steps * p.weights.sum()
    near = gh.run_problem(p, storage=st, rounding=Lb.LBRT_ROUND_NEAREST, want_diag=False)
    sto = gh.run_problem(p, storage=st, rounding=Lb.LBRT_ROUND_STOCHASTIC, want_diag=False)
    # the stored populations (decoded); E is formed before the rounding
    m_near = near["I"].sum(axis=0).mean()
    m_sto = sto["I"].sum(axis=0).mean()
    # each step adds to each stored value a rounding error of zero mean and
    # variance below (ulp / 2)^2 = u^2 (relative); the sum over the box is
    # conserved by the periodic pull, so the mean's error has a standard
    # deviation below u sqrt(steps / (ncell ndir))
    sigma = u * np.sqrt(p.steps / (p.ncell * p.ndir))
    print(f"{storage}: exact {exact:.6f}  nearest {m_near:.6f}  stochastic {m_sto:.6f} "
          f"(sigma {sigma:.1e})", flush=True)
    # round-to-nearest: every stored value stays at its start (the sum of the
    # FP32 weights); stochastic: the exact decay within the noise
    assert abs(m_near - p.weights.sum()) < 1e-6
    assert abs(m_sto - exact) < 5 * sigma
