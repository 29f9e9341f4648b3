"""lbrt_step_noalloc (the entry point that allocates nothing) against
lbrt_step, through the C ABI: the same kernels, so every output must carry
the same bits.  Two calls in a row, the second on a smaller problem (the
scratch keeps the first call's contents), then a size the scratch cannot
hold, which must be rejected before any launch."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _run(prob, entry, storage):
    torch = gh.torch_mod()
    L = gh.lib()
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=storage))
    Ia, _ = gh.host_encoded_state(np.asarray(prob.I0).reshape(prob.ndir, -1), prob.weights,
                                  storage)
    Ia = Ia.reshape(-1).contiguous()
    Ib = torch.empty_like(Ia)
    ka, ks, eta, vel, inflow = gh.upload_fields(prob)
    mdt = torch.float64 if storage == L.LBRT_FP64 else torch.float32
    E = torch.full((prob.ncell,), np.nan, dtype=mdt, device="cuda")
    F = torch.full((3 * prob.ncell,), np.nan, dtype=mdt, device="cuda")
    diag = torch.full((L.LBRT_DIAG_LEN,), np.nan, dtype=torch.float64, device="cuda")
    entry(ctx, Ia, Ib, ka, ks, eta, vel=vel, inflow=inflow or None, nsteps=prob.steps, E=E, F=F,
          diag=diag)
    torch.cuda.synchronize()
    out = Ib if prob.steps % 2 == 1 else Ia
    res = {"I": out.cpu(), "E": E.cpu(), "F": F.cpu(), "diag": diag.cpu()}
    ctx.close()
    return res


def _same(a, b, what):
    for k in ("I", "E", "F", "diag"):
        x, y = a[k], b[k]
        assert x.shape == y.shape, (what, k)
        assert bool(gh.torch_mod().equal(x.view(-1), y.view(-1))), (what, k)
        assert bool(gh.torch_mod().isfinite(x.double()).all()), (what, k)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_noalloc_equals_step_two_calls(storage):
    L = gh.lib()
    st = {"fp32": L.LBRT_FP32, "bf16": L.LBRT_BF16}[storage]
    big = wl.random_problem(81, shape=(20, 18, 140), npoints=50, steps=3,
                            bc=(wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_OUTFLOW,
                                wl.BC_INFLOW, wl.BC_OUTFLOW), inflow_planes=5)
    small = wl.random_problem(82, shape=(6, 9, 70), npoints=26, steps=2,
                              bc=(wl.BC_OUTFLOW, wl.BC_INFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC,
                                  wl.BC_OUTFLOW, wl.BC_OUTFLOW), inflow_planes=2)
    for prob in (big, small):
        print(f"noalloc vs step: {prob.name} {prob.shape} x {prob.ndir} {storage}", flush=True)
        ref = _run(prob, L.lbrt_step, st)
        got = _run(prob, L.lbrt_step_noalloc, st)
        _same(got, ref, prob.name)


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    torch = gh.torch_mod()
    L = gh.lib()
    dirs, w = wl.lebedev(6)
    desc = L.Desc(nx=64, ny=64, nz=2048, dt=0.5, dirs=dirs, weights=w)
    ctx = L.lbrt_init(desc)
    # one z-plane per block: 62 interior rows x 2048 planes of main blocks
    L.lbrt_set_tiling(ctx, 64, 1, 1, 1)
    n = desc.ndir * desc.ncell
    Ia = torch.zeros(n, device="cuda")
    Ib = torch.zeros(n, device="cuda")
    f = torch.zeros(desc.ncell, device="cuda")
    diag = torch.zeros(L.LBRT_DIAG_LEN, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LbrtError) as ei:
        L.lbrt_step_noalloc(ctx, Ia, Ib, f, f, f, nsteps=1, diag=diag)
    assert ei.value.code == L.LBRT_E_INVAL
    assert "scratch" in str(ei.value)
    # without diagnostics the same call needs no partials and runs
    L.lbrt_step_noalloc(ctx, Ia, Ib, f, f, f, nsteps=1)
    torch.cuda.synchronize()
    assert float(Ib.abs().sum()) == 0.0
    ctx.close()
