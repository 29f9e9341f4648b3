"""GPU parity of lbrt_coupling: the moments E, F, P, the fluid-frame J, H and
the radiative sources S of a state (Sec. 3.2 eq. higher_moments; Sec. 5
eq. J and coupling item 4) against the FP64 oracle, element by element.

Bounds.  The GPU sums the same stored values in FP64 in the same direction
order as the oracle; the two differ only by FP64 rounding (a few units of
1e-16 of the terms, which are bounded by W^3 sum_i |I_i| per cell times the
opacities for S) and, for FP32 outputs, by the final rounding to FP32
(2^-24 relative to the value).  Each element is checked against
    |got - ref| <= 2^-24 |ref| [FP32 outputs] + 1e-13 * bound_cell,
bound_cell = W^3 sum_i |I_i| (E, F, P, J, H), times (1 + kappa_a + k) plus
W eta for S.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _outputs(torch, n, dtype):
    return {k: torch.full((m * n,), float("nan"), dtype=dtype, device="cuda")
            for k, m in (("E", 1), ("F", 3), ("P", 6), ("J", 1), ("H", 4), ("S", 4))}


def _compare(got, ref, absI, W, ka, kt, eta, fp32):
    base = 1e-13 * W ** 3 * absI
    bounds = {"E": base, "F": base, "P": base, "J": base, "H": base,
              "S": base * (1.0 + ka + kt) + 1e-13 * W * np.abs(eta)}
    for k, r in ref.items():
        g = got[k].reshape(r.shape)
        lim = bounds[k] + (2.0 ** -24 * np.abs(r) if fp32 else 0.0)
        err = np.abs(g - r)
        worst = float(np.max(err / lim))
        print(f"  {k}: max |err| {err.max():.3e}  worst err/bound {worst:.3f}", flush=True)
        assert np.all(np.isfinite(g)), k
        assert np.all(err <= lim), k


def _run(storage, npoints, shape, lam, vmax, seed):
    torch = gh.torch_mod()
    L = gh.lib()
    st = {"fp64": L.LBRT_FP64, "fp32": L.LBRT_FP32, "bf16": L.LBRT_BF16,
          "fp16": L.LBRT_FP16}[storage]
    p = wl.random_problem(seed, shape=shape, npoints=npoints, lam=lam)
    rng = np.random.default_rng(seed + 100)
    v = rng.standard_normal((3,) + shape)
    v *= rng.uniform(0.0, vmax, shape) / np.linalg.norm(v, axis=0)
    v = v.astype(np.float32).astype(np.float64)
    print(f"coupling: {storage} {shape} x {npoints} lam {lam} vmax {vmax}", flush=True)
    desc = L.Desc.from_problem(p, storage=st)
    ctx = L.lbrt_init(desc)
    I_dev, I_eff = gh.host_encoded_state(p.I0, p.weights, st)
    ka, ks, eta, _, _ = gh.upload_fields(p)
    vel = None if vmax == 0 else torch.from_numpy(v.astype(np.float32)).reshape(-1).cuda()
    mdt = torch.float64 if st == L.LBRT_FP64 else torch.float32
    out = _outputs(torch, p.ncell, mdt)
    L.lbrt_coupling(ctx, I_dev.reshape(-1), vel=vel, kappa_a=ka, kappa_s=ks, eta=eta, **out)
    torch.cuda.synchronize()
    got = {k: t.double().cpu().numpy() for k, t in out.items()}
    v = None if vmax == 0 else v
    ref = orc.coupling(I_eff, p.dirs, v, p.kappa_a, p.kappa_s, p.eta, lam)
    ref = {k: np.asarray(r) for k, r in ref.items()}
    W = 1.0 if v is None else 1.0 / np.sqrt(1.0 - (v ** 2).sum(axis=0))
    absI = np.abs(I_eff).sum(axis=0)
    ka64 = p.kappa_a.astype(np.float64)
    kt = ka64 + p.kappa_s.astype(np.float64) * (1.0 - lam / 9.0)
    _compare(got, ref, absI, W, ka64, kt, p.eta.astype(np.float64), mdt == torch.float32)
    ctx.close()


@pytest.mark.parametrize("storage,npoints,shape,lam,vmax,seed", [
    ("fp64", 50, (6, 7, 45), 0.0, 0.9, 1),
    ("fp64", 26, (5, 6, 33), 0.5, 0.0, 2),
    ("fp32", 110, (9, 10, 131), 0.0, 0.6, 3),
    ("fp32", 146, (4, 5, 77), -0.25, 0.95, 4),
    ("bf16", 110, (7, 8, 64), 0.0, 0.5, 5),
    ("fp16", 50, (3, 4, 11), 0.5, 0.3, 6),
])
def test_coupling_against_oracle(storage, npoints, shape, lam, vmax, seed):
    _run(storage, npoints, shape, lam, vmax, seed)


def test_coupling_writes_only_what_is_asked():
    """Outputs not passed are not touched; without the opacities the sources
    are refused (LBRT_E_INVAL), and so is nothing else."""
    torch = gh.torch_mod()
    L = gh.lib()
    p = wl.random_problem(7, shape=(4, 5, 19), npoints=26)
    ctx = L.lbrt_init(L.Desc.from_problem(p, storage=L.LBRT_FP32))
    I_dev, I_eff = gh.host_encoded_state(p.I0, p.weights, L.LBRT_FP32)
    out = _outputs(torch, p.ncell, torch.float32)
    L.lbrt_coupling(ctx, I_dev.reshape(-1), P=out["P"], J=out["J"])
    torch.cuda.synchronize()
    for k in ("E", "F", "H", "S"):
        assert torch.isnan(out[k]).all(), k
    ref = orc.coupling(I_eff, p.dirs)
    np.testing.assert_allclose(out["J"].double().cpu().numpy().reshape(p.shape), ref["E"],
                               rtol=2.0 ** -23, atol=0)
    np.testing.assert_allclose(out["P"].double().cpu().numpy().reshape(ref["P"].shape), ref["P"],
                               rtol=2.0 ** -23, atol=1e-13 * ref["E"].max())
    with pytest.raises(L.LbrtError) as e:
        L.lbrt_coupling(ctx, I_dev.reshape(-1), S=out["S"])
    assert e.value.code == L.LBRT_E_INVAL
    ctx.close()


def test_coupling_full_size_sampled_cells():
    """256^3 cells x 110 directions, FP32 state (the crossing-beams box with a
    sheared flow), sampled cells against the oracle on their populations."""
    torch = gh.torch_mod()
    L = gh.lib()
    prob = wl.beams(n=256, alloc_state=False)
    n = prob.ncell
    print(prob.name, prob.shape, prob.ndir, flush=True)
    g = torch.Generator(device="cuda").manual_seed(31)
    I = torch.rand(prob.ndir * n, generator=g, device="cuda", dtype=torch.float32)
    I.view(prob.ndir, n).mul_(torch.as_tensor(np.abs(prob.weights), dtype=torch.float32,
                                              device="cuda")[:, None])
    y = torch.arange(prob.ny, device="cuda", dtype=torch.float32)
    vx = (0.5 * torch.tanh((y - 96.0) / 8.0))[None, :, None].expand(prob.shape)
    vel = torch.zeros(3, *prob.shape, device="cuda", dtype=torch.float32)
    vel[0] = vx
    vel[2] = 0.1
    vel = vel.reshape(-1)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    ka, ks, eta = f(prob.kappa_a), f(prob.kappa_s), f(prob.eta)
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=L.LBRT_FP32))
    out = _outputs(torch, n, torch.float32)
    L.lbrt_coupling(ctx, I, vel=vel, kappa_a=ka, kappa_s=ks, eta=eta, **out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    cells = np.stack([rng.integers(0, s, 300) for s in prob.shape], axis=1)
    idx = torch.as_tensor(cells[:, 0] * prob.ny * prob.nx + cells[:, 1] * prob.nx + cells[:, 2],
                          device="cuda")
    Ic = I.view(prob.ndir, n)[:, idx].double().cpu().numpy()[:, None, None, :]
    vc = vel.view(3, n)[:, idx].double().cpu().numpy()[:, None, None, :]
    pick = lambda a: a.reshape(-1)[idx.cpu().numpy()][None, None, :]
    kac, ksc, etc = pick(prob.kappa_a), pick(prob.kappa_s), pick(prob.eta)
    ref = orc.coupling(Ic, prob.dirs, vc, kac, ksc, etc, prob.lam)
    got = {k: v.view(-1, n)[:, idx].double().cpu().numpy().reshape(ref[k].shape)
           for k, v in out.items()}
    del I, out
    ctx.close()
    torch.cuda.empty_cache()
    W = 1.0 / np.sqrt(1.0 - (vc ** 2).sum(axis=0))
    ka64 = kac.astype(np.float64)
    kt = ka64 + ksc.astype(np.float64) * (1.0 - prob.lam / 9.0)
    _compare(got, {k: np.asarray(r) for k, r in ref.items()}, np.abs(Ic).sum(axis=0), W, ka64,
             kt, etc.astype(np.float64), True)
