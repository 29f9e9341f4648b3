"""GPU parity of the adjoint: gradients of the detected energy from the
library's reverse sweep (lbrt_adjoint_step through the checkpointed
torch.autograd.Function) against the FP64 oracle's reverse-mode gradient,
which the CPU tests pin to finite differences.

Tolerances: FP64 storage 1e-10 relative (global L2 of each gradient field);
FP32 storage 2e-5 on the small boxes and 1e-4 on the 32^3 x 146 shear-flow
workload (16 steps: FP32 rounding accumulates along the run and back).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _f64(p):
    for k in ("kappa_a", "kappa_s", "eta"):
        setattr(p, k, np.asarray(getattr(p, k), dtype=np.float64))
    if p.vel is not None:
        p.vel = np.asarray(p.vel, dtype=np.float64)
    return p


def _gpu_gradient(p, storage, steps, face, K, lte=False):
    """L and (g_kappa_a, g_kappa_s, g_eta) from the library; with lte, eta is
    composed in torch as kappa_a * 1 and only kappa_a, kappa_s are leaves."""
    torch = gh.torch_mod()
    L = gh.lib()
    from paper_2007_05718_amd import autodiff
    desc = L.Desc.from_problem(p, storage=storage)
    ctx = L.lbrt_init(desc)
    I0, I0_eff = gh.host_encoded_state(np.asarray(p.I0).reshape(p.ndir, -1), p.weights, storage)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    vel = None if p.vel is None else f(p.vel)
    inflow = [(q.face, q.direction, f(q.values)) for q in p.inflow] or None
    I0 = I0.reshape(-1).contiguous()
    out = dict(I0_eff=I0_eff.reshape((p.ndir,) + p.shape))
    if lte:
        # through the autograd Function, eta composed in torch
        ka = f(p.kappa_a).requires_grad_(True)
        ks = f(p.kappa_s).requires_grad_(True)
        Lval = autodiff.detected_energy(ctx, I0, ka, ks, ka * 1.0, steps, face=face,
                                        checkpoint_every=K, vel=vel, inflow=inflow)
        Lval.backward()
        gka, gks = ka.grad, ks.grad
    else:
        Lval, gka, gks, geta = autodiff.detected_energy_gradient(
            ctx, I0, f(p.kappa_a), f(p.kappa_s), f(p.eta), steps, face=face,
            checkpoint_every=K, vel=vel, inflow=inflow)
        out["eta"] = geta.double().cpu().numpy().reshape(p.shape)
    torch.cuda.synchronize()
    out["L"] = float(Lval.item())
    out["ka"] = gka.double().cpu().numpy().reshape(p.shape)
    out["ks"] = gks.double().cpu().numpy().reshape(p.shape)
    ctx.close()
    return out


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
@pytest.mark.parametrize("moving,bc,planes", [
    (False, (wl.BC_OUTFLOW,) * 6, 0),
    (True, (wl.BC_INFLOW, wl.BC_OUTFLOW, wl.BC_PERIODIC, wl.BC_PERIODIC, wl.BC_OUTFLOW,
            wl.BC_INFLOW), 3),
])
def test_adjoint_matches_oracle(storage, tol, moving, bc, planes):
    st = {"fp64": gh.lib().LBRT_FP64, "fp32": gh.lib().LBRT_FP32}[storage]
    p = _f64(wl.random_problem(61, shape=(7, 9, 70), npoints=26, steps=5, moving_fluid=moving,
                               vmax=0.5, bc=bc, inflow_planes=planes, kappa_range=(-1.5, 1.5)))
    got = _gpu_gradient(p, st, steps=5, face=wl.FACE_PX, K=2)
    L, gka, gks, geta = orc.detected_energy_gradient(p, 5, face=wl.FACE_PX, I0=got["I0_eff"])
    errs = {k: gh.rel_l2(got[k], ref) for k, ref in (("ka", gka), ("ks", gks), ("eta", geta))}
    print(f"L {got['L']:.12g} vs {L:.12g}; grad rel L2 {errs}", flush=True)
    assert abs(got["L"] - L) < tol * abs(L)
    assert max(errs.values()) < tol


@pytest.mark.parametrize("face", [wl.FACE_MY, wl.FACE_PY, wl.FACE_PZ, wl.FACE_MZ])
def test_adjoint_detector_on_y_and_z_faces(face):
    """Detector faces other than x on a box with non-periodic x and y: at
    edge and corner cells part of a population's outflux is booked on an
    earlier face (x before y before z), so the adjoint's detector weights
    must follow that rule for the returned L and gradient to belong to one
    objective.  FP64, against the oracle's L and gradient."""
    p = _f64(wl.random_problem(63, shape=(7, 9, 70), npoints=26, steps=4, moving_fluid=True,
                               vmax=0.4, bc=(wl.BC_OUTFLOW,) * 6, kappa_range=(-1.0, 1.0)))
    got = _gpu_gradient(p, gh.lib().LBRT_FP64, steps=4, face=face, K=2)
    L, gka, gks, geta = orc.detected_energy_gradient(p, 4, face=face, I0=got["I0_eff"])
    errs = {k: gh.rel_l2(got[k], ref) for k, ref in (("ka", gka), ("ks", gks), ("eta", geta))}
    print(f"face {face}: L {got['L']:.15g} vs {L:.15g}; grad rel L2 {errs}", flush=True)
    assert abs(got["L"] - L) < 1e-12 * abs(L)
    assert max(errs.values()) < 1e-10


_SHEAR32 = {}


def _shear32_oracle():
    """The oracle's L and gradient for the 32^3 shear-flow run over the full
    64 steps (computed once: about a minute of numpy)."""
    if not _SHEAR32:
        p = _f64(wl.moving(n=32, steps=64))
        _SHEAR32["p"] = p
        _SHEAR32["ref"] = orc.detected_energy_gradient(p, 64, face=wl.FACE_PX)
    return _SHEAR32["p"], _SHEAR32["ref"]


@pytest.mark.parametrize("storage,tol_L,tol_g", [("fp64", 1e-12, 1e-10), ("fp32", 1e-5, 5e-4)])
def test_adjoint_shear_flow_32(storage, tol_L, tol_g):
    """The moving-fluid workload (log-normal kappa_a, relativistic shear flow,
    146 directions) at 32^3 over its full 64 steps, checkpointed every 8,
    gradient of the energy leaving through +x with eta = kappa_a (B = 1):
    d/dkappa_a = g_kappa_a + g_eta.  FP64 storage to 1e-10; FP32 to 5e-4
    (its rounding accumulates over 64 steps forward and 64 back)."""
    p, (L, gka, gks, geta) = _shear32_oracle()
    st = {"fp64": gh.lib().LBRT_FP64, "fp32": gh.lib().LBRT_FP32}[storage]
    # FP32: through the autograd Function (float32 leaves, so float32
    # gradients); FP64: the library's FP64 gradients, eta a field of its own
    # equal to kappa_a, so d/dkappa_a = g_kappa_a + g_eta
    got = _gpu_gradient(p, st, steps=64, face=wl.FACE_PX, K=8, lte=storage == "fp32")
    if storage == "fp64":
        got["ka"] = got["ka"] + got["eta"]
    e_ka = gh.rel_l2(got["ka"], gka + geta)
    e_ks = gh.rel_l2(got["ks"], gks)
    print(f"{storage}: L {got['L']:.12g} vs {L:.12g}; grad rel L2 ka {e_ka:.3e} ks {e_ks:.3e}",
          flush=True)
    assert abs(got["L"] - L) < tol_L * abs(L)
    assert e_ka < tol_g and e_ks < tol_g


def test_adjoint_rejects_unsupported_modes():
    L = gh.lib()
    torch = gh.torch_mod()
    p = wl.random_problem(3, shape=(6, 6, 6), npoints=14, steps=1)
    for kw in ({"storage": L.LBRT_BF16}, {"collision": L.LBRT_COLL_EXPLICIT}):
        ctx = L.lbrt_init(L.Desc.from_problem(p, **kw))
        st = kw.get("storage", L.LBRT_FP32)
        dt = gh.pop_torch_dtype(st)
        n = p.ndir * p.ncell
        a = torch.zeros(n, dtype=dt, device="cuda")
        b = torch.zeros(n, dtype=dt, device="cuda")
        c = torch.zeros(n, dtype=dt, device="cuda")
        g = torch.zeros(p.ncell, dtype=torch.float32, device="cuda")
        with pytest.raises(L.LbrtError) as ei:
            L.lbrt_adjoint_step(ctx, a, b, c, 1, g, g.clone(), g.clone(), g, g, g)
        assert ei.value.code == L.LBRT_E_UNSUPPORTED
        ctx.close()
