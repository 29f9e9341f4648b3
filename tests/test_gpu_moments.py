"""GPU test of lbrt_moments (E and F of a stored state) against the oracle's
moments, for FP32 and BF16 storage, including the optically thick diffusion
state whose flux is a small difference of terms of size E."""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _moments(prob, storage, I0):
    torch = gh.torch_mod()
    L = gh.lib()
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=storage))
    state, eff = gh.host_encoded_state(np.asarray(I0).reshape(prob.ndir, -1), prob.weights,
                                       storage)
    E = torch.empty(prob.ncell, device="cuda")
    F = torch.empty(3 * prob.ncell, device="cuda")
    L.lbrt_moments(ctx, state.reshape(-1).contiguous(), E=E, F=F)
    torch.cuda.synchronize()
    ctx.close()
    Er, Fr = orc.moments(eff.reshape((prob.ndir,) + prob.shape), prob.dirs)
    return (E.double().cpu().numpy().reshape(prob.shape),
            F.double().cpu().numpy().reshape((3,) + prob.shape), Er, Fr)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_moments_of_random_state(storage):
    L = gh.lib()
    st = {"fp32": L.LBRT_FP32, "bf16": L.LBRT_BF16}[storage]
    p = wl.random_problem(61, shape=(9, 14, 70), npoints=110)
    E, F, Er, Fr = _moments(p, st, p.I0)
    assert gh.rel_l2(E, Er) < 1e-6
    assert gh.rel_l2(F, Fr) < 1e-6


def test_moments_of_thick_state_keep_the_flux():
    L = gh.lib()
    p = wl.diffusion(n=64, sigma=4.0)
    # one oracle step builds a thick-cell flux of ~1e-4 E
    I1 = orc.step(np.asarray(p.I0, dtype=np.float64), p)
    E, F, Er, Fr = _moments(p, L.LBRT_FP32, I1)
    print(f"|F|/|E| {np.linalg.norm(Fr) / np.linalg.norm(Er):.2e} "
          f"E {gh.rel_l2(E, Er):.2e} F {gh.rel_l2(F, Fr):.2e}", flush=True)
    assert gh.rel_l2(E, Er) < 1e-6
    assert gh.rel_l2(F, Fr) < 1e-5
