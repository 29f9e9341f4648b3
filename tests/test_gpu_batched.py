"""GPU tests of the batched form: domains of uneven size, opacity and step
count advanced together (one launch per step over all running domains) give
bit-for-bit the results of the same domains run one by one with lbrt_step,
replay identically from a captured graph, and match the FP64 oracle on
sampled domains."""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _domains(n, seed=4, edges=(8, 12, 16, 24, 33), steps_range=(1, 9)):
    """Batched-sweep domains (small edges so the oracle finishes) with a
    seeded random initial state."""
    probs = []
    for d in range(n):
        p = wl.batch_domain(d, seed=seed, edges=edges, steps_range=steps_range)
        rng = np.random.default_rng([seed, d, 1])
        p.I0 = rng.uniform(0, 1, (p.ndir,) + p.shape) * p.weights[:, None, None, None]
        probs.append(p)
    return probs


def _setup(probs, L, torch):
    doms = []
    for p in probs:
        ctx = L.lbrt_init(L.Desc.from_problem(p, storage=L.LBRT_FP32))
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
        I0 = f(p.I0)
        doms.append(dict(ctx=ctx, I_a=I0.clone(), I_b=torch.zeros_like(I0), I0=I0,
                         kappa_a=f(p.kappa_a), kappa_s=f(p.kappa_s), eta=f(p.eta),
                         nsteps=p.steps,
                         E=torch.zeros(p.ncell, device="cuda"),
                         F=torch.zeros(3 * p.ncell, device="cuda")))
    return doms


def _result(dm):
    return dm["I_b"] if dm["nsteps"] % 2 == 1 else dm["I_a"]


def test_batched_equals_sequential_bitwise():
    torch = gh.torch_mod()
    L = gh.lib()
    probs = _domains(24)
    doms = _setup(probs, L, torch)
    b = L.lbrt_batch_create(doms)
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    for p, dm in zip(probs, doms):
        Ia, Ib = dm["I0"].clone(), torch.zeros_like(dm["I0"])
        E = torch.zeros(p.ncell, device="cuda")
        L.lbrt_step(dm["ctx"], Ia, Ib, dm["kappa_a"], dm["kappa_s"], dm["eta"],
                    nsteps=p.steps, E=E)
        ref = Ib if p.steps % 2 == 1 else Ia
        torch.cuda.synchronize()
        assert torch.equal(_result(dm), ref), p.name
        assert torch.equal(dm["E"], E), p.name
    b.close()


def test_batched_graph_replays_match_eager():
    torch = gh.torch_mod()
    L = gh.lib()
    probs = _domains(12, seed=9)
    doms = _setup(probs, L, torch)
    b = L.lbrt_batch_create(doms)

    def reset():
        for dm in doms:
            dm["I_a"].copy_(dm["I0"])
            dm["I_b"].zero_()

    reset()
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    eager = [_result(dm).clone() for dm in doms]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        L.lbrt_step_batched(b, stream=s.cuda_stream)
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for dm, ref in zip(doms, eager):
            assert torch.equal(_result(dm), ref), rep
    b.close()


def test_batched_matches_oracle_on_sampled_domains():
    torch = gh.torch_mod()
    L = gh.lib()
    probs = _domains(16, seed=11, edges=(8, 12, 17), steps_range=(1, 4))
    doms = _setup(probs, L, torch)
    b = L.lbrt_batch_create(doms)
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    for p, dm in list(zip(probs, doms))[::3]:
        I0 = dm["I0"].double().cpu().numpy().reshape((p.ndir,) + p.shape)
        ref = orc.run(p, I0=I0)
        got = _result(dm).double().cpu().numpy().reshape(ref.shape)
        err = gh.rel_l2(got, ref)
        print(p.name, p.shape, p.steps, f"{err:.2e}", flush=True)
        assert err < 1e-5
    b.close()


@pytest.mark.skip(reason="the single persistent launch (a step-major work queue with per-domain "
                  "completion counters and spin waits) went silent in both of its GPU runs; "
                  "its polling invalidated the L2 on every iteration.  It is switched off: the "
                  "batched form runs one multi-domain launch per step instead")
def test_persistent_single_launch_batched_kernel():
    pass


def test_c4_recipe_domains_bitwise_and_oracle():
    """16 domains drawn with the sweep's own recipe (edges 24..96, 50..400
    steps, zero start): batched equals one-by-one bit for bit on all, and the
    smallest domain matches the FP64 oracle over its full run."""
    torch = gh.torch_mod()
    L = gh.lib()
    probs = [wl.batch_domain(d, seed=4) for d in range(16)]
    for p in probs:
        p.I0 = np.zeros((p.ndir,) + p.shape)
    print([(p.nx, p.steps) for p in probs], flush=True)
    doms = _setup(probs, L, torch)
    b = L.lbrt_batch_create(doms)
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    for p, dm in zip(probs, doms):
        Ia, Ib = dm["I0"].clone(), torch.zeros_like(dm["I0"])
        E = torch.zeros(p.ncell, device="cuda")
        L.lbrt_step(dm["ctx"], Ia, Ib, dm["kappa_a"], dm["kappa_s"], dm["eta"],
                    nsteps=p.steps, E=E)
        ref = Ib if p.steps % 2 == 1 else Ia
        torch.cuda.synchronize()
        assert torch.equal(_result(dm), ref), p.name
        assert torch.equal(dm["E"], E), p.name
    k = min(range(16), key=lambda j: (probs[j].ncell, probs[j].steps))
    p = probs[k]
    I = orc.run(p, I0=np.zeros((p.ndir,) + p.shape))
    got = _result(doms[k]).double().cpu().numpy().reshape(I.shape)
    err = gh.rel_l2(got, I)
    print(p.name, p.shape, p.steps, f"{err:.2e}", flush=True)
    assert err < 1e-5
    b.close()
