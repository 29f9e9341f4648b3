"""GPU test of the launch-shape autotuner: it times candidate tilings through
the C-ABI, leaves the fastest set on the context, keeps I_a intact, and the
tuned tiling gives bit-identical results to the default one."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def test_tune_step_applies_best_and_changes_no_result():
    torch = gh.torch_mod()
    L = gh.lib()
    from paper_2007_05718_amd import autotune as at

    prob = wl.random_problem(21, shape=(40, 70, 96), npoints=50)
    print(prob.name, prob.shape, prob.ndir, flush=True)
    desc = L.Desc.from_problem(prob, storage=L.LBRT_FP32)
    ctx = L.lbrt_init(desc)
    Ia, _ = gh.host_encoded_state(np.asarray(prob.I0).reshape(prob.ndir, -1), prob.weights,
                                  L.LBRT_FP32)
    Ia = Ia.reshape(-1).contiguous()
    Ia_copy = Ia.clone()
    Ib = torch.empty_like(Ia)
    ka, ks, eta, vel, inflow = gh.upload_fields(prob)

    default = at.Tiling(*L.lbrt_get_tiling(ctx))
    L.lbrt_step(ctx, Ia, Ib, ka, ks, eta, vel=vel, inflow=inflow or None, nsteps=1)
    torch.cuda.synchronize()
    ref = Ib.clone()

    cands = [default, at.Tiling(32, 2, 16, 4), at.Tiling(16, 4, 40, 8), at.Tiling(8, 8, 8, 16)]
    rep = at.tune_step(ctx, Ia, Ib, ka, ks, eta, vel=vel, inflow=inflow or None,
                       candidates=cands, steps=2)
    assert rep.default == default
    assert {t for t, _ in rep.timings} == set(cands)
    assert all(ms > 0 for _, ms in rep.timings)
    assert rep.best_ms == min(ms for _, ms in rep.timings)
    assert L.lbrt_get_tiling(ctx) == rep.best.as_tuple()
    assert torch.equal(Ia, Ia_copy)

    for t in cands:
        L.lbrt_set_tiling(ctx, *t.as_tuple())
        Ib.zero_()
        L.lbrt_step(ctx, Ia, Ib, ka, ks, eta, vel=vel, inflow=inflow or None, nsteps=1)
        torch.cuda.synchronize()
        assert torch.equal(Ib, ref), t
    ctx.close()


def test_tune_batch_per_class_changes_no_result():
    """tune_batch groups a batch's domains by problem key, times candidate
    tilings on batched launches of each group, leaves the fastest set on
    every context of the group, and a batch created afterwards gives the same
    bits as one with the default tilings."""
    torch = gh.torch_mod()
    L = gh.lib()
    from paper_2007_05718_amd import autotune as at

    probs = [wl.batch_domain(d, seed=9, edges=(24, 40), steps_range=(3, 6)) for d in range(10)]

    def domains():
        out = []
        for p in probs:
            ctx = L.lbrt_init(L.Desc.from_problem(p, storage=L.LBRT_FP32))
            f = lambda v: torch.full((p.ncell,), float(v), dtype=torch.float32, device="cuda")
            rng = np.random.default_rng(p.nx)
            I0 = torch.from_numpy((rng.uniform(0, 1, (p.ndir, p.ncell)) *
                                   p.weights[:, None]).astype(np.float32).reshape(-1)).cuda()
            out.append(dict(ctx=ctx, I_a=I0, I_b=torch.empty_like(I0),
                            kappa_a=f(p.meta["kappa_a"]), kappa_s=f(p.meta["kappa_s"]),
                            eta=f(p.meta["kappa_a"]), nsteps=p.steps, start=I0.clone()))
        return out

    ref = domains()
    b = L.lbrt_batch_create([{k: v for k, v in dm.items() if k != "start"} for dm in ref])
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    b.close()

    tuned = domains()
    plain = [{k: v for k, v in dm.items() if k != "start"} for dm in tuned]
    reps = at.tune_batch(plain, steps=1, max_candidates=4, reps=1)
    keys = {at.problem_key(dm["ctx"]) for dm in tuned}
    assert {r.key for r in reps} == keys and sum(r.domains for r in reps) == len(tuned)
    for r in reps:
        assert r.best_ms == min(ms for _, ms in r.timings)
        for dm in tuned:
            if at.problem_key(dm["ctx"]) == r.key:
                assert L.lbrt_get_tiling(dm["ctx"]) == r.best.as_tuple()
    # tuning advanced the states: start again from the same initial states
    for dm in tuned:
        dm["I_a"].copy_(dm["start"])
    b = L.lbrt_batch_create(plain)
    L.lbrt_step_batched(b)
    torch.cuda.synchronize()
    b.close()
    for a, c in zip(ref, tuned):
        out_a = a["I_b"] if a["nsteps"] % 2 else a["I_a"]
        out_c = c["I_b"] if c["nsteps"] % 2 else c["I_a"]
        assert torch.equal(out_a, out_c)
        a["ctx"].close()
        c["ctx"].close()
