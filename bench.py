"""Throughput of the fused radiative-transfer LB stream-collide step on one MI355X.

A step is one fused stream-and-collide pass (trilinear pull with inflow and
vacuum faces, per-cell moments, implicit collision, store of the new
populations, E and F, and the FP64 boundary/energy diagnostics) over the
crossing-beams-plus-shadow workload: 256^3 cells, the 110-direction
degree-17 Lebedev rule, FP32 population storage.

Prints ONE JSON line.  `value` is cell-direction updates per second (GDUPS)
of the FP32 form with all inputs resident in HBM.  The roofline entry is
for the fused step (its main and boundary kernels, one lbrt_step call
without diagnostics): algorithmic bytes per call over the call's mean
duration, timed with HIP events on the stream the kernels run on; beside it
the rate of a hand-written streaming copy on the same GPU.
Further forms on the same GPU:
* BF16 and FP16 storage of the same workload, each with its error against
  the FP64 oracle over the full 500-step run of the workload scaled to 64^3
  (the oracle's moments are the committed tests/golden/beams64_500.npz);
* the collision kinds (explicit, Lambda iteration with 5 cycles, implicit)
  on the beams geometry with capped opacities, where the explicit step is
  stable (the cost comparison of the paper's Sec. 6);
* the batched sweep of 512 uneven domains (two multi-domain launches per
  step), eager and as a replayed graph, against the same domains run one by
  one;
* the moving-fluid run with its adjoint (forward steps and the checkpointed
  reverse sweep).
The CPU baseline is the FP64 oracle (test infrastructure) timed on a bounded
sample of the same workload on this host, on one core and on all cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-direction updates/s (GDUPS) and % HBM peak, FP32 vs BF16-storage"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources that define the timed step launch (its kernels, their launch
# configuration and the diagnostics kernels); the counter summary's traffic
# figure holds while their digest is unchanged.
STEP_SOURCES = ("lbrt_step_kernel.h", "lbrt_internal.h", "lbrt_api.cpp", "lbrt_misc.hip",
                "lbrt_k_f32_112s.hip")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_05718_amd", "csrc")
    for f in STEP_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_cell(ndir: int, pop_bytes: int, moment_bytes: int = 4) -> float:
    """One read and one write of every population, the three coefficient
    fields (kappa_a, kappa_s, eta: 12 B) and the E, F outputs (4 values)."""
    return ndir * 2 * pop_bytes + 12 + 4 * moment_bytes


def time_form(L, torch, prob, storage, steps, warmup, with_outputs=True):
    """Returns (mean ms per step over the timed region, mean kernel ms)."""
    desc = L.Desc.from_problem(prob, storage=storage)
    ctx = L.lbrt_init(desc)
    Ia = L.alloc_state(ctx).zero_()
    Ib = L.alloc_state(ctx).zero_()
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    ka, ks, eta = f(prob.kappa_a), f(prob.kappa_s), f(prob.eta)
    inflow = [(p.face, p.direction, f(p.values)) for p in prob.inflow]
    mdt = torch.float64 if storage == L.LBRT_FP64 else torch.float32
    E = torch.empty(prob.ncell, dtype=mdt, device="cuda") if with_outputs else None
    F = torch.empty(3 * prob.ncell, dtype=mdt, device="cuda") if with_outputs else None
    diag = torch.zeros(L.LBRT_DIAG_LEN, dtype=torch.float64, device="cuda") if with_outputs else None
    bufs = [Ia, Ib]
    stream = torch.cuda.current_stream()

    def one(k, events=None):
        a, b = bufs[k % 2], bufs[(k + 1) % 2]
        if events is not None:
            events[0].record(stream)
        L.lbrt_step(ctx, a, b, ka, ks, eta, inflow=inflow or None, nsteps=1, E=E, F=F,
                    diag=diag, stream=stream.cuda_stream)
        if events is not None:
            events[1].record(stream)

    for k in range(warmup):
        one(k)
    torch.cuda.synchronize()
    # Per-launch kernel time: events bracket each lbrt_step call.  With
    # outputs on, a call is the step kernel plus the tiny diagnostics
    # reduction; kernel-only time comes from a second pass without outputs.
    t0 = time.perf_counter()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for k in range(steps):
        one(warmup + k, evs[k])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per_call = [a.elapsed_time(b) for a, b in evs]
    del Ia, Ib
    ctx.close()
    return wall, float(np.mean(per_call)), float(np.min(per_call))


def kernel_only_ms(L, torch, prob, storage, steps):
    """Mean duration of the step kernel alone (E, F written, no diagnostics)."""
    desc = L.Desc.from_problem(prob, storage=storage)
    ctx = L.lbrt_init(desc)
    Ia = L.alloc_state(ctx).zero_()
    Ib = L.alloc_state(ctx).zero_()
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    ka, ks, eta = f(prob.kappa_a), f(prob.kappa_s), f(prob.eta)
    inflow = [(p.face, p.direction, f(p.values)) for p in prob.inflow]
    E = torch.empty(prob.ncell, dtype=torch.float32, device="cuda")
    F = torch.empty(3 * prob.ncell, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    bufs = [Ia, Ib]
    for k in range(3):
        L.lbrt_step(ctx, bufs[k % 2], bufs[(k + 1) % 2], ka, ks, eta, inflow=inflow or None,
                    E=E, F=F, stream=stream.cuda_stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for k in range(steps):
        evs[k][0].record(stream)
        L.lbrt_step(ctx, bufs[k % 2], bufs[(k + 1) % 2], ka, ks, eta, inflow=inflow or None,
                    E=E, F=F, stream=stream.cuda_stream)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    ctx.close()
    return float(np.mean(ms))


def copy_ceiling_gbs(L, torch, nbytes: int = 4 << 30, reps: int = 10) -> dict:
    """Read+write bandwidth of a plain device-to-device copy: the library's
    hand-written streaming copy (16-byte loads, non-temporal stores) and
    torch's copy kernel, same buffers."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("stream_copy", lambda: L.lbrt_stream_copy(a, b, stream=stream.cuda_stream)),
                     ("torch_copy", lambda: b.copy_(a))):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    return out


def form_error(L, torch, storage) -> dict:
    """Error of a storage form against the FP64 oracle over the full run of
    the beams workload scaled to 64^3 (500 steps from zero): relative L2 and
    max |d| / max |ref| of E and of F."""
    import workloads as wl
    path = os.path.join(ROOT, "tests", "golden", "beams64_500.npz")
    ref = np.load(path)
    prob = wl.beams(n=int(ref["n"]), steps=int(ref["steps"]), alloc_state=False)
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=storage))
    Ia = L.alloc_state(ctx).zero_()
    Ib = L.alloc_state(ctx).zero_()
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    inflow = [(p.face, p.direction, f(p.values)) for p in prob.inflow]
    E = torch.empty(prob.ncell, device="cuda")
    F = torch.empty(3 * prob.ncell, device="cuda")
    L.lbrt_step(ctx, Ia, Ib, f(prob.kappa_a), f(prob.kappa_s), f(prob.eta), inflow=inflow,
                nsteps=prob.steps, E=E, F=F)
    torch.cuda.synchronize()
    e = E.double().cpu().numpy().reshape(prob.shape)
    fl = F.double().cpu().numpy().reshape((3,) + prob.shape)
    ctx.close()
    Er, Fr = ref["E"], ref["F"]
    l2 = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    return {"workload": f"beams {prob.nx}^3 x {prob.ndir}, {prob.steps} steps, vs FP64 oracle",
            "E_rel_l2": float(f"{l2(e, Er):.3e}"), "F_rel_l2": float(f"{l2(fl, Fr):.3e}"),
            "E_max_rel": float(f"{np.max(np.abs(e - Er)) / np.max(np.abs(Er)):.3e}"),
            "F_max_rel": float(f"{np.max(np.abs(fl - Fr)) / np.max(np.abs(Fr)):.3e}")}


def time_collisions(L, torch, n: int, steps: int, warmup: int) -> dict:
    """ms per step of the three collision kinds (FP32, no outputs) on the
    beams geometry with capped opacities, and each one's ratio to the
    implicit (closed-form) step."""
    import workloads as wl
    prob = wl.beams_costs(n=n, alloc_state=False)
    out = {"workload": f"beams geometry {n}^3 x {prob.ndir}, kappa_a <= 1, kappa_s = 0.5, "
                       "FP32, no outputs"}
    kinds = (("implicit", L.LBRT_COLL_IMPLICIT, 1), ("explicit", L.LBRT_COLL_EXPLICIT, 1),
             ("lambda5", L.LBRT_COLL_LAMBDA, 5))
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    ka, ks, eta = f(prob.kappa_a), f(prob.kappa_s), f(prob.eta)
    inflow = [(p.face, p.direction, f(p.values)) for p in prob.inflow]
    nn = prob.ndir * prob.ncell
    Ia = torch.zeros(nn, device="cuda")
    Ib = torch.zeros(nn, device="cuda")
    stream = torch.cuda.current_stream()
    for name, coll, iters in kinds:
        ctx = L.lbrt_init(L.Desc.from_problem(prob, collision=coll, lambda_iters=iters))
        bufs = [Ia, Ib]
        for k in range(warmup):
            L.lbrt_step(ctx, bufs[k % 2], bufs[(k + 1) % 2], ka, ks, eta, inflow=inflow,
                        stream=stream.cuda_stream)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for k in range(steps):
            evs[k][0].record(stream)
            L.lbrt_step(ctx, bufs[k % 2], bufs[(k + 1) % 2], ka, ks, eta, inflow=inflow,
                        stream=stream.cuda_stream)
            evs[k][1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        out[name] = {"ms_per_step": round(ms, 4),
                     "GDUPS": round(prob.ndir * prob.ncell / (ms * 1e-3) / 1e9, 2)}
        ctx.close()
    for name, _, _ in kinds:
        out[name]["ratio_to_implicit"] = round(out[name]["ms_per_step"]
                                               / out["implicit"]["ms_per_step"], 3)
    del Ia, Ib
    return out


def time_coupling(L, torch, prob, reps: int = 10) -> dict:
    """lbrt_coupling on an FP32 state of the workload with a sheared flow:
    every output (E, F, P, J, H, S: 19 values per cell) from the 110
    populations, the velocity and the three opacity fields.  Algorithmic
    bytes per cell: 110 x 4 + 3 x 4 + 3 x 4 read, 19 x 4 written."""
    n = prob.ncell
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=L.LBRT_FP32))
    g = torch.Generator(device="cuda").manual_seed(31)
    I = torch.rand(prob.ndir * n, generator=g, device="cuda")
    y = torch.arange(prob.ny, device="cuda", dtype=torch.float32)
    vel = torch.zeros(3, *prob.shape, device="cuda")
    vel[0] = (0.5 * torch.tanh((y - prob.ny * 0.375) / 8.0))[None, :, None]
    vel = vel.reshape(-1)
    fld = torch.rand(3, n, generator=g, device="cuda")
    outs = {k: torch.empty(m * n, device="cuda")
            for k, m in (("E", 1), ("F", 3), ("P", 6), ("J", 1), ("H", 4), ("S", 4))}
    stream = torch.cuda.current_stream()
    call = lambda: L.lbrt_coupling(ctx, I, vel=vel, kappa_a=fld[0], kappa_s=fld[1], eta=fld[2],
                                   stream=stream.cuda_stream, **outs)
    call()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        call()
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    bpc = prob.ndir * 4 + 24 + 19 * 4
    ctx.close()
    del I, outs, fld, vel
    return {"workload": f"{prob.nx}^3 x {prob.ndir} FP32 state, sheared flow, all 19 outputs "
                        "(FP64 sums)", "ms": round(ms, 4),
            "bytes_per_cell_algorithmic": bpc,
            "hbm_GBs_algorithmic": round(bpc * n / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(bpc * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def time_batched(L, torch, ndomains=512, seed=4, sequential=True, tune=True):
    """The batched opacity sweep: one lbrt_step_batched call against the same
    domains advanced one by one with lbrt_step (unless sequential=False).
    Returns a dict."""
    import workloads as wl
    probs = [wl.batch_domain(d, seed=seed) for d in range(ndomains)]
    f = lambda v, n: torch.full((n,), float(v), dtype=torch.float32, device="cuda")
    doms = []
    updates = 0
    for p in probs:
        ctx = L.lbrt_init(L.Desc.from_problem(p, storage=L.LBRT_FP32))
        n = p.ndir * p.ncell
        doms.append(dict(ctx=ctx, I_a=torch.zeros(n, device="cuda"),
                         I_b=torch.zeros(n, device="cuda"),
                         kappa_a=f(p.meta["kappa_a"], p.ncell),
                         kappa_s=f(p.meta["kappa_s"], p.ncell),
                         eta=f(p.meta["kappa_a"], p.ncell), nsteps=p.steps))
        updates += n * p.steps
    b = L.lbrt_batch_create(doms)
    stream = torch.cuda.current_stream()
    L.lbrt_step_batched(b)          # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.lbrt_step_batched(b)
    e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) * 1e-3
    # the same sweep captured once in a graph and replayed
    gs = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=gs):
        L.lbrt_step_batched(b, stream=gs.cuda_stream)
    g.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    t_graph = e0.elapsed_time(e1) * 1e-3
    out = {"domains": ndomains, "updates": updates,
           "GDUPS": round(updates / t_batch / 1e9, 2), "seconds": round(t_batch, 3),
           "graph_GDUPS": round(updates / t_graph / 1e9, 2), "graph_seconds": round(t_graph, 3),
           "launches": 2 * max(p.steps for p in probs),
           "hbm_GBs_algorithmic": round(updates * algorithmic_bytes_per_cell(50, 4) / 50
                                        / t_batch / 1e9, 1)}
    del g
    if sequential:
        e0.record(stream)
        for dm in doms:
            L.lbrt_step(dm["ctx"], dm["I_a"], dm["I_b"], dm["kappa_a"], dm["kappa_s"],
                        dm["eta"], nsteps=dm["nsteps"])
        e1.record(stream)
        torch.cuda.synchronize()
        t_seq = e0.elapsed_time(e1) * 1e-3
        out.update({"sequential_GDUPS": round(updates / t_seq / 1e9, 2),
                    "sequential_seconds": round(t_seq, 3),
                    "speedup_vs_sequential": round(t_seq / t_batch, 3)})
    b.close()
    if tune:
        # the tiling of each edge class tuned on batched launches of that
        # class alone, then the same sweep again
        from paper_2007_05718_amd import autotune
        reps = autotune.tune_batch(doms)
        b = L.lbrt_batch_create(doms)
        L.lbrt_step_batched(b)
        torch.cuda.synchronize()
        e0.record(stream)
        L.lbrt_step_batched(b)
        e1.record(stream)
        torch.cuda.synchronize()
        t_tuned = e0.elapsed_time(e1) * 1e-3
        out.update({"tuned_GDUPS": round(updates / t_tuned / 1e9, 2),
                    "tuned_seconds": round(t_tuned, 3),
                    "tuned_tilings": {r.key.split("|")[0]: "%dx%d z%d/%d" % r.best.as_tuple()
                                      for r in reps}})
        b.close()
    for dm in doms:
        dm["ctx"].close()
    return out


def time_adjoint(L, torch, n=192, steps=64, K=8):
    """The moving-fluid workload: steps forward FP32 steps, then the gradient of
    the energy leaving through +x with respect to kappa_a (eta = kappa_a)."""
    import workloads as wl
    from paper_2007_05718_amd import autodiff
    p = wl.moving(n=n, steps=steps, alloc_state=False)
    ctx = L.lbrt_init(L.Desc.from_problem(p, storage=L.LBRT_FP32))
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).reshape(-1).cuda()
    ka = f(p.kappa_a).requires_grad_(True)
    ks, vel = f(p.kappa_s), f(p.vel)
    I0 = torch.zeros(p.ndir * p.ncell, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    Lval = autodiff.detected_energy(ctx, I0, ka, ks, ka * 1.0, steps, face=1,
                                    checkpoint_every=K, vel=vel)
    ev[1].record(stream)
    Lval.backward()
    ev[2].record(stream)
    torch.cuda.synchronize()
    tf = ev[0].elapsed_time(ev[1]) * 1e-3
    tb = ev[1].elapsed_time(ev[2]) * 1e-3
    updates = p.ndir * p.ncell * steps
    out = {"cells": p.ncell, "directions": p.ndir, "steps": steps, "checkpoint_every": K,
           "L": float(Lval.item()), "forward_seconds": round(tf, 3),
           "forward_GDUPS": round(updates / tf / 1e9, 2), "backward_seconds": round(tb, 3),
           "grad_norm": float(ka.grad.norm().item())}
    ctx.close()
    return out


def _oracle_slab_step(args):
    """One FP64 oracle step on z-planes [z0, z0 + planes) of the workload
    (a slab with vacuum cut faces); returns (updates, seconds)."""
    n, z0, planes, seed = args
    import copy

    import workloads as wl
    from oracle import lbrt_oracle as orc
    prob = wl.beams(n=n, alloc_state=False)
    q = copy.copy(prob)
    q.nz = planes
    q.kappa_a = prob.kappa_a[z0:z0 + planes]
    q.kappa_s = prob.kappa_s[z0:z0 + planes]
    q.eta = prob.eta[z0:z0 + planes]
    q.inflow = [wl.InflowPlane(p.face, p.direction,
                               p.values[z0:z0 + planes] if p.face in (0, 1, 2, 3) else p.values)
                for p in prob.inflow]
    rng = np.random.default_rng(seed)
    I = rng.uniform(0.0, 1.0, (q.ndir, planes, q.ny, q.nx)) * q.weights[:, None, None, None]
    t0 = time.perf_counter()
    orc.step(I, q)
    return q.ndir * q.ncell, time.perf_counter() - t0


def cpu_baseline(n: int, planes: int = 8, workers: int = 0) -> dict:
    """The FP64 oracle on this host: one step on slabs of `planes` z-planes of
    the workload, first on one core (two slabs in turn), then on all cores
    (one slab per worker process, in parallel).  Runs before the GPU is
    touched, so the worker processes start from a clean parent."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    workers = workers or min(ncpu, 16)
    one = [_oracle_slab_step((n, 8 * k, planes, k)) for k in range(2)]
    upd1 = sum(u for u, _ in one)
    sec1 = sum(t for _, t in one)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))       # start the workers
        t0 = time.perf_counter()
        res = pool.map(_oracle_slab_step,
                       [(n, (planes * k) % (n - planes), planes, 100 + k) for k in range(workers)])
        wall = time.perf_counter() - t0
    updn = sum(u for u, _ in res)
    return {"value": updn / wall / 1e9, "unit": "GDUPS", "cores": workers, "kind": "oracle",
            "single_core_GDUPS": upd1 / sec1 / 1e9, "host_cpus": ncpu,
            "sample": f"FP64 oracle (numpy), one step on {n}x{n}x{planes} slabs of the workload "
                      f"({planes * n * n * 110:.3g} updates each): 2 slabs on 1 core "
                      f"({sec1:.1f} s), then {workers} slabs on {workers} worker processes in "
                      f"parallel ({wall:.1f} s wall); host has {ncpu} CPUs"}


def traffic_entry(ndir, ncell):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled) from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_beams256_fp32_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"^([a-z_]+): (\S+)$", line.strip())
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("kernel_source_digest") != kernel_source_digest():
        return None
    return float(kv["bytes_per_launch"]) if "bytes_per_launch" in kv else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="grid edge (default 256)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--forms",
                    default="bf16,fp16,bf16_shifted,fp16_shifted,collisions,coupling,batched,"
                            "adjoint",
                    help="extra forms to time (bf16, fp16, bf16_shifted, fp16_shifted, "
                         "collisions, coupling, batched, adjoint)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched form: skip the one-domain-at-a-time comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not built).", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu:
        log("timing the oracle on the host (before the GPU is used)")
        cpu = cpu_baseline(args.n)

    import torch
    import paper_2007_05718_amd as L
    import workloads as wl

    log("generating workload")
    prob = wl.beams(n=args.n, alloc_state=False)
    ndir, ncell = prob.ndir, prob.ncell
    updates = ndir * ncell

    log("timing fp32")
    wall, call_ms, call_min = time_form(L, torch, prob, L.LBRT_FP32, args.steps, args.warmup)
    log("timing fp32 kernel alone")
    kms = kernel_only_ms(L, torch, prob, L.LBRT_FP32, args.steps)
    gdups = updates / (wall * 1e-3) / 1e9
    bpc = algorithmic_bytes_per_cell(ndir, 4)
    bytes_launch = bpc * ncell
    achieved = bytes_launch / (kms * 1e-3) / 1e9
    forms = {}
    names = [s for s in args.forms.split(",") if s]
    if any(n.startswith(("bf16", "fp16")) for n in names):
        log("fp32 error against the oracle (64^3, 500 steps)")
        forms["fp32_error_vs_oracle"] = form_error(L, torch, L.LBRT_FP32)
    for name in names:
        if name in ("bf16", "fp16", "bf16_shifted", "fp16_shifted"):
            st = {"bf16": L.LBRT_BF16, "fp16": L.LBRT_FP16, "bf16_shifted": L.LBRT_BF16_SHIFTED,
                  "fp16_shifted": L.LBRT_FP16_SHIFTED}[name]
            log(f"timing {name}")
            w2, c2, _ = time_form(L, torch, prob, st, args.steps, args.warmup)
            k2 = kernel_only_ms(L, torch, prob, st, args.steps)
            # (the shifted forms also read and write the cell's FP32 E: 8 B)
            b2 = (algorithmic_bytes_per_cell(ndir, 2) + (8 if "shifted" in name else 0)) * ncell
            forms[name] = {
                "GDUPS": round(updates / (w2 * 1e-3) / 1e9, 2),
                "ms_per_step": round(w2, 4),
                "kernel_ms": round(k2, 4),
                "hbm_GBs_algorithmic": round(b2 / (k2 * 1e-3) / 1e9, 1),
                "speedup_vs_fp32": round(wall / w2, 3),
                "error_vs_oracle": form_error(L, torch, st),
            }
        elif name == "collisions":
            log("timing the collision kinds")
            forms["collision_costs"] = time_collisions(L, torch, args.n, args.steps, args.warmup)
        elif name == "coupling":
            log("timing the coupling moments and sources")
            forms["coupling"] = time_coupling(L, torch, prob)
        elif name == "batched":
            log("timing the batched sweep (512 domains)")
            try:
                forms["batched_sweep_512"] = time_batched(
                    L, torch, sequential=not args.no_sequential)
            except Exception as exc:   # report, keep the headline line
                forms["batched_sweep_512"] = {"error": repr(exc)}
        elif name == "adjoint":
            log("timing the moving-fluid run and its adjoint")
            try:
                forms["moving_adjoint_192"] = time_adjoint(L, torch)
            except Exception as exc:
                forms["moving_adjoint_192"] = {"error": repr(exc)}
        torch.cuda.empty_cache()
    log("copy ceiling")
    copy_gbs = copy_ceiling_gbs(L, torch)
    tr = traffic_entry(ndir, ncell)
    out = {
        "metric": METRIC,
        "value": round(gdups, 2),
        "unit": "GDUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"crossing beams + opaque sphere, {args.n}^3 cells x {ndir}-direction "
                        "Lebedev (degree 17), FP32 population storage, implicit collision, "
                        "dt=0.5 dx, inflow (-x,-y) and vacuum faces, E/F and FP64 "
                        "diagnostics every step",
            "cells": ncell, "directions": ndir, "updates_per_step": updates,
            "hbm_pct_algorithmic": round(100.0 * gdups * bpc / ndir / HBM_PEAK_GBS, 2),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr,
            "kernel": "step_kernel_main<float,112> + step_kernel_general<float,112>",
            "kernel_ms": round(kms, 4),
            "bytes_per_launch_algorithmic": bytes_launch,
            "copy_kernel_GBs": copy_gbs["stream_copy"],
            "torch_copy_GBs": copy_gbs["torch_copy"],
            "frac_of_copy": round(achieved / copy_gbs["stream_copy"], 4),
        },
        "cpu_baseline": cpu,
        "forms": forms,
        "kernel_source_digest": kernel_source_digest(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
