"""Launch-shape autotuner for the fused step.

The step kernels march xy tiles of 64 cells through z ranges (see
``include/lbrt.h``, ``lbrt_set_tiling``).  The tile shape and the z-range
lengths change only the speed, never the result (every choice gives
bit-identical populations), so the best shape for a grid, direction bucket,
storage type and device can be picked by timing a few steps.

``tune_step`` times candidate tilings on the caller's own buffers and leaves
the fastest one set on the context.  It reads ``I_a`` and overwrites ``I_b``
only, so the state in ``I_a`` survives tuning.  ``TuningCache`` remembers the
choice per problem key in a JSON file, so a serving process tunes once.

The batched form (``lbrt_batch_create``) plans each domain with its context's
tiling at creation time.  ``tune_batch`` groups a batch's domains by problem
key (grid, directions, storage, fluid, boundaries) and times the candidate
tilings of each group on a batched launch of that group alone, since a small
domain runs very differently alone (a few blocks) and among hundreds of
others; the fastest tiling is set on every context of the group before the
caller creates the batch.

There is no direction-blocking dimension: a block owns all the directions of
its cells, because the collision needs every direction's streamed value of
a cell at once (the moments E*, F* over all directions).  Splitting the
directions over blocks would need a cross-block reduction of the moments per
cell and plane, or a second pass over the state, each a per-step cost where
the current split (the directions over the waves of one block, combined
through LDS) has none.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass, field
from typing import Iterable, List, Optional, Sequence, Tuple

from . import (Context, lbrt_batch_create, lbrt_get_tiling, lbrt_set_tiling, lbrt_step,
               lbrt_step_batched)

TILES: Tuple[Tuple[int, int], ...] = ((64, 1), (32, 2), (16, 4), (8, 8))
ZLENS: Tuple[int, ...] = (8, 16, 24, 32, 48, 64, 128)
ZLENS_GENERAL: Tuple[int, ...] = (4, 8, 16)


@dataclass(frozen=True)
class Tiling:
    tx: int
    ty: int
    zlen: int
    zlen_general: int

    def as_tuple(self) -> Tuple[int, int, int, int]:
        return (self.tx, self.ty, self.zlen, self.zlen_general)


@dataclass
class TuneReport:
    best: Tiling
    best_ms: float
    default: Tiling
    default_ms: float
    timings: List[Tuple[Tiling, float]] = field(default_factory=list)

    @property
    def speedup(self) -> float:
        return self.default_ms / self.best_ms if self.best_ms > 0 else 1.0


def candidate_tilings(nx: int, ny: int, nz: int, default: Optional[Tiling] = None,
                      tiles: Sequence[Tuple[int, int]] = TILES,
                      zlens: Sequence[int] = ZLENS,
                      zlens_general: Sequence[int] = ZLENS_GENERAL,
                      max_candidates: int = 24) -> List[Tiling]:
    """Candidate tilings for an nx x ny x nz grid, the default first.

    Tiles wider than the grid in x are skipped (their lanes would be idle);
    z ranges are clipped to nz and de-duplicated.  The z-range length of the
    boundary tiles is varied only around the best main-kernel candidates'
    default, which keeps the list short: the boundary kernel is a small part
    of a launch."""
    out: List[Tiling] = []
    seen = set()

    def add(t: Tiling):
        if t.as_tuple() not in seen:
            seen.add(t.as_tuple())
            out.append(t)

    if default is not None:
        add(default)
    zg0 = default.zlen_general if default is not None else 8
    xcover = max(8, 1 << max(0, int(nx) - 1).bit_length())   # next power of two >= nx
    for tx, ty in tiles:
        if tx * ty != 64 or tx & (tx - 1):
            raise ValueError(f"tile {tx}x{ty}: need tx*ty = 64, tx a power of two")
        if tx > xcover:
            # wider than the row: a narrower tile covers it without idle lanes
            continue
        for z in zlens:
            add(Tiling(tx, ty, min(int(z), nz), zg0))
    if default is not None:
        for zg in zlens_general:
            add(Tiling(default.tx, default.ty, min(default.zlen, nz), int(zg)))
    return out[:max_candidates]


def _time_one(ctx: Context, args: dict, torch, steps: int, stream) -> float:
    """Mean ms of `steps` single steps I_a -> I_b, events on the launch stream."""
    s = stream if stream is not None else torch.cuda.current_stream()
    lbrt_step(ctx, nsteps=1, stream=s.cuda_stream, **args)   # warm-up (and first-touch)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(s)
        lbrt_step(ctx, nsteps=1, stream=s.cuda_stream, **args)
        b.record(s)
    s.synchronize()
    return min(a.elapsed_time(b) for a, b in evs)


def tune_step(ctx: Context, I_a, I_b, kappa_a, kappa_s, eta, vel=None, inflow=None,
              E=None, F=None, diag=None, candidates: Optional[Iterable[Tiling]] = None,
              steps: int = 3, stream=None, apply: bool = True) -> TuneReport:
    """Times each candidate tiling on one step I_a -> I_b (best of `steps`)
    and sets the fastest on `ctx` (unless apply=False, which restores the
    tiling the context had).  Outputs E, F, diag, if given, are written as in
    a normal step: pass the ones the production loop uses so that the timed
    work is the same."""
    import torch

    d = ctx.desc.c
    default = Tiling(*lbrt_get_tiling(ctx))
    cands = list(candidates) if candidates is not None else candidate_tilings(
        d.nx, d.ny, d.nz, default)
    if default not in cands:
        cands.insert(0, default)
    args = dict(I_a=I_a, I_b=I_b, kappa_a=kappa_a, kappa_s=kappa_s, eta=eta, vel=vel,
                inflow=inflow, E=E, F=F, diag=diag)
    timings: List[Tuple[Tiling, float]] = []
    for t in cands:
        lbrt_set_tiling(ctx, *t.as_tuple())
        timings.append((t, _time_one(ctx, args, torch, steps, stream)))
    best, best_ms = min(timings, key=lambda x: x[1])
    default_ms = next(ms for t, ms in timings if t == default)
    lbrt_set_tiling(ctx, *(best if apply else default).as_tuple())
    return TuneReport(best=best, best_ms=best_ms, default=default, default_ms=default_ms,
                      timings=timings)


def problem_key(ctx: Context, device_name: str = "") -> str:
    """Key of a tuning result: grid, direction count, storage, fluid kind,
    boundary kinds and device."""
    d = ctx.desc.c
    bc = "".join(str(int(d.bc[f])) for f in range(6))
    return (f"{d.nx}x{d.ny}x{d.nz}|N{d.ndir}|s{int(d.storage)}|m{int(d.moving_fluid)}"
            f"|bc{bc}|{device_name}")


class TuningCache:
    """Tiling choices per problem key, kept in a JSON file."""

    def __init__(self, path: str):
        self.path = path
        self.entries: dict = {}
        if os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key: str) -> Optional[Tiling]:
        e = self.entries.get(key)
        return Tiling(**e["tiling"]) if e else None

    def put(self, key: str, report: TuneReport) -> None:
        self.entries[key] = {"tiling": asdict(report.best), "ms": report.best_ms,
                             "default_ms": report.default_ms}
        tmp = self.path + ".tmp"
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def apply_or_tune(self, ctx: Context, *args, device_name: str = "", **kw) -> Tiling:
        """Sets the cached tiling for ctx's problem, or tunes (tune_step with
        *args, **kw) and caches the result."""
        key = problem_key(ctx, device_name)
        t = self.get(key)
        if t is not None:
            lbrt_set_tiling(ctx, *t.as_tuple())
            return t
        rep = tune_step(ctx, *args, **kw)
        self.put(key, rep)
        return rep.best


@dataclass
class BatchTuneReport:
    key: str
    domains: int
    best: Tiling
    best_ms: float
    default: Tiling
    default_ms: float
    timings: List[Tuple[Tiling, float]] = field(default_factory=list)


def tune_batch(domains: Sequence[dict], steps: int = 2, device_name: str = "",
               max_candidates: int = 10, reps: int = 2) -> List[BatchTuneReport]:
    """Tunes the tiling of a batch's domains per problem-key group and sets
    the fastest on every context of the group (before the caller's
    ``lbrt_batch_create``).  ``domains`` are the dicts ``lbrt_batch_create``
    takes.  Each candidate is timed as one batched launch of the group alone
    with every domain running ``steps`` steps (best of ``reps``); the timing
    runs advance the domains' states, so tune before setting the initial
    states, or on copies."""
    import torch

    groups: dict = {}
    for dm in domains:
        groups.setdefault(problem_key(dm["ctx"], device_name), []).append(dm)
    reports: List[BatchTuneReport] = []
    for key, ds in groups.items():
        d = ds[0]["ctx"].desc.c
        default = Tiling(*lbrt_get_tiling(ds[0]["ctx"]))
        cands = candidate_tilings(d.nx, d.ny, d.nz, default, max_candidates=max_candidates)
        sub = [dict(dm, nsteps=steps) for dm in ds]
        timings: List[Tuple[Tiling, float]] = []
        for t in cands:
            for dm in ds:
                lbrt_set_tiling(dm["ctx"], *t.as_tuple())
            b = lbrt_batch_create(sub)
            s = torch.cuda.current_stream()
            lbrt_step_batched(b, stream=s.cuda_stream)   # warm-up
            best = float("inf")
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                lbrt_step_batched(b, stream=s.cuda_stream)
                e1.record(s)
                s.synchronize()
                best = min(best, e0.elapsed_time(e1))
            b.close()
            timings.append((t, best))
        bt, bms = min(timings, key=lambda x: x[1])
        dms = next(ms for t, ms in timings if t == default)
        for dm in ds:
            lbrt_set_tiling(dm["ctx"], *bt.as_tuple())
        reports.append(BatchTuneReport(key=key, domains=len(ds), best=bt, best_ms=bms,
                                       default=default, default_ms=dms, timings=timings))
    return reports
