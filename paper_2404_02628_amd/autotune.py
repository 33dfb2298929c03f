"""Autotuning of the launch choices that the library leaves to the caller.

For a fixed set of replicas the knobs are the recursion schedule (`recursion_workgroups`: 0 lets
the library choose, 1 forces one workgroup per replica and direction, k > 1 a cooperative chain
with k-1 helpers), the pair kernel and its work granularity (the symmetric per-slice kernel where
the library would pick it, or the ordered one with 1, 2 or 4 waves per 64-particle tile), the
packing of uneven replicas (work dispatched in replica order or longest replica first), replay of
steady steps from a HIP graph, and, for replicas small enough (N <= 64, d P N <= 512), the
persistent kernel that runs whole steps on chip.  `tune` times every
candidate for a few MD steps on the device and returns the fastest; `tune_replicas` picks the
batch size (replica count) with the highest aggregate replica-steps/s.  Both measure, so they
need a GPU; `candidates` and `pick` are plain functions that tests exercise without one.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Iterable, List, Optional, Sequence

from .workloads import System, initial_state


PERSIST_MAX_N = 64
PERSIST_MAX_DOF = 512


def persistent_fits(systems: Sequence[System]) -> bool:
    """Whether the library runs these replicas in its persistent kernel (unless told not to)."""
    return all(s.n <= PERSIST_MAX_N and s.dim * s.p * s.n <= PERSIST_MAX_DOF for s in systems)


@dataclass(frozen=True)
class Knobs:
    recursion_workgroups: int = 0
    pair_kernel: str = "auto"
    graphs: bool = False
    persistent: bool = False
    order: str = "index"      # "index" or "longest": dispatch order of the per-replica work
    pair_split: int = 0       # waves per tile of the ordered pair kernel (0: chosen by the library)
    wide: bool = False        # eight instead of four waves per one-workgroup recursion chain

    def as_kwargs(self) -> Dict:
        return {"recursion_workgroups": self.recursion_workgroups, "pair_kernel": self.pair_kernel,
                "graphs": self.graphs, "persistent": self.persistent, "order": self.order,
                "pair_split": self.pair_split, "wide_recursion": self.wide}


@dataclass
class TuneResult:
    best: Knobs
    seconds_per_step: Dict[Knobs, float] = field(default_factory=dict)


def candidates(systems: Sequence[System], precision: str, graphs: bool = False) -> List[Knobs]:
    """The candidate set for these replicas: schedules that differ in practice only.  Graph replay
    is a candidate only on request: once a process has captured and replayed a step graph, the
    ROCm runtime adds ~35 us to every later kernel dispatch of that process (measured on MI355X:
    a 15 us spring kernel then takes 46 us), so timing it would slow everything timed after it."""
    has_pair = any(s.pair_amp > 0 for s in systems)
    nblk = max((s.n + 64) // 64 for s in systems)
    scheds = [0, 1]
    if len(systems) <= 8 and nblk > 2:
        # a few cooperative helper counts between "one helper" and "as many as fit"
        scheds += sorted({h + 1 for h in (1, 4, 16, 32, 64, 128) if h < nblk - 1})
    sym = has_pair and precision == "mixed" and sum(s.p for s in systems if s.pair_amp > 0) >= 256
    # pair kernel and granularity: the library's choice, and where the symmetric kernel would run
    # also the ordered one at each tile split; the FP64 ordered kernel at each split
    pairs = [("auto", 0)]
    if has_pair:
        pairs += [("ordered", k) for k in (1, 2, 4)] if sym else [("auto", k) for k in (1, 2, 4)]
    orders = ["index", "longest"] if len({s.n for s in systems}) > 1 else ["index"]
    # eight-wave chains for the one-workgroup schedule while their workgroups (two per replica, one
    # compute unit each) leave room on a 256-CU device
    widths = (False, True) if 2 * len(systems) <= 256 else (False,)
    out = [Knobs(persistent=True)] if persistent_fits(systems) else []
    for r in scheds:
        for pk, split in pairs:
            for o in orders:
                for g in ((False, True) if graphs else (False,)):
                    for wd in (widths if r in (0, 1) else (False,)):
                        out.append(Knobs(r, pk, g, False, o, split, wd))
    return out


def pick(timings: Dict[Knobs, float]) -> Knobs:
    """Fastest candidate; ties go to the simpler one (library defaults first)."""
    def simplicity(k: Knobs):
        return (not k.persistent, k.graphs, k.pair_kernel != "auto", k.pair_split != 0, k.order != "index",
                k.wide, k.recursion_workgroups != 0, k.recursion_workgroups)
    return min(timings, key=lambda k: (timings[k], simplicity(k)))


def _time_steps(systems, precision, knobs: Knobs, steps: int, warmup: int, **ctx_kw) -> float:
    from .pimd import Context
    ctx = Context(systems, precision=precision, **knobs.as_kwargs(), **ctx_kw)
    try:
        for r, s in enumerate(systems):
            x, p = initial_state(s)
            ctx.set_state(r, x, p)
        ctx.step(warmup, 0)
        ctx.synchronize()
        t0 = time.perf_counter()
        ctx.step(steps, 0)
        ctx.synchronize()
        return (time.perf_counter() - t0) / steps
    finally:
        ctx.close()


def tune(systems: Sequence[System], precision: str = "mixed", steps: int = 20, warmup: int = 5,
         cands: Optional[Iterable[Knobs]] = None, **ctx_kw) -> TuneResult:
    timings = {}
    for k in (list(cands) if cands is not None else candidates(systems, precision)):
        timings[k] = _time_steps(systems, precision, k, steps, warmup, **ctx_kw)
    return TuneResult(pick(timings), timings)


def tune_replicas(make_systems: Callable[[int], List[System]], counts: Sequence[int], precision: str = "mixed",
                  steps: int = 20, warmup: int = 5, **ctx_kw) -> Dict[int, float]:
    """Aggregate replica-steps/s for each replica count (the library's default choices)."""
    out = {}
    for R in counts:
        systems = make_systems(R)
        out[R] = R / _time_steps(systems, precision, Knobs(persistent=persistent_fits(systems)), steps, warmup,
                                 **ctx_kw)
    return out
