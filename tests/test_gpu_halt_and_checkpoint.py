"""Non-finite detection inside pimd_step, and checkpoint / restart.

* A replica whose state turns non-finite during pimd_step (here: a NaN position set through
  pimd_set_state, then steps without sampling) is found by the integrator on the device; the next
  synchronising call reports PIMD_ERR_NONFINITE naming that replica, after writing its outputs;
  the run stays halted (the state no longer changes, pimd_step refuses) until the state is set
  again.  Both the multi-kernel path and the persistent path of small replicas are covered.
* get_state of every replica, handed to a fresh context of the same configuration, continues the
  trajectory bit for bit (the evaluation is deterministic: fixed summation orders everywhere).
"""
import ctypes as C

import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state

pytestmark = pytest.mark.gpu


def _systems(n):
    return [System(n=n, p=8, dim=2, beta=2.0, xi=xi, pair_amp=1.0, pair_width=0.5, sigma=1.0, seed=70 + k)
            for k, xi in enumerate((1.0, 0.6, 0.3))]


def _raw_state(ctx, r):
    """get_state through the C ABI, returning (status, x, p) even when the call reports an error."""
    from paper_2404_02628_amd.pimd import load
    s = ctx.systems[r]
    x = np.zeros((s.dim, s.p, s.n))
    p = np.zeros_like(x)
    st = load().pimd_get_state(ctx.h, r, x.ctypes.data, p.ctypes.data, None, 0)
    return st, x, p


@pytest.mark.parametrize("n,persistent", [(70, False), (8, True), (8, False)],
                         ids=["multi-kernel", "persistent", "small-multi-kernel"])
def test_nonfinite_during_steps_is_reported_and_halts(n, persistent):
    from paper_2404_02628_amd.pimd import Context, PimdError, PIMD_ERR_NONFINITE, PIMD_ERR_STATE, load
    systems = _systems(n)
    states = [initial_state(s) for s in systems]
    bad = states[1][0].copy()
    bad[1, 3, n // 2] = np.nan
    print(f"non-finite halt: N={n}, persistent={persistent}", flush=True)

    def fresh():
        c = Context(systems, precision="mixed", persistent=persistent, trace_capacity=64)
        for r, (x, p) in enumerate(states):
            c.set_state(r, x, p)
        c.step(5, 0)
        return c

    # where replica 0 would be after the 7 steps a persistent launch still completes
    ref = fresh()
    try:
        ref.set_state(1, states[1][0], states[1][1])
        ref.step(7, 0)
        x0_after7 = ref.get_state(0)[0]
    finally:
        ref.close()
    ctx = fresh()
    try:
        x0_before = ctx.get_state(0)[0]
        ctx.set_state(1, bad, states[1][1])
        ctx.step(7, 0)
        ctx.step(5, 3)      # enqueued before the host has seen the failure
        with pytest.raises(PimdError) as e:
            ctx.synchronize()
        assert e.value.code == PIMD_ERR_NONFINITE
        assert "replica 1:" in str(e.value)
        assert b"replica 1" in load().pimd_last_error()
        st, x1, p1 = _raw_state(ctx, 0)
        assert st == PIMD_ERR_NONFINITE
        # The device halted the run where the failure appeared: the multi-kernel path finds the
        # non-finite force in the first evaluation after set_state, before any replica moved; a
        # persistent launch runs its steps to the end and halts every later launch.
        assert np.array_equal(x1, x0_after7 if persistent else x0_before)
        # halted: further steps are refused and nothing was sampled
        with pytest.raises(PimdError) as e:
            ctx.step(3, 1)
        assert e.value.code == PIMD_ERR_STATE
        assert load().pimd_trace(ctx.h, 0, None, 0, C.byref(C.c_int64())) == PIMD_ERR_NONFINITE
        # restarting replica 1 from a finite state resumes the whole batch
        ctx.set_state(1, states[1][0], states[1][1])
        ctx.step(4, 2)
        ctx.synchronize()
        for r in range(3):
            x, p, _ = ctx.get_state(r)
            assert np.all(np.isfinite(x)) and np.all(np.isfinite(p))
            assert np.isfinite(ctx.energies(r)["e_vir"])
        assert not np.array_equal(ctx.get_state(0)[0], x1)
    finally:
        ctx.close()


@pytest.mark.parametrize("precision,n,persistent,sched", [
    ("mixed", 300, False, 0), ("fp64", 300, False, 0), ("fp64", 300, False, 4), ("fp64", 8, True, 0)],
    ids=["mixed", "fp64", "fp64-cooperative", "fp64-persistent"])
def test_checkpoint_restart_is_bitwise(precision, n, persistent, sched):
    from paper_2404_02628_amd.pimd import Context
    systems = _systems(n)
    print(f"checkpoint: {precision} N={n} persistent={persistent} schedule={sched}", flush=True)
    kw = dict(precision=precision, persistent=persistent, recursion_workgroups=sched, nhc_len=4)
    a = Context(systems, **kw)
    try:
        for r, s in enumerate(systems):
            a.set_state(r, *initial_state(s))
        a.step(25, 0)
        ckpt = [a.get_state(r) for r in range(3)]
        a.step(30, 0)
        end_a = [a.get_state(r) for r in range(3)]
    finally:
        a.close()
    b = Context(systems, **kw)
    try:
        for r, (x, p, nhc) in enumerate(ckpt):
            b.set_state(r, x, p, nhc)
        b.step(30, 0)
        end_b = [b.get_state(r) for r in range(3)]
    finally:
        b.close()
    for r in range(3):
        for k in range(3):
            assert np.array_equal(end_a[r][k], end_b[r][k]), (r, k)
    assert not np.array_equal(end_a[0][0], ckpt[0][0])
