"""Steady MD steps replayed from the captured HIP graph against the same steps run by direct
kernel launches: the trajectories must agree bit for bit (same kernels, same inputs, same
order), across several replays with sampled (directly launched) steps in between."""
import numpy as np
import pytest

from paper_2404_02628_amd.pimd import Context
from paper_2404_02628_amd.workloads import WORKLOADS, initial_state

pytestmark = pytest.mark.gpu


def _systems(name):
    if name == "batched_medium":
        base = WORKLOADS["medium_gauss"]
        return [base.with_(seed=base.seed + r, n=base.n - 7 * r) for r in range(4)]
    return [WORKLOADS[name]]


def _run(systems, precision, sched, graphs):
    # the graph belongs to the multi-kernel path (small systems would otherwise run persistent)
    ctx = Context(systems, precision=precision, recursion_workgroups=sched, graphs=graphs, persistent=False)
    try:
        for r, s in enumerate(systems):
            x0, p0 = initial_state(s)
            ctx.set_state(r, x0, p0)
        for _ in range(3):
            ctx.step(12, sample_every=5)
        states = [ctx.get_state(r) for r in range(len(systems))]
        energies = [ctx.energies(r) for r in range(len(systems))]
        info = ctx.graph_info()
    finally:
        ctx.close()
    return states, energies, info


@pytest.mark.parametrize("name,precision,sched", [
    ("small_ideal", "fp64", 1),
    ("medium_gauss", "mixed", 1),
    ("large_gauss", "fp64", 0),      # cooperative chain + helpers
    ("large_gauss", "mixed", 0),
    ("batched_medium", "fp64", 0),
])
def test_graph_replay_matches_direct_launches(name, precision, sched):
    systems = _systems(name)
    print(f"graph replay: {name} {precision} sched={sched}", flush=True)
    sg, eg, (state_g, nrep_g) = _run(systems, precision, sched, True)
    sd, ed, (state_d, nrep_d) = _run(systems, precision, sched, False)
    assert state_g == 1 and nrep_g > 0, "the step graph was not built and replayed"
    assert state_d == 2 and nrep_d == 0
    for (xg, pg, ng), (xd, pd, nd) in zip(sg, sd):
        np.testing.assert_array_equal(xg, xd)
        np.testing.assert_array_equal(pg, pd)
        np.testing.assert_array_equal(ng, nd)
    for a, b in zip(eg, ed):
        assert a == b
