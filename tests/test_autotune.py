"""Candidate generation and selection of the autotuner (host logic; the timing itself needs a GPU)."""
from paper_2404_02628_amd.autotune import Knobs, candidates, pick
from paper_2404_02628_amd.workloads import WORKLOADS, batched_systems


def test_candidates_cover_the_schedules_that_apply():
    big = WORKLOADS["large_gauss"]
    one = candidates([big], "fp64")
    assert Knobs(0, "auto", False) in one and not any(k.graphs for k in one)   # graphs only on request
    assert Knobs(1, "auto", True) in candidates([big], "fp64", graphs=True)
    assert any(k.recursion_workgroups > 1 for k in one)          # cooperative helper counts
    assert all(k.pair_kernel == "auto" for k in one)             # FP64: ordered kernel only
    many = candidates([big.with_(seed=k) for k in range(16)], "mixed")
    assert {k.pair_kernel for k in many} == {"auto", "ordered"}  # 512 slices: both pair kernels
    assert all(k.recursion_workgroups in (0, 1) for k in many)   # batched: no helpers
    tiny = candidates([WORKLOADS["small_ideal"]], "fp64")
    assert all(k.recursion_workgroups in (0, 1) for k in tiny)   # one row block: nothing to help
    assert Knobs(persistent=True) in tiny                        # small enough for the persistent kernel
    assert not any(k.persistent for k in one) and not any(k.persistent for k in many)
    assert len(set(candidates(batched_systems(64, 505), "mixed"))) == len(candidates(batched_systems(64, 505), "mixed"))


def test_candidates_cover_packing_and_pair_granularity():
    uneven = candidates(batched_systems(64, 505), "mixed")
    assert {k.order for k in uneven} == {"index", "longest"}               # uneven N: both packings
    assert {(k.pair_kernel, k.pair_split) for k in uneven} == {("auto", 0), ("ordered", 1), ("ordered", 2),
                                                               ("ordered", 4)}
    even = candidates([WORKLOADS["large_gauss"].with_(seed=k) for k in range(16)], "mixed")
    assert {k.order for k in even} == {"index"}                            # equal N: order is moot
    fp64 = candidates([WORKLOADS["large_gauss"]], "fp64")
    assert {k.pair_split for k in fp64} == {0, 1, 2, 4}                    # ordered FP64 kernel splits
    ideal = candidates([WORKLOADS["huge_ideal_10k"]], "fp64")
    assert {k.pair_split for k in ideal} == {0}                            # no pair term: nothing to split


def test_pick_prefers_library_defaults_for_packing():
    t = {Knobs(order="longest"): 1.0, Knobs(): 1.0, Knobs(pair_split=2): 1.0}
    assert pick(t) == Knobs()
    t = {Knobs(order="longest"): 0.9, Knobs(): 1.0}
    assert pick(t) == Knobs(order="longest")


def test_pick_takes_the_fastest_and_breaks_ties_toward_defaults():
    t = {Knobs(0, "auto", False): 2.0, Knobs(1, "ordered", True): 1.0, Knobs(5, "auto", False): 3.0}
    assert pick(t) == Knobs(1, "ordered", True)
    t = {Knobs(1, "auto", True): 1.0, Knobs(0, "auto", False): 1.0, Knobs(1, "auto", False): 1.0}
    assert pick(t) == Knobs(0, "auto", False)
    t = {Knobs(persistent=True): 1.0, Knobs(0, "auto", False): 1.0}
    assert pick(t) == Knobs(persistent=True)                     # the library default for small replicas


def test_candidates_offer_wide_chains_where_they_fit():
    c5 = candidates(batched_systems(64, 505), "mixed")
    assert {k.wide for k in c5} == {False, True}                 # 128 chains fit a 256-CU device
    assert all(not k.wide for k in c5 if k.recursion_workgroups > 1)
    big = candidates([WORKLOADS["large_gauss"].with_(seed=k) for k in range(256)], "mixed")
    assert not any(k.wide for k in big)                          # 512 chains: four waves only
    assert pick({Knobs(wide=True): 1.0, Knobs(): 1.0}) == Knobs()
