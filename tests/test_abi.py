"""CPU-side checks of the C ABI: the library loads, exports every function that
include/pimd.h declares, and validates configurations on the host (no GPU call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pimd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:pimd_status|int|const char\*)\s+(pimd_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2404_02628_amd import pimd
    if not os.path.exists(pimd.LIB_PATH):
        from paper_2404_02628_amd.build import build
        build()
    pimd.load()
    return pimd


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    raw = C.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    assert set(names) == set(lib.EXPORTED)
    assert lib.pimd_abi_version() == 8


def _cfg(lib, **over):
    reps = (lib.pimd_replica * 2)()
    reps[0] = lib.pimd_replica(100, 0, 3.0, 1.0, 1.0, 1.0, 1.0, 2.0, 0.5, 0.01, 0.0, 0.0)
    reps[1] = lib.pimd_replica(37, 0, 2.0, 1.0, 1.0, 1.0, 0.4, 0.0, 1.0, 0.01, 0.0, 0.0)
    rep_over = over.pop("rep", {})
    for k, v in rep_over.items():
        setattr(reps[1], k, v)
    kw = dict(n_replicas=2, p=12, dim=2, precision=1, nhc_len=4, sy_order=3, density_bins=50,
              trace_capacity=10, recursion_workgroups=0, flags=0, density_rmax=5.0)
    kw.update(over)
    cfg = lib.pimd_config(kw["n_replicas"], kw["p"], kw["dim"], kw["precision"], kw["nhc_len"], kw["sy_order"],
                          kw["density_bins"], kw["trace_capacity"], kw["recursion_workgroups"], kw["flags"],
                          kw["density_rmax"], reps)
    return cfg, reps


def test_workspace_size_is_positive_and_monotone(lib):
    cfg, _keep = _cfg(lib)
    b1 = lib.pimd_workspace_bytes(cfg)
    cfg2, _keep2 = _cfg(lib, rep={"n": 500})
    b2 = lib.pimd_workspace_bytes(cfg2)
    assert 0 < b1 < b2 and b1 % 256 == 0


@pytest.mark.parametrize("over", [
    {"p": 1}, {"dim": 0}, {"dim": 4}, {"precision": 7}, {"nhc_len": 9}, {"sy_order": 2},
    {"density_bins": 0}, {"density_rmax": 0.0}, {"trace_capacity": -1}, {"n_replicas": 0},
    {"recursion_workgroups": -1}, {"flags": 128}, {"flags": 256}, {"flags": -1},
    {"rep": {"n": 0}}, {"rep": {"xi": -0.1}}, {"rep": {"xi": 1.5}}, {"rep": {"beta": 0.0}},
    {"rep": {"pair_amp": -1.0}}, {"rep": {"pair_amp": 1.0, "pair_width": 0.0}}, {"rep": {"dt": 0.0}},
    {"rep": {"n2": -1}}, {"rep": {"n2": 37}}, {"rep": {"n2": 65}}, {"rep": {"mass": -1.0}},
])
def test_invalid_configs_are_rejected(lib, over):
    cfg, _keep = _cfg(lib, **over)
    with pytest.raises(lib.PimdError) as ei:
        lib.pimd_workspace_bytes(cfg)
    assert ei.value.code == lib.PIMD_ERR_INVALID
    assert len(lib.pimd_last_error()) > 0


def test_create_rejects_missing_workspace_without_touching_the_gpu(lib):
    cfg, _keep = _cfg(lib)
    with pytest.raises(lib.PimdError) as ei:
        lib.pimd_create(cfg, 0, 0, 0)
    assert ei.value.code == lib.PIMD_ERR_WORKSPACE


@pytest.mark.parametrize("flags", [8, 16, 32, 48, 8 | 32 | 2, 64, 64 | 8])
def test_packing_and_split_flags_are_accepted(lib, flags):
    cfg, _keep = _cfg(lib, flags=flags)
    assert lib.pimd_workspace_bytes(cfg) > 0



def test_noalloc_entry_point_rejects_bad_calls_on_the_host(lib):
    """pimd_compute_forces_noalloc checks its arguments and the scratch size before any HIP call."""
    one = (lib.pimd_replica * 1)(lib.pimd_replica(100, 0, 3.0, 1.0, 1.0, 1.0, 1.0, 2.0, 0.5, 0.01, 0.0, 0.0))
    cfg = lib.pimd_config(1, 12, 2, 1, 4, 3, 50, 0, 0, 0, 5.0, one)
    raw = C.CDLL(lib.LIB_PATH)
    raw.pimd_compute_forces_noalloc.restype = C.c_int
    raw.pimd_compute_forces_noalloc.argtypes = [C.POINTER(lib.pimd_config), C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p]
    assert raw.pimd_compute_forces_noalloc(C.byref(cfg), None, 256, None, None) == lib.PIMD_ERR_INVALID
    assert raw.pimd_compute_forces_noalloc(C.byref(cfg), 256, None, None, None) == lib.PIMD_ERR_INVALID
    two = (lib.pimd_replica * 2)(one[0], one[0])
    cfg2 = lib.pimd_config(2, 12, 2, 1, 4, 3, 50, 0, 0, 0, 5.0, two)
    assert raw.pimd_compute_forces_noalloc(C.byref(cfg2), 256, 256, None, None) == lib.PIMD_ERR_INVALID
    big = (lib.pimd_replica * 1)(lib.pimd_replica(60000, 0, 2.0, 1.0, 1.0, 1.0, 1.0, 0.0, 1.0, 0.01, 0.0, 0.0))
    cfg3 = lib.pimd_config(1, 16, 3, 0, 4, 3, 50, 0, 0, 0, 5.0, big)
    assert raw.pimd_compute_forces_noalloc(C.byref(cfg3), 256, 256, None, None) == lib.PIMD_ERR_WORKSPACE
    assert "bytes of scratch" in lib.pimd_last_error()
