"""Thin ctypes binding of libpimd (include/pimd.h).

The functions ``pimd_*`` mirror the C ABI one to one (argument marshalling only).
``Context`` is a convenience owner: it asks the library for the workspace size,
allocates that many bytes as a torch CUDA tensor (device memory), passes torch's
current stream, and forwards every call.  Every step of the computation runs in
the HIP kernels of libpimd; there is no CPU fallback: if the library is missing,
``load()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

from .workloads import System

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpimd.so")

PIMD_OK, PIMD_ERR_INVALID, PIMD_ERR_DEVICE, PIMD_ERR_NONFINITE, PIMD_ERR_WORKSPACE, PIMD_ERR_STATE = 0, -1, -2, -3, -4, -5
PIMD_FP64, PIMD_MIXED = 0, 1
PIMD_HOST, PIMD_DEVICE = 0, 1
PIMD_FLAG_GRAPH = 1
PIMD_FLAG_PAIR_ORDERED = 2
PIMD_FLAG_NO_PERSISTENT = 4
PIMD_FLAG_LONGEST_FIRST = 8
PIMD_FLAG_PAIR_SPLIT_1 = 16
PIMD_FLAG_PAIR_SPLIT_MASK = 48
PIMD_FLAG_RECURSION_WIDE = 64

EXPORTED = [
    "pimd_abi_version", "pimd_last_error", "pimd_workspace_bytes", "pimd_create", "pimd_destroy",
    "pimd_set_state", "pimd_get_state", "pimd_compute_forces", "pimd_get_forces", "pimd_step",
    "pimd_energies", "pimd_trace", "pimd_density", "pimd_reset_accumulators", "pimd_debug_potentials",
    "pimd_debug_probs", "pimd_profile", "pimd_kernel_times", "pimd_kernel_name", "pimd_synchronize",
    "pimd_graph_info", "pimd_cycle_energies", "pimd_init_system", "pimd_debug_fail_waits",
    "pimd_compute_forces_noalloc",
]


class pimd_replica(C.Structure):
    _fields_ = [("n", C.c_int32), ("n2", C.c_int32), ("beta", C.c_double), ("hbar", C.c_double),
                ("mass", C.c_double), ("omega", C.c_double), ("xi", C.c_double), ("pair_amp", C.c_double),
                ("pair_width", C.c_double), ("dt", C.c_double), ("nhc_q", C.c_double), ("bead_mass", C.c_double)]


class pimd_config(C.Structure):
    _fields_ = [("n_replicas", C.c_int32), ("p", C.c_int32), ("dim", C.c_int32), ("precision", C.c_int32),
                ("nhc_len", C.c_int32), ("sy_order", C.c_int32), ("density_bins", C.c_int32),
                ("trace_capacity", C.c_int32), ("recursion_workgroups", C.c_int32), ("flags", C.c_int32),
                ("density_rmax", C.c_double),
                ("replicas", C.POINTER(pimd_replica))]


class pimd_estimates(C.Structure):
    _fields_ = [("v_exch", C.c_double), ("u_trap", C.c_double), ("u_pair", C.c_double),
                ("spring_expect", C.c_double), ("virial", C.c_double), ("e_prim", C.c_double),
                ("e_vir", C.c_double), ("kinetic", C.c_double), ("nhc_energy", C.c_double),
                ("h_conserved", C.c_double), ("step", C.c_int64)]


_lib = None
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p


def load(path: str = LIB_PATH):
    """Loads libpimd.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpimd.so not found at {path}; build it with "
                           f"`python -m paper_2404_02628_amd.build` (hipcc, gfx950)")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 and owns the device
    # memory and stream handles this library is given, so it must be loaded first; libpimd's
    # dependency on libamdhip64.so.7 then resolves to that same runtime.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    sig = {
        "pimd_abi_version": (C.c_int, []),
        "pimd_last_error": (C.c_char_p, []),
        "pimd_workspace_bytes": (C.c_int, [C.POINTER(pimd_config), C.POINTER(C.c_size_t)]),
        "pimd_create": (C.c_int, [C.POINTER(pimd_config), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
        "pimd_destroy": (C.c_int, [_vp]),
        "pimd_set_state": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, C.c_int]),
        "pimd_get_state": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, C.c_int]),
        "pimd_compute_forces": (C.c_int, [_vp]),
        "pimd_get_forces": (C.c_int, [_vp, C.c_int32, _vp, C.c_int]),
        "pimd_step": (C.c_int, [_vp, C.c_int64, C.c_int32]),
        "pimd_energies": (C.c_int, [_vp, C.c_int32, C.POINTER(pimd_estimates)]),
        "pimd_trace": (C.c_int, [_vp, C.c_int32, C.POINTER(pimd_estimates), C.c_int64, C.POINTER(C.c_int64)]),
        "pimd_density": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_uint64), C.POINTER(C.c_int64)]),
        "pimd_reset_accumulators": (C.c_int, [_vp]),
        "pimd_debug_potentials": (C.c_int, [_vp, C.c_int32, _dp, _dp]),
        "pimd_debug_probs": (C.c_int, [_vp, C.c_int32, _dp]),
        "pimd_profile": (C.c_int, [_vp, C.c_int]),
        "pimd_kernel_times": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]),
        "pimd_kernel_name": (C.c_char_p, [C.c_int32]),
        "pimd_synchronize": (C.c_int, [_vp]),
        "pimd_graph_info": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
        "pimd_cycle_energies": (C.c_int, [_vp, C.c_int32, _dp, _dp]),
        "pimd_init_system": (C.c_int, [_vp, _dp, C.POINTER(C.c_uint64)]),
        "pimd_debug_fail_waits": (C.c_int, [_vp]),
        "pimd_compute_forces_noalloc": (C.c_int, [C.POINTER(pimd_config), _vp, _vp, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PimdError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().pimd_last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _chk(code: int, where: str):
    if code != PIMD_OK:
        raise PimdError(code, where)


# ------------------------------------------------------------------ same-name wrappers

def pimd_abi_version() -> int:
    return load().pimd_abi_version()


def pimd_last_error() -> str:
    return load().pimd_last_error().decode(errors="replace")


def pimd_workspace_bytes(cfg: pimd_config) -> int:
    n = C.c_size_t()
    _chk(load().pimd_workspace_bytes(C.byref(cfg), C.byref(n)), "pimd_workspace_bytes")
    return n.value


def pimd_create(cfg: pimd_config, d_workspace: int, nbytes: int, stream: int):
    h = _vp()
    _chk(load().pimd_create(C.byref(cfg), _vp(d_workspace), nbytes, _vp(stream), C.byref(h)), "pimd_create")
    return h


def pimd_destroy(h):
    _chk(load().pimd_destroy(h), "pimd_destroy")


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def pimd_set_state(h, r: int, x, p=None, nhc=None, where: int = PIMD_HOST):
    ptr = lambda a: None if a is None else (a.ctypes.data if isinstance(a, np.ndarray) else int(a))
    _chk(load().pimd_set_state(h, r, ptr(x), ptr(p), ptr(nhc), where), "pimd_set_state")


def pimd_get_state(h, r: int, x=None, p=None, nhc=None, where: int = PIMD_HOST):
    ptr = lambda a: None if a is None else (a.ctypes.data if isinstance(a, np.ndarray) else int(a))
    _chk(load().pimd_get_state(h, r, ptr(x), ptr(p), ptr(nhc), where), "pimd_get_state")


def pimd_compute_forces(h):
    _chk(load().pimd_compute_forces(h), "pimd_compute_forces")


def pimd_compute_forces_noalloc(cfg: pimd_config, d_x: int, d_f: int, d_est: Optional[int], stream: int):
    """Device pointers in, nothing allocated: one replica's forces (and estimators, d_est may be None)."""
    _chk(load().pimd_compute_forces_noalloc(C.byref(cfg), d_x, d_f, d_est, stream), "pimd_compute_forces_noalloc")


def pimd_get_forces(h, r: int, f, where: int = PIMD_HOST):
    _chk(load().pimd_get_forces(h, r, f.ctypes.data if isinstance(f, np.ndarray) else int(f), where),
         "pimd_get_forces")


def pimd_step(h, n_steps: int, sample_every: int):
    _chk(load().pimd_step(h, int(n_steps), int(sample_every)), "pimd_step")


def pimd_energies(h, r: int) -> pimd_estimates:
    e = pimd_estimates()
    _chk(load().pimd_energies(h, r, C.byref(e)), "pimd_energies")
    return e


def pimd_trace(h, r: int, max_samples: int) -> List[pimd_estimates]:
    buf = (pimd_estimates * max(max_samples, 1))()
    n = C.c_int64()
    _chk(load().pimd_trace(h, r, buf, max_samples, C.byref(n)), "pimd_trace")
    return [buf[k] for k in range(n.value)]


def pimd_density(h, r: int, bins: int):
    counts = np.zeros(bins + 1, dtype=np.uint64)
    ns = C.c_int64()
    _chk(load().pimd_density(h, r, counts.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(ns)), "pimd_density")
    return counts, ns.value


def pimd_reset_accumulators(h):
    _chk(load().pimd_reset_accumulators(h), "pimd_reset_accumulators")


def pimd_debug_potentials(h, r: int, n: int):
    X = np.zeros(n + 1)
    Y = np.zeros(n + 2)
    _chk(load().pimd_debug_potentials(h, r, X.ctypes.data_as(_dp), Y.ctypes.data_as(_dp)), "pimd_debug_potentials")
    return X, Y


def pimd_debug_probs(h, r: int, n: int) -> np.ndarray:
    G = np.zeros((n, n))
    _chk(load().pimd_debug_probs(h, r, G.ctypes.data_as(_dp)), "pimd_debug_probs")
    return G


def pimd_init_system(h, pos_sigma, seeds):
    sig = np.ascontiguousarray(pos_sigma, dtype=np.float64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    _chk(load().pimd_init_system(h, sig.ctypes.data_as(_dp), sd.ctypes.data_as(C.POINTER(C.c_uint64))),
         "pimd_init_system")


def pimd_cycle_energies(h, r: int, n: int):
    """(E, ms): the N x N table E^{[u,v]} evaluated entry by entry, and its kernel time."""
    E = np.zeros((n, n))
    ms = C.c_double()
    _chk(load().pimd_cycle_energies(h, r, E.ctypes.data_as(_dp), C.byref(ms)), "pimd_cycle_energies")
    return E, ms.value


def pimd_profile(h, enable: bool):
    _chk(load().pimd_profile(h, 1 if enable else 0), "pimd_profile")


def pimd_kernel_times(h) -> Dict[str, tuple]:
    ms = (C.c_double * 32)()
    nl = (C.c_int64 * 32)()
    nk = C.c_int32()
    _chk(load().pimd_kernel_times(h, ms, nl, 32, C.byref(nk)), "pimd_kernel_times")
    return {load().pimd_kernel_name(k).decode(): (ms[k], nl[k]) for k in range(min(nk.value, 32))}


def pimd_synchronize(h):
    _chk(load().pimd_synchronize(h), "pimd_synchronize")


def pimd_debug_fail_waits(h):
    _chk(load().pimd_debug_fail_waits(h), "pimd_debug_fail_waits")


def pimd_graph_info(h):
    """(state, replays): state 0 not built, 1 replayed, 2 not requested, 3 capture failed."""
    st, n = C.c_int32(), C.c_int64()
    _chk(load().pimd_graph_info(h, C.byref(st), C.byref(n)), "pimd_graph_info")
    return st.value, n.value


# ------------------------------------------------------------------ convenience owner

def estimates_dict(e: pimd_estimates) -> Dict[str, float]:
    return {k: getattr(e, k) for k, _ in pimd_estimates._fields_}


class Context:
    """Owns one libpimd context, its torch-allocated device workspace and its stream."""

    def __init__(self, systems: Sequence[System], precision: str = "mixed", nhc_len: Optional[int] = None,
                 sy_order: int = 3, density_bins: int = 64, density_rmax: float = 6.0, trace_capacity: int = 0,
                 recursion_workgroups: int = 0, graphs: bool = False, pair_kernel: str = "auto",
                 persistent: bool = True, order: str = "index", pair_split: int = 0, wide_recursion: bool = False,
                 device: str = "cuda:0"):
        import torch  # device memory and streams only

        if not systems:
            raise ValueError("need at least one system")
        if pair_kernel not in ("auto", "ordered"):
            raise ValueError("pair_kernel must be 'auto' or 'ordered'")
        if order not in ("index", "longest"):
            raise ValueError("order must be 'index' or 'longest'")
        split_code = {0: 0, 1: 1, 2: 2, 4: 3}.get(pair_split)
        if split_code is None:
            raise ValueError("pair_split must be 0 (automatic), 1, 2 or 4")
        p, dim = systems[0].p, systems[0].dim
        if any(s.p != p or s.dim != dim for s in systems):
            raise ValueError("all replicas of one context share P and dim")
        self.systems = list(systems)
        self.p, self.dim = p, dim
        self.bins = density_bins
        reps = (pimd_replica * len(systems))()
        for k, s in enumerate(systems):
            reps[k] = pimd_replica(s.n, s.n2, s.beta, s.hbar, s.mass, s.omega, s.xi, s.pair_amp,
                                   s.pair_width if s.pair_amp > 0 else 1.0, s.dt, 0.0, s.bead_mass)
        self._reps = reps
        m = systems[0].nhc_len if nhc_len is None else nhc_len
        self.nhc_len = m
        self.cfg = pimd_config(len(systems), p, dim, PIMD_MIXED if precision == "mixed" else PIMD_FP64, m,
                               sy_order, density_bins, trace_capacity, recursion_workgroups,
                               (PIMD_FLAG_GRAPH if graphs else 0) |
                               (PIMD_FLAG_PAIR_ORDERED if pair_kernel == "ordered" else 0) |
                               (0 if persistent else PIMD_FLAG_NO_PERSISTENT) |
                               (PIMD_FLAG_LONGEST_FIRST if order == "longest" else 0) |
                               split_code * PIMD_FLAG_PAIR_SPLIT_1 |
                               (PIMD_FLAG_RECURSION_WIDE if wide_recursion else 0), density_rmax, reps)
        self.nbytes = pimd_workspace_bytes(self.cfg)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            self.h = pimd_create(self.cfg, aligned, self.nbytes, self.stream.cuda_stream)

    # -- state
    def set_state(self, r: int, x, p=None, nhc=None):
        s = self.systems[r]
        shape = (s.dim, s.p, s.n)
        x = _f64(x, shape)
        p = None if p is None else _f64(p, shape)
        nhc = None if nhc is None else _f64(nhc, (self.nhc_len * s.dim * s.p * s.n + 1,))
        pimd_set_state(self.h, r, x, p, nhc)

    def get_state(self, r: int):
        s = self.systems[r]
        shape = (s.dim, s.p, s.n)
        x, p = np.zeros(shape), np.zeros(shape)
        # thermostat: chain velocities [nhc_len][dim][P][N], then the sum of the chain positions
        nhc = np.zeros(self.nhc_len * s.dim * s.p * s.n + 1)
        pimd_get_state(self.h, r, x, p, nhc if self.nhc_len else None)
        return x, p, nhc

    def compute_forces(self):
        pimd_compute_forces(self.h)

    def forces(self, r: int) -> np.ndarray:
        s = self.systems[r]
        f = np.zeros((s.dim, s.p, s.n))
        pimd_get_forces(self.h, r, f)
        return f

    def step(self, n_steps: int, sample_every: int = 0):
        pimd_step(self.h, n_steps, sample_every)

    def energies(self, r: int) -> Dict[str, float]:
        return estimates_dict(pimd_energies(self.h, r))

    def trace(self, r: int, max_samples: int) -> List[Dict[str, float]]:
        return [estimates_dict(e) for e in pimd_trace(self.h, r, max_samples)]

    def density(self, r: int):
        return pimd_density(self.h, r, self.bins)

    def reset_accumulators(self):
        pimd_reset_accumulators(self.h)

    def potentials(self, r: int):
        return pimd_debug_potentials(self.h, r, self.systems[r].n)

    def probabilities(self, r: int) -> np.ndarray:
        return pimd_debug_probs(self.h, r, self.systems[r].n)

    def init_system(self, pos_sigma, seeds):
        """Seeded N(0, sigma_r^2) positions and Maxwell-Boltzmann momenta on the device."""
        if len(pos_sigma) != len(self.systems) or len(seeds) != len(self.systems):
            raise ValueError("one pos_sigma and one seed per replica")
        pimd_init_system(self.h, pos_sigma, seeds)

    def cycle_energies(self, r: int):
        return pimd_cycle_energies(self.h, r, self.systems[r].n)

    def profile(self, on: bool):
        pimd_profile(self.h, on)

    def kernel_times(self):
        return pimd_kernel_times(self.h)

    def synchronize(self):
        pimd_synchronize(self.h)

    def graph_info(self):
        return pimd_graph_info(self.h)

    def debug_fail_waits(self):
        pimd_debug_fail_waits(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            pimd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
