"""ctypes wrapper of the CPU FP64 oracle (test infrastructure only).

Arrays use the layout [dim][P][N] (numpy shape ``(dim, P, N)``, float64, C order).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pimd_oracle.c")
# PIMD_ORACLE_LIB points the wrapper at another build of the same source (used by the
# mutation test, which compiles deliberately broken copies into a temporary directory).
_LIB = os.environ.get("PIMD_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, no OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("dim", C.c_int32),
                ("beta", C.c_double), ("hbar", C.c_double), ("mass", C.c_double),
                ("omega", C.c_double), ("xi", C.c_double), ("pair_amp", C.c_double),
                ("pair_width", C.c_double), ("n2", C.c_int32)]


class _Energies(C.Structure):
    _fields_ = [("v_exch", C.c_double), ("u_trap", C.c_double), ("u_pair", C.c_double),
                ("spring_expect", C.c_double), ("virial", C.c_double),
                ("e_prim", C.c_double), ("e_vir", C.c_double)]


class _MD(C.Structure):
    _fields_ = [("dt", C.c_double), ("nhc_len", C.c_int32), ("nhc_q", C.c_double),
                ("sy_order", C.c_int32), ("bead_mass", C.c_double)]


@dataclass
class OracleParams:
    n: int
    p: int
    dim: int
    beta: float
    xi: float = 1.0
    pair_amp: float = 0.0
    pair_width: float = 1.0
    hbar: float = 1.0
    mass: float = 1.0
    omega: float = 1.0
    n2: int = 0          # particles of a second species (the last n2); 0 = one species

    def c(self) -> _Params:
        return _Params(self.n, self.p, self.dim, self.beta, self.hbar, self.mass,
                       self.omega, self.xi, self.pair_amp, self.pair_width, self.n2)


@dataclass
class OracleMD:
    dt: float = 0.01
    nhc_len: int = 4
    nhc_q: float = 0.0
    sy_order: int = 3
    bead_mass: float = 0.0

    def c(self) -> _MD:
        return _MD(self.dt, self.nhc_len, self.nhc_q, self.sy_order, self.bead_mass)


_lib = None
_dp = C.POINTER(C.c_double)


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER(_Params)
        lib.oracle_ring_energy.restype = C.c_double
        lib.oracle_ring_energy.argtypes = [P, _dp, C.c_int, C.c_int]
        for name, args in [
            ("oracle_internal_energies", [P, _dp, _dp]),
            ("oracle_cycle_energies", [P, _dp, _dp]),
            ("oracle_forward_potentials", [P, _dp, _dp]),
            ("oracle_backward_potentials", [P, _dp, _dp]),
            ("oracle_connection_probabilities", [P, _dp, _dp, _dp, _dp]),
            ("oracle_exchange_forces", [P, _dp, _dp, _dp]),
            ("oracle_interaction", [P, _dp, _dp, _dp, _dp, _dp]),
            ("oracle_compute_forces", [P, _dp, _dp, C.POINTER(_Energies), _dp, _dp, _dp]),
            ("oracle_step", [P, C.POINTER(_MD), _dp, _dp, _dp, _dp, _dp, C.c_int64]),
            ("oracle_density", [P, _dp, C.c_int, C.c_double, C.POINTER(C.c_uint64)]),
        ]:
            fn = getattr(lib, name)
            fn.restype = C.c_int
            fn.argtypes = args
        lib.oracle_conserved.restype = C.c_double
        lib.oracle_conserved.argtypes = [P, C.POINTER(_MD), _dp, _dp, _dp, _dp]
        lib.oracle_exact_energy.restype = C.c_double
        lib.oracle_exact_energy.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double]
        lib.oracle_exact_energy_signed.restype = C.c_double
        lib.oracle_exact_energy_signed.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        lib.oracle_init_state.restype = C.c_int
        lib.oracle_init_state.argtypes = [P, C.POINTER(_MD), C.c_double, C.c_uint64, _dp, _dp]
        _lib = lib
    return _lib


def _arr(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def ring_energy(par: OracleParams, x, u: int, v: int) -> float:
    x = _arr(x, (par.dim, par.p, par.n))
    return load().oracle_ring_energy(C.byref(par.c()), _ptr(x), u, v)


def internal_energies(par: OracleParams, x) -> np.ndarray:
    x = _arr(x, (par.dim, par.p, par.n))
    out = np.zeros(par.n)
    _check(load().oracle_internal_energies(C.byref(par.c()), _ptr(x), _ptr(out)), "internal_energies")
    return out


def cycle_energies(par: OracleParams, x) -> np.ndarray:
    """E[u-1, v-1] = E^{[u,v]} for u <= v (Eqs. 8-10)."""
    x = _arr(x, (par.dim, par.p, par.n))
    E = np.zeros((par.n, par.n))
    _check(load().oracle_cycle_energies(C.byref(par.c()), _ptr(x), _ptr(E)), "cycle_energies")
    return E


def forward_potentials(par: OracleParams, E) -> np.ndarray:
    E = _arr(E, (par.n, par.n))
    X = np.zeros(par.n + 1)
    _check(load().oracle_forward_potentials(C.byref(par.c()), _ptr(E), _ptr(X)), "forward")
    return X


def backward_potentials(par: OracleParams, E) -> np.ndarray:
    E = _arr(E, (par.n, par.n))
    Y = np.zeros(par.n + 2)
    _check(load().oracle_backward_potentials(C.byref(par.c()), _ptr(E), _ptr(Y)), "backward")
    return Y


def connection_probabilities(par: OracleParams, E, X, Y) -> np.ndarray:
    E = _arr(E, (par.n, par.n))
    X = _arr(X, (par.n + 1,))
    Y = _arr(Y, (par.n + 2,))
    G = np.zeros((par.n, par.n))
    _check(load().oracle_connection_probabilities(C.byref(par.c()), _ptr(E), _ptr(X), _ptr(Y), _ptr(G)),
           "probabilities")
    return G


def exchange_forces(par: OracleParams, x, G) -> np.ndarray:
    x = _arr(x, (par.dim, par.p, par.n))
    G = _arr(G, (par.n, par.n))
    f = np.zeros_like(x)
    _check(load().oracle_exchange_forces(C.byref(par.c()), _ptr(x), _ptr(G), _ptr(f)), "exchange_forces")
    return f


def interaction(par: OracleParams, x):
    """Returns (f = -(1/P) grad U, u_trap, u_pair, virial)."""
    x = _arr(x, (par.dim, par.p, par.n))
    f = np.zeros_like(x)
    ut, up, vir = C.c_double(), C.c_double(), C.c_double()
    _check(load().oracle_interaction(C.byref(par.c()), _ptr(x), _ptr(f), C.byref(ut), C.byref(up),
                                     C.byref(vir)), "interaction")
    return f, ut.value, up.value, vir.value


def compute_forces(par: OracleParams, x, want_tables: bool = False):
    """Returns (forces, energies dict[, X, Y, G])."""
    x = _arr(x, (par.dim, par.p, par.n))
    f = np.zeros_like(x)
    e = _Energies()
    if want_tables:
        X = np.zeros(par.n + 1)
        Y = np.zeros(par.n + 2)
        G = np.zeros((par.n, par.n))
        rc = load().oracle_compute_forces(C.byref(par.c()), _ptr(x), _ptr(f), C.byref(e),
                                          _ptr(X), _ptr(Y), _ptr(G))
    else:
        rc = load().oracle_compute_forces(C.byref(par.c()), _ptr(x), _ptr(f), C.byref(e), None, None, None)
    _check(rc, "compute_forces")
    en = {k: getattr(e, k) for k, _ in _Energies._fields_}
    if want_tables:
        return f, en, X, Y, G
    return f, en


def step(par: OracleParams, md: OracleMD, x, p, eta, veta, f, n_steps: int):
    """Advance in place; arrays must be float64 C-contiguous numpy arrays."""
    for a in (x, p, f) + ((eta, veta) if md.nhc_len else ()):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
            raise ValueError("step needs float64 C-contiguous numpy arrays (updated in place)")
    e_ptr = _ptr(eta) if md.nhc_len else None
    v_ptr = _ptr(veta) if md.nhc_len else None
    _check(load().oracle_step(C.byref(par.c()), C.byref(md.c()), _ptr(x), _ptr(p), e_ptr, v_ptr,
                              _ptr(f), int(n_steps)), "step")


def conserved(par: OracleParams, md: OracleMD, x, p, eta=None, veta=None) -> float:
    x = _arr(x)
    p = _arr(p)
    e_ptr = _ptr(_arr(eta)) if md.nhc_len else None
    v_ptr = _ptr(_arr(veta)) if md.nhc_len else None
    if md.nhc_len:
        eta = _arr(eta)
        veta = _arr(veta)
        e_ptr, v_ptr = _ptr(eta), _ptr(veta)
    return load().oracle_conserved(C.byref(par.c()), C.byref(md.c()), _ptr(x), _ptr(p), e_ptr, v_ptr)


def density(par: OracleParams, x, bins: int, rmax: float, counts=None) -> np.ndarray:
    x = _arr(x, (par.dim, par.p, par.n))
    if counts is None:
        counts = np.zeros(bins + 1, dtype=np.uint64)
    _check(load().oracle_density(C.byref(par.c()), _ptr(x), bins, rmax,
                                 counts.ctypes.data_as(C.POINTER(C.c_uint64))), "density")
    return counts


def exact_energy(n: int, dim: int, beta: float, p: int = 0, xi: float = 1.0) -> float:
    """Exact canonical energy of n free trapped particles (hbar = m = omega = 1); p = 0: continuum."""
    return load().oracle_exact_energy(n, dim, beta, p, xi)


def exact_energy_signed(n: int, dim: int, beta: float, p: int = 0, xi: float = 1.0) -> float:
    """The same for any real xi (fermions: xi = -1), linear-domain signed recursion; small n."""
    return load().oracle_exact_energy_signed(n, dim, beta, p, xi)


def philox4x32_10(ctr, key) -> tuple:
    """Philox4x32-10 of a 4-word counter and a 2-word key (four 32-bit words)."""
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    out = (C.c_uint32 * 4)()
    load().oracle_philox4x32_10(c, k, out)
    return tuple(out)


def init_state(par: OracleParams, md: OracleMD, sigma: float, seed: int):
    """(x, p): seeded positions N(0, sigma^2) and momenta N(0, m'/beta), layout (dim, P, N)."""
    x = np.zeros((par.dim, par.p, par.n))
    p = np.zeros_like(x)
    _check(load().oracle_init_state(C.byref(par.c()), C.byref(md.c()), C.c_double(sigma), C.c_uint64(seed),
                                    _ptr(x), _ptr(p)), "init_state")
    return x, p
