"""The no-allocation entry point pimd_compute_forces_noalloc against pimd_compute_forces.

It is called through the C ABI with torch device arrays, several times in a row on one GPU, each
later call on a smaller replica than the one before (the scratch still holds the larger
layout's contents).  The cases cover both precisions and both recursion schedules: one workgroup,
and the cooperative chain with helpers, whose progress flags the call must clear.  The pair
kernels are the symmetric per-slice one (mixed, >= 256 slices) and the ordered ones.  Each call's
forces and estimators must match a context-based evaluation of the same positions within the
parity bars: 1e-10 (FP64) or 1e-5 (mixed) of the largest force, 1e-10 relative for the FP64 parts
of the estimators.  A replica too large for the scratch is rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, random_positions

pytestmark = pytest.mark.gpu

# (label, N, P, dim, xi, A, s, sigma, seed, precision, recursion_workgroups), largest first
SEQUENCE = [
    ("fp64 coop d=2", 700, 8, 2, 0.7, 1.0, 0.5, 1.5, 31, "fp64", 0),
    ("mixed symmetric pair", 220, 256, 2, 1.0, 0.5, 0.5, 2.0, 32, "mixed", 1),
    ("fp64 one workgroup d=3", 150, 4, 3, 0.4, 1.0, 0.6, 1.0, 33, "fp64", 1),
    ("mixed ordered pair coop", 100, 6, 2, 0.9, 2.0, 0.5, 1.0, 34, "mixed", 0),
    ("fp64 ideal d=1", 40, 3, 1, 1.0, 0.0, 0.5, 0.8, 35, "fp64", 0),
]


def _cfg(pm, s, precision, sched):
    reps = (pm.pimd_replica * 1)()
    reps[0] = pm.pimd_replica(s.n, s.n2, s.beta, s.hbar, s.mass, s.omega, s.xi, s.pair_amp,
                              s.pair_width if s.pair_amp > 0 else 1.0, s.dt, 0.0, s.bead_mass)
    cfg = pm.pimd_config(1, s.p, s.dim, pm.PIMD_MIXED if precision == "mixed" else pm.PIMD_FP64, 4, 3, 64, 0,
                         sched, 0, 6.0, reps)
    cfg._keep = reps
    return cfg


def _noalloc(pm, s, x, precision, sched):
    import torch
    cfg = _cfg(pm, s, precision, sched)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    fd = torch.full_like(xd, float("nan"))
    nest = C.sizeof(pm.pimd_estimates) // 8
    est = torch.full((nest,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    pm.pimd_compute_forces_noalloc(cfg, xd.data_ptr(), fd.data_ptr(), est.data_ptr(), stream)
    torch.cuda.synchronize()
    e = pm.pimd_estimates.from_buffer_copy(est.cpu().numpy().tobytes())
    return fd.cpu().numpy(), pm.estimates_dict(e)


def _context(s, x, precision, sched):
    from paper_2404_02628_amd.pimd import Context
    ctx = Context([s], precision=precision, recursion_workgroups=sched)
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        return ctx.forces(0), ctx.energies(0)
    finally:
        ctx.close()


def test_noalloc_matches_context_evaluation_in_sequence():
    import paper_2404_02628_amd.pimd as pm
    pm.load()
    for label, n, p, dim, xi, A, sw, sigma, seed, prec, sched in SEQUENCE:
        print(f"no-allocation call: {label} (N={n}, P={p}, d={dim}, {prec}, schedule {sched})", flush=True)
        s = System(n=n, p=p, dim=dim, beta=2.0, xi=xi, pair_amp=A, pair_width=sw, sigma=sigma, seed=seed)
        x = random_positions(n, p, dim, sigma, seed)
        f_na, e_na = _noalloc(pm, s, x, prec, sched)
        f_cx, e_cx = _context(s, x, prec, sched)
        scale = float(np.max(np.abs(f_cx)))
        err = float(np.max(np.abs(f_na - f_cx))) / scale
        print(f"  force difference {err:.3e} of the largest force", flush=True)
        assert np.all(np.isfinite(f_na))
        assert err <= (1e-5 if prec == "mixed" else 1e-10), (label, err)
        for k in ("v_exch", "u_trap", "spring_expect", "e_prim"):
            tol = 1e-10 if (prec == "fp64" or k in ("v_exch", "u_trap", "spring_expect")) else 1e-5
            ref = e_cx[k]
            d = abs(e_na[k] - ref)
            if k == "e_prim":   # carries U/P, FP32 pair terms in mixed precision
                d_ok = d <= tol * (abs(ref) + abs(e_cx["u_pair"]) / p + abs(e_cx["u_trap"]) / p)
            else:
                d_ok = d <= tol * max(abs(ref), 1e-300)
            assert d_ok, (label, k, e_na[k], ref)
        tol_u = 1e-5 if prec == "mixed" else 1e-10
        assert abs(e_na["u_pair"] - e_cx["u_pair"]) <= tol_u * (abs(e_cx["u_pair"]) + abs(e_cx["u_trap"])), label
        assert abs(e_na["e_vir"] - e_cx["e_vir"]) <= tol_u * abs(e_cx["e_vir"]), label
        assert e_na["kinetic"] == 0.0 and e_na["step"] == 0


def test_noalloc_rejects_what_does_not_fit():
    import paper_2404_02628_amd.pimd as pm
    pm.load()
    s = System(n=60000, p=16, dim=3, beta=2.0, xi=1.0, pair_amp=0.0, pair_width=1.0, sigma=1.0, seed=1)
    cfg = _cfg(pm, s, "fp64", 0)
    with pytest.raises(pm.PimdError) as ei:
        pm.pimd_compute_forces_noalloc(cfg, 256, 256, None, 0)
    assert ei.value.code == pm.PIMD_ERR_WORKSPACE
    two = (pm.pimd_replica * 2)(cfg.replicas[0], cfg.replicas[0])
    cfg2 = pm.pimd_config(2, 16, 3, pm.PIMD_FP64, 4, 3, 64, 0, 0, 0, 6.0, two)
    with pytest.raises(pm.PimdError) as ei:
        pm.pimd_compute_forces_noalloc(cfg2, 256, 256, None, 0)
    assert ei.value.code == pm.PIMD_ERR_INVALID
