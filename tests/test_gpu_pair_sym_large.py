"""The symmetric pair kernel at slice sizes that need more than 64 KiB of LDS per workgroup.

gfx950 gives a workgroup up to 160 KiB of LDS, so the once-per-pair kernel serves mixed-precision
slices of up to 9,024 particles in 2-D and 5,184 in 3-D (it holds a slice's FP32 positions and
FP32 force accumulators in LDS, 16 and 28 bytes per particle, beside eight waves' transpose
buffers).  Eight replicas of P = 32 make 256 interacting slices, so mixed precision selects it here.
The first and the last replica are compared with the CPU oracle at the mixed-precision bars
(forces 1e-5 of the largest force, U_pair 1e-5), and every replica with the ordered kernel."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,dim", [(4800, 2), (3800, 3)])
def test_symmetric_kernel_beyond_64k_lds(orc, n, dim):
    from paper_2404_02628_amd.pimd import Context
    systems = [System(n=n, p=32, dim=dim, beta=3.0, xi=1.0, pair_amp=0.5, pair_width=0.5, sigma=2.0, seed=900 + r)
               for r in range(8)]
    xs = [initial_state(s)[0] for s in systems]
    out = {}
    for kernel in ("auto", "ordered"):
        print(f"N={n} d={dim}: {kernel} pair kernel", flush=True)
        ctx = Context(systems, precision="mixed", pair_kernel=kernel)
        try:
            for r, x in enumerate(xs):
                ctx.set_state(r, x)
            ctx.compute_forces()
            out[kernel] = [(ctx.forces(r), ctx.energies(r)) for r in range(len(systems))]
        finally:
            ctx.close()
    for r in range(len(systems)):
        fa, ea = out["auto"][r]
        fo, eo = out["ordered"][r]
        assert float(np.max(np.abs(fa - fo))) <= 2e-5 * float(np.max(np.abs(fo))), r
        assert abs(ea["u_pair"] - eo["u_pair"]) <= 2e-5 * abs(eo["u_pair"]), r
    for r in (0, len(systems) - 1):
        s = systems[r]
        print(f"oracle, replica {r}", flush=True)
        par = orc.OracleParams(n=s.n, p=s.p, dim=s.dim, beta=s.beta, xi=s.xi, pair_amp=s.pair_amp,
                               pair_width=s.pair_width)
        f_or, en_or = orc.compute_forces(par, xs[r])
        f, en = out["auto"][r]
        assert float(np.max(np.abs(f - f_or))) <= 1e-5 * float(np.max(np.abs(f_or))), r
        assert abs(en["u_pair"] - en_or["u_pair"]) <= 1e-5 * abs(en_or["u_pair"]), r
        assert abs(en["v_exch"] - en_or["v_exch"]) <= 1e-10 * abs(en_or["v_exch"]), r


# The largest slices the symmetric kernel takes in mixed precision fill 162.9 KB of a compute
# unit's 160 KiB of LDS (2-D: N = 9024, 3-D: N = 5184); one particle more and the context falls
# back to the ordered kernel.  The symmetric kernel sums in another order than the ordered one, so
# its forces differ from the ordered kernel's in the last FP32 bits, while the fallback reproduces
# them exactly: that tells which kernel ran.  Eight replicas of P = 32 (256 slices), one force
# evaluation, compared with the ordered kernel (itself held to the oracle by the parity tests).
@pytest.mark.parametrize("n,dim,symmetric", [(9024, 2, True), (9025, 2, False), (5184, 3, True), (5185, 3, False)])
def test_symmetric_kernel_at_its_lds_limit(n, dim, symmetric):
    from paper_2404_02628_amd.pimd import Context
    systems = [System(n=n, p=32, dim=dim, beta=3.0, xi=1.0, pair_amp=0.5, pair_width=0.5, sigma=3.0, seed=950 + r)
               for r in range(8)]
    xs = [initial_state(s)[0] for s in systems]
    out = {}
    for kernel in ("auto", "ordered"):
        print(f"N={n} d={dim}: {kernel} pair kernel", flush=True)
        ctx = Context(systems, precision="mixed", pair_kernel=kernel)
        try:
            for r, x in enumerate(xs):
                ctx.set_state(r, x)
            ctx.compute_forces()
            out[kernel] = [(ctx.forces(r), ctx.energies(r)["u_pair"]) for r in (0, len(systems) - 1)]
        finally:
            ctx.close()
    for (fa, ua), (fo, uo) in zip(out["auto"], out["ordered"]):
        assert np.all(np.isfinite(fa)) and np.isfinite(ua)
        if symmetric:
            assert float(np.max(np.abs(fa - fo))) > 0.0, "the symmetric kernel was not chosen"
            assert float(np.max(np.abs(fa - fo))) <= 2e-5 * float(np.max(np.abs(fo)))
            assert abs(ua - uo) <= 2e-5 * abs(uo)
        else:
            assert np.array_equal(fa, fo) and ua == uo, "the ordered kernel was not chosen"
