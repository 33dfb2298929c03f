"""The FP64 kernels' table-driven exponential (csrc/fast_exp.h), compiled for the host with
hipcc and compared with the C library exp: at most 2 ulp over [-745, 705]."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fast_exp_accuracy():
    src = os.path.join(ROOT, "tests", "native", "fast_exp_check.hip")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "chk")
        subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        out = subprocess.check_output([exe], text=True).split("\n")
    worst = float(out[0].split()[1])
    nsamp = int(out[0].split()[-1])
    assert nsamp > 3_000_000
    assert worst <= 2.0, out[0]
    one, zero_inf, zero_under, ratio_sub, isnan = out[1].split()[1:]
    assert float(one) == 1.0 and float(zero_inf) == 0.0 and float(zero_under) == 0.0
    assert abs(float(ratio_sub) - 1.0) < 1e-6 and isnan == "1"
    assert out[2].split()[1:] == ["1", "1", "1"], out[2]
