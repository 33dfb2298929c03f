"""The FP64 kernels' table-driven exponential and branch-free logarithm (csrc/fast_exp.h),
compiled for the host with hipcc and compared with the C library: exp at most 2 ulp over
[-745, 705], log at most 2 ulp of the result over [2^-1000, 2^1000] (with the recursions' range
[1, 2^64] and the integers up to 2^20 sampled densely)."""
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


def test_fast_log_accuracy():
    src = os.path.join(ROOT, "tests", "native", "fast_log_check.hip")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "chk")
        subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-o", exe, src],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        out = subprocess.check_output([exe], text=True).split("\n")
    worst = float(out[0].split()[1])
    assert int(out[0].split()[-1]) == 4_000_000
    assert worst <= 2.0, out[0]
    one, zero, inf, neg_nan, nan_nan, sub_ratio = out[1].split()[1:]
    assert float(one) == 0.0 and zero == "-inf" and inf == "inf" and neg_nan == "1" and nan_nan == "1"
    assert abs(float(sub_ratio) - 1.0) < 1e-12          # subnormal argument
