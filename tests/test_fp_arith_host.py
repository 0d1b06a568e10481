"""Host-side check of the FP64 modular arithmetic the gfx950 NTT uses for
primes below 2^50: the kernels' own header (modarith.h) is compiled for the
CPU and every product is compared with exact 128-bit integer arithmetic, and
the value ranges of the NTT register rounds are checked against 2^53."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fp64_modmul_exact_and_round_ranges_bounded():
    src = os.path.join(HERE, "host", "fp_arith_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fpcheck")
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-ffp-contract=off", src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
