"""Host-side check of the 64-bit integer modular arithmetic the gfx950 kernels
use for primes of 2^50 and above (exact products, 128-bit reduction, Shoup and
variable products) and of the carry accounting of the base conversion's
column sums: the kernels' own header (modarith.h) is compiled for the CPU and
compared with exact 128-bit integer arithmetic on edge and seeded operands."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_int_modmul_exact_on_edges_and_column_sums():
    src = os.path.join(HERE, "host", "int_arith_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "intcheck")
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
