"""Host-side check of the assignment of NTT grid workgroups to (limb, tile)
units: the kernels' own header (unit_map.h) is compiled for the CPU and the
assignment is checked to be a bijection, in range, with the integer-path limbs
spread two tiles per XCD."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_ntt_unit_assignment_is_a_bijection():
    src = os.path.join(HERE, "host", "unit_map_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "unitmap")
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
