"""Host checks of the bench line's byte accounting (CPU): the algorithmic bytes
that the roofline fractions divide by, restated from the operation's
definition (which rows of which operands one launch reads and writes), and the
parsing of the committed profiles' machine-readable lines."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_limb_and_peaks():
    b = _bench()
    assert b.LIMB == 65536 * 8
    assert b.HBM_PEAK_GBS == 8000.0
    assert b.VALU_ISSUE_PEAK == 256 * 2.4e9


def test_inner_product_bytes_from_its_operands():
    # l = 30, K = 4, dnum = 3: 35 rows, 3 digits
    rows, beta, nq_rows, k = 35, 3, 31, 4
    limb = 65536 * 8
    plain = (beta * rows + 2 * beta * rows + 2 * rows) * limb  # digits, key halves, two accumulators
    assert plain == (3 * beta + 2) * rows * limb == 201850880
    # HMult's form: a q-row reads the beta - 1 other digits, the key and a0, a1, b0, b1;
    # a special row reads every digit and the key; every row writes two
    tensor = (nq_rows * ((beta - 1) + 2 * beta + 4) + k * (beta + 2 * beta) + 2 * rows) * limb
    assert tensor == 250609664


def test_step_inner_products_parse_the_committed_profile():
    b = _bench()
    prof = os.path.join(ROOT, "profiles", "inner_product_logn16_l30_hbm_counters.md")
    lines = [l for l in open(prof).read().splitlines() if l.startswith("step_kernel:")]
    assert {l.split()[1] for l in lines} == {"k_inner_product_tensor_rowpass", "k_inner_product_rowpass"}
    alg = {l.split()[1]: int(dict(x.split("=") for x in l.split()[3:])["algorithmic_bytes"]) for l in lines}
    assert alg == {"k_inner_product_tensor_rowpass": 250609664, "k_inner_product_rowpass": 201850880}
    out = b.step_inner_products()
    if out is not None:  # None while the kernel sources differ from the profiled ones
        for e in out:
            assert 0.0 < e["frac"] < 1.0
            assert abs(e["achieved"] - e["algorithmic_bytes_per_launch"] / e["profiled_us"] / 1e3) < 0.1
