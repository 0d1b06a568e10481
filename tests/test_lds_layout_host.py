"""Host check of the LDS layouts of the 4-element inverse NTT passes
(row4_slot, col4_slot in csrc/ntt.hip): every slot function is a bijection
onto its words, and in each of the four element layouts A..D a half-wave (32
lanes) touches 32 distinct 8-byte banks, so an exchange costs no conflicts.
The formulas are restated from the kernel source, which the test reads to
make sure they are still the ones it checks."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

LAYOUTS = {
    "A": lambda s, i: 4 * s + i,
    "B": lambda s, i: 16 * (s >> 2) + (s & 3) + 4 * i,
    "C": lambda s, i: 64 * (s >> 4) + (s & 15) + 16 * i,
    "D": lambda s, i: s + 64 * i,
}


def row4_slot(e):
    return (e & ~31) | ((e ^ (9 * (e >> 5)) ^ (4 * (e >> 6))) & 31)


def col4_slot(e, col):
    return 8 * (e + (e >> 2)) + col


def _src():
    return open(os.path.join(ROOT, "paper_2507_04775_amd", "csrc", "ntt.hip")).read()


def test_formulas_match_the_kernel_source():
    src = re.sub(r"\s+", " ", _src())
    assert "return (e & ~31u) | ((e ^ (9 * (e >> 5)) ^ (4 * (e >> 6))) & 31u);" in src
    assert "return 8 * (e + (e >> 2)) + col; }" in src
    assert "constexpr int kLds4 = 8 * (255 + 63 + 1);" in src
    for name, body in (("p4a", "4 * s + i"), ("p4b", "16 * (s >> 2) + (s & 3) + 4 * i"),
                       ("p4c", "64 * (s >> 4) + (s & 15) + 16 * i"), ("p4d", "s + 64 * i")):
        assert "%s(uint32_t s, int i) { return %s; }" % (name, body) in src


def test_layouts_cover_each_row_once():
    for name, f in LAYOUTS.items():
        assert sorted(f(s, i) for s in range(64) for i in range(4)) == list(range(256)), name


def test_row_slots_are_a_bijection_and_conflict_free():
    assert sorted(row4_slot(e) for e in range(256)) == list(range(256))
    for name, f in LAYOUTS.items():
        for half in (0, 1):
            for i in range(4):
                banks = [row4_slot(f(s, i)) % 32 for s in range(32 * half, 32 * half + 32)]
                assert len(set(banks)) == 32, (name, half, i)


def test_column_slots_fit_and_are_conflict_free():
    words = 8 * (255 + 63 + 1)
    slots = [col4_slot(e, c) for e in range(256) for c in range(8)]
    assert len(set(slots)) == len(slots) and max(slots) < words
    # a half-wave is 8 columns x 4 consecutive threads s
    for name, f in LAYOUTS.items():
        for s0 in range(0, 64, 4):
            for i in range(4):
                banks = [col4_slot(f(s, i), c) % 32 for s in range(s0, s0 + 4) for c in range(8)]
                assert len(set(banks)) == 32, (name, s0, i)
