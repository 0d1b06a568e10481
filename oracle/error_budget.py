"""Error budget of the oracle's full-slot bootstrap, phase by phase (test
infrastructure: the oracle's own client and executor on the CPU, no GPU code).

The bootstrap of Sec. III-F.7 is run step by step with the secret key at hand,
and the decrypted value after each phase is compared with what that phase
should produce exactly:
- ModRaise: the raised plaintext t is the input times the gain plus q_0 I; the
  table gives max |I| against the EvalMod range K (the sine is only valid
  inside it);
- CoeffToSlot: slots against t / (2 q_0 K), permuted (t exact, so this is
  CoeffToSlot's own noise);
- EvalMod: each half against sin(2 pi K y) of its own decrypted input (the
  approximation plus the noise of the squarings), and against the sine of the
  exact CoeffToSlot output (that plus the incoming noise, amplified);
- SlotToCoeff: the output slots against the input message (everything).

usage: python -m oracle.error_budget [--logn 16|12] [--uniform] [--gain G]
Defaults: N = 2^16 (31 limbs, ten special primes, dnum 3), sparse-secret
encapsulation with degree 31, K = 12, 3 double angles, gain 128; --uniform:
degree 119, K = 512, 6 double angles, gain 1024.
"""
from __future__ import annotations

import argparse
import time

import numpy as np

from . import Params, galois_conjugate, galois_for_rotation, intt
from . import bootstrap as B
from . import client


def _bits(a, b) -> float:
    d = float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
    return float(np.log2(d)) if d > 0 else float("-inf")


def _br(x: int, bits: int) -> int:
    return int(format(x, "0%db" % bits)[::-1], 2)


def run(logn: int = 16, uniform: bool = False, gain: int | None = None, seed: int = 31, verbose: bool = True):
    from paper_2507_04775_amd import inputs  # the seeded generators only

    say = print if verbose else (lambda *a, **k: None)
    t0 = time.time()
    ps = inputs.params("large-nv" if logn == 16 else "boot-small")
    P = Params(ps.logn, ps.q, ps.p, ps.dnum)
    parts = [(ps.logn - 1) // 3 + (1 if i < (ps.logn - 1) % 3 else 0) for i in range(3)]
    if uniform:
        ev = dict(cheb_degree=119, double_angles=6, k_range=512.0) if logn == 16 else \
            dict(cheb_degree=63, double_angles=5, k_range=128.0)
        g_default = 1024 if logn == 16 else 16
    else:
        ev = dict(cheb_degree=31, double_angles=3, k_range=12.0)
        g_default = 128 if logn == 16 else 16
    G = g_default if gain is None else gain
    scale = 2.0 ** ps.log_scale
    bp = B.BootParams(logn=ps.logn, cts_radix_logs=parts, stc_radix_logs=parts[::-1], top_scale=scale,
                      in_scale=scale, hoist_moddown=True, input_gain=G, **ev)
    pl = B.plan(P, bp)
    g = inputs.rng(seed)
    sk = client.SecretKey(P, inputs.ternary(g, ps.N))
    allm = list(ps.q) + list(ps.p)

    def masks_errors():
        return ([inputs.uniform_residues(g, allm, ps.N) for _ in range(ps.dnum)],
                [inputs.gaussian(g, ps.N, ps.sigma) for _ in range(ps.dnum)])

    rk = {k: client.gen_galois_key(P, sk, galois_for_rotation(ps.logn, k), *masks_errors())
          for k in B.rotations_needed(bp)}
    ck = client.gen_galois_key(P, sk, galois_conjugate(ps.logn), *masks_errors())
    rlk = client.gen_relin_key(P, sk, *masks_errors())
    to_sp = from_sp = None
    if not uniform:
        sp = client.SecretKey(P, inputs.sparse_ternary(g, ps.N, 32))
        to_sp = client.gen_switch_key(P, sp, sk.eval_all, *masks_errors())
        from_sp = client.gen_switch_key(P, sk, sp.eval_all, *masks_errors())
    ex = B.Executor(P, pl, rlk, ck, rk, to_sp, from_sp)
    say("keys and plan: %.1f s" % (time.time() - t0))

    n, N, q0, K = ps.N // 2, ps.N, ps.q[0], bp.k_range
    z = inputs.complex_slots(inputs.rng(seed + 1), n)
    pt = client.encode(P, z, 0, scale)
    ct = client.encrypt(P, sk, pt, 0, inputs.uniform_residues(g, ps.q[:1], N), inputs.gaussian(g, N, ps.sigma))
    ct = (ct[0], ct[1], 0)

    def dec(c):
        return client.decode(P, client.decrypt(P, sk, (c[0], c[1]), c[2]), c[2], ex.sc[c[2]])

    def coeffs(c):
        m = client.decrypt(P, sk, (c[0], c[1]), c[2])
        return np.array(client.crt_centred(intt(P.q[: c[2] + 1], m, P.logn), P.q[: c[2] + 1]), dtype=object)

    rows = []
    m0 = coeffs(ct)  # level-0 plaintext, centred mod q_0
    x = ex.scalar_mul_int(ct, G) if G != 1 else ct
    if to_sp is not None:
        x = ex.switch(x, to_sp)
    x = ex.modraise(x)
    if from_sp is not None:
        x = ex.switch(x, from_sp)
    t = coeffs(x)
    I = max(abs(int(round((int(a) - G * int(b)) / q0))) for a, b in zip(t, m0))
    rows.append(("ModRaise", "max |I| = %d against K = %g" % (I, K)))
    say(rows[-1], "%.1f s" % (time.time() - t0))

    c = ex.coeff_to_slot(x)
    perm = np.array([_br(i, ps.logn - 1) for i in range(n)])
    w_exact = (t[:n].astype(float) + 1j * t[n:].astype(float))[perm] / (2 * q0 * K)
    rows.append(("CoeffToSlot", "2^%.2f (own noise; level %d)" % (_bits(dec(c), w_exact), c[2])))
    say(rows[-1], "%.1f s" % (time.time() - t0))

    cj = ex.conj(c)
    re_in = ex.add(c, cj)
    im_in = ex.monomial(ex.add(c, cj, "sub"), 3 * N // 2)
    halves = []
    for name, y_in, y_exact in (("re", re_in, 2 * w_exact.real), ("im", im_in, 2 * w_exact.imag)):
        y_dec = dec(y_in).real
        y_out = ex.eval_mod(y_in)
        got = dec(y_out).real
        own = _bits(got, np.sin(2 * np.pi * K * y_dec))
        tot = _bits(got, np.sin(2 * np.pi * K * y_exact))
        rows.append(("EvalMod " + name, "2^%.2f own, 2^%.2f against the exact sine (level %d)" % (own, tot, y_out[2])))
        say(rows[-1], "%.1f s" % (time.time() - t0))
        halves.append(y_out)
    out = ex.slot_to_coeff(ex.add(halves[0], ex.monomial(halves[1], N // 2)))
    rows.append(("SlotToCoeff", "2^%.2f against the input slots (level %d)" % (_bits(dec(out), z), out[2])))
    say(rows[-1], "%.1f s" % (time.time() - t0))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--logn", type=int, default=16, choices=[12, 16])
    ap.add_argument("--uniform", action="store_true")
    ap.add_argument("--gain", type=int, default=None)
    a = ap.parse_args()
    for phase, res in run(a.logn, a.uniform, a.gain):
        print("| %s | %s |" % (phase, res))


if __name__ == "__main__":
    main()
