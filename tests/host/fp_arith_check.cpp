// Host-side check of the FP64 modular arithmetic used by the gfx950 NTT for
// primes below 2^50 (the same header the kernels include, run on the CPU):
// every product must be exact modulo q, and the value ranges of the NTT
// rounds (four stages between centred reductions) must stay below 2^53.
// Prints "ok" and exits 0 on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../../paper_2507_04775_amd/csrc/modarith.h"

using namespace ckks;
typedef __int128 i128;

static int fails = 0;

static void check_mul(double y, double w, FpMod m, double bound_factor)
{
    double r = fp_mulmod(y, w, m);
    i128 q = (i128)m.q;
    i128 want = ((i128)(long long)y * (i128)(long long)w) % q;
    if (want < 0) want += q;
    i128 got = (i128)(long long)r % q;
    if (got < 0) got += q;
    double lim = (0.5 + 0.375 * std::fabs(y) / std::ldexp(1.0, 50)) * m.q + 1.0;
    if (got != want || std::fabs(r) > lim || r != std::rint(r)) {
        if (fails++ < 10) std::printf("mulmod mismatch y=%.0f w=%.0f r=%.0f\n", y, w, r);
    }
    (void)bound_factor;
}

// 16 values through four forward (CT) stages, as one register round
static double fwd_round(double v[16], const double w[4][8], FpMod m)
{
    double mx = 0;
    for (int st = 0; st < 4; ++st) {
        int h = 8 >> st;
        for (int g = 0; g < (1 << st); ++g)
            for (int k = 0; k < h; ++k) {
                double &x = v[g * 2 * h + k], &y = v[g * 2 * h + k + h];
                double t = fp_mulmod(y, w[st][g], m), a = x;
                x = a + t;
                y = a - t;
                mx = std::fmax(mx, std::fmax(std::fabs(x), std::fabs(y)));
            }
    }
    return mx;
}

static double inv_round(double v[16], const double w[4][8], FpMod m)
{
    double mx = 0;
    for (int st = 0; st < 4; ++st) {
        int h = 1 << st;
        for (int g = 0; g < (8 >> st); ++g)
            for (int k = 0; k < h; ++k) {
                double &x = v[g * 2 * h + k], &y = v[g * 2 * h + k + h];
                double s = x + y, d = x - y;
                mx = std::fmax(mx, std::fabs(s));
                x = st == 2 ? fp_reduce(s, m) : s;
                y = fp_mulmod(d, w[st][g], m);
                mx = std::fmax(mx, std::fmax(std::fabs(x), std::fabs(y)));
            }
    }
    return mx;
}

int main()
{
    const unsigned long long primes[] = {1125899903827969ull, 1125899834490881ull, 562949951979521ull, 1125899906842597ull};
    std::mt19937_64 rng(250704775);
    double worst_fwd = 0, worst_inv = 0;
    for (unsigned long long qq : primes) {
        FpMod m;
        m.q = (double)qq;
        m.qinv = 1.0 / (double)qq;
        for (int i = 0; i < 200000; ++i) {
            double y = (double)(long long)(rng() % (unsigned long long)(7.2 * qq)) - (i & 1 ? std::rint(3.6 * qq) : 0);
            double w = (double)(rng() % qq);
            check_mul(std::rint(y), w, m, 0);
        }
        check_mul(std::rint(7.1 * m.q) - 1, m.q - 1, m, 0);
        check_mul(-(std::rint(7.1 * m.q) - 1), m.q - 1, m, 0);
        // round ranges: canonical start (first round of a pass), then centred starts
        for (int trial = 0; trial < 20000; ++trial) {
            double v[16], w[4][8];
            bool extreme = trial < 100;
            for (int st = 0; st < 4; ++st)
                for (int g = 0; g < 8; ++g) w[st][g] = extreme ? m.q - 1 : (double)(rng() % qq);
            for (int k = 0; k < 16; ++k) v[k] = extreme ? m.q - 1 : (double)(rng() % qq);
            worst_fwd = std::fmax(worst_fwd, fwd_round(v, w, m) / m.q);
            for (int k = 0; k < 16; ++k) v[k] = fp_reduce(v[k], m);
            worst_fwd = std::fmax(worst_fwd, fwd_round(v, w, m) / m.q);
            for (int k = 0; k < 16; ++k) v[k] = extreme ? m.q - 1 : (double)(rng() % qq);
            for (int k = 0; k < 16; ++k) v[k] = fp_reduce(v[k], m);
            worst_inv = std::fmax(worst_inv, inv_round(v, w, m) / m.q);
            for (int k = 0; k < 16; ++k) v[k] = fp_reduce(v[k], m);
            worst_inv = std::fmax(worst_inv, inv_round(v, w, m) / m.q);
            for (int k = 0; k < 16; ++k) {
                uint64_t c = fp_canonical(v[k], m);
                if (c >= qq) { if (fails++ < 10) std::printf("canonical out of range\n"); }
            }
        }
    }
    // the proven limits: forward < 7.1 q, inverse < 8 q; both far below 2^53 / 2^50 = 8 q only with margin
    std::printf("max |x|/q: forward %.3f inverse %.3f\n", worst_fwd, worst_inv);
    if (worst_fwd >= 7.1 || worst_inv >= 7.9) fails++;
    if (fails) { std::printf("FAILED (%d)\n", fails); return 1; }
    std::printf("ok\n");
    return 0;
}
