// Host-side check of the 64-bit integer modular arithmetic of the gfx950
// kernels (the same header the kernels include, run on the CPU): the exact
// 64x64->128 product, the 128-bit reduction, Shoup products and the modular
// product, for the 40-, 50- and 60-bit primes of the parameter sets, on edge
// operands (0, 1, q-2, q-1, the 32-bit word boundaries, 2^64-1) and on seeded
// random ones, against unsigned __int128 arithmetic.  The column sums of
// mac_cols (inline assembly, GPU only) are checked through an emulation of
// their instruction sequence: each v_mad_u64_u32 is a 32x32+64 product with a
// carry-out bit, each v_addc_co_u32 a 32-bit add with carry-in; mac_total of
// the emulated columns must equal the exact 128-bit sum, with operands at
// 2^61 - 1 and up to 2^16 - 1 terms.  The split columns (MacSplit) are checked
// at their limits (constants below 2^50, inputs below 2^62, 16 terms), and
// ModDown's centred conversion from inputs shifted by p_k against the exact
// signed sum.  Prints "ok" and exits 0 on success.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2507_04775_amd/csrc/modarith.h"

using namespace ckks;
typedef unsigned __int128 u128x;

static int fails = 0;

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond) && fails++ < 20) {                    \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                     \
            std::printf("\n");                            \
        }                                                 \
    } while (0)

static u128x to128(u128 z) { return ((u128x)z.hi << 64) | z.lo; }

static u128 from128(u128x z)
{
    u128 r;
    r.lo = (uint64_t)z;
    r.hi = (uint64_t)(z >> 64);
    return r;
}

// floor(w 2^64 / q), the Shoup companion, by exact 128-bit division
static uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((u128x)w << 64) / q); }

static Prime prime_of(uint64_t q)
{
    Prime P;
    P.q = q;
    P.two_q = 2 * q;
    P.r64 = (uint64_t)(((u128x)1 << 64) % q);
    P.r64_s = shoup_of(P.r64, q);
    P.one_s = shoup_of(1, q);
    P.ninv = P.ninv_s = 0;
    P.qinv = 1.0 / (double)q;
    return P;
}

static bool is_prime(uint64_t n)
{
    if (n < 2) return false;
    for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int r = 0;
    while (!(d & 1)) d >>= 1, ++r;
    auto mulm = [&](uint64_t a, uint64_t b) { return (uint64_t)((u128x)a * b % n); };
    for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        uint64_t x = 1, b = a, e = d;
        for (; e; e >>= 1, b = mulm(b, b))
            if (e & 1) x = mulm(x, b);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r && comp; ++i) {
            x = mulm(x, x);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

// the first primes q = 2^bits - t 2N + 1 below 2^bits (N = 2^16), as the parameter sets use
static std::vector<uint64_t> primes_of(int bits, int count)
{
    std::vector<uint64_t> out;
    const uint64_t two_n = 1ull << 17;
    for (uint64_t t = 1; (int)out.size() < count; ++t) {
        uint64_t q = (1ull << bits) - t * two_n + 1;
        if (is_prime(q)) out.push_back(q);
    }
    return out;
}

// ----------------------------------------------- emulation of mac_cols
struct Emu {
    uint64_t lo = 0, mid = 0, hi = 0;
    uint32_t clo = 0, cmid = 0;
};

// v_mad_u64_u32 d, c, a, b, s: d = a b + s mod 2^64, c = the carry out of 2^64
static uint64_t mad_co(uint32_t a, uint32_t b, uint64_t s, uint32_t &c)
{
    const u128x t = (u128x)a * b + s;
    c = (uint32_t)(t >> 64);
    return (uint64_t)t;
}

// v_addc_co_u32 d, _, 0, x, c: d = x + c mod 2^32
static uint32_t addc(uint32_t x, uint32_t c) { return x + c; }

static void emu_mac(Emu &e, uint64_t y, uint64_t h)
{
    const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32), h0 = (uint32_t)h, h1 = (uint32_t)(h >> 32);
    uint32_t c0, c1, c2, cd;
    e.lo = mad_co(y0, h0, e.lo, c0);
    e.mid = mad_co(y0, h1, e.mid, c1);
    e.mid = mad_co(y1, h0, e.mid, c2);
    e.hi = mad_co(y1, h1, e.hi, cd);
    e.clo = addc(e.clo, c0);
    e.cmid = addc(e.cmid, c1);
    e.cmid = addc(e.cmid, c2);
}

static u128x emu_total(const Emu &e)
{
    MacCols c;
    c.lo = e.lo;
    c.mid = e.mid;
    c.hi = e.hi;
    c.clo = e.clo;
    c.cmid = e.cmid;
    return to128(mac_total(c));
}

int main()
{
    std::mt19937_64 rng(250704775);
    std::vector<uint64_t> qs;
    for (int bits : {40, 50, 60})
        for (uint64_t q : primes_of(bits, 3)) qs.push_back(q);

    // exact product of any two 64-bit words
    std::vector<uint64_t> words = {0, 1, 2, 0xFFFFFFFFull, 0x100000000ull, 0x100000001ull, (1ull << 61) - 1,
                                   (1ull << 63), ~0ull, ~0ull - 1};
    for (int i = 0; i < 2000; ++i) words.push_back(rng());
    for (uint64_t a : words)
        for (size_t j = 0; j < words.size(); j += 7) {
            const uint64_t b = words[j];
            CHECK(to128(mul_wide(a, b)) == (u128x)a * b, "mul_wide %llx %llx", (unsigned long long)a,
                  (unsigned long long)b);
            CHECK(mul_hi(a, b) == (uint64_t)(((u128x)a * b) >> 64), "mul_hi");
        }

    for (uint64_t q : qs) {
        const Prime P = prime_of(q);
        std::vector<uint64_t> ops = {0, 1, 2, q - 2, q - 1, (q - 1) / 2, (q + 1) / 2, 0xFFFFFFFFull,
                                     0x100000000ull, 0x100000001ull, 1ull << 31};
        for (int i = 0; i < 300; ++i) ops.push_back(rng() % q);
        // reduce128 on any 128-bit value
        std::vector<u128x> zs = {0, 1, (u128x)q, (u128x)q * q, ~(u128x)0, ((u128x)1 << 127), (u128x)(~0ull),
                                 ((u128x)(~0ull) << 64), (u128x)q * (~0ull)};
        for (int i = 0; i < 3000; ++i) zs.push_back(((u128x)rng() << 64) | rng());
        for (u128x z : zs) CHECK(reduce128(from128(z), P) == (uint64_t)(z % q), "reduce128 q=%llu", (unsigned long long)q);
        for (uint64_t x : ops)
            for (uint64_t y : ops) {
                const uint64_t want = (uint64_t)((u128x)x * y % q);
                CHECK(mulmod(x, y, P) == want, "mulmod q=%llu x=%llu y=%llu", (unsigned long long)q,
                      (unsigned long long)x, (unsigned long long)y);
                // Shoup with y as the constant; x may be any lazy value below 4q (and any 64-bit word)
                const uint64_t ys = shoup_of(y, q);
                for (uint64_t xx : {x, x + q, x + 2 * q, x + 3 * q}) {
                    const uint64_t l = shoup_lazy(xx, y, ys, q);
                    CHECK(l < 2 * q && l % q == (uint64_t)((u128x)xx * y % q), "shoup_lazy");
                    CHECK(shoup(xx, y, ys, q) == (uint64_t)((u128x)xx * y % q), "shoup");
                }
                CHECK(addmod(x, y, q) == (uint64_t)(((u128x)x + y) % q), "addmod");
                CHECK(submod(x, y, q) == (uint64_t)(((u128x)x + q - y) % q), "submod");
            }
        for (uint64_t x : {~0ull, ~0ull - q, 1ull << 63})
            for (uint64_t y : ops) {
                const uint64_t ys = shoup_of(y, q);
                CHECK(shoup(x, y, ys, q) == (uint64_t)((u128x)x * y % q), "shoup on a full word");
            }
    }

    // column sums: y, h < 2^61, short sums at the maxima and long seeded sums
    const uint64_t top = (1ull << 61) - 1;
    std::vector<std::vector<std::pair<uint64_t, uint64_t>>> sums;
    for (int n : {1, 2, 11, 16, 255, 4096, 65535}) {
        std::vector<std::pair<uint64_t, uint64_t>> t;
        for (int i = 0; i < n; ++i) t.push_back({top, top});
        sums.push_back(t);
        std::vector<std::pair<uint64_t, uint64_t>> r;
        for (int i = 0; i < n; ++i) r.push_back({rng() & top, rng() & top});
        sums.push_back(r);
        std::vector<std::pair<uint64_t, uint64_t>> m;
        for (int i = 0; i < n; ++i)
            m.push_back({i % 3 ? top : 0xFFFFFFFFull, i % 2 ? 0x100000001ull : top - (uint64_t)i});
        sums.push_back(m);
    }
    for (const auto &t : sums) {
        Emu e;
        u128x want = 0;
        for (const auto &yh : t) {
            emu_mac(e, yh.first, yh.second);
            want += (u128x)yh.first * yh.second;
        }
        CHECK(emu_total(e) == want, "mac_cols columns, %zu terms", t.size());
    }

    // split columns (MacSplit): constants below 2^50, inputs below 2^62, up to 16 terms
    {
        const uint64_t hmax = (1ull << 50) - 1, ymax = (1ull << 62) - 1;
        const std::vector<uint64_t> hs = {0, 1, (1ull << 27) - 1, 1ull << 27, (1ull << 27) + 1, 0xFFFFFFFFull, hmax};
        const std::vector<uint64_t> ys = {0, 1, 0xFFFFFFFFull, 1ull << 32, ymax, (1ull << 61) + (1ull << 60) - 1};
        for (int n : {1, 2, 4, 11, 15, 16}) {
            for (uint64_t h : hs)
                for (uint64_t y : ys) {
                    MacSplit m;
                    u128x want = 0;
                    for (int i = 0; i < n; ++i) {
                        m.add(y, split_const(h));
                        want += (u128x)y * h;
                    }
                    CHECK(to128(m.total()) == want, "MacSplit %d terms of %llx * %llx", n, (unsigned long long)y,
                          (unsigned long long)h);
                }
            for (int rep = 0; rep < 200; ++rep) {
                MacSplit m;
                u128x want = 0;
                for (int i = 0; i < n; ++i) {
                    const uint64_t y = rep % 4 ? rng() & ymax : ymax - (rng() & 0xFF);
                    const uint64_t h = rep % 3 ? rng() & hmax : hmax - (rng() & 0xFF);
                    m.add(y, split_const(h));
                    want += (u128x)y * h;
                }
                CHECK(to128(m.total()) == want, "MacSplit %d seeded terms", n);
            }
        }
    }

    // ModDown's centred conversion from shifted inputs: the inverse NTT stores u_k = y_k + p_k
    // when y_k <= (p_k - 1)/2, else y_k; the conversion sums u_k [P/p_k]_q exactly, reduces, and
    // subtracts K [P]_q.  That must equal sum_k yc_k [P/p_k]_q mod q with yc_k the centred
    // representative, for 50-bit targets (split columns) and 60-bit ones (mac_cols).
    {
        auto mulm = [](uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128x)a * b % m); };
        const std::vector<uint64_t> sp = primes_of(60, 16);
        std::vector<uint64_t> targets = primes_of(50, 2);
        for (uint64_t q : primes_of(60, 18))
            if (std::find(sp.begin(), sp.end(), q) == sp.end()) targets.push_back(q);
        for (int K : {1, 2, 4, 10, 16})
            for (uint64_t q : targets) {
                const Prime P = prime_of(q);
                uint64_t pq = 1;  // [P]_q
                for (int k = 0; k < K; ++k) pq = mulm(pq, sp[k] % q, q);
                std::vector<uint64_t> h(K);  // [P/p_k]_q
                for (int k = 0; k < K; ++k) {
                    h[k] = 1;
                    for (int j = 0; j < K; ++j)
                        if (j != k) h[k] = mulm(h[k], sp[j] % q, q);
                }
                const uint64_t corr = reduce128(mul_wide((uint64_t)K, pq), P);
                for (int rep = 0; rep < 300; ++rep) {
                    std::vector<uint64_t> y(K);
                    for (int k = 0; k < K; ++k) {
                        const uint64_t p = sp[k];
                        const uint64_t edge[] = {0, 1, (p - 1) / 2, (p + 1) / 2, p - 1};
                        y[k] = rep < 5 ? edge[rep] : (rep % 7 == 0 ? edge[rng() % 5] : rng() % p);
                    }
                    // exact centred sum, reduced
                    __int128 exact = 0;
                    for (int k = 0; k < K; ++k) {
                        const __int128 yc = y[k] <= (sp[k] - 1) / 2 ? (__int128)y[k] : (__int128)y[k] - sp[k];
                        exact += yc * (__int128)h[k];
                    }
                    __int128 rm = exact % (__int128)q;
                    if (rm < 0) rm += q;
                    u128x z = 0;
                    MacSplit ms;
                    Emu e;
                    for (int k = 0; k < K; ++k) {
                        const uint64_t u = y[k] <= (sp[k] >> 1) ? y[k] + sp[k] : y[k];
                        CHECK(u < (1ull << 62), "shifted input below 2^62");
                        z += (u128x)u * h[k];
                        if (q < kSplitMaxConst)
                            ms.add(u, split_const(h[k]));
                        else
                            emu_mac(e, u, h[k]);
                    }
                    const u128x tot = q < kSplitMaxConst ? to128(ms.total()) : emu_total(e);
                    CHECK(tot == z, "conversion sum, K=%d q=%llu", K, (unsigned long long)q);
                    const uint64_t got = submod(reduce128(from128(tot), P), corr, q);
                    CHECK(got == (uint64_t)rm, "centred conversion from shifted inputs, K=%d q=%llu", K,
                          (unsigned long long)q);
                }
            }
    }

    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
