// Context creation: host-side precomputation of every constant the kernels
// use (Sec. III-E of the paper: precomputation happens once, when the context
// is created) and its upload to the device in a single allocation.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace ckks {

thread_local std::string g_last_error;

ckks_status fail(ckks_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

hipError_t scratch_setup(int device);  // noalloc.hip

typedef unsigned __int128 wide;

// Host modular arithmetic shared by the context builders (internal.h).
uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((wide)a * b % m); }

uint64_t pow_mod(uint64_t base, uint64_t e, uint64_t m)
{
    uint64_t acc = 1 % m;
    for (base %= m; e; e >>= 1, base = mul_mod(base, base, m))
        if (e & 1) acc = mul_mod(acc, base, m);
    return acc;
}

uint64_t inv_mod(uint64_t a, uint64_t m)  // m prime
{
    return pow_mod(a % m, m - 2, m);
}

bool probably_prime(uint64_t n)
{
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t b : bases)
        if (n % b == 0) return n == b;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t b : bases) {
        uint64_t x = pow_mod(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int r = 1; r < s && composite; ++r) {
            x = mul_mod(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

namespace {

uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((wide)w << 64) / q); }

ulonglong2 pair(uint64_t w, uint64_t q)
{
    ulonglong2 r;
    r.x = w;
    r.y = shoup_of(w, q);
    return r;
}

}  // namespace

// Smallest primitive 2N-th root of unity modulo q: a candidate g^((q-1)/2N) of
// order exactly 2N (its N-th power is -1) generates them all as its odd powers.
uint64_t smallest_2n_root(uint64_t q, uint64_t two_n)
{
    uint64_t half = two_n / 2, root = 0;
    for (uint64_t g = 2; g < q && !root; ++g) {
        uint64_t c = pow_mod(g, (q - 1) / two_n, q);
        if (pow_mod(c, half, q) == q - 1) root = c;
    }
    uint64_t step = mul_mod(root, root, q), best = root;
    for (uint64_t e = 3, cur = root; e < two_n; e += 2) {
        cur = mul_mod(cur, step, q);
        best = std::min(best, cur);
    }
    return best;
}

uint32_t reverse_bits(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t b = 0; b < bits; ++b, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace ckks

using namespace ckks;

extern "C" const char *ckks_last_error(void) { return g_last_error.c_str(); }

extern "C" ckks_status ckks_ctx_create(uint32_t log_n, const uint64_t *q, uint32_t n_q, const uint64_t *p,
                                       uint32_t n_p, uint32_t dnum, int hip_device, ckks_ctx **out)
{
    if (!out || !q || !p) return fail(CKKS_E_ARG, "ckks_ctx_create: null pointer");
    *out = nullptr;
    if (log_n != 12 && log_n != 16) return fail(CKKS_E_UNSUPPORTED, "ckks_ctx_create: log_n must be 12 or 16");
    if (n_q < 1 || n_p < 1 || dnum < 1 || dnum > n_q)
        return fail(CKKS_E_ARG, "ckks_ctx_create: need n_q >= 1, n_p >= 1, 1 <= dnum <= n_q");
    uint32_t alpha = (n_q + dnum - 1) / dnum;
    if (n_q + n_p > (uint32_t)kMaxPrimes || alpha > (uint32_t)kMaxDigitPrimes || n_p > (uint32_t)kMaxDigitPrimes ||
        dnum > (uint32_t)kMaxDigits)
        return fail(CKKS_E_UNSUPPORTED, "ckks_ctx_create: at most 64 primes, 16 per digit, 16 special, 16 digits");
    const uint64_t N = 1ull << log_n, two_n = 2 * N;
    std::vector<uint64_t> primes(q, q + n_q);
    primes.insert(primes.end(), p, p + n_p);
    for (size_t i = 0; i < primes.size(); ++i) {
        uint64_t m = primes[i];
        if (m >= (1ull << 61) || m % two_n != 1 || !probably_prime(m))
            return fail(CKKS_E_ARG, "ckks_ctx_create: prime " + std::to_string(i) +
                                        " is not a prime below 2^61 congruent to 1 mod 2N");
        for (size_t k = 0; k < i; ++k)
            if (primes[k] == m) return fail(CKKS_E_ARG, "ckks_ctx_create: primes must be distinct");
    }
    if (hipSetDevice(hip_device) != hipSuccess) return fail(CKKS_E_DEVICE, "ckks_ctx_create: hipSetDevice failed");
    // the device address of the no-allocation entry point's static scratch, once per device (a
    // failure is kept and reported by that entry point; the other calls do not use the scratch)
    (void)scratch_setup(hip_device);

    ckks_ctx *ctx = new ckks_ctx();
    ctx->device = hip_device;
    ctx->logn = log_n;
    ctx->N = (uint32_t)N;
    ctx->nq = n_q;
    ctx->np = n_p;
    ctx->dnum = dnum;
    ctx->alpha = alpha;
    ctx->primes = primes;
    const uint32_t np_all = n_q + n_p;

    // ---- host tables
    std::vector<Prime> hp(np_all);
    std::vector<ulonglong2> tw_f((size_t)np_all * N), tw_i((size_t)np_all * N);
    std::vector<double> twd_f((size_t)np_all * N), twd_i((size_t)np_all * N);
    for (uint32_t i = 0; i < np_all; ++i) {
        uint64_t m = primes[i];
        Prime &P = hp[i];
        P.q = m;
        P.two_q = 2 * m;
        P.r64 = (uint64_t)(((wide)1 << 64) % m);
        P.r64_s = shoup_of(P.r64, m);
        P.one_s = shoup_of(1, m);
        P.ninv = inv_mod(N % m, m);
        P.ninv_s = shoup_of(P.ninv, m);
        P.qinv = 1.0 / (double)m;
        uint64_t psi = smallest_2n_root(m, two_n), ipsi = inv_mod(psi, m);
        uint64_t f = 1, b = 1;
        for (uint32_t k = 0; k < N; ++k) {
            uint32_t pos = reverse_bits(k, log_n);
            tw_f[(size_t)i * N + pos] = pair(f, m);
            tw_i[(size_t)i * N + pos] = pair(b, m);
            twd_f[(size_t)i * N + pos] = m < kFpMaxPrime ? (double)f : 0.0;
            twd_i[(size_t)i * N + pos] = m < kFpMaxPrime ? (double)b : 0.0;
            f = mul_mod(f, psi, m);
            b = mul_mod(b, ipsi, m);
        }
    }
    // base-conversion sets: every digit j of every possible size, then P
    ctx->nsets = dnum * alpha + 1;
    const size_t hm_stride = (size_t)np_all * kMaxDigitPrimes;
    std::vector<ulonglong2> bc_hinv((size_t)ctx->nsets * kMaxDigitPrimes);
    std::vector<uint64_t> bc_hmod((size_t)ctx->nsets * hm_stride, 0);
    std::vector<ulonglong2> bc_ys((size_t)ctx->nsets * kMaxDigitPrimes);
    std::vector<double> bc_ysd((size_t)ctx->nsets * kMaxDigitPrimes, 0.0);
    auto build_set = [&](uint32_t set, const uint64_t *src, uint32_t ns) {
        for (uint32_t i = 0; i < ns; ++i) {
            uint64_t prod = 1;
            for (uint32_t k = 0; k < ns; ++k)
                if (k != i) prod = mul_mod(prod, src[k] % src[i], src[i]);
            uint64_t hinv = inv_mod(prod, src[i]);
            bc_hinv[(size_t)set * kMaxDigitPrimes + i] = pair(hinv, src[i]);
            uint64_t ys = mul_mod(hinv, inv_mod(N % src[i], src[i]), src[i]);
            bc_ys[(size_t)set * kMaxDigitPrimes + i] = pair(ys, src[i]);
            bc_ysd[(size_t)set * kMaxDigitPrimes + i] = (double)ys;
            for (uint32_t c = 0; c < np_all; ++c) {
                uint64_t v = 1;
                for (uint32_t k = 0; k < ns; ++k)
                    if (k != i) v = mul_mod(v, src[k] % primes[c], primes[c]);
                // targets below 2^50 keep the constant split for the conversions' MacSplit sums
                bc_hmod[(size_t)set * hm_stride + (size_t)c * kMaxDigitPrimes + i] =
                    primes[c] < kSplitMaxConst ? split_const(v) : v;
            }
        }
    };
    for (uint32_t j = 0; j < dnum; ++j)
        for (uint32_t s = 1; s <= alpha; ++s) {
            uint32_t lo = j * alpha;
            if (lo + s <= n_q) build_set(ctx->set_index(j, s), &primes[lo], s);
        }
    build_set(ctx->pset_index(), &primes[n_q], n_p);
    std::vector<ulonglong2> pinv(np_all);
    std::vector<uint64_t> pmod(np_all, 0);
    for (uint32_t i = 0; i < np_all; ++i) {
        uint64_t P = 1;
        for (uint32_t k = 0; k < n_p; ++k) P = mul_mod(P, p[k] % primes[i], primes[i]);
        pinv[i] = i < n_q ? pair(inv_mod(P, primes[i]), primes[i]) : pair(0, primes[i]);
        pmod[i] = i < n_q ? P : 0;
    }
    std::vector<ulonglong2> rs_inv((size_t)n_q * n_q);
    std::vector<uint64_t> rs_mod((size_t)n_q * n_q, 0);
    for (uint32_t l = 0; l < n_q; ++l)
        for (uint32_t i = 0; i < n_q; ++i) {
            uint64_t qi = primes[i];
            rs_mod[(size_t)l * n_q + i] = primes[l] % qi;
            rs_inv[(size_t)l * n_q + i] = i < l ? pair(inv_mod(primes[l] % qi, qi), qi) : pair(0, qi);
        }

    // ---- one device block
    size_t off_primes = 0;
    size_t off_twf = align_up(off_primes + np_all * sizeof(Prime));
    size_t off_twi = align_up(off_twf + tw_f.size() * sizeof(ulonglong2));
    size_t off_twdf = align_up(off_twi + tw_i.size() * sizeof(ulonglong2));
    size_t off_twdi = align_up(off_twdf + twd_f.size() * sizeof(double));
    size_t off_hinv = align_up(off_twdi + twd_i.size() * sizeof(double));
    size_t off_hmod = align_up(off_hinv + bc_hinv.size() * sizeof(ulonglong2));
    size_t off_ys = align_up(off_hmod + bc_hmod.size() * sizeof(uint64_t));
    size_t off_ysd = align_up(off_ys + bc_ys.size() * sizeof(ulonglong2));
    size_t off_pinv = align_up(off_ysd + bc_ysd.size() * sizeof(double));
    size_t off_rsi = align_up(off_pinv + pinv.size() * sizeof(ulonglong2));
    size_t off_rsm = align_up(off_rsi + rs_inv.size() * sizeof(ulonglong2));
    size_t off_pmod = align_up(off_rsm + rs_mod.size() * sizeof(uint64_t));
    size_t total = align_up(off_pmod + pmod.size() * sizeof(uint64_t));
    char *blk = nullptr;
    if (hipMalloc((void **)&blk, total) != hipSuccess) {
        delete ctx;
        return fail(CKKS_E_NOMEM, "ckks_ctx_create: hipMalloc of the tables failed");
    }
    ctx->dev_block = blk;
    ctx->d_primes = (Prime *)(blk + off_primes);
    ctx->d_tw_fwd = (ulonglong2 *)(blk + off_twf);
    ctx->d_tw_inv = (ulonglong2 *)(blk + off_twi);
    ctx->d_twd_fwd = (double *)(blk + off_twdf);
    ctx->d_twd_inv = (double *)(blk + off_twdi);
    ctx->d_bc_hinv = (ulonglong2 *)(blk + off_hinv);
    ctx->d_bc_hmod = (uint64_t *)(blk + off_hmod);
    ctx->d_bc_ys = (ulonglong2 *)(blk + off_ys);
    ctx->d_bc_ysd = (double *)(blk + off_ysd);
    ctx->d_pinv = (ulonglong2 *)(blk + off_pinv);
    ctx->d_rs_inv = (ulonglong2 *)(blk + off_rsi);
    ctx->d_rs_mod = (uint64_t *)(blk + off_rsm);
    ctx->d_pmod = (uint64_t *)(blk + off_pmod);
    bool ok = hipMemcpy(ctx->d_primes, hp.data(), hp.size() * sizeof(Prime), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(ctx->d_tw_fwd, tw_f.data(), tw_f.size() * sizeof(ulonglong2), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_tw_inv, tw_i.data(), tw_i.size() * sizeof(ulonglong2), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_twd_fwd, twd_f.data(), twd_f.size() * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_twd_inv, twd_i.data(), twd_i.size() * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_bc_hinv, bc_hinv.data(), bc_hinv.size() * sizeof(ulonglong2),
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(ctx->d_bc_hmod, bc_hmod.data(), bc_hmod.size() * sizeof(uint64_t), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_bc_ys, bc_ys.data(), bc_ys.size() * sizeof(ulonglong2), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_bc_ysd, bc_ysd.data(), bc_ysd.size() * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_pinv, pinv.data(), pinv.size() * sizeof(ulonglong2), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_rs_inv, rs_inv.data(), rs_inv.size() * sizeof(ulonglong2), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_rs_mod, rs_mod.data(), rs_mod.size() * sizeof(uint64_t), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(ctx->d_pmod, pmod.data(), pmod.size() * sizeof(uint64_t), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(blk);
        delete ctx;
        return fail(CKKS_E_DEVICE, "ckks_ctx_create: upload of the tables failed");
    }
    *out = ctx;
    return CKKS_OK;
}

extern "C" void ckks_ctx_destroy(ckks_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->dev_block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(ctx->device);
        (void)hipFree(ctx->dev_block);
        (void)hipSetDevice(cur);
    }
    delete ctx;
}

extern "C" ckks_status ckks_get_twiddles(const ckks_ctx *ctx, uint32_t limb, uint64_t *host_out)
{
    if (!ctx || !host_out) return fail(CKKS_E_ARG, "ckks_get_twiddles: null pointer");
    if (limb >= ctx->nq + ctx->np) return fail(CKKS_E_ARG, "ckks_get_twiddles: limb out of range");
    std::vector<ulonglong2> tmp(ctx->N);
    if (hipMemcpy(tmp.data(), ctx->d_tw_fwd + (size_t)limb * ctx->N, ctx->N * sizeof(ulonglong2),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CKKS_E_DEVICE, "ckks_get_twiddles: copy failed");
    for (uint32_t k = 0; k < ctx->N; ++k) host_out[k] = tmp[k].x;
    return CKKS_OK;
}
