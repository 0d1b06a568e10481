/*
 * Plain CPU oracle for the RNS-CKKS key-switching hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may use it.  It shares no code, header, table or constant
 * generator with the GPU library: every constant it needs (the 2N-th root psi,
 * twiddle powers, CRT constants) is derived here again from the prime list.
 *
 * Style: textbook loops, exact 128-bit products reduced with '%', canonical
 * residues in [0, m) everywhere.  OpenMP only splits independent limbs or
 * coefficient indices, so results do not depend on the thread count.
 *
 * Notation follows the paper (FIDESlib, arXiv 2507.04775): N = 2^logn, the
 * ciphertext basis q_0..q_L, the special basis p_0..p_{K-1}, dnum digits of
 * alpha = ceil((L+1)/dnum) limbs, level l meaning limbs q_0..q_l.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- scalars */

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }
static uint64_t addm(uint64_t a, uint64_t b, uint64_t m) { uint64_t s = a + b; return s >= m ? s - m : s; }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t m) { return a >= b ? a - b : a + m - b; }
static uint64_t powm(uint64_t b, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = mulm(r, b, m);
        b = mulm(b, b, m);
        e >>= 1;
    }
    return r;
}
/* inverse modulo a prime by Fermat's little theorem */
static uint64_t invm(uint64_t a, uint64_t m) { return powm(a % m, m - 2, m); }

static uint32_t bitrev(uint32_t x, uint32_t bits)
{
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

/*
 * psi: the smallest primitive 2N-th root of unity modulo q (Table II names psi
 * as the root used by the (i)NTT; the paper does not say which root, the
 * smallest one is the reading taken here).  A root r is found as x^((q-1)/2N)
 * with r^N = -1; every primitive 2N-th root is an odd power of r.
 * Returns 0 when q != 1 (mod 2N).
 */
uint64_t orc_psi(uint64_t q, uint32_t logn)
{
    uint64_t N = 1ull << logn, two_n = 2 * N;
    if ((q - 1) % two_n != 0) return 0;
    uint64_t r = 0;
    for (uint64_t x = 2; x < q; x++) {
        uint64_t c = powm(x, (q - 1) / two_n, q);
        if (powm(c, N, q) == q - 1) { r = c; break; }
    }
    uint64_t best = r, r2 = mulm(r, r, q), cur = r;
    for (uint64_t k = 3; k < two_n; k += 2) {
        cur = mulm(cur, r2, q);
        if (cur < best) best = cur;
    }
    return best;
}

/* ------------------------------------------------------------ (i)NTT, III-F.4 */

/*
 * Forward negacyclic NTT of one limb, in place: radix-2 Cooley-Tukey with the
 * twist by psi merged into the butterflies; natural-order coefficients in,
 * bit-reversed evaluations out, so that out[i] = sum_j a_j psi^((2 br(i)+1) j).
 */
static void ntt_one(uint64_t q, uint32_t logn, uint64_t psi, uint64_t *a)
{
    uint64_t N = 1ull << logn;
    uint64_t *tab = (uint64_t *)malloc(N * sizeof(uint64_t));
    uint64_t pw = 1;
    for (uint64_t k = 0; k < N; k++) { tab[bitrev((uint32_t)k, logn)] = pw; pw = mulm(pw, psi, q); }
    uint64_t t = N;
    for (uint64_t m = 1; m < N; m <<= 1) {
        t >>= 1;
        for (uint64_t i = 0; i < m; i++) {
            uint64_t j1 = 2 * i * t, S = tab[m + i];
            for (uint64_t j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = mulm(a[j + t], S, q);
                a[j] = addm(U, V, q);
                a[j + t] = subm(U, V, q);
            }
        }
    }
    free(tab);
}

/*
 * Inverse negacyclic NTT of one limb, in place: radix-2 Gentleman-Sande
 * butterflies take the bit-reversed evaluations back to natural-order
 * coefficients with no explicit bit reversal, then scale by N^-1.
 */
static void intt_one(uint64_t q, uint32_t logn, uint64_t psi, uint64_t *a)
{
    uint64_t N = 1ull << logn;
    uint64_t ipsi = invm(psi, q);
    uint64_t *tab = (uint64_t *)malloc(N * sizeof(uint64_t));
    uint64_t pw = 1;
    for (uint64_t k = 0; k < N; k++) { tab[bitrev((uint32_t)k, logn)] = pw; pw = mulm(pw, ipsi, q); }
    uint64_t t = 1;
    for (uint64_t m = N >> 1; m >= 1; m >>= 1) {
        uint64_t j1 = 0;
        for (uint64_t i = 0; i < m; i++) {
            uint64_t S = tab[m + i];
            for (uint64_t j = j1; j < j1 + t; j++) {
                uint64_t U = a[j], V = a[j + t];
                a[j] = addm(U, V, q);
                a[j + t] = mulm(subm(U, V, q), S, q);
            }
            j1 += 2 * t;
        }
        t <<= 1;
    }
    uint64_t ninv = invm(N % q, q);
    for (uint64_t j = 0; j < N; j++) a[j] = mulm(a[j], ninv, q);
    free(tab);
}

/* (i)NTT of n limbs a[i] (row i under modulus mods[i]); inverse != 0 selects the iNTT */
void orc_ntt(const uint64_t *mods, uint32_t n, uint32_t logn, uint64_t *a, int inverse)
{
    uint64_t N = 1ull << logn;
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        uint64_t psi = orc_psi(mods[i], logn);
        if (inverse) intt_one(mods[i], logn, psi, a + (uint64_t)i * N);
        else ntt_one(mods[i], logn, psi, a + (uint64_t)i * N);
    }
}

/* ----------------------------------------------- fast base conversion, Eq. (1) */

/*
 * Conv_{B->C}: every coefficient x = (x_0..x_{r-1}) in basis B (coefficient
 * domain) is first scaled limb-wise, y_i = [x_i * (B/b_i)^-1]_{b_i}, then the
 * modular matrix-vector product out_c = [sum_i y_i * [B/b_i]_c]_c is taken for
 * every target prime c.  The products are summed exactly in 128 bits and
 * reduced once (the paper accumulates in 128 bits as well).
 */
void orc_bconv(const uint64_t *src, uint32_t ns, const uint64_t *dst, uint32_t nd, uint32_t logn,
               const uint64_t *x, uint64_t *out)
{
    uint64_t N = 1ull << logn;
    uint64_t *hat_inv = (uint64_t *)malloc(ns * sizeof(uint64_t));
    uint64_t *hat_mod = (uint64_t *)malloc((size_t)ns * nd * sizeof(uint64_t));
    for (uint32_t i = 0; i < ns; i++) {
        uint64_t prod = 1;
        for (uint32_t k = 0; k < ns; k++)
            if (k != i) prod = mulm(prod, src[k] % src[i], src[i]);
        hat_inv[i] = invm(prod, src[i]);
        for (uint32_t c = 0; c < nd; c++) {
            uint64_t pc = 1;
            for (uint32_t k = 0; k < ns; k++)
                if (k != i) pc = mulm(pc, src[k] % dst[c], dst[c]);
            hat_mod[(size_t)c * ns + i] = pc;
        }
    }
#pragma omp parallel
    {
        uint64_t *y = (uint64_t *)malloc(ns * sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t n = 0; n < (int64_t)N; n++) {
            for (uint32_t i = 0; i < ns; i++) y[i] = mulm(x[(uint64_t)i * N + n], hat_inv[i], src[i]);
            for (uint32_t c = 0; c < nd; c++) {
                u128 acc = 0;
                for (uint32_t i = 0; i < ns; i++) acc += (u128)y[i] * hat_mod[(size_t)c * ns + i];
                out[(uint64_t)c * N + n] = (uint64_t)(acc % dst[c]);
            }
        }
        free(y);
    }
    free(hat_inv);
    free(hat_mod);
}

/* ----------------------------------------------------- hybrid key switching */

/* row r of an extended polynomial at level l: q_0..q_l, then p_0..p_{K-1} */
static uint64_t row_mod(const uint64_t *q, const uint64_t *p, uint32_t level, uint32_t r)
{
    return r <= level ? q[r] : p[r - level - 1];
}
/* the matching row of a top-level key laid out [dnum][2][nq+np][N] */
static uint32_t key_row(uint32_t nq, uint32_t level, uint32_t r)
{
    return r <= level ? r : nq + (r - level - 1);
}

static uint32_t alpha_of(uint32_t nq, uint32_t dnum) { return (nq + dnum - 1) / dnum; }

/*
 * ModUp (hybrid key switching, Sec. II-A and III-F.3): the eval-domain input
 * d at level l is brought to coefficients, cut into beta = ceil((l+1)/alpha)
 * digits of consecutive limbs (the digit layout is fixed by the top level), and
 * every digit is extended by fast base conversion to all other rows of
 * Q_l u P, which are then brought back to the evaluation domain.  The digit's
 * own rows are copied from d unchanged.  ext has shape [beta][l+1+K][N].
 */
void orc_modup(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
               uint32_t dnum, uint32_t level, const uint64_t *d, uint64_t *ext)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1, rows = n + np, alpha = alpha_of(nq, dnum);
    uint32_t beta = (n + alpha - 1) / alpha;
    uint64_t *dc = (uint64_t *)malloc((size_t)n * N * sizeof(uint64_t));
    memcpy(dc, d, (size_t)n * N * sizeof(uint64_t));
    orc_ntt(q, n, logn, dc, 1);
    uint64_t *mods = (uint64_t *)malloc(rows * sizeof(uint64_t));
    for (uint32_t r = 0; r < rows; r++) mods[r] = row_mod(q, p, level, r);
    for (uint32_t j = 0; j < beta; j++) {
        uint32_t lo = j * alpha, hi = (j + 1) * alpha < n ? (j + 1) * alpha : n;
        uint64_t *e = ext + (size_t)j * rows * N;
        uint32_t nd = rows - (hi - lo);
        uint64_t *dst = (uint64_t *)malloc(nd * sizeof(uint64_t));
        uint32_t *dst_row = (uint32_t *)malloc(nd * sizeof(uint32_t));
        uint32_t c = 0;
        for (uint32_t r = 0; r < rows; r++)
            if (r < lo || r >= hi) { dst[c] = mods[r]; dst_row[c] = r; c++; }
        uint64_t *conv = (uint64_t *)malloc((size_t)nd * N * sizeof(uint64_t));
        orc_bconv(q + lo, hi - lo, dst, nd, logn, dc + (size_t)lo * N, conv);
        orc_ntt(dst, nd, logn, conv, 0);
        for (uint32_t k = 0; k < nd; k++) memcpy(e + (size_t)dst_row[k] * N, conv + (size_t)k * N, N * sizeof(uint64_t));
        for (uint32_t r = lo; r < hi; r++) memcpy(e + (size_t)r * N, d + (size_t)r * N, N * sizeof(uint64_t));
        free(conv);
        free(dst);
        free(dst_row);
    }
    free(mods);
    free(dc);
}

/* the eval-domain automorphism X -> X^g as a gather: out[i] = in[src(i)] */
static uint32_t galois_src(uint32_t i, uint64_t g, uint32_t logn)
{
    uint64_t N = 1ull << logn, two_n = 2 * N;
    uint64_t e = (2 * (uint64_t)bitrev(i, logn) + 1) * (g % two_n) % two_n; /* odd exponent */
    return bitrev((uint32_t)((e - 1) / 2), logn);
}

/*
 * Key inner product (the dot-product step of hybrid key switching):
 * acc_t[r] = sum_j phi_g(ext_j)[r] * key[j][t][row r], t = 0, 1, over all
 * l+1+K rows.  g = 1 is the plain inner product; another odd g applies the
 * automorphism to the extended digits first (hoisted rotation, III-F.6).
 * key is the top-level key [dnum][2][nq+np][N]; acc is [2][l+1+K][N].
 */
void orc_inner_product(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                       uint32_t dnum, uint32_t level, const uint64_t *ext, const uint64_t *key,
                       uint64_t g, uint64_t *acc)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1, rows = n + np, alpha = alpha_of(nq, dnum);
    uint32_t beta = (n + alpha - 1) / alpha, krows = nq + np;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)rows; r++) {
        uint64_t m = row_mod(q, p, level, (uint32_t)r);
        uint32_t kr = key_row(nq, level, (uint32_t)r);
        for (uint64_t i = 0; i < N; i++) {
            uint32_t si = (g == 1) ? (uint32_t)i : galois_src((uint32_t)i, g, logn);
            for (uint32_t t = 0; t < 2; t++) {
                uint64_t s = 0;
                for (uint32_t j = 0; j < beta; j++) {
                    uint64_t v = ext[((size_t)j * rows + r) * N + si];
                    uint64_t k = key[(((size_t)j * 2 + t) * krows + kr) * N + i];
                    s = addm(s, mulm(v, k, m), m);
                }
                acc[((size_t)t * rows + r) * N + i] = s;
            }
        }
    }
}

/*
 * Centred fast base conversion from the special basis: the same sum as
 * orc_bconv, with every y_k taken as its representative in
 * [-(p_k-1)/2, (p_k-1)/2].  The value it represents is v = sum_k y_k P/p_k,
 * congruent to x mod P with |v| < K P / 2 and no bias in sign.
 */
static void bconv_centred(const uint64_t *src, uint32_t ns, const uint64_t *dst, uint32_t nd, uint32_t logn,
                          const uint64_t *x, uint64_t *out)
{
    uint64_t N = 1ull << logn;
    uint64_t *hat_inv = (uint64_t *)malloc(ns * sizeof(uint64_t));
    uint64_t *hat_mod = (uint64_t *)malloc((size_t)ns * nd * sizeof(uint64_t));
    for (uint32_t i = 0; i < ns; i++) {
        uint64_t prod = 1;
        for (uint32_t k = 0; k < ns; k++)
            if (k != i) prod = mulm(prod, src[k] % src[i], src[i]);
        hat_inv[i] = invm(prod, src[i]);
        for (uint32_t c = 0; c < nd; c++) {
            uint64_t pc = 1;
            for (uint32_t k = 0; k < ns; k++)
                if (k != i) pc = mulm(pc, src[k] % dst[c], dst[c]);
            hat_mod[(size_t)c * ns + i] = pc;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < (int64_t)N; n++) {
        for (uint32_t c = 0; c < nd; c++) {
            uint64_t m = dst[c], s = 0;
            for (uint32_t i = 0; i < ns; i++) {
                uint64_t y = mulm(x[(uint64_t)i * N + n], hat_inv[i], src[i]);
                uint64_t t = mulm(y % m, hat_mod[(size_t)c * ns + i], m);      /* y * [B/b_i]_c */
                if (y > (src[i] - 1) / 2) {                                     /* y - b_i instead of y */
                    uint64_t bmod = mulm(src[i] % m, hat_mod[(size_t)c * ns + i], m);
                    t = subm(t, bmod, m);
                }
                s = addm(s, t, m);
            }
            out[(uint64_t)c * N + n] = s;
        }
    }
    free(hat_inv);
    free(hat_mod);
}

/*
 * ModDown: x has rows q_0..q_l, p_0..p_{K-1} (eval domain).  The P rows are
 * brought to coefficients, converted to Q_l with the centred conversion above,
 * brought back, and out_i = [P^-1]_{q_i} * (x_i - NTT(conv_i)) (the ModDown
 * fusion sequence of III-F.5).  The result is (x - v) / P with v = x mod P up
 * to a multiple u P, |v| < K P / 2: x / P rounded with an error of zero mean
 * (a floor division, or a canonical conversion whose overshoot u lies in
 * [0, K), would leave a bias of about K / 2 in every coefficient).  out is
 * [l+1][N].
 */
void orc_moddown(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                 uint32_t level, const uint64_t *x, uint64_t *out)
{
    (void)nq;
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1;
    uint64_t *a = (uint64_t *)malloc((size_t)np * N * sizeof(uint64_t));
    memcpy(a, x + (size_t)n * N, (size_t)np * N * sizeof(uint64_t));
    orc_ntt(p, np, logn, a, 1);
    uint64_t *conv = (uint64_t *)malloc((size_t)n * N * sizeof(uint64_t));
    bconv_centred(p, np, q, n, logn, a, conv);
    orc_ntt(q, n, logn, conv, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        uint64_t P = 1;
        for (uint32_t k = 0; k < np; k++) P = mulm(P, p[k] % q[i], q[i]);
        uint64_t pinv = invm(P, q[i]);
        for (uint64_t c = 0; c < N; c++)
            out[(size_t)i * N + c] = mulm(pinv, subm(x[(size_t)i * N + c], conv[(size_t)i * N + c], q[i]), q[i]);
    }
    free(a);
    free(conv);
}

/* KeySwitch(d) = ModDown(InnerProduct(ModUp(d), key)) for both key halves */
void orc_keyswitch(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                   uint32_t dnum, uint32_t level, const uint64_t *d, const uint64_t *key,
                   uint64_t *out0, uint64_t *out1)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1, rows = n + np, alpha = alpha_of(nq, dnum);
    uint32_t beta = (n + alpha - 1) / alpha;
    uint64_t *ext = (uint64_t *)malloc((size_t)beta * rows * N * sizeof(uint64_t));
    uint64_t *acc = (uint64_t *)malloc((size_t)2 * rows * N * sizeof(uint64_t));
    orc_modup(logn, q, nq, p, np, dnum, level, d, ext);
    orc_inner_product(logn, q, nq, p, np, dnum, level, ext, key, 1, acc);
    orc_moddown(logn, q, nq, p, np, level, acc, out0);
    orc_moddown(logn, q, nq, p, np, level, acc + (size_t)rows * N, out1);
    free(ext);
    free(acc);
}

/* ------------------------------------------------------------- elementwise */

/* out[i] = a[i] op b[i] under mods[i]; op 0 add, 1 sub, 2 mul */
void orc_vec(const uint64_t *mods, uint32_t n, uint32_t logn, const uint64_t *a, const uint64_t *b,
             uint64_t *out, int op)
{
    uint64_t N = 1ull << logn;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        uint64_t m = mods[i];
        for (uint64_t c = 0; c < N; c++) {
            uint64_t u = a[(size_t)i * N + c], v = b[(size_t)i * N + c], r;
            if (op == 0) r = addm(u, v, m);
            else if (op == 1) r = subm(u, v, m);
            else r = mulm(u, v, m);
            out[(size_t)i * N + c] = r;
        }
    }
}

/*
 * HMult with relinearisation (Table I): d0 = a0 b0, d1 = a0 b1 + a1 b0,
 * d2 = a1 b1 limb-wise in the evaluation domain, (k0, k1) = KeySwitch(d2)
 * with the relinearisation key, out = (d0 + k0, d1 + k1).  No rescale.
 */
void orc_hmult_relin(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                     uint32_t dnum, uint32_t level, const uint64_t *a0, const uint64_t *a1,
                     const uint64_t *b0, const uint64_t *b1, const uint64_t *key,
                     uint64_t *out0, uint64_t *out1)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1;
    size_t sz = (size_t)n * N;
    uint64_t *d0 = (uint64_t *)malloc(sz * 8), *d1 = (uint64_t *)malloc(sz * 8), *d2 = (uint64_t *)malloc(sz * 8);
    uint64_t *t = (uint64_t *)malloc(sz * 8), *k0 = (uint64_t *)malloc(sz * 8), *k1 = (uint64_t *)malloc(sz * 8);
    orc_vec(q, n, logn, a0, b0, d0, 2);
    orc_vec(q, n, logn, a0, b1, d1, 2);
    orc_vec(q, n, logn, a1, b0, t, 2);
    orc_vec(q, n, logn, d1, t, d1, 0);
    orc_vec(q, n, logn, a1, b1, d2, 2);
    orc_keyswitch(logn, q, nq, p, np, dnum, level, d2, key, k0, k1);
    orc_vec(q, n, logn, d0, k0, out0, 0);
    orc_vec(q, n, logn, d1, k1, out1, 0);
    free(d0); free(d1); free(d2); free(t); free(k0); free(k1);
}

/*
 * Rescale (Table I, III-F.5 rescale fusion): for one polynomial c at level l,
 * v = INTT_{q_l}(c_l); SwitchModulo lifts v centred ((q_l-1)/2 is the largest
 * value taken as non-negative) into every q_i, i < l; then
 * out_i = [q_l^-1]_{q_i} * (c_i - NTT_{q_i}(SwitchModulo_i(v))).  out is [l][N].
 */
void orc_rescale(uint32_t logn, const uint64_t *q, uint32_t level, const uint64_t *c, uint64_t *out)
{
    uint64_t N = 1ull << logn;
    uint64_t ql = q[level];
    uint64_t *v = (uint64_t *)malloc(N * sizeof(uint64_t));
    memcpy(v, c + (size_t)level * N, N * sizeof(uint64_t));
    orc_ntt(&ql, 1, logn, v, 1);
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < (int64_t)level; i++) {
        uint64_t qi = q[i];
        uint64_t *s = (uint64_t *)malloc(N * sizeof(uint64_t));
        for (uint64_t k = 0; k < N; k++) {
            if (v[k] <= (ql - 1) / 2) s[k] = v[k] % qi;
            else s[k] = subm(v[k] % qi, ql % qi, qi); /* v - q_l, taken mod q_i */
        }
        ntt_one(qi, logn, orc_psi(qi, logn), s);
        uint64_t qlinv = invm(ql % qi, qi);
        for (uint64_t k = 0; k < N; k++)
            out[(size_t)i * N + k] = mulm(qlinv, subm(c[(size_t)i * N + k], s[k], qi), qi);
        free(s);
    }
    free(v);
}

/* -------------------------------------------------------------- automorphism */

/*
 * phi_g on the evaluation domain (X -> X^g, g odd): the value stored at
 * position i is A(psi^(2 br(i)+1)); the automorphism moves A(psi^(e g)) to the
 * slot of psi^e, so out[i] = in[br(((2 br(i)+1) g mod 2N - 1)/2)].
 */
void orc_automorph_eval(uint32_t logn, uint32_t n, uint64_t g, const uint64_t *in, uint64_t *out)
{
    uint64_t N = 1ull << logn;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < (int64_t)n; l++)
        for (uint64_t i = 0; i < N; i++)
            out[(size_t)l * N + i] = in[(size_t)l * N + galois_src((uint32_t)i, g, logn)];
}

/* phi_g on the coefficient domain: a_j X^j -> a_j X^(j g mod 2N), X^N = -1 */
void orc_automorph_coef(const uint64_t *mods, uint32_t n, uint32_t logn, uint64_t g, const uint64_t *in, uint64_t *out)
{
    uint64_t N = 1ull << logn, two_n = 2 * N;
    for (uint32_t l = 0; l < n; l++)
        for (uint64_t j = 0; j < N; j++) {
            uint64_t e = j * (g % two_n) % two_n;
            uint64_t v = in[(size_t)l * N + j];
            if (e >= N) out[(size_t)l * N + (e - N)] = v ? mods[l] - v : 0;
            else out[(size_t)l * N + e] = v;
        }
}

/*
 * HRotate / Conjugate (Table I): phi_g is applied to both halves, the second
 * half is key-switched with the key for g, and out = (phi_g(c0) + k0, k1).
 */
void orc_apply_galois(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                      uint32_t dnum, uint32_t level, const uint64_t *c0, const uint64_t *c1, uint64_t g,
                      const uint64_t *key, uint64_t *out0, uint64_t *out1)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1;
    size_t sz = (size_t)n * N;
    uint64_t *r0 = (uint64_t *)malloc(sz * 8), *r1 = (uint64_t *)malloc(sz * 8), *k0 = (uint64_t *)malloc(sz * 8);
    orc_automorph_eval(logn, n, g, c0, r0);
    orc_automorph_eval(logn, n, g, c1, r1);
    orc_keyswitch(logn, q, nq, p, np, dnum, level, r1, key, k0, out1);
    orc_vec(q, n, logn, r0, k0, out0, 0);
    free(r0); free(r1); free(k0);
}

/*
 * Hoisted rotations (III-F.6): one ModUp of c1 is shared by every Galois
 * element; for each g the automorphism is applied to the extended digits, the
 * inner product is taken with that g's key, ModDown follows, and
 * out_k = (phi_g(c0) + k0, k1).  keys[k] points to a full top-level key,
 * out0/out1 are [count][l+1][N].
 */
void orc_hoisted_rotate(uint32_t logn, const uint64_t *q, uint32_t nq, const uint64_t *p, uint32_t np,
                        uint32_t dnum, uint32_t level, const uint64_t *c0, const uint64_t *c1,
                        uint32_t count, const uint64_t *gs, const uint64_t *const *keys,
                        uint64_t *out0, uint64_t *out1)
{
    uint64_t N = 1ull << logn;
    uint32_t n = level + 1, rows = n + np, alpha = alpha_of(nq, dnum);
    uint32_t beta = (n + alpha - 1) / alpha;
    size_t sz = (size_t)n * N;
    uint64_t *ext = (uint64_t *)malloc((size_t)beta * rows * N * 8);
    uint64_t *acc = (uint64_t *)malloc((size_t)2 * rows * N * 8);
    uint64_t *r0 = (uint64_t *)malloc(sz * 8), *k0 = (uint64_t *)malloc(sz * 8);
    orc_modup(logn, q, nq, p, np, dnum, level, c1, ext);
    for (uint32_t k = 0; k < count; k++) {
        orc_inner_product(logn, q, nq, p, np, dnum, level, ext, keys[k], gs[k], acc);
        orc_moddown(logn, q, nq, p, np, level, acc, k0);
        orc_moddown(logn, q, nq, p, np, level, acc + (size_t)rows * N, out1 + (size_t)k * sz);
        orc_automorph_eval(logn, n, gs[k], c0, r0);
        orc_vec(q, n, logn, r0, k0, out0 + (size_t)k * sz, 0);
    }
    free(ext); free(acc); free(r0); free(k0);
}

/* --------------------------------------------------------- plaintext encoding
 * Residues of integer-valued doubles (the bootstrap planner's plaintext
 * coefficients).  A double v = M 2^e with |M| < 2^53 an integer is reduced as
 * [M]_m [2^e]_m when e > 0, else directly; out[i][k] for modulus mods[i].   */
void orc_reduce_f64(const uint64_t *mods, uint32_t nmods, uint32_t count, const double *x, uint64_t *out)
{
#pragma omp parallel for
    for (uint32_t i = 0; i < nmods; i++) {
        uint64_t m = mods[i];
        for (uint32_t k = 0; k < count; k++) {
            double v = x[k];
            int neg = v < 0;
            double a = neg ? -v : v;
            int e = 0;
            uint64_t r;
            if (a < 9007199254740992.0) {               /* 2^53: an exact integer */
                r = (uint64_t)a % m;
            } else {
                while (a >= 9007199254740992.0) { a *= 0.5; e++; }   /* exact halvings */
                r = mulm((uint64_t)a % m, powm(2, (uint64_t)e, m), m);
            }
            out[(size_t)i * count + k] = neg && r ? m - r : r;
        }
    }
}

/* Thread count of the OpenMP loops (timing of the oracle on 1 or all cores);
 * results do not depend on it. */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
