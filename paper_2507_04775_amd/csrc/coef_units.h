// Coefficient-wise units of the key-switching path, shared by the grid and
// persistent kernels (kernels.hip) and the one-launch batch kernel (ntt.hip):
// the fast base conversion (paper Eq. (1), Sec. III-F.3), the key inner
// product (dot-product fusion of III-F.5) and the HMult tensor.  A unit runs
// on kCoefThreads threads, thread `tid` (0 .. kCoefThreads - 1) owning one
// coefficient index of each 256-coefficient block, so every global access is
// a fully coalesced 8-byte-per-lane row segment.  The inner product's staging
// buffer and barriers are the caller's: every thread of the workgroup must
// call the same unit with the same record.
#pragma once
#include "internal.h"

namespace ckks {
namespace coef {

constexpr uint32_t kCoefThreads = 256;

__device__ __forceinline__ uint32_t row_prime(uint32_t r, uint32_t level, uint32_t nq)
{
    return r <= level ? r : nq + (r - level - 1);
}

// Read-only tables read through the scalar cache when the address is uniform.
typedef const __attribute__((address_space(4))) uint64_t ConstU64;

// Conv_{B->C}: y_i = [x_i (B/b_i)^-1]_{b_i} (Shoup; skipped when the inverse
// NTT already produced y_i), then every output row c gets
// [sum_i y_i [B/b_i]_c]_c, accumulated exactly in 128 bits and reduced once
// (as the paper does): by MacSplit's four carry-free columns when the row's
// prime is below 2^50 (its constants stored split), else by mac_cols.  `job` selects the digit (or polynomial),
// `bz` a group of kBconvRowGroup output rows.  The source count NS is a
// template parameter (no predicated iterations), and the constants [B/b_i]_c,
// uniform over the workgroup, come through the scalar cache.
template <class Acc, int NS>
__device__ __forceinline__ uint64_t conv_sum(const uint64_t (&y)[NS], ConstU64 *h, const Prime &P)
{
    Acc acc;
#pragma unroll
    for (int i = 0; i < NS; ++i) acc.add(y[i], h[i]);
    return reduce128(acc.total(), P);
}

template <int NS>
__device__ __forceinline__ void bconv_rows(const BconvArgs &a, const BconvJob &J, uint32_t n, uint32_t r0,
                                           uint32_t r1)
{
    const uint32_t N = a.N;
    uint64_t y[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const uint64_t x = J.src[(size_t)i * N + n];
        if (a.prescaled) {
            y[i] = x;
        } else {
            const ulonglong2 h = J.hinv[i];
            y[i] = shoup(x, h.x, h.y, a.primes[J.src_prime0 + i].q);
        }
    }
    for (uint32_t r = r0; r < r1; ++r) {
        if (r >= J.lo && r < J.hi) {
            if (J.copy_src)
                J.dst[(size_t)r * N + n] =
                    J.copy_src[(size_t)r * N + (a.copy_galois == 1 ? n : galois_src(n, a.copy_galois, a.logn))];
            continue;
        }
        const uint32_t pi = row_prime(r, a.level, a.nq);
        ConstU64 *h = (ConstU64 *)(J.hmod + (size_t)pi * kMaxDigitPrimes);
        const Prime &P = a.primes[pi];
        J.dst[(size_t)r * N + n] = P.q < kSplitMaxConst ? conv_sum<MacSplit, NS>(y, h, P) : conv_sum<MacColsAcc, NS>(y, h, P);
    }
}

__device__ __forceinline__ void bconv_unit(const BconvArgs &a, uint32_t job, uint32_t bx, uint32_t bz, uint32_t tid)
{
    const BconvJob &J = a.job[job];
    const uint32_t n = bx * kCoefThreads + tid;
    const uint32_t r0 = bz * kBconvRowGroup;
    if (r0 >= a.nrows) return;
    const uint32_t r1 = min(r0 + kBconvRowGroup, a.nrows);
    switch (J.ns) {
#define BC_CASE(k) \
    case k: bconv_rows<k>(a, J, n, r0, r1); break;
        BC_CASE(1) BC_CASE(2) BC_CASE(3) BC_CASE(4) BC_CASE(5) BC_CASE(6) BC_CASE(7) BC_CASE(8)
        BC_CASE(9) BC_CASE(10) BC_CASE(11) BC_CASE(12) BC_CASE(13) BC_CASE(14) BC_CASE(15) BC_CASE(16)
#undef BC_CASE
    default: break;
    }
}

// acc[t][r] = sum_j phi_g(ext_j)[r] * key[j][t][r] over the beta digits.
// Under X -> X^g the 256 positions of a block all come from one source block
// (the low bits of the natural index are fixed inside a block of bit-reversed
// positions), so a gathered row is read as one coalesced block into LDS and
// permuted there.  The source blocks of up to kIpStage digits are loaded
// before one barrier, so their load latencies overlap: a barrier per digit
// would expose one HBM round trip per digit and block.
constexpr uint32_t kIpStage = 4;

// Where a unit's two reduced sums go: the accumulator rows by default, or the
// caller's registers (RegStore: the inner product that also runs the first
// inverse pass of ModDown's special rows).
struct AccStore {
    __device__ __forceinline__ void operator()(const IpArgs &a, uint32_t r, uint32_t n, uint64_t v0, uint64_t v1) const
    {
        const size_t N = (size_t)1 << a.logn;
        a.acc[(size_t)r * N + n] = v0;
        a.acc[((size_t)a.rows + r) * N + n] = v1;
    }
};
struct RegStore {
    uint64_t *v0, *v1;
    __device__ __forceinline__ void operator()(const IpArgs &, uint32_t, uint32_t, uint64_t x0, uint64_t x1) const
    {
        *v0 = x0;
        *v1 = x1;
    }
};

// Row r of one key switch's inner product on block bx; stage holds
// kIpStage * kCoefThreads words.
template <class Store = AccStore>
__device__ __forceinline__ void ip_unit(const IpArgs &a, uint32_t r, uint32_t bx, uint64_t *stage, uint32_t tid,
                                        Store store = Store())
{
    const uint32_t N = 1u << a.logn;
    const uint32_t n = bx * kCoefThreads + tid;
    const uint32_t pi = row_prime(r, a.level, a.nq);  // also the key row
    const size_t krows = a.nq + a.np;
    const bool gather = a.galois != 1 || (a.own && a.own_galois != 1);
    u128 s0 = {0, 0}, s1 = {0, 0};
    for (uint32_t j0 = 0; j0 < a.beta; j0 += kIpStage) {
        const uint32_t nj = min(kIpStage, a.beta - j0);
        uint64_t x[kIpStage];
        uint32_t g[kIpStage], sb[kIpStage];
#pragma unroll
        for (uint32_t t = 0; t < kIpStage; ++t) {
            if (t >= nj) break;
            const uint32_t j = j0 + t;
            const bool own = a.own && r >= j * a.alpha && r < min(j * a.alpha + a.alpha, a.level + 1);
            const uint64_t *row = own ? a.own + (size_t)r * N : a.ext + ((size_t)j * a.rows + r) * N;
            g[t] = own ? a.own_galois : a.galois;
            sb[t] = g[t] == 1 ? bx * kCoefThreads : galois_src(bx * kCoefThreads, g[t], a.logn) & ~(uint32_t)(kCoefThreads - 1);
            x[t] = row[sb[t] + tid];
        }
        if (gather) {
            __syncthreads();  // the previous group's permuted reads are done
#pragma unroll
            for (uint32_t t = 0; t < kIpStage; ++t)
                if (t < nj) stage[t * kCoefThreads + tid] = x[t];
            __syncthreads();
#pragma unroll
            for (uint32_t t = 0; t < kIpStage; ++t)
                if (t < nj && g[t] != 1) x[t] = stage[t * kCoefThreads + galois_src(n, g[t], a.logn) - sb[t]];
        }
#pragma unroll
        for (uint32_t t = 0; t < kIpStage; ++t) {
            if (t >= nj) break;
            const uint32_t j = j0 + t;
            const uint64_t k0 = a.key[(((size_t)j * 2 + 0) * krows + pi) * N + n];
            const uint64_t k1 = a.key[(((size_t)j * 2 + 1) * krows + pi) * N + n];
            s0 = add128(s0, mul_wide(x[t], k0));
            s1 = add128(s1, mul_wide(x[t], k1));
        }
    }
    const Prime P = a.primes[pi];
    if (a.fold_tot) {  // a hoisted giant step: add [P]_q phi_g(c0) and accumulate into tot
        if (a.fold_c0 && r <= a.level) {
            const uint32_t g = a.own_galois;
            const uint32_t sb = g == 1 ? bx * kCoefThreads : galois_src(bx * kCoefThreads, g, a.logn) & ~(uint32_t)(kCoefThreads - 1);
            uint64_t x = a.fold_c0[(size_t)r * N + sb + tid];
            if (g != 1) {
                __syncthreads();  // the digits' permuted reads are done
                stage[tid] = x;
                __syncthreads();
                x = stage[galois_src(n, g, a.logn) - sb];
            }
            s0 = add128(s0, mul_wide(x, a.pmod[pi]));
        }
        uint64_t *t0 = a.fold_tot + (size_t)r * N + n, *t1 = a.fold_tot + ((size_t)a.rows + r) * N + n;
        const uint64_t v0 = reduce128(s0, P), v1 = reduce128(s1, P);
        *t0 = a.fold_first ? v0 : addmod(*t0, v0, P.q);
        *t1 = a.fold_first ? v1 : addmod(*t1, v1, P.q);
        return;
    }
    store(a, r, n, reduce128(s0, P), reduce128(s1, P));
}

// Blocks bx0 .. bx0 + nb - 1 of row r, software-pipelined when all digits fit
// one staging group (beta <= kIpStage): the digit and key loads of block i + 1
// are issued before block i's barriers, so a unit exposes one HBM round trip
// instead of one per block.
__device__ __forceinline__ void ip_blocks(const IpArgs &a, uint32_t r, uint32_t bx0, uint32_t nb, uint64_t *stage,
                                          uint32_t tid)
{
    if (a.beta > kIpStage) {
        for (uint32_t i = 0; i < nb; ++i) ip_unit(a, r, bx0 + i, stage, tid);
        return;
    }
    const uint32_t N = 1u << a.logn;
    const uint32_t pi = row_prime(r, a.level, a.nq);
    const size_t krows = a.nq + a.np;
    const bool gather = a.galois != 1 || (a.own && a.own_galois != 1);
    const uint64_t *row[kIpStage];
    uint32_t g[kIpStage];
#pragma unroll
    for (uint32_t j = 0; j < kIpStage; ++j) {
        if (j >= a.beta) break;
        const bool own = a.own && r >= j * a.alpha && r < min(j * a.alpha + a.alpha, a.level + 1);
        row[j] = own ? a.own + (size_t)r * N : a.ext + ((size_t)j * a.rows + r) * N;
        g[j] = own ? a.own_galois : a.galois;
    }
    struct Loaded {
        uint64_t x[kIpStage], k0[kIpStage], k1[kIpStage];
        uint32_t sb[kIpStage];
    };
    auto load = [&](uint32_t bx, Loaded &L) {
        const uint32_t n = bx * kCoefThreads + tid;
#pragma unroll
        for (uint32_t j = 0; j < kIpStage; ++j) {
            if (j >= a.beta) break;
            L.sb[j] = g[j] == 1 ? bx * kCoefThreads : galois_src(bx * kCoefThreads, g[j], a.logn) & ~(uint32_t)(kCoefThreads - 1);
            L.x[j] = row[j][L.sb[j] + tid];
            L.k0[j] = a.key[(((size_t)j * 2 + 0) * krows + pi) * N + n];
            L.k1[j] = a.key[(((size_t)j * 2 + 1) * krows + pi) * N + n];
        }
    };
    const Prime P = a.primes[pi];
    Loaded cur, nxt;
    load(bx0, cur);
    for (uint32_t i = 0; i < nb; ++i) {
        const uint32_t bx = bx0 + i, n = bx * kCoefThreads + tid;
        if (i + 1 < nb) load(bx + 1, nxt);
        if (gather) {
            __syncthreads();  // the previous block's permuted reads are done
#pragma unroll
            for (uint32_t j = 0; j < kIpStage; ++j)
                if (j < a.beta) stage[j * kCoefThreads + tid] = cur.x[j];
            __syncthreads();
#pragma unroll
            for (uint32_t j = 0; j < kIpStage; ++j)
                if (j < a.beta && g[j] != 1) cur.x[j] = stage[j * kCoefThreads + galois_src(n, g[j], a.logn) - cur.sb[j]];
        }
        u128 s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (uint32_t j = 0; j < kIpStage; ++j) {
            if (j >= a.beta) break;
            s0 = add128(s0, mul_wide(cur.x[j], cur.k0[j]));
            s1 = add128(s1, mul_wide(cur.x[j], cur.k1[j]));
        }
        a.acc[(size_t)r * N + n] = reduce128(s0, P);
        a.acc[((size_t)a.rows + r) * N + n] = reduce128(s1, P);
        if (i + 1 < nb) cur = nxt;
    }
}

// Row r of HMult's key inner product with the tensor folded in (IpArgs::ta0
// set; no automorphism).  The key-switched polynomial is d2 = a1 b1: a digit's
// own rows are formed from a1 and b1 here instead of being read from d2, and
// a row under q_r (r <= l) also accumulates [P]_{q_r} d0 into half 0 and
// [P]_{q_r} d1 into half 1, d0 = a0 b0, d1 = a0 b1 + a1 b0, so that ModDown's
// P^-1 (acc - Conv) leaves KS_t + d_t.  At most kMaxDigits + 1 products below
// 2^122 each: the 128-bit sums are exact and reduced once.
template <class Store = AccStore>
__device__ __forceinline__ void ip_unit_tensor(const IpArgs &a, uint32_t r, uint32_t bx, uint32_t tid,
                                               Store store = Store())
{
    const uint32_t N = 1u << a.logn;
    const uint32_t n = bx * kCoefThreads + tid;
    const uint32_t pi = row_prime(r, a.level, a.nq);  // also the key row
    const size_t krows = a.nq + a.np;
    const Prime P = a.primes[pi];
    const bool qrow = r <= a.level;
    uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (qrow) {
        const size_t i = (size_t)r * N + n;
        a0 = a.ta0[i];
        a1 = a.ta1[i];
        b0 = a.tb0[i];
        b1 = a.tb1[i];
    }
    u128 s0 = {0, 0}, s1 = {0, 0};
    for (uint32_t j0 = 0; j0 < a.beta; j0 += kIpStage) {
        uint64_t x[kIpStage], k0[kIpStage], k1[kIpStage];
#pragma unroll
        for (uint32_t t = 0; t < kIpStage; ++t) {
            const uint32_t j = j0 + t;
            if (j >= a.beta) break;
            const bool own = qrow && r >= j * a.alpha && r < min(j * a.alpha + a.alpha, a.level + 1);
            x[t] = own ? 0 : a.ext[((size_t)j * a.rows + r) * N + n];
            k0[t] = a.key[(((size_t)j * 2 + 0) * krows + pi) * N + n];
            k1[t] = a.key[(((size_t)j * 2 + 1) * krows + pi) * N + n];
            if (own) x[t] = reduce128(mul_wide(a1, b1), P);
        }
#pragma unroll
        for (uint32_t t = 0; t < kIpStage; ++t) {
            if (j0 + t >= a.beta) break;
            s0 = add128(s0, mul_wide(x[t], k0[t]));
            s1 = add128(s1, mul_wide(x[t], k1[t]));
        }
    }
    if (qrow) {
        const uint64_t pm = a.pmod[pi];
        const uint64_t d0 = reduce128(mul_wide(a0, b0), P);
        const uint64_t d1 = reduce128(add128(mul_wide(a0, b1), mul_wide(a1, b0)), P);
        s0 = add128(s0, mul_wide(d0, pm));
        s1 = add128(s1, mul_wide(d1, pm));
    }
    store(a, r, n, reduce128(s0, P), reduce128(s1, P));
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 (limb l under q_l)
__device__ __forceinline__ void tensor_unit(const TensorArgs &a, uint32_t l, uint32_t bx, uint32_t tid)
{
    const size_t i = ((size_t)l << a.logn) + bx * kCoefThreads + tid;
    const Prime P = a.primes[l];
    const uint64_t x0 = a.a0[i], x1 = a.a1[i], y0 = a.b0[i], y1 = a.b1[i];
    a.d0[i] = reduce128(mul_wide(x0, y0), P);
    a.d1[i] = reduce128(add128(mul_wide(x0, y1), mul_wide(x1, y0)), P);
    a.d2[i] = reduce128(mul_wide(x1, y1), P);
}


}  // namespace coef
}  // namespace ckks
