// Modular arithmetic on 64-bit words for gfx950, built from 32x32->64
// multiply-adds (v_mad_u64_u32 runs at full rate on CDNA4; there is no
// 64x64->128 instruction).  Methods follow the paper's choice (Table III and
// Sec. III-F.2): Shoup multiplication when one operand is a precomputed
// constant, and a two-step Shoup-style folding of exact 128-bit products when
// both operands vary.  Every modulus is below 2^61, so lazy values up to 4q
// fit a word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

struct u128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ uint64_t mad32(uint32_t a, uint32_t b, uint64_t c)
{
    return (uint64_t)a * (uint64_t)b + c;  // one v_mad_u64_u32
}

// exact 64x64 -> 128 product from four 32x32 products
__device__ __forceinline__ u128 mul_wide(uint64_t a, uint64_t b)
{
    uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    uint64_t p00 = mad32(a0, b0, 0);
    uint64_t p10 = mad32(a1, b0, p00 >> 32);          // < 2^64
    uint64_t p01 = mad32(a0, b1, (uint32_t)p10);      // < 2^64
    uint64_t hi = mad32(a1, b1, (p10 >> 32) + (p01 >> 32));
    u128 r;
    r.lo = (p01 << 32) | (uint32_t)p00;
    r.hi = hi;
    return r;
}

// high 64 bits of a 64x64 product
__device__ __forceinline__ uint64_t mul_hi(uint64_t a, uint64_t b)
{
    return mul_wide(a, b).hi;
}

__device__ __forceinline__ u128 add128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
    return r;
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// Shoup: x * w mod q for any 64-bit x, with ws = floor(w 2^64 / q); result in [0, 2q)
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t ws, uint64_t q)
{
    uint64_t qt = mul_hi(x, ws);
    return x * w - qt * q;
}

__device__ __forceinline__ uint64_t shoup(uint64_t x, uint64_t w, uint64_t ws, uint64_t q)
{
    return csub(shoup_lazy(x, w, ws, q), q);
}

// Per-prime constants needed by the reductions.
struct Prime {
    uint64_t q;
    uint64_t two_q;
    uint64_t r64, r64_s;  // 2^64 mod q and its Shoup companion
    uint64_t one_s;       // floor(2^64 / q): Shoup companion of 1
    uint64_t ninv, ninv_s;  // N^-1 mod q
    double qinv;            // 1/q rounded to double (FP64 path)
};

// Reduce an exact 128-bit value z (any z < 2^128) modulo q:
// z = h 2^64 + l == h (2^64 mod q) + l, both terms folded with Shoup.
__device__ __forceinline__ uint64_t reduce128(u128 z, const Prime &P)
{
    uint64_t a = shoup_lazy(z.hi, P.r64, P.r64_s, P.q);   // [0, 2q)
    uint64_t b = z.lo - mul_hi(z.lo, P.one_s) * P.q;       // [0, 2q)
    uint64_t s = a + b;                                     // [0, 4q)
    s = csub(s, P.two_q);
    return csub(s, P.q);
}

// variable x variable: x, y < 2^64 with x y < 2^128
__device__ __forceinline__ uint64_t mulmod(uint64_t x, uint64_t y, const Prime &P)
{
    return reduce128(mul_wide(x, y), P);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }

// ---------------------------------------------------------------- FP64 path
// For primes below 2^50, residues are exact integers in doubles and a modular
// product is exact through error-free transformations (full-rate FP64 FMA on
// CDNA4).  With u = 2^-53 and |y| <= Y, w in [0, q):
//   h = fl(y w), l = y w - h exactly (FMA), |l| <= u |y w|;
//   k = rint(fl(h fl(1/q))) differs from y w / q by at most 1/2 + 3u |y w| / q;
//   r = (h - k q) + l = y w - k q exactly, since every partial result is an
//   integer of magnitude below 2^53.
// Hence |r| <= (1/2 + 3u Y) q = (1/2 + 0.375 Y / 2^50) q for q < 2^50: the
// result is a centred-ish representative, never canonical; callers keep every
// intermediate below 2^53 in magnitude (see the NTT rounds).
constexpr uint64_t kFpMaxPrime = 1ull << 50;

struct FpMod {
    double q, qinv;
};

__host__ __device__ __forceinline__ double fp_mulmod(double y, double w, FpMod m)
{
    double h = y * w;
    double l = fma(y, w, -h);
    double k = rint(h * m.qinv);
    double r = fma(-k, m.q, h);
    return r + l;
}

// centred reduction: |result| <= q/2 + 1 for |x| < 2^53
__host__ __device__ __forceinline__ double fp_reduce(double x, FpMod m)
{
    double k = rint(x * m.qinv);
    return fma(-k, m.q, x);
}

// canonical residue in [0, q) of an exact integer |x| < 2^53
__host__ __device__ __forceinline__ uint64_t fp_canonical(double x, FpMod m)
{
    double r = fp_reduce(x, m);
    r = r < 0.0 ? r + m.q : r;
    return (uint64_t)r;
}
__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

}  // namespace ckks
