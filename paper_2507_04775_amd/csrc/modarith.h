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

__host__ __device__ __forceinline__ uint64_t mad32(uint32_t a, uint32_t b, uint64_t c)
{
    return (uint64_t)a * (uint64_t)b + c;  // one v_mad_u64_u32
}

// exact 64x64 -> 128 product from four 32x32 products
__host__ __device__ __forceinline__ u128 mul_wide(uint64_t a, uint64_t b)
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
__host__ __device__ __forceinline__ uint64_t mul_hi(uint64_t a, uint64_t b)
{
    return mul_wide(a, b).hi;
}

__host__ __device__ __forceinline__ u128 add128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
    return r;
}

// Exact sum of products y_i h_i (y_i, h_i < 2^61, fewer than 2^16 terms) with
// h_i wave-uniform, accumulated by 32-bit columns: lo = sum y0 h0,
// mid = sum (y0 h1 + y1 h0), hi = sum y1 h1, and the carries out of lo and mid
// counted from the hardware carry-out of v_mad_u64_u32.  A term costs four
// multiply-adds and three carry additions, where mul_wide + add128 spend
// about twenty instructions (half of them register moves).  hi stays below
// 2^62 (y1, h1 < 2^29), so it needs no carry.  The carry-outs go to separate
// scalar pairs and are read three or more instructions later, after an
// s_nop, which covers the VALU-writes-SGPR read hazard.
struct MacCols {
    uint64_t lo = 0, mid = 0, hi = 0;
    uint32_t clo = 0, cmid = 0;
};

__device__ __forceinline__ void mac_cols(MacCols &c, uint64_t y, uint64_t h)
{
    const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
    const uint32_t h0 = (uint32_t)h, h1 = (uint32_t)(h >> 32);
    uint64_t k0, k1, k2, kd;
    asm("v_mad_u64_u32 %[lo], %[c0], %[y0], %[h0], %[lo]\n\t"
        "v_mad_u64_u32 %[mid], %[c1], %[y0], %[h1], %[mid]\n\t"
        "v_mad_u64_u32 %[mid], %[c2], %[y1], %[h0], %[mid]\n\t"
        "v_mad_u64_u32 %[hi], %[cd], %[y1], %[h1], %[hi]\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32_e64 %[clo], %[cd], 0, %[clo], %[c0]\n\t"
        "v_addc_co_u32_e64 %[cmid], %[cd], 0, %[cmid], %[c1]\n\t"
        "v_addc_co_u32_e64 %[cmid], %[cd], 0, %[cmid], %[c2]"
        : [lo] "+v"(c.lo), [mid] "+v"(c.mid), [hi] "+v"(c.hi), [clo] "+v"(c.clo), [cmid] "+v"(c.cmid),
          [c0] "=&s"(k0), [c1] "=&s"(k1), [c2] "=&s"(k2), [cd] "=&s"(kd)
        : [y0] "v"(y0), [y1] "v"(y1), [h0] "s"(h0), [h1] "s"(h1));
}

// The 128-bit value of the columns: lo + mid 2^32 + (hi + clo) 2^64 + cmid 2^96.
__host__ __device__ __forceinline__ u128 mac_total(const MacCols &c)
{
    u128 r;
    r.lo = c.lo + (c.mid << 32);
    r.hi = c.hi + (c.mid >> 32) + ((uint64_t)c.cmid << 32) + c.clo + (r.lo < c.lo ? 1 : 0);
    return r;
}

// Exact sum of products y_i h_i for constants h_i < 2^50 and inputs y_i < 2^62,
// at most 16 terms.  h is split at bit 27 and y at bit 32, so the four columns
// y0 h0 (< 2^59), y0 h1 (< 2^55), y1 h0 (< 2^57) and y1 h1 (< 2^53) each stay
// below 2^63 over 16 terms: a term is four multiply-adds with no carry to
// count.  The value is c00 + c01 2^27 + c10 2^32 + c11 2^59.  The constant
// arrives split (split_const: h0 in the low word, h1 in the high word), so
// both halves are ready in scalar registers.  On the GPU the four
// multiply-adds of a term go in one block, so consecutive terms interleave
// four independent chains (the carry-outs, always zero here, are discarded).
constexpr uint64_t kSplitMaxConst = 1ull << 50;
constexpr int kSplitShift = 27;

__host__ __device__ __forceinline__ uint64_t split_const(uint64_t h)
{
    return ((h >> kSplitShift) << 32) | (h & ((1ull << kSplitShift) - 1));
}

struct MacSplit {
    uint64_t c00 = 0, c01 = 0, c10 = 0, c11 = 0;

    // y < 2^62; hs = split_const(h) with h < 2^50
    __host__ __device__ __forceinline__ void add(uint64_t y, uint64_t hs)
    {
        const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
        const uint32_t h0 = (uint32_t)hs, h1 = (uint32_t)(hs >> 32);
#if defined(__HIP_DEVICE_COMPILE__)
        uint64_t k;
        asm("v_mad_u64_u32 %[c00], %[k], %[y0], %[h0], %[c00]\n\t"
            "v_mad_u64_u32 %[c01], %[k], %[y0], %[h1], %[c01]\n\t"
            "v_mad_u64_u32 %[c10], %[k], %[y1], %[h0], %[c10]\n\t"
            "v_mad_u64_u32 %[c11], %[k], %[y1], %[h1], %[c11]"
            : [c00] "+v"(c00), [c01] "+v"(c01), [c10] "+v"(c10), [c11] "+v"(c11), [k] "=&s"(k)
            : [y0] "v"(y0), [y1] "v"(y1), [h0] "s"(h0), [h1] "s"(h1));
#else
        c00 = mad32(y0, h0, c00);
        c01 = mad32(y0, h1, c01);
        c10 = mad32(y1, h0, c10);
        c11 = mad32(y1, h1, c11);
#endif
    }
    __host__ __device__ __forceinline__ u128 total() const
    {
        u128 r = {c00, 0};
        r = add128(r, u128{c01 << kSplitShift, c01 >> (64 - kSplitShift)});
        r = add128(r, u128{c10 << 32, c10 >> 32});
        r = add128(r, u128{c11 << (kSplitShift + 32), c11 >> (32 - kSplitShift)});
        return r;
    }
};

// The same interface over mac_cols, for constants up to 2^61.
struct MacColsAcc {
    MacCols c;
    __device__ __forceinline__ void add(uint64_t y, uint64_t h) { mac_cols(c, y, h); }
    __host__ __device__ __forceinline__ u128 total() const { return mac_total(c); }
};

__host__ __device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// Shoup: x * w mod q for any 64-bit x, with ws = floor(w 2^64 / q); result in [0, 2q)
__host__ __device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t ws, uint64_t q)
{
    uint64_t qt = mul_hi(x, ws);
    return x * w - qt * q;
}

__host__ __device__ __forceinline__ uint64_t shoup(uint64_t x, uint64_t w, uint64_t ws, uint64_t q)
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
__host__ __device__ __forceinline__ uint64_t reduce128(u128 z, const Prime &P)
{
    uint64_t a = shoup_lazy(z.hi, P.r64, P.r64_s, P.q);   // [0, 2q)
    uint64_t b = z.lo - mul_hi(z.lo, P.one_s) * P.q;       // [0, 2q)
    uint64_t s = a + b;                                     // [0, 4q)
    s = csub(s, P.two_q);
    return csub(s, P.q);
}

// variable x variable: x, y < 2^64 with x y < 2^128
__host__ __device__ __forceinline__ uint64_t mulmod(uint64_t x, uint64_t y, const Prime &P)
{
    return reduce128(mul_wide(x, y), P);
}

__host__ __device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }

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
__host__ __device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

}  // namespace ckks
