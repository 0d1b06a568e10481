// 32-bit word limbs (the paper's limb type is templated on the word size,
// Sec. III-C; only 64-bit words are verified there): the key-switching path
// with every residue in a 32-bit word, for primes below 2^30 at N = 2^16.
//
// Half the bytes of the 64-bit path per limb, and every modular product is
// native: a twiddle multiplication is Shoup's method on 32-bit words (one
// multiply, one high multiply, one multiply-subtract), the butterflies are
// Harvey's lazy forms ([0, 4q) forward, [0, 2q) inverse, below 2^32 since
// q < 2^30), and sums of products (base conversion, inner product, tensor)
// accumulate exact 64-bit sums reduced once by Barrett.  The same modulus
// budget takes about twice the limbs.
//
// Operations (include/ckks.h, ckks32_*): NTT / INTT, ModUp, ModDown, key
// switching, HMult with relinearisation, Rescale and the Galois automorphism
// with its key switch, all on limb-major [limbs][N] u32 polynomials.
//
// Kernels:
// - NTT passes: N = 2^16 as a 256 x 256 matrix, a column pass (the first
//   eight stages, each column an independent 256-point transform) and a row
//   pass (the last eight), four global accesses per element as in the paper.
//   A workgroup of 512 threads takes 32 columns (rows), 16 threads per column
//   (row) with 16 elements each, in two register rounds of four stages and
//   one exchange through LDS; row passes load and store 16 consecutive words
//   per thread with 128-bit accesses and exchange once more.
// - Base conversion, inner product, tensor, automorphism, lift: one thread
//   per coefficient index of a 256-coefficient block.
// - ModDown's P^-1 (x - Conv(x)) (+ add) and Rescale's q_l^-1 (c - .) run in
//   the store of the last forward pass.
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
}

using namespace ckks;

namespace {

constexpr uint32_t kN = 65536;
constexpr uint32_t kLogN = 16;
constexpr int kT = 512;                 // threads per pass workgroup
constexpr uint32_t kMaxPrimes32 = 64;   // q and p together
constexpr uint32_t kMaxRows32 = 64;     // rows of one polynomial in a launch (l + 1 + K)
constexpr uint32_t kMaxLaunch32 = 256;  // rows of one launch (polynomials x rows)
constexpr uint32_t kMaxDigit32 = 16;    // primes per digit and in the special basis
constexpr uint32_t kQBound = 1u << 30;

struct Pair32 {
    uint32_t w, s;  // a constant and its Shoup companion floor(w 2^32 / q)
};

struct Prime32 {
    uint32_t q, pad;
    uint64_t mu;  // floor(2^64 / q), for Barrett reduction of 64-bit sums
};

// -------------------------------------------------------- modular arithmetic

__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t q) { return x >= q ? x - q : x; }

// w y - floor(ws y / 2^32) q: in [0, 2q) for every y < 2^32 (Shoup)
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t y, Pair32 w, uint32_t q)
{
    return w.w * y - __umulhi(w.s, y) * q;
}

__device__ __forceinline__ uint32_t shoup(uint32_t y, Pair32 w, uint32_t q) { return csub(shoup_lazy(y, w, q), q); }

// x mod q for any 64-bit x: x - floor(x mu / 2^64) q is in [0, 2q) (Barrett with mu = floor(2^64 / q))
__device__ __forceinline__ uint32_t reduce64(uint64_t x, const Prime32 &P)
{
    const uint64_t r = x - __umul64hi(x, P.mu) * P.q;
    return csub((uint32_t)r, P.q);
}

__device__ __forceinline__ uint64_t mul32(uint32_t a, uint32_t b) { return (uint64_t)a * b; }

// ------------------------------------------------------------- NTT passes

// Launch row y = poly * rows + r: polynomial `poly`, row r under prime
// prime[r]; rows whose bit is set in skip are left alone.
struct Ntt32Args {
    const uint32_t *src;
    uint32_t *dst;              // pass 0 writes here, pass 1 transforms it in place
    int64_t src_poly_stride, dst_poly_stride;
    uint32_t rows, npoly;
    const Prime32 *primes;
    const Pair32 *tw;           // [n_primes][N]: psi^(+-br(i))
    // last inverse multiplication (N^-1, times a conversion scale) per row r
    Pair32 scale[kMaxRows32];
    // forward epilogue: 0 plain; 1 ModDown out_p = cst (aux_p - x) + add_p; 2 Rescale out_p = cst (aux_p - x)
    uint32_t epi;
    const uint32_t *aux[2];
    const uint32_t *add[2];
    uint32_t *out[2];
    const Pair32 *cst;          // per prime index
    uint32_t skip[kMaxLaunch32 / 32];
    uint8_t prime[kMaxRows32];
};

struct RowPos {
    uint32_t poly, r, pi;
    bool skip;
};

__device__ __forceinline__ RowPos row_pos(const Ntt32Args &a, uint32_t y)
{
    RowPos p;
    p.poly = y / a.rows;
    p.r = y - p.poly * a.rows;
    p.pi = a.prime[p.r];
    p.skip = (a.skip[y >> 5] >> (y & 31)) & 1;
    return p;
}

// Stage k (0..7) of a 256-point transform on element e of block B: the
// butterfly's twiddle is T[(B << k) + (e >> (8 - k))] (B = 1 for the column
// pass, 256 + row for the row pass), its partner e + (128 >> k).
__device__ __forceinline__ Pair32 twk(const Pair32 *T, uint32_t B, int k, uint32_t e)
{
    return T[(B << k) + (e >> (8 - k))];
}

// Four forward (Cooley-Tukey) stages k0..k0+3 on v[i], element e(i) =
// base + stride i, partners i + (8 >> (k - k0)).  Values stay in [0, 4q).
template <class E>
__device__ __forceinline__ void fwd4(uint32_t (&v)[16], const Pair32 *T, uint32_t B, int k0, uint32_t q, E e)
{
    const uint32_t q2 = 2 * q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int h = 8 >> st;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i & h) continue;
            const Pair32 w = twk(T, B, k0 + st, e(i));
            const uint32_t x = v[i] >= q2 ? v[i] - q2 : v[i];
            const uint32_t t = shoup_lazy(v[i + h], w, q);
            v[i] = x + t;
            v[i + h] = x - t + q2;
        }
    }
}

// Four inverse (Gentleman-Sande) stages k0, k0-1, .., k0-3, partners i + (1 << st).
// Values stay in [0, 2q).
template <class E>
__device__ __forceinline__ void inv4(uint32_t (&v)[16], const Pair32 *T, uint32_t B, int k0, uint32_t q, E e)
{
    const uint32_t q2 = 2 * q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int h = 1 << st;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i & h) continue;
            const Pair32 w = twk(T, B, k0 - st, e(i));
            const uint32_t x = v[i], y = v[i + h];
            const uint32_t s = x + y;
            v[i] = s >= q2 ? s - q2 : s;
            v[i + h] = shoup_lazy(x - y + q2, w, q);
        }
    }
}

constexpr uint32_t kColStride = 33;               // LDS words per matrix row in a column pass (32 + 1)
constexpr uint32_t kRowStride = 256 + 16;         // LDS words per row in a row pass
__device__ __forceinline__ uint32_t rslot(uint32_t e) { return e + (e >> 4); }  // conflict-free both ways
constexpr uint32_t kLds32 = 256 * kColStride > 32 * kRowStride ? 256 * kColStride : 32 * kRowStride;

// Forward column pass: 32 columns per workgroup; round 1 on rows s + 16 i,
// round 2 on rows 16 s + i.
__global__ __launch_bounds__(kT) void k32_fwd_col(Ntt32Args a)
{
    __shared__ uint32_t L[kLds32];
    const RowPos p = row_pos(a, blockIdx.y);
    if (p.skip) return;
    const uint32_t q = a.primes[p.pi].q;
    const Pair32 *T = a.tw + (size_t)p.pi * kN;
    const uint32_t col = threadIdx.x & 31, s = threadIdx.x >> 5, c = blockIdx.x * 32 + col;
    const uint32_t *src = a.src + p.poly * a.src_poly_stride + (size_t)p.r * kN;
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = src[(s + 16 * i) * 256 + c];
    fwd4(v, T, 1, 0, q, [&](int i) { return s + 16 * i; });
#pragma unroll
    for (int i = 0; i < 16; ++i) L[(s + 16 * i) * kColStride + col] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[(16 * s + i) * kColStride + col];
    fwd4(v, T, 1, 4, q, [&](int i) { return 16 * s + i; });
    uint32_t *dst = a.dst + p.poly * a.dst_poly_stride + (size_t)p.r * kN;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[(16 * s + i) * 256 + c] = v[i];
}

__device__ __forceinline__ void load16(uint32_t (&v)[16], const uint32_t *m)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint4 x = ((const uint4 *)m)[j];
        v[4 * j] = x.x;
        v[4 * j + 1] = x.y;
        v[4 * j + 2] = x.z;
        v[4 * j + 3] = x.w;
    }
}

__device__ __forceinline__ void store16(uint32_t *m, const uint32_t (&v)[16])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) ((uint4 *)m)[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
}

// Forward row pass: 32 rows per workgroup, 16 threads per row.  Loaded as 16
// consecutive words per thread, exchanged to e = s + 16 i for round 1, back to
// e = 16 s + i for round 2 and the store (with the epilogue).
__global__ __launch_bounds__(kT) void k32_fwd_row(Ntt32Args a)
{
    __shared__ uint32_t L[kLds32];
    const RowPos p = row_pos(a, blockIdx.y);
    if (p.skip) return;
    const Prime32 P = a.primes[p.pi];
    const uint32_t q = P.q;
    const Pair32 *T = a.tw + (size_t)p.pi * kN;
    const uint32_t rw = threadIdx.x >> 4, s = threadIdx.x & 15, b = blockIdx.x * 32 + rw;
    uint32_t *m = a.dst + p.poly * a.dst_poly_stride + (size_t)p.r * kN + b * 256;
    uint32_t *Lr = L + rw * kRowStride;
    uint32_t v[16];
    load16(v, m + 16 * s);
#pragma unroll
    for (int i = 0; i < 16; ++i) Lr[rslot(16 * s + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = Lr[rslot(s + 16 * i)];
    fwd4(v, T, 256 + b, 0, q, [&](int i) { return s + 16 * i; });
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) Lr[rslot(s + 16 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = Lr[rslot(16 * s + i)];
    fwd4(v, T, 256 + b, 4, q, [&](int i) { return 16 * s + i; });
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = csub(csub(v[i], 2 * q), q);
    const size_t off = (size_t)p.r * kN + b * 256 + 16 * s;
    if (a.epi == 0) {
        store16(m + 16 * s, v);
        return;
    }
    const Pair32 c = a.cst[p.pi];
    uint32_t x[16], o[16];
    load16(x, (p.poly ? a.aux[1] : a.aux[0]) + off);
#pragma unroll
    for (int i = 0; i < 16; ++i) o[i] = shoup(x[i] - v[i] + q, c, q);
    const uint32_t *add = p.poly ? a.add[1] : a.add[0];
    if (a.epi == 1 && add) {
        load16(x, add + off);
#pragma unroll
        for (int i = 0; i < 16; ++i) o[i] = csub(o[i] + x[i], q);
    }
    store16((p.poly ? a.out[1] : a.out[0]) + off, o);
}

// Inverse row pass: round 1 (stages 7..4) on e = 16 s + i as loaded, round 2
// (stages 3..0) on e = s + 16 i; stored from that layout.
__global__ __launch_bounds__(kT) void k32_inv_row(Ntt32Args a)
{
    __shared__ uint32_t L[kLds32];
    const RowPos p = row_pos(a, blockIdx.y);
    if (p.skip) return;
    const uint32_t q = a.primes[p.pi].q;
    const Pair32 *T = a.tw + (size_t)p.pi * kN;
    const uint32_t rw = threadIdx.x >> 4, s = threadIdx.x & 15, b = blockIdx.x * 32 + rw;
    const uint32_t *m = a.src + p.poly * a.src_poly_stride + (size_t)p.r * kN + b * 256;
    uint32_t *Lr = L + rw * kRowStride;
    uint32_t v[16];
    load16(v, m + 16 * s);
    inv4(v, T, 256 + b, 7, q, [&](int i) { return 16 * s + i; });
#pragma unroll
    for (int i = 0; i < 16; ++i) Lr[rslot(16 * s + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = Lr[rslot(s + 16 * i)];
    inv4(v, T, 256 + b, 3, q, [&](int i) { return s + 16 * i; });
    uint32_t *d = a.dst + p.poly * a.dst_poly_stride + (size_t)p.r * kN + b * 256;
#pragma unroll
    for (int i = 0; i < 16; ++i) d[s + 16 * i] = v[i];
}

// Inverse column pass: round 1 (stages 7..4) on rows 16 s + i, round 2 (3..0)
// on rows s + 16 i, then the last multiplication (N^-1 and the row's scale).
__global__ __launch_bounds__(kT) void k32_inv_col(Ntt32Args a)
{
    __shared__ uint32_t L[kLds32];
    const RowPos p = row_pos(a, blockIdx.y);
    if (p.skip) return;
    const uint32_t q = a.primes[p.pi].q;
    const Pair32 *T = a.tw + (size_t)p.pi * kN;
    const uint32_t col = threadIdx.x & 31, s = threadIdx.x >> 5, c = blockIdx.x * 32 + col;
    uint32_t *d = a.dst + p.poly * a.dst_poly_stride + (size_t)p.r * kN;
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = d[(16 * s + i) * 256 + c];
    inv4(v, T, 1, 7, q, [&](int i) { return 16 * s + i; });
#pragma unroll
    for (int i = 0; i < 16; ++i) L[(16 * s + i) * kColStride + col] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[(s + 16 * i) * kColStride + col];
    inv4(v, T, 1, 3, q, [&](int i) { return s + 16 * i; });
    const Pair32 f = a.scale[p.r];
#pragma unroll
    for (int i = 0; i < 16; ++i) d[(s + 16 * i) * 256 + c] = shoup(v[i], f, q);
}

// ----------------------------------------------------- coefficient kernels

constexpr int kB = 256;

// Fast base conversion (Eq. (1)) of job j = blockIdx.y: y_i = src row i (already
// scaled by [(B/b_i)^-1]_{b_i} in the inverse NTT), out row c = [sum_i y_i [B/b_i]_c]_c
// for the rows c outside [lo, hi), in groups of 8 rows (blockIdx.z).  With
// centred, every y_i above (b_i - 1)/2 stands for y_i - b_i: the sum gains
// h (q_c - [B]_{q_c}) for the h such inputs.
struct Bconv32Job {
    const uint32_t *src;
    uint32_t *dst;
    const uint32_t *hmod;       // [prime][kMaxDigit32]: [B/b_i]_{prime}
    uint32_t ns, lo, hi, pad;
    uint32_t half[kMaxDigit32]; // (b_i - 1) / 2
};

struct Bconv32Args {
    Bconv32Job job[kMaxDigit32];
    const Prime32 *primes;
    const uint32_t *bmod;       // centred: [prime] B mod q
    uint32_t nrows, centred;
    uint8_t prime[kMaxRows32];
};

__global__ __launch_bounds__(kB) void k32_bconv(Bconv32Args a)
{
    const Bconv32Job &J = a.job[blockIdx.y];
    const uint32_t n = blockIdx.x * kB + threadIdx.x, r0 = blockIdx.z * 8;
    if (r0 >= a.nrows) return;
    uint32_t y[kMaxDigit32];
    uint32_t h = 0;
    for (uint32_t i = 0; i < J.ns; ++i) {
        y[i] = J.src[(size_t)i * kN + n];
        h += y[i] > J.half[i];
    }
    const uint32_t r1 = min(r0 + 8, a.nrows);
    for (uint32_t r = r0; r < r1; ++r) {
        if (r >= J.lo && r < J.hi) continue;
        const uint32_t pi = a.prime[r];
        const Prime32 P = a.primes[pi];
        const uint32_t *hm = J.hmod + (size_t)pi * kMaxDigit32;
        uint64_t acc = a.centred ? (uint64_t)h * (P.q - a.bmod[pi]) : 0;
        for (uint32_t i = 0; i < J.ns; ++i) acc += mul32(y[i], hm[i]);
        J.dst[(size_t)r * kN + n] = reduce64(acc, P);
    }
}

// Key inner product: acc_t[r] = sum_j x_j[r] key[j][t][prime(r)], x_j[r] = d[r]
// for the digit's own rows (d at level l, evaluation domain), ext_j[r] else.
struct Ip32Args {
    const uint32_t *ext, *d, *key;
    uint32_t *acc;
    const Prime32 *primes;
    uint32_t beta, rows, n, alpha, krows, pad;
    uint8_t prime[kMaxRows32];
};

__global__ __launch_bounds__(kB) void k32_inner_product(Ip32Args a)
{
    const uint32_t n = blockIdx.x * kB + threadIdx.x, r = blockIdx.y, pi = a.prime[r];
    uint64_t s0 = 0, s1 = 0;
    for (uint32_t j = 0; j < a.beta; ++j) {
        const bool own = r < a.n && r >= j * a.alpha && r < j * a.alpha + a.alpha;
        const uint32_t x = own ? a.d[(size_t)r * kN + n] : a.ext[((size_t)j * a.rows + r) * kN + n];
        s0 += mul32(x, a.key[(((size_t)j * 2 + 0) * a.krows + pi) * kN + n]);
        s1 += mul32(x, a.key[(((size_t)j * 2 + 1) * a.krows + pi) * kN + n]);
    }
    const Prime32 P = a.primes[pi];
    a.acc[(size_t)r * kN + n] = reduce64(s0, P);
    a.acc[((size_t)a.rows + r) * kN + n] = reduce64(s1, P);
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 on limb blockIdx.y (prime index = limb)
__global__ __launch_bounds__(kB) void k32_tensor(const uint32_t *a0, const uint32_t *a1, const uint32_t *b0,
                                                 const uint32_t *b1, uint32_t *d0, uint32_t *d1, uint32_t *d2,
                                                 const Prime32 *primes)
{
    const size_t i = (size_t)blockIdx.y * kN + blockIdx.x * kB + threadIdx.x;
    const Prime32 P = primes[blockIdx.y];
    const uint32_t x0 = a0[i], x1 = a1[i], y0 = b0[i], y1 = b1[i];
    d0[i] = reduce64(mul32(x0, y0), P);
    d1[i] = reduce64(mul32(x0, y1) + mul32(x1, y0), P);
    d2[i] = reduce64(mul32(x1, y1), P);
}

// out[limb][e] = in[limb][src of e under X -> X^g] (evaluation domain)
__global__ __launch_bounds__(kB) void k32_automorph(const uint32_t *in, uint32_t *out, uint32_t g)
{
    const uint32_t e = blockIdx.x * kB + threadIdx.x;
    const size_t row = (size_t)blockIdx.y * kN;
    out[row + e] = in[row + galois_src(e, g, kLogN)];
}

// Rescale's SwitchModulo: v (coefficients under q_l, [2][N]) lifted centred
// into q_i for the l limbs i < l of both halves: out[t][i] = v_t - q_l [v_t > (q_l-1)/2] mod q_i
__global__ __launch_bounds__(kB) void k32_lift(const uint32_t *v, uint32_t *out, const Prime32 *primes,
                                               const uint32_t *qlmod, uint32_t ql, uint32_t l)
{
    const uint32_t n = blockIdx.x * kB + threadIdx.x, i = blockIdx.y, t = blockIdx.z;
    const uint32_t u = v[(size_t)t * kN + n], q = primes[i].q;
    const uint32_t um = u % q;  // u < 2^30
    const uint32_t r = u <= (ql - 1) / 2 ? um : csub(um + q - qlmod[i], q);
    out[((size_t)t * l + i) * kN + n] = r;
}

}  // namespace

// --------------------------------------------------------------- host side

struct ckks32_ctx {
    int device = 0;
    uint32_t nq = 0, np = 0, dnum = 0, alpha = 0;
    std::vector<uint32_t> primes;  // q_0..q_L, p_0..p_{K-1}
    void *dev = nullptr;
    Prime32 *d_primes = nullptr;
    Pair32 *d_tw_fwd = nullptr, *d_tw_inv = nullptr;
    uint32_t *d_hmod = nullptr;    // [nsets][n_primes][kMaxDigit32]
    uint32_t *d_pmod = nullptr;    // [n_primes]: P mod prime
    Pair32 *d_pinv = nullptr;      // [n_primes]: P^-1 mod q_i
    Pair32 *d_qlinv = nullptr;     // [nq][nq]: (l, i) -> q_l^-1 mod q_i
    uint32_t *d_qlmod = nullptr;   // [nq][nq]: (l, i) -> q_l mod q_i
    // host copies of per-set constants
    std::vector<Pair32> ys;        // [nsets][kMaxDigit32]: N^-1 [(B/b_i)^-1]_{b_i}
    std::vector<Pair32> ninv;      // [n_primes]
    std::vector<Pair32> qlinv;     // [nq][nq]
    uint32_t nsets = 0;
    uint32_t set_index(uint32_t digit, uint32_t size) const { return digit * alpha + size - 1; }
    uint32_t pset() const { return dnum * alpha; }
};

namespace {

#define TRY32(x)                        \
    do {                                \
        ckks_status _s = (x);           \
        if (_s != CKKS_OK) return _s;   \
    } while (0)

Pair32 pair32(uint64_t w, uint64_t q)
{
    Pair32 p;
    p.w = (uint32_t)w;
    p.s = (uint32_t)((w << 32) / q);
    return p;
}

ckks_status dev32(hipError_t e, const char *what)
{
    if (e == hipSuccess) return CKKS_OK;
    return fail(CKKS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Sizes32 {
    uint32_t n, rows, beta;
};

Sizes32 sizes(const ckks32_ctx *c, uint32_t level)
{
    Sizes32 s;
    s.n = level + 1;
    s.rows = s.n + c->np;
    s.beta = (s.n + c->alpha - 1) / c->alpha;
    return s;
}

// prime index of row r of an extended polynomial at `level`
uint32_t ext_prime(const ckks32_ctx *c, uint32_t level, uint32_t r) { return r <= level ? r : c->nq + r - level - 1; }

Ntt32Args base_args(const ckks32_ctx *c, bool inverse)
{
    Ntt32Args a;
    memset(&a, 0, sizeof(a));
    a.primes = c->d_primes;
    a.tw = inverse ? c->d_tw_inv : c->d_tw_fwd;
    return a;
}

hipError_t launch_ntt32(const Ntt32Args &a, bool inverse, hipStream_t st)
{
    const uint32_t ny = a.npoly * a.rows;
    if (ny == 0) return hipSuccess;
    if (ny > kMaxLaunch32 || a.rows > kMaxRows32) return hipErrorInvalidValue;
    const dim3 grid(8, ny), block(kT);
    if (inverse) {
        hipLaunchKernelGGL(k32_inv_row, grid, block, 0, st, a);
        hipLaunchKernelGGL(k32_inv_col, grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL(k32_fwd_col, grid, block, 0, st, a);
        hipLaunchKernelGGL(k32_fwd_row, grid, block, 0, st, a);
    }
    return hipGetLastError();
}

ckks_status check_ptr32(const void *p, const char *what)
{
    if (!p || ((uintptr_t)p & 15)) return fail(CKKS_E_ARG, std::string(what) + ": null or not 16-byte aligned");
    return CKKS_OK;
}

// Workspace layout of a key switch at `level` (words): dc [n], ext [beta][rows],
// acc [2][rows], pc [2][K], conv [2][n].
struct Ws32 {
    uint32_t *dc, *ext, *acc, *pc, *conv;
};

size_t ks_words(const ckks32_ctx *c, uint32_t level)
{
    const Sizes32 s = sizes(c, level);
    return ((size_t)s.n + (size_t)s.beta * s.rows + 2 * (size_t)s.rows + 2 * (size_t)c->np + 2 * (size_t)s.n) * kN;
}

size_t ks_bytes(const ckks32_ctx *c, uint32_t level) { return align256(ks_words(c, level) * 4); }

Ws32 ks_ws(const ckks32_ctx *c, uint32_t level, void *ws)
{
    const Sizes32 s = sizes(c, level);
    Ws32 w;
    w.dc = (uint32_t *)ws;
    w.ext = w.dc + (size_t)s.n * kN;
    w.acc = w.ext + (size_t)s.beta * s.rows * kN;
    w.pc = w.acc + 2 * (size_t)s.rows * kN;
    w.conv = w.pc + 2 * (size_t)c->np * kN;
    return w;
}

hipError_t launch_bconv32(const Bconv32Args &a, uint32_t njobs, hipStream_t st)
{
    static_assert(sizeof(Bconv32Args) <= 4096, "the conversion's argument block is a kernel argument");
    hipLaunchKernelGGL(k32_bconv, dim3(kN / kB, njobs, (a.nrows + 7) / 8), dim3(kB), 0, st, a);
    return hipGetLastError();
}

// ModUp of d (evaluation domain, level l) into ext (evaluation domain, the
// digits' own rows left out: the inner product reads them from d).
hipError_t modup32(const ckks32_ctx *c, const uint32_t *d, uint32_t level, const Ws32 &w, hipStream_t st)
{
    const Sizes32 s = sizes(c, level);
    Ntt32Args ia = base_args(c, true);
    ia.src = d;
    ia.dst = w.dc;
    ia.rows = s.n;
    ia.npoly = 1;
    for (uint32_t i = 0; i < s.n; ++i) {
        const uint32_t j = i / c->alpha, lo = j * c->alpha, hi = std::min(lo + c->alpha, s.n);
        ia.prime[i] = (uint8_t)i;
        ia.scale[i] = c->ys[(size_t)c->set_index(j, hi - lo) * kMaxDigit32 + (i - lo)];
    }
    hipError_t e = launch_ntt32(ia, true, st);
    if (e != hipSuccess) return e;
    Bconv32Args bh;
    memset(&bh, 0, sizeof(bh));
    bh.primes = c->d_primes;
    bh.nrows = s.rows;
    const size_t hstride = (size_t)(c->nq + c->np) * kMaxDigit32;
    for (uint32_t r = 0; r < s.rows; ++r) bh.prime[r] = (uint8_t)ext_prime(c, level, r);
    for (uint32_t j = 0; j < s.beta; ++j) {
        const uint32_t lo = j * c->alpha, hi = std::min(lo + c->alpha, s.n);
        Bconv32Job &J = bh.job[j];
        J.src = w.dc + (size_t)lo * kN;
        J.dst = w.ext + (size_t)j * s.rows * kN;
        J.hmod = c->d_hmod + (size_t)c->set_index(j, hi - lo) * hstride;
        J.ns = hi - lo;
        J.lo = lo;
        J.hi = hi;
        for (uint32_t i = 0; i < J.ns; ++i) J.half[i] = 0xFFFFFFFFu;  // not centred
    }
    e = launch_bconv32(bh, s.beta, st);
    if (e != hipSuccess) return e;
    Ntt32Args fa = base_args(c, false);
    fa.src = fa.dst = w.ext;
    fa.src_poly_stride = fa.dst_poly_stride = (int64_t)s.rows * kN;
    fa.rows = s.rows;
    fa.npoly = s.beta;
    for (uint32_t r = 0; r < s.rows; ++r) fa.prime[r] = (uint8_t)ext_prime(c, level, r);
    for (uint32_t j = 0; j < s.beta; ++j)
        for (uint32_t r = j * c->alpha; r < std::min(j * c->alpha + c->alpha, s.n); ++r) {
            const uint32_t y = j * s.rows + r;
            fa.skip[y >> 5] |= 1u << (y & 31);
        }
    return launch_ntt32(fa, false, st);
}

// ModDown of the pair acc [2][rows] into out_t = P^-1 (acc_t - Conv(acc_t|P)) + add_t.
hipError_t moddown32(const ckks32_ctx *c, const uint32_t *acc, uint32_t level, const Ws32 &w, uint32_t *out0,
                     uint32_t *out1, const uint32_t *add0, const uint32_t *add1, hipStream_t st)
{
    const Sizes32 s = sizes(c, level);
    const uint32_t K = c->np;
    Ntt32Args ia = base_args(c, true);
    ia.src = acc + (size_t)s.n * kN;
    ia.dst = w.pc;
    ia.src_poly_stride = (int64_t)s.rows * kN;
    ia.dst_poly_stride = (int64_t)K * kN;
    ia.rows = K;
    ia.npoly = 2;
    for (uint32_t k = 0; k < K; ++k) {
        ia.prime[k] = (uint8_t)(c->nq + k);
        ia.scale[k] = c->ys[(size_t)c->pset() * kMaxDigit32 + k];
    }
    hipError_t e = launch_ntt32(ia, true, st);
    if (e != hipSuccess) return e;
    Bconv32Args bh;
    memset(&bh, 0, sizeof(bh));
    bh.primes = c->d_primes;
    bh.bmod = c->d_pmod;
    bh.centred = 1;
    bh.nrows = s.n;
    for (uint32_t r = 0; r < s.n; ++r) bh.prime[r] = (uint8_t)r;
    const size_t hstride = (size_t)(c->nq + c->np) * kMaxDigit32;
    for (uint32_t t = 0; t < 2; ++t) {
        Bconv32Job &J = bh.job[t];
        J.src = w.pc + (size_t)t * K * kN;
        J.dst = w.conv + (size_t)t * s.n * kN;
        J.hmod = c->d_hmod + (size_t)c->pset() * hstride;
        J.ns = K;
        J.lo = J.hi = 0xFFFFFFFFu;
        for (uint32_t k = 0; k < K; ++k) J.half[k] = (c->primes[c->nq + k] - 1) / 2;
    }
    e = launch_bconv32(bh, 2, st);
    if (e != hipSuccess) return e;
    Ntt32Args fa = base_args(c, false);
    fa.src = fa.dst = w.conv;
    fa.src_poly_stride = fa.dst_poly_stride = (int64_t)s.n * kN;
    fa.rows = s.n;
    fa.npoly = 2;
    for (uint32_t r = 0; r < s.n; ++r) fa.prime[r] = (uint8_t)r;
    fa.epi = 1;
    fa.aux[0] = acc;
    fa.aux[1] = acc + (size_t)s.rows * kN;
    fa.add[0] = add0;
    fa.add[1] = add1;
    fa.out[0] = out0;
    fa.out[1] = out1;
    fa.cst = c->d_pinv;
    return launch_ntt32(fa, false, st);
}

hipError_t inner_product32(const ckks32_ctx *c, const uint32_t *d, uint32_t level, const uint32_t *key,
                           const Ws32 &w, hipStream_t st)
{
    const Sizes32 s = sizes(c, level);
    Ip32Args a;
    memset(&a, 0, sizeof(a));
    a.ext = w.ext;
    a.d = d;
    a.key = key;
    a.acc = w.acc;
    a.primes = c->d_primes;
    a.beta = s.beta;
    a.rows = s.rows;
    a.n = s.n;
    a.alpha = c->alpha;
    a.krows = c->nq + c->np;
    for (uint32_t r = 0; r < s.rows; ++r) a.prime[r] = (uint8_t)ext_prime(c, level, r);
    hipLaunchKernelGGL(k32_inner_product, dim3(kN / kB, s.rows), dim3(kB), 0, st, a);
    return hipGetLastError();
}

hipError_t keyswitch32(ckks32_ctx *c, const uint32_t *d, uint32_t level, const uint32_t *key, uint32_t *out0,
                       uint32_t *out1, const uint32_t *add0, const uint32_t *add1, void *ws, hipStream_t st)
{
    const Ws32 w = ks_ws(c, level, ws);
    hipError_t e = modup32(c, d, level, w, st);
    if (e == hipSuccess) e = inner_product32(c, d, level, key, w, st);
    if (e == hipSuccess) e = moddown32(c, w.acc, level, w, out0, out1, add0, add1, st);
    return e;
}

ckks_status check_ctx32(const ckks32_ctx *c, uint32_t level)
{
    if (!c) return fail(CKKS_E_ARG, "ckks32: null context");
    if (level >= c->nq) return fail(CKKS_E_LEVEL, "ckks32: level " + std::to_string(level) + " out of range");
    return CKKS_OK;
}

}  // namespace

extern "C" ckks_status ckks32_ctx_create(uint32_t log_n, const uint32_t *q, uint32_t n_q, const uint32_t *p,
                                         uint32_t n_p, uint32_t dnum, int hip_device, ckks32_ctx **out)
{
    if (!out || !q || !p) return fail(CKKS_E_ARG, "ckks32_ctx_create: null pointer");
    *out = nullptr;
    if (log_n != kLogN) return fail(CKKS_E_UNSUPPORTED, "ckks32_ctx_create: log_n must be 16");
    if (n_q < 1 || n_p < 1 || dnum < 1 || dnum > n_q)
        return fail(CKKS_E_ARG, "ckks32_ctx_create: need n_q >= 1, n_p >= 1, 1 <= dnum <= n_q");
    const uint32_t alpha = (n_q + dnum - 1) / dnum;
    if (n_q + n_p > kMaxPrimes32 || alpha > kMaxDigit32 || n_p > kMaxDigit32 || dnum > kMaxDigit32 ||
        n_q + n_p > kMaxRows32)
        return fail(CKKS_E_UNSUPPORTED, "ckks32_ctx_create: at most 64 primes, 16 per digit, 16 special, 16 digits");
    std::vector<uint32_t> primes(q, q + n_q);
    primes.insert(primes.end(), p, p + n_p);
    const uint64_t N = kN, two_n = 2 * N;
    for (size_t i = 0; i < primes.size(); ++i) {
        const uint64_t m = primes[i];
        if (m >= kQBound || m % two_n != 1 || !probably_prime(m))
            return fail(CKKS_E_ARG, "ckks32_ctx_create: prime " + std::to_string(i) +
                                        " is not a prime below 2^30 congruent to 1 mod 2N");
        for (size_t k = 0; k < i; ++k)
            if (primes[k] == m) return fail(CKKS_E_ARG, "ckks32_ctx_create: primes must be distinct");
    }
    if (hipSetDevice(hip_device) != hipSuccess) return fail(CKKS_E_DEVICE, "ckks32_ctx_create: hipSetDevice failed");
    ckks32_ctx *c = new ckks32_ctx();
    c->device = hip_device;
    c->nq = n_q;
    c->np = n_p;
    c->dnum = dnum;
    c->alpha = alpha;
    c->primes = primes;
    const uint32_t np_all = n_q + n_p;
    c->nsets = dnum * alpha + 1;

    std::vector<Prime32> pr(np_all);
    std::vector<Pair32> twf((size_t)np_all * N), twi((size_t)np_all * N);
    c->ninv.resize(np_all);
    for (uint32_t i = 0; i < np_all; ++i) {
        const uint64_t m = primes[i];
        pr[i].q = (uint32_t)m;
        pr[i].pad = 0;
        pr[i].mu = (uint64_t)((((unsigned __int128)1) << 64) / m);
        const uint64_t psi = smallest_2n_root(m, two_n), psi_inv = inv_mod(psi, m);
        uint64_t a = 1, b = 1;
        std::vector<uint64_t> pw(N), pwi(N);
        for (uint64_t k = 0; k < N; ++k, a = mul_mod(a, psi, m), b = mul_mod(b, psi_inv, m)) {
            pw[k] = a;
            pwi[k] = b;
        }
        for (uint32_t k = 0; k < N; ++k) {
            const uint32_t e = reverse_bits(k, kLogN);
            twf[(size_t)i * N + k] = pair32(pw[e], m);
            twi[(size_t)i * N + k] = pair32(pwi[e], m);
        }
        c->ninv[i] = pair32(inv_mod(N % m, m), m);
    }
    // conversion constants: digit sets (j, size) and the special basis
    std::vector<uint32_t> hmod((size_t)c->nsets * np_all * kMaxDigit32, 0);
    c->ys.assign((size_t)c->nsets * kMaxDigit32, Pair32{0, 0});
    auto fill_set = [&](uint32_t set, const std::vector<uint32_t> &src) {
        for (size_t i = 0; i < src.size(); ++i) {
            const uint64_t bi = primes[src[i]];
            uint64_t hat_i = 1;  // (B / b_i) mod b_i
            for (size_t k = 0; k < src.size(); ++k)
                if (k != i) hat_i = mul_mod(hat_i, primes[src[k]] % bi, bi);
            const uint64_t y = mul_mod(inv_mod(hat_i, bi), c->ninv[src[i]].w, bi);
            c->ys[(size_t)set * kMaxDigit32 + i] = pair32(y, bi);
            for (uint32_t t = 0; t < np_all; ++t) {
                const uint64_t qt = primes[t];
                uint64_t h = 1;
                for (size_t k = 0; k < src.size(); ++k)
                    if (k != i) h = mul_mod(h, primes[src[k]] % qt, qt);
                hmod[((size_t)set * np_all + t) * kMaxDigit32 + i] = (uint32_t)h;
            }
        }
    };
    for (uint32_t j = 0; j < dnum; ++j)
        for (uint32_t size = 1; size <= alpha; ++size) {
            if (j * alpha + size > n_q) continue;
            std::vector<uint32_t> src;
            for (uint32_t i = 0; i < size; ++i) src.push_back(j * alpha + i);
            fill_set(c->set_index(j, size), src);
        }
    {
        std::vector<uint32_t> src;
        for (uint32_t k = 0; k < n_p; ++k) src.push_back(n_q + k);
        fill_set(c->pset(), src);
    }
    std::vector<uint32_t> pmod(np_all);
    std::vector<Pair32> pinv(np_all);
    for (uint32_t t = 0; t < np_all; ++t) {
        const uint64_t qt = primes[t];
        uint64_t P = 1;
        for (uint32_t k = 0; k < n_p; ++k) P = mul_mod(P, primes[n_q + k] % qt, qt);
        pmod[t] = (uint32_t)P;
        pinv[t] = t < n_q ? pair32(inv_mod(P, qt), qt) : Pair32{0, 0};
    }
    std::vector<Pair32> qlinv((size_t)n_q * n_q, Pair32{0, 0});
    std::vector<uint32_t> qlmod((size_t)n_q * n_q, 0);
    for (uint32_t l = 1; l < n_q; ++l)
        for (uint32_t i = 0; i < l; ++i) {
            qlmod[(size_t)l * n_q + i] = (uint32_t)(primes[l] % primes[i]);
            qlinv[(size_t)l * n_q + i] = pair32(inv_mod(primes[l] % primes[i], primes[i]), primes[i]);
        }
    c->qlinv = qlinv;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t o_pr = take(pr.size() * sizeof(Prime32)), o_twf = take(twf.size() * sizeof(Pair32)),
                 o_twi = take(twi.size() * sizeof(Pair32)), o_hm = take(hmod.size() * 4),
                 o_pm = take(pmod.size() * 4), o_pi = take(pinv.size() * sizeof(Pair32)),
                 o_ql = take(qlinv.size() * sizeof(Pair32)), o_qm = take(qlmod.size() * 4);
    if (hipMalloc(&c->dev, off) != hipSuccess) {
        delete c;
        return fail(CKKS_E_NOMEM, "ckks32_ctx_create: table allocation failed");
    }
    char *base = (char *)c->dev;
    c->d_primes = (Prime32 *)(base + o_pr);
    c->d_tw_fwd = (Pair32 *)(base + o_twf);
    c->d_tw_inv = (Pair32 *)(base + o_twi);
    c->d_hmod = (uint32_t *)(base + o_hm);
    c->d_pmod = (uint32_t *)(base + o_pm);
    c->d_pinv = (Pair32 *)(base + o_pi);
    c->d_qlinv = (Pair32 *)(base + o_ql);
    c->d_qlmod = (uint32_t *)(base + o_qm);
    hipError_t e = hipMemcpy(c->d_primes, pr.data(), pr.size() * sizeof(Prime32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_tw_fwd, twf.data(), twf.size() * sizeof(Pair32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_tw_inv, twi.data(), twi.size() * sizeof(Pair32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_hmod, hmod.data(), hmod.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_pmod, pmod.data(), pmod.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_pinv, pinv.data(), pinv.size() * sizeof(Pair32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_qlinv, qlinv.data(), qlinv.size() * sizeof(Pair32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_qlmod, qlmod.data(), qlmod.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(c->dev);
        delete c;
        return fail(CKKS_E_DEVICE, "ckks32_ctx_create: table upload failed");
    }
    *out = c;
    return CKKS_OK;
}

extern "C" void ckks32_ctx_destroy(ckks32_ctx *c)
{
    if (!c) return;
    if (c->dev) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(c->device);
        (void)hipFree(c->dev);
        (void)hipSetDevice(cur);
    }
    delete c;
}

extern "C" size_t ckks32_workspace_bytes(const ckks32_ctx *c, uint32_t op, uint32_t level)
{
    if (!c || level >= c->nq) return 0;
    const size_t n = level + 1;
    switch (op) {
    case CKKS_OP_KEYSWITCH: return ks_bytes(c, level);
    case CKKS_OP_HMULT:
    case CKKS_OP_ROTATE: return ks_bytes(c, level) + align256(2 * n * kN * 4);
    case CKKS_OP_RESCALE: return (2 + 2 * (size_t)level) * kN * 4;
    default: return 0;
    }
}

static ckks_status ntt32_common(ckks32_ctx *c, uint32_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream,
                                bool inverse)
{
    if (!c) return fail(CKKS_E_ARG, "ckks32_(i)ntt: null context");
    TRY32(check_ptr32(poly, "ckks32_(i)ntt poly"));
    if (n_limbs == 0 || limb0 + n_limbs > c->nq + c->np || n_limbs > kMaxRows32)
        return fail(CKKS_E_ARG, "ckks32_(i)ntt: limb range outside q_0..q_L, p_0..p_{K-1}");
    Ntt32Args a = base_args(c, inverse);
    a.src = a.dst = poly;
    a.rows = n_limbs;
    a.npoly = 1;
    for (uint32_t r = 0; r < n_limbs; ++r) {
        a.prime[r] = (uint8_t)(limb0 + r);
        a.scale[r] = c->ninv[limb0 + r];
    }
    return dev32(launch_ntt32(a, inverse, (hipStream_t)stream), inverse ? "ckks32_intt" : "ckks32_ntt");
}

extern "C" ckks_status ckks32_ntt(ckks32_ctx *c, uint32_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream)
{
    return ntt32_common(c, poly, limb0, n_limbs, stream, false);
}

extern "C" ckks_status ckks32_intt(ckks32_ctx *c, uint32_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream)
{
    return ntt32_common(c, poly, limb0, n_limbs, stream, true);
}

extern "C" ckks_status ckks32_modup(ckks32_ctx *c, const uint32_t *d, uint32_t level, uint32_t *ext, void *ws,
                                    void *stream)
{
    TRY32(check_ctx32(c, level));
    TRY32(check_ptr32(d, "ckks32_modup d"));
    TRY32(check_ptr32(ext, "ckks32_modup ext"));
    TRY32(check_ptr32(ws, "ckks32_modup ws"));
    const hipStream_t st = (hipStream_t)stream;
    const Sizes32 s = sizes(c, level);
    Ws32 w = ks_ws(c, level, ws);
    w.ext = ext;  // the caller's buffer: its own rows are copied from d afterwards
    hipError_t e = modup32(c, d, level, w, st);
    for (uint32_t j = 0; j < s.beta && e == hipSuccess; ++j) {
        const uint32_t lo = j * c->alpha, hi = std::min(lo + c->alpha, s.n);
        e = hipMemcpyAsync(ext + ((size_t)j * s.rows + lo) * kN, d + (size_t)lo * kN, (size_t)(hi - lo) * kN * 4,
                           hipMemcpyDeviceToDevice, st);
    }
    return dev32(e, "ckks32_modup");
}

extern "C" ckks_status ckks32_moddown(ckks32_ctx *c, const uint32_t *x, uint32_t level, uint32_t *out0,
                                      uint32_t *out1, void *ws, void *stream)
{
    TRY32(check_ctx32(c, level));
    TRY32(check_ptr32(x, "ckks32_moddown x"));
    TRY32(check_ptr32(out0, "ckks32_moddown out0"));
    TRY32(check_ptr32(out1, "ckks32_moddown out1"));
    TRY32(check_ptr32(ws, "ckks32_moddown ws"));
    const hipStream_t st = (hipStream_t)stream;
    const Ws32 w = ks_ws(c, level, ws);
    return dev32(moddown32(c, x, level, w, out0, out1, nullptr, nullptr, st), "ckks32_moddown");
}

extern "C" ckks_status ckks32_keyswitch(ckks32_ctx *c, const uint32_t *d, uint32_t level, const uint32_t *key,
                                        uint32_t *out0, uint32_t *out1, void *ws, void *stream)
{
    TRY32(check_ctx32(c, level));
    TRY32(check_ptr32(d, "ckks32_keyswitch d"));
    TRY32(check_ptr32(key, "ckks32_keyswitch key"));
    TRY32(check_ptr32(out0, "ckks32_keyswitch out0"));
    TRY32(check_ptr32(out1, "ckks32_keyswitch out1"));
    TRY32(check_ptr32(ws, "ckks32_keyswitch ws"));
    return dev32(keyswitch32(c, d, level, key, out0, out1, nullptr, nullptr, ws, (hipStream_t)stream),
                 "ckks32_keyswitch");
}

extern "C" ckks_status ckks32_hmult_relin(ckks32_ctx *c, const uint32_t *a0, const uint32_t *a1, const uint32_t *b0,
                                          const uint32_t *b1, uint32_t level, const uint32_t *rlk, uint32_t *out0,
                                          uint32_t *out1, void *ws, void *stream)
{
    TRY32(check_ctx32(c, level));
    const void *ptrs[] = {a0, a1, b0, b1, rlk, out0, out1, ws};
    for (const void *q : ptrs) TRY32(check_ptr32(q, "ckks32_hmult_relin"));
    const hipStream_t st = (hipStream_t)stream;
    const size_t n = level + 1;
    uint32_t *d2 = (uint32_t *)((char *)ws + ks_bytes(c, level));
    hipLaunchKernelGGL(k32_tensor, dim3(kN / kB, n), dim3(kB), 0, st, a0, a1, b0, b1, out0, out1, d2, c->d_primes);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = keyswitch32(c, d2, level, rlk, out0, out1, out0, out1, ws, st);
    return dev32(e, "ckks32_hmult_relin");
}

extern "C" ckks_status ckks32_apply_galois(ckks32_ctx *c, const uint32_t *c0, const uint32_t *c1, uint32_t level,
                                           uint32_t galois, const uint32_t *key, uint32_t *out0, uint32_t *out1,
                                           void *ws, void *stream)
{
    TRY32(check_ctx32(c, level));
    const void *ptrs[] = {c0, c1, key, out0, out1, ws};
    for (const void *q : ptrs) TRY32(check_ptr32(q, "ckks32_apply_galois"));
    if (galois % 2 == 0 || galois >= 2 * kN) return fail(CKKS_E_ARG, "ckks32_apply_galois: galois must be odd, below 2N");
    const hipStream_t st = (hipStream_t)stream;
    const size_t n = level + 1;
    uint32_t *g0 = (uint32_t *)((char *)ws + ks_bytes(c, level)), *g1 = g0 + n * kN;
    hipLaunchKernelGGL(k32_automorph, dim3(kN / kB, n), dim3(kB), 0, st, c0, g0, galois);
    hipLaunchKernelGGL(k32_automorph, dim3(kN / kB, n), dim3(kB), 0, st, c1, g1, galois);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = keyswitch32(c, g1, level, key, out0, out1, g0, nullptr, ws, st);
    return dev32(e, "ckks32_apply_galois");
}

extern "C" ckks_status ckks32_rescale(ckks32_ctx *c, const uint32_t *c0, const uint32_t *c1, uint32_t level,
                                      uint32_t *out0, uint32_t *out1, void *ws, void *stream)
{
    TRY32(check_ctx32(c, level));
    if (level < 1) return fail(CKKS_E_LEVEL, "ckks32_rescale: level 0 cannot be rescaled");
    const void *ptrs[] = {c0, c1, out0, out1, ws};
    for (const void *q : ptrs) TRY32(check_ptr32(q, "ckks32_rescale"));
    const hipStream_t st = (hipStream_t)stream;
    const uint32_t l = level;
    uint32_t *v = (uint32_t *)ws, *lift = v + 2 * (size_t)kN;
    // v_t = INTT_{q_l}(c_t[l]): copy the two last limbs, transform in place
    hipError_t e = hipMemcpyAsync(v, c0 + (size_t)l * kN, kN * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(v + kN, c1 + (size_t)l * kN, kN * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return dev32(e, "ckks32_rescale");
    Ntt32Args ia = base_args(c, true);
    ia.src = ia.dst = v;
    ia.src_poly_stride = ia.dst_poly_stride = kN;
    ia.rows = 1;
    ia.npoly = 2;
    ia.prime[0] = (uint8_t)l;
    ia.scale[0] = c->ninv[l];
    e = launch_ntt32(ia, true, st);
    if (e != hipSuccess) return dev32(e, "ckks32_rescale");
    hipLaunchKernelGGL(k32_lift, dim3(kN / kB, l, 2), dim3(kB), 0, st, v, lift, c->d_primes, c->d_qlmod + (size_t)l * c->nq,
                       c->primes[l], l);
    Ntt32Args fa = base_args(c, false);
    fa.src = fa.dst = lift;
    fa.src_poly_stride = fa.dst_poly_stride = (int64_t)l * kN;
    fa.rows = l;
    fa.npoly = 2;
    for (uint32_t r = 0; r < l; ++r) fa.prime[r] = (uint8_t)r;
    fa.epi = 2;
    fa.aux[0] = c0;
    fa.aux[1] = c1;
    fa.out[0] = out0;
    fa.out[1] = out1;
    fa.cst = c->d_qlinv + (size_t)l * c->nq;
    return dev32(launch_ntt32(fa, false, st), "ckks32_rescale");
}
