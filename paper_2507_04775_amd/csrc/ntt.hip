// Negacyclic NTT / inverse NTT for gfx950 (paper Sec. III-F.4).
//
// Forward: radix-2 Cooley-Tukey with the psi twist merged into the
// butterflies, natural coefficients -> bit-reversed evaluations.  Inverse:
// Gentleman-Sande butterflies, bit-reversed -> natural, times N^-1.  The
// butterfly of stage m at index j uses w = psi^br(m + j div 2t) from the
// context tables.
//
// Layout of the work: threads own a few elements each and run several radix-2
// stages on them in registers ("rounds"); rounds exchange data through LDS.
// N = 2^12 fits one workgroup of 256 threads with 16 elements each (three
// rounds of four stages).  N = 2^16 is the paper's 2-D / hierarchical scheme:
// viewed as a 256 x 256 matrix, a column pass runs the first eight stages
// (each column is an independent 256-point problem) and a row pass runs the
// last eight (each row of 256 contiguous elements is independent, with its own
// twiddle subset).  Each pass reads and writes every element once: four global
// accesses per element in total.  A pass workgroup holds 16 columns (rows) with
// 32 threads on each and 8 elements per thread, in rounds of 3, 3 and 2
// stages: short dependency chains per thread and twice the waves of a
// 16-element layout, which matters most for the slower integer path.
//
// Two arithmetic paths, chosen per limb (uniform per workgroup):
// - primes below 2^50: exact FP64 arithmetic (modarith.h).  Values are
//   signed representatives; a centred reduction at the start of each round
//   keeps |x| <= q/2 + 1, after which four forward stages stay below 5.3 q
//   (7.1 q when a round starts from canonical input) and four inverse stages,
//   with the sums of the third stage re-centred, below 4 q; all < 2^53.
// - other primes (up to 2^61): 64-bit integers with Shoup twiddles and
//   Harvey's lazy butterflies ([0, 4q) forward, [0, 2q) inverse).
// Outputs of every transform are canonical.
#include <atomic>

#include "coef_units.h"
#include "internal.h"
#include "unit_map.h"

namespace ckks {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t pad(uint32_t x) { return x + (x >> 4); }


// ----------------------------------------------------------- integer path

struct IntArith {
    typedef uint64_t V;
    typedef ulonglong2 W;
    const ulonglong2 *T;
    uint64_t q, q2, fc, fc_s;  // fc: constant of the last inverse multiplication

    __device__ __forceinline__ V from_u64(uint64_t x) const { return x; }
    __device__ __forceinline__ V from_bits(uint64_t x) const { return x; }
    __device__ __forceinline__ uint64_t to_bits(V x) const { return x; }
    __device__ __forceinline__ W tw(uint32_t i) const { return T[i]; }
    // the twiddle at hi + k (k below the lowest set bit of hi): read from the table
    __device__ __forceinline__ W tw_split(uint32_t hi, uint32_t k) const { return T[hi + k]; }
    // [x y]_q of two canonical residues (HMult's d2 = a1 b1 as it is loaded)
    __device__ __forceinline__ V product(uint64_t x, uint64_t y, const Prime &P) const
    {
        return reduce128(mul_wide(x, y), P);
    }
    template <int NV>
    __device__ __forceinline__ void reduce_all(V (&)[NV]) const {}
    // Harvey forward butterfly: x, y in [0, 4q) -> [0, 4q)
    __device__ __forceinline__ void ct(V &x, V &y, W w) const
    {
        uint64_t a = x >= q2 ? x - q2 : x;
        uint64_t t = shoup_lazy(y, w.x, w.y, q);
        x = a + t;
        y = a - t + q2;
    }
    // Harvey inverse butterfly: x, y in [0, 2q) -> [0, 2q)
    __device__ __forceinline__ void gs(V &x, V &y, W w, int) const
    {
        uint64_t s = x + y;
        s = s >= q2 ? s - q2 : s;
        uint64_t d = x - y + q2;
        x = s;
        y = shoup_lazy(d, w.x, w.y, q);
    }
    __device__ __forceinline__ uint64_t fwd_final(V x) const { return csub(csub(x, q2), q); }
    __device__ __forceinline__ uint64_t inv_final(V x) const { return shoup(x, fc, fc_s, q); }
    __device__ __forceinline__ uint64_t modulus() const { return q; }
    // key inner product on canonical values
    __device__ __forceinline__ V mac_in(V x) const { return fwd_final(x); }
    __device__ __forceinline__ V own(uint64_t x) const { return x; }
    __device__ __forceinline__ void mac(V &acc, V v, uint64_t k, const Prime &P) const
    {
        acc = addmod(acc, mulmod(v, k, P), q);
    }
    __device__ __forceinline__ uint64_t acc_final(V acc) const { return acc; }
};

// ----------------------------------------------------------- FP64 path

struct FpArith {
    typedef double V;
    typedef double W;
    const double *T;
    FpMod m;
    double fc;  // constant of the last inverse multiplication

    __device__ __forceinline__ V from_u64(uint64_t x) const { return (double)x; }
    __device__ __forceinline__ V from_bits(uint64_t x) const { return __longlong_as_double((long long)x); }
    __device__ __forceinline__ uint64_t to_bits(V x) const { return (uint64_t)__double_as_longlong(x); }
    __device__ __forceinline__ W tw(uint32_t i) const { return T[i]; }
    // the twiddle at hi + k, k below the lowest set bit of hi: the table holds psi^br(i) (or its
    // inverse), and br(hi + k) = br(hi) + br(k) for such k, so it is T[hi] T[k], formed here (a
    // centred representative) from the row's one entry and the first entries shared by every row
    __device__ __forceinline__ W tw_split(uint32_t hi, uint32_t k) const { return fp_mulmod(T[hi], T[k], m); }
    // [x y]_q of two canonical residues below 2^50, a centred representative
    __device__ __forceinline__ V product(uint64_t x, uint64_t y, const Prime &) const
    {
        return fp_mulmod((double)x, (double)y, m);
    }
    template <int NV>
    __device__ __forceinline__ void reduce_all(V (&v)[NV]) const
    {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = fp_reduce(v[i], m);
    }
    __device__ __forceinline__ void ct(V &x, V &y, W w) const
    {
        double t = fp_mulmod(y, w, m);
        double a = x;
        x = a + t;
        y = a - t;
    }
    // the sums of the third stage of a round (st == 2) are re-centred
    __device__ __forceinline__ void gs(V &x, V &y, W w, int st) const
    {
        double s = x + y, d = x - y;
        x = st == 2 ? fp_reduce(s, m) : s;
        y = fp_mulmod(d, w, m);
    }
    __device__ __forceinline__ uint64_t fwd_final(V x) const { return fp_canonical(x, m); }
    __device__ __forceinline__ uint64_t inv_final(V x) const { return fp_canonical(fp_mulmod(x, fc, m), m); }
    __device__ __forceinline__ uint64_t modulus() const { return (uint64_t)m.q; }
    // key inner product: |v| < 5.3 q from a forward round, the running sum re-centred each step
    __device__ __forceinline__ V mac_in(V x) const { return x; }
    __device__ __forceinline__ V own(uint64_t x) const { return (double)x; }
    __device__ __forceinline__ void mac(V &acc, V v, uint64_t k, const Prime &) const
    {
        acc = fp_reduce(acc + fp_mulmod(v, (double)k, m), m);
    }
    __device__ __forceinline__ uint64_t acc_final(V acc) const { return fp_canonical(acc, m); }
};

// Stores the last inverse pass's outputs.  For ModDown's centred conversion
// (ys_mode 2) each canonical y of the special limb p is stored as y + p when
// y <= (p - 1)/2, else as y: the centred representative plus p, in
// [(p + 1)/2, 3 (p - 1)/2], below 2^62, so the conversion's sums take no
// per-term comparison (bconv_load removes the shift).
template <int NV, class A, class Idx>
__device__ __forceinline__ void inv_store(uint64_t *dst, const typename A::V (&v)[NV], const A &ar, uint32_t ys_mode,
                                          Idx idx)
{
    if (ys_mode == 2) {
        const uint64_t q = ar.modulus(), half = q >> 1;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const uint64_t y = ar.inv_final(v[i]);
            dst[idx(i)] = y <= half ? y + q : y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) dst[idx(i)] = ar.inv_final(v[i]);
    }
}

// LOG forward stages on v[i] = element base + STRIDE i (i < 2^LOG) of an
// NS-point problem: t = 2^(LOG-1) STRIDE, ..., STRIDE.  base = a 2^LOG STRIDE
// + s with s < STRIDE.  Twiddles come from T[m B + j div 2t], m = NS / 2t.
// tw_fwd loads the 2^LOG - 1 twiddles a round uses (stage by stage, group by
// group) and fwd_rw applies them, so a pass can issue a round's twiddle loads
// before the barrier that precedes the round.
//
// Row passes (ROW, B = 256 + row) take the stages with NS / 2t >= kTwSplit
// groups per row as tw_split(m B, j div 2t): one table entry per row and
// stage, and the first entries of the table, which every row shares.  A row
// then reads 34 of its 255 twiddles from the table instead of all of them.
constexpr uint32_t kTwSplit = 32;

template <int LOG, int NS, int STRIDE, class A, bool ROW = false>
__device__ __forceinline__ void tw_fwd(typename A::W *w, uint32_t base, const A &ar, uint32_t B)
{
    int k = 0;
#pragma unroll
    for (int st = 0; st < LOG; ++st) {
        const uint32_t t = ((1u << (LOG - 1)) >> st) * STRIDE;
        const uint32_t hi = (NS / (2 * t)) * B, g0 = base / (2 * t);
#pragma unroll
        for (int g = 0; g < (1 << st); ++g)
            w[k++] = ROW && NS / (2 * t) >= kTwSplit ? ar.tw_split(hi, g0 + g) : ar.tw(hi + g0 + g);
    }
}

template <int LOG, class A>
__device__ __forceinline__ void fwd_rw(typename A::V *v, const typename A::W *w, const A &ar)
{
    int k = 0;
#pragma unroll
    for (int st = 0; st < LOG; ++st) {
        const int h = (1 << (LOG - 1)) >> st;
#pragma unroll
        for (int g = 0; g < (1 << st); ++g) {
            const typename A::W ww = w[k++];
#pragma unroll
            for (int kk = 0; kk < h; ++kk) ar.ct(v[g * 2 * h + kk], v[g * 2 * h + kk + h], ww);
        }
    }
}

template <int LOG, int NS, int STRIDE, class A>
__device__ __forceinline__ void fwd_r(typename A::V *v, uint32_t base, const A &ar, uint32_t B)
{
    typename A::W w[(1 << LOG) - 1];
    tw_fwd<LOG, NS, STRIDE>(w, base, ar, B);
    fwd_rw<LOG>(v, w, ar);
}

// LOG inverse stages: t = STRIDE, 2 STRIDE, ..., 2^(LOG-1) STRIDE.  Rounds
// of four stages re-centre the sums of their third stage (FP64 path); three
// stages from a centred start stay below 4 q + 8 without it.
template <int LOG, int NS, int STRIDE, class A, bool ROW = false>
__device__ __forceinline__ void tw_inv(typename A::W *w, uint32_t base, const A &ar, uint32_t B)
{
    int k = 0;
#pragma unroll
    for (int st = 0; st < LOG; ++st) {
        const uint32_t t = (1u << st) * STRIDE;
        const uint32_t hi = (NS / (2 * t)) * B, g0 = base / (2 * t);
#pragma unroll
        for (int g = 0; g < ((1 << (LOG - 1)) >> st); ++g)
            w[k++] = ROW && NS / (2 * t) >= kTwSplit ? ar.tw_split(hi, g0 + g) : ar.tw(hi + g0 + g);
    }
}

template <int LOG, class A>
__device__ __forceinline__ void inv_rw(typename A::V *v, const typename A::W *w, const A &ar)
{
    int k = 0;
#pragma unroll
    for (int st = 0; st < LOG; ++st) {
        const int h = 1 << st;
#pragma unroll
        for (int g = 0; g < ((1 << (LOG - 1)) >> st); ++g) {
            const typename A::W ww = w[k++];
#pragma unroll
            for (int kk = 0; kk < h; ++kk) ar.gs(v[g * 2 * h + kk], v[g * 2 * h + kk + h], ww, LOG == 4 ? st : -1);
        }
    }
}

template <int LOG, int NS, int STRIDE, class A>
__device__ __forceinline__ void inv_r(typename A::V *v, uint32_t base, const A &ar, uint32_t B)
{
    typename A::W w[(1 << LOG) - 1];
    tw_inv<LOG, NS, STRIDE>(w, base, ar, B);
    inv_rw<LOG>(v, w, ar);
}

template <int NS, int STRIDE, class A>
__device__ __forceinline__ void fwd16(typename A::V (&v)[16], uint32_t base, const A &ar, uint32_t B)
{
    fwd_r<4, NS, STRIDE>(v, base, ar, B);
}

template <int NS, int STRIDE, class A>
__device__ __forceinline__ void inv16(typename A::V (&v)[16], uint32_t base, const A &ar, uint32_t B)
{
    inv_r<4, NS, STRIDE>(v, base, ar, B);
}

// The thread's index, opaque to loop-invariant code motion, for the pass
// bodies of the persistent kernels at N = 2^16.  Those run a body once per
// claimed unit; offsets derived from threadIdx.x and hoisted out of that loop
// stay live in vector registers across the whole body (ModDown's conversion
// pass needed 154 per thread that way, 124 with this index, and the forward
// column pass 118 against 70).  Grid kernels pass threadIdx.x itself.
__device__ __forceinline__ uint32_t thread_index()
{
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

struct LimbPos {
    uint32_t poly, row, prime;
    bool skip;
};

// Field of polynomial p (0 or 1) of a two-entry argument array, as a select:
// the argument block then has no dynamically indexed field and a persistent
// kernel keeps it in scalar registers.
template <class T>
__device__ __forceinline__ T pick(T const (&v)[2], uint32_t p)
{
    return p ? v[1] : v[0];
}

__host__ __device__ __forceinline__ LimbPos limb_pos(const LimbMap &m, uint32_t limb)
{
    LimbPos p;
    if (m.dense && m.skip_alpha) {
        // the limb-th row that is not skipped: polynomial j leaves out its rows
        // [j alpha, min(j alpha + alpha, level + 1)) (row0 = 0 in such launches)
        uint32_t rem = limb, poly = 0;
        for (;;) {
            const uint32_t lo = poly * m.skip_alpha;
            const uint32_t hi = lo + m.skip_alpha < m.level + 1 ? lo + m.skip_alpha : m.level + 1;
            const uint32_t gap = hi > lo ? hi - lo : 0, kept = m.rows - gap;
            if (rem < kept) {
                p.poly = poly;
                p.row = rem < lo ? rem : rem + gap;
                break;
            }
            rem -= kept;
            ++poly;
        }
        p.skip = false;
    } else {
        p.poly = limb / m.rows;
        p.row = limb - p.poly * m.rows;
        p.skip = limb_skipped(m, p.poly, p.row);
    }
    p.prime = limb_prime(m, p.row);
    return p;
}

// SwitchModulo of the rescale: u in [0, q_l) lifted centred and reduced mod q
__device__ __forceinline__ uint64_t switch_modulo(uint64_t u, uint64_t half, uint64_t qlmod, const Prime &P)
{
    uint64_t um = csub(u - mul_hi(u, P.one_s) * P.q, P.q);
    return u <= half ? um : submod(um, qlmod, P.q);
}

template <int PRO>
__device__ __forceinline__ uint64_t load_fwd(const NttArgs &a, const LimbPos &lp, const uint64_t *src, uint32_t e,
                                             const Prime &P)
{
    if (PRO == PRO_RESCALE) {
        return switch_modulo(pick(a.rs_src, lp.poly)[e], (a.rs_ql - 1) >> 1, a.rs_qlmod[lp.prime], P);
    } else {
        return src[e];
    }
}

// Final forward value x (canonical) at element e of the limb; `addv` is the
// addend of the ModDown epilogue (already gathered, 0 without addend).
template <int EPI>
__device__ __forceinline__ void store_fwd(const NttArgs &a, const LimbPos &lp, uint64_t *dst, uint32_t e, uint64_t x,
                                          uint64_t addv, uint64_t auxv, const Prime &P, size_t N)
{
    if (EPI == EPI_PLAIN) {
        dst[e] = x;
    } else {
        const size_t off = (size_t)lp.row * N;
        const ulonglong2 c = a.cst[lp.prime];
        uint64_t r = shoup(submod(auxv, x, P.q), c.x, c.y, P.q);
        if (EPI == EPI_MODDOWN) r = addmod(r, addv, P.q);
        pick(a.out, lp.poly)[off + e] = r;
    }
}

__device__ __forceinline__ IntArith int_arith(const ulonglong2 *tw, const Prime &P, uint32_t prime, uint32_t N)
{
    IntArith r;
    r.T = tw + (size_t)prime * N;
    r.q = P.q;
    r.q2 = P.two_q;
    r.fc = P.ninv;
    r.fc_s = P.ninv_s;
    return r;
}

__device__ __forceinline__ FpArith fp_arith(const double *twd, const Prime &P, uint32_t prime, uint32_t N)
{
    FpArith r;
    r.T = twd + (size_t)prime * N;
    r.m.q = (double)P.q;
    r.m.qinv = P.qinv;
    r.fc = (double)P.ninv;
    return r;
}

__device__ __forceinline__ IntArith int_arith(const NttArgs &a, const Prime &P, uint32_t prime, uint32_t N)
{
    return int_arith(a.tw, P, prime, N);
}

__device__ __forceinline__ FpArith fp_arith(const NttArgs &a, const Prime &P, uint32_t prime, uint32_t N)
{
    return fp_arith(a.twd, P, prime, N);
}

// Constant of the last inverse multiplication of a limb: N^-1, or the
// base-conversion input scale N^-1 [(B/b_i)^-1]_{b_i} (ys_mode 1 / 2).
__device__ __forceinline__ uint32_t ys_index(const NttArgs &a, const LimbPos &lp)
{
    if (a.ys_mode == 1) {
        const uint32_t r = lp.row + a.map.row0, j = r / a.alpha, lo = j * a.alpha;
        const uint32_t ns = min(a.alpha, a.nlev - lo);
        return (j * a.alpha + ns - 1) * kMaxDigitPrimes + (r - lo);
    }
    return a.pset * kMaxDigitPrimes + lp.row;
}

__device__ __forceinline__ IntArith inv_int_arith(const NttArgs &a, const LimbPos &lp, const Prime &P, uint32_t N)
{
    IntArith r = int_arith(a, P, lp.prime, N);
    if (a.ys_mode) {
        const ulonglong2 c = a.ys[ys_index(a, lp)];
        r.fc = c.x;
        r.fc_s = c.y;
    }
    return r;
}

__device__ __forceinline__ FpArith inv_fp_arith(const NttArgs &a, const LimbPos &lp, const Prime &P, uint32_t N)
{
    FpArith r = fp_arith(a, P, lp.prime, N);
    if (a.ys_mode) r.fc = a.ysd[ys_index(a, lp)];
    return r;
}

// Source of a base conversion computed in the first forward pass (PRO_BCONV).
struct BcSrc {
    const uint64_t *y;   // ns scaled source rows, stride N
    const uint64_t *hm;  // [B/b_i] mod the target prime, i < ns
    uint32_t ns;
    const Prime *src;    // centred conversion (ModDown, inputs shifted by p_k): the source primes, else null
    uint64_t bq;         // [B]_q of the target prime (centred conversion)
};

__device__ __forceinline__ BcSrc bc_source(const NttArgs &a, uint32_t poly, uint32_t prime, size_t N)
{
    BcSrc b;
    uint32_t set;
    if (a.bc_mode == 1) {
        const uint32_t lo = poly * a.alpha;
        b.ns = min(a.alpha, a.nlev - lo);
        set = poly * a.alpha + b.ns - 1;
        b.y = a.bc_src + (size_t)lo * N;
        b.src = nullptr;
        b.bq = 0;
    } else {
        b.ns = a.nprimes - a.map.nq;
        set = a.pset;
        b.y = a.bc_src + (int64_t)poly * a.bc_poly_stride;
        b.src = a.primes + a.map.nq;
        b.bq = a.pmod[prime];
    }
    b.hm = a.hmod + ((size_t)set * a.nprimes + prime) * kMaxDigitPrimes;
    return b;
}

// v[i] = Conv(y)[pos(i)]: sum_k y_k[pos] [B/b_k]_q accumulated exactly, reduced
// once.  Acc sums by 32-bit columns: MacSplit (four multiply-adds per term)
// when the target prime, and so every constant, is below 2^50 (the table holds
// those constants split), else MacCols
// (four multiply-adds and three carry additions; the constants in scalar
// registers either way).  Groups of four elements keep the column sums in few
// registers.  The loads of source row k+1 are issued before the products of
// row k, so the latency of the source rows overlaps the arithmetic.  For
// ModDown's centred conversion the inverse NTT stored u_k = y_k + p_k with
// y_k centred: sum_k p_k [P/p_k]_q = K [P]_q (mod q), which `corr` removes
// after the reduction.
template <class Acc, int NV, class A, class Pos>
__device__ __forceinline__ void bconv_sum(typename A::V (&v)[NV], const A &ar, const BcSrc &b, const Prime &P,
                                          size_t N, Pos pos, uint64_t corr)
{
    constexpr int G = 4;
    static_assert(NV % G == 0, "groups of four elements");
#pragma unroll
    for (int grp = 0; grp < NV / G; ++grp) {
        Acc acc[G];
        uint64_t cur[G];
#pragma unroll
        for (int i = 0; i < G; ++i) cur[i] = b.y[pos(G * grp + i)];
        for (uint32_t k = 0; k < b.ns; ++k) {
            const bool more = k + 1 < b.ns;
            uint64_t nxt[G];
            if (more) {
                const uint64_t *yn = b.y + (size_t)(k + 1) * N;
#pragma unroll
                for (int i = 0; i < G; ++i) nxt[i] = yn[pos(G * grp + i)];
            }
            const uint64_t h = ((const __attribute__((address_space(4))) uint64_t *)b.hm)[k];  // scalar cache
#pragma unroll
            for (int i = 0; i < G; ++i) acc[i].add(cur[i], h);
            if (more) {
#pragma unroll
                for (int i = 0; i < G; ++i) cur[i] = nxt[i];
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) v[G * grp + i] = ar.from_u64(submod(reduce128(acc[i].total(), P), corr, P.q));
    }
}

// The same for at most kConvBatch source rows: every load of a group is
// issued before its first product, one wait per group instead of one per row.
constexpr uint32_t kConvBatch = 4;

template <class Acc, int NV, class A, class Pos>
__device__ __forceinline__ void bconv_sum_few(typename A::V (&v)[NV], const A &ar, const BcSrc &b, const Prime &P,
                                              size_t N, Pos pos, uint64_t corr)
{
    constexpr int G = 4;
    static_assert(NV % G == 0, "groups of four elements");
#pragma unroll
    for (int grp = 0; grp < NV / G; ++grp) {
        uint64_t y[kConvBatch][G];
#pragma unroll
        for (uint32_t k = 0; k < kConvBatch; ++k)
            if (k < b.ns) {
#pragma unroll
                for (int i = 0; i < G; ++i) y[k][i] = b.y[(size_t)k * N + pos(G * grp + i)];
            }
        Acc acc[G];
#pragma unroll
        for (uint32_t k = 0; k < kConvBatch; ++k)
            if (k < b.ns) {
                const uint64_t h = ((const __attribute__((address_space(4))) uint64_t *)b.hm)[k];  // scalar cache
#pragma unroll
                for (int i = 0; i < G; ++i) acc[i].add(y[k][i], h);
            }
#pragma unroll
        for (int i = 0; i < G; ++i) v[G * grp + i] = ar.from_u64(submod(reduce128(acc[i].total(), P), corr, P.q));
    }
}

template <int NV, class A, class Pos>
__device__ __forceinline__ void bconv_load(typename A::V (&v)[NV], const A &ar, const BcSrc &b, const Prime &P,
                                           size_t N, Pos pos)
{
    const uint64_t corr = b.src ? reduce128(mul_wide((uint64_t)b.ns, b.bq), P) : 0;
    if (b.ns <= kConvBatch) {
        if (P.q < kSplitMaxConst)
            bconv_sum_few<MacSplit>(v, ar, b, P, N, pos, corr);
        else
            bconv_sum_few<MacColsAcc>(v, ar, b, P, N, pos, corr);
    } else if (P.q < kSplitMaxConst) {
        bconv_sum<MacSplit>(v, ar, b, P, N, pos, corr);
    } else {
        bconv_sum<MacColsAcc>(v, ar, b, P, N, pos, corr);
    }
}

// ------------------------------------------------------------------ N = 2^16
// Every kernel body processes one "unit": tile `tile` (16 columns or 16 rows
// of the 256 x 256 view) of limb `limb` of a launch described by NttArgs.
// Grid kernels take (tile, limb) from (blockIdx.x, blockIdx.y); persistent
// kernels claim units from a work queue (see the end of this file).
//
// A unit runs on 512 threads: 32 per column (row), each holding 8 of its 256
// elements.  Element positions within the 256-point problem in the three
// layouts a thread s < 32 takes:
//   wide   s + 32 i          (stages t = 128, 64, 32; coalesced global access)
//   mid    32 (s/4) + s%4 + 4 i (stages t = 16, 8, 4)
//   narrow 8 s + i            (stages t = 2, 1 as two radix-4 groups)
// Between layouts each thread stores what it holds and, after one barrier,
// loads the next layout; a thread only ever overwrites slots it loaded itself,
// so one barrier per exchange suffices.

constexpr int kThreads16 = 512;

// The 32 threads of a row lie in one 64-wide wave (a wave holds two rows), so
// the row passes exchange data through LDS within the wave: a release fence,
// a wave barrier and an acquire fence order the LDS stores before the loads of
// other lanes, with no workgroup barrier.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t pos_wide(uint32_t s, int i) { return s + 32 * i; }
__device__ __forceinline__ uint32_t pos_mid(uint32_t s, int i) { return 32 * (s >> 2) + (s & 3) + 4 * i; }
__device__ __forceinline__ uint32_t pos_narrow(uint32_t s, int i) { return 8 * s + i; }

// LDS slot of element e of column `col` in a column pass over a tile of TW
// columns: the columns interleaved (element-major) and every group of 8
// elements padded by one word.  A half-wave (TW columns x 32/TW threads) then
// touches 32 consecutive words in the wide and mid layouts and 32 / TW groups
// of TW words spread over all banks in the narrow one (TW = 16, 8, 4).
template <int TW>
__device__ __forceinline__ uint32_t col_slot(uint32_t e, uint32_t col) { return TW * (e + (e >> 3)) + col; }
constexpr int kColLds = 16 * (255 + 31 + 1);

// LDS slot of element e of a row (256 words per row): the low five bits are
// XOR-swizzled with f(e / 32), f(h) = h ^ 4h, so that the 32 threads of a row
// (one half-wave) hit 32 distinct banks in each of the three layouts.
__device__ __forceinline__ uint32_t row_slot(uint32_t e)
{
    const uint32_t h = e >> 5;
    return (e & ~31u) | ((e ^ h ^ (h << 2)) & 31u);
}
constexpr int kLds16 = kColLds > 16 * 256 ? kColLds : 16 * 256;
// Tile widths: 16 columns (rows) of the 256 x 256 view per workgroup of 512
// threads, the layout of every persistent pass and of grid launches over many
// limbs; 8 or 4 per workgroup of 256 or 128 threads for launches over few
// limbs, which then have two or four times the workgroups to spread over the
// 256 CUs.  LDS per workgroup: TW (255 + 31 + 1) words.
template <int TW>
constexpr int lds_words() { return TW * (255 + 31 + 1); }

template <int PRO, int TW, class A>
__device__ __forceinline__ void fwd_col_body(const NttArgs &a, const LimbPos &lp, const Prime &P, const A &ar,
                                             uint64_t *lds, uint32_t tile, uint32_t tx)
{
    const uint32_t col = tx & (TW - 1), s = tx / TW, c = tile * TW + col;
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 65536;
    typename A::W wa[7], wb[7], wc[6];
    typename A::V v[8];
    if (PRO == PRO_BCONV) {  // the twiddles after the conversion: not live across its loop
        bconv_load(v, ar, bc_source(a, lp.poly, lp.prime, 65536), P, 65536,
                   [&](int i) { return pos_wide(s, i) * 256 + c; });
        tw_fwd<3, 256, 32>(wa, s, ar, 1);
    } else {
        tw_fwd<3, 256, 32>(wa, s, ar, 1);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = ar.from_u64(load_fwd<PRO>(a, lp, src, pos_wide(s, i) * 256 + c, P));
    }
    fwd_rw<3>(v, wa, ar);
    tw_fwd<3, 256, 4>(wb, pos_mid(s, 0), ar, 1);  // in flight across the exchange
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[col_slot<TW>(pos_wide(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(lds[col_slot<TW>(pos_mid(s, i), col)]);
    ar.reduce_all(v);
    fwd_rw<3>(v, wb, ar);
    tw_fwd<2, 256, 1>(wc, 8 * s, ar, 1);
    tw_fwd<2, 256, 1>(wc + 3, 8 * s + 4, ar, 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[col_slot<TW>(pos_mid(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(lds[col_slot<TW>(pos_narrow(s, i), col)]);
    ar.reduce_all(v);
    fwd_rw<2>(v, wc, ar);
    fwd_rw<2>(v + 4, wc + 3, ar);
    uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536;
#pragma unroll
    for (int i = 0; i < 8; ++i) m[pos_narrow(s, i) * 256 + c] = ar.to_bits(v[i]);
}

template <int PRO, int TW = 16>
__device__ __forceinline__ void fwd_col_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                             uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        fwd_col_body<PRO, TW>(a, lp, P, fp_arith(a, P, lp.prime, 65536), lds, tile, tx);
    else
        fwd_col_body<PRO, TW>(a, lp, P, int_arith(a, P, lp.prime, 65536), lds, tile, tx);
}

template <int EPI, int TW, class A>
__device__ __forceinline__ void fwd_row_body(const NttArgs &a, const LimbPos &lp, const Prime &P, const A &ar,
                                             uint64_t *lds, uint32_t tile, uint32_t tx)
{
    const uint32_t blk = tx >> 5, s = tx & 31, b = tile * TW + blk;
    const uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536 + b * 256;
    uint64_t *L = lds + blk * 256;
    typename A::W wa[7], wb[7], wc[6];
    tw_fwd<3, 256, 32, A, true>(wa, s, ar, 256 + b);
    typename A::V v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(m[pos_wide(s, i)]);
    ar.reduce_all(v);
    fwd_rw<3>(v, wa, ar);
    tw_fwd<3, 256, 4, A, true>(wb, pos_mid(s, 0), ar, 256 + b);  // in flight across the exchange
#pragma unroll
    for (int i = 0; i < 8; ++i) L[row_slot(pos_wide(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(L[row_slot(pos_mid(s, i))]);
    ar.reduce_all(v);
    fwd_rw<3>(v, wb, ar);
    // the epilogue's operands are loaded here, so their latency overlaps the last round: the
    // subtrahend row (ModDown, Rescale) and the addend (ModDown; block b's addend under X -> X^g
    // comes from one block sb and is permuted through LDS at the end)
    uint64_t auxv[8], addv[8];
    const uint64_t *add = EPI == EPI_MODDOWN ? pick(a.add, lp.poly) : nullptr;
    uint32_t sb = b * 256;
#pragma unroll
    for (int i = 0; i < 8; ++i) auxv[i] = addv[i] = 0;
    if (EPI != EPI_PLAIN) {
        const uint64_t *ax = pick(a.aux, lp.poly) + (size_t)lp.row * 65536 + b * 256;
#pragma unroll
        for (int i = 0; i < 8; ++i) auxv[i] = ax[pos_wide(s, i)];
    }
    if (add) {
        add += (size_t)lp.row * 65536;
        if (a.galois != 1) sb = galois_src(b * 256, a.galois, 16) & ~255u;
#pragma unroll
        for (int i = 0; i < 8; ++i) addv[i] = add[sb + pos_wide(s, i)];
    }
    tw_fwd<2, 256, 1, A, true>(wc, 8 * s, ar, 256 + b);
    tw_fwd<2, 256, 1, A, true>(wc + 3, 8 * s + 4, ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 8; ++i) L[row_slot(pos_mid(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(L[row_slot(pos_narrow(s, i))]);
    ar.reduce_all(v);
    fwd_rw<2>(v, wc, ar);
    fwd_rw<2>(v + 4, wc + 3, ar);
#pragma unroll
    for (int i = 0; i < 8; ++i) L[row_slot(pos_narrow(s, i))] = ar.fwd_final(v[i]);
    wave_sync();
    uint64_t x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = L[row_slot(pos_wide(s, i))];
    if (add && a.galois != 1) {
        wave_sync();
#pragma unroll
        for (int i = 0; i < 8; ++i) L[row_slot(pos_wide(s, i))] = addv[i];
        wave_sync();
#pragma unroll
        for (int i = 0; i < 8; ++i) addv[i] = L[row_slot(galois_src(b * 256 + pos_wide(s, i), a.galois, 16) - sb)];
    }
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 65536;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        store_fwd<EPI>(a, lp, dst, b * 256 + pos_wide(s, i), x[i], addv[i], auxv[i], P, 65536);
}

template <int EPI, int TW = 16>
__device__ __forceinline__ void fwd_row_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                             uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        fwd_row_body<EPI, TW>(a, lp, P, fp_arith(a, P, lp.prime, 65536), lds, tile, tx);
    else
        fwd_row_body<EPI, TW>(a, lp, P, int_arith(a, P, lp.prime, 65536), lds, tile, tx);
}

template <int PRO, int TW, class A>
__device__ __forceinline__ void inv_row_body(const NttArgs &a, const LimbPos &lp, const Prime &P, const A &ar,
                                             uint64_t *lds, uint32_t tile, uint32_t tx)
{
    const uint32_t blk = tx >> 5, s = tx & 31, b = tile * TW + blk;
    const size_t row_off = (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 65536;
    const uint64_t *src = a.src + row_off;
    uint64_t *L = lds + blk * 256;
    typename A::W wa[6], wb[7], wc[7];
    tw_inv<2, 256, 1, A, true>(wa, 8 * s, ar, 256 + b);
    tw_inv<2, 256, 1, A, true>(wa + 3, 8 * s + 4, ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t e = b * 256 + pos_wide(s, i);
        if (PRO == PRO_TENSOR)  // HMult's d2 = a1 b1, formed on the fly in the limb's arithmetic
            L[row_slot(pos_wide(s, i))] = ar.to_bits(ar.product(src[e], a.src2[row_off + e], P));
        else
            L[row_slot(pos_wide(s, i))] = src[PRO == PRO_GALOIS ? galois_src(e, a.galois, 16) : e];
    }
    wave_sync();
    typename A::V v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        v[i] = PRO == PRO_TENSOR ? ar.from_bits(L[row_slot(pos_narrow(s, i))]) : ar.from_u64(L[row_slot(pos_narrow(s, i))]);
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    inv_rw<2>(v + 4, wa + 3, ar);
    tw_inv<3, 256, 4, A, true>(wb, pos_mid(s, 0), ar, 256 + b);  // in flight across the exchange
#pragma unroll
    for (int i = 0; i < 8; ++i) L[row_slot(pos_narrow(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(L[row_slot(pos_mid(s, i))]);
    ar.reduce_all(v);
    inv_rw<3>(v, wb, ar);
    tw_inv<3, 256, 32, A, true>(wc, s, ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 8; ++i) L[row_slot(pos_mid(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(L[row_slot(pos_wide(s, i))]);
    ar.reduce_all(v);
    inv_rw<3>(v, wc, ar);
    uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536 + b * 256;
#pragma unroll
    for (int i = 0; i < 8; ++i) m[pos_wide(s, i)] = ar.to_bits(v[i]);
}

template <int PRO, int TW = 16>
__device__ __forceinline__ void inv_row_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                             uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        inv_row_body<PRO, TW>(a, lp, P, fp_arith(a, P, lp.prime, 65536), lds, tile, tx);
    else
        inv_row_body<PRO, TW>(a, lp, P, int_arith(a, P, lp.prime, 65536), lds, tile, tx);
}

template <int TW, class A>
__device__ __forceinline__ void inv_col_body(const NttArgs &a, const LimbPos &lp, const A &ar, uint64_t *lds,
                                             uint32_t tile, uint32_t tx)
{
    const uint32_t col = tx & (TW - 1), s = tx / TW, c = tile * TW + col;
    const uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536;
    typename A::W wa[6], wb[7], wc[7];
    tw_inv<2, 256, 1>(wa, 8 * s, ar, 1);
    tw_inv<2, 256, 1>(wa + 3, 8 * s + 4, ar, 1);
    typename A::V v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(m[pos_narrow(s, i) * 256 + c]);
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    inv_rw<2>(v + 4, wa + 3, ar);
    tw_inv<3, 256, 4>(wb, pos_mid(s, 0), ar, 1);  // in flight across the exchange
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[col_slot<TW>(pos_narrow(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(lds[col_slot<TW>(pos_mid(s, i), col)]);
    ar.reduce_all(v);
    inv_rw<3>(v, wb, ar);
    tw_inv<3, 256, 32>(wc, s, ar, 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[col_slot<TW>(pos_mid(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = ar.from_bits(lds[col_slot<TW>(pos_wide(s, i), col)]);
    ar.reduce_all(v);
    inv_rw<3>(v, wc, ar);
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 65536;
    inv_store(dst, v, ar, a.ys_mode, [&](int i) { return pos_wide(s, i) * 256 + c; });
}

template <int TW = 16>
__device__ __forceinline__ void inv_col_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                             uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        inv_col_body<TW>(a, lp, inv_fp_arith(a, lp, P, 65536), lds, tile, tx);
    else
        inv_col_body<TW>(a, lp, inv_int_arith(a, lp, P, 65536), lds, tile, tx);
}

// Inverse passes with 4 elements per thread, 64 threads per 256-point problem,
// for launches over few limbs: those are latency-bound with one wave per SIMD
// in the 8-element layout, and this one gives them twice the waves.  A
// workgroup of 512 threads takes 8 rows (one wave each) or 8 columns.  Rounds
// of two stages (t = 1, 2 | 4, 8 | 16, 32 | 64, 128) in four layouts, thread
// s < 64 holding positions
//   A 4s + i,  B 16 (s/4) + s%4 + 4i,  C 64 (s/16) + s%16 + 16i,  D s + 64i.
__device__ __forceinline__ uint32_t p4a(uint32_t s, int i) { return 4 * s + i; }
__device__ __forceinline__ uint32_t p4b(uint32_t s, int i) { return 16 * (s >> 2) + (s & 3) + 4 * i; }
__device__ __forceinline__ uint32_t p4c(uint32_t s, int i) { return 64 * (s >> 4) + (s & 15) + 16 * i; }
__device__ __forceinline__ uint32_t p4d(uint32_t s, int i) { return s + 64 * i; }
// LDS slot of element e of a row (256 words): the low five bits XOR-ed with
// 9 (e/32) and 4 (e/64) (mod 32), so that each half-wave hits 32 distinct
// 8-byte banks in all four layouts (checked exhaustively on the host).
__device__ __forceinline__ uint32_t row4_slot(uint32_t e)
{
    return (e & ~31u) | ((e ^ (9 * (e >> 5)) ^ (4 * (e >> 6))) & 31u);
}
// LDS slot of element e of column `col` of an 8-column tile: columns
// interleaved, one word of padding every 4 elements (conflict-free likewise).
__device__ __forceinline__ uint32_t col4_slot(uint32_t e, uint32_t col) { return 8 * (e + (e >> 2)) + col; }
constexpr int kLds4 = 8 * (255 + 63 + 1);

// The rounds of one row: thread s < 64 of the row's wave, element loads
// load(i) at position p4a(s, i), scratch L (256 words), output row m.
template <class A, class Load>
__device__ __forceinline__ void inv_row4_rounds(const A &ar, uint64_t *L, uint32_t s, uint32_t b, Load load,
                                                uint64_t *m)
{
    typename A::W wa[3], wb[3];
    typename A::V v[4];
    tw_inv<2, 256, 1, A, true>(wa, p4a(s, 0), ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_u64(load(i));
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    tw_inv<2, 256, 4, A, true>(wb, p4b(s, 0), ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 4; ++i) L[row4_slot(p4a(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(L[row4_slot(p4b(s, i))]);
    ar.reduce_all(v);
    inv_rw<2>(v, wb, ar);
    tw_inv<2, 256, 16, A, true>(wa, p4c(s, 0), ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 4; ++i) L[row4_slot(p4b(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(L[row4_slot(p4c(s, i))]);
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    tw_inv<2, 256, 64, A, true>(wb, p4d(s, 0), ar, 256 + b);
#pragma unroll
    for (int i = 0; i < 4; ++i) L[row4_slot(p4c(s, i))] = ar.to_bits(v[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(L[row4_slot(p4d(s, i))]);
    ar.reduce_all(v);
    inv_rw<2>(v, wb, ar);
#pragma unroll
    for (int i = 0; i < 4; ++i) m[p4d(s, i)] = ar.to_bits(v[i]);
}

template <class A>
__device__ __forceinline__ void inv_row4_body(const NttArgs &a, const LimbPos &lp, const A &ar, uint64_t *lds,
                                              uint32_t tile, uint32_t tx)
{
    const uint32_t blk = tx >> 6, s = tx & 63, b = tile * 8 + blk;
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 65536 + b * 256;
    uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536 + b * 256;
    inv_row4_rounds(ar, lds + blk * 256, s, b, [&](int i) { return src[p4a(s, i)]; }, m);
}

template <class A>
__device__ __forceinline__ void inv_col4_body(const NttArgs &a, const LimbPos &lp, const A &ar, uint64_t *lds,
                                              uint32_t tile, uint32_t tx)
{
    const uint32_t col = tx & 7, s = tx >> 3, c = tile * 8 + col;
    const uint64_t *m = a.mid + (int64_t)lp.poly * a.mid_stride + (size_t)lp.row * 65536;
    typename A::W wa[3], wb[3];
    typename A::V v[4];
    tw_inv<2, 256, 1>(wa, p4a(s, 0), ar, 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(m[p4a(s, i) * 256 + c]);
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    tw_inv<2, 256, 4>(wb, p4b(s, 0), ar, 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) lds[col4_slot(p4a(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(lds[col4_slot(p4b(s, i), col)]);
    ar.reduce_all(v);
    inv_rw<2>(v, wb, ar);
    tw_inv<2, 256, 16>(wa, p4c(s, 0), ar, 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) lds[col4_slot(p4b(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(lds[col4_slot(p4c(s, i), col)]);
    ar.reduce_all(v);
    inv_rw<2>(v, wa, ar);
    tw_inv<2, 256, 64>(wb, p4d(s, 0), ar, 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) lds[col4_slot(p4c(s, i), col)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ar.from_bits(lds[col4_slot(p4d(s, i), col)]);
    ar.reduce_all(v);
    inv_rw<2>(v, wb, ar);
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 65536;
    inv_store(dst, v, ar, a.ys_mode, [&](int i) { return p4d(s, i) * 256 + c; });
}

__device__ __forceinline__ void inv_row4_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                              uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        inv_row4_body(a, lp, fp_arith(a, P, lp.prime, 65536), lds, tile, tx);
    else
        inv_row4_body(a, lp, int_arith(a, P, lp.prime, 65536), lds, tile, tx);
}

__device__ __forceinline__ void inv_col4_unit(const NttArgs &a, uint32_t limb, uint32_t tile, uint64_t *lds,
                                              uint32_t tx)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        inv_col4_body(a, lp, inv_fp_arith(a, lp, P, 65536), lds, tile, tx);
    else
        inv_col4_body(a, lp, inv_int_arith(a, lp, P, 65536), lds, tile, tx);
}

// ------------------------------------------------------------------ N = 2^12

template <int PRO, int EPI, class A>
__device__ __forceinline__ void fwd12_body(const NttArgs &a, const LimbPos &lp, const Prime &P, const A &ar,
                                           uint64_t *lds)
{
    const uint32_t t = threadIdx.x, base2 = (t >> 4) * 256 + (t & 15);
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 4096;
    typename A::V v[16];
    if (PRO == PRO_BCONV) {
        bconv_load(v, ar, bc_source(a, lp.poly, lp.prime, 4096), P, 4096, [&](int i) { return t + 256 * i; });
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = ar.from_u64(load_fwd<PRO>(a, lp, src, t + 256 * i, P));
    }
    fwd16<4096, 256>(v, t, ar, 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(t + 256 * i)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = ar.from_bits(lds[pad(base2 + 16 * i)]);
    ar.reduce_all(v);
    fwd16<4096, 16>(v, base2, ar, 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(base2 + 16 * i)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = ar.from_bits(lds[pad(16 * t + i)]);
    ar.reduce_all(v);
    fwd16<4096, 1>(v, 16 * t, ar, 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(16 * t + i)] = ar.fwd_final(v[i]);
    __syncthreads();
    uint64_t x[16], addv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        x[i] = lds[pad(t + 256 * i)];
        addv[i] = 0;
    }
    const uint64_t *add = EPI == EPI_MODDOWN ? pick(a.add, lp.poly) : nullptr;
    if (add) {
        add += (size_t)lp.row * 4096;
        if (a.galois == 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) addv[i] = add[t + 256 * i];
        } else {  // the whole limb's addend through LDS, then permuted
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) lds[pad(t + 256 * i)] = add[t + 256 * i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) addv[i] = lds[pad(galois_src(t + 256 * i, a.galois, 12))];
        }
    }
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 4096;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint64_t auxv = EPI == EPI_PLAIN ? 0 : pick(a.aux, lp.poly)[(size_t)lp.row * 4096 + t + 256 * i];
        store_fwd<EPI>(a, lp, dst, t + 256 * i, x[i], addv[i], auxv, P, 4096);
    }
}

template <int PRO, int EPI>
__device__ __forceinline__ void fwd12_unit(const NttArgs &a, uint32_t limb, uint32_t, uint64_t *lds, uint32_t)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        fwd12_body<PRO, EPI>(a, lp, P, fp_arith(a, P, lp.prime, 4096), lds);
    else
        fwd12_body<PRO, EPI>(a, lp, P, int_arith(a, P, lp.prime, 4096), lds);
}

template <int PRO, class A>
__device__ __forceinline__ void inv12_body(const NttArgs &a, const LimbPos &lp, const A &ar, uint64_t *lds)
{
    const uint32_t t = threadIdx.x, base2 = (t >> 4) * 256 + (t & 15);
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 4096;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t e = t + 256 * i;
        lds[pad(e)] = src[PRO == PRO_GALOIS ? galois_src(e, a.galois, 12) : e];
    }
    __syncthreads();
    typename A::V v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = ar.from_u64(lds[pad(16 * t + i)]);
    ar.reduce_all(v);
    inv16<4096, 1>(v, 16 * t, ar, 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(16 * t + i)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = ar.from_bits(lds[pad(base2 + 16 * i)]);
    ar.reduce_all(v);
    inv16<4096, 16>(v, base2, ar, 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(base2 + 16 * i)] = ar.to_bits(v[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = ar.from_bits(lds[pad(t + 256 * i)]);
    ar.reduce_all(v);
    inv16<4096, 256>(v, t, ar, 1);
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 4096;
    inv_store(dst, v, ar, a.ys_mode, [&](int i) { return t + 256 * i; });
}

template <int PRO>
__device__ __forceinline__ void inv12_unit(const NttArgs &a, uint32_t limb, uint32_t, uint64_t *lds, uint32_t)
{
    const LimbPos lp = limb_pos(a.map, limb);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    if (P.q < kFpMaxPrime)
        inv12_body<PRO>(a, lp, inv_fp_arith(a, lp, P, 4096), lds);
    else
        inv12_body<PRO>(a, lp, inv_int_arith(a, lp, P, 4096), lds);
}

// ---------------------------------------------------- kernels: grid and queue
// Every NTT stage exists as a grid kernel (one launch = one NttArgs, unit =
// (blockIdx.x, blockIdx.y)) and as a persistent kernel that claims units
// (instance, limb, tile) of many launches from a work queue, so a whole batch
// of ciphertexts at different levels goes through one launch per stage.

__device__ __forceinline__ UnitId grid_unit(const NttArgs &a)
{
    if (gridDim.x != 16 || (a.map.skip_alpha != 0 && !a.map.dense)) {  // N = 2^12, or skipped limbs in the grid
        UnitId u;
        u.limb = blockIdx.y;
        u.tile = blockIdx.x;
        return u;
    }
    return unit_of(blockIdx.y * 16 + blockIdx.x, gridDim.y, a.n_heavy, a.heavy);
}

constexpr int kLds12 = 4352;

// Persistent kernels at N = 2^16 read their argument block with scalar loads
// (run_work_queue_uniform).  Those at N = 2^12 keep it in LDS: with 16
// elements per thread they already need close to the scalar register file,
// and a scalar copy would spill to scratch.
#define NTT_KERNELS(NAME, LDS, THREADS, UNIFORM, GRID_ATTR, ...)                                \
    __global__ __launch_bounds__(THREADS) GRID_ATTR void k_##NAME(NttArgs a)                     \
    {                                                                                             \
        __shared__ uint64_t lds[LDS];                                                             \
        const UnitId u = grid_unit(a);                                                            \
        __VA_ARGS__(a, u.limb, u.tile, lds, threadIdx.x);                                         \
    }                                                                                             \
    __global__ __launch_bounds__(THREADS) void q_##NAME(const NttArgs *insts, WorkQueue q)        \
    {                                                                                             \
        __shared__ uint64_t lds[LDS];                                                             \
        __shared__ uint32_t claim;                                                                \
        auto body = [&](const NttArgs &a, uint32_t limb, uint32_t tile) {                        \
            __VA_ARGS__(a, limb, tile, lds, UNIFORM ? thread_index() : threadIdx.x);              \
        };                                                                                        \
        if constexpr (UNIFORM) {                                                                  \
            run_work_queue_uniform(insts, q, &claim, body);                                       \
        } else {                                                                                  \
            __shared__ NttArgs sa;                                                                \
            run_work_queue(insts, q, sa, &claim, body);                                           \
        }                                                                                         \
    }

// Three 512-thread workgroups per CU for the plain passes: the column passes
// fit in 72 VGPRs; the row passes spill 12 to 16 bytes per lane and still gain
// over 35 limbs (not over 74, and the tensor prologue's pass loses, so it
// keeps two workgroups per CU).
#define OCC6 __attribute__((amdgpu_waves_per_eu(6)))

NTT_KERNELS(fwd_col_plain, kLds16, kThreads16, true, OCC6, fwd_col_unit<PRO_PLAIN>)
NTT_KERNELS(fwd_col_rescale, kLds16, kThreads16, true, , fwd_col_unit<PRO_RESCALE>)
NTT_KERNELS(fwd_col_bconv, kLds16, kThreads16, true, , fwd_col_unit<PRO_BCONV>)
NTT_KERNELS(fwd_row_plain, kLds16, kThreads16, true, OCC6, fwd_row_unit<EPI_PLAIN>)
NTT_KERNELS(fwd_row_moddown, kLds16, kThreads16, true, , fwd_row_unit<EPI_MODDOWN>)
NTT_KERNELS(fwd_row_rescale, kLds16, kThreads16, true, , fwd_row_unit<EPI_RESCALE>)
NTT_KERNELS(inv_row_plain, kLds16, kThreads16, true, OCC6, inv_row_unit<PRO_PLAIN>)
NTT_KERNELS(inv_row_galois, kLds16, kThreads16, true, , inv_row_unit<PRO_GALOIS>)
NTT_KERNELS(inv_row_tensor, kLds16, kThreads16, true, , inv_row_unit<PRO_TENSOR>)
NTT_KERNELS(inv_col, kLds16, kThreads16, true, OCC6, inv_col_unit)
// Grid kernels with narrower tiles (TW = 8, 4 columns or rows per workgroup of
// 32 TW threads), for launches over few limbs; unit = (blockIdx.x, blockIdx.y).
#define NTT_NARROW(NAME, UNIT_T)                                                                    \
    __global__ __launch_bounds__(256) void k_##NAME##_w8(NttArgs a)                                \
    {                                                                                               \
        __shared__ uint64_t lds[lds_words<8>()];                                                    \
        UNIT_T(8)(a, blockIdx.y, blockIdx.x, lds, threadIdx.x);                                     \
    }                                                                                               \
    __global__ __launch_bounds__(128) void k_##NAME##_w4(NttArgs a)                                \
    {                                                                                               \
        __shared__ uint64_t lds[lds_words<4>()];                                                    \
        UNIT_T(4)(a, blockIdx.y, blockIdx.x, lds, threadIdx.x);                                     \
    }
// The 4-element inverse passes (tile code 2: 8 rows or columns, 512 threads).
__global__ __launch_bounds__(512) void k_inv_row4(NttArgs a)
{
    __shared__ uint64_t lds[kLds4];
    inv_row4_unit(a, blockIdx.y, blockIdx.x, lds, threadIdx.x);
}
__global__ __launch_bounds__(512) void k_inv_col4(NttArgs a)
{
    __shared__ uint64_t lds[kLds4];
    inv_col4_unit(a, blockIdx.y, blockIdx.x, lds, threadIdx.x);
}
#define U_FCP(W) fwd_col_unit<PRO_PLAIN, W>
#define U_FCR(W) fwd_col_unit<PRO_RESCALE, W>
#define U_FCB(W) fwd_col_unit<PRO_BCONV, W>
#define U_FRP(W) fwd_row_unit<EPI_PLAIN, W>
#define U_FRM(W) fwd_row_unit<EPI_MODDOWN, W>
#define U_FRR(W) fwd_row_unit<EPI_RESCALE, W>
#define U_IRP(W) inv_row_unit<PRO_PLAIN, W>
#define U_IRG(W) inv_row_unit<PRO_GALOIS, W>
#define U_IRT(W) inv_row_unit<PRO_TENSOR, W>
#define U_IC(W) inv_col_unit<W>
NTT_NARROW(fwd_col_plain, U_FCP)
NTT_NARROW(fwd_col_rescale, U_FCR)
NTT_NARROW(fwd_col_bconv, U_FCB)
NTT_NARROW(fwd_row_plain, U_FRP)
NTT_NARROW(fwd_row_moddown, U_FRM)
NTT_NARROW(fwd_row_rescale, U_FRR)
NTT_NARROW(inv_row_plain, U_IRP)
NTT_NARROW(inv_row_galois, U_IRG)
NTT_NARROW(inv_row_tensor, U_IRT)
NTT_NARROW(inv_col, U_IC)
#undef U_FCP
#undef U_FCR
#undef U_FCB
#undef U_FRP
#undef U_FRM
#undef U_FRR
#undef U_IRP
#undef U_IRG
#undef U_IRT
#undef U_IC
#undef NTT_NARROW

#define FWD12_PP fwd12_unit<PRO_PLAIN, EPI_PLAIN>
#define FWD12_PM fwd12_unit<PRO_PLAIN, EPI_MODDOWN>
#define FWD12_RR fwd12_unit<PRO_RESCALE, EPI_RESCALE>
#define FWD12_RP fwd12_unit<PRO_RESCALE, EPI_PLAIN>
#define FWD12_BM fwd12_unit<PRO_BCONV, EPI_MODDOWN>
NTT_KERNELS(fwd12_plain, kLds12, kThreads, false, , FWD12_PP)
NTT_KERNELS(fwd12_moddown, kLds12, kThreads, false, , FWD12_PM)
NTT_KERNELS(fwd12_rescale, kLds12, kThreads, false, , FWD12_RR)
NTT_KERNELS(fwd12_lift, kLds12, kThreads, false, , FWD12_RP)
NTT_KERNELS(fwd12_bconv_moddown, kLds12, kThreads, false, , FWD12_BM)
NTT_KERNELS(inv12_plain, kLds12, kThreads, false, , inv12_unit<PRO_PLAIN>)
NTT_KERNELS(inv12_galois, kLds12, kThreads, false, , inv12_unit<PRO_GALOIS>)
#undef FWD12_PP
#undef FWD12_PM
#undef FWD12_RR
#undef FWD12_RP
#undef FWD12_BM
#undef NTT_KERNELS
#undef OCC6

// ------------------------------------------- one launch for a whole batch
// The persistent kernel of a batch of key switches in one launch (N = 2^16):
// every step of every key switch is a group of units in one list, and a unit
// starts once the group it depends on (the previous step of the same key
// switch) is done, so the steps of different key switches overlap instead of
// meeting at eleven launch boundaries.  Dependencies go through per-group
// counters: a unit's stores are complete in every wave before the workgroup
// counts it done with an agent-scope release, and a waiting workgroup
// acquires at agent scope before it reads, which makes the data of other
// workgroups, on any XCD, visible.  The coefficient-wise steps run their
// 256-thread units on the two halves of the 512-thread workgroup, each half
// taking eight of the unit's sixteen 256-coefficient blocks.
//
constexpr uint32_t kFusedIpStage = 2 * coef::kIpStage * coef::kCoefThreads;
constexpr int kFusedLds = kLds16 > (int)kFusedIpStage ? kLds16 : (int)kFusedIpStage;
static_assert(kQueueBlocks % 2 == 0, "the two halves take half of a unit's blocks each");

__shared__ uint64_t g_fused_lds[kFusedLds];
__shared__ BconvArgs g_fused_bc;

// Completions a workgroup has not yet published: up to f.publish_every
// (at most kFusedPending) groups with their unit counts, kept by thread 0.
// Publishing costs one agent-scope release (a write-back of the XCD's L2), so
// it is done for several units at once: when publish_every groups are
// pending, before the workgroup blocks on a wait, and when it runs out of
// units.  A workgroup that blocks has published everything it finished, so
// the earliest unfinished unit can always proceed, and a workgroup that does
// not block publishes within publish_every units.
constexpr uint32_t kFusedPending = 32;
constexpr uint32_t kFusedSeen = 4;
struct Pending {
    uint32_t group[kFusedPending], count[kFusedPending], n;
    // groups this workgroup has seen complete (and acquired after): a later unit waiting for one of
    // them needs neither a poll nor another acquire, since a complete group's data no longer changes
    uint32_t seen[kFusedSeen], seen_next;
};

__device__ __forceinline__ void fused_publish(const FusedArgs &f, Pending &p)
{
    if (p.n == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (uint32_t i = 0; i < p.n; ++i)
        __hip_atomic_fetch_add(f.done + (size_t)p.group[i] * f.done_stride, p.count[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    p.n = 0;
}

__device__ __forceinline__ void fused_finished(const FusedArgs &f, Pending &p, uint32_t g)
{
    for (uint32_t i = 0; i < p.n; ++i)
        if (p.group[i] == g) {
            ++p.count[i];
            return;
        }
    p.group[p.n] = g;
    p.count[p.n] = 1;
    if (++p.n >= f.publish_every) fused_publish(f, p);
}

// Waits (thread 0 only) until every unit of group g is done, publishing the
// workgroup's own completions first if it has to wait; gives up after
// spin_limit polls and raises the fault flag, so that the launch always ends.
__device__ __forceinline__ void fused_wait(const FusedArgs &f, Pending &p, uint32_t g)
{
    for (uint32_t i = 0; i < kFusedSeen; ++i)
        if (p.seen[i] == g) return;
    const uint32_t want = f.target[g];
    const uint32_t *cnt = f.done + (size_t)g * f.done_stride;
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        fused_publish(f, p);
        uint32_t polls = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
            if (++polls > f.spin_limit) {
                __hip_atomic_store(f.fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    p.seen[p.seen_next] = g;
    p.seen_next = (p.seen_next + 1) % kFusedSeen;
}

template <class Args>
__device__ __forceinline__ Args uniform_args(const Args *base, uint32_t inst)
{
    typedef const __attribute__((address_space(4))) uint32_t ConstWord;
    static_assert(sizeof(Args) % 4 == 0, "argument blocks are read as 4-byte words");
    ConstWord *src = (ConstWord *)((uintptr_t)base + (uintptr_t)inst * sizeof(Args));
    Args a;
#pragma unroll
    for (uint32_t i = 0; i < sizeof(Args) / 4; ++i) ((uint32_t *)&a)[i] = src[i];
    return a;
}

// The argument block of the unit's step: the pointer passes through an empty
// asm statement, so that the scalar loads of one step's block are not
// hoisted above the switch (speculated for every step, the blocks of all
// steps would be live at once).
template <class Args>
__device__ __forceinline__ Args step_args(const Args *base, uint32_t inst)
{
    uint64_t p = (uint64_t)(uintptr_t)base;
    asm volatile("" : "+s"(p));
    return uniform_args((const Args *)(uintptr_t)p, inst);
}

__global__ __launch_bounds__(kThreads16) __attribute__((amdgpu_waves_per_eu(4))) void q_fused16(FusedArgs f)
{
    typedef const __attribute__((address_space(4))) uint32_t ConstWord;
    __shared__ uint32_t claim;
    __shared__ Pending pend;  // thread 0's
    if (threadIdx.x == 0) {
        claim = atomicAdd(f.claim, 1u);
        pend.n = 0;
        for (uint32_t i = 0; i < kFusedSeen; ++i) pend.seen[i] = kNoGroup;
        pend.seen_next = 0;
    }
    __syncthreads();
    uint32_t u = __builtin_amdgcn_readfirstlane(claim);
    uint32_t have_bc = 0xFFFFFFFFu;
    while (u < f.nunits) {
        ConstWord *w = (ConstWord *)((uintptr_t)f.units + (uintptr_t)u * sizeof(FusedUnit));
        const uint32_t inst = __builtin_amdgcn_readfirstlane(w[0]);
        const uint32_t code = __builtin_amdgcn_readfirstlane(w[1]);
        const uint32_t wait = __builtin_amdgcn_readfirstlane(w[2]);
        const uint32_t signal = __builtin_amdgcn_readfirstlane(w[3]);
        __syncthreads();  // every thread has read claim and is done with the previous unit's LDS
        if (threadIdx.x == 0) claim = atomicAdd(f.claim, 1u);
        if (wait != kNoGroup) {
            if (threadIdx.x == 0) fused_wait(f, pend, wait);
            __syncthreads();
        }
        const uint32_t step = code >> 28, tile = (code >> 16) & 0xFFFu, limb = code & 0xFFFFu;
        // the thread index is taken anew for every unit: offsets derived from it and hoisted out of
        // the loop would stay live across every step's body
        const uint32_t tx = thread_index();
        switch (step) {
        case QI_TENSOR: {
            const TensorArgs a = step_args(f.tensor, inst);
            for (uint32_t i = tx / coef::kCoefThreads; i < kQueueBlocks; i += 2)
                coef::tensor_unit(a, limb, tile * kQueueBlocks + i, tx % coef::kCoefThreads);
            break;
        }
        case QI_UP_INTT0_PLAIN: inv_row_unit<PRO_PLAIN>(step_args(f.ntt[0], inst), limb, tile, g_fused_lds, tx); break;
        case QI_UP_INTT0_GALOIS: inv_row_unit<PRO_GALOIS>(step_args(f.ntt[0], inst), limb, tile, g_fused_lds, tx); break;
        case QI_UP_INTT1: inv_col_unit(step_args(f.ntt[0], inst), limb, tile, g_fused_lds, tx); break;
        case QI_UP_BCONV: {
            if (inst != have_bc) {  // its job fields are indexed per thread: the block goes through LDS
                const uint64_t *src = (const uint64_t *)(f.bconv + inst);
                uint64_t *dst = (uint64_t *)&g_fused_bc;
                for (uint32_t i = threadIdx.x; i < sizeof(BconvArgs) / 8; i += blockDim.x) dst[i] = src[i];
                have_bc = inst;
                __syncthreads();
            }
            const uint32_t nb = g_fused_bc.N / (coef::kCoefThreads * kQueueBlocks);
            for (uint32_t i = tx / coef::kCoefThreads; i < kQueueBlocks; i += 2)
                coef::bconv_unit(g_fused_bc, limb, (tile % nb) * kQueueBlocks + i, tile / nb, tx % coef::kCoefThreads);
            break;
        }
        case QI_UP_NTT0: fwd_col_unit<PRO_PLAIN>(step_args(f.ntt[1], inst), limb, tile, g_fused_lds, tx); break;
        case QI_UP_NTT1: fwd_row_unit<EPI_PLAIN>(step_args(f.ntt[1], inst), limb, tile, g_fused_lds, tx); break;
        case QI_IP: {
            const uint32_t half = tx / coef::kCoefThreads;
            coef::ip_blocks(step_args(f.ip, inst), limb, tile * kQueueBlocks + half * (kQueueBlocks / 2),
                            kQueueBlocks / 2, g_fused_lds + half * coef::kIpStage * coef::kCoefThreads,
                            tx % coef::kCoefThreads);
            break;
        }
        case QI_DN_INTT0: inv_row_unit<PRO_PLAIN>(step_args(f.ntt[2], inst), limb, tile, g_fused_lds, tx); break;
        case QI_DN_INTT1: inv_col_unit(step_args(f.ntt[2], inst), limb, tile, g_fused_lds, tx); break;
        case QI_DN_NTT0: fwd_col_unit<PRO_BCONV>(step_args(f.ntt[3], inst), limb, tile, g_fused_lds, tx); break;
        case QI_DN_NTT1: fwd_row_unit<EPI_MODDOWN>(step_args(f.ntt[3], inst), limb, tile, g_fused_lds, tx); break;
        default: break;
        }
        // the barrier does not wait for global stores: every wave waits for its own first, so
        // the unit's stores are complete before thread 0 records (and later publishes) it
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        if (threadIdx.x == 0) fused_finished(f, pend, signal);
        u = __builtin_amdgcn_readfirstlane(claim);
    }
    if (threadIdx.x == 0) fused_publish(f, pend);
}

typedef void (*GridKernel)(NttArgs);
typedef void (*QueueKernel)(const NttArgs *, WorkQueue);

struct StageKernels {
    GridKernel grid;
    QueueKernel queue;
};

// The key inner product (N = 2^16) with the first inverse pass of ModDown's
// special rows run by the same workgroups (Sec. III-F.5: the inner product
// feeds ModDown directly).  A block bx of 256 coefficients of a row is the
// 256-point row problem b = bx of that row's inverse NTT, so a workgroup of a
// special row reduces its sums over two blocks, stages them in LDS, and its
// four waves run the row passes (4 elements per thread), writing their output
// where ModDown's INTT keeps it; the INTT then runs its column pass only.  The
// special rows' accumulators never reach memory.  Their workgroups come first
// in the launch, so their longer units overlap the q-rows' streaming instead
// of forming its tail.  `ia` is ModDown's INTT (the rows p_0..p_{K-1} of both
// accumulators, in that order).
constexpr uint32_t kIpRowpassLds = coef::kIpStage * coef::kCoefThreads + 4 * 256;

template <bool TENSOR>
__device__ __forceinline__ void ip_rowpass_unit(const IpArgs &ip, const NttArgs &ia, uint32_t y, uint32_t bx,
                                                uint64_t *lds, uint32_t tid)
{
    const uint32_t nqr = ip.level + 1, nsp = ip.rows - nqr;
    const uint32_t r = y < nsp ? nqr + y : y - nsp;
    if (r < nqr) {
        if (TENSOR)
            coef::ip_unit_tensor(ip, r, bx, tid);
        else
            coef::ip_unit(ip, r, bx, lds, tid);
        return;
    }
    // a special row: blocks 2 bx and 2 bx + 1 (the upper half of the grid row has no work), so
    // that all four waves run a row pass (block 2 bx + w / 2, polynomial w % 2)
    if (bx >= (1u << ip.logn) / (2 * coef::kCoefThreads)) return;
    uint64_t v[4];
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
        const coef::RegStore st{&v[2 * h], &v[2 * h + 1]};
        if (TENSOR)
            coef::ip_unit_tensor(ip, r, 2 * bx + h, tid, st);
        else
            coef::ip_unit(ip, r, 2 * bx + h, lds, tid, st);
    }
    // the four rows' inputs; after the barrier the staging area is the row passes' scratch
    uint64_t *in = lds + coef::kIpStage * coef::kCoefThreads;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) in[i * coef::kCoefThreads + tid] = v[i];
    __syncthreads();
    const uint32_t w = tid >> 6, s = tid & 63, k = r - nqr, prime = ip.nq + k;
    const uint32_t poly = w & 1, b = 2 * bx + (w >> 1);
    const Prime P = ia.primes[prime];
    const uint64_t *x = in + ((w >> 1) * 2 + poly) * coef::kCoefThreads;
    uint64_t *L = lds + w * 256;
    uint64_t *m = ia.mid + (int64_t)poly * ia.mid_stride + (size_t)k * 65536 + b * 256;
    auto load = [&](int i) { return x[p4a(s, i)]; };
    if (P.q < kFpMaxPrime)
        inv_row4_rounds(fp_arith(ia, P, prime, 65536), L, s, b, load, m);
    else
        inv_row4_rounds(int_arith(ia, P, prime, 65536), L, s, b, load, m);
}

__global__ __launch_bounds__(coef::kCoefThreads) void k_inner_product_rowpass(IpArgs ip, NttArgs ia)
{
    __shared__ uint64_t lds[kIpRowpassLds];
    ip_rowpass_unit<false>(ip, ia, blockIdx.y, blockIdx.x, lds, threadIdx.x);
}

__global__ __launch_bounds__(coef::kCoefThreads) void k_inner_product_tensor_rowpass(IpArgs ip, NttArgs ia)
{
    __shared__ uint64_t lds[kIpRowpassLds];
    ip_rowpass_unit<true>(ip, ia, blockIdx.y, blockIdx.x, lds, threadIdx.x);
}

// The kernel that runs one pass of a stage (pass 0 = first, 1 = second at N =
// 2^16) with tiles of tw columns (rows); the narrow tiles have grid kernels only.
bool stage_kernels(NttStage st, uint32_t logn, int pass, StageKernels &k, uint32_t tw = 16)
{
#define SK(G) \
    k.grid = tw == 8 ? k_##G##_w8 : tw == 4 ? k_##G##_w4 : k_##G; \
    k.queue = tw == 16 ? q_##G : nullptr; \
    return true;
#define SK12(G) \
    k.grid = k_##G; \
    k.queue = q_##G; \
    return true;
    if (logn == 12) {
        if (pass != 0) return false;
        switch (st) {
        case STAGE_FWD_PLAIN: SK12(fwd12_plain)
        case STAGE_FWD_MODDOWN: SK12(fwd12_moddown)
        case STAGE_FWD_RESCALE: SK12(fwd12_rescale)
        case STAGE_FWD_LIFT: SK12(fwd12_lift)
        case STAGE_FWD_BCONV_MODDOWN: SK12(fwd12_bconv_moddown)
        case STAGE_INV_PLAIN: SK12(inv12_plain)
        case STAGE_INV_GALOIS: SK12(inv12_galois)
        default: return false;
        }
    }
    if (tw == 2) {  // 4 elements per thread: the column pass of every inverse, the plain row pass
        const bool inv = st == STAGE_INV_PLAIN || st == STAGE_INV_GALOIS || st == STAGE_INV_TENSOR;
        if (inv && (pass == 1 || st == STAGE_INV_PLAIN)) {
            k.grid = pass == 0 ? k_inv_row4 : k_inv_col4;
            k.queue = nullptr;
            return true;
        }
        tw = 8;  // the other row passes take tiles of 8
    }
    switch (st) {
    case STAGE_FWD_PLAIN:
        if (pass == 0) { SK(fwd_col_plain) } else { SK(fwd_row_plain) }
    case STAGE_FWD_MODDOWN:
        if (pass == 0) { SK(fwd_col_plain) } else { SK(fwd_row_moddown) }
    case STAGE_FWD_RESCALE:
        if (pass == 0) { SK(fwd_col_rescale) } else { SK(fwd_row_rescale) }
    case STAGE_FWD_LIFT:
        if (pass == 0) { SK(fwd_col_rescale) } else { SK(fwd_row_plain) }
    case STAGE_FWD_BCONV_MODDOWN:
        if (pass == 0) { SK(fwd_col_bconv) } else { SK(fwd_row_moddown) }
    case STAGE_INV_PLAIN:
        if (pass == 0) { SK(inv_row_plain) } else { SK(inv_col) }
    case STAGE_INV_GALOIS:
        if (pass == 0) { SK(inv_row_galois) } else { SK(inv_col) }
    case STAGE_INV_TENSOR:
        if (pass == 0) { SK(inv_row_tensor) } else { SK(inv_col) }
    default: return false;
    }
#undef SK
#undef SK12
}

}  // namespace

uint32_t ntt_passes(uint32_t logn) { return logn == 12 ? 1 : 2; }
uint32_t ntt_tiles(uint32_t logn) { return logn == 12 ? 1 : 16; }
static uint32_t ntt_threads(uint32_t logn) { return logn == 12 ? kThreads : kThreads16; }

// Fills a.heavy with the launch limbs on the integer path.  It leaves none when
// they do not fit the list, when every limb is on that path, or in launches of
// more than kHeavyMaxLimbs limbs: the assignment is then the whole-limb one.
// Measured side by side, placing the heavy limbs apart makes the passes over
// 31 and 35 limbs 5 to 12 % faster, leaves the 62-limb ModDown passes
// unchanged and makes the 74-limb ModUp passes 2 to 4 % slower: those run in
// more than one round of workgroups per CU, where the position of a workgroup
// in the launch no longer decides its CU.
constexpr uint32_t kHeavyMaxLimbs = 48;
static void set_heavy(NttArgs &a, uint32_t nlimbs)
{
    a.n_heavy = 0;
    if (a.logn != 16 || (a.map.skip_alpha != 0 && !a.map.dense) || nlimbs > kHeavyMaxLimbs) return;
    uint32_t nh = 0;
    for (uint32_t l = 0; l < nlimbs; ++l) {
        const LimbPos lp = limb_pos(a.map, l);
        if (lp.prime >= 64 || !((a.int_primes >> lp.prime) & 1)) continue;
        if (nh == (uint32_t)kMaxHeavy) return;
        a.heavy[nh++] = (uint8_t)l;
    }
    a.n_heavy = nh < nlimbs ? nh : 0;  // all limbs alike: whole-limb placement
}

// Tile width of the grid launches at N = 2^16, per direction and launch size
// (0: the default rule below).  Set by ckks_ntt_tile_set (an autotuner), read
// by every grid launch.
static std::atomic<uint8_t> g_tile[2][kMaxTileLimbs + 1];

static uint32_t default_tile(uint32_t nlimbs)
{
    if (nlimbs >= 24) return 16;
    return nlimbs >= 6 ? 8 : 4;
}

// tile code 2 (the 4-element inverse passes) applies to inverse stages only; a pass without a
// 4-element kernel (the gathered or tensor row passes) runs with tiles of 8
static uint32_t effective_tile(NttStage st, uint32_t tw)
{
    const bool inv = st == STAGE_INV_PLAIN || st == STAGE_INV_GALOIS || st == STAGE_INV_TENSOR;
    return tw == 2 && !inv ? 8 : tw;
}
static bool four_element_pass(NttStage st, uint32_t pass, uint32_t tw)
{
    return tw == 2 && (pass == 1 || st == STAGE_INV_PLAIN);
}

static uint32_t tile_width(NttStage st, uint32_t logn, uint32_t nlimbs)
{
    if (logn != 16) return 16;
    const int inv = st == STAGE_INV_PLAIN || st == STAGE_INV_GALOIS || st == STAGE_INV_TENSOR;
    const uint32_t t = nlimbs <= kMaxTileLimbs ? g_tile[inv][nlimbs].load(std::memory_order_relaxed) : 0;
    if (t) return t;
    return inv && nlimbs <= 8 ? 2 : default_tile(nlimbs);
}

hipError_t launch_ntt_stage(NttStage st, const NttArgs &a0, uint32_t nlimbs, hipStream_t stream, uint32_t first_pass)
{
    if (nlimbs == 0) return hipSuccess;
    if (first_pass >= ntt_passes(a0.logn)) return hipErrorInvalidValue;
    NttArgs a = a0;
    const uint32_t tw = effective_tile(st, tile_width(st, a.logn, nlimbs));
    if (tw == 16) set_heavy(a, nlimbs);
    else a.n_heavy = 0;
    for (uint32_t pass = first_pass; pass < ntt_passes(a.logn); ++pass) {
        StageKernels k;
        if (!stage_kernels(st, a.logn, pass, k, tw)) return hipErrorInvalidValue;
        const bool four = a.logn == 16 && four_element_pass(st, pass, tw);
        const uint32_t pw = tw == 2 ? 8 : tw;  // rows or columns per workgroup
        const uint32_t tiles = a.logn == 12 ? 1 : 256 / pw;
        const uint32_t threads = a.logn == 12 ? kThreads : four ? 512 : 32 * pw;
        hipLaunchKernelGGL(k.grid, dim3(tiles, nlimbs), dim3(threads), 0, stream, a);
    }
    return hipGetLastError();
}

bool ntt_tile_set(uint32_t inverse, uint32_t nlimbs, uint32_t tile)
{
    if (inverse > 1 || nlimbs == 0 || nlimbs > kMaxTileLimbs ||
        !(tile == 0 || tile == 4 || tile == 8 || tile == 16 || (tile == 2 && inverse == 1)))
        return false;
    g_tile[inverse][nlimbs].store((uint8_t)tile, std::memory_order_relaxed);
    return true;
}

uint32_t ntt_tile_get(uint32_t inverse, uint32_t nlimbs)
{
    return tile_width(inverse ? STAGE_INV_PLAIN : STAGE_FWD_PLAIN, 16, nlimbs);
}

hipError_t launch_inner_product_rowpass(const IpArgs &ip, const NttArgs &ia, hipStream_t stream)
{
    if (ip.logn != 16 || ia.logn != 16 || ip.fold_tot || ip.rows != ip.level + 1 + ip.np || ia.map.rows != ip.np ||
        ia.ys_mode != 2 || !ia.mid)
        return hipErrorInvalidValue;
    const dim3 grid((1u << ip.logn) / coef::kCoefThreads, ip.rows);
    if (ip.ta0) {
        if (ip.galois != 1 || !ip.ta1 || !ip.tb0 || !ip.tb1 || !ip.pmod) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_inner_product_tensor_rowpass, grid, dim3(coef::kCoefThreads), 0, stream, ip, ia);
    } else {
        hipLaunchKernelGGL(k_inner_product_rowpass, grid, dim3(coef::kCoefThreads), 0, stream, ip, ia);
    }
    return hipGetLastError();
}

hipError_t launch_ntt_stage_queue(NttStage st, uint32_t logn, uint32_t pass, const NttArgs *insts,
                                  const WorkQueue &q, uint32_t grid, hipStream_t stream)
{
    StageKernels k;
    if (!stage_kernels(st, logn, pass, k)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k.queue, dim3(grid), dim3(ntt_threads(logn)), 0, stream, insts, q);
    return hipGetLastError();
}

hipError_t launch_fused_batch(const FusedArgs &f, uint32_t grid, hipStream_t stream)
{
    if (f.nunits == 0) return hipSuccess;
    hipLaunchKernelGGL(q_fused16, dim3(grid), dim3(kThreads16), 0, stream, f);
    return hipGetLastError();
}

// Compatibility wrappers used by the single-operation paths.
hipError_t launch_ntt_fwd(const NttArgs &a0, uint32_t nlimbs, NttPro pro, NttEpi epi, hipStream_t stream,
                          uint64_t *mid, int64_t mid_poly_stride)
{
    NttArgs a = a0;
    a.mid = mid;
    a.mid_stride = mid_poly_stride;
    NttStage st;
    if (pro == PRO_PLAIN && epi == EPI_PLAIN) st = STAGE_FWD_PLAIN;
    else if (pro == PRO_PLAIN && epi == EPI_MODDOWN) st = STAGE_FWD_MODDOWN;
    else if (pro == PRO_RESCALE && epi == EPI_RESCALE) st = STAGE_FWD_RESCALE;
    else if (pro == PRO_RESCALE && epi == EPI_PLAIN) st = STAGE_FWD_LIFT;
    else if (pro == PRO_BCONV && epi == EPI_MODDOWN) st = STAGE_FWD_BCONV_MODDOWN;
    else return hipErrorInvalidValue;
    return launch_ntt_stage(st, a, nlimbs, stream);
}

hipError_t launch_ntt_inv(const NttArgs &a0, uint32_t nlimbs, NttPro pro, hipStream_t stream, uint64_t *mid,
                          int64_t mid_poly_stride)
{
    NttArgs a = a0;
    a.mid = mid;
    a.mid_stride = mid_poly_stride;
    return launch_ntt_stage(pro == PRO_GALOIS ? STAGE_INV_GALOIS : STAGE_INV_PLAIN, a, nlimbs, stream);
}

}  // namespace ckks
