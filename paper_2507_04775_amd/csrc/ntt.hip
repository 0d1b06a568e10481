// Negacyclic NTT / inverse NTT for gfx950 (paper Sec. III-F.4).
//
// Forward: radix-2 Cooley-Tukey with the psi twist merged into the
// butterflies, natural coefficients -> bit-reversed evaluations.  Inverse:
// Gentleman-Sande butterflies, bit-reversed -> natural, times N^-1.  Twiddle
// w for the butterfly of stage m at index j is psi^br(m + j div 2t), with its
// Shoup companion (Table III), read from the context tables.
//
// Layout of the work: every thread owns 16 elements and runs four radix-2
// stages on them in registers ("radix-16 rounds"); rounds exchange data
// through LDS.  N = 2^12 fits one workgroup (three rounds).  N = 2^16 is the
// paper's 2-D / hierarchical scheme: viewed as a 256 x 256 matrix, a column
// pass runs the first eight stages (each column is an independent 256-point
// problem) and a row pass runs the last eight (each row of 256 contiguous
// elements is independent, with its own twiddle subset).  Each pass reads and
// writes every element once: four global accesses per element in total.
// Values stay lazily reduced (Harvey butterflies: [0, 4q) forward, [0, 2q)
// inverse) and are made canonical in the last pass.
#include "internal.h"

namespace ckks {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t pad(uint32_t x) { return x + (x >> 4); }

// Harvey forward butterfly: x, y in [0, 4q) -> [0, 4q)
__device__ __forceinline__ void ct_bfly(uint64_t &x, uint64_t &y, ulonglong2 w, uint64_t q, uint64_t q2)
{
    uint64_t a = x >= q2 ? x - q2 : x;
    uint64_t t = shoup_lazy(y, w.x, w.y, q);
    x = a + t;
    y = a - t + q2;
}

// Harvey inverse butterfly: x, y in [0, 2q) -> [0, 2q)
__device__ __forceinline__ void gs_bfly(uint64_t &x, uint64_t &y, ulonglong2 w, uint64_t q, uint64_t q2)
{
    uint64_t s = x + y;
    s = s >= q2 ? s - q2 : s;
    uint64_t d = x - y + q2;
    x = s;
    y = shoup_lazy(d, w.x, w.y, q);
}

// Four forward stages on v[i] = element base + STRIDE i of an NS-point
// problem: t = 8 STRIDE, 4 STRIDE, 2 STRIDE, STRIDE.  base = a 16 STRIDE + s
// with s < STRIDE.  Twiddles come from T[m B + j div 2t], m = NS / 2t.
template <int NS, int STRIDE>
__device__ __forceinline__ void fwd16(uint64_t (&v)[16], uint32_t base, const ulonglong2 *__restrict__ T, uint32_t B,
                                      uint64_t q, uint64_t q2)
{
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int h = 8 >> st;
        const uint32_t t = h * STRIDE;
        const uint32_t m = NS / (2 * t);
        const uint32_t g0 = m * B + base / (2 * t);
#pragma unroll
        for (int g = 0; g < (1 << st); ++g) {
            const ulonglong2 w = T[g0 + g];
#pragma unroll
            for (int k = 0; k < h; ++k) ct_bfly(v[g * 2 * h + k], v[g * 2 * h + k + h], w, q, q2);
        }
    }
}

// Four inverse stages: t = STRIDE, 2 STRIDE, 4 STRIDE, 8 STRIDE.
template <int NS, int STRIDE>
__device__ __forceinline__ void inv16(uint64_t (&v)[16], uint32_t base, const ulonglong2 *__restrict__ T, uint32_t B,
                                      uint64_t q, uint64_t q2)
{
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int h = 1 << st;
        const uint32_t t = h * STRIDE;
        const uint32_t m = NS / (2 * t);
        const uint32_t g0 = m * B + base / (2 * t);
#pragma unroll
        for (int g = 0; g < (8 >> st); ++g) {
            const ulonglong2 w = T[g0 + g];
#pragma unroll
            for (int k = 0; k < h; ++k) gs_bfly(v[g * 2 * h + k], v[g * 2 * h + k + h], w, q, q2);
        }
    }
}

struct LimbPos {
    uint32_t poly, row, prime;
    bool skip;
};

__device__ __forceinline__ LimbPos limb_pos(const LimbMap &m)
{
    LimbPos p;
    p.poly = blockIdx.y / m.rows;
    p.row = blockIdx.y - p.poly * m.rows;
    p.skip = limb_skipped(m, p.poly, p.row);
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
        return switch_modulo(a.rs_src[lp.poly][e], (a.rs_ql - 1) >> 1, a.rs_qlmod[lp.prime], P);
    } else {
        return src[e];
    }
}

// Final forward value x (canonical) at element e of the limb.
template <int EPI>
__device__ __forceinline__ void store_fwd(const NttArgs &a, const LimbPos &lp, uint64_t *dst, uint32_t e, uint64_t x,
                                          const Prime &P, size_t N)
{
    if (EPI == EPI_PLAIN) {
        dst[e] = x;
    } else {
        const size_t off = (size_t)lp.row * N;
        const ulonglong2 c = a.cst[lp.prime];
        uint64_t r = shoup(submod(a.aux[lp.poly][off + e], x, P.q), c.x, c.y, P.q);
        if (EPI == EPI_MODDOWN) {
            const uint64_t *add = a.add[lp.poly];
            if (add) r = addmod(r, add[off + (a.galois == 1 ? e : galois_src(e, a.galois, a.logn))], P.q);
        }
        a.out[lp.poly][off + e] = r;
    }
}

// ------------------------------------------------------------------ N = 2^16

template <int PRO>
__global__ __launch_bounds__(kThreads) void k_ntt16_fwd_col(NttArgs a, uint64_t *mid, int64_t mid_stride)
{
    __shared__ uint64_t lds[16 * 272];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 65536;
    const uint32_t col = threadIdx.x & 15, s = threadIdx.x >> 4, c = blockIdx.x * 16 + col;
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 65536;
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = load_fwd<PRO>(a, lp, src, (s + 16 * i) * 256 + c, P);
    fwd16<256, 16>(v, s, T, 1, q, q2);
    uint64_t *L = lds + col * 272;
#pragma unroll
    for (int i = 0; i < 16; ++i) L[pad(s + 16 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(16 * s + i)];
    fwd16<256, 1>(v, 16 * s, T, 1, q, q2);
    uint64_t *m = mid + (int64_t)lp.poly * mid_stride + (size_t)lp.row * 65536;
#pragma unroll
    for (int i = 0; i < 16; ++i) m[(16 * s + i) * 256 + c] = v[i];
}

template <int EPI>
__global__ __launch_bounds__(kThreads) void k_ntt16_fwd_row(NttArgs a, const uint64_t *mid, int64_t mid_stride)
{
    __shared__ uint64_t lds[16 * 272];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 65536;
    const uint32_t blk = threadIdx.x >> 4, s = threadIdx.x & 15, b = blockIdx.x * 16 + blk;
    const uint64_t *m = mid + (int64_t)lp.poly * mid_stride + (size_t)lp.row * 65536 + b * 256;
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = m[s + 16 * i];
    fwd16<256, 16>(v, s, T, 256 + b, q, q2);
    uint64_t *L = lds + blk * 272;
#pragma unroll
    for (int i = 0; i < 16; ++i) L[pad(s + 16 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(16 * s + i)];
    fwd16<256, 1>(v, 16 * s, T, 256 + b, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) L[pad(16 * s + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(s + 16 * i)];
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 65536;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint64_t x = csub(csub(v[i], q2), q);
        store_fwd<EPI>(a, lp, dst, b * 256 + s + 16 * i, x, P, 65536);
    }
}

template <int PRO>
__global__ __launch_bounds__(kThreads) void k_ntt16_inv_row(NttArgs a, uint64_t *mid, int64_t mid_stride)
{
    __shared__ uint64_t lds[16 * 272];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 65536;
    const uint32_t blk = threadIdx.x >> 4, s = threadIdx.x & 15, b = blockIdx.x * 16 + blk;
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 65536;
    uint64_t *L = lds + blk * 272;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t e = b * 256 + s + 16 * i;
        L[pad(s + 16 * i)] = src[PRO == PRO_GALOIS ? galois_src(e, a.galois, 16) : e];
    }
    __syncthreads();
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(16 * s + i)];
    inv16<256, 1>(v, 16 * s, T, 256 + b, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) L[pad(16 * s + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(s + 16 * i)];
    inv16<256, 16>(v, s, T, 256 + b, q, q2);
    uint64_t *m = mid + (int64_t)lp.poly * mid_stride + (size_t)lp.row * 65536 + b * 256;
#pragma unroll
    for (int i = 0; i < 16; ++i) m[s + 16 * i] = v[i];
}

__global__ __launch_bounds__(kThreads) void k_ntt16_inv_col(NttArgs a, const uint64_t *mid, int64_t mid_stride)
{
    __shared__ uint64_t lds[16 * 272];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 65536;
    const uint32_t col = threadIdx.x & 15, s = threadIdx.x >> 4, c = blockIdx.x * 16 + col;
    const uint64_t *m = mid + (int64_t)lp.poly * mid_stride + (size_t)lp.row * 65536;
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = m[(16 * s + i) * 256 + c];
    inv16<256, 1>(v, 16 * s, T, 1, q, q2);
    uint64_t *L = lds + col * 272;
#pragma unroll
    for (int i = 0; i < 16; ++i) L[pad(16 * s + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[pad(s + 16 * i)];
    inv16<256, 16>(v, s, T, 1, q, q2);
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 65536;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[(s + 16 * i) * 256 + c] = shoup(v[i], P.ninv, P.ninv_s, q);
}

// ------------------------------------------------------------------ N = 2^12

template <int PRO, int EPI>
__global__ __launch_bounds__(kThreads) void k_ntt12_fwd(NttArgs a)
{
    __shared__ uint64_t lds[4352];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 4096;
    const uint32_t t = threadIdx.x, base2 = (t >> 4) * 256 + (t & 15);
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 4096;
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = load_fwd<PRO>(a, lp, src, t + 256 * i, P);
    fwd16<4096, 256>(v, t, T, 1, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(t + 256 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(base2 + 16 * i)];
    fwd16<4096, 16>(v, base2, T, 1, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(base2 + 16 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(16 * t + i)];
    fwd16<4096, 1>(v, 16 * t, T, 1, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(16 * t + i)] = v[i];
    __syncthreads();
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 4096;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint64_t x = csub(csub(lds[pad(t + 256 * i)], q2), q);
        store_fwd<EPI>(a, lp, dst, t + 256 * i, x, P, 4096);
    }
}

template <int PRO>
__global__ __launch_bounds__(kThreads) void k_ntt12_inv(NttArgs a)
{
    __shared__ uint64_t lds[4352];
    const LimbPos lp = limb_pos(a.map);
    if (lp.skip) return;
    const Prime P = a.primes[lp.prime];
    const uint64_t q = P.q, q2 = P.two_q;
    const ulonglong2 *T = a.tw + (size_t)lp.prime * 4096;
    const uint32_t t = threadIdx.x, base2 = (t >> 4) * 256 + (t & 15);
    const uint64_t *src = a.src + (int64_t)lp.poly * a.map.src_poly_stride + (size_t)lp.row * 4096;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t e = t + 256 * i;
        lds[pad(e)] = src[PRO == PRO_GALOIS ? galois_src(e, a.galois, 12) : e];
    }
    __syncthreads();
    uint64_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(16 * t + i)];
    inv16<4096, 1>(v, 16 * t, T, 1, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(16 * t + i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(base2 + 16 * i)];
    inv16<4096, 16>(v, base2, T, 1, q, q2);
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(base2 + 16 * i)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(t + 256 * i)];
    inv16<4096, 256>(v, t, T, 1, q, q2);
    uint64_t *dst = a.dst + (int64_t)lp.poly * a.map.dst_poly_stride + (size_t)lp.row * 4096;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[t + 256 * i] = shoup(v[i], P.ninv, P.ninv_s, q);
}

}  // namespace

hipError_t launch_ntt_fwd(const NttArgs &a, uint32_t nlimbs, NttPro pro, NttEpi epi, hipStream_t stream,
                          uint64_t *mid, int64_t mid_poly_stride)
{
    if (nlimbs == 0) return hipSuccess;
    dim3 block(kThreads);
    if (a.logn == 12) {
        dim3 grid(1, nlimbs);
#define K12(P, E)                                                                            \
    if (pro == P && epi == E) {                                                              \
        hipLaunchKernelGGL((k_ntt12_fwd<P, E>), grid, block, 0, stream, a);                 \
        return hipGetLastError();                                                            \
    }
        K12(PRO_PLAIN, EPI_PLAIN)
        K12(PRO_PLAIN, EPI_MODDOWN)
        K12(PRO_RESCALE, EPI_RESCALE)
#undef K12
        return hipErrorInvalidValue;
    }
    dim3 grid(16, nlimbs);
    if (pro == PRO_PLAIN)
        hipLaunchKernelGGL((k_ntt16_fwd_col<PRO_PLAIN>), grid, block, 0, stream, a, mid, mid_poly_stride);
    else if (pro == PRO_RESCALE)
        hipLaunchKernelGGL((k_ntt16_fwd_col<PRO_RESCALE>), grid, block, 0, stream, a, mid, mid_poly_stride);
    else
        return hipErrorInvalidValue;
    if (epi == EPI_PLAIN)
        hipLaunchKernelGGL((k_ntt16_fwd_row<EPI_PLAIN>), grid, block, 0, stream, a, mid, mid_poly_stride);
    else if (epi == EPI_MODDOWN)
        hipLaunchKernelGGL((k_ntt16_fwd_row<EPI_MODDOWN>), grid, block, 0, stream, a, mid, mid_poly_stride);
    else
        hipLaunchKernelGGL((k_ntt16_fwd_row<EPI_RESCALE>), grid, block, 0, stream, a, mid, mid_poly_stride);
    return hipGetLastError();
}

hipError_t launch_ntt_inv(const NttArgs &a, uint32_t nlimbs, NttPro pro, hipStream_t stream, uint64_t *mid,
                          int64_t mid_poly_stride)
{
    if (nlimbs == 0) return hipSuccess;
    dim3 block(kThreads);
    if (a.logn == 12) {
        dim3 grid(1, nlimbs);
        if (pro == PRO_GALOIS)
            hipLaunchKernelGGL((k_ntt12_inv<PRO_GALOIS>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_ntt12_inv<PRO_PLAIN>), grid, block, 0, stream, a);
        return hipGetLastError();
    }
    dim3 grid(16, nlimbs);
    if (pro == PRO_GALOIS)
        hipLaunchKernelGGL((k_ntt16_inv_row<PRO_GALOIS>), grid, block, 0, stream, a, mid, mid_poly_stride);
    else
        hipLaunchKernelGGL((k_ntt16_inv_row<PRO_PLAIN>), grid, block, 0, stream, a, mid, mid_poly_stride);
    hipLaunchKernelGGL(k_ntt16_inv_col, grid, block, 0, stream, a, mid, mid_poly_stride);
    return hipGetLastError();
}

}  // namespace ckks
