// Coefficient-wise kernels of the key-switching path for gfx950: the fast
// base conversion (paper Eq. (1), Sec. III-F.3), the key inner product
// (dot-product fusion of III-F.5), the HMult tensor (their units are in
// coef_units.h) and the limb-wise support operations of Table I.  One thread
// per coefficient index, so every global access is a fully coalesced
// 8-byte-per-lane row segment.
#include "internal.h"
#include "coef_units.h"

namespace ckks {

namespace {

constexpr int kThreads = 256;
using namespace coef;

__global__ __launch_bounds__(kThreads) void k_bconv(BconvArgs a)
{
    bconv_unit(a, blockIdx.y, blockIdx.x, blockIdx.z, threadIdx.x);
}

// persistent: tile t of record (inst, job) covers kQueueBlocks coefficient blocks
// ((t % (N / (256 kQueueBlocks))) kQueueBlocks ..) of row group t / (N / (256 kQueueBlocks))
__global__ __launch_bounds__(kThreads) void q_bconv(const BconvArgs *insts, WorkQueue q)
{
    __shared__ BconvArgs sa;
    __shared__ uint32_t claim;
    run_work_queue(insts, q, sa, &claim, [&](const BconvArgs &a, uint32_t job, uint32_t t) {
        const uint32_t nb = a.N / (kThreads * kQueueBlocks);
        for (uint32_t i = 0; i < kQueueBlocks; ++i) bconv_unit(a, job, (t % nb) * kQueueBlocks + i, t / nb, threadIdx.x);
    });
}

__global__ __launch_bounds__(kThreads) void k_inner_product(IpArgs a)
{
    __shared__ uint64_t stage[kIpStage * kThreads];
    ip_unit(a, blockIdx.y, blockIdx.x, stage, threadIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_inner_product_tensor(IpArgs a)
{
    ip_unit_tensor(a, blockIdx.y, blockIdx.x, threadIdx.x);
}

__global__ __launch_bounds__(kThreads) void q_inner_product(const IpArgs *insts, WorkQueue q)
{
    __shared__ uint64_t stage[kIpStage * kThreads];
    __shared__ IpArgs sa;
    __shared__ uint32_t claim;
    run_work_queue(insts, q, sa, &claim, [&](const IpArgs &a, uint32_t row, uint32_t t) {
        ip_blocks(a, row, t * kQueueBlocks, kQueueBlocks, stage, threadIdx.x);
    });
}

__global__ __launch_bounds__(kThreads) void k_tensor(TensorArgs a) { tensor_unit(a, blockIdx.y, blockIdx.x, threadIdx.x); }

__global__ __launch_bounds__(kThreads) void q_tensor(const TensorArgs *insts, WorkQueue q)
{
    __shared__ TensorArgs sa;
    __shared__ uint32_t claim;
    run_work_queue(insts, q, sa, &claim, [&](const TensorArgs &a, uint32_t limb, uint32_t t) {
        for (uint32_t i = 0; i < kQueueBlocks; ++i) tensor_unit(a, limb, t * kQueueBlocks + i, threadIdx.x);
    });
}

// zeroes n counters (a fill kernel: safe inside captured graphs)
__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

struct Scalars {
    uint64_t v[kMaxPrimes];
};

template <int OP>
__global__ __launch_bounds__(kThreads) void k_elementwise(const uint64_t *a, const uint64_t *b, const uint64_t *c,
                                                          uint64_t *out, Scalars scalars, const Prime *primes,
                                                          uint32_t logn)
{
    const uint32_t l = blockIdx.y;
    const size_t i = ((size_t)l << logn) + blockIdx.x * kThreads + threadIdx.x;
    const Prime P = primes[l];
    const uint64_t x = a[i];
    uint64_t r;
    if (OP == 0) r = addmod(x, b[i], P.q);
    else if (OP == 1) r = submod(x, b[i], P.q);
    else if (OP == 2) r = mulmod(x, b[i], P);
    else if (OP == 3) r = reduce128(add128(mul_wide(x, b[i]), u128{c[i], 0}), P);
    else if (OP == 4) r = mulmod(x, scalars.v[l], P);
    else r = addmod(x, scalars.v[l], P.q);
    out[i] = r;
}

// Ciphertext-level support operations of Table I over both halves in one
// launch (blockIdx.z = half t): HAdd a_t + b_t; PtAdd a_0 + pt and a copy of
// a_1; PtMult a_t pt; ScalarAdd a_0 + s and a copy of a_1; ScalarMult a_t s.
// The copy half is skipped (grid z = 1) when the output is the input.
template <int OP>
__global__ __launch_bounds__(kThreads) void k_ct_op(CtOpArgs a)
{
    const uint32_t l = blockIdx.y, t = blockIdx.z;
    const size_t i = ((size_t)l << a.logn) + blockIdx.x * kThreads + threadIdx.x;
    const Prime P = a.primes[l];
    const uint64_t x = a.a[t][i];
    uint64_t r;
    if (OP == CT_HADD) r = addmod(x, a.b[t][i], P.q);
    else if (OP == CT_PTADD) r = t == 0 ? addmod(x, a.b[0][i], P.q) : x;
    else if (OP == CT_PTMULT) r = mulmod(x, a.b[0][i], P);
    else if (OP == CT_SCALAR_ADD) r = t == 0 ? addmod(x, a.s[l], P.q) : x;
    else r = mulmod(x, a.s[l], P);
    a.out[t][i] = r;
}

__global__ __launch_bounds__(kThreads) void k_fold_ext(FoldArgs a)
{
    const uint32_t r = blockIdx.y, t = blockIdx.z, N = 1u << a.logn;
    const uint32_t n = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t pi = row_prime(r, a.level, a.nq);
    const Prime P = a.primes[pi];
    const size_t i = (size_t)r * N + n;
    uint64_t v = a.acc[t] ? a.acc[t][i] : 0;
    if (a.s[t] && r <= a.level) {
        const uint64_t x = a.s[t][(size_t)r * N + (a.galois == 1 ? n : galois_src(n, a.galois, a.logn))];
        v = addmod(v, mulmod(a.pmod[r], x, P), P.q);
    }
    a.tot[t][i] = a.first ? v : addmod(a.tot[t][i], v, P.q);
}

__global__ __launch_bounds__(kThreads) void k_automorph(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                        uint32_t logn, uint32_t g)
{
    const uint32_t l = blockIdx.y;
    const uint32_t e = blockIdx.x * kThreads + threadIdx.x;
    const size_t base = (size_t)l << logn;
    out[base + e] = in[base + galois_src(e, g, logn)];
}

// out_t[o] = sum_b a_t[b] pt[o][b] on every coefficient of every limb: the
// products are summed exactly in 128 bits (n <= 16 products below 2^122 each)
// and reduced once; each baby coefficient is read once for all NOUT outputs.
template <int NOUT>
__global__ __launch_bounds__(kThreads) void k_lincomb(LincombArgs a)
{
    const uint32_t l = blockIdx.y;
    const size_t i = ((size_t)l << a.logn) + blockIdx.x * kThreads + threadIdx.x;
    const Prime P = a.primes[l];
    u128 s0[NOUT], s1[NOUT];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) s0[o] = s1[o] = u128{0, 0};
    // the loads of four baby steps are issued before their products, so their latencies overlap
    constexpr uint32_t G = 4;
    for (uint32_t b0 = 0; b0 < a.n; b0 += G) {
        uint64_t x0[G], x1[G], w[NOUT][G];
#pragma unroll
        for (uint32_t t = 0; t < G; ++t) {
            if (b0 + t >= a.n) break;
            x0[t] = a.a0[b0 + t][i];
            x1[t] = a.a1[b0 + t][i];
#pragma unroll
            for (int o = 0; o < NOUT; ++o) w[o][t] = a.pt[o][b0 + t][i];
        }
#pragma unroll
        for (uint32_t t = 0; t < G; ++t) {
            if (b0 + t >= a.n) break;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                s0[o] = add128(s0[o], mul_wide(x0[t], w[o][t]));
                s1[o] = add128(s1[o], mul_wide(x1[t], w[o][t]));
            }
        }
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        a.out0[o][i] = reduce128(s0[o], P);
        a.out1[o][i] = reduce128(s1[o], P);
    }
}

// out_t = acc_t + sum_b a_t[b] c_b (c_b a residue per limb), summed exactly in
// 128 bits and reduced once; acc may be the output itself (read first).
__global__ __launch_bounds__(kThreads) void k_scalar_lincomb(ScalarLincombArgs a)
{
    const uint32_t l = blockIdx.y;
    const size_t i = ((size_t)l << a.logn) + blockIdx.x * kThreads + threadIdx.x;
    const Prime P = a.primes[l];
    u128 s0 = {a.acc0 ? a.acc0[i] : 0, 0}, s1 = {a.acc1 ? a.acc1[i] : 0, 0};
    constexpr uint32_t G = 4;  // loads of four terms before their products
    for (uint32_t b0 = 0; b0 < a.n; b0 += G) {
        uint64_t x0[G], x1[G], w[G];
#pragma unroll
        for (uint32_t t = 0; t < G; ++t) {
            if (b0 + t >= a.n) break;
            x0[t] = a.a0[b0 + t][i];
            x1[t] = a.a1[b0 + t][i];
            w[t] = a.cst[(size_t)(b0 + t) * a.cst_stride + l];
        }
#pragma unroll
        for (uint32_t t = 0; t < G; ++t) {
            if (b0 + t >= a.n) break;
            s0 = add128(s0, mul_wide(x0[t], w[t]));
            s1 = add128(s1, mul_wide(x1[t], w[t]));
        }
    }
    a.out0[i] = reduce128(s0, P);
    a.out1[i] = reduce128(s1, P);
}

__device__ uint64_t pow2_mod(uint32_t e, const Prime &P)
{
    uint64_t r = 1, b = 2 % P.q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, b, P);
        b = mulmod(b, b, P);
    }
    return r;
}

// Residue of an integer-valued double v = +-m 2^e (m < 2^53 from its bit
// fields): m >> -e when e <= 0, else [m]_q [2^e]_q.
__global__ __launch_bounds__(kThreads) void k_reduce_f64(const double *__restrict__ x, uint64_t *__restrict__ out,
                                                         const Prime *primes, uint32_t nlimbs, uint32_t logn)
{
    const uint32_t l = blockIdx.y, d = blockIdx.z;
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    const Prime P = primes[l];
    const uint64_t bits = (uint64_t)__double_as_longlong(x[((size_t)d << logn) + k]);
    const uint32_t ex = (uint32_t)(bits >> 52) & 0x7ff;
    uint64_t r = 0;
    if (ex != 0) {  // zero has ex = 0; an integer-valued double is never subnormal
        const uint64_t m = (bits & ((1ull << 52) - 1)) | (1ull << 52);
        const int e = (int)ex - 1075;
        r = e <= 0 ? (m >> (uint32_t)(-e)) % P.q : mulmod(m % P.q, pow2_mod((uint32_t)e, P), P);
    }
    if ((bits >> 63) && r) r = P.q - r;
    out[(((size_t)d * nlimbs + l) << logn) + k] = r;
}

__global__ __launch_bounds__(kThreads) void k_half_monomial(uint64_t *out, uint32_t logn)
{
    const size_t i = ((size_t)blockIdx.y << logn) + blockIdx.x * kThreads + threadIdx.x;
    const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
    out[i] = k == (1u << (logn - 1)) ? 1 : 0;
}

}  // namespace

hipError_t launch_lincomb(const LincombArgs &a, uint32_t nlimbs, hipStream_t stream)
{
    if (a.n == 0 || a.n > kMaxLincomb) return hipErrorInvalidValue;
    if (a.nout == 1)
        hipLaunchKernelGGL(k_lincomb<1>, dim3((1u << a.logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, a);
    else if (a.nout == 2)
        hipLaunchKernelGGL(k_lincomb<2>, dim3((1u << a.logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_scalar_lincomb(const ScalarLincombArgs &a, uint32_t nlimbs, hipStream_t stream)
{
    if (a.n == 0 || a.n > kMaxLincomb || nlimbs > a.cst_stride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scalar_lincomb, dim3((1u << a.logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_reduce_f64(const double *x, uint64_t *out, const Prime *primes, uint32_t ndiag, uint32_t nlimbs,
                             uint32_t logn, hipStream_t stream)
{
    if (ndiag == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_f64, dim3((1u << logn) / kThreads, nlimbs, ndiag), dim3(kThreads), 0, stream, x,
                       out, primes, nlimbs, logn);
    return hipGetLastError();
}

hipError_t launch_half_monomial(uint64_t *out, uint32_t nlimbs, uint32_t logn, hipStream_t stream)
{
    hipLaunchKernelGGL(k_half_monomial, dim3((1u << logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, out, logn);
    return hipGetLastError();
}

hipError_t launch_bconv(const BconvArgs &a, uint32_t njobs, hipStream_t stream)
{
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bconv, dim3(a.N / kThreads, njobs, (a.nrows + kBconvRowGroup - 1) / kBconvRowGroup),
                       dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_inner_product(const IpArgs &a, hipStream_t stream)
{
    if (a.ta0) {
        if (a.galois != 1 || !a.ta1 || !a.tb0 || !a.tb1 || !a.pmod) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_inner_product_tensor, dim3((1u << a.logn) / kThreads, a.rows), dim3(kThreads), 0, stream,
                           a);
    } else {
        hipLaunchKernelGGL(k_inner_product, dim3((1u << a.logn) / kThreads, a.rows), dim3(kThreads), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_tensor(const uint64_t *a0, const uint64_t *a1, const uint64_t *b0, const uint64_t *b1, uint64_t *d0,
                         uint64_t *d1, uint64_t *d2, const Prime *primes, uint32_t nlimbs, uint32_t logn,
                         hipStream_t stream)
{
    TensorArgs a = {a0, a1, b0, b1, d0, d1, d2, primes, logn, 0};
    hipLaunchKernelGGL(k_tensor, dim3((1u << logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_bconv_queue(const BconvArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL(q_bconv, dim3(grid), dim3(kThreads), 0, stream, insts, q);
    return hipGetLastError();
}

hipError_t launch_inner_product_queue(const IpArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL(q_inner_product, dim3(grid), dim3(kThreads), 0, stream, insts, q);
    return hipGetLastError();
}

hipError_t launch_tensor_queue(const TensorArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL(q_tensor, dim3(grid), dim3(kThreads), 0, stream, insts, q);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_elementwise(int op, const uint64_t *a, const uint64_t *b, const uint64_t *c, uint64_t *out,
                              const uint64_t *host_scalars, const Prime *primes, uint32_t nlimbs, uint32_t logn,
                              hipStream_t stream)
{
    dim3 grid((1u << logn) / kThreads, nlimbs), block(kThreads);
    Scalars sc = {};
    if (host_scalars)
        for (uint32_t l = 0; l < nlimbs && l < (uint32_t)kMaxPrimes; ++l) sc.v[l] = host_scalars[l];
    switch (op) {
    case 0: hipLaunchKernelGGL((k_elementwise<0>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    case 1: hipLaunchKernelGGL((k_elementwise<1>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    case 2: hipLaunchKernelGGL((k_elementwise<2>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    case 3: hipLaunchKernelGGL((k_elementwise<3>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    case 4: hipLaunchKernelGGL((k_elementwise<4>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    case 5: hipLaunchKernelGGL((k_elementwise<5>), grid, block, 0, stream, a, b, c, out, sc, primes, logn); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fold_ext(const FoldArgs &a, uint32_t rows, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fold_ext, dim3((1u << a.logn) / kThreads, rows, 2), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_ct_op(int op, const CtOpArgs &a, uint32_t nlimbs, uint32_t halves, hipStream_t stream)
{
    dim3 grid((1u << a.logn) / kThreads, nlimbs, halves), block(kThreads);
    switch (op) {
    case CT_HADD: hipLaunchKernelGGL((k_ct_op<CT_HADD>), grid, block, 0, stream, a); break;
    case CT_PTADD: hipLaunchKernelGGL((k_ct_op<CT_PTADD>), grid, block, 0, stream, a); break;
    case CT_PTMULT: hipLaunchKernelGGL((k_ct_op<CT_PTMULT>), grid, block, 0, stream, a); break;
    case CT_SCALAR_ADD: hipLaunchKernelGGL((k_ct_op<CT_SCALAR_ADD>), grid, block, 0, stream, a); break;
    case CT_SCALAR_MULT: hipLaunchKernelGGL((k_ct_op<CT_SCALAR_MULT>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_automorph(const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint32_t logn, uint32_t galois,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(k_automorph, dim3((1u << logn) / kThreads, nlimbs), dim3(kThreads), 0, stream, in, out, logn,
                       galois);
    return hipGetLastError();
}

}  // namespace ckks
