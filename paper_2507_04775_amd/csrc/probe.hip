// Measurement probe: the issue rate of the 32x32->64 integer multiply-add
// (v_mad_u64_u32) that every 64-bit modular product of the kernels is built
// from.  The integer-VALU fraction reported for the key-switching kernels is
// taken against this rate and against the chip's issue peak (one wave64 VALU
// instruction per CU per cycle).  Not part of any CKKS operation.
#include <string>

#include "internal.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
}

using namespace ckks;

namespace {

constexpr int kChains = 8;       // independent multiply-add chains per thread
constexpr int kProbeThreads = 256;

// Each thread runs kChains dependent chains of `iters` multiply-adds,
// acc = lo32(acc) * b + acc, one v_mad_u64_u32 each, and writes their sum so
// the work is not removed.
__global__ __launch_bounds__(kProbeThreads) void k_probe_mad64(uint64_t *out, uint32_t iters, uint32_t b)
{
    uint64_t acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = (uint64_t)(threadIdx.x + 1) * (k + 3) + blockIdx.x;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = (uint64_t)(uint32_t)acc[k] * (uint64_t)b + acc[k];
    }
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" ckks_status ckks_probe_mad64(uint64_t *out, uint32_t blocks, uint32_t iters, void *stream,
                                        uint64_t *mads_per_launch)
{
    if (!out || blocks == 0 || iters == 0 || !mads_per_launch)
        return fail(CKKS_E_ARG, "ckks_probe_mad64: null pointer or zero size");
    hipLaunchKernelGGL(k_probe_mad64, dim3(blocks), dim3(kProbeThreads), 0, (hipStream_t)stream, out, iters,
                       0x9E3779B9u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_probe_mad64: ") + hipGetErrorString(e));
    *mads_per_launch = (uint64_t)blocks * kProbeThreads * iters * kChains;
    return CKKS_OK;
}
