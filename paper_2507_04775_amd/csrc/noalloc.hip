// Hybrid key switching for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the same kernels as ckks_keyswitch, with the workspace taken
// from a static device array instead of a caller buffer.
//
// The array lives in this file's code object, so every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Host
// code never passes `scratch` itself to a kernel (in host code that name is
// a host-side stand-in, not a device address): scratch_setup() resolves the
// device address once per device with hipGetSymbolAddress, and the entry
// point hands that address to the kernels.
#include <mutex>
#include <string>

#include "internal.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
ckks_status check_keyswitch_args(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key,
                                 const uint64_t *out0, const uint64_t *out1, const char *what);
}  // namespace ckks

#define TRY(x)                              \
    do {                                    \
        ckks_status _s = (x);               \
        if (_s != CKKS_OK) return _s;       \
    } while (0)

namespace {

// 160 MiB: the key-switch workspace at N = 2^16 and 31 ciphertext limbs with up
// to ten special primes (159 MiB at the top level) fits.
constexpr size_t kScratchBytes = (size_t)160 << 20;
static_assert(kScratchBytes % 256 == 0, "the scratch array is a whole number of 256-byte lines");

static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

namespace ckks {

// Resolves the device address of `scratch` on `device`, which must be the
// current device; once per device, later calls return the first result.
hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_done[device] = true;
    }
    return g_err[device];
}

}  // namespace ckks

using namespace ckks;

extern "C" size_t ckks_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" ckks_status ckks_keyswitch_noalloc(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key,
                                              uint64_t *out0, uint64_t *out1, void *stream)
{
    TRY(check_keyswitch_args(ctx, d, level, key, out0, out1, "ckks_keyswitch_noalloc"));
    const size_t need = ckks_workspace_bytes(ctx, CKKS_OP_KEYSWITCH, level);
    if (need > kScratchBytes)
        return fail(CKKS_E_ARG, "ckks_keyswitch_noalloc: the key switch at level " + std::to_string(level) +
                                    " needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                    std::to_string(kScratchBytes) + "-byte static scratch");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices && g_done[ctx->device]) ws = g_ptr[ctx->device];
    }
    if (!ws)
        return fail(CKKS_E_DEVICE, "ckks_keyswitch_noalloc: the static scratch has no address on device " +
                                       std::to_string(ctx->device) + " (hipGetSymbolAddress failed at context creation)");
    // the scratch lies in no caller buffer, so only d, out0 and out1 can overlap (checked above)
    const hipError_t e = keyswitch_core(ctx, d, 1, level, key->data, out0, out1, nullptr, nullptr, 1, ws,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_keyswitch_noalloc: ") + hipGetErrorString(e));
    return CKKS_OK;
}
