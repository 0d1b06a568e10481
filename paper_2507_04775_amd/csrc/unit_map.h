// Assignment of the workgroups of an N = 2^16 NTT grid launch to (limb, tile)
// units, shared by the kernels and a host-side check.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

// XCD-aware unit of a grid launch.  Workgroups go to the eight XCDs round
// robin (linear id k to XCD k mod 8, position j = k div 8 in that XCD's
// order), each XCD with its own L2, and each XCD receives 2 n of the 16 n
// units of an n-limb launch.
// - Limbs on the 64-bit integer path (NttArgs::heavy) cost about 2.4 times an
//   FP64 limb.  Each XCD takes two tiles of every such limb, at consecutive
//   positions starting at (2 n) mod 32 when 2 n > 32: within an XCD,
//   consecutive workgroups go to different CUs, and the CUs that receive the
//   first (2 n) mod 32 positions also receive a third workgroup.  The heavy
//   tiles then share a CU with as little other work as the launch allows.
// - The other limbs keep whole-limb placement: XCD x takes limbs x, x + 8, …
//   of the first 8 floor(m/8) of them, and the last m mod 8 are spread evenly
//   over all XCDs.  A limb's two passes then run on the same XCD, so the row
//   pass finds the column pass's output and the limb's twiddles in its L2.
// The assignment is a bijection on the units.  Grid launches whose limb
// indices include skipped limbs keep the plain assignment, which spreads every
// limb's tiles over all XCDs: contiguous runs would leave some XCDs with
// skipped limbs only.  ModUp's single-operation launch enumerates only the
// converted rows (LimbMap::dense) instead.
struct UnitId {
    uint32_t limb, tile;
};

// Unit of workgroup k of an n-limb launch at N = 2^16 (16 tiles per limb),
// with nh heavy limbs at ascending launch indices heavy[].
__host__ __device__ __forceinline__ UnitId unit_of(uint32_t k, uint32_t n, uint32_t nh, const uint8_t *heavy)
{
    UnitId u;
    const uint32_t x = k & 7, j = k >> 3, per = 2 * n, hh = 2 * nh;
    uint32_t s = per > 32 ? per % 32 : 0;
    s = s + hh <= per ? s : per - hh;
    if (j - s < hh) {  // j in [s, s + hh)
        const uint32_t i = j - s;
        u.limb = heavy[i >> 1];
        u.tile = x + 8 * (i & 1);
        return u;
    }
    const uint32_t p = j < s ? j : j - hh;
    const uint32_t m = n - nh, whole = m >> 3, rest = m - 8 * whole;
    uint32_t li;
    if (p < 16 * whole) {
        li = x + 8 * (p >> 4);
        u.tile = p & 15;
    } else {  // XCD x's 2 rest units of the remaining limbs
        const uint32_t v = x * 2 * rest + (p - 16 * whole);
        li = 8 * whole + (v >> 4);
        u.tile = v & 15;
    }
    for (uint32_t h = 0; h < nh; ++h) li += heavy[h] <= li ? 1u : 0u;  // the li-th limb that is not heavy
    u.limb = li;
    return u;
}

}  // namespace ckks
