// Host-side check of the workgroup-to-unit assignment of the N = 2^16 NTT grid
// launches (the kernels' own header, run on the CPU): for every launch size up
// to 200 limbs and random sets of integer-path ("heavy") limbs, the assignment
// must be a bijection onto the 16 n units with every limb and tile in range;
// without heavy limbs it must be the whole-limb placement; with them, each XCD
// must hold two tiles of every heavy limb at consecutive positions starting at
// (2 n) mod 32 (or where they fit).  Prints "ok" and exits 0 on success.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2507_04775_amd/csrc/unit_map.h"

using namespace ckks;

static int fails = 0;

static void fail(const char *what, uint32_t n, uint32_t nh, uint32_t k)
{
    if (fails++ < 10) std::printf("%s: n=%u nh=%u k=%u\n", what, n, nh, k);
}

int main()
{
    std::mt19937 rng(7);
    long units = 0;
    for (uint32_t n = 1; n <= 200; ++n) {
        for (int trial = 0; trial < 40; ++trial) {
            const uint32_t nh = trial == 0 ? 0 : rng() % (std::min<uint32_t>(n, 32) + 1);
            std::vector<uint32_t> idx(n);
            for (uint32_t i = 0; i < n; ++i) idx[i] = i;
            std::shuffle(idx.begin(), idx.end(), rng);
            std::vector<uint8_t> heavy(idx.begin(), idx.begin() + nh);
            std::sort(heavy.begin(), heavy.end());
            std::vector<int> seen(16 * n, 0), is_heavy(n, 0);
            for (uint8_t h : heavy) is_heavy[h] = 1;
            const uint32_t per = 2 * n, hh = 2 * nh;
            uint32_t s = per > 32 ? per % 32 : 0;
            s = s + hh <= per ? s : per - hh;
            for (uint32_t k = 0; k < 16 * n; ++k) {
                const UnitId u = unit_of(k, n, nh, heavy.data());
                ++units;
                if (u.limb >= n || u.tile >= 16) {
                    fail("out of range", n, nh, k);
                    continue;
                }
                ++seen[u.limb * 16 + u.tile];
                const uint32_t x = k & 7, j = k >> 3;
                const bool in_window = j >= s && j < s + hh;
                if (in_window != (bool)is_heavy[u.limb]) fail("heavy tile outside its window", n, nh, k);
                if (is_heavy[u.limb] && u.tile % 8 != x) fail("heavy tile on another XCD", n, nh, k);
                if (nh == 0) {  // whole-limb placement
                    const uint32_t whole = n >> 3, rest = n - 8 * whole;
                    uint32_t limb, tile;
                    if (j < 16 * whole) {
                        limb = x + 8 * (j >> 4);
                        tile = j & 15;
                    } else {
                        const uint32_t v = x * 2 * rest + (j - 16 * whole);
                        limb = 8 * whole + (v >> 4);
                        tile = v & 15;
                    }
                    if (u.limb != limb || u.tile != tile) fail("not the whole-limb placement", n, nh, k);
                }
            }
            for (uint32_t i = 0; i < 16 * n; ++i)
                if (seen[i] != 1) fail("not a bijection", n, nh, i);
        }
    }
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("%ld units checked\nok\n", units);
    return 0;
}
