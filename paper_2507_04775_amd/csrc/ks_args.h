// Argument blocks of the key-switching steps, built on the host for the
// single-operation calls (launched at once) and for batches (stored in device
// tables and run by the persistent stage kernels).
#pragma once
#include "internal.h"

namespace ckks {

struct KsSizes {
    uint32_t n, rows, beta;  // limbs l+1, extended rows l+1+K, digits at level l
    size_t N;
};

// workspace layout of one key switch: dc [n], ext [beta][rows], acc [2][rows], pc [2][K], conv [2][n]
struct KsWs {
    uint64_t *dc, *ext, *acc, *pc, *conv;
};

KsSizes ks_sizes(const ckks_ctx *c, uint32_t level);
size_t ks_ws_elems(const ckks_ctx *c, uint32_t level);
KsWs ks_ws(const ckks_ctx *c, uint32_t level, void *ws);
NttArgs base_args(const ckks_ctx *c, bool inverse);

// ModUp: INTT of d (gathered through g) leaving scaled conversion inputs (n limbs)
NttArgs args_modup_intt(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, uint64_t *dc);
// ModUp: conversion of every digit (beta jobs); own rows copied from d when copy_own
BconvArgs args_modup_bconv(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *dc,
                           uint64_t *ext, bool copy_own);
// ModUp: forward NTT of the converted rows (beta * rows limbs, own rows skipped)
NttArgs args_modup_ntt(const ckks_ctx *c, uint32_t level, uint64_t *ext);
// key inner product (rows rows); own rows read from `own` when non-null
IpArgs args_ip(const ckks_ctx *c, const uint64_t *ext, uint32_t level, const uint64_t *key, uint32_t g,
               uint64_t *acc, const uint64_t *own, uint32_t own_galois);
// ModDown: INTT of the special rows of npoly accumulators (npoly * K limbs)
NttArgs args_moddown_intt(const ckks_ctx *c, const uint64_t *acc, int64_t acc_stride, uint32_t level, uint64_t *pc);
// ModDown: conversion + forward NTT + P^-1 (x - .) + add (npoly * n limbs)
NttArgs args_moddown_ntt(const ckks_ctx *c, const uint64_t *acc, int64_t acc_stride, uint32_t npoly, uint32_t level,
                         uint64_t *const *out, const uint64_t *const *add, uint32_t g, const uint64_t *pc,
                         uint64_t *conv);

}  // namespace ckks
