// C-ABI entry points: host-side validation, then the launch sequence of each
// operation on the caller's stream.  The composition of key switching follows
// hybrid key switching (paper Sec. II-A, III-F.3): INTT -> ModUp base
// conversion -> NTT -> key inner product -> INTT of the special rows ->
// ModDown base conversion -> NTT with the fused P^-1 (x - .) epilogue
// (III-F.5), into which the HMult / rotation additions are folded as well.
#include <string.h>

#include <string>

#include "internal.h"
#include "ks_args.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
}

using namespace ckks;

namespace {

hipStream_t S(void *stream) { return (hipStream_t)stream; }

ckks_status dev(hipError_t e, const char *what)
{
    if (e == hipSuccess) return CKKS_OK;
    return fail(CKKS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned(const void *p) { return ((uintptr_t)p & 7) == 0; }

bool overlap(const void *a, size_t an, const void *b, size_t bn)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

ckks_status check_ptr(const void *p, const char *what)
{
    if (!p) return fail(CKKS_E_ARG, std::string(what) + ": null pointer");
    if (!aligned(p)) return fail(CKKS_E_ARG, std::string(what) + ": pointer not 8-byte aligned");
    return CKKS_OK;
}

#define TRY(x)                              \
    do {                                    \
        ckks_status _s = (x);               \
        if (_s != CKKS_OK) return _s;       \
    } while (0)

hipError_t modup_intt(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, uint64_t *dc, hipStream_t st)
{
    return launch_ntt_stage(g == 1 ? STAGE_INV_PLAIN : STAGE_INV_GALOIS, args_modup_intt(c, d, g, level, dc), level + 1,
                            st);
}

hipError_t modup_from_coeffs(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *dc,
                             uint64_t *ext, bool copy_own, hipStream_t st)
{
    KsSizes s = ks_sizes(c, level);
    hipError_t e = launch_bconv(args_modup_bconv(c, d, g, level, dc, ext, copy_own), s.beta, st);
    if (e != hipSuccess) return e;
    // only the converted rows: every digit leaves out its own rows, which partition q_0..q_l
    NttArgs a = args_modup_ntt(c, level, ext);
    a.map.dense = 1;
    return launch_ntt_stage(STAGE_FWD_PLAIN, a, s.beta * s.rows - s.n, st);
}

hipError_t inner_product(const ckks_ctx *c, const uint64_t *ext, uint32_t level, const uint64_t *key, uint32_t g,
                         uint64_t *acc, hipStream_t st, const uint64_t *own = nullptr, uint32_t own_galois = 1)
{
    return launch_inner_product(args_ip(c, ext, level, key, g, acc, own, own_galois), st);
}

// ModDown of npoly accumulators acc[t] (rows q_0..q_l, p_0..p_{K-1}, stride
// acc_stride) into out[t] = P^-1 (acc_t - NTT(Conv_{P->q}(INTT(acc_t|P)))) + add_t
// (add gathered through g).  The special rows' iNTT leaves the scaled
// conversion inputs y_k = [a_k (P/p_k)^-1] (N^-1 folded into the same
// constant); the forward NTT computes the conversion in its first pass and the
// P^-1 (x - .) + add sequence in its last (III-F.5 ModDown fusion).
// row_done: the inner product already ran the INTT's first pass (launch_inner_product_rowpass).
hipError_t moddown(const ckks_ctx *c, const uint64_t *acc, int64_t acc_stride, uint32_t npoly, uint32_t level,
                   uint64_t *const *out, const uint64_t *const *add, uint32_t g, uint64_t *pc, uint64_t *conv,
                   hipStream_t st, bool row_done = false)
{
    KsSizes s = ks_sizes(c, level);
    hipError_t e = launch_ntt_stage(STAGE_INV_PLAIN, args_moddown_intt(c, acc, acc_stride, level, pc), npoly * c->np, st,
                                    row_done ? 1 : 0);
    if (e != hipSuccess) return e;
    return launch_ntt_stage(STAGE_FWD_BCONV_MODDOWN,
                            args_moddown_ntt(c, acc, acc_stride, npoly, level, out, add, g, pc, conv), npoly * s.n, st);
}

}  // namespace

namespace ckks {

// Full key switch of d (gathered through g_in) with `key`; outputs
// out_t = KS_t + add_t (add gathered through g_add).  The digits' own rows are
// never copied: the inner product reads them from d directly.
// tin (N = 2^16, d, add0, add1 null, g_in = g_add = 1): HMult's relinearisation
// of a x b with the tensor folded in.  d2 = a1 b1 is formed by ModUp's first
// inverse pass and by the inner product (its digit-own rows), and the inner
// product adds [P]_q d0 and [P]_q d1 to the accumulators over q_0..q_l, so
// that ModDown returns KS(d2) + (d0, d1): no tensor kernel and no d0, d1, d2
// in memory.
hipError_t keyswitch_core(const ckks_ctx *c, const uint64_t *d, uint32_t g_in, uint32_t level, const uint64_t *key,
                          uint64_t *out0, uint64_t *out1, const uint64_t *add0, const uint64_t *add1, uint32_t g_add,
                          void *ws, hipStream_t st, const TensorIn *tin)
{
    KsSizes s = ks_sizes(c, level);
    KsWs w = ks_ws(c, level, ws);
    hipError_t e;
    if (tin) {
        if (c->logn != 16 || d || add0 || add1 || g_in != 1 || g_add != 1) return hipErrorInvalidValue;
        NttArgs ia = args_modup_intt(c, tin->a1, 1, level, w.dc);
        ia.src2 = tin->b1;
        e = launch_ntt_stage(STAGE_INV_TENSOR, ia, level + 1, st);
    } else {
        e = modup_intt(c, d, g_in, level, w.dc, st);
    }
    if (e == hipSuccess) e = modup_from_coeffs(c, d, g_in, level, w.dc, w.ext, false, st);
    if (e != hipSuccess) return e;
    IpArgs ip = args_ip(c, w.ext, level, key, 1, w.acc, d, g_in);
    if (tin) {
        ip.own = nullptr;
        ip.ta0 = tin->a0;
        ip.ta1 = tin->a1;
        ip.tb0 = tin->b0;
        ip.tb1 = tin->b1;
    }
    // at N = 2^16 the inner product also runs the first pass of ModDown's INTT on the special rows
    const int64_t acc_stride = (int64_t)s.rows * s.N;
    const bool rowpass = c->logn == 16;
    e = rowpass ? launch_inner_product_rowpass(ip, args_moddown_intt(c, w.acc, acc_stride, level, w.pc), st)
                : launch_inner_product(ip, st);
    if (e != hipSuccess) return e;
    uint64_t *outs[2] = {out0, out1};
    const uint64_t *adds[2] = {add0, add1};
    return moddown(c, w.acc, acc_stride, 2, level, outs, adds, g_add, w.pc, w.conv, st, rowpass);
}

}  // namespace ckks

namespace {

ckks_status check_ctx(const ckks_ctx *c)
{
    if (!c) return fail(CKKS_E_ARG, "null context");
    return CKKS_OK;
}

ckks_status check_level(const ckks_ctx *c, uint32_t level)
{
    if (level >= c->nq) return fail(CKKS_E_LEVEL, "level " + std::to_string(level) + " out of range");
    return CKKS_OK;
}

ckks_status check_ct(const ckks_ctx *c, const ckks_ct *ct, const char *what)
{
    if (!ct) return fail(CKKS_E_ARG, std::string(what) + ": null ciphertext");
    TRY(check_ptr(ct->c0, what));
    TRY(check_ptr(ct->c1, what));
    TRY(check_level(c, ct->level));
    size_t bytes = (size_t)(ct->level + 1) * c->N * 8;
    if (overlap(ct->c0, bytes, ct->c1, bytes))
        return fail(CKKS_E_ARG, std::string(what) + ": c0 and c1 overlap");
    return CKKS_OK;
}

ckks_status check_key(const ckks_ctx *c, const ckks_key *k)
{
    if (!k || !k->data) return fail(CKKS_E_KEY, "null key");
    if (k->ctx != c) return fail(CKKS_E_KEY, "key belongs to another context");
    return CKKS_OK;
}

size_t poly_bytes(const ckks_ctx *c, uint32_t level) { return (size_t)(level + 1) * c->N * 8; }

ckks_status check_disjoint(const ckks_ctx *c, const ckks_ct *out, const ckks_ct *in, uint32_t lvl_out,
                           uint32_t lvl_in, const char *what)
{
    size_t bo = poly_bytes(c, lvl_out), bi = poly_bytes(c, lvl_in);
    const void *o[2] = {out->c0, out->c1}, *i[2] = {in->c0, in->c1};
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            if (overlap(o[x], bo, i[y], bi)) return fail(CKKS_E_ARG, std::string(what) + ": output overlaps input");
    return CKKS_OK;
}

uint32_t galois_of_rotation(const ckks_ctx *c, int32_t k)
{
    const uint64_t two_n = 2ull * c->N, half = c->N / 2;
    int64_t kk = k % (int64_t)half;
    if (kk < 0) kk += half;
    uint64_t g = 1, b = 5;
    for (uint64_t e = (uint64_t)kk; e; e >>= 1, b = b * b % two_n)
        if (e & 1) g = g * b % two_n;
    return (uint32_t)g;
}

}  // namespace

namespace ckks {

hipError_t keyswitch_extended(ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *key,
                              void *ws, hipStream_t st, uint64_t **acc)
{
    KsWs w = ks_ws(c, level, ws);
    *acc = w.acc;
    hipError_t e = modup_intt(c, d, g, level, w.dc, st);
    if (e == hipSuccess) e = modup_from_coeffs(c, d, g, level, w.dc, w.ext, false, st);
    if (e == hipSuccess) e = inner_product(c, w.ext, level, key, 1, w.acc, st, d, g);
    return e;
}

hipError_t keyswitch_extended_fold(ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *key,
                                   void *ws, hipStream_t st, const uint64_t *c0, uint64_t *tot, bool first)
{
    KsWs w = ks_ws(c, level, ws);
    hipError_t e = modup_intt(c, d, g, level, w.dc, st);
    if (e == hipSuccess) e = modup_from_coeffs(c, d, g, level, w.dc, w.ext, false, st);
    if (e != hipSuccess) return e;
    IpArgs ip = args_ip(c, w.ext, level, key, 1, w.acc, d, g);
    ip.fold_c0 = c0;
    ip.fold_tot = tot;
    ip.fold_first = first ? 1 : 0;
    return launch_inner_product(ip, st);
}

hipError_t moddown_pair(ckks_ctx *c, const uint64_t *x, uint32_t level, uint64_t *out0, uint64_t *out1, void *ws,
                        hipStream_t st)
{
    const KsSizes s = ks_sizes(c, level);
    KsWs w = ks_ws(c, level, ws);
    uint64_t *outs[2] = {out0, out1};
    const uint64_t *adds[2] = {nullptr, nullptr};
    return moddown(c, x, (int64_t)s.rows * s.N, 2, level, outs, adds, 1, w.pc, w.conv, st);
}

}  // namespace ckks

extern "C" ckks_status ckks_sync(ckks_ctx *ctx, void *stream)
{
    TRY(check_ctx(ctx));
    hipError_t e = hipStreamSynchronize(S(stream));
    if (e == hipSuccess) e = hipGetLastError();
    return dev(e, "ckks_sync");
}

extern "C" size_t ckks_workspace_bytes(const ckks_ctx *c, uint32_t op, uint32_t level)
{
    if (!c || level >= c->nq) return 0;
    const size_t N = c->N, n = level + 1;
    switch (op) {
    case CKKS_OP_MODUP: return n * N * 8;
    case CKKS_OP_MODDOWN: return ((size_t)c->np + n) * N * 8;
    case CKKS_OP_KEYSWITCH:
    case CKKS_OP_ROTATE:
    case CKKS_OP_HOISTED: return ks_ws_elems(c, level) * 8;
    case CKKS_OP_HMULT: return (ks_ws_elems(c, level) + n * N) * 8;
    case CKKS_OP_RESCALE: return (2 * N + 2 * (size_t)level * N) * 8;
    default: return 0;
    }
}

static ckks_status ntt_common(ckks_ctx *ctx, uint64_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream,
                              bool inverse)
{
    TRY(check_ctx(ctx));
    TRY(check_ptr(poly, inverse ? "ckks_intt" : "ckks_ntt"));
    if (n_limbs == 0 || limb0 + n_limbs > ctx->nq + ctx->np)
        return fail(CKKS_E_ARG, "ckks_(i)ntt: limb range outside q_0..q_L, p_0..p_{K-1}");
    NttArgs a = base_args(ctx, inverse);
    a.src = poly;
    a.dst = poly;
    a.map.rows = n_limbs;
    a.map.prime0 = limb0;
    hipError_t e = inverse ? launch_ntt_inv(a, n_limbs, PRO_PLAIN, S(stream), poly, 0)
                           : launch_ntt_fwd(a, n_limbs, PRO_PLAIN, EPI_PLAIN, S(stream), poly, 0);
    return dev(e, inverse ? "ckks_intt" : "ckks_ntt");
}

extern "C" ckks_status ckks_ntt_tile_set(uint32_t inverse, uint32_t n_limbs, uint32_t tile)
{
    if (!ntt_tile_set(inverse, n_limbs, tile))
        return fail(CKKS_E_ARG, "ckks_ntt_tile_set: inverse must be 0 or 1, n_limbs in [1, 128], tile 0, 4, 8 or 16");
    return CKKS_OK;
}

extern "C" uint32_t ckks_ntt_tile_get(uint32_t inverse, uint32_t n_limbs)
{
    return inverse <= 1 && n_limbs ? ntt_tile_get(inverse, n_limbs) : 0;
}

extern "C" ckks_status ckks_ntt(ckks_ctx *ctx, uint64_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream)
{
    return ntt_common(ctx, poly, limb0, n_limbs, stream, false);
}

extern "C" ckks_status ckks_intt(ckks_ctx *ctx, uint64_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream)
{
    return ntt_common(ctx, poly, limb0, n_limbs, stream, true);
}

extern "C" ckks_status ckks_modup(ckks_ctx *ctx, const uint64_t *d, uint32_t level, uint64_t *ext, void *ws,
                                  void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_level(ctx, level));
    TRY(check_ptr(d, "ckks_modup d"));
    TRY(check_ptr(ext, "ckks_modup ext"));
    TRY(check_ptr(ws, "ckks_modup ws"));
    KsSizes s = ks_sizes(ctx, level);
    size_t eb = (size_t)s.beta * s.rows * s.N * 8, db = poly_bytes(ctx, level);
    if (overlap(ext, eb, d, db) || overlap(ext, eb, ws, db) || overlap(d, db, ws, db))
        return fail(CKKS_E_ARG, "ckks_modup: d, ext and ws must not overlap");
    hipError_t e = modup_intt(ctx, d, 1, level, (uint64_t *)ws, S(stream));
    if (e == hipSuccess) e = modup_from_coeffs(ctx, d, 1, level, (uint64_t *)ws, ext, true, S(stream));
    return dev(e, "ckks_modup");
}

extern "C" ckks_status ckks_inner_product(ckks_ctx *ctx, const uint64_t *ext, uint32_t level, const ckks_key *key,
                                          uint32_t galois, uint64_t *acc, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_level(ctx, level));
    TRY(check_key(ctx, key));
    TRY(check_ptr(ext, "ckks_inner_product ext"));
    TRY(check_ptr(acc, "ckks_inner_product acc"));
    if (galois % 2 == 0 || galois >= 2 * ctx->N) return fail(CKKS_E_ARG, "ckks_inner_product: galois must be odd < 2N");
    KsSizes s = ks_sizes(ctx, level);
    if (overlap(ext, (size_t)s.beta * s.rows * s.N * 8, acc, 2 * (size_t)s.rows * s.N * 8))
        return fail(CKKS_E_ARG, "ckks_inner_product: acc overlaps ext");
    return dev(inner_product(ctx, ext, level, key->data, galois, acc, S(stream)), "ckks_inner_product");
}

extern "C" ckks_status ckks_moddown(ckks_ctx *ctx, const uint64_t *x, uint32_t level, uint64_t *out, void *ws,
                                    void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_level(ctx, level));
    TRY(check_ptr(x, "ckks_moddown x"));
    TRY(check_ptr(out, "ckks_moddown out"));
    TRY(check_ptr(ws, "ckks_moddown ws"));
    KsSizes s = ks_sizes(ctx, level);
    size_t xb = (size_t)s.rows * s.N * 8, ob = poly_bytes(ctx, level), wb = ckks_workspace_bytes(ctx, CKKS_OP_MODDOWN, level);
    if (overlap(x, xb, out, ob) || overlap(x, xb, ws, wb) || overlap(out, ob, ws, wb))
        return fail(CKKS_E_ARG, "ckks_moddown: x, out and ws must not overlap");
    uint64_t *pc = (uint64_t *)ws, *conv = pc + (size_t)ctx->np * s.N;
    uint64_t *outs[1] = {out};
    return dev(moddown(ctx, x, 0, 1, level, outs, nullptr, 1, pc, conv, S(stream)), "ckks_moddown");
}

extern "C" ckks_status ckks_key_wrap(ckks_ctx *ctx, const uint64_t *dev_key, uint32_t galois, ckks_key **out)
{
    TRY(check_ctx(ctx));
    if (!out) return fail(CKKS_E_ARG, "ckks_key_wrap: null output");
    TRY(check_ptr(dev_key, "ckks_key_wrap key"));
    if (galois != 0 && (galois % 2 == 0 || galois >= 2 * ctx->N || galois == 1))
        return fail(CKKS_E_KEY, "ckks_key_wrap: galois must be 0 or odd in (1, 2N)");
    ckks_key *k = new ckks_key();
    k->data = dev_key;
    k->galois = galois;
    k->ctx = ctx;
    *out = k;
    return CKKS_OK;
}

extern "C" void ckks_key_release(ckks_key *key) { delete key; }

namespace ckks {

// Validation shared by ckks_keyswitch and ckks_keyswitch_noalloc (everything but the workspace).
ckks_status check_keyswitch_args(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key,
                                 const uint64_t *out0, const uint64_t *out1, const char *what)
{
    TRY(check_ctx(ctx));
    TRY(check_level(ctx, level));
    TRY(check_key(ctx, key));
    TRY(check_ptr(d, (std::string(what) + " d").c_str()));
    TRY(check_ptr(out0, (std::string(what) + " out0").c_str()));
    TRY(check_ptr(out1, (std::string(what) + " out1").c_str()));
    const size_t pb = poly_bytes(ctx, level);
    if (overlap(out0, pb, d, pb) || overlap(out1, pb, d, pb) || overlap(out0, pb, out1, pb))
        return fail(CKKS_E_ARG, std::string(what) + ": d, out0 and out1 must not overlap");
    return CKKS_OK;
}

}  // namespace ckks

extern "C" ckks_status ckks_keyswitch(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key,
                                      uint64_t *out0, uint64_t *out1, void *ws, void *stream)
{
    TRY(check_keyswitch_args(ctx, d, level, key, out0, out1, "ckks_keyswitch"));
    TRY(check_ptr(ws, "ckks_keyswitch ws"));
    size_t pb = poly_bytes(ctx, level), wb = ckks_workspace_bytes(ctx, CKKS_OP_KEYSWITCH, level);
    if (overlap(ws, wb, d, pb) || overlap(ws, wb, out0, pb) || overlap(ws, wb, out1, pb))
        return fail(CKKS_E_ARG, "ckks_keyswitch: d, out0, out1 and ws must not overlap");
    return dev(keyswitch_core(ctx, d, 1, level, key->data, out0, out1, nullptr, nullptr, 1, ws, S(stream)),
               "ckks_keyswitch");
}

extern "C" ckks_status ckks_hmult_relin(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, const ckks_key *rlk,
                                        ckks_ct *out, void *ws, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_ct(ctx, a, "ckks_hmult_relin a"));
    TRY(check_ct(ctx, b, "ckks_hmult_relin b"));
    if (a->level != b->level) return fail(CKKS_E_LEVEL, "ckks_hmult_relin: operands at different levels");
    TRY(check_key(ctx, rlk));
    if (rlk->galois != 0) return fail(CKKS_E_KEY, "ckks_hmult_relin: key is not a relinearisation key");
    if (!out) return fail(CKKS_E_ARG, "ckks_hmult_relin: null output");
    uint32_t level = a->level;
    ckks_ct o = *out;
    o.level = level;
    TRY(check_ct(ctx, &o, "ckks_hmult_relin out"));
    TRY(check_ptr(ws, "ckks_hmult_relin ws"));
    TRY(check_disjoint(ctx, &o, a, level, level, "ckks_hmult_relin"));
    TRY(check_disjoint(ctx, &o, b, level, level, "ckks_hmult_relin"));
    size_t wb = ckks_workspace_bytes(ctx, CKKS_OP_HMULT, level), pb = poly_bytes(ctx, level);
    const void *all[6] = {a->c0, a->c1, b->c0, b->c1, o.c0, o.c1};
    for (int i = 0; i < 6; ++i)
        if (overlap(ws, wb, all[i], pb)) return fail(CKKS_E_ARG, "ckks_hmult_relin: workspace overlaps a polynomial");
    const size_t N = ctx->N;
    uint64_t *d2 = (uint64_t *)ws;
    void *ks_ws = d2 + (size_t)(level + 1) * N;
    hipError_t e;
    if (ctx->logn == 16) {
        const TensorIn tin = {a->c0, a->c1, b->c0, b->c1};
        e = keyswitch_core(ctx, nullptr, 1, level, rlk->data, o.c0, o.c1, nullptr, nullptr, 1, ks_ws, S(stream), &tin);
    } else {
        e = launch_tensor(a->c0, a->c1, b->c0, b->c1, o.c0, o.c1, d2, ctx->d_primes, level + 1, ctx->logn, S(stream));
        if (e == hipSuccess)
            e = keyswitch_core(ctx, d2, 1, level, rlk->data, o.c0, o.c1, o.c0, o.c1, 1, ks_ws, S(stream));
    }
    TRY(dev(e, "ckks_hmult_relin"));
    out->level = level;
    out->scale = a->scale * b->scale;
    return CKKS_OK;
}

extern "C" ckks_status ckks_rescale(ckks_ctx *ctx, const ckks_ct *in, ckks_ct *out, void *ws, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_ct(ctx, in, "ckks_rescale in"));
    if (in->level < 1) return fail(CKKS_E_LEVEL, "ckks_rescale: level 0 cannot be rescaled");
    if (!out) return fail(CKKS_E_ARG, "ckks_rescale: null output");
    const uint32_t l = in->level;
    ckks_ct o = *out;
    o.level = l - 1;
    TRY(check_ct(ctx, &o, "ckks_rescale out"));
    TRY(check_ptr(ws, "ckks_rescale ws"));
    const size_t N = ctx->N, ib = poly_bytes(ctx, l), ob = poly_bytes(ctx, l - 1);
    // in place (same buffers) is allowed, any other overlap is not
    const void *I[2] = {in->c0, in->c1}, *O[2] = {o.c0, o.c1};
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            if (overlap(O[x], ob, I[y], ib) && !(x == y && O[x] == I[y]))
                return fail(CKKS_E_ARG, "ckks_rescale: output overlaps input other than exactly in place");
    size_t wb = ckks_workspace_bytes(ctx, CKKS_OP_RESCALE, l);
    for (int x = 0; x < 2; ++x)
        if (overlap(ws, wb, I[x], ib) || overlap(ws, wb, O[x], ob))
            return fail(CKKS_E_ARG, "ckks_rescale: workspace overlaps a polynomial");
    uint64_t *v = (uint64_t *)ws, *mid = v + 2 * N;
    NttArgs ia = base_args(ctx, true);
    ia.src = in->c0 + (size_t)l * N;
    ia.dst = v;
    ia.map.rows = 1;
    ia.map.prime0 = l;
    ia.map.src_poly_stride = (int64_t)(in->c1 - in->c0);
    ia.map.dst_poly_stride = (int64_t)N;
    hipError_t e = launch_ntt_inv(ia, 2, PRO_PLAIN, S(stream), v, (int64_t)N);
    if (e == hipSuccess) {
        NttArgs a = base_args(ctx, false);
        a.src = v;
        a.dst = mid;
        a.map.rows = l;
        a.map.prime0 = 0;
        a.map.src_poly_stride = 0;
        a.map.dst_poly_stride = (int64_t)l * N;
        a.rs_src[0] = v;
        a.rs_src[1] = v + N;
        a.rs_qlmod = ctx->d_rs_mod + (size_t)l * ctx->nq;
        a.rs_ql = ctx->primes[l];
        a.cst = ctx->d_rs_inv + (size_t)l * ctx->nq;
        a.aux[0] = in->c0;
        a.aux[1] = in->c1;
        a.out[0] = o.c0;
        a.out[1] = o.c1;
        e = launch_ntt_fwd(a, 2 * l, PRO_RESCALE, EPI_RESCALE, S(stream), mid, (int64_t)l * N);
    }
    TRY(dev(e, "ckks_rescale"));
    out->level = l - 1;
    out->scale = in->scale / (double)ctx->primes[l];
    return CKKS_OK;
}

extern "C" ckks_status ckks_apply_galois(ckks_ctx *ctx, const ckks_ct *in, uint32_t galois, const ckks_key *key,
                                         ckks_ct *out, void *ws, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_ct(ctx, in, "ckks_apply_galois in"));
    TRY(check_key(ctx, key));
    if (galois % 2 == 0 || galois <= 1 || galois >= 2 * ctx->N)
        return fail(CKKS_E_ARG, "ckks_apply_galois: galois must be odd in (1, 2N)");
    if (key->galois != galois) return fail(CKKS_E_KEY, "ckks_apply_galois: key is for another Galois element");
    if (!out) return fail(CKKS_E_ARG, "ckks_apply_galois: null output");
    const uint32_t level = in->level;
    ckks_ct o = *out;
    o.level = level;
    TRY(check_ct(ctx, &o, "ckks_apply_galois out"));
    TRY(check_ptr(ws, "ckks_apply_galois ws"));
    TRY(check_disjoint(ctx, &o, in, level, level, "ckks_apply_galois"));
    size_t wb = ckks_workspace_bytes(ctx, CKKS_OP_ROTATE, level), pb = poly_bytes(ctx, level);
    const void *all[4] = {in->c0, in->c1, o.c0, o.c1};
    for (int i = 0; i < 4; ++i)
        if (overlap(ws, wb, all[i], pb)) return fail(CKKS_E_ARG, "ckks_apply_galois: workspace overlaps a polynomial");
    hipError_t e =
        keyswitch_core(ctx, in->c1, galois, level, key->data, o.c0, o.c1, in->c0, nullptr, galois, ws, S(stream));
    TRY(dev(e, "ckks_apply_galois"));
    out->level = level;
    out->scale = in->scale;
    return CKKS_OK;
}

extern "C" ckks_status ckks_hrotate(ckks_ctx *ctx, const ckks_ct *in, int32_t k, const ckks_key *key, ckks_ct *out,
                                    void *ws, void *stream)
{
    TRY(check_ctx(ctx));
    uint32_t g = galois_of_rotation(ctx, k);
    if (g == 1) return fail(CKKS_E_ARG, "ckks_hrotate: rotation by a multiple of N/2 is the identity");
    return ckks_apply_galois(ctx, in, g, key, out, ws, stream);
}

extern "C" ckks_status ckks_conjugate(ckks_ctx *ctx, const ckks_ct *in, const ckks_key *key, ckks_ct *out, void *ws,
                                      void *stream)
{
    TRY(check_ctx(ctx));
    return ckks_apply_galois(ctx, in, 2 * ctx->N - 1, key, out, ws, stream);
}

extern "C" ckks_status ckks_hrotate_hoisted(ckks_ctx *ctx, const ckks_ct *in, uint32_t n, const int32_t *k,
                                            const ckks_key *const *keys, ckks_ct *out, void *ws, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_ct(ctx, in, "ckks_hrotate_hoisted in"));
    if (n == 0) return CKKS_OK;
    if (!k || !keys || !out) return fail(CKKS_E_ARG, "ckks_hrotate_hoisted: null array");
    TRY(check_ptr(ws, "ckks_hrotate_hoisted ws"));
    const uint32_t level = in->level;
    size_t wb = ckks_workspace_bytes(ctx, CKKS_OP_HOISTED, level), pb = poly_bytes(ctx, level);
    std::vector<uint32_t> gs(n);
    for (uint32_t i = 0; i < n; ++i) {
        gs[i] = galois_of_rotation(ctx, k[i]);
        if (gs[i] == 1) return fail(CKKS_E_ARG, "ckks_hrotate_hoisted: rotation by a multiple of N/2");
        TRY(check_key(ctx, keys[i]));
        if (keys[i]->galois != gs[i]) return fail(CKKS_E_KEY, "ckks_hrotate_hoisted: key " + std::to_string(i) +
                                                                  " is for another Galois element");
        ckks_ct o = out[i];
        o.level = level;
        TRY(check_ct(ctx, &o, "ckks_hrotate_hoisted out"));
        TRY(check_disjoint(ctx, &o, in, level, level, "ckks_hrotate_hoisted"));
        if (overlap(ws, wb, o.c0, pb) || overlap(ws, wb, o.c1, pb))
            return fail(CKKS_E_ARG, "ckks_hrotate_hoisted: workspace overlaps an output");
        for (uint32_t j = 0; j < i; ++j) {
            ckks_ct p = out[j];
            p.level = level;
            TRY(check_disjoint(ctx, &o, &p, level, level, "ckks_hrotate_hoisted outputs"));
        }
    }
    if (overlap(ws, wb, in->c0, pb) || overlap(ws, wb, in->c1, pb))
        return fail(CKKS_E_ARG, "ckks_hrotate_hoisted: workspace overlaps the input");
    KsSizes s = ks_sizes(ctx, level);
    KsWs w = ks_ws(ctx, level, ws);
    hipError_t e = modup_intt(ctx, in->c1, 1, level, w.dc, S(stream));
    if (e == hipSuccess) e = modup_from_coeffs(ctx, in->c1, 1, level, w.dc, w.ext, false, S(stream));
    const int64_t acc_stride = (int64_t)s.rows * s.N;
    const bool rowpass = ctx->logn == 16;  // the inner product runs the special rows' first INTT pass
    for (uint32_t i = 0; i < n && e == hipSuccess; ++i) {
        const IpArgs ip = args_ip(ctx, w.ext, level, keys[i]->data, gs[i], w.acc, in->c1, gs[i]);
        e = rowpass ? launch_inner_product_rowpass(ip, args_moddown_intt(ctx, w.acc, acc_stride, level, w.pc), S(stream))
                    : launch_inner_product(ip, S(stream));
        if (e != hipSuccess) break;
        uint64_t *outs[2] = {out[i].c0, out[i].c1};
        const uint64_t *adds[2] = {in->c0, nullptr};
        e = moddown(ctx, w.acc, acc_stride, 2, level, outs, adds, gs[i], w.pc, w.conv, S(stream), rowpass);
    }
    TRY(dev(e, "ckks_hrotate_hoisted"));
    for (uint32_t i = 0; i < n; ++i) {
        out[i].level = level;
        out[i].scale = in->scale;
    }
    return CKKS_OK;
}

static ckks_status elementwise(ckks_ctx *ctx, int op, const uint64_t *a, const uint64_t *b, const uint64_t *c,
                               uint64_t *out, const uint64_t *host_scalars, uint32_t level, void *stream,
                               const char *what)
{
    TRY(check_ctx(ctx));
    if (level >= ctx->nq + ctx->np) return fail(CKKS_E_LEVEL, std::string(what) + ": more rows than primes");
    TRY(check_ptr(a, what));
    TRY(check_ptr(out, what));
    if (op <= 3) TRY(check_ptr(b, what));
    if (op == 3) TRY(check_ptr(c, what));
    if (op >= 4) {
        if (!host_scalars) return fail(CKKS_E_ARG, std::string(what) + ": null scalars");
        for (uint32_t i = 0; i <= level; ++i)
            if (host_scalars[i] >= ctx->primes[i])
                return fail(CKKS_E_ARG, std::string(what) + ": scalar not reduced modulo its prime");
    }
    size_t pb = poly_bytes(ctx, level);
    const uint64_t *ins[3] = {a, op <= 3 ? b : nullptr, op == 3 ? c : nullptr};
    for (int i = 0; i < 3; ++i)
        if (ins[i] && ins[i] != out && overlap(ins[i], pb, out, pb))
            return fail(CKKS_E_ARG, std::string(what) + ": output partially overlaps an input");
    return dev(launch_elementwise(op, a, b, c, out, host_scalars, ctx->d_primes, level + 1, ctx->logn, S(stream)),
               what);
}

extern "C" ckks_status ckks_poly_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                     uint32_t level, void *stream)
{
    return elementwise(ctx, 0, a, b, nullptr, out, nullptr, level, stream, "ckks_poly_add");
}

extern "C" ckks_status ckks_poly_sub(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                     uint32_t level, void *stream)
{
    return elementwise(ctx, 1, a, b, nullptr, out, nullptr, level, stream, "ckks_poly_sub");
}

extern "C" ckks_status ckks_poly_mul(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                     uint32_t level, void *stream)
{
    return elementwise(ctx, 2, a, b, nullptr, out, nullptr, level, stream, "ckks_poly_mul");
}

extern "C" ckks_status ckks_poly_mul_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, const uint64_t *c,
                                         uint64_t *out, uint32_t level, void *stream)
{
    return elementwise(ctx, 3, a, b, c, out, nullptr, level, stream, "ckks_poly_mul_add");
}

extern "C" ckks_status ckks_poly_scalar_mul(ckks_ctx *ctx, const uint64_t *a, const uint64_t *s, uint64_t *out,
                                            uint32_t level, void *stream)
{
    return elementwise(ctx, 4, a, nullptr, nullptr, out, s, level, stream, "ckks_poly_scalar_mul");
}

extern "C" ckks_status ckks_poly_scalar_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *s, uint64_t *out,
                                            uint32_t level, void *stream)
{
    return elementwise(ctx, 5, a, nullptr, nullptr, out, s, level, stream, "ckks_poly_scalar_add");
}

// Table I support operations on whole ciphertexts (one launch over both halves)
static ckks_status ct_op(ckks_ctx *ctx, int op, const ckks_ct *a, const ckks_ct *b, const uint64_t *pt,
                         const uint64_t *s, double scale_mul, ckks_ct *out, void *stream, const char *what)
{
    TRY(check_ctx(ctx));
    TRY(check_ct(ctx, a, what));
    const uint32_t level = a->level;
    if (op == CT_HADD) {
        TRY(check_ct(ctx, b, what));
        if (b->level != level) return fail(CKKS_E_LEVEL, std::string(what) + ": operands at different levels");
    }
    const bool uses_pt = op == CT_PTADD || op == CT_PTMULT, uses_s = op == CT_SCALAR_ADD || op == CT_SCALAR_MULT;
    if (uses_pt) TRY(check_ptr(pt, what));
    if (uses_s) {
        if (!s) return fail(CKKS_E_ARG, std::string(what) + ": null scalars");
        for (uint32_t i = 0; i <= level; ++i)
            if (s[i] >= ctx->primes[i]) return fail(CKKS_E_ARG, std::string(what) + ": scalar not reduced modulo its prime");
    }
    if (!out) return fail(CKKS_E_ARG, std::string(what) + ": null output");
    ckks_ct o = *out;
    o.level = level;
    TRY(check_ct(ctx, &o, what));
    const size_t pb = poly_bytes(ctx, level);
    // the output is either exactly an input's buffers (in place) or disjoint from every input
    const ckks_ct *ins[2] = {a, op == CT_HADD ? b : nullptr};
    for (const ckks_ct *x : ins)
        if (x && !(o.c0 == x->c0 && o.c1 == x->c1))
            TRY(check_disjoint(ctx, &o, x, level, level, what));
    if (uses_pt && (overlap(pt, pb, o.c0, pb) || overlap(pt, pb, o.c1, pb)))
        return fail(CKKS_E_ARG, std::string(what) + ": output overlaps the plaintext");
    CtOpArgs args;
    memset(&args, 0, sizeof(args));
    args.a[0] = a->c0;
    args.a[1] = a->c1;
    args.b[0] = op == CT_HADD ? b->c0 : pt;
    args.b[1] = op == CT_HADD ? b->c1 : pt;
    args.out[0] = o.c0;
    args.out[1] = o.c1;
    args.primes = ctx->d_primes;
    args.logn = ctx->logn;
    if (uses_s)
        for (uint32_t i = 0; i <= level; ++i) args.s[i] = s[i];
    const bool copy_half = op == CT_PTADD || op == CT_SCALAR_ADD;
    const uint32_t halves = copy_half && o.c1 == a->c1 ? 1 : 2;
    TRY(dev(launch_ct_op(op, args, level + 1, halves, S(stream)), what));
    out->level = level;
    out->scale = a->scale * scale_mul;
    return CKKS_OK;
}

extern "C" ckks_status ckks_hadd(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, void *stream)
{
    return ct_op(ctx, CT_HADD, a, b, nullptr, nullptr, 1.0, out, stream, "ckks_hadd");
}

extern "C" ckks_status ckks_ptadd(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *pt, ckks_ct *out, void *stream)
{
    return ct_op(ctx, CT_PTADD, a, nullptr, pt, nullptr, 1.0, out, stream, "ckks_ptadd");
}

extern "C" ckks_status ckks_ptmult(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *pt, double pt_scale, ckks_ct *out,
                                   void *stream)
{
    return ct_op(ctx, CT_PTMULT, a, nullptr, pt, nullptr, pt_scale, out, stream, "ckks_ptmult");
}

extern "C" ckks_status ckks_scalar_add(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *s, ckks_ct *out, void *stream)
{
    return ct_op(ctx, CT_SCALAR_ADD, a, nullptr, nullptr, s, 1.0, out, stream, "ckks_scalar_add");
}

extern "C" ckks_status ckks_scalar_mult(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *s, double s_scale,
                                        ckks_ct *out, void *stream)
{
    return ct_op(ctx, CT_SCALAR_MULT, a, nullptr, nullptr, s, s_scale, out, stream, "ckks_scalar_mult");
}

extern "C" ckks_status ckks_hsquare(ckks_ctx *ctx, const ckks_ct *a, const ckks_key *rlk, ckks_ct *out, void *ws,
                                    void *stream)
{
    return ckks_hmult_relin(ctx, a, a, rlk, out, ws, stream);
}

extern "C" ckks_status ckks_automorph(ckks_ctx *ctx, const uint64_t *in, uint32_t galois, uint64_t *out,
                                      uint32_t n_limbs, void *stream)
{
    TRY(check_ctx(ctx));
    TRY(check_ptr(in, "ckks_automorph in"));
    TRY(check_ptr(out, "ckks_automorph out"));
    if (n_limbs == 0 || n_limbs > ctx->nq + ctx->np) return fail(CKKS_E_ARG, "ckks_automorph: bad limb count");
    if (galois % 2 == 0 || galois >= 2 * ctx->N) return fail(CKKS_E_ARG, "ckks_automorph: galois must be odd < 2N");
    size_t b = (size_t)n_limbs * ctx->N * 8;
    if (overlap(in, b, out, b)) return fail(CKKS_E_ARG, "ckks_automorph: out overlaps in");
    return dev(launch_automorph(in, out, n_limbs, ctx->logn, galois, S(stream)), "ckks_automorph");
}
