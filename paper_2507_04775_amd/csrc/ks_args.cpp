// Argument blocks of the key-switching steps (paper Sec. II-A, III-F.3 to
// III-F.5), shared by the single-operation calls and the batch planner.
#include "ks_args.h"

#include <string.h>

namespace ckks {

KsSizes ks_sizes(const ckks_ctx *c, uint32_t level)
{
    KsSizes s;
    s.n = level + 1;
    s.rows = s.n + c->np;
    s.beta = (s.n + c->alpha - 1) / c->alpha;
    s.N = c->N;
    return s;
}

size_t ks_ws_elems(const ckks_ctx *c, uint32_t level)
{
    KsSizes s = ks_sizes(c, level);
    return ((size_t)s.n + (size_t)s.beta * s.rows + 2 * (size_t)s.rows + 2 * (size_t)c->np + 2 * (size_t)s.n) * s.N;
}

KsWs ks_ws(const ckks_ctx *c, uint32_t level, void *ws)
{
    KsSizes s = ks_sizes(c, level);
    KsWs w;
    w.dc = (uint64_t *)ws;
    w.ext = w.dc + (size_t)s.n * s.N;
    w.acc = w.ext + (size_t)s.beta * s.rows * s.N;
    w.pc = w.acc + 2 * (size_t)s.rows * s.N;
    w.conv = w.pc + 2 * (size_t)c->np * s.N;
    return w;
}

NttArgs base_args(const ckks_ctx *c, bool inverse)
{
    NttArgs a;
    memset(&a, 0, sizeof(a));
    a.primes = c->d_primes;
    a.tw = inverse ? c->d_tw_inv : c->d_tw_fwd;
    a.twd = inverse ? c->d_twd_inv : c->d_twd_fwd;
    a.logn = c->logn;
    a.galois = 1;
    a.map.nq = c->nq;
    a.map.level = kAllPrimes;
    for (size_t i = 0; i < c->primes.size() && i < 64; ++i)
        if (c->primes[i] >= kFpMaxPrime) a.int_primes |= 1ull << i;
    return a;
}

NttArgs args_modup_intt(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, uint64_t *dc)
{
    NttArgs a = base_args(c, true);
    a.src = d;
    a.dst = dc;
    a.mid = dc;
    a.mid_stride = 0;
    a.galois = g;
    a.map.rows = level + 1;
    a.map.prime0 = 0;
    a.ys_mode = 1;
    a.alpha = c->alpha;
    a.nlev = level + 1;
    a.ys = c->d_bc_ys;
    a.ysd = c->d_bc_ysd;
    return a;
}

BconvArgs args_modup_bconv(const ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *dc,
                           uint64_t *ext, bool copy_own)
{
    KsSizes s = ks_sizes(c, level);
    BconvArgs b;
    memset(&b, 0, sizeof(b));
    const size_t hm_stride = (size_t)(c->nq + c->np) * kMaxDigitPrimes;
    for (uint32_t j = 0; j < s.beta; ++j) {
        uint32_t lo = j * c->alpha, hi = lo + c->alpha < s.n ? lo + c->alpha : s.n;
        uint32_t set = c->set_index(j, hi - lo);
        BconvJob &J = b.job[j];
        J.src = dc + (size_t)lo * s.N;
        J.dst = ext + (size_t)j * s.rows * s.N;
        J.copy_src = copy_own ? d : nullptr;
        J.hinv = c->d_bc_hinv + (size_t)set * kMaxDigitPrimes;
        J.hmod = c->d_bc_hmod + (size_t)set * hm_stride;
        J.ns = hi - lo;
        J.src_prime0 = lo;
        J.lo = lo;
        J.hi = hi;
    }
    b.primes = c->d_primes;
    b.nrows = s.rows;
    b.level = level;
    b.nq = c->nq;
    b.N = c->N;
    b.logn = c->logn;
    b.copy_galois = g;
    b.prescaled = 1;
    return b;
}

NttArgs args_modup_ntt(const ckks_ctx *c, uint32_t level, uint64_t *ext)
{
    KsSizes s = ks_sizes(c, level);
    NttArgs a = base_args(c, false);
    a.src = ext;
    a.dst = ext;
    a.mid = ext;
    a.mid_stride = (int64_t)s.rows * s.N;
    a.map.rows = s.rows;
    a.map.level = level;
    a.map.skip_alpha = c->alpha;
    a.map.src_poly_stride = a.map.dst_poly_stride = (int64_t)s.rows * s.N;
    return a;
}

IpArgs args_ip(const ckks_ctx *c, const uint64_t *ext, uint32_t level, const uint64_t *key, uint32_t g,
               uint64_t *acc, const uint64_t *own, uint32_t own_galois)
{
    KsSizes s = ks_sizes(c, level);
    IpArgs a;
    a.ext = ext;
    a.key = key;
    a.acc = acc;
    a.primes = c->d_primes;
    a.beta = s.beta;
    a.rows = s.rows;
    a.level = level;
    a.nq = c->nq;
    a.np = c->np;
    a.logn = c->logn;
    a.alpha = c->alpha;
    a.galois = g;
    a.own = own;
    a.own_galois = own_galois;
    a.ta0 = a.ta1 = a.tb0 = a.tb1 = nullptr;
    a.pmod = c->d_pmod;
    a.fold_c0 = nullptr;
    a.fold_tot = nullptr;
    a.fold_first = a.fold_pad = 0;
    return a;
}

NttArgs args_moddown_intt(const ckks_ctx *c, const uint64_t *acc, int64_t acc_stride, uint32_t level, uint64_t *pc)
{
    KsSizes s = ks_sizes(c, level);
    const int64_t kN = (int64_t)c->np * s.N, nN = (int64_t)s.n * s.N;
    NttArgs ia = base_args(c, true);
    ia.src = acc + nN;
    ia.dst = pc;
    ia.mid = pc;
    ia.mid_stride = kN;
    ia.map.rows = c->np;
    ia.map.level = level;
    ia.map.row0 = s.n;
    ia.map.src_poly_stride = acc_stride;
    ia.map.dst_poly_stride = kN;
    ia.ys_mode = 2;
    ia.pset = c->pset_index();
    ia.ys = c->d_bc_ys;
    ia.ysd = c->d_bc_ysd;
    return ia;
}

NttArgs args_moddown_ntt(const ckks_ctx *c, const uint64_t *acc, int64_t acc_stride, uint32_t npoly, uint32_t level,
                         uint64_t *const *out, const uint64_t *const *add, uint32_t g, const uint64_t *pc,
                         uint64_t *conv)
{
    KsSizes s = ks_sizes(c, level);
    const int64_t kN = (int64_t)c->np * s.N, nN = (int64_t)s.n * s.N;
    NttArgs a = base_args(c, false);
    a.src = conv;
    a.dst = conv;
    a.mid = conv;
    a.mid_stride = nN;
    a.map.rows = s.n;
    a.map.level = level;
    a.map.src_poly_stride = a.map.dst_poly_stride = nN;
    a.galois = g;
    a.cst = c->d_pinv;
    a.bc_mode = 2;
    a.bc_src = pc;
    a.bc_poly_stride = kN;
    a.pset = c->pset_index();
    a.nprimes = c->nq + c->np;
    a.hmod = c->d_bc_hmod;
    a.pmod = c->d_pmod;
    for (uint32_t t = 0; t < npoly; ++t) {
        a.aux[t] = acc + t * acc_stride;
        a.add[t] = add ? add[t] : nullptr;
        a.out[t] = out[t];
    }
    return a;
}

}  // namespace ckks
