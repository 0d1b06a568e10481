// Bootstrapping executor (paper Sec. III-F.7): ModRaise, CoeffToSlot as
// merged special-FFT stages evaluated with baby-step/giant-step over hoisted
// rotations, EvalMod as a Chebyshev product tree plus double-angle steps, and
// SlotToCoeff.  EvalMod evaluates the Chebyshev series by baby-step/giant-step
// (a tree of Chebyshev divisions p = q T_G + r over power-of-two giants, with
// integer combinations of the babies at the leaves).  The schedule (levels, layouts, rotations, constants) is
// derived here from the descriptor; the plaintext diagonals arrive as
// integer-valued doubles and are reduced and transformed on the device once,
// at creation.  A run is a fixed host-side sequence of library operations on
// one stream, so it can be captured into a HIP graph.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "internal.h"
#include "ks_args.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
}

using namespace ckks;

namespace {

#define TRY(x)                              \
    do {                                    \
        ckks_status _s = (x);               \
        if (_s != CKKS_OK) return _s;       \
    } while (0)

hipStream_t S(void *stream) { return (hipStream_t)stream; }

ckks_status dev(hipError_t e, const char *what)
{
    if (e == hipSuccess) return CKKS_OK;
    return fail(CKKS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Layout {
    int32_t m_lo;
    uint32_t count, baby, giants, h0;
};

// Diagonals of a group of r stages with smallest half-size h0 sit at offsets
// m h0, m in [m_lo, m_lo + count); index i = m - m_lo = g baby + b.
Layout group_layout(uint32_t n, uint32_t r, uint32_t h0)
{
    Layout L;
    const uint32_t R = 1u << r;
    L.h0 = h0;
    if ((uint64_t)R * h0 == n) {
        L.m_lo = 0;
        L.count = R;
    } else {
        L.m_lo = -(int32_t)(R - 1);
        L.count = 2 * R - 1;
    }
    L.baby = 1;
    while (L.baby * L.baby < L.count) L.baby *= 2;
    L.giants = (L.count + L.baby - 1) / L.baby;
    return L;
}

double round_half_away(double v)
{
    const double a = floor(fabs(v) + 0.5);
    return v >= 0 ? a : -a;
}

struct Group {
    Layout lay;
    uint32_t level;      // input level
    uint32_t rescales;
    std::vector<int32_t> giant;   // G_g
    std::vector<int32_t> baby_k;  // b h0, b = 1..min(baby, count)-1
    uint64_t *pt = nullptr;       // [count][level+1][N], evaluation domain
};

// One node of the baby-step/giant-step Chebyshev evaluation: a leaf
// c_0 + sum_k c_k T_k below the baby size, or a split p = q T_G + r.
struct ChebNode {
    bool leaf = false;
    std::vector<double> c;  // leaf coefficients c_0..c_D
    size_t cst = 0;         // leaf: offset of its [D][t+2] constant residues in the device table
    uint32_t G = 0;
    int q = -1, r = -1;     // children; q = -1 when the quotient is the constant q0
    double q0 = 0;
    int level = 0;          // level of the result relative to the EvalMod input
};

// p = q T_G + r for Chebyshev coefficients c of degree D, G <= D < 2G:
// q_0 = c_G, q_i = 2 c_(G+i), r_(G-i) = c_(G-i) - c_(G+i).
void cheb_split(const std::vector<double> &c, uint32_t G, std::vector<double> &q, std::vector<double> &r)
{
    const uint32_t D = (uint32_t)c.size() - 1;
    q.assign(D - G + 1, 0.0);
    r.assign(c.begin(), c.begin() + G);
    q[0] = c[G];
    for (uint32_t i = 1; i <= D - G; ++i) {
        q[i] = 2.0 * c[G + i];
        r[G - i] = r[G - i] - c[G + i];
    }
}

// Resources of one execution lane: the caller's stream (lane 0) or an
// internal stream, its own workspace and buffers, so lanes never share a
// buffer.  Independent work (giant steps of a linear transform, the two EvalMod
// halves) runs on different lanes and overlaps on the GPU; every lane's work
// is forked from and joined back into the caller's stream with events, which
// also makes the whole bootstrap capturable as one graph.  Lanes 0 and 1 run
// an EvalMod half each and hold its buffers; lanes 2 and 3 only giant steps.
struct Lane {
    hipStream_t aux = nullptr;       // internal stream (null for lane 0)
    void *ws = nullptr;
    uint32_t p = 0, r = 0, acc = 0;  // BSGS partial sum, rotated partial sum, lane accumulator
    uint32_t d = 0;                  // three level-down temporaries d, d+1, d+2
    uint32_t t = 0, g = 0, pool = 0; // babies T_2.., giants, Chebyshev buffer pool
};

constexpr uint32_t kLanes = 4;

// A ciphertext held in one of the executor's buffers (or the caller's output).
struct Ct {
    uint64_t *c0, *c1;
    uint32_t level;
};

}  // namespace

struct ckks_boot {
    ckks_ctx *ctx = nullptr;
    bool owns_dev = false;  // dev was allocated by the handle (else it is the caller's buffer)
    uint32_t L = 0, n = 0, N = 0;
    std::vector<Group> cts, stc;
    uint32_t degree = 0, double_angles = 0, evalmod_in = 0, out_level = 0, keyswitches = 0;
    std::vector<double> cheb, sc;  // Chebyshev coefficients; level scales
    // baby-step/giant-step evaluation: baby size, giants (2b, 4b, ..), levels of T_k relative
    // to the EvalMod input, leaf level, the node tree (root last) and the leaf constants
    uint32_t baby = 0, nbaby = 0;
    std::vector<uint32_t> giants;
    std::map<uint32_t, int> lvT;
    int t_leaf = 0;
    std::vector<ChebNode> nodes;
    uint64_t *leaf_cst = nullptr;
    const ckks_key *relin = nullptr, *conj = nullptr, *to_sparse = nullptr, *from_sparse = nullptr;
    std::map<uint32_t, const ckks_key *> rot;  // slot rotation mod n -> key
    void *dev = nullptr;
    size_t bytes = 0;
    uint64_t *mono = nullptr;   // [L+1][N]: X^(N/2) in the evaluation domain
    uint64_t *slots = nullptr;  // nslots buffers of 2 (L+1) N words
    size_t slot_words = 0;
    uint32_t nslots = 0, max_baby = 1;
    size_t ws_bytes = 0;
    // hoisted ModDown: per lane an extended accumulator pair [2][l+1+K][N] (qp_words per lane)
    bool hoist = false;
    uint64_t gain = 1;  // integer the level-0 input is multiplied by before ModRaise
    uint64_t *qp = nullptr;
    size_t qp_words = 0;
    Lane lanes[kLanes];
    // Fork / join events: one run records each event once, so within a capture
    // no event is re-recorded after a wait on it has been captured.  The count
    // is fixed by the schedule (events_per_run).  lane_open[l] is set while lane
    // l has work that is not yet joined back into the caller's stream.
    std::vector<hipEvent_t> events;
    uint32_t next_event = 0;
    bool lane_open[kLanes] = {};
    hipEvent_t close_events[kLanes] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    // buffers shared by the lanes: hoisted babies, group outputs, the split and EvalMod halves
    uint32_t s_babies() const { return 0; }  // max_baby - 1 buffers
    uint32_t s_out(uint32_t i) const { return max_baby - 1 + i; }  // i = 0, 1
    uint32_t s_x() const { return max_baby + 1; }
    uint32_t s_cj() const { return max_baby + 2; }
    uint32_t s_re(uint32_t i) const { return max_baby + 3 + i; }
    uint32_t s_im(uint32_t i) const { return max_baby + 5 + i; }
    uint32_t shared_slots() const { return max_baby + 7; }
    uint32_t pool_size() const { return 2 * (uint32_t)giants.size() + 6; }
    // lane 0 accumulates into the transform's output buffer, the others into their own
    uint32_t lane_slots(uint32_t l) const
    {
        return 2 + (l > 0) + (l < 2 ? 3 + (nbaby - 1) + (uint32_t)giants.size() + pool_size() : 0);
    }
    uint32_t slot_count() const
    {
        uint32_t c = shared_slots();
        for (uint32_t l = 0; l < kLanes; ++l) c += lane_slots(l);
        return c;
    }
    void assign_lanes(uint8_t *ws_base)
    {
        uint32_t next = shared_slots();
        for (uint32_t l = 0; l < kLanes; ++l) {
            Lane &ln = lanes[l];
            const uint32_t b0 = next;
            ln.p = b0;
            ln.r = b0 + 1;
            ln.acc = l > 0 ? b0 + 2 : UINT32_MAX;
            ln.d = b0 + 2 + (l > 0);
            ln.t = ln.d + 3;
            ln.g = ln.t + (nbaby - 1);
            ln.pool = ln.g + (uint32_t)giants.size();
            next += lane_slots(l);
            ln.ws = ws_base + l * ws_bytes;
        }
    }
    hipEvent_t event() { return next_event < events.size() ? events[next_event++] : nullptr; }

    Ct slot(uint32_t i, uint32_t level) const
    {
        uint64_t *b = slots + (size_t)i * slot_words;
        return Ct{b, b + (size_t)(L + 1) * N, level};
    }
};

namespace {

ckks_ct as_ct(const Ct &c) { return ckks_ct{c.c0, c.c1, c.level, 1.0}; }

struct Runner {
    ckks_boot *b;
    hipStream_t st;
    const Lane *ln;
    std::vector<uint64_t> res;

    ckks_ctx *ctx() const { return b->ctx; }

    // Lanes 1..nl-1 start after the work issued so far on the caller's stream.
    ckks_status fork(uint32_t nl)
    {
        if (nl < 2) return CKKS_OK;
        hipEvent_t e = b->event();
        if (!e) return fail(CKKS_E_DEVICE, "ckks_bootstrap: fork/join events exhausted");
        TRY(dev(hipEventRecord(e, st), "ckks_bootstrap fork"));
        for (uint32_t l = 1; l < nl; ++l) {
            TRY(dev(hipStreamWaitEvent(b->lanes[l].aux, e, 0), "ckks_bootstrap fork"));
            b->lane_open[l] = true;
        }
        return CKKS_OK;
    }

    // The caller's stream continues after everything issued so far on lane l.
    ckks_status join(uint32_t l)
    {
        hipEvent_t e = b->event();
        if (!e) return fail(CKKS_E_DEVICE, "ckks_bootstrap: fork/join events exhausted");
        TRY(dev(hipEventRecord(e, b->lanes[l].aux), "ckks_bootstrap join"));
        TRY(dev(hipStreamWaitEvent(st, e, 0), "ckks_bootstrap join"));
        b->lane_open[l] = false;
        return CKKS_OK;
    }

    const uint64_t *residues(int64_t C, uint32_t level)
    {
        res.resize(level + 1);
        for (uint32_t i = 0; i <= level; ++i) {
            const int64_t q = (int64_t)ctx()->primes[i];
            int64_t r = C % q;
            res[i] = (uint64_t)(r < 0 ? r + q : r);
        }
        return res.data();
    }

    ckks_status rescale(Ct &c, const Ct *dst = nullptr)
    {
        ckks_ct in = as_ct(c), out = dst ? as_ct(*dst) : in;
        TRY(ckks_rescale(ctx(), &in, &out, ln->ws, st));
        c = Ct{out.c0, out.c1, c.level - 1};
        return CKKS_OK;
    }

    ckks_status scalar_mul(const Ct &src, const Ct &dst, int64_t C)
    {
        const uint64_t *r = residues(C, src.level);
        TRY(ckks_poly_scalar_mul(ctx(), src.c0, r, dst.c0, src.level, st));
        return ckks_poly_scalar_mul(ctx(), src.c1, r, dst.c1, src.level, st);
    }

    ckks_status scalar_add(const Ct &c, double v)
    {
        return ckks_poly_scalar_add(ctx(), c.c0, residues((int64_t)round_half_away(v * b->sc[c.level]), c.level),
                                    c.c0, c.level, st);
    }

    ckks_status add(const Ct &x, const Ct &y, const Ct &out, bool sub = false)
    {
        auto f = sub ? ckks_poly_sub : ckks_poly_add;
        TRY(f(ctx(), x.c0, y.c0, out.c0, x.level, st));
        return f(ctx(), x.c1, y.c1, out.c1, x.level, st);
    }

    // src times the real c, taken to level t < src.level, written to dst
    ckks_status mult_const_to(const Ct &src, double c, uint32_t t, const Ct &dst_buf, Ct &out)
    {
        const double X = (b->sc[t] * (double)ctx()->primes[t + 1]) / b->sc[src.level];
        Ct d{dst_buf.c0, dst_buf.c1, t + 1};
        TRY(scalar_mul(Ct{src.c0, src.c1, t + 1}, d, (int64_t)round_half_away(c * X)));
        TRY(rescale(d));
        out = d;
        return CKKS_OK;
    }

    ckks_status level_down(const Ct &src, uint32_t t, const Ct &buf, Ct &out)
    {
        if (src.level == t) {
            out = src;
            return CKKS_OK;
        }
        return mult_const_to(src, 1.0, t, buf, out);
    }

    // dst = rescale(relin(x y)) at the lower of the two levels
    ckks_status mul(const Ct &x, const Ct &y, const Ct &dst_buf, Ct &out)
    {
        const uint32_t l = std::min(x.level, y.level);
        Ct a, c;
        TRY(level_down(x, l, b->slot(ln->d, 0), a));
        if (y.c0 == x.c0) {
            c = a;
        } else {
            TRY(level_down(y, l, b->slot(ln->d + 1, 0), c));
        }
        ckks_ct A = as_ct(a), B = as_ct(c), O = as_ct(Ct{dst_buf.c0, dst_buf.c1, l});
        TRY(ckks_hmult_relin(ctx(), &A, &B, b->relin, &O, ln->ws, st));
        out = Ct{dst_buf.c0, dst_buf.c1, l};
        return rescale(out);
    }

    // Giant steps with the ModDown hoisted out of the loop: each lane sums its
    // giants' parts over Q u P (a key switch left in the extended basis plus
    // P phi_G(s_0), or P s for G = 0), the lanes' sums are added after the
    // join, and one ModDown per half brings the total back to Q.
    ckks_status giants_hoisted(const Group &g, const std::vector<Ct> &src, uint32_t acc_slot)
    {
        const uint32_t lvl = g.level, rows = lvl + 1 + ctx()->np;
        const size_t N = b->N, limb = (size_t)(lvl + 1) * N;
        Runner lr[kLanes] = {*this, *this, *this, *this};
        const uint32_t nl = std::min<uint32_t>(kLanes, g.lay.giants);
        TRY(fork(nl));
        for (uint32_t l = 1; l < nl; ++l) {
            lr[l].st = b->lanes[l].aux;
            lr[l].ln = &b->lanes[l];
        }
        auto tot = [&](uint32_t l) { return b->qp + (size_t)l * b->qp_words; };
        FoldArgs base;
        memset(&base, 0, sizeof(base));
        base.pmod = ctx()->d_pmod;
        base.primes = ctx()->d_primes;
        base.level = lvl;
        base.nq = ctx()->nq;
        base.logn = ctx()->logn;
        bool started[kLanes] = {};
        // each lane takes giants gi = lane mod nl; two of them with the same number of babies share
        // one lincomb, which reads the babies once (outputs in the lane's slots p and r)
        std::vector<uint32_t> mine[kLanes];
        for (uint32_t gi = 0; gi < g.lay.giants; ++gi) mine[gi % nl].push_back(gi);
        auto babies = [&](uint32_t gi) { return std::min(g.lay.baby, g.lay.count - gi * g.lay.baby); };
        size_t next[kLanes] = {};
        for (bool more = true; more;) {
            more = false;
            for (uint32_t ln = 0; ln < nl; ++ln) {
                if (next[ln] >= mine[ln].size()) continue;
                more = true;
                Runner &R_ = lr[ln];
                const Lane &L_ = *R_.ln;
                uint32_t pair[2] = {mine[ln][next[ln]], 0}, cnt = 1;
                if (next[ln] + 1 < mine[ln].size() && babies(mine[ln][next[ln] + 1]) == babies(pair[0]))
                    pair[cnt++] = mine[ln][next[ln] + 1];
                next[ln] += cnt;
                const Ct outs[2] = {b->slot(L_.p, lvl), b->slot(L_.r, lvl)};
                const uint32_t nb = babies(pair[0]);
                LincombArgs la;
                memset(&la, 0, sizeof(la));
                for (uint32_t j = 0; j < nb; ++j) {
                    la.a0[j] = src[j].c0;
                    la.a1[j] = src[j].c1;
                    for (uint32_t o = 0; o < cnt; ++o) la.pt[o][j] = g.pt + (size_t)(pair[o] * g.lay.baby + j) * limb;
                }
                for (uint32_t o = 0; o < cnt; ++o) {
                    la.out0[o] = outs[o].c0;
                    la.out1[o] = outs[o].c1;
                }
                la.primes = ctx()->d_primes;
                la.n = nb;
                la.nout = cnt;
                la.logn = ctx()->logn;
                TRY(dev(launch_lincomb(la, lvl + 1, R_.st), "ckks_bootstrap lincomb"));
                for (uint32_t o = 0; o < cnt; ++o) {
                    const Ct &P = outs[o];
                    const uint32_t G = (uint32_t)(((int64_t)g.giant[pair[o]] % b->n + b->n) % b->n);
                    const bool first = !started[ln];
                    started[ln] = true;
                    if (G != 0) {
                        // the giant step's key switch accumulates acc + [P]_q phi_g(c0) into the lane's
                        // total in its inner product's launch (no acc in memory, no fold launch)
                        const ckks_key *rk = b->rot.at(G);
                        TRY(dev(keyswitch_extended_fold(ctx(), P.c1, rk->galois, lvl, rk->data, L_.ws, R_.st, P.c0,
                                                        tot(ln), first),
                                "ckks_bootstrap giant key switch"));
                    } else {
                        FoldArgs fa = base;
                        fa.tot[0] = tot(ln);
                        fa.tot[1] = tot(ln) + (size_t)rows * N;
                        fa.first = first;
                        fa.s[0] = P.c0;
                        fa.s[1] = P.c1;
                        fa.galois = 1;
                        TRY(dev(launch_fold_ext(fa, rows, R_.st), "ckks_bootstrap fold"));
                    }
                }
            }
        }
        for (uint32_t l = 1; l < nl; ++l) {
            TRY(join(l));
            FoldArgs fa = base;
            fa.tot[0] = tot(0);
            fa.tot[1] = tot(0) + (size_t)rows * N;
            fa.acc[0] = tot(l);
            fa.acc[1] = tot(l) + (size_t)rows * N;
            fa.galois = 1;
            TRY(dev(launch_fold_ext(fa, rows, st), "ckks_bootstrap fold"));
        }
        const Ct acc = b->slot(acc_slot, lvl);
        return dev(moddown_pair(ctx(), tot(0), lvl, acc.c0, acc.c1, ln->ws, st), "ckks_bootstrap moddown");
    }

    ckks_status linear_transform(const Group &g, const Ct &in, uint32_t acc_slot, const Ct *final_out, Ct &out)
    {
        const uint32_t lvl = in.level;
        if (lvl != g.level) return fail(CKKS_E_LEVEL, "ckks_bootstrap: schedule level mismatch");
        const size_t N = b->N, limb = (size_t)(lvl + 1) * N;
        std::vector<Ct> src(1, in);
        if (!g.baby_k.empty()) {
            std::vector<const ckks_key *> keys;
            std::vector<ckks_ct> outs;
            for (size_t i = 0; i < g.baby_k.size(); ++i) {
                keys.push_back(b->rot.at((uint32_t)g.baby_k[i] % b->n));
                Ct o = b->slot(b->s_babies() + (uint32_t)i, lvl);
                src.push_back(o);
                outs.push_back(as_ct(o));
            }
            ckks_ct I = as_ct(in);
            TRY(ckks_hrotate_hoisted(ctx(), &I, (uint32_t)g.baby_k.size(), g.baby_k.data(), keys.data(), outs.data(),
                                     ln->ws, st));
        }
        if (b->hoist) {
            TRY(giants_hoisted(g, src, acc_slot));
            Ct c = b->slot(acc_slot, lvl);
            for (uint32_t r = 0; r < g.rescales; ++r) TRY(rescale(c, (r + 1 == g.rescales) ? final_out : nullptr));
            out = c;
            return CKKS_OK;
        }
        // giant steps round-robin over the lanes, each accumulating its own sum
        Runner lr[kLanes] = {*this, *this, *this, *this};
        const uint32_t nl = std::min<uint32_t>(kLanes, g.lay.giants);
        TRY(fork(nl));
        for (uint32_t l = 1; l < nl; ++l) {
            lr[l].st = b->lanes[l].aux;
            lr[l].ln = &b->lanes[l];
        }
        bool started[kLanes] = {};
        for (uint32_t gi = 0; gi < g.lay.giants; ++gi) {
            Runner &R_ = lr[gi % nl];
            const Lane &L_ = *R_.ln;
            const Ct acc = b->slot(gi % nl == 0 ? acc_slot : L_.acc, lvl), P = b->slot(L_.p, lvl),
                     R = b->slot(L_.r, lvl);
            const bool first = !started[gi % nl];
            started[gi % nl] = true;
            const uint32_t i0 = gi * g.lay.baby, nb = std::min(g.lay.baby, g.lay.count - i0);
            const uint32_t G = (uint32_t)(((int64_t)g.giant[gi] % b->n + b->n) % b->n);
            LincombArgs la;
            memset(&la, 0, sizeof(la));
            for (uint32_t j = 0; j < nb; ++j) {
                la.a0[j] = src[j].c0;
                la.a1[j] = src[j].c1;
                la.pt[0][j] = g.pt + (size_t)(i0 + j) * limb;
            }
            const Ct &target = (G == 0 && first) ? acc : P;
            la.out0[0] = target.c0;
            la.out1[0] = target.c1;
            la.primes = ctx()->d_primes;
            la.n = nb;
            la.nout = 1;
            la.logn = ctx()->logn;
            TRY(dev(launch_lincomb(la, lvl + 1, R_.st), "ckks_bootstrap lincomb"));
            Ct part = P;
            if (G != 0) {
                part = first ? acc : R;
                ckks_ct I = as_ct(P), O = as_ct(part);
                TRY(ckks_hrotate(ctx(), &I, (int32_t)G, b->rot.at(G), &O, L_.ws, R_.st));
            }
            if (!first) TRY(R_.add(acc, part, acc));
        }
        const Ct acc = b->slot(acc_slot, lvl);
        for (uint32_t l = 1; l < nl; ++l) {
            TRY(join(l));
            TRY(add(acc, b->slot(b->lanes[l].acc, lvl), acc));
        }
        Ct c = acc;
        for (uint32_t r = 0; r < g.rescales; ++r) TRY(rescale(c, (r + 1 == g.rescales) ? final_out : nullptr));
        out = c;
        return CKKS_OK;
    }

    // buffers of the Chebyshev evaluation
    std::vector<uint32_t> pool;
    std::map<uint32_t, Ct> T;

    ckks_status take(uint32_t &s)
    {
        if (pool.empty()) return fail(CKKS_E_UNSUPPORTED, "ckks_bootstrap: Chebyshev buffer pool exhausted");
        s = pool.back();
        pool.pop_back();
        return CKKS_OK;
    }

    ckks_status poly(int ni, Ct &out, uint32_t &slot)
    {
        const ChebNode &nd = b->nodes[ni];
        if (nd.leaf) {
            // sum_k C_k T_k on the limbs 0..t+1, rescaled once, plus c_0
            const uint32_t t = (uint32_t)((int)b->evalmod_in + nd.level), D = (uint32_t)nd.c.size() - 1;
            TRY(take(slot));
            const Ct dst = b->slot(slot, t + 1);
            for (uint32_t k0 = 1; k0 <= D; k0 += kMaxLincomb) {
                ScalarLincombArgs la;
                memset(&la, 0, sizeof(la));
                la.n = std::min<uint32_t>(kMaxLincomb, D - k0 + 1);
                for (uint32_t j = 0; j < la.n; ++j) {
                    la.a0[j] = T.at(k0 + j).c0;
                    la.a1[j] = T.at(k0 + j).c1;
                }
                la.cst = b->leaf_cst + nd.cst + (size_t)(k0 - 1) * (t + 2);
                la.cst_stride = t + 2;
                la.acc0 = k0 > 1 ? dst.c0 : nullptr;
                la.acc1 = k0 > 1 ? dst.c1 : nullptr;
                la.out0 = dst.c0;
                la.out1 = dst.c1;
                la.primes = ctx()->d_primes;
                la.logn = ctx()->logn;
                TRY(dev(launch_scalar_lincomb(la, t + 2, st), "ckks_bootstrap leaf"));
            }
            out = dst;
            TRY(rescale(out));
            return scalar_add(out, nd.c[0]);
        }
        Ct R, P;
        uint32_t sr, sp;
        TRY(poly(nd.r, R, sr));
        const Ct &TG = T.at(nd.G);
        TRY(take(sp));
        if (nd.q < 0) {
            TRY(mult_const_to(TG, nd.q0, TG.level - 1, b->slot(sp, 0), P));
        } else {
            Ct Q;
            uint32_t sq;
            TRY(poly(nd.q, Q, sq));
            TRY(mul(Q, TG, b->slot(sp, 0), P));
            pool.push_back(sq);
        }
        const uint32_t l = std::min(P.level, R.level);
        TRY(level_down(P, l, P, P));
        TRY(level_down(R, l, R, R));
        TRY(add(P, R, P));
        pool.push_back(sr);
        out = P;
        slot = sp;
        return CKKS_OK;
    }

    // EvalMod of the ciphertext in buffer s0 (s1 is its partner); result in s0 or s1
    ckks_status eval_mod(uint32_t s0, uint32_t s1, Ct &out)
    {
        T.clear();
        pool.clear();
        for (uint32_t i = 0; i < b->pool_size(); ++i) pool.push_back(ln->pool + i);
        T[1] = b->slot(s0, b->evalmod_in);
        Ct tmp;
        for (uint32_t k = 2; k <= b->nbaby; ++k) {
            const Ct buf = b->slot(ln->t + (k - 2), 0);
            Ct v;
            if (k % 2 == 0) {
                TRY(mul(T.at(k / 2), T.at(k / 2), buf, v));
                TRY(scalar_mul(v, v, 2));
                TRY(scalar_add(v, -1.0));
            } else {
                TRY(mul(T.at(k / 2), T.at(k / 2 + 1), buf, v));
                TRY(scalar_mul(v, v, 2));
                TRY(level_down(T.at(1), v.level, b->slot(ln->d + 2, 0), tmp));
                TRY(add(v, tmp, v, true));
            }
            T[k] = v;
        }
        for (size_t j = 0; j < b->giants.size(); ++j) {
            const uint32_t G = b->giants[j];
            Ct v;
            TRY(mul(T.at(G / 2), T.at(G / 2), b->slot(ln->g + (uint32_t)j, 0), v));
            TRY(scalar_mul(v, v, 2));
            TRY(scalar_add(v, -1.0));
            T[G] = v;
        }
        Ct acc;
        uint32_t sa;
        TRY(poly((int)b->nodes.size() - 1, acc, sa));
        // double angles y <- 2 y^2 - 1, alternating between s1 and s0 (T_1 is no longer read)
        uint32_t other = s1;
        for (uint32_t r = 0; r < b->double_angles; ++r) {
            Ct y;
            TRY(mul(acc, acc, b->slot(other, 0), y));
            TRY(scalar_mul(y, y, 2));
            TRY(scalar_add(y, -1.0));
            acc = y;
            other = other == s1 ? s0 : s1;
        }
        if (b->double_angles == 0) {  // the result must leave the shared pool
            const Ct dst = b->slot(s1, acc.level);
            const size_t bytes = (size_t)(acc.level + 1) * b->N * 8;
            TRY(dev(hipMemcpyAsync(dst.c0, acc.c0, bytes, hipMemcpyDeviceToDevice, st), "ckks_bootstrap copy"));
            TRY(dev(hipMemcpyAsync(dst.c1, acc.c1, bytes, hipMemcpyDeviceToDevice, st), "ckks_bootstrap copy"));
            acc = dst;
        }
        out = acc;
        return CKKS_OK;
    }

    ckks_status modraise(const ckks_ct &in, const Ct &x)
    {
        const ckks_ctx *c = ctx();
        const size_t N = c->N;
        uint64_t *v = (uint64_t *)ln->ws;
        NttArgs ia = base_args(c, true);
        ia.src = in.c0;
        ia.dst = v;
        ia.map.rows = 1;
        ia.map.prime0 = 0;
        ia.map.src_poly_stride = (int64_t)(in.c1 - in.c0);
        ia.map.dst_poly_stride = (int64_t)N;
        TRY(dev(launch_ntt_inv(ia, 2, PRO_PLAIN, st, v, (int64_t)N), "ckks_bootstrap modraise"));
        NttArgs a = base_args(c, false);
        a.src = v;
        a.dst = x.c0;
        a.map.rows = b->L + 1;
        a.map.prime0 = 0;
        a.map.src_poly_stride = 0;
        a.map.dst_poly_stride = (int64_t)(x.c1 - x.c0);
        a.rs_src[0] = v;
        a.rs_src[1] = v + N;
        a.rs_qlmod = c->d_rs_mod;  // row 0: q_0 mod q_i
        a.rs_ql = c->primes[0];
        return dev(launch_ntt_fwd(a, 2 * (b->L + 1), PRO_RESCALE, EPI_PLAIN, st, x.c0, (int64_t)(x.c1 - x.c0)),
                   "ckks_bootstrap modraise");
    }

    // (c0, c1) -> (c0 + k0, k1), (k0, k1) = KeySwitch(c1, key); the result's c1 lives in tmp
    ckks_status switch_key(const Ct &c, const ckks_key *key, const Ct &tmp, Ct &out)
    {
        TRY(ckks_keyswitch(ctx(), c.c1, c.level, key, tmp.c0, tmp.c1, ln->ws, st));
        TRY(ckks_poly_add(ctx(), c.c0, tmp.c0, c.c0, c.level, st));
        out = Ct{c.c0, tmp.c1, c.level};
        return CKKS_OK;
    }

    // One bootstrap.  On failure every lane that was forked is joined back, so
    // the caller's stream (and a capture on it) is never left with work of
    // another stream that it does not wait for.
    ckks_status run(const ckks_ct &in, const ckks_ct &out)
    {
        b->next_event = 0;
        for (bool &o : b->lane_open) o = false;
        ckks_status s = run_steps(in, out);
        if (s != CKKS_OK) {
            close_lanes();
            return s;
        }
        for (uint32_t l = 1; l < kLanes; ++l)
            if (b->lane_open[l]) return fail(CKKS_E_DEVICE, "ckks_bootstrap: a lane was not joined");
        return CKKS_OK;
    }

    // Joins every open lane into the caller's stream with events outside the
    // run's own set (error path only; later errors are not reported).
    void close_lanes()
    {
        for (uint32_t l = 1; l < kLanes; ++l) {
            if (!b->lane_open[l]) continue;
            if (hipEventRecord(b->close_events[l], b->lanes[l].aux) == hipSuccess)
                (void)hipStreamWaitEvent(st, b->close_events[l], 0);
            b->lane_open[l] = false;
        }
    }

    ckks_status run_steps(const ckks_ct &in0, const ckks_ct &out)
    {
        Ct x = b->slot(b->s_x(), b->L);
        ckks_ct in = in0;
        if (b->gain > 1) {  // G m: the integer gain on the level-0 input, exact
            const Ct g = b->slot(b->s_im(0), 0);
            TRY(scalar_mul(Ct{in.c0, in.c1, 0}, g, (int64_t)b->gain));
            in = ckks_ct{g.c0, g.c1, 0, in0.scale};
        }
        if (b->to_sparse) {  // encapsulation: switch the input to the sparse secret first
            const Ct c = b->slot(b->s_re(0), 0), tmp = b->slot(b->s_cj(), 0);
            const size_t bytes = b->N * 8;
            TRY(dev(hipMemcpyAsync(c.c0, in.c0, bytes, hipMemcpyDeviceToDevice, st), "ckks_bootstrap copy"));
            Ct sp;
            TRY(switch_key(Ct{c.c0, in.c1, 0}, b->to_sparse, tmp, sp));
            TRY(modraise(ckks_ct{sp.c0, sp.c1, 0, 1.0}, x));
            TRY(switch_key(x, b->from_sparse, b->slot(b->s_cj(), b->L), x));
        } else {
            TRY(modraise(in, x));
        }
        uint32_t ai = 0;
        for (const Group &g : b->cts) {
            TRY(linear_transform(g, x, b->s_out(ai), nullptr, x));
            ai ^= 1;
        }
        // split: re = x + conj(x), im = (conj(x) - x) X^(N/2)
        const uint32_t l = x.level;
        const Ct cj = b->slot(b->s_cj(), l), re = b->slot(b->s_re(0), l), im = b->slot(b->s_im(0), l);
        ckks_ct X = as_ct(x), CJ = as_ct(cj);
        TRY(ckks_conjugate(ctx(), &X, b->conj, &CJ, ln->ws, st));
        TRY(add(x, cj, re));
        TRY(add(cj, x, im, true));
        TRY(ckks_poly_mul(ctx(), im.c0, b->mono, im.c0, l, st));
        TRY(ckks_poly_mul(ctx(), im.c1, b->mono, im.c1, l, st));
        // the two halves on lanes 0 and 1
        Ct yr, yi;
        Runner im_r = *this;
        im_r.st = b->lanes[1].aux;
        im_r.ln = &b->lanes[1];
        TRY(fork(2));
        TRY(im_r.eval_mod(b->s_im(0), b->s_im(1), yi));
        TRY(eval_mod(b->s_re(0), b->s_re(1), yr));
        TRY(join(1));
        TRY(ckks_poly_mul(ctx(), yi.c0, b->mono, yi.c0, yi.level, st));
        TRY(ckks_poly_mul(ctx(), yi.c1, b->mono, yi.c1, yi.level, st));
        TRY(add(yr, yi, yi));
        x = yi;
        const Ct fin{out.c0, out.c1, b->out_level};
        for (size_t i = 0; i < b->stc.size(); ++i) {
            TRY(linear_transform(b->stc[i], x, b->s_out(ai), i + 1 == b->stc.size() ? &fin : nullptr, x));
            ai ^= 1;
        }
        return CKKS_OK;
    }
};

// Fork and join events of one run: a transform group whose giant steps go to
// nl > 1 lanes takes one fork and nl - 1 joins; the EvalMod halves take two.
uint32_t events_per_run(const ckks_boot &b)
{
    uint32_t n = 2;
    for (const auto *gs : {&b.cts, &b.stc})
        for (const Group &g : *gs) {
            const uint32_t nl = std::min<uint32_t>(kLanes, g.lay.giants);
            if (nl > 1) n += nl;
        }
    return n;
}

uint32_t keyswitches_of(const ckks_boot &b)
{
    uint32_t ks = 1 + (b.to_sparse ? 2 : 0);  // conjugation, encapsulation
    for (const auto *gs : {&b.cts, &b.stc})
        for (const Group &g : *gs) {
            ks += (uint32_t)g.baby_k.size();
            for (int32_t G : g.giant) ks += (((int64_t)G % b.n + b.n) % b.n) != 0;
        }
    uint32_t products = 0;
    for (const ChebNode &nd : b.nodes) products += !nd.leaf && nd.q >= 0;
    ks += 2 * ((b.nbaby - 1) + (uint32_t)b.giants.size() + products + b.double_angles);  // both halves
    return ks;
}

}  // namespace

// Builds a handle; with size_only, stops once the device bytes are known and
// stores them there (nothing is allocated or uploaded).
static ckks_status boot_create(ckks_ctx *ctx, const ckks_boot_desc *desc, ckks_boot **out, size_t *size_only)
{
    if (!ctx || !desc || !out) return fail(CKKS_E_ARG, "ckks_boot_create: null argument");
    *out = nullptr;
    const uint32_t logn = ctx->logn, N = ctx->N, n = N / 2, L = ctx->nq - 1;
    if (desc->n_cts == 0 || desc->n_stc == 0 || !desc->cts_radix_logs || !desc->stc_radix_logs || !desc->cts_diags ||
        !desc->stc_diags || !desc->cheb || desc->cheb_degree < 1 || !(desc->top_scale > 0))
        return fail(CKKS_E_ARG, "ckks_boot_create: incomplete descriptor");
    if (!desc->relin || desc->relin->galois != 0 || desc->relin->ctx != ctx)
        return fail(CKKS_E_KEY, "ckks_boot_create: missing relinearisation key");
    if (!desc->conj || desc->conj->galois != 2 * N - 1 || desc->conj->ctx != ctx)
        return fail(CKKS_E_KEY, "ckks_boot_create: missing conjugation key");
    if (desc->n_rot && (!desc->rot_steps || !desc->rot_keys))
        return fail(CKKS_E_ARG, "ckks_boot_create: null rotation arrays");

    ckks_boot *b = new ckks_boot();
    b->ctx = ctx;
    b->L = L;
    b->n = n;
    b->N = N;
    b->degree = desc->cheb_degree;
    if (b->degree < 2) {
        delete b;
        return fail(CKKS_E_ARG, "ckks_boot_create: cheb_degree must be at least 2");
    }
    b->double_angles = desc->double_angles;
    b->cheb.assign(desc->cheb, desc->cheb + desc->cheb_degree + 1);
    b->relin = desc->relin;
    b->conj = desc->conj;
    if ((desc->to_sparse == nullptr) != (desc->from_sparse == nullptr) ||
        (desc->to_sparse && (desc->to_sparse->ctx != ctx || desc->from_sparse->ctx != ctx))) {
        delete b;
        return fail(CKKS_E_KEY, "ckks_boot_create: sparse-secret keys must be given together");
    }
    b->to_sparse = desc->to_sparse;
    b->hoist = desc->hoist_moddown != 0;
    b->gain = desc->input_gain > 1 ? desc->input_gain : 1;
    if (b->gain >= ctx->primes[0]) {
        delete b;
        return fail(CKKS_E_ARG, "ckks_boot_create: input_gain must be below q_0");
    }
    b->from_sparse = desc->from_sparse;
    auto bail = [&](ckks_status s, const std::string &m) {
        ckks_boot_destroy(b);
        return fail(s, "ckks_boot_create: " + m);
    };
    for (uint32_t i = 0; i < desc->n_rot; ++i) {
        const ckks_key *k = desc->rot_keys[i];
        const uint32_t r = (uint32_t)(((int64_t)desc->rot_steps[i] % n + n) % n);
        uint64_t g = 1, p = 5;
        for (uint32_t e = r; e; e >>= 1, p = p * p % (2ull * N))
            if (e & 1) g = g * p % (2ull * N);
        if (!k || k->ctx != ctx || k->galois != g) return bail(CKKS_E_KEY, "rotation key " + std::to_string(i) +
                                                                             " does not match its step");
        b->rot[r] = k;
    }

    // level scales and the Chebyshev tree depths (same recurrences as the documented schedule)
    b->sc.assign(L + 1, 0.0);
    b->sc[L] = desc->top_scale;
    for (uint32_t l = L; l >= 1; --l) b->sc[l - 1] = (b->sc[l] * b->sc[l]) / (double)ctx->primes[l];
    // baby-step/giant-step plan: levels of T_k relative to the EvalMod input, then the node tree
    b->baby = desc->cheb_baby;
    if (b->baby == 0) {
        b->baby = 2;
        while (b->baby * b->baby <= b->degree) b->baby *= 2;
    }
    if (b->baby < 2 || (b->baby & (b->baby - 1))) return bail(CKKS_E_ARG, "cheb_baby must be a power of two >= 2");
    b->nbaby = std::min(b->baby, b->degree);
    b->lvT[1] = 0;
    for (uint32_t k = 2; k <= b->nbaby; ++k)
        b->lvT[k] = k % 2 == 0 ? b->lvT[k / 2] - 1 : std::min(b->lvT[k / 2], b->lvT[k / 2 + 1]) - 1;
    for (uint32_t G = b->baby; 2 * G <= b->degree; G *= 2) {
        b->giants.push_back(2 * G);
        b->lvT[2 * G] = b->lvT[G] - 1;
    }
    b->t_leaf = 0;
    for (uint32_t k = 1; k <= std::min(b->baby - 1, b->degree); ++k) b->t_leaf = std::min(b->t_leaf, b->lvT[k]);
    b->t_leaf -= 1;
    std::function<int(const std::vector<double> &)> build = [&](const std::vector<double> &c) -> int {
        const uint32_t D = (uint32_t)c.size() - 1;
        ChebNode nd;
        if (D < b->baby) {
            nd.leaf = true;
            nd.c = c;
            nd.level = b->t_leaf;
        } else {
            uint32_t G = b->baby;
            while (2 * G <= D) G *= 2;
            std::vector<double> q, r;
            cheb_split(c, G, q, r);
            nd.G = G;
            nd.r = build(r);
            nd.q0 = q[0];
            if (q.size() > 1) nd.q = build(q);
            const int p = nd.q < 0 ? b->lvT[G] - 1 : std::min(b->nodes[nd.q].level, b->lvT[G]) - 1;
            nd.level = std::min(p, b->nodes[nd.r].level);
        }
        b->nodes.push_back(nd);
        return (int)b->nodes.size() - 1;
    };
    build(b->cheb);
    const uint32_t depth = (uint32_t)(-b->nodes.back().level);

    // groups and levels
    uint32_t sum_c = 0, sum_s = 0;
    for (uint32_t i = 0; i < desc->n_cts; ++i) sum_c += desc->cts_radix_logs[i];
    for (uint32_t i = 0; i < desc->n_stc; ++i) sum_s += desc->stc_radix_logs[i];
    if (sum_c != logn - 1 || sum_s != logn - 1) return bail(CKKS_E_ARG, "radix logs must cover log2(N/2) stages");
    int64_t lvl = L;
    auto make_group = [&](uint32_t r, uint32_t h0, uint32_t rescales) {
        Group g;
        g.lay = group_layout(n, r, h0);
        g.level = (uint32_t)std::max<int64_t>(lvl, 0);
        g.rescales = rescales;
        for (uint32_t gi = 0; gi < g.lay.giants; ++gi) g.giant.push_back(((int32_t)(gi * g.lay.baby) + g.lay.m_lo) * (int32_t)h0);
        for (uint32_t k = 1; k < std::min(g.lay.baby, g.lay.count); ++k) g.baby_k.push_back((int32_t)(k * h0));
        lvl -= rescales;
        return g;
    };
    uint32_t stage = 0;
    for (uint32_t i = 0; i < desc->n_cts; ++i) {
        const uint32_t r = desc->cts_radix_logs[i];
        b->cts.push_back(make_group(r, n >> (stage + r), i == 0 ? 2 : 1));
        stage += r;
    }
    b->evalmod_in = (uint32_t)std::max<int64_t>(lvl, 0);
    lvl -= depth + b->double_angles;
    if ((int64_t)b->evalmod_in + b->t_leaf < 0 || lvl < 0)
        return bail(CKKS_E_UNSUPPORTED, "the schedule needs more levels than the context has");
    stage = 0;
    for (uint32_t i = 0; i < desc->n_stc; ++i) {
        const uint32_t r = desc->stc_radix_logs[i];
        b->stc.push_back(make_group(r, 1u << stage, 1));
        stage += r;
    }
    if (lvl < 0) return bail(CKKS_E_UNSUPPORTED, "the schedule needs more levels than the context has");
    b->out_level = (uint32_t)lvl;
    for (const auto *gs : {&b->cts, &b->stc})
        for (const Group &g : *gs) {
            if (g.lay.baby > kMaxLincomb) return bail(CKKS_E_UNSUPPORTED, "more than 16 baby steps in a group");
            b->max_baby = std::max(b->max_baby, g.lay.baby);
            for (int32_t k : g.baby_k)
                if (!b->rot.count((uint32_t)k % n)) return bail(CKKS_E_KEY, "no key for rotation " + std::to_string(k));
            for (int32_t G : g.giant) {
                const uint32_t r = (uint32_t)(((int64_t)G % n + n) % n);
                if (r && !b->rot.count(r)) return bail(CKKS_E_KEY, "no key for rotation " + std::to_string(r));
            }
        }
    b->keyswitches = keyswitches_of(*b);

    // one device allocation: plaintexts, X^(N/2), buffers, workspace
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t pt_words = 0;
    for (const auto *gs : {&b->cts, &b->stc})
        for (const Group &g : *gs) pt_words += (size_t)g.lay.count * (g.level + 1) * N;
    b->slot_words = 2 * (size_t)(L + 1) * N;
    b->nslots = b->slot_count();
    size_t wsb = 0;
    for (uint32_t op : {CKKS_OP_HMULT, CKKS_OP_ROTATE, CKKS_OP_HOISTED, CKKS_OP_RESCALE})
        wsb = std::max(wsb, ckks_workspace_bytes(ctx, op, L));
    wsb = std::max(wsb, 2 * (size_t)N * 8);
    // leaf constants: for each leaf, C_k = round(c_k (D_t q_(t+1)) / D_level(T_k)) mod q_0..q_(t+1)
    std::vector<uint64_t> cst;
    {
        const uint32_t t = (uint32_t)((int)b->evalmod_in + b->t_leaf);
        for (ChebNode &nd : b->nodes) {
            if (!nd.leaf) continue;
            nd.cst = cst.size();
            for (uint32_t k = 1; k < nd.c.size(); ++k) {
                const double X = (b->sc[t] * (double)ctx->primes[t + 1]) / b->sc[b->evalmod_in + b->lvT[k]];
                const int64_t C = (int64_t)round_half_away(nd.c[k] * X);
                for (uint32_t i = 0; i <= t + 1; ++i) {
                    const int64_t qi = (int64_t)ctx->primes[i];
                    const int64_t m = C % qi;
                    cst.push_back((uint64_t)(m < 0 ? m + qi : m));
                }
            }
        }
    }
    const size_t off_cst = up(pt_words * 8);
    const size_t off_mono = off_cst + up(std::max<size_t>(cst.size(), 1) * 8),
                 off_slots = off_mono + up((size_t)(L + 1) * N * 8);
    // the lanes' workspaces double as the staging buffer of the plaintext upload below
    size_t max_count = 0;
    for (const auto *gs : {&b->cts, &b->stc})
        for (const Group &g : *gs) max_count = std::max(max_count, (size_t)g.lay.count);
    wsb = std::max(wsb, (max_count * N * sizeof(double) + kLanes - 1) / kLanes);
    const size_t off_ws = off_slots + up(b->nslots * b->slot_words * 8);
    b->qp_words = b->hoist ? 2 * (size_t)(L + 1 + ctx->np) * N : 0;
    const size_t off_qp = off_ws + kLanes * up(wsb);
    b->ws_bytes = up(wsb);
    b->bytes = off_qp + kLanes * b->qp_words * 8;
    if (size_only) {
        *size_only = b->bytes;
        ckks_boot_destroy(b);
        return CKKS_OK;
    }
    if (desc->device_buffer) {
        if (((uintptr_t)desc->device_buffer & 255) || desc->device_buffer_bytes < b->bytes)
            return bail(CKKS_E_ARG, "device_buffer must be 256-byte aligned and hold " + std::to_string(b->bytes) +
                                        " bytes (ckks_boot_bytes)");
        b->dev = desc->device_buffer;
    } else {
        if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc(&b->dev, b->bytes) != hipSuccess) {
            b->dev = nullptr;
            return bail(CKKS_E_NOMEM, "device allocation of " + std::to_string(b->bytes) + " bytes failed");
        }
        b->owns_dev = true;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return bail(CKKS_E_DEVICE, "hipSetDevice failed");
    uint8_t *base = (uint8_t *)b->dev;
    b->mono = (uint64_t *)(base + off_mono);
    b->leaf_cst = (uint64_t *)(base + off_cst);
    b->slots = (uint64_t *)(base + off_slots);
    b->assign_lanes(base + off_ws);
    b->qp = b->hoist ? (uint64_t *)(base + off_qp) : nullptr;
    for (uint32_t l = 1; l < kLanes; ++l)
        if (hipStreamCreateWithFlags(&b->lanes[l].aux, hipStreamNonBlocking) != hipSuccess) {
            b->lanes[l].aux = nullptr;
            return bail(CKKS_E_DEVICE, "stream creation failed");
        }
    b->events.assign(events_per_run(*b), nullptr);
    for (hipEvent_t &ev : b->events)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            return bail(CKKS_E_DEVICE, "event creation failed");
        }
    for (hipEvent_t &ev : b->close_events)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            return bail(CKKS_E_DEVICE, "event creation failed");
        }

    // plaintexts: integer-valued doubles -> residues -> evaluation domain, staged in the
    // lanes' workspaces (unused until the first run)
    double *stage_buf = (double *)(base + off_ws);
    uint64_t *pt = (uint64_t *)base;
    hipError_t e = hipSuccess;
    std::vector<double> host;
    for (int side = 0; side < 2 && e == hipSuccess; ++side) {
        std::vector<Group> &gs = side == 0 ? b->cts : b->stc;
        const double *const *diags = side == 0 ? desc->cts_diags : desc->stc_diags;
        for (size_t i = 0; i < gs.size() && e == hipSuccess; ++i) {
            Group &g = gs[i];
            if (!diags[i]) {
                e = hipErrorInvalidValue;
                break;
            }
            const size_t words = (size_t)g.lay.count * N;
            host.assign(diags[i], diags[i] + words);
            for (double v : host)
                if (!(v == floor(v)) || fabs(v) > 1e300)
                    return bail(CKKS_E_ARG, "plaintext coefficients must be finite integers");
            g.pt = pt;
            e = hipMemcpy(stage_buf, host.data(), words * sizeof(double), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = launch_reduce_f64(stage_buf, g.pt, ctx->d_primes, g.lay.count, g.level + 1, logn, 0);
            if (e == hipSuccess) {
                NttArgs a = base_args(ctx, false);
                a.src = g.pt;
                a.dst = g.pt;
                a.map.rows = g.level + 1;
                a.map.prime0 = 0;
                a.map.src_poly_stride = a.map.dst_poly_stride = (int64_t)(g.level + 1) * N;
                e = launch_ntt_fwd(a, g.lay.count * (g.level + 1), PRO_PLAIN, EPI_PLAIN, 0, g.pt,
                                   (int64_t)(g.level + 1) * N);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(0);  // the staging buffer is reused
            pt += (size_t)g.lay.count * (g.level + 1) * N;
        }
    }
    if (e == hipSuccess && !cst.empty())
        e = hipMemcpy(b->leaf_cst, cst.data(), cst.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_half_monomial(b->mono, L + 1, logn, 0);
    if (e == hipSuccess) {
        NttArgs a = base_args(ctx, false);
        a.src = a.dst = b->mono;
        a.map.rows = L + 1;
        a.map.prime0 = 0;
        a.map.src_poly_stride = a.map.dst_poly_stride = 0;
        e = launch_ntt_fwd(a, L + 1, PRO_PLAIN, EPI_PLAIN, 0, b->mono, 0);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(0);
    if (e != hipSuccess) return bail(CKKS_E_DEVICE, std::string("plaintext upload: ") + hipGetErrorString(e));
    *out = b;
    return CKKS_OK;
}

extern "C" ckks_status ckks_boot_create(ckks_ctx *ctx, const ckks_boot_desc *desc, ckks_boot **out)
{
    return boot_create(ctx, desc, out, nullptr);
}

extern "C" ckks_status ckks_boot_bytes(ckks_ctx *ctx, const ckks_boot_desc *desc, size_t *bytes)
{
    if (!bytes) return fail(CKKS_E_ARG, "ckks_boot_bytes: null output");
    *bytes = 0;
    ckks_boot *unused = nullptr;
    return boot_create(ctx, desc, &unused, bytes);
}

extern "C" uint32_t ckks_boot_output_level(const ckks_boot *b) { return b ? b->out_level : 0; }
extern "C" uint32_t ckks_boot_keyswitches(const ckks_boot *b) { return b ? b->keyswitches : 0; }
extern "C" size_t ckks_boot_device_bytes(const ckks_boot *b) { return b ? b->bytes : 0; }

static ckks_status check_io(const ckks_boot *b, const ckks_ct *in, const ckks_ct *out, const char *what)
{
    if (!b || !in || !out) return fail(CKKS_E_ARG, std::string(what) + ": null argument");
    if (in->level != 0) return fail(CKKS_E_LEVEL, std::string(what) + ": the input must be at level 0");
    const void *p[4] = {in->c0, in->c1, out->c0, out->c1};
    for (const void *x : p)
        if (!x || ((uintptr_t)x & 7)) return fail(CKKS_E_ARG, std::string(what) + ": null or misaligned polynomial");
    const size_t N = b->N, ob = (size_t)(b->out_level + 1) * N * 8, ib = N * 8;
    auto ov = [](const void *a, size_t an, const void *c, size_t cn) {
        return (uintptr_t)a < (uintptr_t)c + cn && (uintptr_t)c < (uintptr_t)a + an;
    };
    if (ov(out->c0, ob, out->c1, ob) || ov(out->c0, ob, in->c0, ib) || ov(out->c0, ob, in->c1, ib) ||
        ov(out->c1, ob, in->c0, ib) || ov(out->c1, ob, in->c1, ib))
        return fail(CKKS_E_ARG, std::string(what) + ": output overlaps the input or itself");
    for (const void *x : p)
        if (ov(x, 8, b->dev, b->bytes)) return fail(CKKS_E_ARG, std::string(what) + ": operand inside the handle's buffers");
    return CKKS_OK;
}

extern "C" ckks_status ckks_bootstrap(ckks_boot *b, const ckks_ct *in, ckks_ct *out, void *stream)
{
    TRY(check_io(b, in, out, "ckks_bootstrap"));
    Runner r{b, S(stream), &b->lanes[0], {}};
    TRY(r.run(*in, *out));
    out->level = b->out_level;
    out->scale = b->sc[b->out_level];
    return CKKS_OK;
}

extern "C" ckks_status ckks_boot_capture(ckks_boot *b, const ckks_ct *in, ckks_ct *out, void *stream)
{
    TRY(check_io(b, in, out, "ckks_boot_capture"));
    hipStream_t st = S(stream);
    if (!st) return fail(CKKS_E_ARG, "ckks_boot_capture: the default stream cannot be captured");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return fail(CKKS_E_DEVICE, std::string("ckks_boot_capture: begin capture: ") + hipGetErrorString(e));
    Runner r{b, st, &b->lanes[0], {}};
    const ckks_status s = r.run(*in, *out);  // every forked lane is joined, also on failure
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (s != CKKS_OK || e != hipSuccess) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        if (s != CKKS_OK) return s;
        return fail(CKKS_E_DEVICE, std::string("ckks_boot_capture: end capture: ") + hipGetErrorString(e));
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->exec = nullptr;
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        return fail(CKKS_E_DEVICE, std::string("ckks_boot_capture: instantiate: ") + hipGetErrorString(e));
    }
    out->level = b->out_level;
    out->scale = b->sc[b->out_level];
    return CKKS_OK;
}

extern "C" ckks_status ckks_boot_replay(ckks_boot *b, void *stream)
{
    if (!b || !b->exec) return fail(CKKS_E_ARG, "ckks_boot_replay: nothing captured");
    hipError_t e = hipGraphLaunch(b->exec, S(stream));
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_boot_replay: ") + hipGetErrorString(e));
    return CKKS_OK;
}

extern "C" void ckks_boot_destroy(ckks_boot *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t ev : b->events)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : b->close_events)
        if (ev) (void)hipEventDestroy(ev);
    for (uint32_t l = 1; l < kLanes; ++l)
        if (b->lanes[l].aux) (void)hipStreamDestroy(b->lanes[l].aux);
    if (b->dev && b->owns_dev) (void)hipFree(b->dev);
    delete b;
}
