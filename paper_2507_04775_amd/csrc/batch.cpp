// Batched key switching (the paper's limb batching, Sec. III-F.1, done the
// MI355X way): every step of every work item of a batch (HMult+relin, key
// switch, rotation, hoisted rotations; any mix of levels) becomes a list of
// (instance, limb) records, and each step runs as ONE launch of a persistent
// kernel whose workgroups claim (record, tile) units from an atomic counter.
// The host builds all argument blocks and records once (ckks_batch_create);
// a run is a zeroing kernel plus one launch per step on one stream, which can
// be captured into a hipGraph and replayed.  The autotuner times each step's
// persistent grid size and keeps the fastest.
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ks_args.h"

namespace ckks {
ckks_status fail(ckks_status s, const std::string &msg);
}

using namespace ckks;

#define TRY(x)                              \
    do {                                    \
        ckks_status _s = (x);               \
        if (_s != CKKS_OK) return _s;       \
    } while (0)

namespace {

enum QKind { Q_NTT = 0, Q_BCONV, Q_IP, Q_TENSOR };

struct QueueSpec {
    QKind kind;
    NttStage stage;
    uint32_t pass;
    int set;  // instance array (NTT sets 0..3)
    std::vector<UnitRec> recs;
    uint32_t tiles;
    UnitRec *recs_dev;
    uint32_t grid_mult;
};

hipStream_t S(void *s) { return (hipStream_t)s; }

uint32_t galois_of(const ckks_ctx *c, int32_t k)
{
    const uint64_t two_n = 2ull * c->N, half = c->N / 2;
    int64_t kk = k % (int64_t)half;
    if (kk < 0) kk += half;
    uint64_t g = 1, b = 5;
    for (uint64_t e = (uint64_t)kk; e; e >>= 1, b = b * b % two_n)
        if (e & 1) g = g * b % two_n;
    return (uint32_t)g;
}

size_t item_ws_elems(const ckks_ctx *c, const ckks_work &w)
{
    const uint32_t level = w.a.level;
    KsSizes s = ks_sizes(c, level);
    switch (w.kind) {
    case CKKS_WORK_HMULT_RELIN: return ks_ws_elems(c, level) + (size_t)s.n * s.N;
    case CKKS_WORK_KEYSWITCH:
    case CKKS_WORK_ROTATE: return ks_ws_elems(c, level);
    case CKKS_WORK_HOISTED:
        return ((size_t)s.n + (size_t)s.beta * s.rows +
                (size_t)w.n_rot * (2 * (size_t)s.rows + 2 * (size_t)c->np + 2 * (size_t)s.n)) *
               s.N;
    default: return 0;
    }
}

bool ptr_ok(const void *p) { return p && ((uintptr_t)p & 7) == 0; }

ckks_status check_ct(const ckks_ctx *c, const ckks_ct &ct, const char *what)
{
    if (!ptr_ok(ct.c0) || !ptr_ok(ct.c1)) return fail(CKKS_E_ARG, std::string(what) + ": null or misaligned pointer");
    if (ct.level >= c->nq) return fail(CKKS_E_LEVEL, std::string(what) + ": level out of range");
    return CKKS_OK;
}

}  // namespace

struct ckks_batch {
    ckks_ctx *ctx = nullptr;
    std::vector<NttArgs> ntt[4];  // ModUp INTT, ModUp NTT, ModDown INTT, ModDown NTT
    std::vector<BconvArgs> bconv;
    std::vector<IpArgs> ip;
    std::vector<TensorArgs> tensor;
    QueueSpec q[QI_COUNT];
    char *dev = nullptr;
    const NttArgs *ntt_dev[4] = {};
    const BconvArgs *bconv_dev = nullptr;
    const IpArgs *ip_dev = nullptr;
    const TensorArgs *tensor_dev = nullptr;
    uint32_t *counters = nullptr;
    uint32_t bconv_tiles = 0;
    uint32_t keyswitches = 0;
    int cus = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // One-launch schedule: every step of every key switch is a group of units that waits for
    // the group before it (kNoGroup: none).  `window` > 0 selects that schedule.
    struct Group {
        uint32_t step, inst, wait, item, tiles;
        std::vector<uint32_t> limbs;
    };
    std::vector<Group> groups;
    uint32_t cur_item = 0;
    uint32_t window = 0;
    uint32_t fused_mult = 2;
    char *fdev = nullptr;
    FusedArgs fused = {};
};

namespace {

void add_recs(ckks_batch *b, int qi, uint32_t inst, uint32_t n)
{
    for (uint32_t l = 0; l < n; ++l) b->q[qi].recs.push_back(UnitRec{inst, l});
}

// A group of the one-launch schedule: records (limbs) of instance inst of step qi, each of
// `tiles` units, waiting for group `wait`.  Returns its index.
uint32_t add_group(ckks_batch *b, int qi, uint32_t inst, uint32_t wait, uint32_t tiles, std::vector<uint32_t> limbs)
{
    b->groups.push_back(ckks_batch::Group{(uint32_t)qi, inst, wait, b->cur_item, tiles, std::move(limbs)});
    return (uint32_t)b->groups.size() - 1;
}

std::vector<uint32_t> iota(uint32_t n)
{
    std::vector<uint32_t> v(n);
    for (uint32_t i = 0; i < n; ++i) v[i] = i;
    return v;
}

// ModDown of npoly accumulators (two INTT passes and two NTT passes at N = 2^16)
void plan_moddown(ckks_batch *b, const uint64_t *acc, int64_t stride, uint32_t level, uint64_t *const *out,
                  const uint64_t *const *add, uint32_t g, uint64_t *pc, uint64_t *conv, uint32_t wait)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    const uint32_t nt = ntt_tiles(c->logn);
    uint32_t di = (uint32_t)b->ntt[2].size();
    b->ntt[2].push_back(args_moddown_intt(c, acc, stride, level, pc));
    add_recs(b, QI_DN_INTT0, di, 2 * c->np);
    add_recs(b, QI_DN_INTT1, di, 2 * c->np);
    uint32_t mi = (uint32_t)b->ntt[3].size();
    b->ntt[3].push_back(args_moddown_ntt(c, acc, stride, 2, level, out, add, g, pc, conv));
    add_recs(b, QI_DN_NTT0, mi, 2 * s.n);
    add_recs(b, QI_DN_NTT1, mi, 2 * s.n);
    wait = add_group(b, QI_DN_INTT0, di, wait, nt, iota(2 * c->np));
    wait = add_group(b, QI_DN_INTT1, di, wait, nt, iota(2 * c->np));
    wait = add_group(b, QI_DN_NTT0, mi, wait, nt, iota(2 * s.n));
    add_group(b, QI_DN_NTT1, mi, wait, nt, iota(2 * s.n));
}

// ModUp of d (gathered through g) into ext; returns nothing, records the steps
// ModUp of d (gathered through g) into ext, after group `wait`; returns the group of its last step
uint32_t plan_modup(ckks_batch *b, const uint64_t *d, uint32_t g, uint32_t level, uint64_t *dc, uint64_t *ext,
                    uint32_t wait)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    const uint32_t nt = ntt_tiles(c->logn);
    uint32_t ui = (uint32_t)b->ntt[0].size();
    b->ntt[0].push_back(args_modup_intt(c, d, g, level, dc));
    const int q0 = g == 1 ? QI_UP_INTT0_PLAIN : QI_UP_INTT0_GALOIS;
    add_recs(b, q0, ui, s.n);
    add_recs(b, QI_UP_INTT1, ui, s.n);
    uint32_t bi = (uint32_t)b->bconv.size();
    b->bconv.push_back(args_modup_bconv(c, d, g, level, dc, ext, false));
    add_recs(b, QI_UP_BCONV, bi, s.beta);
    uint32_t ni = (uint32_t)b->ntt[1].size();
    NttArgs na = args_modup_ntt(c, level, ext);
    b->ntt[1].push_back(na);
    std::vector<uint32_t> conv_rows;
    for (uint32_t l = 0; l < s.beta * s.rows; ++l) {
        const uint32_t poly = l / na.map.rows, row = l - poly * na.map.rows;
        if (limb_skipped(na.map, poly, row)) continue;  // the digit's own rows are read from d
        b->q[QI_UP_NTT0].recs.push_back(UnitRec{ni, l});
        b->q[QI_UP_NTT1].recs.push_back(UnitRec{ni, l});
        conv_rows.push_back(l);
    }
    const uint32_t row_groups = (s.rows + kBconvRowGroup - 1) / kBconvRowGroup;
    wait = add_group(b, q0, ui, wait, nt, iota(s.n));
    wait = add_group(b, QI_UP_INTT1, ui, wait, nt, iota(s.n));
    wait = add_group(b, QI_UP_BCONV, bi, wait, (c->N / (256 * kQueueBlocks)) * row_groups, iota(s.beta));
    wait = add_group(b, QI_UP_NTT0, ni, wait, nt, conv_rows);
    return add_group(b, QI_UP_NTT1, ni, wait, nt, conv_rows);
}

void plan_keyswitch(ckks_batch *b, const uint64_t *d, uint32_t g_in, uint32_t level, const uint64_t *key,
                    uint64_t *out0, uint64_t *out1, const uint64_t *add0, const uint64_t *add1, uint32_t g_add,
                    uint64_t *ws, uint32_t wait)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    KsWs w = ks_ws(c, level, ws);
    wait = plan_modup(b, d, g_in, level, w.dc, w.ext, wait);
    uint32_t ii = (uint32_t)b->ip.size();
    b->ip.push_back(args_ip(c, w.ext, level, key, 1, w.acc, d, g_in));
    add_recs(b, QI_IP, ii, s.rows);
    wait = add_group(b, QI_IP, ii, wait, c->N / (256 * kQueueBlocks), iota(s.rows));
    uint64_t *outs[2] = {out0, out1};
    const uint64_t *adds[2] = {add0, add1};
    plan_moddown(b, w.acc, (int64_t)s.rows * s.N, level, outs, adds, g_add, w.pc, w.conv, wait);
    b->keyswitches += 1;
}

ckks_status plan_item(ckks_batch *b, const ckks_work &w, uint64_t *ws)
{
    const ckks_ctx *c = b->ctx;
    const uint32_t level = w.a.level;
    KsSizes s = ks_sizes(c, level);
    switch (w.kind) {
    case CKKS_WORK_HMULT_RELIN: {
        uint64_t *d2 = ws;
        uint32_t ti = (uint32_t)b->tensor.size();
        b->tensor.push_back(TensorArgs{w.a.c0, w.a.c1, w.b.c0, w.b.c1, w.out->c0, w.out->c1, d2, c->d_primes, c->logn, 0});
        add_recs(b, QI_TENSOR, ti, s.n);
        const uint32_t tg = add_group(b, QI_TENSOR, ti, kNoGroup, c->N / (256 * kQueueBlocks), iota(s.n));
        plan_keyswitch(b, d2, 1, level, w.key->data, w.out->c0, w.out->c1, w.out->c0, w.out->c1, 1,
                       d2 + (size_t)s.n * s.N, tg);
        return CKKS_OK;
    }
    case CKKS_WORK_KEYSWITCH:
        plan_keyswitch(b, w.a.c0, 1, level, w.key->data, w.out->c0, w.out->c1, nullptr, nullptr, 1, ws, kNoGroup);
        return CKKS_OK;
    case CKKS_WORK_ROTATE:
        plan_keyswitch(b, w.a.c1, w.galois, level, w.key->data, w.out->c0, w.out->c1, w.a.c0, nullptr, w.galois, ws,
                       kNoGroup);
        return CKKS_OK;
    case CKKS_WORK_HOISTED: {
        uint64_t *dc = ws, *ext = dc + (size_t)s.n * s.N, *per = ext + (size_t)s.beta * s.rows * s.N;
        const uint32_t up = plan_modup(b, w.a.c1, 1, level, dc, ext, kNoGroup);
        const size_t per_rot = (2 * (size_t)s.rows + 2 * (size_t)c->np + 2 * (size_t)s.n) * s.N;
        for (uint32_t r = 0; r < w.n_rot; ++r) {
            const uint32_t g = galois_of(c, w.rot[r]);
            uint64_t *acc = per + r * per_rot, *pc = acc + 2 * (size_t)s.rows * s.N, *conv = pc + 2 * (size_t)c->np * s.N;
            uint32_t ii = (uint32_t)b->ip.size();
            b->ip.push_back(args_ip(c, ext, level, w.rot_keys[r]->data, g, acc, w.a.c1, g));
            add_recs(b, QI_IP, ii, s.rows);
            const uint32_t ig = add_group(b, QI_IP, ii, up, c->N / (256 * kQueueBlocks), iota(s.rows));
            uint64_t *outs[2] = {w.out[r].c0, w.out[r].c1};
            const uint64_t *adds[2] = {w.a.c0, nullptr};
            plan_moddown(b, acc, (int64_t)s.rows * s.N, level, outs, adds, g, pc, conv, ig);
            b->keyswitches += 1;
        }
        return CKKS_OK;
    }
    default: return fail(CKKS_E_ARG, "ckks_batch_create: unknown work kind");
    }
}

ckks_status validate_item(const ckks_ctx *c, const ckks_work &w, uint32_t idx)
{
    const std::string what = "ckks_batch_create item " + std::to_string(idx);
    ckks_status st;
    if (w.kind == CKKS_WORK_KEYSWITCH) {
        if (!ptr_ok(w.a.c0)) return fail(CKKS_E_ARG, what + ": null input");
        if (w.a.level >= c->nq) return fail(CKKS_E_LEVEL, what + ": level out of range");
    } else if ((st = check_ct(c, w.a, what.c_str())) != CKKS_OK) {
        return st;
    }
    if (!w.out) return fail(CKKS_E_ARG, what + ": null output");
    auto key_ok = [&](const ckks_key *k) { return k && k->data && k->ctx == c; };
    switch (w.kind) {
    case CKKS_WORK_HMULT_RELIN:
        if ((st = check_ct(c, w.b, what.c_str())) != CKKS_OK) return st;
        if (w.b.level != w.a.level) return fail(CKKS_E_LEVEL, what + ": operands at different levels");
        if (!key_ok(w.key) || w.key->galois != 0) return fail(CKKS_E_KEY, what + ": needs a relinearisation key");
        if (!ptr_ok(w.out->c0) || !ptr_ok(w.out->c1)) return fail(CKKS_E_ARG, what + ": bad output");
        return CKKS_OK;
    case CKKS_WORK_KEYSWITCH:
        if (!key_ok(w.key)) return fail(CKKS_E_KEY, what + ": null key");
        if (!ptr_ok(w.out->c0) || !ptr_ok(w.out->c1)) return fail(CKKS_E_ARG, what + ": bad output");
        return CKKS_OK;
    case CKKS_WORK_ROTATE:
        if (w.galois % 2 == 0 || w.galois <= 1 || w.galois >= 2 * c->N)
            return fail(CKKS_E_ARG, what + ": galois must be odd in (1, 2N)");
        if (!key_ok(w.key) || w.key->galois != w.galois) return fail(CKKS_E_KEY, what + ": key for another element");
        if (!ptr_ok(w.out->c0) || !ptr_ok(w.out->c1)) return fail(CKKS_E_ARG, what + ": bad output");
        return CKKS_OK;
    case CKKS_WORK_HOISTED:
        if (w.n_rot == 0 || !w.rot || !w.rot_keys) return fail(CKKS_E_ARG, what + ": no rotations");
        for (uint32_t r = 0; r < w.n_rot; ++r) {
            const uint32_t g = galois_of(c, w.rot[r]);
            if (g == 1) return fail(CKKS_E_ARG, what + ": rotation by a multiple of N/2");
            if (!key_ok(w.rot_keys[r]) || w.rot_keys[r]->galois != g)
                return fail(CKKS_E_KEY, what + ": rotation key " + std::to_string(r) + " for another element");
            if (!ptr_ok(w.out[r].c0) || !ptr_ok(w.out[r].c1)) return fail(CKKS_E_ARG, what + ": bad output");
        }
        return CKKS_OK;
    default: return fail(CKKS_E_ARG, what + ": unknown work kind");
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

hipError_t launch_queue(ckks_batch *b, int qi, uint32_t mult, hipStream_t st)
{
    QueueSpec &Q = b->q[qi];
    if (Q.recs.empty()) return hipSuccess;
    WorkQueue wq;
    wq.recs = Q.recs_dev;
    wq.nrecs = (uint32_t)Q.recs.size();
    wq.tiles = Q.tiles;
    wq.counter = b->counters + qi;
    const uint64_t units = (uint64_t)wq.nrecs * wq.tiles;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(units, (uint64_t)mult * b->cus);
    switch (Q.kind) {
    case Q_NTT: return launch_ntt_stage_queue(Q.stage, b->ctx->logn, Q.pass, b->ntt_dev[Q.set], wq, grid, st);
    case Q_BCONV: return launch_bconv_queue(b->bconv_dev, wq, grid, st);
    case Q_IP: return launch_inner_product_queue(b->ip_dev, wq, grid, st);
    case Q_TENSOR: return launch_tensor_queue(b->tensor_dev, wq, grid, st);
    }
    return hipErrorInvalidValue;
}

uint32_t fused_counter_words(const ckks_batch *b);
size_t fused_units(const ckks_batch *b);
size_t fused_region_bytes(const ckks_batch *b);

hipError_t run(ckks_batch *b, hipStream_t st)
{
    if (b->window) {  // one launch: the claim counter, the fault flag and the group counters start at zero
        hipError_t e = launch_zero_u32(b->fused.claim, fused_counter_words(b), st);
        const uint32_t grid = (uint32_t)std::min<uint64_t>(b->fused.nunits, (uint64_t)b->fused_mult * b->cus);
        return e == hipSuccess ? launch_fused_batch(b->fused, grid, st) : e;
    }
    hipError_t e = launch_zero_u32(b->counters, QI_COUNT, st);
    for (int qi = 0; qi < QI_COUNT && e == hipSuccess; ++qi) e = launch_queue(b, qi, b->q[qi].grid_mult, st);
    return e;
}

// Counters of the one-launch schedule: the claim counter and the fault flag in
// the first 128-byte line, then one line per group's done counter, so that
// the atomics and polls of different groups never share a line.
constexpr uint32_t kDoneStride = 32;
uint32_t fused_counter_words(const ckks_batch *b) { return kDoneStride * (1 + (uint32_t)b->groups.size()); }

// Finished units a workgroup records before it publishes them with one release
// (fewer releases, later signals; measured on the 128-item batch).
constexpr uint32_t kPublishEvery = 32;

// Polls a waiting workgroup makes before it gives up (and raises the fault flag): far beyond
// any real wait (each poll sleeps and reads a counter), but finite, so a launch always ends.
constexpr uint32_t kFusedSpinLimit = 1u << 22;

// The unit list of the one-launch schedule.  Groups are ordered by
// (item / window + step), then by step, latest first, then by item: the items
// form windows of `window` consecutive items, and window w runs step s in
// slot w + s, so consecutive windows overlap step by step (a software
// pipeline over the batch), and a group always comes after the group it
// waits for (an earlier step of the same item, hence an earlier slot).  With
// window >= the number of items it is the step-by-step order of the
// per-step launches, without their barriers.
ckks_status build_fused(ckks_batch *b, uint32_t window)
{
    const uint32_t ng = (uint32_t)b->groups.size();
    std::vector<uint32_t> order(ng);
    for (uint32_t i = 0; i < ng; ++i) order[i] = i;
    auto slot = [&](uint32_t g) { return b->groups[g].item / window + b->groups[g].step; };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        const uint32_t sx = slot(x), sy = slot(y);
        if (sx != sy) return sx < sy;
        if (b->groups[x].step != b->groups[y].step) return b->groups[x].step > b->groups[y].step;
        return b->groups[x].item < b->groups[y].item;
    });
    std::vector<uint32_t> pos(ng), target(ng);
    for (uint32_t i = 0; i < ng; ++i) pos[order[i]] = i;
    std::vector<FusedUnit> units;
    for (uint32_t g : order) {
        const ckks_batch::Group &G = b->groups[g];
        if (G.wait != kNoGroup && (G.wait >= ng || pos[G.wait] >= pos[g]))
            return fail(CKKS_E_ARG, "ckks_batch_set_schedule: internal error, a group before the one it waits for");
        if (G.tiles >= 4096) return fail(CKKS_E_UNSUPPORTED, "ckks_batch_set_schedule: too many tiles per record");
        for (uint32_t limb : G.limbs)
            for (uint32_t t = 0; t < G.tiles; ++t)
                units.push_back(FusedUnit{G.inst, limb | (t << 16) | (G.step << 28), G.wait, g});
        target[g] = (uint32_t)G.limbs.size() * G.tiles;
    }
    const size_t off_cnt = 0, off_tgt = align256((size_t)fused_counter_words(b) * 4),
                 off_units = off_tgt + align256((size_t)ng * 4);
    if (units.size() != fused_units(b) || off_units + units.size() * sizeof(FusedUnit) > fused_region_bytes(b))
        return fail(CKKS_E_ARG, "ckks_batch_set_schedule: internal error, unit list larger than its region");
    char *dev = b->fdev;
    // the region may be in use by a run of the previous schedule on any stream
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(dev + off_tgt, target.data(), (size_t)ng * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && !units.empty())
        e = hipMemcpy(dev + off_units, units.data(), units.size() * sizeof(FusedUnit), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return fail(CKKS_E_DEVICE, std::string("ckks_batch_set_schedule: upload failed: ") + hipGetErrorString(e));
    FusedArgs &f = b->fused;
    f.units = (const FusedUnit *)(dev + off_units);
    f.target = (const uint32_t *)(dev + off_tgt);
    f.claim = (uint32_t *)(dev + off_cnt);
    f.fault = f.claim + 1;
    f.done = f.claim + kDoneStride;
    f.done_stride = kDoneStride;
    f.publish_every = kPublishEvery;
    f.nunits = (uint32_t)units.size();
    f.spin_limit = kFusedSpinLimit;
    for (int s = 0; s < 4; ++s) f.ntt[s] = b->ntt_dev[s];
    f.bconv = b->bconv_dev;
    f.ip = b->ip_dev;
    f.tensor = b->tensor_dev;
    return CKKS_OK;
}

}  // namespace

namespace {

size_t items_bytes(const ckks_ctx *ctx, const ckks_work *items, uint32_t n)
{
    size_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += align256(item_ws_elems(ctx, items[i]) * 8);
    return total;
}

// Validates and plans every item, with the items' workspaces from `ws` on
// (planning only computes addresses; nothing is read or written there).
ckks_status plan_batch(ckks_ctx *ctx, const ckks_work *items, uint32_t n, char *ws, ckks_batch **out)
{
    *out = nullptr;
    for (uint32_t i = 0; i < n; ++i) {
        ckks_status st = validate_item(ctx, items[i], i);
        if (st != CKKS_OK) return st;
    }
    ckks_batch *b = new ckks_batch();
    b->ctx = ctx;
    const uint32_t nt = ntt_tiles(ctx->logn);
    const bool two_pass = ntt_passes(ctx->logn) == 2;
    const struct {
        QKind k;
        NttStage st;
        uint32_t pass;
        int set;
    } spec[QI_COUNT] = {
        {Q_TENSOR, STAGE_FWD_PLAIN, 0, -1},          {Q_NTT, STAGE_INV_PLAIN, 0, 0},
        {Q_NTT, STAGE_INV_GALOIS, 0, 0},             {Q_NTT, STAGE_INV_PLAIN, 1, 0},
        {Q_BCONV, STAGE_FWD_PLAIN, 0, -1},           {Q_NTT, STAGE_FWD_PLAIN, 0, 1},
        {Q_NTT, STAGE_FWD_PLAIN, 1, 1},              {Q_IP, STAGE_FWD_PLAIN, 0, -1},
        {Q_NTT, STAGE_INV_PLAIN, 0, 2},              {Q_NTT, STAGE_INV_PLAIN, 1, 2},
        {Q_NTT, STAGE_FWD_BCONV_MODDOWN, 0, 3},      {Q_NTT, STAGE_FWD_BCONV_MODDOWN, 1, 3},
    };
    for (int qi = 0; qi < QI_COUNT; ++qi) {
        b->q[qi].kind = spec[qi].k;
        b->q[qi].stage = spec[qi].st;
        b->q[qi].pass = spec[qi].pass;
        b->q[qi].set = spec[qi].set;
        b->q[qi].tiles = spec[qi].k == Q_NTT ? nt : ctx->N / (256 * kQueueBlocks);
        b->q[qi].grid_mult = 2;
    }
    char *w = ws;
    uint32_t max_rows = 0;
    for (uint32_t i = 0; i < n; ++i) {
        b->cur_item = i;
        ckks_status st = plan_item(b, items[i], (uint64_t *)w);
        if (st != CKKS_OK) {
            delete b;
            return st;
        }
        w += align256(item_ws_elems(ctx, items[i]) * 8);
        max_rows = std::max(max_rows, ks_sizes(ctx, items[i].a.level).rows);
    }
    b->bconv_tiles = (ctx->N / (256 * kQueueBlocks)) * ((max_rows + kBconvRowGroup - 1) / kBconvRowGroup);
    b->q[QI_UP_BCONV].tiles = b->bconv_tiles;
    if (!two_pass) {  // one pass per transform at N = 2^12: the second-pass steps are empty
        b->q[QI_UP_INTT1].recs.clear();
        b->q[QI_UP_NTT1].recs.clear();
        b->q[QI_DN_INTT1].recs.clear();
        b->q[QI_DN_NTT1].recs.clear();
        for (ckks_batch::Group &g : b->groups)
            if (g.step == QI_UP_INTT1 || g.step == QI_UP_NTT1 || g.step == QI_DN_INTT1 || g.step == QI_DN_NTT1)
                g.limbs.clear();
    }
    *out = b;
    return CKKS_OK;
}

// Launch tables of the per-step schedule: argument blocks, unit records, step counters.
struct TableLayout {
    size_t off_ntt[4], off_bc, off_ip, off_tn, off_rec[QI_COUNT], off_cnt, bytes;
};

TableLayout table_layout(const ckks_batch *b)
{
    TableLayout t;
    size_t off = 0;
    for (int s = 0; s < 4; ++s) {
        t.off_ntt[s] = off;
        off = align256(off + b->ntt[s].size() * sizeof(NttArgs));
    }
    t.off_bc = off;
    off = align256(off + b->bconv.size() * sizeof(BconvArgs));
    t.off_ip = off;
    off = align256(off + b->ip.size() * sizeof(IpArgs));
    t.off_tn = off;
    off = align256(off + b->tensor.size() * sizeof(TensorArgs));
    for (int qi = 0; qi < QI_COUNT; ++qi) {
        t.off_rec[qi] = off;
        off = align256(off + b->q[qi].recs.size() * sizeof(UnitRec));
    }
    t.off_cnt = off;
    t.bytes = align256(off + QI_COUNT * sizeof(uint32_t));
    return t;
}

// The one-launch schedule's region: counters (the claim counter and fault flag,
// then one 128-byte line per group), group sizes, and the unit list (the same
// length for every window).
size_t fused_units(const ckks_batch *b)
{
    size_t n = 0;
    for (const ckks_batch::Group &g : b->groups) n += g.limbs.size() * g.tiles;
    return n;
}

size_t fused_region_bytes(const ckks_batch *b)
{
    const size_t ng = b->groups.size();
    return align256((size_t)fused_counter_words(b) * 4) + align256(ng * 4) + align256(fused_units(b) * sizeof(FusedUnit));
}

}  // namespace

extern "C" size_t ckks_batch_workspace_bytes(const ckks_ctx *ctx, const ckks_work *items, uint32_t n)
{
    if (!ctx || !items || n == 0) return 0;
    for (uint32_t i = 0; i < n; ++i)
        if (items[i].a.level >= ctx->nq) return 0;
    ckks_batch *b = nullptr;
    // addresses only: a nonzero aligned base stands in for the workspace
    if (plan_batch((ckks_ctx *)ctx, items, n, (char *)(uintptr_t)4096, &b) != CKKS_OK) return 0;
    const size_t total = items_bytes(ctx, items, n) + table_layout(b).bytes + fused_region_bytes(b);
    delete b;
    return total;
}

extern "C" ckks_status ckks_batch_create(ckks_ctx *ctx, const ckks_work *items, uint32_t n, void *ws,
                                         ckks_batch **out)
{
    if (!ctx || !items || !out || n == 0) return fail(CKKS_E_ARG, "ckks_batch_create: null argument or empty batch");
    if (!ptr_ok(ws) || ((uintptr_t)ws & 255)) return fail(CKKS_E_ARG, "ckks_batch_create: null or misaligned workspace");
    ckks_batch *b = nullptr;
    TRY(plan_batch(ctx, items, n, (char *)ws, &b));
    // the launch tables follow the items' workspaces, then the one-launch region
    const TableLayout t = table_layout(b);
    std::vector<char> img(t.bytes, 0);
    for (int s = 0; s < 4; ++s)
        if (!b->ntt[s].empty()) memcpy(&img[t.off_ntt[s]], b->ntt[s].data(), b->ntt[s].size() * sizeof(NttArgs));
    if (!b->bconv.empty()) memcpy(&img[t.off_bc], b->bconv.data(), b->bconv.size() * sizeof(BconvArgs));
    if (!b->ip.empty()) memcpy(&img[t.off_ip], b->ip.data(), b->ip.size() * sizeof(IpArgs));
    if (!b->tensor.empty()) memcpy(&img[t.off_tn], b->tensor.data(), b->tensor.size() * sizeof(TensorArgs));
    for (int qi = 0; qi < QI_COUNT; ++qi)
        if (!b->q[qi].recs.empty())
            memcpy(&img[t.off_rec[qi]], b->q[qi].recs.data(), b->q[qi].recs.size() * sizeof(UnitRec));
    b->dev = (char *)ws + items_bytes(ctx, items, n);
    b->fdev = b->dev + t.bytes;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipMemcpy(b->dev, img.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        delete b;
        return fail(CKKS_E_DEVICE, "ckks_batch_create: upload of the launch tables failed");
    }
    for (int s = 0; s < 4; ++s) b->ntt_dev[s] = (const NttArgs *)(b->dev + t.off_ntt[s]);
    b->bconv_dev = (const BconvArgs *)(b->dev + t.off_bc);
    b->ip_dev = (const IpArgs *)(b->dev + t.off_ip);
    b->tensor_dev = (const TensorArgs *)(b->dev + t.off_tn);
    for (int qi = 0; qi < QI_COUNT; ++qi) b->q[qi].recs_dev = (UnitRec *)(b->dev + t.off_rec[qi]);
    b->counters = (uint32_t *)(b->dev + t.off_cnt);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
        b->cus = prop.multiProcessorCount;
    *out = b;
    return CKKS_OK;
}

extern "C" ckks_status ckks_batch_run(ckks_batch *b, void *stream)
{
    if (!b) return fail(CKKS_E_ARG, "ckks_batch_run: null batch");
    hipError_t e = run(b, S(stream));
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_batch_run: ") + hipGetErrorString(e));
    return CKKS_OK;
}

// Persistent grid per step, in workgroups per CU: every candidate runs the
// whole batch once to warm caches and code, then kTuneReps more times; each
// step keeps the candidate with the smallest median time.
extern "C" ckks_status ckks_batch_tune(ckks_batch *b, void *stream)
{
    if (!b) return fail(CKKS_E_ARG, "ckks_batch_tune: null batch");
    static const uint32_t cand[] = {1, 2, 3, 4, 6, 8};
    constexpr int nc = sizeof(cand) / sizeof(cand[0]), kTuneReps = 5;
    std::vector<float> ms((size_t)nc * QI_COUNT * kTuneReps, 0.f);
    hipEvent_t ev[QI_COUNT + 1];
    for (int i = 0; i <= QI_COUNT; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
            return fail(CKKS_E_DEVICE, "ckks_batch_tune: events");
        }
    hipStream_t st = S(stream);
    hipError_t e = hipSuccess;
    for (int rep = -1; rep < kTuneReps && e == hipSuccess; ++rep)
        for (int ci = 0; ci < nc && e == hipSuccess; ++ci) {
            e = launch_zero_u32(b->counters, QI_COUNT, st);
            for (int qi = 0; qi < QI_COUNT && e == hipSuccess; ++qi) {
                (void)hipEventRecord(ev[qi], st);
                e = launch_queue(b, qi, cand[ci], st);
            }
            (void)hipEventRecord(ev[QI_COUNT], st);
            if (e == hipSuccess) e = hipEventSynchronize(ev[QI_COUNT]);
            for (int qi = 0; qi < QI_COUNT && e == hipSuccess && rep >= 0; ++qi)
                (void)hipEventElapsedTime(&ms[((size_t)ci * QI_COUNT + qi) * kTuneReps + rep], ev[qi], ev[qi + 1]);
        }
    for (int i = 0; i <= QI_COUNT; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_batch_tune: ") + hipGetErrorString(e));
    for (int qi = 0; qi < QI_COUNT; ++qi) {
        float best = 1e30f;
        uint32_t pick = 2;
        for (int ci = 0; ci < nc; ++ci) {
            float *x = &ms[((size_t)ci * QI_COUNT + qi) * kTuneReps];
            std::sort(x, x + kTuneReps);
            if (x[kTuneReps / 2] < best) {
                best = x[kTuneReps / 2];
                pick = cand[ci];
            }
        }
        b->q[qi].grid_mult = pick;
    }
    return CKKS_OK;
}

extern "C" ckks_status ckks_batch_set_grid(ckks_batch *b, uint32_t step, uint32_t wg_per_cu)
{
    if (!b || step >= QI_COUNT || wg_per_cu == 0 || wg_per_cu > 16)
        return fail(CKKS_E_ARG, "ckks_batch_set_grid: null batch, step out of range or grid not in [1, 16]");
    b->q[step].grid_mult = wg_per_cu;
    return CKKS_OK;
}

// A captured graph holds the launches of the schedule it was captured with: dropped on a change.
void drop_graph(ckks_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" ckks_status ckks_batch_set_schedule(ckks_batch *b, uint32_t window, uint32_t wg_per_cu)
{
    if (!b) return fail(CKKS_E_ARG, "ckks_batch_set_schedule: null batch");
    if (window == 0) {
        if (b->window != 0) drop_graph(b);
        b->window = 0;
        return CKKS_OK;
    }
    if (b->ctx->logn != 16)
        return fail(CKKS_E_UNSUPPORTED, "ckks_batch_set_schedule: the one-launch schedule needs N = 2^16");
    if (wg_per_cu == 0 || wg_per_cu > 2)
        return fail(CKKS_E_ARG, "ckks_batch_set_schedule: 1 or 2 workgroups per CU (the kernel's occupancy)");
    if (b->window != window) TRY(build_fused(b, window));
    if (b->window != window || b->fused_mult != wg_per_cu) drop_graph(b);
    b->window = window;
    b->fused_mult = wg_per_cu;
    return CKKS_OK;
}

extern "C" uint32_t ckks_batch_schedule(const ckks_batch *b) { return b ? b->window : 0; }

extern "C" ckks_status ckks_batch_faults(ckks_batch *b, void *stream)
{
    if (!b) return fail(CKKS_E_ARG, "ckks_batch_faults: null batch");
    if (hipStreamSynchronize(S(stream)) != hipSuccess) return fail(CKKS_E_DEVICE, "ckks_batch_faults: synchronize");
    if (!b->window && !b->fused.fault) return CKKS_OK;
    uint32_t flag = 0;
    if (hipMemcpy(&flag, b->fused.fault, 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CKKS_E_DEVICE, "ckks_batch_faults: read back");
    if (flag) return fail(CKKS_E_DEVICE, "ckks_batch: a one-launch run gave up waiting for a dependency");
    return CKKS_OK;
}

extern "C" uint32_t ckks_batch_steps(void) { return QI_COUNT; }

extern "C" ckks_status ckks_batch_capture(ckks_batch *b, void *stream)
{
    if (!b) return fail(CKKS_E_ARG, "ckks_batch_capture: null batch");
    hipStream_t st = S(stream);
    if (!st) return fail(CKKS_E_ARG, "ckks_batch_capture: the default stream cannot be captured");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(CKKS_E_DEVICE, "ckks_batch_capture: begin capture failed");
    const hipError_t e = run(b, st);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (e2 == hipSuccess && g) (void)hipGraphDestroy(g);
        return fail(CKKS_E_DEVICE, std::string("ckks_batch_capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        return fail(CKKS_E_DEVICE, "ckks_batch_capture: instantiate failed");
    }
    return CKKS_OK;
}

extern "C" ckks_status ckks_batch_replay(ckks_batch *b, void *stream)
{
    if (!b || !b->exec) return fail(CKKS_E_ARG, "ckks_batch_replay: nothing captured");
    hipError_t e = hipGraphLaunch(b->exec, S(stream));
    if (e != hipSuccess) return fail(CKKS_E_DEVICE, std::string("ckks_batch_replay: ") + hipGetErrorString(e));
    return CKKS_OK;
}

extern "C" uint32_t ckks_batch_keyswitches(const ckks_batch *b) { return b ? b->keyswitches : 0; }

extern "C" uint32_t ckks_batch_grid(const ckks_batch *b, uint32_t step)
{
    return (b && step < QI_COUNT) ? b->q[step].grid_mult : 0;
}

extern "C" void ckks_batch_destroy(ckks_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;  // the tables are in the caller's workspace
}
