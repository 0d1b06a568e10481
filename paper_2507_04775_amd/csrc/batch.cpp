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

namespace {

enum QKind { Q_NTT = 0, Q_BCONV, Q_IP, Q_TENSOR };

// launch order of the steps of a batch
enum QIndex {
    QI_TENSOR = 0,
    QI_UP_INTT0_PLAIN,
    QI_UP_INTT0_GALOIS,
    QI_UP_INTT1,
    QI_UP_BCONV,
    QI_UP_NTT0,
    QI_UP_NTT1,
    QI_IP,
    QI_DN_INTT0,
    QI_DN_INTT1,
    QI_DN_NTT0,
    QI_DN_NTT1,
    QI_COUNT
};

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
};

namespace {

void add_recs(ckks_batch *b, int qi, uint32_t inst, uint32_t n)
{
    for (uint32_t l = 0; l < n; ++l) b->q[qi].recs.push_back(UnitRec{inst, l});
}

// ModDown of npoly accumulators (two INTT passes and two NTT passes at N = 2^16)
void plan_moddown(ckks_batch *b, const uint64_t *acc, int64_t stride, uint32_t level, uint64_t *const *out,
                  const uint64_t *const *add, uint32_t g, uint64_t *pc, uint64_t *conv)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    uint32_t di = (uint32_t)b->ntt[2].size();
    b->ntt[2].push_back(args_moddown_intt(c, acc, stride, level, pc));
    add_recs(b, QI_DN_INTT0, di, 2 * c->np);
    add_recs(b, QI_DN_INTT1, di, 2 * c->np);
    uint32_t mi = (uint32_t)b->ntt[3].size();
    b->ntt[3].push_back(args_moddown_ntt(c, acc, stride, 2, level, out, add, g, pc, conv));
    add_recs(b, QI_DN_NTT0, mi, 2 * s.n);
    add_recs(b, QI_DN_NTT1, mi, 2 * s.n);
}

// ModUp of d (gathered through g) into ext; returns nothing, records the steps
void plan_modup(ckks_batch *b, const uint64_t *d, uint32_t g, uint32_t level, uint64_t *dc, uint64_t *ext)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    uint32_t ui = (uint32_t)b->ntt[0].size();
    b->ntt[0].push_back(args_modup_intt(c, d, g, level, dc));
    add_recs(b, g == 1 ? QI_UP_INTT0_PLAIN : QI_UP_INTT0_GALOIS, ui, s.n);
    add_recs(b, QI_UP_INTT1, ui, s.n);
    uint32_t bi = (uint32_t)b->bconv.size();
    b->bconv.push_back(args_modup_bconv(c, d, g, level, dc, ext, false));
    add_recs(b, QI_UP_BCONV, bi, s.beta);
    uint32_t ni = (uint32_t)b->ntt[1].size();
    NttArgs na = args_modup_ntt(c, level, ext);
    b->ntt[1].push_back(na);
    for (uint32_t l = 0; l < s.beta * s.rows; ++l) {
        const uint32_t poly = l / na.map.rows, row = l - poly * na.map.rows;
        if (limb_skipped(na.map, poly, row)) continue;  // the digit's own rows are read from d
        b->q[QI_UP_NTT0].recs.push_back(UnitRec{ni, l});
        b->q[QI_UP_NTT1].recs.push_back(UnitRec{ni, l});
    }
}

void plan_keyswitch(ckks_batch *b, const uint64_t *d, uint32_t g_in, uint32_t level, const uint64_t *key,
                    uint64_t *out0, uint64_t *out1, const uint64_t *add0, const uint64_t *add1, uint32_t g_add,
                    uint64_t *ws)
{
    const ckks_ctx *c = b->ctx;
    KsSizes s = ks_sizes(c, level);
    KsWs w = ks_ws(c, level, ws);
    plan_modup(b, d, g_in, level, w.dc, w.ext);
    uint32_t ii = (uint32_t)b->ip.size();
    b->ip.push_back(args_ip(c, w.ext, level, key, 1, w.acc, d, g_in));
    add_recs(b, QI_IP, ii, s.rows);
    uint64_t *outs[2] = {out0, out1};
    const uint64_t *adds[2] = {add0, add1};
    plan_moddown(b, w.acc, (int64_t)s.rows * s.N, level, outs, adds, g_add, w.pc, w.conv);
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
        plan_keyswitch(b, d2, 1, level, w.key->data, w.out->c0, w.out->c1, w.out->c0, w.out->c1, 1,
                       d2 + (size_t)s.n * s.N);
        return CKKS_OK;
    }
    case CKKS_WORK_KEYSWITCH:
        plan_keyswitch(b, w.a.c0, 1, level, w.key->data, w.out->c0, w.out->c1, nullptr, nullptr, 1, ws);
        return CKKS_OK;
    case CKKS_WORK_ROTATE:
        plan_keyswitch(b, w.a.c1, w.galois, level, w.key->data, w.out->c0, w.out->c1, w.a.c0, nullptr, w.galois, ws);
        return CKKS_OK;
    case CKKS_WORK_HOISTED: {
        uint64_t *dc = ws, *ext = dc + (size_t)s.n * s.N, *per = ext + (size_t)s.beta * s.rows * s.N;
        plan_modup(b, w.a.c1, 1, level, dc, ext);
        const size_t per_rot = (2 * (size_t)s.rows + 2 * (size_t)c->np + 2 * (size_t)s.n) * s.N;
        for (uint32_t r = 0; r < w.n_rot; ++r) {
            const uint32_t g = galois_of(c, w.rot[r]);
            uint64_t *acc = per + r * per_rot, *pc = acc + 2 * (size_t)s.rows * s.N, *conv = pc + 2 * (size_t)c->np * s.N;
            uint32_t ii = (uint32_t)b->ip.size();
            b->ip.push_back(args_ip(c, ext, level, w.rot_keys[r]->data, g, acc, w.a.c1, g));
            add_recs(b, QI_IP, ii, s.rows);
            uint64_t *outs[2] = {w.out[r].c0, w.out[r].c1};
            const uint64_t *adds[2] = {w.a.c0, nullptr};
            plan_moddown(b, acc, (int64_t)s.rows * s.N, level, outs, adds, g, pc, conv);
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

hipError_t run(ckks_batch *b, hipStream_t st)
{
    hipError_t e = launch_zero_u32(b->counters, QI_COUNT, st);
    for (int qi = 0; qi < QI_COUNT && e == hipSuccess; ++qi) e = launch_queue(b, qi, b->q[qi].grid_mult, st);
    return e;
}

}  // namespace

extern "C" size_t ckks_batch_workspace_bytes(const ckks_ctx *ctx, const ckks_work *items, uint32_t n)
{
    if (!ctx || !items) return 0;
    size_t total = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (items[i].a.level >= ctx->nq) return 0;
        total += align256(item_ws_elems(ctx, items[i]) * 8);
    }
    return total;
}

extern "C" ckks_status ckks_batch_create(ckks_ctx *ctx, const ckks_work *items, uint32_t n, void *ws,
                                         ckks_batch **out)
{
    if (!ctx || !items || !out || n == 0) return fail(CKKS_E_ARG, "ckks_batch_create: null argument or empty batch");
    if (!ptr_ok(ws)) return fail(CKKS_E_ARG, "ckks_batch_create: null or misaligned workspace");
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
    char *w = (char *)ws;
    uint32_t max_rows = 0;
    for (uint32_t i = 0; i < n; ++i) {
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
    }
    // device tables
    size_t off = 0, off_ntt[4], off_bc, off_ip, off_tn, off_rec[QI_COUNT], off_cnt;
    for (int s = 0; s < 4; ++s) {
        off_ntt[s] = off;
        off = align256(off + b->ntt[s].size() * sizeof(NttArgs));
    }
    off_bc = off;
    off = align256(off + b->bconv.size() * sizeof(BconvArgs));
    off_ip = off;
    off = align256(off + b->ip.size() * sizeof(IpArgs));
    off_tn = off;
    off = align256(off + b->tensor.size() * sizeof(TensorArgs));
    for (int qi = 0; qi < QI_COUNT; ++qi) {
        off_rec[qi] = off;
        off = align256(off + b->q[qi].recs.size() * sizeof(UnitRec));
    }
    off_cnt = off;
    off = align256(off + QI_COUNT * sizeof(uint32_t));
    std::vector<char> img(off, 0);
    for (int s = 0; s < 4; ++s)
        if (!b->ntt[s].empty()) memcpy(&img[off_ntt[s]], b->ntt[s].data(), b->ntt[s].size() * sizeof(NttArgs));
    if (!b->bconv.empty()) memcpy(&img[off_bc], b->bconv.data(), b->bconv.size() * sizeof(BconvArgs));
    if (!b->ip.empty()) memcpy(&img[off_ip], b->ip.data(), b->ip.size() * sizeof(IpArgs));
    if (!b->tensor.empty()) memcpy(&img[off_tn], b->tensor.data(), b->tensor.size() * sizeof(TensorArgs));
    for (int qi = 0; qi < QI_COUNT; ++qi)
        if (!b->q[qi].recs.empty())
            memcpy(&img[off_rec[qi]], b->q[qi].recs.data(), b->q[qi].recs.size() * sizeof(UnitRec));
    if (hipSetDevice(ctx->device) != hipSuccess || hipMalloc((void **)&b->dev, off) != hipSuccess) {
        delete b;
        return fail(CKKS_E_NOMEM, "ckks_batch_create: device tables");
    }
    if (hipMemcpy(b->dev, img.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(b->dev);
        delete b;
        return fail(CKKS_E_DEVICE, "ckks_batch_create: upload failed");
    }
    for (int s = 0; s < 4; ++s) b->ntt_dev[s] = (const NttArgs *)(b->dev + off_ntt[s]);
    b->bconv_dev = (const BconvArgs *)(b->dev + off_bc);
    b->ip_dev = (const IpArgs *)(b->dev + off_ip);
    b->tensor_dev = (const TensorArgs *)(b->dev + off_tn);
    for (int qi = 0; qi < QI_COUNT; ++qi) b->q[qi].recs_dev = (UnitRec *)(b->dev + off_rec[qi]);
    b->counters = (uint32_t *)(b->dev + off_cnt);
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
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}
