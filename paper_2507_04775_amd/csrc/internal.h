// Internal declarations of the gfx950 CKKS library: the context with its
// device tables, kernel argument blocks and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ckks.h"
#include "modarith.h"

namespace ckks {

constexpr int kMaxDigitPrimes = 16;  // primes per digit / in the special basis
constexpr int kMaxDigits = 16;
constexpr int kMaxPrimes = 64;
constexpr uint32_t kAllPrimes = 0xFFFFFFFFu;
constexpr int kMaxHeavy = 32;  // integer-path limbs a grid launch places apart

// Row -> prime map of a launch over limbs.  Limb y of a launch is row
// (y % rows) of polynomial (y / rows).  With level == kAllPrimes row r uses
// prime prime0 + r; otherwise logical row lr = row0 + r uses q_lr for
// lr <= level and p_{lr-level-1} (prime index nq + lr - level - 1) above.
// skip_alpha > 0 skips, in polynomial j, the logical rows of digit j.
struct LimbMap {
    uint32_t rows;
    uint32_t level;
    uint32_t prime0;
    uint32_t nq;
    uint32_t row0;
    uint32_t skip_alpha;
    uint32_t dense;           // with skip_alpha: limb indices enumerate only the rows that are not skipped
    int64_t src_poly_stride;  // elements between polynomials of the input (may be negative)
    int64_t dst_poly_stride;  // elements between polynomials of the output
};

__host__ __device__ inline uint32_t limb_prime(const LimbMap &m, uint32_t r)
{
    uint32_t lr = r + m.row0;
    if (m.level == kAllPrimes) return m.prime0 + lr;
    return lr <= m.level ? lr : m.nq + (lr - m.level - 1);
}

__host__ __device__ inline bool limb_skipped(const LimbMap &m, uint32_t poly, uint32_t r)
{
    if (m.skip_alpha == 0) return false;
    uint32_t lr = r + m.row0;
    uint32_t lo = poly * m.skip_alpha;
    uint32_t hi = lo + m.skip_alpha < m.level + 1 ? lo + m.skip_alpha : m.level + 1;
    return lr >= lo && lr < hi;
}

__device__ __forceinline__ uint32_t bitrev(uint32_t x, uint32_t logn) { return __brev(x) >> (32 - logn); }

// Position whose value moves to position e under X -> X^g in the evaluation
// domain: out[e] = in[br(((2 br(e) + 1) g mod 2N - 1) / 2)].
__device__ __forceinline__ uint32_t galois_src(uint32_t e, uint32_t g, uint32_t logn)
{
    uint32_t i = bitrev(e, logn);
    uint32_t x = ((2 * i + 1) * g) & ((2u << logn) - 1);  // wraps mod 2^32, exact mod 2N
    return bitrev((x - 1) >> 1, logn);
}

// Prologue of the first forward pass / epilogue of the last forward pass.
enum NttPro { PRO_PLAIN = 0, PRO_RESCALE = 1, PRO_GALOIS = 2, PRO_BCONV = 3, PRO_TENSOR = 4 };
enum NttEpi { EPI_PLAIN = 0, EPI_MODDOWN = 1, EPI_RESCALE = 2 };

struct NttArgs {
    uint64_t *dst;
    const uint64_t *src;
    uint64_t *mid;              // output of the first pass / input of the second (N = 2^16)
    int64_t mid_stride;         // elements between polynomials in mid
    LimbMap map;
    const Prime *primes;
    const ulonglong2 *tw;       // [n_primes][N] {w, floor(w 2^64 / q)}
    const double *twd;          // [n_primes][N] w as a double (primes below 2^50)
    uint32_t logn;
    uint32_t galois;            // PRO_GALOIS gather / addend gather (1 = none)
    // EPI_MODDOWN: out_p = Pinv (aux_p - x) + add_p ; EPI_RESCALE: out_p = qlinv (aux_p - x)
    const uint64_t *aux[2];     // per polynomial (row r at aux[p] + r N)
    const uint64_t *add[2];     // per polynomial, may be null
    uint64_t *out[2];           // per polynomial
    const ulonglong2 *cst;      // per prime index: Pinv or q_l^-1 pair
    // PRO_RESCALE: input limb per polynomial (coefficients under q_l), q_l mod q_i per prime
    const uint64_t *rs_src[2];
    const uint64_t *rs_qlmod;
    uint64_t rs_ql;
    // Last inverse pass: multiply by N^-1 (ys_mode 0), or by N^-1 [(B/b_i)^-1]_{b_i}, the scale
    // that turns the row into the input of a fast base conversion from basis B: the ModUp digits
    // of level nlev-1 (ys_mode 1, row i in digit i / alpha) or the special basis (ys_mode 2).
    uint32_t ys_mode;
    uint32_t alpha, nlev, nprimes, pset;
    const ulonglong2 *ys;       // [nsets][kMaxDigitPrimes] Shoup pairs
    const double *ysd;          // the same constants as doubles
    // PRO_BCONV: the first forward pass computes its input as a fast base conversion of scaled
    // rows (written by an inverse with ys_mode 1 or 2).  bc_mode 1: ModUp, polynomial j of the
    // launch is digit j and its source rows are bc_src rows j alpha ..; bc_mode 2: ModDown,
    // polynomial t reads the K rows at bc_src + t bc_poly_stride.
    const uint64_t *bc_src;
    int64_t bc_poly_stride;
    uint32_t bc_mode;
    const uint64_t *hmod;       // [nsets][n_primes][kMaxDigitPrimes]
    // bc_mode 2 converts with centred inputs y_k in [-(p_k-1)/2, (p_k-1)/2]: every y_k above
    // (p_k-1)/2 subtracts [P]_q once, read from pmod[prime]
    const uint64_t *pmod;
    // Grid launches at N = 2^16 place the limbs on the 64-bit integer path (primes of 2^50 and
    // above, about 2.4 times the work of an FP64 limb) apart from the others; see grid_unit.
    uint64_t int_primes;        // bit i: prime i is on the integer path
    uint32_t n_heavy, heavy_pad;
    uint8_t heavy[kMaxHeavy];   // launch limbs on the integer path, ascending (n_heavy of them)
    // PRO_TENSOR (first inverse pass): the input row is [src * src2]_q, HMult's d2 = a1 b1
    const uint64_t *src2;
};

// A unit of work of a persistent stage kernel is one tile of limb `limb` of
// instance `inst` (an NttArgs / BconvArgs / IpArgs of the batch); units are
// claimed in order from `counter`, which must be zero when the stage starts.
struct UnitRec {
    uint32_t inst, limb;
};
static_assert(sizeof(UnitRec) == 8, "a unit record is two words: inst, then limb");

struct WorkQueue {
    const UnitRec *recs;
    uint32_t nrecs;
    uint32_t tiles;             // units per record
    uint32_t *counter;
};

// Persistent work-queue loop shared by every stage kernel: units are claimed
// from q.counter (the next claim is issued while the current unit runs), the
// unit's argument block is copied into LDS (`sa`) whenever the instance
// changes, and body(sa, limb, tile) processes the unit with the whole block.
template <class Args, class Body>
__device__ __forceinline__ void run_work_queue(const Args *insts, const WorkQueue &q, Args &sa, uint32_t *claim,
                                               Body body)
{
    static_assert(sizeof(Args) % 8 == 0, "argument blocks are copied as 8-byte words");
    const uint32_t total = q.nrecs * q.tiles;
    if (threadIdx.x == 0) *claim = atomicAdd(q.counter, 1u);
    __syncthreads();
    uint32_t u = *claim;
    uint32_t have = 0xFFFFFFFFu;
    while (u < total) {
        const UnitRec rec = q.recs[u / q.tiles];
        __syncthreads();  // every thread has read *claim and is done with sa and the unit's LDS
        if (threadIdx.x == 0) *claim = atomicAdd(q.counter, 1u);
        if (rec.inst != have) {
            const uint64_t *src = (const uint64_t *)(insts + rec.inst);
            uint64_t *dst = (uint64_t *)&sa;
            for (uint32_t i = threadIdx.x; i < sizeof(Args) / 8; i += blockDim.x) dst[i] = src[i];
            have = rec.inst;
        }
        __syncthreads();
        body(sa, rec.limb, u % q.tiles);
        __syncthreads();
        u = *claim;
    }
}

// The same loop for argument blocks without dynamically indexed fields (the
// NTT passes): the claim is made wave-uniform and the unit record and the
// argument block are read through the constant address space, so they come in
// with scalar loads into scalar registers, as a grid kernel receives its
// arguments.  An argument block in LDS occupies vector registers instead,
// 8 to 14 more per thread in these passes, which put the Rescale prologue
// pass and the first inverse pass above the 128 that two 512-thread
// workgroups per CU allow.  Both blocks are written before the launch and
// only read here.
template <class Args, class Body>
__device__ __forceinline__ void run_work_queue_uniform(const Args *insts, const WorkQueue &q, uint32_t *claim,
                                                       Body body)
{
    static_assert(sizeof(Args) % 4 == 0, "argument blocks are read as 4-byte words");
    typedef const __attribute__((address_space(4))) uint32_t ConstWord;
    const uint32_t total = q.nrecs * q.tiles;
    if (threadIdx.x == 0) *claim = atomicAdd(q.counter, 1u);
    __syncthreads();
    uint32_t u = __builtin_amdgcn_readfirstlane(*claim);
    while (u < total) {
        const uint32_t ri = __builtin_amdgcn_readfirstlane(u / q.tiles);
        ConstWord *rec = (ConstWord *)((uintptr_t)q.recs + (uintptr_t)ri * sizeof(UnitRec));
        const uint32_t inst = __builtin_amdgcn_readfirstlane(rec[0]);  // UnitRec::inst
        const uint32_t limb = __builtin_amdgcn_readfirstlane(rec[1]);  // UnitRec::limb
        __syncthreads();  // every thread has read *claim and is done with the unit's LDS
        if (threadIdx.x == 0) *claim = atomicAdd(q.counter, 1u);
        Args a;
        ConstWord *src = (ConstWord *)((uintptr_t)insts + (uintptr_t)inst * sizeof(Args));
#pragma unroll
        for (uint32_t i = 0; i < sizeof(Args) / 4; ++i) ((uint32_t *)&a)[i] = src[i];
        body(a, limb, u - ri * q.tiles);
        __syncthreads();
        u = __builtin_amdgcn_readfirstlane(*claim);
    }
}

// The steps of a batch of key switches, in the order of their dependencies
// (one persistent launch each, or one unit kind each of the one-launch batch
// kernel).
enum BatchStep {
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

// One unit of the one-launch batch kernel: tile `tile` of limb (record)
// `limb` of instance `inst` of step `step`, which starts once every unit of
// group `wait` is done and counts itself done in group `signal`.  A group is
// the set of units of one step of one key switch (one instance).  Units are
// listed in an order in which every group comes after the group it waits
// for, and claimed in that order, so the wait of the earliest unfinished unit
// is always satisfied and the launch cannot deadlock.
constexpr uint32_t kNoGroup = 0xFFFFFFFFu;
struct BconvArgs;
struct IpArgs;
struct TensorArgs;
struct FusedUnit {
    uint32_t inst;
    uint32_t code;              // limb | tile << 16 | step << 28
    uint32_t wait;              // group to wait for, or kNoGroup
    uint32_t signal;            // group of this unit
};
static_assert(sizeof(FusedUnit) == 16, "a fused unit is four words");

struct FusedArgs {
    const FusedUnit *units;
    const uint32_t *target;     // per group: its number of units
    uint32_t *claim;            // next unit to claim; zero at launch
    uint32_t *done;             // per group g: units done, at done[g * done_stride]; zero at launch
    uint32_t *fault;            // set to 1 when a wait gave up (spin_limit polls)
    uint32_t nunits, spin_limit, done_stride;
    uint32_t publish_every;     // completions are published after at most this many groups (1..32)
    const NttArgs *ntt[4];      // ModUp INTT, ModUp NTT, ModDown INTT, ModDown NTT instances
    const BconvArgs *bconv;
    const IpArgs *ip;
    const TensorArgs *tensor;
};

enum NttStage {
    STAGE_FWD_PLAIN = 0,
    STAGE_FWD_MODDOWN,
    STAGE_FWD_RESCALE,
    STAGE_FWD_BCONV_MODDOWN,
    STAGE_INV_PLAIN,
    STAGE_INV_GALOIS,
    STAGE_FWD_LIFT,             // centred lift of one source limb into every row, then forward NTT
    STAGE_INV_TENSOR            // inverse NTT of the product of two polynomials (N = 2^16)
};

struct BconvJob {
    const uint64_t *src;        // ns coefficient-domain limbs, stride N
    uint64_t *dst;              // output rows at dst + r N
    const uint64_t *copy_src;   // rows [lo, hi) copied from here to dst (may be null)
    const ulonglong2 *hinv;     // ns pairs {[(B/b_i)^-1]_{b_i}, shoup}
    const uint64_t *hmod;       // [n_primes][kMaxDigitPrimes]: [B/b_i]_c (split_const form for c < 2^50)
    uint32_t ns;
    uint32_t src_prime0;
    uint32_t lo, hi;            // output rows not converted
};

struct BconvArgs {
    BconvJob job[kMaxDigits];
    const Prime *primes;
    uint32_t nrows;             // output rows 0..nrows-1
    uint32_t level, nq;         // row -> prime map as in LimbMap
    uint32_t N, logn;
    uint32_t copy_galois;       // copied rows are gathered through X -> X^g (1 = plain copy)
    uint32_t prescaled;         // sources already hold y_i (the iNTT folded the scaling in)
};

constexpr uint32_t kBconvRowGroup = 8;  // output rows per workgroup (grid z splits the rows)
constexpr uint32_t kQueueBlocks = 16;   // 256-coefficient blocks per unit of the persistent coefficient-wise kernels

struct IpArgs {
    const uint64_t *ext;        // [beta][rows][N]
    const uint64_t *key;        // [dnum][2][nq+np][N]
    uint64_t *acc;              // [2][rows][N]
    const Prime *primes;
    uint32_t beta, rows, level, nq, np, logn, alpha;
    uint32_t galois;            // every digit row gathered through X -> X^g (hoisted rotation; 1 = none)
    const uint64_t *own;        // non-null: digit j's own rows are read from own[r] (gathered through
    uint32_t own_galois;        // own_galois), not from ext
    // HMult's tensor folded in (grid launches, galois = own_galois = 1): the key-switched
    // polynomial is d2 = a1 b1, whose digit-own rows are formed from ta1, tb1 (own unused),
    // and rows q_0..q_l also accumulate [P]_q d0 (half 0) and [P]_q d1 (half 1),
    // d0 = a0 b0, d1 = a0 b1 + a1 b0; pmod[prime] = [P]_q.  ta0 null: no tensor.
    const uint64_t *ta0, *ta1, *tb0, *tb1;
    const uint64_t *pmod;
    // A hoisted giant step of the bootstrap folded in (grid launches; fold_tot set): instead of
    // acc, tot_t = (fold_first ? 0 : tot_t) + acc_t + (t == 0 and r <= l ? [P]_q phi_g(fold_c0) : 0),
    // g = own_galois, tot laid out as acc ([2][rows][N])
    const uint64_t *fold_c0;
    uint64_t *fold_tot;
    uint32_t fold_first, fold_pad;
};

enum CtOp { CT_HADD = 0, CT_PTADD, CT_PTMULT, CT_SCALAR_ADD, CT_SCALAR_MULT };

// One ciphertext-level support operation: halves t = 0, 1 of a (and b, or the
// plaintext in b[0]), scalars s[l] per limb, written to out[t].
struct CtOpArgs {
    const uint64_t *a[2], *b[2];
    uint64_t *out[2];
    const Prime *primes;
    uint32_t logn, pad;
    uint64_t s[kMaxPrimes];
};

// Accumulation of one giant step in the extended basis (hoisted ModDown):
// for half t and row r (q_0..q_l, then p_0..p_{K-1}),
//   part = (acc[t] ? acc[t][r] : 0) + (s[t] && r <= l ? [P]_(q_r) phi_g(s[t])[r] : 0)
//   tot[t][r] = first ? part : tot[t][r] + part.
struct FoldArgs {
    uint64_t *tot[2];
    const uint64_t *acc[2];
    const uint64_t *s[2];
    const uint64_t *pmod;       // [n_primes] P mod q_i
    const Prime *primes;
    uint32_t level, nq, logn, galois, first, pad;
};

struct TensorArgs {
    const uint64_t *a0, *a1, *b0, *b1;
    uint64_t *d0, *d1, *d2;
    const Prime *primes;
    uint32_t logn, pad;
};

// Linear combinations of ciphertexts with plaintexts (the baby-step sums of
// the bootstrap's linear transforms): for each output o < nout (1 or 2),
// out_t[o] = sum_b a_t[b] * pt[o][b], t = 0, 1.  Two outputs (two giant steps
// over the same babies) read the babies once.
constexpr uint32_t kMaxLincomb = 16;
constexpr uint32_t kLincombOut = 2;

struct LincombArgs {
    const uint64_t *a0[kMaxLincomb], *a1[kMaxLincomb], *pt[kLincombOut][kMaxLincomb];
    uint64_t *out0[kLincombOut], *out1[kLincombOut];
    const Prime *primes;
    uint32_t n, logn, nout, pad;
};

// out_t = acc_t + sum_b a_t[b] * c[b][limb] with per-limb scalar residues
// c[b][limb] = cst[b * cst_stride + limb] (integer combination of ciphertexts).
struct ScalarLincombArgs {
    const uint64_t *a0[kMaxLincomb], *a1[kMaxLincomb];
    const uint64_t *cst;
    uint32_t cst_stride;
    const uint64_t *acc0, *acc1;  // may be null; may equal out
    uint64_t *out0, *out1;
    const Prime *primes;
    uint32_t n, logn;
};

// Host modular arithmetic (context.cpp), for the context builders.
uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t m);
uint64_t pow_mod(uint64_t base, uint64_t e, uint64_t m);
uint64_t inv_mod(uint64_t a, uint64_t m);  // m prime
bool probably_prime(uint64_t n);
uint64_t smallest_2n_root(uint64_t q, uint64_t two_n);
uint32_t reverse_bits(uint32_t x, uint32_t bits);

// Launchers (all asynchronous on `stream`).
hipError_t launch_ntt_fwd(const NttArgs &a, uint32_t nlimbs, NttPro pro, NttEpi epi, hipStream_t stream,
                          uint64_t *mid, int64_t mid_poly_stride);
hipError_t launch_ntt_inv(const NttArgs &a, uint32_t nlimbs, NttPro pro, hipStream_t stream, uint64_t *mid,
                          int64_t mid_poly_stride);
uint32_t ntt_passes(uint32_t logn);
uint32_t ntt_tiles(uint32_t logn);  // tiles per limb of the persistent passes
// Tile width (16, 8 or 4 columns / rows per workgroup) of the N = 2^16 grid
// launches over nlimbs limbs, per direction; 0 restores the default rule.
constexpr uint32_t kMaxTileLimbs = 128;
bool ntt_tile_set(uint32_t inverse, uint32_t nlimbs, uint32_t tile);
uint32_t ntt_tile_get(uint32_t inverse, uint32_t nlimbs);
// first_pass 1 (N = 2^16): the second pass only, the first pass's output already in a.mid
hipError_t launch_ntt_stage(NttStage st, const NttArgs &a, uint32_t nlimbs, hipStream_t stream,
                            uint32_t first_pass = 0);
hipError_t launch_ntt_stage_queue(NttStage st, uint32_t logn, uint32_t pass, const NttArgs *insts,
                                  const WorkQueue &q, uint32_t grid, hipStream_t stream);
hipError_t launch_bconv(const BconvArgs &a, uint32_t njobs, hipStream_t stream);
hipError_t launch_bconv_queue(const BconvArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream);
hipError_t launch_inner_product_queue(const IpArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream);
hipError_t launch_tensor_queue(const TensorArgs *insts, const WorkQueue &q, uint32_t grid, hipStream_t stream);
hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t stream);
// The one-launch batch kernel (N = 2^16 only): `grid` workgroups of 512 threads.
hipError_t launch_fused_batch(const FusedArgs &f, uint32_t grid, hipStream_t stream);
hipError_t launch_inner_product(const IpArgs &a, hipStream_t stream);  // ta0 set: the tensor form
// N = 2^16: the inner product of a key switch whose ModDown INTT is `ia` (args_moddown_intt over the
// same accumulators), with that INTT's first pass on the special rows run by the same launch; the
// INTT then runs with first_pass 1.  The special rows of ip.acc are not written.
hipError_t launch_inner_product_rowpass(const IpArgs &ip, const NttArgs &ia, hipStream_t stream);
hipError_t launch_tensor(const uint64_t *a0, const uint64_t *a1, const uint64_t *b0, const uint64_t *b1,
                         uint64_t *d0, uint64_t *d1, uint64_t *d2, const Prime *primes, uint32_t nlimbs,
                         uint32_t logn, hipStream_t stream);
// op: 0 add, 1 sub, 2 mul, 3 mul-add (a*b+c), 4 scalar mul (host_scalars[limb]), 5 scalar add
hipError_t launch_elementwise(int op, const uint64_t *a, const uint64_t *b, const uint64_t *c, uint64_t *out,
                              const uint64_t *host_scalars, const Prime *primes, uint32_t nlimbs, uint32_t logn,
                              hipStream_t stream);
// rows = l+1+K extended rows
hipError_t launch_fold_ext(const FoldArgs &a, uint32_t rows, hipStream_t stream);
// halves: 2, or 1 to leave half 1 untouched (in place PtAdd / ScalarAdd)
hipError_t launch_ct_op(int op, const CtOpArgs &a, uint32_t nlimbs, uint32_t halves, hipStream_t stream);
hipError_t launch_automorph(const uint64_t *in, uint64_t *out, uint32_t nlimbs, uint32_t logn, uint32_t galois,
                            hipStream_t stream);
hipError_t launch_lincomb(const LincombArgs &a, uint32_t nlimbs, hipStream_t stream);
hipError_t launch_scalar_lincomb(const ScalarLincombArgs &a, uint32_t nlimbs, hipStream_t stream);
// x: [ndiag][N] integer-valued doubles -> out: [ndiag][nlimbs][N] residues modulo primes 0..nlimbs-1
hipError_t launch_reduce_f64(const double *x, uint64_t *out, const Prime *primes, uint32_t ndiag, uint32_t nlimbs,
                             uint32_t logn, hipStream_t stream);
// out[l][N/2] = 1 on every limb l < nlimbs, zeros elsewhere (coefficient domain X^(N/2))
hipError_t launch_half_monomial(uint64_t *out, uint32_t nlimbs, uint32_t logn, hipStream_t stream);

}  // namespace ckks

// The opaque context of the C ABI.
struct ckks_ctx {
    int device = 0;
    uint32_t logn = 0, N = 0, nq = 0, np = 0, dnum = 0, alpha = 0;
    std::vector<uint64_t> primes;  // q_0..q_L, p_0..p_{K-1}
    void *dev_block = nullptr;     // one allocation holding every table
    ckks::Prime *d_primes = nullptr;
    ulonglong2 *d_tw_fwd = nullptr;     // [n][N]
    ulonglong2 *d_tw_inv = nullptr;     // [n][N]
    double *d_twd_fwd = nullptr;        // [n][N] same twiddles as doubles (primes below 2^50)
    double *d_twd_inv = nullptr;
    // base-conversion sets: digit sets indexed (j * alpha + size - 1), then the P set
    ulonglong2 *d_bc_hinv = nullptr;    // [nsets][kMaxDigitPrimes]
    uint64_t *d_bc_hmod = nullptr;      // [nsets][n_primes][kMaxDigitPrimes], split_const form for c < 2^50
    ulonglong2 *d_bc_ys = nullptr;      // [nsets][kMaxDigitPrimes]: N^-1 [(B/b_i)^-1]_{b_i}
    double *d_bc_ysd = nullptr;         // the same as doubles (primes below 2^50)
    ulonglong2 *d_pinv = nullptr;       // [n_primes] P^-1 mod q_i
    uint64_t *d_pmod = nullptr;         // [n_primes] P mod q_i (0 on the special primes)
    ulonglong2 *d_rs_inv = nullptr;     // [nq][nq]: (level l, prime i) -> q_l^-1 mod q_i
    uint64_t *d_rs_mod = nullptr;       // [nq][nq]: q_l mod q_i
    uint32_t nsets = 0;

    uint32_t set_index(uint32_t digit, uint32_t size) const { return digit * alpha + size - 1; }
    uint32_t pset_index() const { return dnum * alpha; }
};

struct ckks_key {
    const uint64_t *data;
    uint32_t galois;
    const ckks_ctx *ctx;
};

namespace ckks {

// HMult's operands a = (a0, a1), b = (b0, b1) at the level of the key switch.
struct TensorIn {
    const uint64_t *a0, *a1, *b0, *b1;
};

// Full key switch of phi_{g_in}(d) into out_t = KS_t + phi_{g_add}(add_t) (add_t
// may be null), workspace of CKKS_OP_KEYSWITCH size; tin: HMult's tensor folded
// in instead of d and add (N = 2^16).
hipError_t keyswitch_core(const ckks_ctx *c, const uint64_t *d, uint32_t g_in, uint32_t level, const uint64_t *key,
                          uint64_t *out0, uint64_t *out1, const uint64_t *add0, const uint64_t *add1, uint32_t g_add,
                          void *ws, hipStream_t st, const TensorIn *tin = nullptr);

// keyswitch_extended of a hoisted giant step whose sum with [P]_q phi_g(c0) (rows
// q_0..q_l of half 0) is accumulated into tot ([2][l+1+K][N], outside the
// workspace): tot = (first ? 0 : tot) + that, in the inner product's launch.
hipError_t keyswitch_extended_fold(ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *key,
                                   void *ws, hipStream_t st, const uint64_t *c0, uint64_t *tot, bool first);

// Key switch of phi_g(d) (d at `level`, eval domain) without the ModDown: the
// two accumulators [2][l+1+K][N] over q_0..q_l, p_0..p_{K-1} are left in the
// workspace (CKKS_OP_KEYSWITCH size) at *acc.
hipError_t keyswitch_extended(ckks_ctx *c, const uint64_t *d, uint32_t g, uint32_t level, const uint64_t *key,
                              void *ws, hipStream_t st, uint64_t **acc);
// ModDown of an extended pair x = [2][l+1+K][N] into out0, out1 at `level`
// (workspace of CKKS_OP_KEYSWITCH size; x must not lie in it).
hipError_t moddown_pair(ckks_ctx *c, const uint64_t *x, uint32_t level, uint64_t *out0, uint64_t *out1, void *ws,
                        hipStream_t st);

}  // namespace ckks
