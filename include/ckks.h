/*
 * ckks.h - C ABI of the MI355X (gfx950) RNS-CKKS key-switching library.
 *
 * The operations are the server-side CKKS primitives of the FIDESlib paper
 * (arXiv 2507.04775), Table I, and the steps of hybrid key switching they are
 * built from (Sec. II-A; Sec. III-F.3 to III-F.6).
 *
 * Conventions shared by every call
 * --------------------------------
 * - N = 2^log_n.  The ciphertext basis is q_0..q_L (n_q = L+1 primes), the
 *   special basis p_0..p_{K-1} (n_p = K primes).  Every prime is below 2^61
 *   and congruent to 1 mod 2N.
 * - A polynomial at level l has l+1 limbs q_0..q_l.  Limbs are u64 arrays of N
 *   canonical residues in [0, q), stored limb-major and contiguous:
 *   poly[i*N + k] is coefficient / evaluation k of limb i.  The evaluation
 *   domain holds A(psi^(2 br(k) + 1)) at position k (bit-reversed order), psi
 *   being the smallest primitive 2N-th root of unity modulo the limb's prime.
 * - "Extended" polynomials (ModUp output, inner-product accumulators, ModDown
 *   input) have l+1+K rows: q_0..q_l, then p_0..p_{K-1}.
 * - Key-switching keys are top-level keys laid out [dnum][2][n_q+n_p][N]
 *   (rows q_0..q_L, then p_0..p_{K-1}); at level l rows 0..l and the K special
 *   rows are read.  Digit j covers q_{j alpha}..q_{min((j+1) alpha, l+1)-1}
 *   with alpha = ceil(n_q / dnum).
 * - Every data pointer is a device pointer owned by the caller (the library
 *   never allocates per call).  Workspaces are caller-owned device buffers of
 *   at least ckks_workspace_bytes() bytes.  The context owns only its
 *   precomputed tables.
 * - Every call is asynchronous on the given HIP stream (a hipStream_t passed as
 *   void*; NULL is the default stream).  Arguments are validated on the host
 *   before anything is launched; on an error nothing is written and the call
 *   returns a negative status; ckks_last_error() gives the reason.  Device-side
 *   faults surface as CKKS_E_DEVICE from ckks_sync().
 * - Outputs must not overlap inputs unless a call says otherwise.
 * - A context may be used from several host threads on distinct streams with
 *   disjoint buffers and workspaces.
 */
#ifndef CKKS_H
#define CKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CKKS_OK = 0,
    CKKS_E_ARG = -1,         /* null pointer, bad size, misalignment, forbidden aliasing */
    CKKS_E_LEVEL = -2,       /* level out of range or operands at different levels */
    CKKS_E_KEY = -3,         /* wrong key kind or Galois element */
    CKKS_E_NOMEM = -4,       /* table allocation failed at context creation */
    CKKS_E_DEVICE = -5,      /* a HIP runtime call failed */
    CKKS_E_UNSUPPORTED = -6  /* parameter shape this build does not handle */
} ckks_status;

typedef struct ckks_ctx ckks_ctx;
typedef struct ckks_key ckks_key;

/* A ciphertext: two caller-owned device polynomials at `level`. */
typedef struct {
    uint64_t *c0;
    uint64_t *c1;
    uint32_t level;
    double scale; /* host-side metadata, carried but never read by kernels */
} ckks_ct;

/* Operation codes for ckks_workspace_bytes. */
enum {
    CKKS_OP_MODUP = 1,
    CKKS_OP_MODDOWN = 2,
    CKKS_OP_KEYSWITCH = 3,
    CKKS_OP_HMULT = 4,
    CKKS_OP_RESCALE = 5,
    CKKS_OP_ROTATE = 6,
    CKKS_OP_HOISTED = 7 /* per call, independent of the number of rotations */
};

/*
 * Context creation (Sec. III-E: precomputation at context creation).
 * q[0..n_q-1], p[0..n_p-1]: host arrays of the primes.  dnum: number of digits
 * of the hybrid key-switching decomposition (1 <= dnum <= n_q).  Builds, on the
 * host, the twiddle tables with their Shoup companions and the constants of the
 * base conversions, ModDown and Rescale, and uploads them to `hip_device`.
 * Supported: log_n in {12, 16}; n_q + n_p <= 64; every digit and the special
 * basis have at most 16 primes.  *out receives the context; free it with
 * ckks_ctx_destroy.  Synchronous.
 */
ckks_status ckks_ctx_create(uint32_t log_n, const uint64_t *q, uint32_t n_q, const uint64_t *p, uint32_t n_p,
                            uint32_t dnum, int hip_device, ckks_ctx **out);
void ckks_ctx_destroy(ckks_ctx *ctx);

/* Thread-local text of the last error, never NULL. */
const char *ckks_last_error(void);

/* Waits for the stream and reports any asynchronous device error. */
ckks_status ckks_sync(ckks_ctx *ctx, void *stream);

/* Workspace bytes needed by an operation at `level` (0 for an unknown op). */
size_t ckks_workspace_bytes(const ckks_ctx *ctx, uint32_t op, uint32_t level);

/* Copies one prime's forward twiddle table psi^br(k), k < N, into host memory
 * (for table checks); limb indexes q_0..q_L then p_0..p_{K-1}. Synchronous. */
ckks_status ckks_get_twiddles(const ckks_ctx *ctx, uint32_t limb, uint64_t *host_out);

/*
 * Negacyclic NTT / inverse NTT in place (Sec. III-F.4): radix-2 Cooley-Tukey
 * forward (natural coefficients to bit-reversed evaluations) and Gentleman-
 * Sande inverse (back, scaled by N^-1).  poly holds n_limbs limbs; limb i is
 * transformed under the prime with limb index limb0 + i (q_0..q_L are
 * 0..n_q-1, p_0..p_{K-1} are n_q..n_q+n_p-1).
 */
ckks_status ckks_ntt(ckks_ctx *ctx, uint64_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream);
ckks_status ckks_intt(ckks_ctx *ctx, uint64_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream);

/*
 * Launch shape of the NTT passes at N = 2^16 (Sec. III-F.4 runs the transform
 * as a column pass and a row pass over the 256 x 256 view): a workgroup takes
 * `tile` columns (rows) with 32 threads on each, tile 16 (512 threads), 8 (256)
 * or 4 (128).  Narrow tiles give a launch over few limbs more workgroups to
 * spread over the CUs.  Inverse launches also take tile code 2: 8 columns
 * (rows) with 64 threads on each, 4 elements per thread (512 threads), twice
 * the waves for latency-bound launches over few limbs; every inverse column
 * pass has this form, and the plain inverse row pass (the ModDown and Rescale
 * INTTs, ckks_intt); the gathered and tensor row passes then use tiles of 8.  The choice holds per direction (inverse 0 / 1) and per number of
 * limbs in the launch (1..128), for every NTT launch of every operation in the
 * process; tile 0 restores the default (16 from 24 limbs up, 8 from 6, else 4;
 * inverse launches of at most 8 limbs 2).  Results do not depend on it.  An
 * autotuner sets it from measurements.  ckks_ntt_tile_get returns the code in
 * effect (0 for bad arguments).  Persistent batch kernels always use 16.
 */
ckks_status ckks_ntt_tile_set(uint32_t inverse, uint32_t n_limbs, uint32_t tile);
uint32_t ckks_ntt_tile_get(uint32_t inverse, uint32_t n_limbs);

/*
 * ModUp of hybrid key switching (Sec. II-A, III-F.3, Eq. (1)):
 * d [l+1][N] (evaluation domain) -> ext [beta][l+1+K][N] (evaluation domain),
 * beta = ceil((l+1)/alpha).  Row r of ext[j] is d's row r for r in digit j;
 * every other row is NTT(Conv_{D_j -> row}(INTT(d)|D_j)) with the fast base
 * conversion y_i = [x_i (D_j/d_i)^-1]_{d_i}, out = [sum_i y_i [D_j/d_i]]_row.
 * ws: ckks_workspace_bytes(CKKS_OP_MODUP, l).
 */
ckks_status ckks_modup(ckks_ctx *ctx, const uint64_t *d, uint32_t level, uint64_t *ext, void *ws, void *stream);

/*
 * Key inner product (dot-product step of hybrid key switching, III-F.5):
 * acc[t][r] = sum_{j<beta} phi_g(ext_j)[r] * key[j][t][row r], t = 0, 1.
 * ext [beta][l+1+K][N], acc [2][l+1+K][N].  galois 1 is the plain product;
 * another odd g < 2N applies the automorphism X -> X^g to the digits first
 * (hoisted rotation, III-F.6).  The key's own Galois element is not checked.
 */
ckks_status ckks_inner_product(ckks_ctx *ctx, const uint64_t *ext, uint32_t level, const ckks_key *key,
                               uint32_t galois, uint64_t *acc, void *stream);

/*
 * ModDown (III-F.3, ModDown fusion of III-F.5): x [l+1+K][N] evaluation domain
 * -> out [l+1][N], out_i = [P^-1]_{q_i} (x_i - NTT(Conv_{P->q_i}(INTT(x|P)))).
 * Conv is the fast base conversion of Eq. (1) with centred inputs: with
 * a_k = INTT(x|P)_k and y_k = [a_k (P/p_k)^-1]_{p_k}, every y_k above
 * (p_k - 1)/2 enters the sum as y_k - p_k, so Conv(a) = sum_k y_k^ctr [P/p_k]_{q_i}
 * and, per coefficient, out = (X - v) / P exactly, with X the integer whose
 * residues are x and v = sum_k y_k^ctr (P/p_k), so v = X (mod P) and
 * |v| < K P / 2.  The error of the division then has zero mean.
 * ws: ckks_workspace_bytes(CKKS_OP_MODDOWN, l).
 */
ckks_status ckks_moddown(ckks_ctx *ctx, const uint64_t *x, uint32_t level, uint64_t *out, void *ws, void *stream);

/*
 * Wraps a caller-owned device key [dnum][2][n_q+n_p][N] (evaluation domain).
 * galois = 0 marks a relinearisation key (for s^2); an odd g < 2N marks the
 * key for the automorphism X -> X^g.  Nothing is copied: the buffer must stay
 * valid while the handle is used.  Release with ckks_key_release.
 */
ckks_status ckks_key_wrap(ckks_ctx *ctx, const uint64_t *dev_key, uint32_t galois, ckks_key **out);
void ckks_key_release(ckks_key *key);

/*
 * Hybrid key switching: (out0, out1) = ModDown(InnerProduct(ModUp(d), key))
 * for both key halves; d, out0, out1 are [l+1][N] evaluation domain.
 * ws: ckks_workspace_bytes(CKKS_OP_KEYSWITCH, l).
 */
ckks_status ckks_keyswitch(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key, uint64_t *out0,
                           uint64_t *out1, void *ws, void *stream);

/*
 * Key switching for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, kernels and output as ckks_keyswitch, with the workspace
 * taken from a static device array of ckks_noalloc_scratch_bytes() bytes
 * (160 MiB: every level of N = 2^16 with 31 ciphertext limbs and up to ten
 * special primes) that the library holds on each GPU it runs on until the
 * process ends.  The call allocates nothing.  A level whose workspace
 * (ckks_workspace_bytes(CKKS_OP_KEYSWITCH, l)) exceeds the scratch returns
 * CKKS_E_ARG.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap in time on one GPU (different streams or host threads without
 * ordering between them) race and give undefined results; calls ordered on
 * one stream are safe.  The scratch needs no initial contents.
 */
ckks_status ckks_keyswitch_noalloc(ckks_ctx *ctx, const uint64_t *d, uint32_t level, const ckks_key *key,
                                   uint64_t *out0, uint64_t *out1, void *stream);
size_t ckks_noalloc_scratch_bytes(void);

/*
 * HMult with relinearisation (Table I): d0 = a0 b0, d1 = a0 b1 + a1 b0,
 * d2 = a1 b1, (k0, k1) = KeySwitch(d2, rlk), out = (d0 + k0, d1 + k1).
 * a, b at the same level (else CKKS_E_LEVEL); rlk must have galois 0
 * (else CKKS_E_KEY).  No rescale; out->level = level, out->scale = a.scale *
 * b.scale.  out may not alias a or b.  ws: CKKS_OP_HMULT.  At N = 2^16 the
 * tensor is folded into the key switch (d2 formed as it is loaded by ModUp's
 * inverse NTT and by the inner product, [P]_q d0 and [P]_q d1 added to the
 * inner product's sums over q_0..q_l), so no d is stored; the result is the
 * same residues.
 */
ckks_status ckks_hmult_relin(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, const ckks_key *rlk, ckks_ct *out,
                             void *ws, void *stream);

/*
 * Rescale (Table I; rescale fusion of III-F.5): for each half c at level l >= 1,
 * v = INTT_{q_l}(c_l) lifted centred into q_i, out_i =
 * [q_l^-1]_{q_i} (c_i - NTT_{q_i}(v)), i < l.  out->level = l - 1,
 * out->scale = in->scale / q_l.  out may be the same buffers as in (in place);
 * any other overlap is an error.  ws: CKKS_OP_RESCALE.
 */
ckks_status ckks_rescale(ckks_ctx *ctx, const ckks_ct *in, ckks_ct *out, void *ws, void *stream);

/*
 * Automorphism plus key switch (HRotate and Conjugate, Table I):
 * out = (phi_g(c0) + k0, k1) with (k0, k1) = KeySwitch(phi_g(c1), key_g).
 * g odd, 1 < g < 2N; the key's galois must equal g (else CKKS_E_KEY).
 * ws: CKKS_OP_ROTATE.
 */
ckks_status ckks_apply_galois(ckks_ctx *ctx, const ckks_ct *in, uint32_t galois, const ckks_key *key, ckks_ct *out,
                              void *ws, void *stream);

/* HRotate by k slots to the left: g = 5^k mod 2N (negative k allowed). */
ckks_status ckks_hrotate(ckks_ctx *ctx, const ckks_ct *in, int32_t k, const ckks_key *key, ckks_ct *out, void *ws,
                         void *stream);

/* Conjugate: g = 2N - 1. */
ckks_status ckks_conjugate(ckks_ctx *ctx, const ckks_ct *in, const ckks_key *key, ckks_ct *out, void *ws,
                           void *stream);

/*
 * Hoisted rotations (III-F.6): one ModUp of in->c1 is shared by n rotations;
 * for each i: acc = sum_j phi_g(ext_j) * key_i, (k0, k1) = ModDown(acc),
 * out[i] = (phi_g(c0) + k0, k1) with g = 5^k[i] mod 2N.  keys[i] must carry
 * that g.  ws: CKKS_OP_HOISTED (independent of n).
 */
ckks_status ckks_hrotate_hoisted(ckks_ctx *ctx, const ckks_ct *in, uint32_t n, const int32_t *k,
                                 const ckks_key *const *keys, ckks_ct *out, void *ws, void *stream);

/*
 * Limb-wise support operations of Table I on evaluation-domain data; all
 * operands at `level` (l+1 limbs), out may alias an input exactly.  Row i
 * uses the i-th prime of q_0..q_L, p_0..p_{K-1}, so l may reach n_q+n_p-1
 * for extended polynomials (key generation); CKKS_E_LEVEL beyond that.
 *   ckks_poly_add/sub/mul : out = a (+,-,*) b              (HAdd, PtAdd, PtMult per polynomial)
 *   ckks_poly_mul_add     : out = a * b + c                (PtMulAdd per polynomial)
 *   ckks_poly_scalar_mul  : out = a * s[i] on limb i       (ScalarMult; s: host array [l+1], s[i] < q_i)
 *   ckks_poly_scalar_add  : out = a + s[i] on limb i       (ScalarAdd on c0; s[i] < q_i)
 */
ckks_status ckks_poly_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t level,
                          void *stream);
ckks_status ckks_poly_sub(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t level,
                          void *stream);
ckks_status ckks_poly_mul(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t level,
                          void *stream);
ckks_status ckks_poly_mul_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *b, const uint64_t *c, uint64_t *out,
                              uint32_t level, void *stream);
ckks_status ckks_poly_scalar_mul(ckks_ctx *ctx, const uint64_t *a, const uint64_t *s, uint64_t *out, uint32_t level,
                                 void *stream);
ckks_status ckks_poly_scalar_add(ckks_ctx *ctx, const uint64_t *a, const uint64_t *s, uint64_t *out, uint32_t level,
                                 void *stream);

/*
 * Ciphertext-level support operations of Table I (ScalarAdd, PtAdd, HAdd,
 * ScalarMult, PtMult), each one launch over both halves at the level of a:
 *   ckks_hadd        : out = (a0 + b0, a1 + b1)        out->scale = a->scale
 *   ckks_ptadd       : out = (a0 + pt, a1)             out->scale = a->scale
 *   ckks_ptmult      : out = (a0 pt, a1 pt)            out->scale = a->scale * pt_scale
 *   ckks_scalar_add  : out = (a0 + s, a1)              out->scale = a->scale
 *   ckks_scalar_mult : out = (a0 s, a1 s)              out->scale = a->scale * s_scale
 * b must be at a's level (else CKKS_E_LEVEL).  pt: device [l+1][N] in the
 * evaluation domain (rows q_0..q_l of an encoded plaintext; the caller keeps
 * its scale).  s: host array [l+1], s[i] < q_i, an integer constant in RNS
 * form (else CKKS_E_ARG).  Scales are host metadata: adding operands of
 * different scales is the caller's error, not detected.  out is either the
 * same buffers as a (or b) or disjoint from them and from pt (else
 * CKKS_E_ARG); out->level = a->level.  No workspace.
 */
ckks_status ckks_hadd(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, void *stream);
ckks_status ckks_ptadd(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *pt, ckks_ct *out, void *stream);
ckks_status ckks_ptmult(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *pt, double pt_scale, ckks_ct *out,
                        void *stream);
ckks_status ckks_scalar_add(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *s, ckks_ct *out, void *stream);
ckks_status ckks_scalar_mult(ckks_ctx *ctx, const ckks_ct *a, const uint64_t *s, double s_scale, ckks_ct *out,
                             void *stream);

/*
 * HSquare: HMult of a ciphertext with itself (d0 = a0^2, d1 = 2 a0 a1,
 * d2 = a1^2), relinearised; the contract of ckks_hmult_relin with b = a.
 * ws: CKKS_OP_HMULT.
 */
ckks_status ckks_hsquare(ckks_ctx *ctx, const ckks_ct *a, const ckks_key *rlk, ckks_ct *out, void *ws, void *stream);

/* Eval-domain automorphism alone: out[k] = in[br(((2 br(k)+1) g mod 2N - 1)/2)] on n_limbs limbs. */
ckks_status ckks_automorph(ckks_ctx *ctx, const uint64_t *in, uint32_t galois, uint64_t *out, uint32_t n_limbs,
                           void *stream);

/*
 * Batched key switching (limb batching, Sec. III-F.1).  A batch is a list of
 * independent work items at any levels:
 *   CKKS_WORK_HMULT_RELIN : out[0] = HMult+relin(a, b) with key (galois 0)
 *   CKKS_WORK_KEYSWITCH   : (out[0].c0, out[0].c1) = KeySwitch(a.c0 at a.level, key)
 *   CKKS_WORK_ROTATE      : out[0] = apply_galois(a, galois, key)
 *   CKKS_WORK_HOISTED     : out[i] = HRotate(a, rot[i], rot_keys[i]) for i < n_rot, one ModUp
 * Each item's result is bit-identical to the corresponding single-operation
 * call.  ckks_batch_create validates every item, binds the caller-owned
 * workspace `ws` (ckks_batch_workspace_bytes bytes, 256-byte aligned, kept
 * for the batch's life) and uploads the batch's launch tables into its tail:
 * a batch allocates no device memory.  ckks_batch_run executes every step of every item as
 * one persistent work-queue launch per step on `stream`; ckks_batch_capture
 * records that launch sequence into a HIP graph that ckks_batch_replay
 * relaunches (a non-default stream is required to capture).  ckks_batch_tune
 * runs the batch with each persistent grid size of {1, 2, 3, 4, 6, 8}
 * workgroups per CU, once to warm up and five times measured, and keeps per
 * step the size with the smallest median time (it runs the batch, overwriting
 * the outputs with the same values).
 * Items must not share outputs, and no output may overlap another item's
 * input or workspace; inputs and keys must stay valid while the batch is used.
 */
enum {
    CKKS_WORK_HMULT_RELIN = 1,
    CKKS_WORK_KEYSWITCH = 2,
    CKKS_WORK_ROTATE = 3,
    CKKS_WORK_HOISTED = 4
};

typedef struct {
    uint32_t kind;
    ckks_ct a;                       /* input ciphertext (KEYSWITCH: a.c0 is the polynomial) */
    ckks_ct b;                       /* second HMult operand */
    const ckks_key *key;             /* HMULT / KEYSWITCH / ROTATE key */
    uint32_t galois;                 /* ROTATE: Galois element (the key's) */
    uint32_t n_rot;                  /* HOISTED: number of rotations */
    const int32_t *rot;              /* HOISTED: slot rotations (host array) */
    const ckks_key *const *rot_keys; /* HOISTED: one key per rotation (host array) */
    ckks_ct *out;                    /* outputs (n_rot for HOISTED, else 1); levels are set */
} ckks_work;

typedef struct ckks_batch ckks_batch;

size_t ckks_batch_workspace_bytes(const ckks_ctx *ctx, const ckks_work *items, uint32_t n);
ckks_status ckks_batch_create(ckks_ctx *ctx, const ckks_work *items, uint32_t n, void *ws, ckks_batch **out);
ckks_status ckks_batch_run(ckks_batch *batch, void *stream);
ckks_status ckks_batch_tune(ckks_batch *batch, void *stream);
ckks_status ckks_batch_capture(ckks_batch *batch, void *stream);
ckks_status ckks_batch_replay(ckks_batch *batch, void *stream);
uint32_t ckks_batch_keyswitches(const ckks_batch *batch); /* key switches performed per run */
uint32_t ckks_batch_grid(const ckks_batch *batch, uint32_t step); /* persistent grid, in workgroups per CU */
/* Sets one step's persistent grid (1..16 workgroups per CU), e.g. from a tuning
 * cache; steps are numbered 0..ckks_batch_steps()-1. */
ckks_status ckks_batch_set_grid(ckks_batch *batch, uint32_t step, uint32_t wg_per_cu);
uint32_t ckks_batch_steps(void);
/*
 * Schedule of ckks_batch_run / ckks_batch_capture (limb batching of
 * Sec. III-F.1 carried to whole key switches).  window = 0: one persistent
 * launch per step (the default above).  window >= 1 (N = 2^16 only): the
 * whole batch in ONE persistent launch of wg_per_cu (1 or 2) workgroups per
 * CU.  Every step of every key switch (ModUp's inverse NTT, conversion and
 * NTT, the inner product, ModDown's inverse NTT and NTT, HMult's tensor) is a
 * group of units; a unit starts once the previous step of its own key switch
 * is done, through per-group counters in device memory, so the steps of
 * different items overlap.  Items are taken in windows of `window` consecutive
 * items and window w runs step s in slot w + s (a software pipeline over the
 * batch); window >= n items is the step-by-step order without barriers.
 * Results are bit-identical to every other schedule.  A change of window
 * waits for the device, then writes the unit list into the workspace's tail.
 * A change of schedule drops a captured graph (ckks_batch_replay then fails
 * until the next ckks_batch_capture).
 * A waiting workgroup gives up after a bounded number of polls, so a launch
 * always ends; ckks_batch_faults then reports CKKS_E_DEVICE.
 */
ckks_status ckks_batch_set_schedule(ckks_batch *batch, uint32_t window, uint32_t wg_per_cu);
uint32_t ckks_batch_schedule(const ckks_batch *batch); /* the window, 0 for per-step launches */
/* Waits for `stream`; CKKS_E_DEVICE if a one-launch run gave up waiting (its outputs are then invalid). */
ckks_status ckks_batch_faults(ckks_batch *batch, void *stream);
void ckks_batch_destroy(ckks_batch *batch);

/*
 * Bootstrapping (Sec. III-F.7): ModRaise, CoeffToSlot, EvalMod, SlotToCoeff
 * for a fully packed ciphertext (N/2 slots).
 *
 * Schedule, derived by the library from the descriptor:
 * - Input gain: with input_gain G > 1 the level-0 input is first multiplied by
 *   the integer G (exact, no rescale), so that the message uses more of q_0
 *   while its share of the EvalMod argument stays small; the caller's
 *   SlotToCoeff constants carry 1/G.
 * - ModRaise: the level-0 input's coefficients are lifted centred from q_0 to
 *   q_0..q_L (L = n_q - 1) and returned to the evaluation domain.  With
 *   sparse-secret encapsulation (to_sparse and from_sparse set), the input is
 *   first key-switched at level 0 with to_sparse (s -> a sparse s'), and the
 *   raised ciphertext is key-switched back at level L with from_sparse.
 * - CoeffToSlot: the inverse special-FFT stages (butterflies pairing slots x
 *   and x + h, half-sizes n/2 down to 1, n = N/2) are merged into groups of
 *   cts_radix_logs[g] stages in that order; SlotToCoeff merges the forward
 *   stages (half-sizes 1 up to n/2) into groups of stc_radix_logs[g].  A
 *   group of r stages with smallest half-size h0 has R = 2^r and diagonals at
 *   slot offsets m h0 for m in [m_lo, m_lo + count): m_lo = 0, count = R when
 *   R h0 = n, else m_lo = -(R-1), count = 2R-1.  Diagonal i = g B + b (B the
 *   smallest power of two with B^2 >= count) is applied as
 *   sum_g rot(sum_b pt_i * rot(ct, b h0), G_g), G_g = (g B + m_lo) h0, with
 *   the baby rotations b = 1..B-1 hoisted.  Each group ends with a rescale;
 *   the first CoeffToSlot group rescales twice.
 * - Between them: ct_re = ct + conj(ct), ct_im = (conj(ct) - ct) X^(N/2);
 *   each goes through EvalMod; then ct = ct_re + ct_im X^(N/2).
 * - EvalMod: the babies T_1..T_min(b,d) (d = cheb_degree, b = cheb_baby)
 *   from T_1 = y, T_2m = 2 T_m^2 - 1, T_2m+1 = 2 T_m T_m+1 - T_1, the giants
 *   T_2b, T_4b, .. up to d by squaring.  A series of degree D >= b is split
 *   at the largest giant G <= D as q T_G + r (q_0 = c_G, q_i = 2 c_(G+i),
 *   r_(G-i) = c_(G-i) - c_(G+i), double arithmetic), r evaluated first, then
 *   q (a constant q_0 is multiplied in as a real constant); q T_G and r are
 *   brought to the lower of their levels and added.  Below degree b a leaf is
 *   sum_k round(c_k (D_t q_(t+1)) / D_level(T_k)) T_k on the limbs 0..t+1,
 *   rescaled once, plus c_0, with t one below the lowest of T_1..T_(b-1).
 *   Then double_angles steps y <- 2 y^2 - 1.
 *
 * Scales: level L has top_scale, level l-1 has (D_l * D_l) / q_l (double
 * arithmetic).  Taking a level-l ciphertext times a real c to level t < l
 * drops its limbs above t+1, multiplies by round(c (D_t q_(t+1)) / D_l) and
 * rescales; a constant c added at level l is round(c D_l); rounding is half
 * away from zero.  Multiplications are HMult+relin followed by a rescale.
 *
 * Descriptor: cts_diags[g] / stc_diags[g] point to count_g host vectors of N
 * integer-valued doubles (the plaintext coefficients of group g's diagonals,
 * already multiplied by their scale, in index order i); cheb[0..d] are the
 * Chebyshev coefficients; relin (galois 0), conj (galois 2N-1) and one key
 * per slot rotation of the schedule (rot_steps[i] taken mod N/2, key galois
 * 5^rot_steps[i] mod 2N) must stay valid while the handle lives.
 *
 * ckks_boot_create validates the descriptor (CKKS_E_KEY when a rotation of
 * the schedule has no key, CKKS_E_UNSUPPORTED when a group needs more than
 * 16 baby steps or the levels run out), uploads and transforms the plaintexts
 * and lays out its buffers in one block of device memory: the caller's
 * device_buffer, or one allocation of its own, freed by ckks_boot_destroy.  ckks_bootstrap runs the whole pipeline on `stream`:
 * in->level must be 0, out receives level ckks_boot_output_level() (out's
 * buffers hold that many limbs + 1) and scale D_out.  Calls on one handle
 * must not overlap in time (they share its buffers).  ckks_boot_capture
 * records the launch sequence for (in, out) into a HIP graph on a
 * non-default stream; ckks_boot_replay relaunches it (same in and out).
 */
typedef struct ckks_boot ckks_boot;

typedef struct {
    uint32_t n_cts, n_stc;               /* numbers of CoeffToSlot / SlotToCoeff groups */
    const uint32_t *cts_radix_logs;      /* stages per group, application order */
    const uint32_t *stc_radix_logs;
    const double *const *cts_diags;      /* [n_cts] host pointers to [count_g][N] doubles */
    const double *const *stc_diags;
    uint32_t cheb_degree;
    const double *cheb;                  /* cheb_degree + 1 coefficients */
    uint32_t cheb_baby;                  /* baby-step size, a power of two >= 2; 0: smallest b with b^2 > d */
    uint32_t double_angles;
    double top_scale;                    /* scale of level L */
    const ckks_key *relin, *conj;
    const ckks_key *to_sparse, *from_sparse;  /* both null, or switching keys s -> s' and s' -> s */
    uint32_t n_rot;
    const int32_t *rot_steps;
    const ckks_key *const *rot_keys;
    uint32_t hoist_moddown;              /* 1: giant steps key-switched without ModDown, summed over Q u P,
                                            one ModDown per group (fewer roundings, less time); 0: the plain
                                            schedule, one ModDown per rotation as in the paper */
    uint64_t input_gain;                 /* 0 or 1: none; else the level-0 input is multiplied by this integer
                                            (below q_0) before ModRaise, so the message fills more of q_0; the
                                            caller folds 1/input_gain into the SlotToCoeff constants */
    void *device_buffer;                 /* null: the handle allocates its device memory itself; else a
                                            caller-owned device buffer, 256-byte aligned, of at least
                                            ckks_boot_bytes() bytes, valid (and not touched by the caller)
                                            while the handle lives; the handle then allocates nothing */
    size_t device_buffer_bytes;
} ckks_boot_desc;

ckks_status ckks_boot_create(ckks_ctx *ctx, const ckks_boot_desc *desc, ckks_boot **out);
/* Device bytes the handle of `desc` needs (plaintexts, buffers, workspaces): the size of a
 * caller-owned device_buffer.  Validates the descriptor as ckks_boot_create does, on the host only. */
ckks_status ckks_boot_bytes(ckks_ctx *ctx, const ckks_boot_desc *desc, size_t *bytes);
uint32_t ckks_boot_output_level(const ckks_boot *boot);
uint32_t ckks_boot_keyswitches(const ckks_boot *boot);  /* key switches per bootstrap */
size_t ckks_boot_device_bytes(const ckks_boot *boot);   /* plaintexts, buffers and workspace */
ckks_status ckks_bootstrap(ckks_boot *boot, const ckks_ct *in, ckks_ct *out, void *stream);
ckks_status ckks_boot_capture(ckks_boot *boot, const ckks_ct *in, ckks_ct *out, void *stream);
ckks_status ckks_boot_replay(ckks_boot *boot, void *stream);
void ckks_boot_destroy(ckks_boot *boot);

/*
 * 32-bit word limbs (Sec. III-C: the limb type is templated on the word size;
 * the paper verifies only 64-bit words).  The key-switching path with every
 * residue in a uint32_t: N = 2^16 (log_n must be 16), every prime below 2^30
 * and congruent to 1 mod 2N, polynomials limb-major [limbs][N] u32 in the
 * layouts of the 64-bit calls (evaluation domain in bit-reversed order,
 * psi the smallest primitive 2N-th root; extended rows q_0..q_l, p_0..p_{K-1};
 * keys [dnum][2][n_q+n_p][N] u32, passed as device pointers; digits as above).
 * Every result equals the 64-bit definition of the same operation on the same
 * primes.  A twiddle product is a 32-bit Shoup multiplication, butterflies
 * are Harvey's lazy forms (below 4q < 2^32), and sums of products are exact
 * 64-bit sums reduced once (Barrett).  Pointers: device, 16-byte aligned.
 * Workspaces: ckks32_workspace_bytes(op, l) with op CKKS_OP_KEYSWITCH (also
 * ModUp and ModDown), CKKS_OP_HMULT, CKKS_OP_ROTATE, CKKS_OP_RESCALE.  All
 * calls are asynchronous on `stream`; errors as for the 64-bit calls.
 *   ckks32_ntt / ckks32_intt: in place on limbs limb0 .. limb0+n_limbs-1 (at most 64).
 *   ckks32_modup:   d [l+1] -> ext [beta][l+1+K] (each digit's own rows copied from d).
 *   ckks32_moddown: x [2][l+1+K] -> out_t = P^-1 (x_t - Conv(x_t|P)) [l+1], with the
 *                   centred conversion of ckks_moddown.
 *   ckks32_keyswitch: (out0, out1) = ModDown(InnerProduct(ModUp(d), key)).
 *   ckks32_hmult_relin: (a0 b0, a0 b1 + a1 b0) + KeySwitch(a1 b1, rlk); out may not alias inputs.
 *   ckks32_apply_galois: (phi_g(c0), 0) + KeySwitch(phi_g(c1), key of g).
 *   ckks32_rescale: out_t = q_l^-1 (c_t - NTT(SwitchModulo(INTT_{q_l}(c_t[l])))) at level l-1;
 *                   out may equal c (in place).
 */
typedef struct ckks32_ctx ckks32_ctx;
ckks_status ckks32_ctx_create(uint32_t log_n, const uint32_t *q, uint32_t n_q, const uint32_t *p, uint32_t n_p,
                              uint32_t dnum, int hip_device, ckks32_ctx **out);
void ckks32_ctx_destroy(ckks32_ctx *ctx);
size_t ckks32_workspace_bytes(const ckks32_ctx *ctx, uint32_t op, uint32_t level);
ckks_status ckks32_ntt(ckks32_ctx *ctx, uint32_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream);
ckks_status ckks32_intt(ckks32_ctx *ctx, uint32_t *poly, uint32_t limb0, uint32_t n_limbs, void *stream);
ckks_status ckks32_modup(ckks32_ctx *ctx, const uint32_t *d, uint32_t level, uint32_t *ext, void *ws, void *stream);
ckks_status ckks32_moddown(ckks32_ctx *ctx, const uint32_t *x, uint32_t level, uint32_t *out0, uint32_t *out1,
                           void *ws, void *stream);
ckks_status ckks32_keyswitch(ckks32_ctx *ctx, const uint32_t *d, uint32_t level, const uint32_t *key, uint32_t *out0,
                             uint32_t *out1, void *ws, void *stream);
ckks_status ckks32_hmult_relin(ckks32_ctx *ctx, const uint32_t *a0, const uint32_t *a1, const uint32_t *b0,
                               const uint32_t *b1, uint32_t level, const uint32_t *rlk, uint32_t *out0, uint32_t *out1,
                               void *ws, void *stream);
ckks_status ckks32_apply_galois(ckks32_ctx *ctx, const uint32_t *c0, const uint32_t *c1, uint32_t level,
                                uint32_t galois, const uint32_t *key, uint32_t *out0, uint32_t *out1, void *ws,
                                void *stream);
ckks_status ckks32_rescale(ckks32_ctx *ctx, const uint32_t *c0, const uint32_t *c1, uint32_t level, uint32_t *out0,
                           uint32_t *out1, void *ws, void *stream);

/*
 * Measurement probe (no CKKS operation): one launch of `blocks` workgroups of
 * 256 threads, each thread running 8 independent chains of `iters` dependent
 * 32x32->64 multiply-adds (v_mad_u64_u32), the instruction every 64-bit
 * modular product of the kernels is built from.  *mads_per_launch receives the
 * number of multiply-adds per lane of the launch (blocks * 256 * iters * 8);
 * timing the launch gives the chip's integer multiply-add rate, the ceiling
 * the integer-VALU fractions of the key-switching kernels are reported against.
 * out: device buffer of blocks * 256 words (each thread writes one sum).
 */
ckks_status ckks_probe_mad64(uint64_t *out, uint32_t blocks, uint32_t iters, void *stream,
                             uint64_t *mads_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* CKKS_H */
