/*
 * yastn.h -- C ABI of the MI355X block-sparse tensordot library.
 *
 * The library contracts two abelian-symmetric (Z_m, U(1) and their direct
 * products) block-sparse tensors, the operation described in Sec. II.B
 * ("Fusion and contractions") of Rams, Wojtowicz, Sinha, Hasik, "YASTN: Yet
 * another symmetric tensor networks" (arXiv:2405.12196):
 *
 *     C_{{i}{j}} = sum_{{x}} A_{{i} u {x}} B_{{j} u {x}}
 *
 * computed as: match A's and B's blocks on the charges of the contracted legs,
 * group the matches by the fused contracted charge X (one dense sector GEMM
 * C_IJ = sum_X A_IX B_XJ per X), and write the result straight into C's
 * blocks.  Tensors follow Sec. II.A: a leg is V(s, t, D) (signature s = +-1,
 * charge sectors t, sector dims D); a block is named by a tuple of charges,
 * one per leg, and a stored block obeys the block form of charge conservation
 * sum_i s_i rho_i = n; all blocks of a tensor live in ONE 1D buffer (lazy
 * storage), each block dense in C (row-major) order.
 *
 * Conventions
 *   - Every call returns yastn_status; nothing throws across the ABI.  On an
 *     error, yastn_last_error() returns a thread-local message.
 *   - Host pointers are marked [host], device pointers [device].  Every
 *     descriptor array is read during the call and copied; the caller keeps
 *     ownership of everything it passes in.
 *   - Device buffers (tensor data, workspace) are owned by the caller.
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream).
 */
#ifndef YASTN_H
#define YASTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YASTN_ABI_VERSION 1
#define YASTN_MAX_RANK 8   /* legs per tensor                                  */
#define YASTN_MAX_NSYM 4   /* charge components (e.g. U(1)xU(1) has nsym = 2)  */

typedef enum {
  YASTN_OK = 0,
  YASTN_ERR_ARG = 1,        /* null pointer, rank/nsym out of range, axes out of range or repeated,
                               axes of unequal length, signature not +-1, negative or overlapping
                               block offsets, unsupported option                                */
  YASTN_ERR_SYM = 2,        /* sym_mod differs between A and B, or an entry is 1 or negative    */
  YASTN_ERR_CHARGE = 3,     /* a block violates sum_i s_i rho_i = n (Sec. II.A)                  */
  YASTN_ERR_SIGNATURE = 4,  /* a contracted leg pair has equal signatures (a leg contracts only
                               with its dual, Sec. II.A footnote on conjugation)                 */
  YASTN_ERR_SHAPE = 5,      /* a dim < 1, one charge with two dims on a leg, or a contracted
                               charge with different dims in A and B                             */
  YASTN_ERR_DUPLICATE = 6,  /* a charge tuple occurs twice in one tensor                         */
  YASTN_ERR_NOMEM = 7,      /* host or device allocation failed                                  */
  YASTN_ERR_HIP = 8,        /* a HIP runtime call failed (no device, launch failure, ...)        */
  YASTN_ERR_STATE = 9       /* call not valid for this plan (e.g. buffer too small, job mix)     */
} yastn_status;

/* Arithmetic of the sector GEMMs.  F64: FP64 MFMA.  F32: FP32 MFMA.  BF16X3 /
 * BF16X6: each FP32 operand split into bf16 terms hi + mid (+ lo), products
 * hi*hi + hi*mid + mid*hi (X3; + mid*mid + hi*lo + lo*hi for X6) on bf16 MFMA;
 * all reduced precisions accumulate in FP32. */
typedef enum { YASTN_F64 = 0, YASTN_F32 = 1, YASTN_BF16X3 = 2, YASTN_BF16X6 = 3 } yastn_precision;

/* Element type of a stored tensor buffer.  C128: complex, (re, im) FP64
 * pairs, interleaved (yastn_zplan_*, yastn_swap_gate only). */
typedef enum { YASTN_DTYPE_F64 = 0, YASTN_DTYPE_F32 = 1, YASTN_DTYPE_C128 = 2 } yastn_dtype;

/* One block-sparse tensor (Sec. II.A).  All arrays [host]. */
typedef struct {
  int32_t rank;              /* number of legs, 0..YASTN_MAX_RANK                               */
  int32_t nsym;              /* charge components, 1..YASTN_MAX_NSYM                            */
  const int32_t *sym_mod;    /* [nsym] 0 = U(1) (charges in Z); m >= 2 = Z_m (reduced mod m)    */
  const int8_t *sig;         /* [rank] leg signatures, +1 or -1                                 */
  const int32_t *n;          /* [nsym] total charge n                                           */
  int64_t nblocks;           /* stored blocks (may be 0)                                        */
  const int32_t *charges;    /* [nblocks][rank][nsym] charge of each block on each leg          */
  const int64_t *shapes;     /* [nblocks][rank] block dims, each >= 1                           */
  const int64_t *offsets;    /* [nblocks] first element of each block in the 1D buffer; blocks
                                must not overlap; any order                                     */
} yastn_tensor_desc;

/* One tensordot: C = tensordot(A, B, axes=(axes_a, axes_b)) (the paper's
 * tensordot listing).  C's legs are A's uncontracted legs in order, then B's. */
typedef struct {
  yastn_tensor_desc a, b;
  int32_t ncontract;         /* number of contracted leg pairs                                  */
  const int32_t *axes_a;     /* [ncontract] [host] legs of A                                    */
  const int32_t *axes_b;     /* [ncontract] [host] matching legs of B                           */
} yastn_problem;

typedef struct {
  yastn_precision precision; /* arithmetic of the sector GEMMs                                  */
  yastn_dtype in_dtype;      /* element type of A and B buffers                                 */
  yastn_dtype out_dtype;     /* element type of C buffers                                       */
  int32_t tile_rows;         /* rows of C_X per wave tile: 16, 32, 64, 128, 256 or 512;
                                0 = plan's choice (tall tiles while the launch keeps enough tiles) */
  int32_t flags;             /* 0, or one of the YASTN_FLAG_* below                             */
} yastn_options;

/* Kernel family of the sector GEMMs when no variant is set.  By default the
 * plan runs MFMA tiles with register-resident B (every sector K <= 64) or MFMA
 * tiles over a packed B (otherwise).  FLAG_MFMA forces the packed-B MFMA
 * tiles; FLAG_ROWS asks for one output row per lane on the vector FMA units
 * (used when every sector has K, N <= 64; BF16 precisions always use MFMA). */
#define YASTN_FLAG_MFMA 1
#define YASTN_FLAG_ROWS 2
/* Plans are kept in a structure cache by default (see yastn_plan);
 * FLAG_NOCACHE (may be or-ed with the flags above) plans afresh and keeps
 * nothing. */
#define YASTN_FLAG_NOCACHE 4

typedef struct {
  int64_t blocks_a, blocks_b;  /* stored blocks of A and B                                      */
  int64_t pairs;               /* matched (A block, B block) pairs                              */
  int64_t sectors;             /* distinct fused contracted charges X with >= 1 pair            */
  int64_t c_blocks;            /* blocks of C                                                   */
  int64_t c_numel;             /* elements of C (contiguous, rule: ascending charge order)      */
  int64_t numel_a, numel_b;    /* stored elements of A and B                                    */
  int64_t max_m, max_k, max_n; /* largest fused sector matrix dims                              */
  int64_t tiles;               /* wave tiles of the grouped GEMM for this problem               */
  double useful_flops;         /* sum over matched pairs of 2*m*k*n                             */
  double mfma_flops;           /* flops the MFMA tiles execute (padding included)               */
  double alg_bytes;            /* (numel_a + numel_b) * in bytes + c_numel * out bytes          */
} yastn_stats;

typedef struct yastn_plan_s *yastn_plan_t;

/* Build a plan for nprob independent problems that will run in one grouped
 * launch.  Validates every descriptor on the host (all error classes above),
 * then matches blocks with the charge-hash join kernel on the device (the
 * plan's device tables are allocated here), reads the matches back, and
 * derives C's structure: blocks (a_free, b_free) reached by at least one
 * matched pair, in ascending lexicographic order of the (normalised) charge
 * tuple, stored contiguously; n_C = n_A + n_B.  A contracted charge present
 * in only one operand contributes nothing (Sec. II.B footnote).
 * Synchronises hip_stream once.  opts may be NULL (F64, F64 in/out, auto). */
yastn_status yastn_plan(const yastn_problem *probs, int32_t nprob, const yastn_options *opts,
                        void *hip_stream, yastn_plan_t *out);

/* Structure cache: CTM runs contract tensors of one block structure in
 * every iteration (Sec. III), so yastn_plan keeps each plan it builds under
 * the exact description of the request (device, options, every descriptor
 * array, compared in full) and answers a later identical request with a new
 * handle to the same plan (up to 64 structures, least recently used
 * dropped).  Handles of one structure share the plan, including its tuned
 * kernel variant; its device tables are released when the last handle is
 * freed and the cache has dropped it (yastn_plan_cache_clear drops every
 * entry).  yastn_plan_profile: the wall time of the plan's construction in
 * ms, ms[0] validation, ms[1] the charge-hash join (device), ms[2] the host
 * tables, ms[3] the upload ([host] array of 4, may be NULL); *cached = 1 if
 * this handle came from the cache. */
yastn_status yastn_plan_profile(yastn_plan_t plan, double *ms, int32_t *cached);
void yastn_plan_cache_clear(void);

/* Tuning store: every choice yastn_plan_autotune makes is kept for the
 * process under a 128-bit fingerprint of the plan request (options, axes and
 * every descriptor array; not the device ordinal) and the device's
 * architecture name (hipDeviceProp_t::gcnArchName).  A new plan whose request
 * and architecture are in the store starts at that variant when it fits the
 * plan, with the stored times (yastn_plan_autotune then returns at once).
 * yastn_tune_save writes the store to a JSON file (path [host]); a later
 * process reads it with yastn_tune_load (*loaded = entries read, may be
 * NULL), so the structures a CTM run repeats are tuned once across runs.
 * The file names the variant count; a file made for another count is
 * rejected with YASTN_ERR_ARG, as is a malformed or unreadable one (the store
 * is then unchanged).  yastn_tune_clear empties the store.  Loading adds to
 * the store, replacing entries with the same key and architecture. */
yastn_status yastn_tune_save(const char *path);
yastn_status yastn_tune_load(const char *path, int32_t *loaded);
void yastn_tune_clear(void);

/* Structure of problem prob's output.  The returned arrays are owned by the
 * plan and live until yastn_free.  c->charges / shapes / offsets are [host]. */
yastn_status yastn_plan_output(yastn_plan_t plan, int32_t prob, yastn_tensor_desc *c,
                               int64_t *c_numel);

/* Options the plan was built with and its number of problems (either output
 * may be NULL). */
yastn_status yastn_plan_info(yastn_plan_t plan, yastn_options *opts, int32_t *nprob);

/* Device workspace yastn_contract needs, in bytes (may be 0). */
yastn_status yastn_plan_workspace(yastn_plan_t plan, size_t *bytes);

yastn_status yastn_plan_stats(yastn_plan_t plan, int32_t prob, yastn_stats *st);

/* Run every problem of the plan in one grouped launch, asynchronously on
 * hip_stream.  a[p], b[p] [device] are the input buffers of problem p (any
 * values with the planned structure; in_dtype elements), c[p] [device] its
 * output buffer of c_numel elements (out_dtype), fully overwritten: C need
 * not be zeroed.  The host arrays a, b, c are read during the call (plans of
 * more than 64 problems: a small kernel first copies the pointers into a
 * table in the workspace; up to 65536 problems run in one grouped launch).
 * workspace [device] must hold yastn_plan_workspace bytes (256-byte aligned)
 * and must not be shared by calls that may overlap.  Results are
 * deterministic: no atomics, fixed summation order per output element. */
yastn_status yastn_contract(yastn_plan_t plan, const void *const *a, const void *const *b,
                            void *const *c, void *workspace, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * yastn_contract, with the workspace taken from a fixed device array of
 * YASTN_SCRATCH_BYTES that the library holds on every GPU it runs on (from
 * the first call on that GPU until the process ends), so the call passes no
 * workspace and allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).  The plan's workspace (yastn_plan_workspace) must fit:
 * larger plans get YASTN_ERR_STATE; so does a call whose current device is
 * not the plan's.  Every call on one GPU shares that GPU's array and leaves
 * its contents behind (each call writes every scratch byte it reads first),
 * so calls that may overlap on one GPU -- on different streams, or on one
 * stream with a plan still running that uses yastn_contract_noalloc -- race:
 * serialise them.  Results are bitwise those of yastn_contract. */
#define YASTN_SCRATCH_BYTES ((size_t)64 << 20)
yastn_status yastn_contract_noalloc(yastn_plan_t plan, const void *const *a, const void *const *b,
                                    void *const *c, void *hip_stream);

/* As yastn_contract for a single-problem plan, and also writes the FP64
 * Frobenius norm and max |x| of the output: norm_out [device] receives
 * out[0] = ||C||_F, out[1] = max |C| (the truncation input's normalisation).
 * The register-resident and pipelined kernels accumulate it in their epilogue
 * (no second pass over C: each tile files its part in the workspace and one
 * small kernel reduces the parts in tile order, so the result is
 * deterministic); other kernel variants run a separate two-pass reduction.
 * The workspace (yastn_plan_workspace bytes) holds the parts. */
yastn_status yastn_contract_norm(yastn_plan_t plan, const void *const *a, const void *const *b,
                                 void *const *c, void *workspace, double *norm_out, void *hip_stream);

/* As yastn_contract, and records HIP events on hip_stream for timing:
 * events[0] before the B pack kernel, events[1] between the pack kernel and
 * the grouped GEMM, events[2] after the GEMM ([host] array of 3 hipEvent_t
 * created by the caller; any entry may be NULL).  The plan must run in one
 * launch (at most 65536 problems), else YASTN_ERR_STATE. */
yastn_status yastn_contract_timed(yastn_plan_t plan, const void *const *a, const void *const *b,
                                  void *const *c, void *workspace, void *hip_stream,
                                  void *const *events);

/* Kernel variants.  A plan starts with variant 0 (the library's heuristic).
 * Variants 1-6: MFMA tiles reading a packed copy of B (six tile shapes);
 * 7: one output row per lane on the vector FMA units (sectors with K, N <= 64);
 * 8-16: MFMA tiles with the tile's B values held in registers and read straight
 * from B's blocks (nine chunk / occupancy shapes; sectors with K <= 64, and
 * K <= 80 for variant 16, which runs one wave per SIMD);
 * 17-19: MFMA tiles over a packed B with the k loop software-pipelined (any K;
 * three shapes);
 * 20-22: as 8-16 for K <= 80, with each workgroup loading the B tile of up
 * to four row tiles of one sector column range into shared memory once
 * (three chunk / occupancy shapes; FP32 arithmetic: variant 22 only);
 * 23: as 22 with A's rows loaded in adjacent pairs (FP64, K <= 40, plans
 * whose A rows run contiguously in even-length runs);
 * 24: as 20-22 for any K, the B tile staged in shared memory in chunks of 32
 * k straight from B's blocks (no packed copy of B), the next chunk's loads in
 * flight during the current chunk's products (FP64, plans whose tiles hold at
 * most 32 rows).
 * yastn_plan_autotune runs every variant that fits the plan `reps` times on
 * the caller's buffers (same arguments as yastn_contract; C is overwritten),
 * times them with HIP events (the variants within 15 % of the fastest a
 * second time, in reverse order, keeping each one's better time), keeps the
 * fastest in the plan and returns its
 * id in *chosen (may be NULL).  times_ms [host], if not NULL, receives
 * YASTN_NUM_VARIANTS floats: [0] = best time per contraction, [v] = time of
 * variant v or -1 if it does not fit.  Synchronises hip_stream.  Results of
 * different variants agree within rounding, and one plan always uses one
 * variant, so repeated contractions stay bitwise reproducible.
 * The choice is kept with the plan's structure: a later yastn_plan_autotune
 * on any handle of a tuned structure (see the structure cache) returns the
 * stored choice and times at once, without timing again.
 * yastn_plan_set_variant sets the variant of this handle only;
 * YASTN_ERR_STATE if the variant does not fit.  A new handle starts at the
 * structure's tuned variant (0, the heuristic, before any tuning). */
#define YASTN_NUM_VARIANTS 25
yastn_status yastn_plan_autotune(yastn_plan_t plan, const void *const *a, const void *const *b,
                                 void *const *c, void *workspace, void *hip_stream, int32_t reps,
                                 int32_t *chosen, float *times_ms);
yastn_status yastn_plan_set_variant(yastn_plan_t plan, int32_t variant);

/* One entry of a multi-plan launch (continuous batching across requests). */
typedef struct {
  yastn_plan_t plan;
  const void *const *a;      /* [host array of nprob device pointers]                           */
  const void *const *b;
  void *const *c;
  void *workspace;           /* [device] this job's workspace                                   */
} yastn_job;

/* Run the problems of several plans in one grouped launch on hip_stream.
 * All plans must share precision and dtypes (else YASTN_ERR_STATE).  Each
 * job's results are bitwise equal to running it alone with yastn_contract. */
yastn_status yastn_contract_jobs(const yastn_job *jobs, int32_t njobs, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of contraction requests from many concurrent
 * CTM runs.  A request is a chain of up to YASTN_MAX_CHAIN contractions of
 * resident tensors (an enlarged-corner step: C.T, .T, .A, .A*), step i > 0
 * taking step i-1's output as its A operand.  The server admits queued
 * requests in arrival order while its device memory pool (one allocation made
 * by yastn_server_create; serving never calls hipMalloc) can hold their
 * intermediate outputs and workspaces (a request that fits may pass a waiting
 * one that does not, at most 16 times per waiting request, after which the
 * waiting request is admitted next); each yastn_server_step merges the next
 * step of every admitted request into one grouped launch (yastn_contract_jobs)
 * on the server's stream, so requests that arrive while others run join the
 * next launch; a request completes when the event after the launch holding
 * its last step has completed, and its pool memory is reused.  Every result is
 * bitwise the one yastn_contract gives alone (deterministic kernels).  Not
 * thread-safe: one host thread drives a server.
 * ------------------------------------------------------------------------- */
#define YASTN_MAX_CHAIN 8
enum { YASTN_REQ_QUEUED = 0, YASTN_REQ_RUNNING = 1, YASTN_REQ_DONE = 2 };

typedef struct {
  int32_t nsteps;              /* contractions in the chain, 1..YASTN_MAX_CHAIN                   */
  const yastn_plan_t *plans;   /* [host, nsteps] single-problem plans                             */
  const void *a0;              /* [device] A operand of step 0 (resident, caller-owned)           */
  const void *const *b;        /* [host, nsteps] [device] B operand of each step (resident)       */
  void *out;                   /* [device] output of the last step (caller-owned, c_numel elements) */
} yastn_request;

typedef struct {
  int64_t submitted, admitted, completed;  /* requests                                          */
  int64_t ticks, launched_steps, max_batch; /* grouped launches, steps launched, most per launch */
  int64_t queued, running;                  /* requests waiting for memory / admitted, now       */
  size_t pool_bytes, pool_used, pool_peak;  /* device pool                                       */
  int64_t bypasses;                         /* admissions past a waiting, larger request         */
  int64_t queued_peak;                      /* most requests waiting at once                     */
} yastn_server_stats;

typedef struct yastn_server_s *yastn_server_t;

/* pool_bytes of device memory for intermediates and workspaces (the HBM
 * budget); at most max_ahead (1..64) launches outstanding before a step waits
 * for the oldest; hip_stream: the server's stream. */
yastn_status yastn_server_create(size_t pool_bytes, int32_t max_ahead, void *hip_stream, yastn_server_t *out);
/* Queue a request (the arrays are read during the call); *id identifies it.
 * YASTN_ERR_NOMEM if its footprint exceeds the pool. */
yastn_status yastn_server_submit(yastn_server_t s, const yastn_request *rq, int64_t *id);
/* One scheduler tick: retire finished launches, admit queued requests, launch
 * the next step of every admitted request (one grouped launch per precision);
 * *launched (may be NULL) = steps launched. */
yastn_status yastn_server_step(yastn_server_t s, int32_t *launched);
/* State of request id (YASTN_REQ_*) and, once done, its latency from submit to
 * the host observing completion, in ms (else -1). */
yastn_status yastn_server_query(yastn_server_t s, int64_t id, int32_t *state, double *latency_ms);
/* Drop a finished request's record. */
yastn_status yastn_server_forget(yastn_server_t s, int64_t id);
/* Run ticks until every submitted request is done. */
yastn_status yastn_server_drain(yastn_server_t s);
yastn_status yastn_server_get_stats(yastn_server_t s, yastn_server_stats *out);
/* Waits for outstanding launches, frees the pool.  NULL is ignored. */
void yastn_server_destroy(yastn_server_t s);

/* FP64 Frobenius norm and max |x| of a [device] buffer of n elements
 * (dtype), written as out[0] = ||x||_F, out[1] = max|x| ([device], FP64).
 * Deterministic two-pass reduction; workspace [device] must hold
 * yastn_norm_workspace() bytes. */
size_t yastn_norm_workspace(void);
yastn_status yastn_norm(const void *x, int64_t n, yastn_dtype dtype, double *out, void *workspace,
                        void *hip_stream);

/* Release a plan handle (the tables go with the last handle that shares
 * them and the cache entry).  NULL is ignored.  The caller must make sure no
 * launch that uses the plan is still running. */
void yastn_free(yastn_plan_t plan);

/* ---- leg permutation (transpose) of a block tensor ----------------------
 * Y = transpose(X, perm): leg i of Y is leg perm[i] of X (numpy convention).
 * Each block of X with charges (t_0..t_{r-1}) becomes the block of Y with
 * charges (t_perm[0]..t_perm[r-1]), its elements permuted the same way
 * (Sec. II.A: a block is a dense array indexed by its legs; permuting legs
 * permutes the charge tuple and the block's axes together).  Y's blocks are
 * ordered ascending by charge tuple and stored contiguously; signature and
 * total charge follow the legs.  yastn_perm_plan validates X as yastn_plan
 * does (perm must be a permutation of 0..rank-1, else YASTN_ERR_ARG) and
 * uploads one table; yastn_permute is asynchronous on hip_stream, reads X
 * [device] (dtype) and overwrites every element of Y [device] (same dtype,
 * yastn_perm_output numel elements).  X and Y must not overlap.  One
 * element per thread, writes coalesced, HBM-bound. */
typedef struct yastn_perm_s *yastn_perm_t;
yastn_status yastn_perm_plan(const yastn_tensor_desc *x, const int32_t *perm, void *hip_stream, yastn_perm_t *out);
yastn_status yastn_perm_output(yastn_perm_t p, yastn_tensor_desc *y, int64_t *y_numel);
yastn_status yastn_permute(yastn_perm_t p, yastn_dtype dtype, const void *x, void *y, void *hip_stream);
void yastn_perm_free(yastn_perm_t p);

/* ---- gradient of a tensordot (reverse mode, real arithmetic) ------------
 * For C = tensordot(A, B, axes) and a scalar loss L with dC = dL/dC (C's
 * structure, as yastn_plan_output gives it), the gradient with respect to
 * A (wrt = 0) is dA = transpose(tensordot(dC, B*, axes = (dC's B-free legs,
 * B's free legs)), back to A's leg order), and with respect to B (wrt = 1)
 * dB = transpose(tensordot(A*, dC, axes = (A's free legs, dC's A-free
 * legs)), back to B's leg order).  B* is B with flipped signatures and total
 * charge, the same real data (the conjugate of Sec. II.A), so the contracted
 * legs are dual and the result carries A's (B's) signature and total charge.
 * The gradient's block list is the structural output of that contraction:
 * every block of A's (B's) charge sectors that some pair reaches, in
 * ascending charge order (blocks of A that no pair reaches are absent, their
 * gradient is zero).  yastn_grad_plan plans both steps (one contraction with
 * opts, one permutation when the leg orders differ); yastn_grad runs them on
 * hip_stream: dc [device] (opts.in_dtype), other = B for wrt 0 or A for
 * wrt 1 [device] (opts.in_dtype), out [device] (opts.out_dtype,
 * yastn_grad_output numel elements), workspace [device] of
 * yastn_grad_workspace bytes. */
typedef struct yastn_grad_s *yastn_grad_t;
yastn_status yastn_grad_plan(const yastn_problem *prob, int32_t wrt, const yastn_options *opts, void *hip_stream,
                             yastn_grad_t *out);
yastn_status yastn_grad_output(yastn_grad_t g, yastn_tensor_desc *d, int64_t *numel);
yastn_status yastn_grad_workspace(yastn_grad_t g, size_t *bytes);
yastn_status yastn_grad(yastn_grad_t g, const void *dc, const void *other, void *out, void *workspace,
                        void *hip_stream);
void yastn_grad_free(yastn_grad_t g);

/* ---- block-sparse truncated SVD (the CTM truncation) --------------------
 * T (FP64) viewed as a matrix: rows = the legs row_legs[0..nrow) (in that
 * order), columns = the other legs in leg order.  Its blocks group into
 * sectors X = sum over the row legs of s_i rho_i (Z_m components reduced
 * into [0, m)); by the block form of charge conservation (Sec. II.A) the
 * column legs of a sector carry n - X, so the matrix is block diagonal, one
 * dense matrix M_X per sector (Sec. II.B fusion of the row legs and of the
 * column legs; constituent charge tuples ascending, each block's row index in
 * C order over its row legs, its column index over its column legs; absent
 * blocks are zeros).  The CTM move truncates the SVD of this block-diagonal
 * matrix to the environment dimension chi (Sec. III, Fig. 3 (c)-(d)).
 *
 * yastn_svd_plan validates T as yastn_plan does (row legs: a non-empty proper
 * subset, no repeats, else YASTN_ERR_ARG) and uploads the sector tables.
 * Sectors are numbered in ascending order of X; yastn_svd_sector gives sector
 * k's charge X ([host] nsym ints), its matrix dims m x n and the index of its
 * first singular value (sector k has min(m, n) of them, sv0 .. sv0 + min - 1).
 *
 * yastn_svd computes every M_X = U_X diag(S_X) V_X^T on the device (FP64
 * block one-sided Jacobi: the columns of the tall orientation of M_X are
 * put in order of descending norm before each sweep and rotated in blocks of
 * 8 until every pair is orthogonal to working precision) and applies one
 * global truncation: values at or below
 * tol * (largest value) are dropped; if more than chi remain and c is the
 * (chi+1)-th largest of them, a value is kept iff it exceeds c (1 + deg_tol),
 * so at most chi are kept and a multiplet within deg_tol of the first dropped
 * value is never split.  sv [device] receives all nsv singular values, each
 * sector's descending; kept [host] (nsectors) the kept count of each sector
 * (a prefix of its values); sweeps [host, may be NULL] the Jacobi sweeps run.
 * t [device]: T's buffer; workspace [device]: yastn_svd_info bytes, 256-byte
 * aligned (per sector the working matrix, V, a copy of the matrix and a
 * scratch copy of both for the column reordering: about 3 m n + 2 n^2
 * doubles for an m x n tall sector, plus per-value arrays), which also holds
 * the factors until the next yastn_svd.  Runs on
 * hip_stream and synchronises it once per sweep (it returns when done);
 * YASTN_ERR_STATE if the sweeps do not converge.
 *
 * yastn_svd_output: the structure of the kept factors of the last yastn_svd:
 * U with legs (row legs..., v), v carrying charge X with signature -1, total
 * charge 0, block (row tuple, X) of dims (row dims..., kept_X); V^T with legs
 * (v', column legs...), v' carrying X with signature +1, T's total charge,
 * block (X, column tuple) of dims (kept_X, column dims...).  Blocks ascending,
 * contiguous; sectors with nothing kept have none.  Arrays owned by the plan.
 * yastn_svd_factors writes them (async on hip_stream) into u and vt [device]
 * from the workspace of the last yastn_svd.  Signs: a singular pair
 * (u_t, v_t) is only defined up to a common sign; the one written is the one
 * whose u_t (as a column of the sector matrix) has its entry of largest
 * magnitude, the first such in row order, positive.  yastn_svd_factors_scaled
 * also multiplies U's kept column t by S_t^pu and V^T's row t by S_t^pv
 * (pu = pv = -0.5 gives the factors U S^-1/2 and S^-1/2 V^T of the CTM
 * projectors; 0 and 0 is yastn_svd_factors); YASTN_ERR_ARG for a power
 * that is not finite.
 *
 * yastn_svd_set_flags: YASTN_SVD_RECOVER_V makes the following yastn_svd
 * calls on this plan form one set of singular vectors after the sweeps
 * instead of accumulating rotations.  When every sector has at most 1024
 * rows (tall orientation), each sector is first factored W = Q R by
 * Householder reflections and the sweeps run on R^T (nearly orthogonal,
 * graded columns: about half the sweeps on the CTM four-corner product);
 * the right vectors of W are then the converged columns and the left ones
 * are formed as w_t = W v_t / s_t.  Otherwise the sweeps run on W without
 * rotating V and v_t = W^T u_t / s_t.  Either way the formed vectors carry
 * an error of about sqrt(n) eps s_max / s_t relative, so the mode is used
 * only when 4 sqrt(rows) eps s_max <= 1e-11 s_min over the kept values;
 * otherwise the call runs again with accumulated rotations (the default,
 * flags 0).  YASTN_ERR_ARG for an unknown flag. */
#define YASTN_SVD_RECOVER_V 1
typedef struct yastn_svd_s *yastn_svd_t;
yastn_status yastn_svd_plan(const yastn_tensor_desc *t, int32_t nrow, const int32_t *row_legs, void *hip_stream,
                            yastn_svd_t *out);
yastn_status yastn_svd_info(yastn_svd_t s, int32_t *nsectors, int64_t *nsv, size_t *workspace_bytes);
yastn_status yastn_svd_set_flags(yastn_svd_t s, int32_t flags);
yastn_status yastn_svd_sector(yastn_svd_t s, int32_t k, int32_t *charge, int64_t *m, int64_t *n, int64_t *sv0);
yastn_status yastn_svd(yastn_svd_t s, const void *t, int32_t chi, double tol, double deg_tol, double *sv,
                       int32_t *kept, int32_t *sweeps, void *workspace, void *hip_stream);
yastn_status yastn_svd_output(yastn_svd_t s, yastn_tensor_desc *u, int64_t *u_numel, yastn_tensor_desc *vt,
                              int64_t *vt_numel);
yastn_status yastn_svd_factors(yastn_svd_t s, void *u, void *vt, const void *workspace, void *hip_stream);
yastn_status yastn_svd_factors_scaled(yastn_svd_t s, void *u, void *vt, double pu, double pv, const void *workspace,
                                      void *hip_stream);
void yastn_svd_free(yastn_svd_t s);

/* ---- one CTM move (Sec. III, Fig. 3) ------------------------------------
 * The left move of the corner-transfer-matrix method for a 1x1 unit cell,
 * all in FP64 on the device.  Inputs: env[9] = C1, C2, C3, C4, T1, T2, T3,
 * T4, A (corners top-left, top-right, bottom-right, bottom-left; edges top,
 * right, bottom, left; the site tensor), with these legs and signatures
 * (every bond joins a +1 leg to a -1 leg of the same space; A* is A with
 * every signature and the total charge flipped and the same values):
 *     C1 (d -, r +)   C2 (l -, d -)   C3 (u +, l -)   C4 (u +, r +)
 *     T1 (l -, k -, b +, r +)    T2 (t +, k +, b -, bot -)
 *     T3 (l -, k +, b -, r +)    T4 (t +, k -, b +, bot -)
 *     A  (t +, l +, b -, r -, p +)
 * (an edge's k / b legs join the ket / bra layer of the site).  The move:
 *  1. enlarged corners (Fig. 3 (b)-(c)), each four contractions:
 *     Q1 = C1.T1.T4.A.A*  legs (T1.r, T4.bot, A.b, A.r, A*.b, A*.r)
 *     Q2 = C2.T2.T1.A.A*  legs (T2.bot, T1.l, A.l, A.b, A*.l, A*.b)
 *     Q3 = C3.T3.T2.A.A*  legs (T3.l, T2.t, A.t, A.l, A*.t, A*.l)
 *     Q4 = C4.T4.T3.A.A*  legs (T4.t, T3.r, A.t, A.r, A*.t, A*.r)
 *  2. halves R_up = Q2.Q1 over (T1, A, A* horizontal legs), legs (Q2's
 *     bottom cut, Q1's bottom cut); R_dn = Q3.Q4, legs (Q3's top cut, Q4's
 *     top cut);
 *  3. the four-corner product M = R_up.R_dn over (Q1's bottom cut, Q4's top
 *     cut) (Fig. 3 (d));
 *  4. its truncated SVD (yastn_svd's rule and sign convention, rows = R_up's
 *     remaining legs) to at most chi values;
 *  5. projectors P_up = R_dn.(S^-1/2 V^T)*, P_dn = R_up.(U S^-1/2)* (F* the
 *     dual of a factor), legs (cut..., k);
 *  6. the new left column C1' = P_up.(C1.T1), C4' = P_dn.(C4.T3) and
 *     T4' = P_dn^T (T4.A.A*) P_up, contracted as Z1 = P_dn.T4, Z2 = Z1.A,
 *     Z3 = Z2.A*, T4' = Z3.P_up, with the legs and signatures of C1, T4, C4;
 *  7. each divided by its largest |entry| (FP64 reduction on the device).
 * Independent contractions share a grouped launch (the four corners' steps,
 * C4.T3, the projectors, C1', C4' and Z1: eleven launches of contractions).
 *
 * yastn_ctm_plan validates the nine descriptors (yastn_plan's error classes;
 * YASTN_ERR_SIGNATURE / _SHAPE when they do not form the network above),
 * plans every contraction before the SVD and allocates the device memory of
 * all intermediates (owned by the handle).  Synchronises hip_stream.
 * yastn_ctm_move runs one move on env [device, 9 buffers, FP64]; it
 * synchronises hip_stream after the SVD (the kept counts decide the
 * projectors' structure, whose plans come from the plan cache when the
 * structure repeats) and returns when the move is done.  flags:
 * YASTN_CTM_AUTOTUNE times the kernel variants of every contraction plan not
 * tuned yet and keeps the fastest.  The results stay in the handle's memory
 * until the next move or yastn_ctm_free; yastn_ctm_tensor gives any tensor
 * of the move (YASTN_CTM_* below): its structure (arrays owned by the handle)
 * and its device buffer; yastn_ctm_copy copies a tensor's values (numel FP64)
 * into dst [device] on hip_stream (async).  yastn_ctm_info [host outputs, each
 * may be NULL]: kept values (sum over sectors), Jacobi sweeps, the time of
 * each phase of the last move in ms from HIP events on hip_stream (ms[0]
 * corners, ms[1] halves and product, ms[2] SVD, ms[3] the plans after the
 * SVD and the scaled factors, ms[4] projectors and the new column, ms[5]
 * normalisation), and the useful flops of its contractions (flops[0] before
 * the SVD, flops[1] after; sums of 2 m k n over matched block pairs). */
typedef struct yastn_ctm_s *yastn_ctm_t;
enum {
  YASTN_CTM_Q1 = 0, YASTN_CTM_Q2, YASTN_CTM_Q3, YASTN_CTM_Q4, YASTN_CTM_RUP, YASTN_CTM_RDN, YASTN_CTM_M,
  YASTN_CTM_US, YASTN_CTM_VTS, YASTN_CTM_PUP, YASTN_CTM_PDN, YASTN_CTM_C1T1, YASTN_CTM_C4T3, YASTN_CTM_Z1,
  YASTN_CTM_Z2, YASTN_CTM_Z3, YASTN_CTM_C1N, YASTN_CTM_T4N, YASTN_CTM_C4N, YASTN_CTM_C1, YASTN_CTM_T4, YASTN_CTM_C4,
  YASTN_CTM_NTENSORS
};
/* YASTN_CTM_US / _VTS: U S^-1/2 and S^-1/2 V^T; _C1N/_T4N/_C4N: the new
 * column before step 7; _C1/_T4/_C4: after it (the move's result). */
#define YASTN_CTM_AUTOTUNE 1
yastn_status yastn_ctm_plan(const yastn_tensor_desc *env, void *hip_stream, yastn_ctm_t *out);
yastn_status yastn_ctm_move(yastn_ctm_t h, const void *const *env, int32_t chi, double tol, double deg_tol,
                            int32_t flags, void *hip_stream);
yastn_status yastn_ctm_tensor(yastn_ctm_t h, int32_t which, yastn_tensor_desc *desc, int64_t *numel,
                              const void **data);
yastn_status yastn_ctm_copy(yastn_ctm_t h, int32_t which, void *dst, void *hip_stream);
yastn_status yastn_ctm_info(yastn_ctm_t h, int32_t *kept, int32_t *sweeps, double *ms, double *flops);
void yastn_ctm_free(yastn_ctm_t h);

/* ---- complex128 tensordot ------------------------------------------------
 * C = tensordot(A', B', axes) for complex tensors stored as interleaved
 * (re, im) FP64 pairs (YASTN_DTYPE_C128; offsets and shapes count complex
 * elements), where A' = conj(A) if conj has YASTN_CONJ_A and A otherwise,
 * B' likewise with YASTN_CONJ_B.  Conjugation maps every leg to its dual:
 * the signatures and the total charge flip and the values are conjugated
 * (Sec. II.A); the descriptors passed are those of A and B themselves.
 * The product runs on the FP64 MFMA kernels as one real contraction (A read
 * in place with its (re, im) pairs as one more contracted leg of dim 2; B
 * expanded in the workspace into 2 x 2 real blocks, one streaming kernel;
 * C written in place with (re, im) as its last leg), so every property of
 * yastn_plan / yastn_contract holds: one grouped launch for all problems,
 * deterministic results, the structure cache.  Operand ranks: A <= 7,
 * B <= 6 (the real form adds one and two legs).  yastn_zplan_output gives
 * C's complex structure; yastn_zplan_workspace the workspace bytes (the real
 * plan's plus 32 bytes per complex element spanned by each B);
 * yastn_zplan_real the underlying real plan (owned by the zplan) for
 * yastn_plan_stats (useful_flops = 8 m k n per matched block pair) and
 * yastn_plan_set_variant; yastn_zplan_autotune is yastn_plan_autotune of the
 * real plan on these complex buffers (it expands B first).  yastn_zcontract
 * is asynchronous on hip_stream; complex buffers must be 16-byte aligned. */
#define YASTN_CONJ_A 1
#define YASTN_CONJ_B 2
typedef struct yastn_zplan_s *yastn_zplan_t;
yastn_status yastn_zplan(const yastn_problem *probs, int32_t nprob, int32_t conj, void *hip_stream,
                         yastn_zplan_t *out);
yastn_status yastn_zplan_output(yastn_zplan_t z, int32_t prob, yastn_tensor_desc *c, int64_t *c_numel);
yastn_status yastn_zplan_workspace(yastn_zplan_t z, size_t *bytes);
yastn_status yastn_zplan_real(yastn_zplan_t z, yastn_plan_t *real);
yastn_status yastn_zcontract(yastn_zplan_t z, const void *const *a, const void *const *b, void *const *c,
                             void *workspace, void *hip_stream);
yastn_status yastn_zplan_autotune(yastn_zplan_t z, const void *const *a, const void *const *b, void *const *c,
                                  void *workspace, void *hip_stream, int32_t reps, int32_t *chosen,
                                  float *times_ms);
void yastn_zplan_free(yastn_zplan_t z);

/* ---- fermionic swap gate -------------------------------------------------
 * The swap gate between leg groups legs1 and legs2 of one tensor (Sec. III,
 * fermionic Hubbard example: swap gates on line crossings impose the
 * fermionic order, changing the sign of blocks with odd-parity charges on
 * both swapped legs).  The parity of a charge is the sum of its fermionic
 * components (fermionic[c] = 1; [host], nsym entries of 0 or 1) mod 2; a
 * group's parity is the sum over its legs mod 2; a block is negated iff both
 * groups are odd -- the product of the swap gates of every pair (i in legs1,
 * j in legs2).  yastn_swap_plan validates T (yastn_plan's classes; legs out
 * of range or a bad mask: YASTN_ERR_ARG) and lists the negated blocks;
 * yastn_swap_info gives their number and elements; yastn_swap_gate negates
 * them in place in data [device] of the given dtype (F64, F32 or C128),
 * asynchronously on hip_stream, touching no other element. */
typedef struct yastn_swap_s *yastn_swap_t;
yastn_status yastn_swap_plan(const yastn_tensor_desc *t, int32_t n1, const int32_t *legs1, int32_t n2,
                             const int32_t *legs2, const int32_t *fermionic, yastn_swap_t *out);
yastn_status yastn_swap_info(yastn_swap_t s, int64_t *blocks, int64_t *elements);
yastn_status yastn_swap_gate(yastn_swap_t s, void *data, yastn_dtype dtype, void *hip_stream);
void yastn_swap_free(yastn_swap_t s);

const char *yastn_last_error(void);
const char *yastn_status_string(yastn_status s);
int32_t yastn_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* YASTN_H */
