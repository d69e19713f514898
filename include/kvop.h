/*
 * kvop — KV-cache-backed semantic operators on AMD MI355X (gfx950).
 *
 * C ABI of the library.  The operations follow the paper's description of its
 * KV cache-enabled operators (Section 5):
 *   - offline, every document is fed once through the decoder and its keys and
 *     values are kept ("Offline: KV Cache Creation")            -> kvop_kv_build
 *   - online, an operator appends its query (instruction suffix) to the cached
 *     documents and one batched forward pass yields one output per item; a
 *     filter reads the logits of the answer tokens, forms their log-odds and
 *     accepts, rejects or marks the item unsure against two thresholds
 *     (Section 5 "Online: Query Execution"; thresholds on log-odds as in
 *     Section 4.1, Eq. 14 at zero temperature); a map decodes a longer output;
 *     a join is a filter over pairs of the cartesian product (Section 4.2)
 *                                                                -> kvop_op_eval
 *   - query-agnostic compression keeps a fraction of each document's rows
 *     (Section 2.3, Section 5); the kept rows are passed in as index lists,
 *     scored and selected by expected attention  -> kvop_kv_build_scored, kvop_ea_select
 *   - the learned proxy is the cheap first stage of a two-stage cascade: it
 *     answers confident items and passes the rest on as unsure (cascade
 *     semantics, Section 4.1 Eqs. 1-3)                           -> kvop_proxy_*
 *   - a cascade over profiles of increasing retention evaluates each item only
 *     until a stage decides it (Section 4.1, Eqs. 1-3)           -> kvop_cascade_eval
 *   - the optimizer chooses the stages and thresholds of such cascades from
 *     profiled log-odds under credible bounds on recall and precision, and
 *     orders the chosen operators (Sections 4.1-4.2; host code)  -> kvop_plan_*
 *   - several operators share every launch of one pass (Section 5, batching)
 *                                                                -> kvop_mixed_eval
 *
 * Conventions for every call:
 *   - "dev" pointers are device (HBM) pointers on the current HIP device,
 *     "host" pointers are ordinary host memory.  All buffers are owned by the
 *     caller unless stated otherwise; the library never frees them.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued on it asynchronously unless a call says it synchronises.
 *   - Errors: every call returns a kvop_status.  No C++ exception crosses the
 *     ABI.  On an argument error (EINVAL, EBADHANDLE, ENOMEM) nothing has been
 *     enqueued and outputs are untouched.  kvop_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Not thread-safe per object: calls on one model/pool from several host
 *     threads must be serialised by the caller.
 */
#ifndef KVOP_H
#define KVOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kvop_status {
  KVOP_OK = 0,
  KVOP_EINVAL = 1,      /* invalid argument, shape or index list */
  KVOP_ENOMEM = 2,      /* device memory or cache pool exhausted */
  KVOP_EBADHANDLE = 3,  /* released, foreign or corrupt cache handle */
  KVOP_EDEVICE = 4      /* a HIP runtime error (also asynchronous faults seen later) */
} kvop_status;

/* Arithmetic of weights and activations.  Accumulation, softmax statistics,
 * RMSNorm statistics and the logit-head reduction are FP32 in both. */
typedef enum kvop_dtype { KVOP_F32 = 0, KVOP_BF16 = 1 } kvop_dtype;

/* Storage of cached keys/values.  FP8 is OCP E4M3 (fn) with one FP32 scale per
 * block of 16 rows of one (layer, kv head, K or V): scale = amax/448. */
typedef enum kvop_kv_dtype { KVOP_KV_F32 = 0, KVOP_KV_BF16 = 1, KVOP_KV_FP8 = 2 } kvop_kv_dtype;

typedef enum kvop_op_kind { KVOP_FILTER = 0, KVOP_MAP = 1, KVOP_JOIN = 2 } kvop_op_kind;

/* Decoder shape: Llama-style pre-norm decoder, RMSNorm, rotary embedding
 * (rotate-half pairs (i, i + head_dim/2), angle pos * rope_theta^(-2i/head_dim)),
 * grouped-query attention (query head h uses kv head h / (n_heads/n_kv_heads)),
 * SwiGLU feed-forward W_down(silu(W_gate x) * W_up x), final RMSNorm, untied head. */
typedef struct kvop_model_cfg {
  int32_t n_layers, d_model, n_heads, n_kv_heads, head_dim, d_ffn, vocab;
  float rms_eps, rope_theta;
} kvop_model_cfg;

typedef struct kvop_model kvop_model;
typedef struct kvop_pool kvop_pool;
typedef struct kvop_proxy kvop_proxy;
typedef uint64_t kvop_handle;

/* Human-readable description of the last error on this thread ("" if none). */
const char* kvop_last_error(void);

/* Number of FP32 elements kvop_model_create expects for this shape. */
int64_t kvop_weights_numel(const kvop_model_cfg* cfg);

/* Create a model from FP32 master weights packed in one device buffer, in this
 * order (row-major, linear maps stored [out, in] and applied as x W^T):
 *   for each layer: attn_norm[d], wq[H*D, d], wk[Hkv*D, d], wv[Hkv*D, d],
 *                   wo[d, H*D], ffn_norm[d], w_gate[F, d], w_up[F, d], w_down[d, F]
 *   then final_norm[d], embed[V, d], head[V, d].
 * The library converts/repacks them into its own buffers in `compute` dtype
 * (norm gains stay FP32); the caller may free `weights_dev` after the call
 * returns (the call synchronises `stream`).
 * Errors: EINVAL on a bad shape (head_dim not 32/64/128, n_heads not a multiple
 * of n_kv_heads, d_model/d_ffn not multiples of 64, n_weights mismatch);
 * ENOMEM; EDEVICE. */
kvop_status kvop_model_create(const kvop_model_cfg* cfg, const float* weights_dev, int64_t n_weights,
                              kvop_dtype compute, void* stream, kvop_model** out);
kvop_status kvop_model_destroy(kvop_model* model);

/* A cache pool: `bytes` of device memory holding documents' caches in
 * `kv_dtype`.  Each document occupies one contiguous region laid out
 * [layer][kv head][K,V][row][head_dim] followed, for FP8, by its FP32 block
 * scales [layer][kv head][K,V][ceil(L/16)].  The pool owns its memory. */
kvop_status kvop_pool_create(kvop_model* model, kvop_kv_dtype kv_dtype, uint64_t bytes, kvop_pool** out);
kvop_status kvop_pool_destroy(kvop_pool* pool);
/* Bytes one document of length L occupies in this pool (rounded to 256). */
uint64_t kvop_doc_bytes(const kvop_pool* pool, int64_t L);
kvop_status kvop_pool_stats(const kvop_pool* pool, uint64_t* used_bytes, uint64_t* capacity_bytes,
                            int32_t* live_docs);

/* Offline cache creation (Section 5, "Offline"): prefill n_docs documents
 * causally at positions 0..L-1 and keep every layer's rotated keys and values.
 *   tokens_dev   : int32 token ids of all documents concatenated (device)
 *   offsets_host : int64[n_docs+1], document i is tokens[offsets[i]:offsets[i+1]]
 *   handles_out  : host array of n_docs handles, written on success
 *   pooled_dev   : optional FP32 [n_docs, d_model] output (NULL to skip): the mean
 *                  over the document's rows of the final-normed hidden state
 *                  (the learned proxy's input feature)
 * Errors: EINVAL (n_docs < 0, empty document, decreasing offsets, a token id outside
 * [0, vocab)); ENOMEM when the pool cannot hold all documents.  On any error no handle
 * is created and nothing is written.  Token ids are checked on the device before any
 * compute is enqueued, which synchronises `stream` once; the caches are then built
 * asynchronously on `stream`. */
kvop_status kvop_kv_build(kvop_pool* pool, const int32_t* tokens_dev, const int64_t* offsets_host,
                          int32_t n_docs, void* stream, kvop_handle* handles_out, float* pooled_dev);

/* Offline cache creation with query-agnostic compression scores (Section 2.3 and Section 5,
 * "Offline": the compressed profiles keep the rows chosen by the Expected Attention method
 * the paper cites).  Builds the caches exactly as kvop_kv_build (same handles, same cache
 * contents) and also writes, per document row, its expected-attention score:
 *   n_future   : the future queries sit at positions L .. L+n_future-1 (1..4096; e.g. the
 *                operators' suffix length); L + n_future must not exceed 65536
 *   scores_dev : FP32 [offsets[n_docs] - offsets[0]] (device), indexed like tokens_dev
 *                from offsets[0]; row score = sum over layers and kv heads of the row's
 *                share of that (layer, kv head)'s expected attention contribution: the
 *                document's pre-rotation queries of each layer and query head taken as a
 *                Gaussian (mean, population covariance), mapped through the rotation
 *                averaged over the future positions; a rotated key k's expected weight is
 *                exp(mean.k/sqrt(D) + k^T cov k/(2D)) normalised over the document's keys,
 *                times |v|, averaged over the query heads of the kv head, and each (layer,
 *                kv head) totals 1 (so a document's scores total n_layers * n_kv_heads).
 * Errors as kvop_kv_build, plus EINVAL (null scores_dev, n_future out of range, L + n_future
 * too long) and ENOMEM (workspace).  Asynchronous on stream like kvop_kv_build. */
kvop_status kvop_kv_build_scored(kvop_pool* pool, const int32_t* tokens_dev, const int64_t* offsets_host,
                                 int32_t n_docs, int32_t n_future, void* stream, kvop_handle* handles_out,
                                 float* pooled_dev, float* scores_dev);

/* Rows kept at retention r of a document of length L (the profile's compression ratio is
 * 1 - r): k = clamp(floor((round(1000 r) * L + 500) / 1000), min(4, L), L).  -1 if L < 1 or
 * r outside [0, 1]. */
int32_t kvop_retained_count(float r, int64_t L);

/* Retained-row lists of a compressed profile from expected-attention scores: per document
 * the kvop_retained_count(r, L) rows of highest score (equal scores: lower row first),
 * ascending, in the list format kvop_op_eval takes.
 *   scores_dev      : FP32 scores as written by kvop_kv_build_scored (device), indexed from
 *                     offsets_host[0]
 *   offsets_host    : int64[n_docs+1] document row offsets (as for kvop_kv_build)
 *   idx_dev         : int32 output (device), room for the sum of the counts
 *   idx_offsets_out : int64[n_docs+1] host output: document i's list is
 *                     idx[idx_offsets[i] : idx_offsets[i+1]] (document-relative rows)
 * Uses the pool's model for metadata staging.  Errors: EINVAL (null pointers, r outside
 * [0, 1], a document length outside [1, 65535]).  Asynchronous on stream. */
kvop_status kvop_ea_select(kvop_pool* pool, const float* scores_dev, const int64_t* offsets_host, int32_t n_docs,
                           float r, void* stream, int32_t* idx_dev, int64_t* idx_offsets_out);

/* Release documents' caches; their handles become invalid.  EBADHANDLE if any
 * handle is not live in this pool (then nothing is released). */
kvop_status kvop_kv_release(kvop_pool* pool, const kvop_handle* handles, int32_t n);

/* Operator descriptor (read during the call only). */
typedef struct kvop_op {
  int32_t kind;               /* kvop_op_kind */
  const int32_t* suffix_host; /* the operator's instruction suffix: token ids (host) */
  int32_t suffix_len;         /* S >= 1 */
  int32_t yes_id, no_id;      /* filter/join answer tokens ('1' and '0') */
  float theta_pos, theta_neg; /* accept iff LO > theta_pos, reject iff LO < theta_neg */
  int32_t label_lo, label_n;  /* map: decode over ids [label_lo, label_lo + label_n) */
  int32_t n_gen;              /* map: number of ids to decode (>= 1) */
  uint32_t flags;             /* KVOP_FLAG_* */
} kvop_op;

/* Skip the check that each list holds exactly k(r, L) rows (the caller may then
 * pass any valid sorted list; r is only range-checked). */
#define KVOP_FLAG_ANY_COUNT 1u
/* Padded batching, the form Section 5 ("Execution-time Batching") describes, kept as an
 * ablation of the variable-length work lists: every item's attention runs over the largest
 * cached key count of its wave (a join: of A and B together); the keys past the item's own
 * are loaded (its own retained rows again, cyclically), multiplied and masked, so results
 * equal the unpadded call's exactly while the work is that of a padded batch.  kvop_op_eval,
 * kvop_op_eval_select and kvop_cascade_eval honour it (kvop_mixed_eval ignores it); only the
 * direct-load attention kernels implement it: EINVAL for FP32 compute, an FP32 cache,
 * head_dim other than 64/128 or attention variant -1. */
#define KVOP_FLAG_PADDED 2u

/* Online execution (Section 5, "Online"): evaluate one operator over n_items
 * items.  A filter/map item is one document; a join item is an ordered pair of
 * documents (A, B) using handles[2i], handles[2i+1] and index lists 2i, 2i+1.
 *   r               : retention in (0, 1]; each list must hold exactly
 *                     k(r, L) = clamp(floor((round(1000 r) L + 500)/1000), min(4, L), L)
 *                     rows unless KVOP_FLAG_ANY_COUNT
 *   idx_dev         : int32 retained row indices of all lists concatenated (device);
 *                     every list strictly increasing within [0, L)
 *   idx_offsets_host: int64[n_lists+1] (n_lists = n_items, or 2 n_items for joins)
 *   handles_host    : n_lists handles
 *   logits_out_dev  : FP32 — filter/join: [n_items, 2] (yes, no);
 *                     map: [n_items, n_gen, label_n] logits over the label slice
 *   decision_out_dev: int8 [n_items] — 1 accept, 0 reject, -1 unsure (filter/join);
 *                     may be NULL for a map
 *   tokens_out_dev  : int32 [n_items, n_gen] decoded ids (map only, else NULL)
 * The suffix is placed after the document's original length (positions L + j;
 * for a join, B's rows sit at L_A + p and the suffix at L_A + L_B + j), sees every
 * retained row and the earlier suffix rows.  The call synchronises `stream` once
 * to validate the index lists before enqueuing any compute; the results are then
 * produced asynchronously on `stream`.
 * Errors: EINVAL (r out of range, wrong list count, unsorted or out-of-range
 * index, bad op fields), EBADHANDLE, ENOMEM, EDEVICE. */
kvop_status kvop_op_eval(kvop_pool* pool, const kvop_op* op, float r, const int32_t* idx_dev,
                         const int64_t* idx_offsets_host, const kvop_handle* handles_host, int32_t n_items,
                         void* stream, float* logits_out_dev, int8_t* decision_out_dev,
                         int32_t* tokens_out_dev);

/* Cascade entry: evaluate only the items listed in select_host (indices into the
 * n_items items described by handles/lists, as for kvop_op_eval), writing their outputs
 * at their own rows of logits_out_dev / decision_out_dev; other rows are untouched.
 * Filters and joins only (a map is rejected with EINVAL).  Used to send the items a
 * cheaper first stage left unsure to the full operator (Section 4.1, Eqs. 1-3). */
kvop_status kvop_op_eval_select(kvop_pool* pool, const kvop_op* op, float r, const int32_t* idx_dev,
                                const int64_t* idx_offsets_host, const kvop_handle* handles_host, int32_t n_items,
                                const int32_t* select_host, int32_t n_select, void* stream, float* logits_out_dev,
                                int8_t* decision_out_dev);

/* One stage of a filter cascade over cache profiles (Section 4.1): the same operator over the
 * profile of retention r with its own thresholds.  The lists are as for kvop_op_eval. */
typedef struct kvop_stage {
  float r;
  float theta_pos, theta_neg;       /* accept iff LO > theta_pos, reject iff LO < theta_neg */
  const int32_t* idx_dev;           /* this profile's retained lists (device) */
  const int64_t* idx_offsets_host;  /* int64[n_items (+1) or 2 n_items (+1) for joins] */
} kvop_stage;

/* A filter (or join) cascade over profiles of increasing cost (Section 4.1, Eqs. 1-3):
 * every item starts unsure; stage i evaluates only the items all earlier stages left unsure
 * (op->theta_* are replaced by the stage's thresholds) and accepts, rejects or leaves them
 * unsure.  Outputs (device, one row per item): the logits and decision of the last stage
 * that evaluated the item (decision -1 if it is still unsure after the last stage) and that
 * stage's index in stage_out_dev (int8).  processed_host[n_stages] receives the number of
 * items each stage evaluated (Eq. 4's unsure counts).  Every stage's lists are validated
 * before the first stage runs, so an argument error leaves the outputs untouched.  The call
 * synchronises `stream` between stages (the unsure set is compacted on the host).  Errors: EINVAL (a map, no
 * stages or more than 127, null pointers, a NaN threshold), and those of kvop_op_eval_select. */
kvop_status kvop_cascade_eval(kvop_pool* pool, const kvop_op* op, const kvop_stage* stages, int32_t n_stages,
                              const kvop_handle* handles_host, int32_t n_items, void* stream, float* logits_out_dev,
                              int8_t* decision_out_dev, int8_t* stage_out_dev, int32_t* processed_host);

/* Parity debugging: the residual stream of the suffix rows after decoder layer `layer`
 * (0 .. n_layers - 1) of a filter or join evaluation (Section 5, "Online: Query Execution":
 * the operator query's forward pass over the cached keys/values), for comparison with a
 * reference layer by layer.  Arguments as kvop_op_eval (map items: EINVAL); output FP32
 * [n_items, suffix_len, d_model] on the device, caller-owned.  At the last layer only each
 * item's last suffix row is carried past the attention (the row the head reads); the
 * item's other rows hold their input to that layer.  Validation, errors and stream
 * behaviour as kvop_op_eval; no logits or decisions are written. */
kvop_status kvop_debug_stage(kvop_pool* pool, const kvop_op* op, float r, const int32_t* idx_dev,
                             const int64_t* idx_offsets_host, const kvop_handle* handles_host, int32_t n_items,
                             int32_t layer, void* stream, float* hidden_out_dev);

/* ---- batching form -----------------------------------------------------------
 * Mixed operators in one pass (the batched execution of Section 5, "Execution-time
 * Batching", with variable-length work lists instead of padding): the items of
 * several filters, joins and at most one map share every projection launch and one
 * attention launch per layer; the map then continues with its decode steps.
 *   ops          : n_ops operators with their own output buffers (device):
 *                  filter/join logits [items of that op, 2] and decisions [items];
 *                  map logits [items, n_gen, label_n] and tokens [items, n_gen];
 *                  an operator's outputs are in the order its items appear
 *   item_op_host : operator index of every item
 *   item_list_host: first list/handle index of every item (a join uses two
 *                  consecutive ones); lists and handles as for kvop_op_eval
 * Work is split into waves of at most kvop_set_wave_rows rows with a fixed number of items
 * per operator.  KVOP_MIXED_PERSISTENT runs the attention as a persistent launch that
 * takes (item, kv head) units from a device counter; KVOP_MIXED_GRAPH captures one full
 * wave's launch sequence in a hipGraph and replays it for the following full waves
 * (the first and the last, partial wave run directly).  The call synchronises `stream`
 * to validate the lists, and again at the end when a graph was used.
 * Errors as kvop_op_eval; EINVAL for more than one map operator. */
typedef struct kvop_mixed_op {
  kvop_op op;
  float* logits_out_dev;
  int8_t* decision_out_dev;   /* filter/join, nullable */
  int32_t* tokens_out_dev;    /* map */
} kvop_mixed_op;
#define KVOP_MIXED_PERSISTENT 1u
#define KVOP_MIXED_GRAPH 2u
/* Suffix rows per wave of kvop_op_eval / kvop_mixed_eval (default 131072; >= 64). */
kvop_status kvop_set_wave_rows(int64_t rows);
kvop_status kvop_mixed_eval(kvop_pool* pool, const kvop_mixed_op* ops, int32_t n_ops, float r, const int32_t* idx_dev,
                            const int64_t* idx_offsets_host, const kvop_handle* handles_host,
                            const int32_t* item_op_host, const int64_t* item_list_host, int32_t n_items,
                            uint32_t flags, void* stream);

/* ---- learned proxy ----------------------------------------------------------
 * The cheap first stage of a two-stage cascade (Section 4.1, Eqs. 1-3: an operator
 * accepts or rejects a tuple, or passes it on as unsure).  Network:
 *   x = (f - mean) * inv_std        (feature standardiser, identity until fitted)
 *   z = W2 gelu(W1 x + b1) + b2,  p = softmax(z);  class 1 = accept
 * with exact (erf) GELU.  Parameters are FP32 masters packed as
 *   W1 [d_hidden, d_in] | b1 [d_hidden] | W2 [2, d_hidden] | b2 [2];
 * the forward projection and the W1 gradient run in BF16 on MFMA with FP32
 * accumulation; everything else is FP32.  Training minimises the mean
 * cross-entropy with bias-corrected Adam (beta 0.9 / 0.999, eps 1e-8). */
kvop_status kvop_proxy_create(int32_t d_in, int32_t d_hidden, const float* params_dev, kvop_proxy** out);
kvop_status kvop_proxy_destroy(kvop_proxy* proxy);
/* mean and 1/std (std floored at 1e-6) of every feature over feats_dev [n, d_in] */
kvop_status kvop_proxy_fit_standardizer(kvop_proxy* proxy, const float* feats_dev, int64_t n, void* stream);
kvop_status kvop_proxy_set_standardizer(kvop_proxy* proxy, const float* mean_dev, const float* inv_std_dev,
                                        void* stream);
/* One Adam step on the minibatch rows_dev[0..batch) of feats_dev/labels_dev (labels in
 * {0, 1}); rows_dev NULL means rows 0..batch-1.  batch must be a multiple of 8.
 * loss_out_dev (nullable) receives the minibatch's mean cross-entropy before the step. */
kvop_status kvop_proxy_train_step(kvop_proxy* proxy, const float* feats_dev, const int32_t* labels_dev,
                                  const int32_t* rows_dev, int32_t batch, float lr, void* stream,
                                  float* loss_out_dev);
/* Gradients of the minibatch's mean cross-entropy, packed like the parameters (no update). */
kvop_status kvop_proxy_grads(kvop_proxy* proxy, const float* feats_dev, const int32_t* labels_dev,
                             const int32_t* rows_dev, int32_t batch, void* stream, float* grads_out_dev,
                             float* loss_out_dev);
/* Inference over n rows: class (0/1), confidence max(p), answered = confidence > tau. */
kvop_status kvop_proxy_infer(kvop_proxy* proxy, const float* feats_dev, int64_t n, float tau, void* stream,
                             int8_t* cls_out_dev, float* conf_out_dev, int8_t* answered_out_dev);
/* kvop_proxy_infer that allocates nothing, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid it).  Same kernels
 * and results as kvop_proxy_infer.  Its scratch (the standardised BF16 features and the
 * FP32 hidden pre-activations of the call's rows) is a fixed device array of
 * KVOP_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; its address is looked
 * up on the first call on each device.  n is limited to
 *   n * (2 d_in + 4 d_hidden) + 256 <= KVOP_NOALLOC_SCRATCH_BYTES
 * (6553 rows for d_in 2048, d_hidden 256); larger n: EINVAL, nothing enqueued.  Every call
 * on one GPU uses the same array: calls that overlap on one GPU (several streams or host
 * threads) race and must be serialised by the caller. */
#define KVOP_NOALLOC_SCRATCH_BYTES (32u << 20)
kvop_status kvop_proxy_infer_noalloc(kvop_proxy* proxy, const float* feats_dev, int64_t n, float tau, void* stream,
                                     int8_t* cls_out_dev, float* conf_out_dev, int8_t* answered_out_dev);
/* Copy the FP32 master parameters (packed as above) into params_out_dev. */
kvop_status kvop_proxy_params(kvop_proxy* proxy, float* params_out_dev, void* stream);

/* ---- diagnostics and tuning ------------------------------------------------
 * Run one projection C = A B^T with an explicit tile configuration `tile`
 * (0 .. kvop_gemm_num_tiles(dtype)-1, or -1 for the library's own choice).  dtype: KVOP_F32 or KVOP_BF16 operands;
 * epilogue 0 = store C in out_dtype, 1 = FP32 C += A B^T, 2 = SwiGLU over 16-row
 * interleaved gate/up rows of B (C has N/2 columns).  Device pointers; strides in
 * elements.  EINVAL when the tile cannot run the shape (K, lda, ldb must be
 * multiples of 16 bytes / element size). */
/* The projection with its rotary epilogue (BF16 operands A [M, K], B [N, K], row-major,
 * K-contiguous; C [M, N] BF16): C = A B^T rounded to BF16, then the heads of width head_dim in
 * columns [0, rot_cols) rotated pairwise (i, i + head_dim/2) by the angles of row r's
 * position pos_dev[r] (cos_dev / sin_dev: [position][head_dim/2] FP32 tables): the decoder's
 * rotary embedding, applied to the operator query that Section 5 appends to each cached item,
 * so a query row j after an item of L cached rows sits at position L + j.  fused = 1 runs the
 * epilogue inside the projection
 * (the form op_eval uses), fused = 0 the plain projection followed by a separate rotation
 * pass; both must give the same bits.  head_dim must divide 128 and be a multiple of 16;
 * N and rot_cols multiples of head_dim; EINVAL otherwise or when the tile cannot run the shape.
 * Device pointers; C is overwritten. */
kvop_status kvop_debug_gemm_rope(int32_t tile, const void* A, const void* B, void* Cm, int32_t M, int32_t N, int32_t K,
                                 int32_t head_dim, int32_t rot_cols, const int32_t* pos_dev, const float* cos_dev,
                                 const float* sin_dev, int32_t fused, void* stream);
int32_t kvop_gemm_num_tiles(int32_t dtype);
const char* kvop_gemm_tile_name(int32_t dtype, int32_t tile);
kvop_status kvop_debug_gemm(int32_t dtype, int32_t out_dtype, int32_t epilogue, int32_t tile, const void* A,
                            const void* B, void* Cm, int32_t M, int32_t N, int32_t K, int64_t lda, int64_t ldb,
                            int64_t ldc, void* stream);
/* Per-kernel-class timing of the library's own launches: while on, each launch of
 * kvop_kv_build / kvop_op_eval is bracketed by HIP events on the caller's stream.
 * kvop_profile_stop synchronises those events and writes, for class i < n, the summed
 * milliseconds and the number of launches (classes named by kvop_profile_class_name). */
kvop_status kvop_profile_start(void);
kvop_status kvop_profile_stop(double* ms_out, int64_t* count_out, int32_t n);
/* Per-launch milliseconds of class cls from the last start/stop interval, in launch order:
 * writes min(n, count) values to ms_out (nullable) and returns the count (-1: bad class). */
int32_t kvop_profile_launches(int32_t cls, double* ms_out, int32_t n);
int32_t kvop_profile_num_classes(void);
const char* kvop_profile_class_name(int32_t i);
/* Autotuner: for each projection of the model (QKV, O, gate/up, down) at M = rows, time
 * every tile candidate (reps launches each, HIP events on `stream`) and record the fastest
 * in the tuning table used by kv_build / op_eval for that (dtype, epilogue, N, K, M bucket
 * = floor(log2 M)).  Allocates temporary scratch; synchronises.  A text report of every
 * timing is written to report (nullable, report_len bytes incl. the terminator). */
kvop_status kvop_autotune(kvop_model* model, int64_t rows, int32_t reps, void* stream, char* report,
                          int32_t report_len);
/* The tuning table as text lines "dtype epilogue N K mbucket tile_name"; returns the full
 * length (write at most len-1 bytes + terminator into buf, which may be NULL). */
int32_t kvop_tuning_export(char* buf, int32_t len);
/* Load lines in the export format into the tuning table; empty lines and lines starting
 * with '#' are skipped (EINVAL if another line is not understood). */
kvop_status kvop_tuning_import(const char* text);
/* Record the best tile for (dtype, epilogue, N, K, M) in the library's tuning table
 * (used by later kvop_kv_build / kvop_op_eval calls). */
kvop_status kvop_gemm_set_tile(int32_t dtype, int32_t epilogue, int32_t N, int32_t K, int32_t M, int32_t tile);
/* The tile the library uses for a projection of M x N x K (operands row-major with lda = ldb = K;
 * epilogue 0 store, 1 FP32 add, 2 SwiGLU, 3 rotary, which takes the store tuning): the tuning
 * table's tile for (dtype, epilogue, N, K, floor(log2 M)), else the built-in default for M.
 * Host state only, no device needed.  -1 for arguments out of range. */
int32_t kvop_gemm_pick_tile(int32_t dtype, int32_t epilogue, int32_t M, int32_t N, int32_t K);
/* Attention kernel used for BF16 compute with a BF16 or FP8 cache and head_dim 64 or 128
 * (all other cases use the register-staged kernel): -1 = register-staged key/value tiles;
 * 0, 1, 2 = tiles fetched by direct global -> LDS loads with 64-key tiles and 2 stages,
 * 64-key tiles and 3 stages, 32-key tiles and 3 stages (the default; head_dim 64 uses
 * 64-key tiles for 2).  Process-wide; EINVAL outside -1 .. 2.  Results agree within the stated
 * bounds; variants with 64-key tiles give the register-staged kernel's results exactly for
 * a BF16 cache. */
kvop_status kvop_set_attention_kernel(int32_t variant);
int32_t kvop_get_attention_kernel(void);
/* Widen n FP8 (E4M3 fn) codes (device bytes) to BF16 bit patterns (device uint16) with the
 * conversion the direct-load attention kernels apply to FP8 cache rows.  n > 0, a multiple
 * of 8 (EINVAL otherwise).  Asynchronous on stream. */
kvop_status kvop_debug_fp8_to_bf16(const uint8_t* codes_dev, int32_t n, uint16_t* out_dev, void* stream);
/* Copy the cached keys (kv = 0) or values (kv = 1) of one document, one layer and one
 * kv head into out_dev as FP32 [L, head_dim] (FP8 entries decoded and scaled). */
kvop_status kvop_debug_read_cache(kvop_pool* pool, kvop_handle handle, int32_t layer, int32_t kv_head, int32_t kv,
                                  float* out_dev, void* stream);

/* ---- plan optimizer over profiled log-odds (host only; no device work) -----------------
 * Section 4.1: every logical filter is a cascade of candidate physical operators in cost
 * order (here typically the same filter over cache profiles of increasing retention).  The
 * choice of operators and their thresholds is relaxed -- pick factor sigmoid(s / tau), soft
 * decision softmax([LO - theta+, theta- - LO, 0] / tau) -- so Eqs. 1-4 carry soft accept /
 * reject / unsure values and a soft cost; Eqs. 5-7 count TP / FP / FN against the gold plan
 * (every filter's most expensive operator; Section 4.2: a tuple passes iff every filter
 * accepts it); Eqs. 8-9 give the Beta(1 + TP, 1 + FN) and Beta(1 + TP, 1 + FP) lower bounds
 * l with P(X >= l) = alpha; Eqs. 10-13 give the loss cost / (|S| sum c) + beta ReLU(T_P -
 * l_P) + beta ReLU(T_R - l_R), minimised by Adam (0.9, 0.999, 1e-8) while tau falls
 * exponentially from tau0 to tau_end.  The plan is read at tau = 0: an operator is selected
 * iff s > 0; thresholds with theta+ < theta- collapse to their midpoint.  A tuple still unsure
 * after a filter's last selected operator is not accepted.
 * Parameters are laid out per operator (s, theta+, theta-), filters in order; pick scores
 * start at 0 and thresholds at +theta0 / -theta0.  All arrays are host memory owned by the
 * caller.  Errors: EINVAL for empty or inconsistent problems (no filter, a filter without
 * operators or with more than 64, a cost <= 0, non-finite log-odds, alpha outside (0, 1),
 * targets outside [0, 1]) and bad options. */
typedef struct kvop_plan_problem {
  int32_t n_filters;             /* logical filters, 1..64 */
  const int32_t* n_ops;          /* [n_filters] candidate operators of every filter, 1..64 */
  const double* cost;            /* [n_total] per-tuple cost of every operator, > 0 */
  const float* log_odds;         /* [n_total][n_tuples] profiled log-odds, operator-major */
  const int8_t* gold;            /* [n_filters][n_tuples] 1 iff the filter's gold operator accepts */
  int32_t n_tuples;              /* profiling sample size |S| >= 1 */
  double target_recall, target_precision;  /* T_R, T_P in [0, 1] */
  double alpha;                  /* credible level in (0, 1) */
} kvop_plan_problem;

typedef struct kvop_plan_opts {
  int32_t steps;                 /* Adam steps >= 1 */
  double lr;                     /* Adam step size > 0 */
  double beta;                   /* constraint weight >= 0 */
  double tau0, tau_end;          /* temperature at the first and the last step, tau0 >= tau_end > 0 */
  double theta0;                 /* initial thresholds +theta0 / -theta0 */
} kvop_plan_opts;

typedef struct kvop_plan_report {
  double tp, fp, fn;             /* Eqs. 5-7 of the discrete plan on the sample */
  double recall_lb, precision_lb;  /* Eqs. 8-9 */
  double cost_frac;              /* Eq. 10's cost term of the discrete plan */
} kvop_plan_report;

/* Optimise.  Outputs: params_out[3 n_total] (nullable) the final relaxed parameters;
 * selected_out[n_total], theta_pos_out / theta_neg_out[n_total] the plan at tau = 0;
 * loss_trace_out[steps] (nullable) the loss at every step before its update; report_out
 * (nullable) the discrete plan evaluated on the sample. */
kvop_status kvop_plan_optimize(const kvop_plan_problem* problem, const kvop_plan_opts* opts, double* params_out,
                               int8_t* selected_out, float* theta_pos_out, float* theta_neg_out,
                               double* loss_trace_out, kvop_plan_report* report_out);

/* The relaxed loss at parameters params[3 n_total] and temperature tau > 0, and its exact
 * gradient into grad_out[3 n_total] (nullable). */
kvop_status kvop_plan_loss(const kvop_plan_problem* problem, const double* params, double tau, double beta,
                           double* loss_out, double* grad_out);

/* A discrete plan on the sample: report, and per operator the inter-operator selectivity
 * (fraction of the sample it does not reject), the intra-operator selectivity (fraction it
 * leaves unsure) -- both over the whole sample, as Section 4.2 defines them -- the tuples it
 * processes in its cascade (0 if not selected), and per tuple whether the plan accepts it.
 * Every output is nullable.  Decisions compare the FP32 log-odds with the FP32 thresholds,
 * as kvop_op_eval does. */
kvop_status kvop_plan_evaluate(const kvop_plan_problem* problem, const int8_t* selected, const float* theta_pos,
                               const float* theta_neg, kvop_plan_report* report_out, double* sel_inter_out,
                               double* sel_intra_out, int32_t* processed_out, int8_t* accept_out);

/* Operator ordering (Section 4.2, Algorithm 1): n_ops (1..20) physical operators, impl[i] the
 * logical operator (0..63) of operator i; running operator i costs cost[i] per pending tuple of
 * its logical operator, then keeps the sel_intra[i] fraction of them pending and the
 * sel_inter[i] fraction of every other logical operator's.  The subset dynamic programme
 * keeps, per subset, the cheapest way to have run exactly it.  Writes the order (operator
 * indices) and its cost for n_tuples initial tuples. */
kvop_status kvop_plan_reorder(int32_t n_ops, const int32_t* impl, const double* cost, const double* sel_inter,
                              const double* sel_intra, double n_tuples, int32_t* order_out, double* cost_out);

/* Eqs. 8-9's bound: l with P(X >= l) = alpha for X ~ Beta(a, b); a, b > 0, alpha in (0, 1). */
kvop_status kvop_beta_lower_bound(double a, double b, double alpha, double* out);

#ifdef __cplusplus
}
#endif

#endif /* KVOP_H */
