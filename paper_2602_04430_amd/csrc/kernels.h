// Launchers of the gfx950 kernels (host side).  Each returns hipSuccess or the first
// HIP error of its launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace kvop {

enum Dt { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };
enum Epi { EPI_STORE = 0, EPI_ADD = 1, EPI_SWIGLU = 2, EPI_ROPE = 3 };

// ---------------------------------------------------------------- GEMM (C = A B^T)
// A [M, K] (lda), B [N, K] (ldb), both in `dt` (f32 or bf16); FP32 accumulation.
//   EPI_STORE : C[M, N] (ldc) in `out_dt`
//   EPI_ADD   : C (FP32) += A B^T           (residual add)
//   EPI_SWIGLU: B rows interleaved in blocks of 16 (16 gate rows, then the 16 matching
//               up rows); C[M, N/2] (ldc) in `out_dt` = silu(gate) * up
//   EPI_ROPE  : BF16 only: C[M, N] in BF16, then the rotary embedding of the D-wide heads in
//               columns [0, rot_cols) at each row's position (pairs (i, i + D/2)), applied
//               to the BF16-rounded products exactly as rope_qk applies it; joins also get
//               the query columns [0, q_cols) rotated at position - shift[row] into q_alt
//               (same layout) where shift[row] >= 0
struct GemmShape {
  int M, N, K;
  int64_t lda, ldb, ldc;
};
struct RopeEpi {
  const int32_t* pos;                  // position of each output row
  const float* cos_t;                  // [position][D/2]
  const float* sin_t;
  int D, rot_cols, q_cols;
  void* q_alt;                         // may be null
  const int32_t* shift;
  int pos_stride;                      // row r's position and shift at index r * pos_stride (0: 1)
};
// Tile configurations (autotuner candidates); see gemm.hip.
int gemm_num_tiles(int dt);
const char* gemm_tile_name(int dt, int tile);
bool gemm_tile_ok(int dt, int tile, const GemmShape& s, int epi);
hipError_t gemm(int dt, int out_dt, int epi, int tile, const void* A, const void* B, void* C, const GemmShape& s,
                hipStream_t st, const RopeEpi* rope = nullptr);
// head dims the rotary epilogue serves (whole heads in every BF16 tile, 8-pair groups)
bool gemm_rope_supported(int D);
// default tile for a shape (from the tuned table when present)
int gemm_pick_tile(int dt, int epi, const GemmShape& s);
void gemm_set_tuned(int dt, int epi, int N, int K, int mbucket, int tile);
int gemm_mbucket(int M);
// tuning table as text lines "dtype epilogue N K mbucket tile_name"
std::string gemm_tuned_export();
bool gemm_tuned_import_line(int dt, int epi, int N, int K, int mb, const std::string& name);

// ---------------------------------------------------------------- attention
// One work item = one (query block, key sources) unit; executed for every kv head.
struct AttnWork {
  int64_t off_a;      // byte offset of document A's cache region in the pool (-1: none)
  int64_t off_b;      // byte offset of document B's region (join), -1 if none
  int64_t idx_a;      // offset of A's retained list in the index array, -1 = rows 0..n_a-1
  int64_t idx_b;      // offset of B's retained list, -1 = rows 0..n_b-1
  int32_t L_a, L_b;   // document lengths (region layout; B's key positions are L_a + p)
  int32_t n_a, n_b;   // keys taken from A and B
  int32_t q_row0;     // activation row of query position 0 of this item
  int32_t q_pos0;     // absolute position of query position 0
  int32_t n_q;        // query positions in this item (<= Pmax)
  int32_t own_row0;   // first own row (suffix/generated keys) in the own-row buffer
  int32_t n_own;      // own keys; own key j sits at position own_pos0 + j
  int32_t own_pos0;
  int32_t pad_a;      // padded batching: keys of A iterated (>= n_a; keys past n_a are loaded,
                      // multiplied and masked); 0 = n_a.  Direct-load kernels only.
};

struct AttnArgs {
  const AttnWork* work;
  int n_work;
  const uint8_t* pool;
  const int32_t* idx;
  const void* q;       // queries [rows][q_stride], head hq at column hq*D (rotated)
  const void* q_alt;   // join: queries rotated at (position - L_a), same layout; may be null
  int64_t q_stride;
  const void* own;     // own keys/values [rows][own_stride]; k of kv head h at own_kcol + h*D
  int64_t own_stride;
  int own_kcol, own_vcol;
  void* out;           // [rows][out_stride], head hq at column hq*D
  int64_t out_stride;
  int layer, n_layers, Hkv, G, Pmax;
  float scale_log2;    // log2(e) / sqrt(D)
  int* counter;        // persistent launch: unit counter (zeroed before the launch), else null
  int persistent_wgs;  // persistent launch: number of workgroups (register-staged kernel)
  int n_cu;            // persistent launch: compute units; the direct-load kernels launch as
                       // many workgroups as fit on them at once
  int decode;          // 1: a decoding step (one query position per item, no document B); the
                       // streaming decode kernel serves it where it supports the shape
};
// cdt: compute/query dtype (f32 or bf16); kvdt: cache dtype (f32 with f32; bf16/fp8 with bf16)
hipError_t attention(int cdt, int kvdt, int D, const AttnArgs& a, hipStream_t st);
// Decoding step (Pmax = 1, no document B), BF16 compute: keys and values streamed from HBM
// into registers, G query heads of one kv head per workgroup (G in {1, 2, 4}, D in {64, 128})
bool attention_decode_ok(int kvdt, int D, int G);
hipError_t attention_decode(int kvdt, int D, const AttnArgs& a, hipStream_t st);
// BF16 compute with a BF16 or FP8 cache, D in {64, 128}: tiles fetched by direct global->LDS
// loads.  variant: 0 = 64-key tiles / 2 stages, 1 = 64 / 3, 2 = 32 / 3.
hipError_t attention_dma(int kvdt, int D, int variant, const AttnArgs& a, hipStream_t st);
// FP8 (E4M3) codes -> BF16 bits with the conversion the direct-load kernels use (n % 8 == 0)
hipError_t fp8_widen(const uint8_t* codes, uint16_t* out, int n, hipStream_t st);
// whether attention() runs the direct-load kernels for this combination (they alone honour pad_a)
bool attention_is_dma(int cdt, int kvdt, int D);
// attention kernel used by attention(): -1 = register-staged, else the attention_dma variant
void attention_set_impl(int impl);
int attention_get_impl();

// ---------------------------------------------------------------- expected-attention compression
// One layer of a prefill chunk (rows of nd documents, chunk-relative row offsets row_off[nd+1],
// qkv = the QKV projection before rotation, dt f32 or bf16, row stride ld): e_ws [rows][H]
// receives every key's expected log-weight per query head, then acc [rows][Hkv] += the
// layer's normalised contributions.  order[nd]: the documents in the order their workgroups
// are launched (longest first); items[n_items][3]: (document, first key, key count) segments
// of the log-weight pass, longest documents first.  Documents need L + n_future <= the rotary
// table length.
hipError_t ea_layer(int dt, int D, const void* qkv, int64_t ld, int H, int Hkv, const int64_t* row_off,
                    const int32_t* order, int nd, const int32_t* items, int n_items, int n_future,
                    const float* cos_tab, const float* sin_tab, float* e_ws, float* acc, hipStream_t st);
hipError_t ea_zero(float* p, int64_t n, hipStream_t st);
// out[row] = sum over kv heads of acc[row][g]
hipError_t ea_finish(const float* acc, int Hkv, int rows, float* out, hipStream_t st);
// per document d (scores rows doc_off[d] .. doc_off[d+1]): the kcount[d] highest scores, equal
// scores lower row first, ascending document-relative rows written at idx + out_off[d]
hipError_t ea_select(const float* scores, const int64_t* doc_off, const int32_t* kcount, const int64_t* out_off,
                     int n_docs, int32_t* idx, hipStream_t st);

// ---------------------------------------------------------------- elementwise / small kernels
// x[row] = embed[tok[row]] (embed in `dt`), FP32 output; ids clamped to [0, V)
hipError_t embed_rows(int dt, const void* embed, const int32_t* tok, int n_rows, int d, int vocab, float* x,
                      hipStream_t st);
// embed rows with per-row token ids (tok[row]); ids clamped to [0, V)
// embed rows whose token is suffix[row % S] (op_eval input)
hipError_t embed_suffix(int dt, const void* embed, const int32_t* suffix, int S, int n_rows, int d, int vocab,
                        float* x, hipStream_t st);
// y[row] = rmsnorm(x[row]) * g, x FP32 with row stride ldx, y in `dt` with stride ldy
hipError_t rmsnorm_rows(int dt, const float* x, int64_t ldx, const float* g, int n_rows, int d, float eps, void* y,
                        int64_t ldy, hipStream_t st);
// rotary embedding in place on q heads and k heads of a qkv buffer (dt), row positions
// pos[row]; when q_alt != null also writes q rotated at pos[row] - alt_shift[row] into q_alt
// BF16 rows r < n_rows of dst [.][ld] from src row r % src_rows (same layout): columns below
// rot_cols rotated at pos[r] as the projection's rotary epilogue rotates them, the rest
// copied; joins: query columns (below q_cols) also rotated at pos[r] - shift[r] into q_alt
// where shift[r] >= 0
hipError_t rope_broadcast(const void* src, int src_rows, void* dst, int64_t ld, int n_rows, int n_cols, int rot_cols,
                          int q_cols, int D, const int32_t* pos, const float* cos_tab, const float* sin_tab, void* q_alt,
                          const int32_t* shift, hipStream_t st);
hipError_t rope_qk(int dt, void* qkv, int64_t ld, int n_rows, int H, int Hkv, int D, const int32_t* pos,
                   const float* cos_tab, const float* sin_tab, void* q_alt, const int32_t* alt_shift,
                   hipStream_t st);
// kv_build: rotate q (in place) and k of document rows and write k, v into the cache
struct KvBlock {      // 16 consecutive rows of one document
  int64_t off;        // document region byte offset
  int32_t L;          // document length
  int32_t p0;         // first position of the block
  int32_t row0;       // activation row of position p0
  int32_t pad;
};
hipError_t rope_write_kv(int dt, int kvdt, void* qkv, int64_t ld, const KvBlock* blocks, int n_blocks, int H,
                         int Hkv, int D, int layer, int n_layers, const float* cos_tab, const float* sin_tab,
                         uint8_t* pool, hipStream_t st);
// map decode bookkeeping: copy k, v of rows into a per-layer own-row buffer
hipError_t copy_kv_rows(int dt, const void* qkv, int64_t ld, int kcol, int n_cols, const int32_t* src_rows,
                        const int32_t* dst_rows, int n, void* dst, int64_t ldd, hipStream_t st);
// pooled[doc] = mean over the document's rows of rmsnorm(x)*g (FP32); row_off[n_docs+1]
// are row offsets into x; inv_scratch holds n_rows floats
hipError_t pooled_mean(const float* x, int d, const int64_t* row_off, int n_docs, int n_rows, const float* g,
                       float eps, float* inv_scratch, float* pooled, hipStream_t st);
// filter/join head: y = rmsnorm(x[row_of_item]) * g; logits (yes, no); log-odds decision
// item i of the launch reads row in_rows[i] of x (or row i when in_rows is null) and writes
// output row out_rows[i]
hipError_t head_filter(int dt, const float* x, int64_t ldx, int n_items, int d, const float* g, float eps,
                       const void* head, int yes_id, int no_id, float th_pos, float th_neg, const int32_t* in_rows,
                       const int32_t* out_rows, float* logits, int8_t* decision, hipStream_t st);
// map head: logits over [lo, lo+n) and argmax (lowest id on ties); the argmax id goes to
// tok_out[out_row * ld_tok] and, when next_tok is set, to next_tok[out_row] (next_by_out) or
// next_tok[item]
hipError_t head_map(int dt, const float* x, int64_t ldx, int n_items, int d, const float* g, float eps,
                    const void* head, int lo, int n, const int32_t* in_rows, const int32_t* out_rows, float* logits,
                    int64_t ld_logits, int32_t* tok_out, int64_t ld_tok, int32_t* next_tok, bool next_by_out,
                    hipStream_t st);
// index-list validation: counts lists that are unsorted or out of range into *bad
struct ListCheck {
  int64_t off;
  int32_t n, L;
};
hipError_t validate_lists(const int32_t* idx, const ListCheck* lists, int n_lists, int* bad, hipStream_t st);
// counts, into *bad, the wavefronts that saw a token id outside [0, vocab)
hipError_t validate_tokens(const int32_t* tok, int64_t n, int vocab, int* bad, hipStream_t st);
// weight conversion: dst (dt) = src (f32); for interleave16 != 0 the rows of two [F, d]
// matrices (src, src2) are interleaved in blocks of 16
hipError_t convert_weights(int dt, const float* src, const float* src2, int64_t rows, int64_t cols, void* dst,
                           int interleave16, hipStream_t st);
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
// decode L rows of one cached (layer, head, K or V) block to FP32
hipError_t read_cache(int kvdt, const uint8_t* region, int L, int D, int layer, int n_layers, int Hkv, int h, int kv,
                      float* out, hipStream_t st);

// ---------------------------------------------------------------- learned proxy
hipError_t proxy_stats(const float* F, int64_t n, int d, float* mean, float* istd, hipStream_t st);
hipError_t proxy_gather(const float* F, int d, const int32_t* rows, int B, const float* mean, const float* istd,
                        uint16_t* x, uint16_t* xT, hipStream_t st);
hipError_t proxy_head_infer(const float* h1, int n, int H, const float* b1, const float* W2, const float* b2,
                            float tau, int8_t* cls, float* conf, int8_t* answered, hipStream_t st);
hipError_t proxy_head_train(const float* h1, int B, int H, const float* b1, const float* W2, const float* b2,
                            const int32_t* labels, const int32_t* rows, float* a, float* dz, float* dh1, uint16_t* dh1T,
                            float* loss_row, hipStream_t st);
hipError_t proxy_reduce(const float* a, const float* dz, const float* dh1, const float* loss_row, int B, int H,
                        float* g_b1, float* g_w2, float* g_b2, float* loss, hipStream_t st);
hipError_t proxy_adam(float* p, const float* g, float* m, float* v, int64_t n, int64_t n_w1, uint16_t* w1b, float lr,
                      float beta1, float beta2, float eps, int step, hipStream_t st);
hipError_t f32_to_bf16(const float* s, uint16_t* d, int64_t n, hipStream_t st);

}  // namespace kvop
