// Host side of the C ABI: model weights, the cache pool (a first-fit allocator of
// contiguous per-document regions with generation-tagged handles), the offline prefill
// (kv_build) and the online operator evaluation (op_eval) for filter, map and join.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/kvop.h"
#include "host_util.h"
#include "kernels.h"

using namespace kvop;

namespace {

constexpr int kRopeMaxPos = 65536;
constexpr int64_t kAlign = 256;
int64_t g_wave_rows = 131072;  // suffix rows per op_eval / mixed wave

// ---- optional per-kernel-class timing: HIP events recorded on the caller's stream around
// each launch while profiling is on; read back (synchronising) by kvop_profile_stop.
enum ProfClass { PC_GEMM_QKV, PC_GEMM_O, PC_GEMM_GATEUP, PC_GEMM_DOWN, PC_ATTENTION, PC_ROPE_KV, PC_RMSNORM,
                 PC_EMBED, PC_HEAD, PC_DECODE, PC_EA, PC_OTHER, PC_COUNT };
// map_decode: one whole greedy decode step (all layers) of a map operator
const char* kProfNames[PC_COUNT] = {"gemm_qkv", "gemm_o", "gemm_gate_up", "gemm_down", "attention", "rope_kv",
                                    "rmsnorm", "embed", "head", "map_decode", "ea_scores", "other"};
struct Prof {
  bool on = false;
  bool capturing = false;  // no event records while a graph is being captured
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[PC_COUNT] = {};
  int64_t cnt[PC_COUNT] = {};
  std::vector<double> launches[PC_COUNT];  // per-launch milliseconds, in launch order
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
Prof g_prof;
struct ProfScope {
  int k;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int k_, hipStream_t st_) : k(k_), st(st_) {
    if (g_prof.on && !g_prof.capturing) { a = g_prof.get(); b = g_prof.get(); (void)hipEventRecord(a, st); }
  }
  ~ProfScope() {
    if (a) { (void)hipEventRecord(b, st); g_prof.pending.push_back({k, {a, b}}); }
  }
};

// Pinned host staging with an event guarding its reuse.
struct HostStage {
  char* p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
  hipError_t reserve(size_t bytes) {
    if (pending) {
      hipError_t e = hipEventSynchronize(ev);
      if (e != hipSuccess) return e;
      pending = false;
    }
    if (!ev) {
      hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipHostFree(p);
    size_t want = std::max(bytes, cap * 2);
    hipError_t e = hipHostMalloc((void**)&p, want, hipHostMallocDefault);
    if (e != hipSuccess) { p = nullptr; cap = 0; return e; }
    cap = want;
    return hipSuccess;
  }
  ~HostStage() {
    if (ev) { (void)hipEventSynchronize(ev); (void)hipEventDestroy(ev); }
    if (p) (void)hipHostFree(p);
  }
};

// Bump layout of one host staging area mirrored into one device area.
struct Mirror {
  std::vector<size_t> offs;
  size_t size = 0;
  size_t add(size_t bytes) {
    size_t o = size;
    size = align_up(size + bytes, 64);
    offs.push_back(o);
    return o;
  }
};

}  // namespace

// ================================================================== model
struct kvop_model {
  kvop_model_cfg cfg;
  int dt;
  struct Layer {
    float* attn_norm;
    float* ffn_norm;
    void* wqkv;
    void* wo;
    void* wgu;
    void* wdown;
  };
  std::vector<Layer> layers;
  void* embed = nullptr;
  void* head = nullptr;
  float* final_norm = nullptr;
  float* cos_tab = nullptr;
  float* sin_tab = nullptr;
  std::vector<void*> allocs;
  // workspaces shared by kv_build and op_eval (calls on one model are serialised)
  DevBuf ws;
  DevBuf meta;
  DevBuf ea;  // expected-attention workspace of kvop_kv_build_scored
  HostStage stage;
  int* dflag = nullptr;   // [0]: list-validation count, [16]: persistent-attention unit counter
  int* hflag = nullptr;
  int n_cu = 0;
  hipStream_t cap_stream = nullptr;  // graph capture (the legacy null stream cannot be captured)
  // completion of the last call that used the workspaces, and the stream it ran on
  hipEvent_t done_ev = nullptr;
  hipStream_t last_stream = nullptr;
  bool done_recorded = false;

  int qkv_cols() const { return (cfg.n_heads + 2 * cfg.n_kv_heads) * cfg.head_dim; }
  int esz() const { return dt == DT_F32 ? 4 : 2; }
  ~kvop_model() {
    if (done_ev) { (void)hipEventSynchronize(done_ev); (void)hipEventDestroy(done_ev); }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
    if (dflag) (void)hipFree(dflag);
    if (hflag) (void)hipHostFree(hflag);
  }
};

namespace {
// Calls on one model share its workspaces (activations, metadata, flags) and its pools'
// freed regions.  A call enqueued on another stream than the previous call first waits for
// that call's completion event, so nothing it overwrites is still being read.  Constructed
// before a call's first enqueue; the destructor records the call's completion.
struct CallOrder {
  kvop_model* m;
  hipStream_t st;
  CallOrder(kvop_model* m_, hipStream_t st_) : m(m_), st(st_) {
    if (m->done_recorded && m->last_stream != st) (void)hipStreamWaitEvent(st, m->done_ev, 0);
  }
  ~CallOrder() {
    if (!m->done_ev && hipEventCreateWithFlags(&m->done_ev, hipEventDisableTiming) != hipSuccess) {
      m->done_ev = nullptr;
      return;
    }
    m->done_recorded = hipEventRecord(m->done_ev, st) == hipSuccess;
    m->last_stream = st;
  }
};
}  // namespace

struct DocSlot {
  uint64_t off = 0, bytes = 0;
  int32_t L = 0;
  uint32_t gen = 0;
  bool live = false;
};

struct kvop_pool {
  kvop_model* m;
  int kvdt;
  uint8_t* base = nullptr;
  uint64_t cap = 0, used = 0;
  uint32_t id;
  std::map<uint64_t, uint64_t> free_list;  // offset -> size
  std::vector<DocSlot> slots;
  std::vector<uint32_t> free_slots;
  int live = 0;
};

namespace {

std::atomic<uint32_t> g_pool_ids{1};

int kv_esz(int kvdt) { return kvdt == DT_F32 ? 4 : (kvdt == DT_BF16 ? 2 : 1); }

uint64_t doc_bytes(const kvop_pool* p, int64_t L) {
  const kvop_model_cfg& c = p->m->cfg;
  int64_t elems = 2LL * c.n_layers * c.n_kv_heads * L * c.head_dim;
  int64_t b = elems * kv_esz(p->kvdt);
  if (p->kvdt == DT_FP8) b += 2LL * c.n_layers * c.n_kv_heads * ((L + 15) / 16) * 4;
  return (uint64_t)align_up(b, kAlign);
}

bool pool_alloc(kvop_pool* p, uint64_t bytes, uint64_t* off) {
  for (auto it = p->free_list.begin(); it != p->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      uint64_t rest = it->second - bytes, noff = it->first + bytes;
      p->free_list.erase(it);
      if (rest) p->free_list[noff] = rest;
      p->used += bytes;
      return true;
    }
  }
  return false;
}

void pool_free(kvop_pool* p, uint64_t off, uint64_t bytes) {
  p->used -= bytes;
  auto it = p->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != p->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    p->free_list.erase(nx);
  }
  if (it != p->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      p->free_list.erase(it);
    }
  }
}

kvop_handle make_handle(const kvop_pool* p, uint32_t slot, uint32_t gen) {
  return ((uint64_t)(p->id & 0xffff) << 48) | ((uint64_t)(gen & 0xffff) << 32) | slot;
}

const DocSlot* lookup(const kvop_pool* p, kvop_handle h) {
  uint32_t pid = (uint32_t)(h >> 48), gen = (uint32_t)((h >> 32) & 0xffff), slot = (uint32_t)(h & 0xffffffffu);
  if (pid != (p->id & 0xffff) || slot >= p->slots.size()) return nullptr;
  const DocSlot& s = p->slots[slot];
  if (!s.live || (s.gen & 0xffff) != gen) return nullptr;
  return &s;
}

int64_t retained_count(float r, int64_t L) {
  int64_t rm = (int64_t)std::llround((double)r * 1000.0);
  int64_t k = (rm * L + 500) / 1000;
  return std::min(std::max(k, std::min<int64_t>(4, L)), L);
}

struct LayerBufs {
  float* x;
  void* h;
  void* qkv;
  void* qalt;
  void* attn;
  void* act;
};

// Rows that continue past the attention: r*stride + off for r < n.
struct SelGroup {
  int n, stride, off;
};
constexpr int kMaxSelGroups = 8;

// Plan of one decoder layer over `rows` activation rows.  Only the rows of the selection
// groups continue past the attention (the K/V of every row are still produced): the last
// layer of op_eval continues with the last suffix row of each item only.
struct LayerPlan {
  int rows;
  const int32_t* pos;
  const int32_t* alt_shift;  // joins: q_alt rotation shift per row (-1: none); may be null
  AttnArgs attn;             // work list etc. (q/out/own filled by run_layer)
  bool own_from_qkv;         // own keys are the rows of this pass
  const void* own;           // otherwise: explicit own buffer
  int64_t own_stride;
  int own_kcol, own_vcol;
  int n_groups;                    // selection groups (all rows: one group {rows, 1, 0})
  SelGroup sel[kMaxSelGroups];
  // expected-attention scoring during prefill (off when ea_row_off is null)
  const int64_t* ea_row_off = nullptr;
  const int32_t* ea_order = nullptr;
  const int32_t* ea_items = nullptr;
  int ea_nd = 0, ea_n_items = 0, ea_n_future = 0;
  float* ea_e = nullptr;
  float* ea_acc = nullptr;
  // blocks of rows that repeat every `period` rows before the rotation (layer 0: every item of
  // an operator starts from the embeddings of that operator's suffix), so each block's first
  // period rows are normalised and projected once; the blocks cover every row
  struct SharedBlock {
    int row0, rows, period;
  };
  SharedBlock shared[kMaxSelGroups];
  int n_shared = 0;
  // > 0: only the last of every q_last rows continues (the last layer of one operator), so
  // queries are projected for those rows only (keys and values for all: that row sees them)
  int q_last = 0;
  void select_all() { n_groups = 1; sel[0] = SelGroup{rows, 1, 0}; }
  void select_one(int n, int stride, int off) { n_groups = 1; sel[0] = SelGroup{n, stride, off}; }
};

// skip_tail: stop once this layer's keys/values exist (prefill's last layer when the final
// hidden states are not needed)
kvop_status run_layer(kvop_model* m, int l, const LayerBufs& b, LayerPlan& lp, uint8_t* pool, int kvdt,
                      const KvBlock* kvblocks, int n_kvblocks, hipStream_t st, bool skip_tail = false) {
  const kvop_model_cfg& c = m->cfg;
  const kvop_model::Layer& W = m->layers[l];
  const int d = c.d_model, H = c.n_heads, Hkv = c.n_kv_heads, D = c.head_dim, F = c.d_ffn;
  const int qc = m->qkv_cols();
  const int rows = lp.rows;
  const int dt = m->dt;
  // BF16 suffix rows: the rotation of queries and keys is fused into the projection's epilogue
  // (prefill keeps it separate: expected-attention scoring reads the unrotated queries, and
  // the keys are rotated by the cache writer)
  const bool fuse_rope = dt == DT_BF16 && n_kvblocks == 0 && !lp.ea_row_off && gemm_rope_supported(D);
  // rows shared by every item of a block: normalise and project them once (into the attention
  // output buffer, free until the attention runs), then copy them to every item rotated at its
  // positions; the result equals the per-row path bit for bit
  const int e = m->esz();
  bool shared = fuse_rope && lp.n_shared > 0;
  {
    int64_t covered = 0, periods = 0;
    for (int i = 0; i < lp.n_shared; i++) {
      const LayerPlan::SharedBlock& sb = lp.shared[i];
      if (sb.period < 1 || sb.rows < 0 || sb.rows % sb.period) shared = false;
      covered += sb.rows;
      periods += sb.period;
    }
    if (covered != rows || periods * qc > (int64_t)rows * H * D) shared = false;
  }
  const int qlast = fuse_rope && !shared && lp.q_last > 0 && rows % lp.q_last == 0 ? lp.q_last : 0;
  {
    ProfScope ps(PC_RMSNORM, st);
    if (shared) {
      for (int i = 0; i < lp.n_shared; i++) {
        const LayerPlan::SharedBlock& sb = lp.shared[i];
        if (sb.rows == 0) continue;
        HIPTRY(rmsnorm_rows(dt, b.x + (int64_t)sb.row0 * d, d, W.attn_norm, sb.period, d, c.rms_eps,
                            (char*)b.h + (int64_t)sb.row0 * d * e, d, st));
      }
    } else {
      HIPTRY(rmsnorm_rows(dt, b.x, d, W.attn_norm, rows, d, c.rms_eps, b.h, d, st));
    }
  }
  {
    ProfScope ps(PC_GEMM_QKV, st);
    GemmShape s{rows, qc, d, d, d, qc};
    if (shared) {
      int64_t off = 0;
      for (int i = 0; i < lp.n_shared; i++) {
        const LayerPlan::SharedBlock& sb = lp.shared[i];
        if (sb.rows == 0) continue;
        GemmShape sg{sb.period, qc, d, d, d, qc};
        HIPTRY(gemm(dt, dt, EPI_STORE, gemm_pick_tile(dt, EPI_STORE, sg), (const char*)b.h + (int64_t)sb.row0 * d * e,
                    W.wqkv, (char*)b.attn + off * qc * e, sg, st));
        off += sb.period;
      }
    } else if (qlast) {
      const int nq = rows / qlast;
      // keys and values of every row (output columns H D .. qc; keys rotated)
      GemmShape kv{rows, 2 * Hkv * D, d, d, d, qc};
      const RopeEpi rk{lp.pos, m->cos_tab, m->sin_tab, D, Hkv * D, 0, nullptr, nullptr, 1};
      HIPTRY(gemm(dt, dt, EPI_ROPE, gemm_pick_tile(dt, EPI_ROPE, kv), b.h,
                  (const char*)W.wqkv + (int64_t)H * D * d * e, (char*)b.qkv + (int64_t)H * D * e, kv, st, &rk));
      // queries of the last row of every item (rows q_last - 1, 2 q_last - 1, ...)
      GemmShape qs{nq, H * D, d, (int64_t)qlast * d, d, (int64_t)qlast * qc};
      const int64_t r0 = qlast - 1;
      const RopeEpi rq{lp.pos + r0, m->cos_tab, m->sin_tab, D, H * D, H * D,
                       lp.alt_shift ? (char*)b.qalt + r0 * qc * e : nullptr, lp.alt_shift ? lp.alt_shift + r0 : nullptr,
                       qlast};
      HIPTRY(gemm(dt, dt, EPI_ROPE, gemm_pick_tile(dt, EPI_ROPE, qs), (const char*)b.h + r0 * d * e, W.wqkv,
                  (char*)b.qkv + r0 * qc * e, qs, st, &rq));
    } else if (fuse_rope) {
      const RopeEpi re{lp.pos, m->cos_tab, m->sin_tab, D, (H + Hkv) * D, H * D, lp.alt_shift ? b.qalt : nullptr,
                       lp.alt_shift};
      HIPTRY(gemm(dt, dt, EPI_ROPE, gemm_pick_tile(dt, EPI_ROPE, s), b.h, W.wqkv, b.qkv, s, st, &re));
    } else {
      HIPTRY(gemm(dt, dt, EPI_STORE, gemm_pick_tile(dt, EPI_STORE, s), b.h, W.wqkv, b.qkv, s, st));
    }
  }
  if (lp.ea_row_off) {  // before the rotation: the statistics are of the pre-rotation queries
    ProfScope ps(PC_EA, st);
    HIPTRY(ea_layer(dt, D, b.qkv, qc, H, Hkv, lp.ea_row_off, lp.ea_order, lp.ea_nd, lp.ea_items, lp.ea_n_items,
                    lp.ea_n_future, m->cos_tab, m->sin_tab, lp.ea_e, lp.ea_acc, st));
  }
  if (n_kvblocks > 0) {
    ProfScope ps(PC_ROPE_KV, st);
    // prefill: rotate queries here; keys are rotated by the cache writer
    HIPTRY(rope_qk(dt, b.qkv, qc, rows, H, 0, D, lp.pos, m->cos_tab, m->sin_tab, nullptr, nullptr, st));
    HIPTRY(rope_write_kv(dt, kvdt, b.qkv, qc, kvblocks, n_kvblocks, H, Hkv, D, l, c.n_layers, m->cos_tab, m->sin_tab,
                         pool, st));
  } else if (shared) {
    ProfScope ps(PC_ROPE_KV, st);
    int64_t off = 0;
    for (int i = 0; i < lp.n_shared; i++) {
      const LayerPlan::SharedBlock& sb = lp.shared[i];
      if (sb.rows == 0) continue;
      const int64_t r0 = sb.row0;
      HIPTRY(rope_broadcast((char*)b.attn + off * qc * e, sb.period, (char*)b.qkv + r0 * qc * e, qc, sb.rows, qc,
                            (H + Hkv) * D, H * D, D, lp.pos + r0, m->cos_tab, m->sin_tab,
                            lp.alt_shift ? (char*)b.qalt + r0 * qc * e : nullptr,
                            lp.alt_shift ? lp.alt_shift + r0 : nullptr, st));
      off += sb.period;
    }
  } else if (!fuse_rope) {
    ProfScope ps(PC_ROPE_KV, st);
    HIPTRY(rope_qk(dt, b.qkv, qc, rows, H, Hkv, D, lp.pos, m->cos_tab, m->sin_tab, lp.alt_shift ? b.qalt : nullptr,
                   lp.alt_shift, st));
  }
  if (skip_tail) return KVOP_OK;
  AttnArgs a = lp.attn;
  a.q = b.qkv;
  a.q_alt = lp.alt_shift ? b.qalt : nullptr;
  a.q_stride = qc;
  if (lp.own_from_qkv) {
    a.own = b.qkv;
    a.own_stride = qc;
    a.own_kcol = H * D;
    a.own_vcol = (H + Hkv) * D;
  } else {
    a.own = lp.own;
    a.own_stride = lp.own_stride;
    a.own_kcol = lp.own_kcol;
    a.own_vcol = lp.own_vcol;
  }
  a.out = b.attn;
  a.out_stride = H * D;
  a.layer = l;
  a.n_layers = c.n_layers;
  a.Hkv = Hkv;
  a.G = H / Hkv;
  a.pool = pool;
  a.scale_log2 = (float)(1.4426950408889634 / std::sqrt((double)D));
  {
    ProfScope ps(PC_ATTENTION, st);
    if (a.counter) HIPTRY(fill_i32(a.counter, 0, 1, st));
    HIPTRY(attention(dt, kvdt, D, a, st));
  }
  // rows continuing: all, or strided selections (last row of each item)
  for (int gi = 0; gi < lp.n_groups; gi++) {
  const int n = lp.sel[gi].n;
  if (n <= 0) continue;
  const int64_t sa = (int64_t)lp.sel[gi].stride;
  const char* attn_sel = (const char*)b.attn + (int64_t)lp.sel[gi].off * H * D * m->esz();
  float* x_sel = b.x + (int64_t)lp.sel[gi].off * d;
  {
    ProfScope ps(PC_GEMM_O, st);
    GemmShape s{n, d, H * D, sa * H * D, H * D, sa * d};
    HIPTRY(gemm(dt, DT_F32, EPI_ADD, gemm_pick_tile(dt, EPI_ADD, s), attn_sel, W.wo, x_sel, s, st));
  }
  { ProfScope ps(PC_RMSNORM, st); HIPTRY(rmsnorm_rows(dt, x_sel, sa * d, W.ffn_norm, n, d, c.rms_eps, b.h, d, st)); }
  {
    ProfScope ps(PC_GEMM_GATEUP, st);
    GemmShape s{n, 2 * F, d, d, d, F};
    HIPTRY(gemm(dt, dt, EPI_SWIGLU, gemm_pick_tile(dt, EPI_SWIGLU, s), b.h, W.wgu, b.act, s, st));
  }
  {
    ProfScope ps(PC_GEMM_DOWN, st);
    GemmShape s{n, d, F, F, F, sa * d};
    HIPTRY(gemm(dt, DT_F32, EPI_ADD, gemm_pick_tile(dt, EPI_ADD, s), b.act, W.wdown, x_sel, s, st));
  }
  }
  return KVOP_OK;
}

size_t act_bytes(const kvop_model* m, int64_t rows, bool join) {
  const kvop_model_cfg& c = m->cfg;
  int e = m->esz();
  size_t b = 0;
  b += align_up(rows * c.d_model * 4, kAlign);                          // x
  b += align_up(rows * c.d_model * e, kAlign);                          // h
  b += align_up(rows * (int64_t)m->qkv_cols() * e, kAlign);             // qkv
  b += join ? align_up(rows * (int64_t)m->qkv_cols() * e, kAlign) : 0;  // q_alt (qkv layout)
  b += align_up(rows * (int64_t)c.n_heads * c.head_dim * e, kAlign);    // attn
  b += align_up(rows * (int64_t)c.d_ffn * e, kAlign);                   // act
  return b;
}

LayerBufs carve(kvop_model* m, char* base, int64_t rows, bool join) {
  const kvop_model_cfg& c = m->cfg;
  int e = m->esz();
  LayerBufs b{};
  char* p = base;
  b.x = (float*)p; p += align_up(rows * c.d_model * 4, kAlign);
  b.h = p; p += align_up(rows * c.d_model * e, kAlign);
  b.qkv = p; p += align_up(rows * (int64_t)m->qkv_cols() * e, kAlign);
  if (join) { b.qalt = p; p += align_up(rows * (int64_t)m->qkv_cols() * e, kAlign); }
  b.attn = p; p += align_up(rows * (int64_t)c.n_heads * c.head_dim * e, kAlign);
  b.act = p;
  return b;
}

}  // namespace

extern "C" {

const char* kvop_last_error(void) { return last_error().c_str(); }

int64_t kvop_weights_numel(const kvop_model_cfg* c) {
  if (!c) return -1;
  int64_t d = c->d_model, hd = c->head_dim, F = c->d_ffn;
  int64_t per = d + (int64_t)c->n_heads * hd * d + 2LL * c->n_kv_heads * hd * d + d * c->n_heads * hd + d +
                3LL * F * d;
  return per * c->n_layers + d + 2LL * c->vocab * d;
}

kvop_status kvop_model_create(const kvop_model_cfg* cfg, const float* w, int64_t n_weights, kvop_dtype compute,
                              void* stream, kvop_model** out) {
  if (!cfg || !w || !out) return fail(KVOP_EINVAL, "null argument");
  const kvop_model_cfg c = *cfg;
  if (c.n_layers < 1 || c.n_heads < 1 || c.n_kv_heads < 1 || c.n_heads % c.n_kv_heads)
    return fail(KVOP_EINVAL, "bad head configuration");
  if (c.head_dim != 32 && c.head_dim != 64 && c.head_dim != 128) return fail(KVOP_EINVAL, "head_dim must be 32/64/128");
  if (c.d_model % 64 || c.d_ffn % 64 || c.vocab < 2) return fail(KVOP_EINVAL, "d_model and d_ffn must be multiples of 64");
  if ((c.n_heads / c.n_kv_heads) > 64) return fail(KVOP_EINVAL, "group too large");
  if (compute != KVOP_F32 && compute != KVOP_BF16) return fail(KVOP_EINVAL, "bad compute dtype");
  if (n_weights != kvop_weights_numel(cfg)) return fail(KVOP_EINVAL, "weight count mismatch");
  hipStream_t st = (hipStream_t)stream;
  kvop_model* m = new (std::nothrow) kvop_model();
  if (!m) return fail(KVOP_ENOMEM, "host allocation");
  m->cfg = c;
  m->dt = compute == KVOP_F32 ? DT_F32 : DT_BF16;
  const int64_t d = c.d_model, H = c.n_heads, Hkv = c.n_kv_heads, D = c.head_dim, F = c.d_ffn, V = c.vocab;
  const int e = m->esz();
  auto dalloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    m->allocs.push_back(p);
    return p;
  };
  kvop_status st_ok = KVOP_OK;
  auto conv = [&](const float* src, const float* src2, int64_t rows, int64_t cols, void* dst, int inter) {
    if (st_ok == KVOP_OK && convert_weights(m->dt, src, src2, rows, cols, dst, inter, st) != hipSuccess)
      st_ok = fail(KVOP_EDEVICE, "weight conversion launch failed");
  };
  const float* p = w;
  for (int l = 0; l < c.n_layers; l++) {
    kvop_model::Layer L{};
    L.attn_norm = (float*)dalloc(d * 4);
    L.ffn_norm = (float*)dalloc(d * 4);
    L.wqkv = dalloc((H + 2 * Hkv) * D * d * e);
    L.wo = dalloc(d * H * D * e);
    L.wgu = dalloc(2 * F * d * e);
    L.wdown = dalloc(d * F * e);
    if (!L.attn_norm || !L.ffn_norm || !L.wqkv || !L.wo || !L.wgu || !L.wdown) {
      delete m;
      return fail(KVOP_ENOMEM, "weight allocation");
    }
    if (hipMemcpyAsync(L.attn_norm, p, d * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) st_ok = KVOP_EDEVICE;
    p += d;
    conv(p, nullptr, H * D, d, L.wqkv, 0);
    p += H * D * d;
    conv(p, nullptr, Hkv * D, d, (char*)L.wqkv + H * D * d * e, 0);
    p += Hkv * D * d;
    conv(p, nullptr, Hkv * D, d, (char*)L.wqkv + (H + Hkv) * D * d * e, 0);
    p += Hkv * D * d;
    conv(p, nullptr, d, H * D, L.wo, 0);
    p += d * H * D;
    if (hipMemcpyAsync(L.ffn_norm, p, d * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) st_ok = KVOP_EDEVICE;
    p += d;
    conv(p, p + F * d, F, d, L.wgu, 1);
    p += 2 * F * d;
    conv(p, nullptr, d, F, L.wdown, 0);
    p += d * F;
    m->layers.push_back(L);
  }
  m->final_norm = (float*)dalloc(d * 4);
  m->embed = dalloc(V * d * e);
  m->head = dalloc(V * d * e);
  if (!m->final_norm || !m->embed || !m->head) {
    delete m;
    return fail(KVOP_ENOMEM, "weight allocation");
  }
  if (hipMemcpyAsync(m->final_norm, p, d * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) st_ok = KVOP_EDEVICE;
  p += d;
  conv(p, nullptr, V, d, m->embed, 0);
  p += V * d;
  conv(p, nullptr, V, d, m->head, 0);
  // rotary tables, evaluated in double precision: angle(pos, i) = pos * theta^(-2i/D)
  {
    const int half = (int)D / 2;
    std::vector<float> ct((size_t)kRopeMaxPos * half), sn((size_t)kRopeMaxPos * half);
    for (int i = 0; i < half; i++) {
      double inv = std::pow((double)c.rope_theta, -2.0 * i / (double)D);
      for (int ps = 0; ps < kRopeMaxPos; ps++) {
        double a = (double)ps * inv;
        ct[(size_t)ps * half + i] = (float)std::cos(a);
        sn[(size_t)ps * half + i] = (float)std::sin(a);
      }
    }
    m->cos_tab = (float*)dalloc(ct.size() * 4);
    m->sin_tab = (float*)dalloc(sn.size() * 4);
    if (!m->cos_tab || !m->sin_tab) {
      delete m;
      return fail(KVOP_ENOMEM, "rope table allocation");
    }
    if (hipMemcpyAsync(m->cos_tab, ct.data(), ct.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess) st_ok = KVOP_EDEVICE;
    if (hipMemcpyAsync(m->sin_tab, sn.data(), sn.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess) st_ok = KVOP_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) st_ok = KVOP_EDEVICE;
  }
  {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (m->n_cu <= 0) m->n_cu = 256;
  }
  if (hipMalloc((void**)&m->dflag, 256) != hipSuccess || hipHostMalloc((void**)&m->hflag, 64, 0) != hipSuccess) {
    delete m;
    return fail(KVOP_ENOMEM, "flag allocation");
  }
  if (st_ok != KVOP_OK) {
    delete m;
    return fail(KVOP_EDEVICE, last_error().empty() ? "model upload failed" : last_error());
  }
  *out = m;
  return KVOP_OK;
}

kvop_status kvop_model_destroy(kvop_model* m) {
  if (!m) return fail(KVOP_EINVAL, "null model");
  (void)hipDeviceSynchronize();
  delete m;
  return KVOP_OK;
}

kvop_status kvop_pool_create(kvop_model* m, kvop_kv_dtype kvd, uint64_t bytes, kvop_pool** out) {
  if (!m || !out) return fail(KVOP_EINVAL, "null argument");
  int kvdt = kvd == KVOP_KV_F32 ? DT_F32 : (kvd == KVOP_KV_BF16 ? DT_BF16 : (kvd == KVOP_KV_FP8 ? DT_FP8 : -1));
  if (kvdt < 0) return fail(KVOP_EINVAL, "bad kv dtype");
  if (m->dt == DT_F32 && kvdt != DT_F32) return fail(KVOP_EINVAL, "an FP32 model keeps an FP32 cache");
  if (m->dt == DT_BF16 && kvdt == DT_F32) return fail(KVOP_EINVAL, "a BF16 model keeps a BF16 or FP8 cache");
  bytes = (uint64_t)align_up((int64_t)bytes, kAlign);
  if (bytes == 0) return fail(KVOP_EINVAL, "empty pool");
  kvop_pool* p = new (std::nothrow) kvop_pool();
  if (!p) return fail(KVOP_ENOMEM, "host allocation");
  p->m = m;
  p->kvdt = kvdt;
  p->cap = bytes;
  p->id = g_pool_ids.fetch_add(1);
  if (hipMalloc((void**)&p->base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(KVOP_ENOMEM, "pool allocation of " + std::to_string(bytes) + " bytes failed");
  }
  p->free_list[0] = bytes;
  *out = p;
  return KVOP_OK;
}

kvop_status kvop_pool_destroy(kvop_pool* p) {
  if (!p) return fail(KVOP_EINVAL, "null pool");
  (void)hipDeviceSynchronize();
  (void)hipFree(p->base);
  delete p;
  return KVOP_OK;
}

uint64_t kvop_doc_bytes(const kvop_pool* p, int64_t L) { return p && L > 0 ? doc_bytes(p, L) : 0; }

kvop_status kvop_pool_stats(const kvop_pool* p, uint64_t* used, uint64_t* cap, int32_t* live) {
  if (!p) return fail(KVOP_EINVAL, "null pool");
  if (used) *used = p->used;
  if (cap) *cap = p->cap;
  if (live) *live = p->live;
  return KVOP_OK;
}

kvop_status kvop_kv_release(kvop_pool* p, const kvop_handle* hs, int32_t n) {
  if (!p || (n > 0 && !hs) || n < 0) return fail(KVOP_EINVAL, "bad arguments");
  std::vector<uint32_t> slots;
  for (int i = 0; i < n; i++) {
    if (!lookup(p, hs[i])) return fail(KVOP_EBADHANDLE, "handle " + std::to_string(i) + " is not live in this pool");
    uint32_t s = (uint32_t)(hs[i] & 0xffffffffu);
    if (std::find(slots.begin(), slots.end(), s) != slots.end())
      return fail(KVOP_EBADHANDLE, "handle released twice in one call");
    slots.push_back(s);
  }
  for (uint32_t s : slots) {
    DocSlot& d = p->slots[s];
    pool_free(p, d.off, d.bytes);
    d.live = false;
    d.gen++;
    p->free_slots.push_back(s);
    p->live--;
  }
  return KVOP_OK;
}

// ------------------------------------------------------------------ kv_build
static kvop_status kv_build_impl(kvop_pool* p, const int32_t* tokens, const int64_t* offsets, int32_t n,
                                 void* stream, kvop_handle* handles_out, float* pooled, int n_future,
                                 float* scores) {
  if (!p || n < 0 || (n > 0 && (!tokens || !offsets || !handles_out))) return fail(KVOP_EINVAL, "bad arguments");
  if (n == 0) return KVOP_OK;
  kvop_model* m = p->m;
  const kvop_model_cfg& c = m->cfg;
  hipStream_t st = (hipStream_t)stream;
  CallOrder order(m, st);
  for (int i = 0; i < n; i++) {
    int64_t L = offsets[i + 1] - offsets[i];
    if (L < 1) return fail(KVOP_EINVAL, "document " + std::to_string(i) + " is empty or offsets decrease");
    if (L >= kRopeMaxPos) return fail(KVOP_EINVAL, "document longer than the rotary table");
    if (scores && L + n_future > kRopeMaxPos)
      return fail(KVOP_EINVAL, "document " + std::to_string(i) + ": L + n_future exceeds the rotary table");
  }
  // token ids must lie in [0, V): checked on the device, before anything is allocated or
  // any compute is enqueued (one synchronisation of the stream)
  HIPTRY(hipMemsetAsync(m->dflag, 0, 4, st));
  HIPTRY(validate_tokens(tokens + offsets[0], offsets[n] - offsets[0], c.vocab, m->dflag, st));
  HIPTRY(hipMemcpyAsync(m->hflag, m->dflag, 4, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  if (m->hflag[0] != 0) return fail(KVOP_EINVAL, "token id outside [0, vocab)");
  // expected-attention workspace (model-owned, grown on demand): per chunk row, H
  // log-weights and Hkv accumulators
  float* ea_ws = nullptr;
  int64_t ea_rows = 0;
  if (scores) {
    ea_rows = 65536;
    for (int i = 0; i < n; i++) ea_rows = std::max<int64_t>(ea_rows, offsets[i + 1] - offsets[i]);
    if (p->m->ea.reserve((size_t)ea_rows * (p->m->cfg.n_heads + p->m->cfg.n_kv_heads) * 4, (hipStream_t)stream) !=
        hipSuccess) {
      (void)hipGetLastError();
      return fail(KVOP_ENOMEM, "expected-attention workspace");
    }
    ea_ws = (float*)p->m->ea.p;
  }
  // allocate every region first (all or nothing)
  std::vector<uint64_t> offs(n), sizes(n);
  for (int i = 0; i < n; i++) {
    sizes[i] = doc_bytes(p, offsets[i + 1] - offsets[i]);
    if (!pool_alloc(p, sizes[i], &offs[i])) {
      for (int j = 0; j < i; j++) pool_free(p, offs[j], sizes[j]);
      return fail(KVOP_ENOMEM, "cache pool full after " + std::to_string(i) + " of " + std::to_string(n) + " documents");
    }
  }
  auto rollback = [&]() { for (int j = 0; j < n; j++) pool_free(p, offs[j], sizes[j]); };

  const int d = c.d_model, H = c.n_heads, Hkv = c.n_kv_heads, D = c.head_dim, G = H / Hkv;
  const int Pmax = std::max(1, std::min(64 / G, 64));
  const int64_t chunk_rows = 65536;
  int i0 = 0;
  while (i0 < n) {
    // documents [i0, i1) in this chunk
    int i1 = i0;
    int64_t rows = 0;
    while (i1 < n && (i1 == i0 || rows + (offsets[i1 + 1] - offsets[i1]) <= chunk_rows)) {
      rows += offsets[i1 + 1] - offsets[i1];
      i1++;
    }
    const int nd = i1 - i0;
    // host-built metadata
    std::vector<int32_t> pos(rows);
    std::vector<KvBlock> blocks;
    std::vector<AttnWork> work;
    std::vector<int64_t> row_off(nd + 1);
    int64_t r = 0;
    for (int i = i0; i < i1; i++) {
      int L = (int)(offsets[i + 1] - offsets[i]);
      row_off[i - i0] = r;
      for (int q = 0; q < L; q++) pos[r + q] = q;
      for (int p0 = 0; p0 < L; p0 += 16) blocks.push_back(KvBlock{(int64_t)offs[i], L, p0, (int32_t)(r + p0), 0});
      for (int p0 = 0; p0 < L; p0 += Pmax) {
        AttnWork w{};
        w.off_a = (int64_t)offs[i];
        w.off_b = -1;
        w.idx_a = -1;
        w.idx_b = -1;
        w.L_a = L;
        w.n_a = std::min(L, p0 + Pmax);
        w.q_row0 = (int32_t)(r + p0);
        w.q_pos0 = p0;
        w.n_q = std::min(Pmax, L - p0);
        work.push_back(w);
      }
      r += L;
    }
    row_off[nd] = r;
    // longest key ranges first
    std::stable_sort(work.begin(), work.end(), [](const AttnWork& a, const AttnWork& b) { return a.n_a > b.n_a; });
    // expected-attention workgroups: longest documents first
    std::vector<int32_t> ea_ord(nd);
    for (int i = 0; i < nd; i++) ea_ord[i] = i;
    std::stable_sort(ea_ord.begin(), ea_ord.end(), [&](int32_t a, int32_t b2) {
      return row_off[a + 1] - row_off[a] > row_off[b2 + 1] - row_off[b2];
    });
    // log-weight work items: key segments of at most 1024 rows, so that one long document
    // spreads over several workgroups
    std::vector<int32_t> ea_items;
    for (int32_t dd : ea_ord) {
      const int32_t Ld = (int32_t)(row_off[dd + 1] - row_off[dd]);
      for (int32_t k0 = 0; k0 < Ld; k0 += 1024) {
        ea_items.push_back(dd);
        ea_items.push_back(k0);
        ea_items.push_back(std::min<int32_t>(1024, Ld - k0));
      }
    }
    Mirror mir;
    size_t o_pos = mir.add(pos.size() * 4), o_blk = mir.add(blocks.size() * sizeof(KvBlock)),
           o_work = mir.add(work.size() * sizeof(AttnWork)), o_roff = mir.add(row_off.size() * 8),
           o_ord = mir.add(nd * 4), o_items = mir.add(ea_items.size() * 4), o_inv = mir.add(rows * 4);
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess) {
      rollback();
      return fail(KVOP_ENOMEM, "metadata staging");
    }
    memcpy(m->stage.p + o_pos, pos.data(), pos.size() * 4);
    memcpy(m->stage.p + o_blk, blocks.data(), blocks.size() * sizeof(KvBlock));
    memcpy(m->stage.p + o_work, work.data(), work.size() * sizeof(AttnWork));
    memcpy(m->stage.p + o_roff, row_off.data(), row_off.size() * 8);
    memcpy(m->stage.p + o_ord, ea_ord.data(), nd * 4);
    memcpy(m->stage.p + o_items, ea_items.data(), ea_items.size() * 4);
    char* md = (char*)m->meta.p;
    if (hipMemcpyAsync(md, m->stage.p, o_inv, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(m->stage.ev, st) != hipSuccess) {
      rollback();
      return fail(KVOP_EDEVICE, "metadata upload");
    }
    m->stage.pending = true;
    if (m->ws.reserve(act_bytes(m, rows, false), st) != hipSuccess) {
      rollback();
      return fail(KVOP_ENOMEM, "activation workspace for " + std::to_string(rows) + " rows");
    }
    LayerBufs b = carve(m, (char*)m->ws.p, rows, false);
    if (embed_rows(m->dt, m->embed, tokens + offsets[i0], (int)rows, d, c.vocab, b.x, st) != hipSuccess) {
      rollback();
      return fail(KVOP_EDEVICE, "embedding launch");
    }
    LayerPlan lp{};
    lp.rows = (int)rows;
    lp.pos = (const int32_t*)(md + o_pos);
    lp.alt_shift = nullptr;
    lp.attn.work = (const AttnWork*)(md + o_work);
    lp.attn.n_work = (int)work.size();
    lp.attn.idx = nullptr;
    lp.attn.Pmax = Pmax;
    lp.own_from_qkv = false;
    lp.own = nullptr;
    lp.select_all();
    float* ea_acc = ea_ws ? ea_ws + (size_t)ea_rows * H : nullptr;
    if (ea_ws) {
      lp.ea_row_off = (const int64_t*)(md + o_roff);
      lp.ea_order = (const int32_t*)(md + o_ord);
      lp.ea_items = (const int32_t*)(md + o_items);
      lp.ea_n_items = (int)(ea_items.size() / 3);
      lp.ea_nd = nd;
      lp.ea_n_future = n_future;
      lp.ea_e = ea_ws;
      lp.ea_acc = ea_acc;
      if (ea_zero(ea_acc, rows * Hkv, st) != hipSuccess) {
        rollback();
        return fail(KVOP_EDEVICE, "expected-attention launch");
      }
    }
    for (int l = 0; l < c.n_layers; l++) {
      bool tail = (l + 1 < c.n_layers) || pooled != nullptr;
      kvop_status s = run_layer(m, l, b, lp, p->base, p->kvdt, (const KvBlock*)(md + o_blk), (int)blocks.size(), st,
                                !tail);
      if (s != KVOP_OK) {
        rollback();
        return s;
      }
    }
    if (ea_ws && ea_finish(ea_acc, Hkv, (int)rows, scores + (offsets[i0] - offsets[0]), st) != hipSuccess) {
      rollback();
      return fail(KVOP_EDEVICE, "expected-attention launch");
    }
    if (pooled) {
      if (pooled_mean(b.x, d, (const int64_t*)(md + o_roff), nd, (int)rows, m->final_norm, c.rms_eps,
                      (float*)(md + o_inv), pooled + (int64_t)i0 * d, st) != hipSuccess) {
        rollback();
        return fail(KVOP_EDEVICE, "pooled launch");
      }
    }
    i0 = i1;
  }
  // publish handles
  for (int i = 0; i < n; i++) {
    uint32_t slot;
    if (!p->free_slots.empty()) {
      slot = p->free_slots.back();
      p->free_slots.pop_back();
    } else {
      slot = (uint32_t)p->slots.size();
      p->slots.push_back(DocSlot{});
    }
    DocSlot& s = p->slots[slot];
    s.off = offs[i];
    s.bytes = sizes[i];
    s.L = (int32_t)(offsets[i + 1] - offsets[i]);
    s.live = true;
    handles_out[i] = make_handle(p, slot, s.gen);
    p->live++;
  }
  return KVOP_OK;
}

kvop_status kvop_kv_build(kvop_pool* p, const int32_t* tokens, const int64_t* offsets, int32_t n, void* stream,
                          kvop_handle* handles_out, float* pooled) {
  return kv_build_impl(p, tokens, offsets, n, stream, handles_out, pooled, 0, nullptr);
}

kvop_status kvop_kv_build_scored(kvop_pool* p, const int32_t* tokens, const int64_t* offsets, int32_t n,
                                 int32_t n_future, void* stream, kvop_handle* handles_out, float* pooled,
                                 float* scores) {
  if (!scores || n_future < 1 || n_future > 4096) return fail(KVOP_EINVAL, "scores output and 1 <= n_future <= 4096");
  return kv_build_impl(p, tokens, offsets, n, stream, handles_out, pooled, n_future, scores);
}

int32_t kvop_retained_count(float r, int64_t L) {
  if (L < 1 || !(r >= 0.f) || r > 1.f) return -1;
  const int64_t rm = (int64_t)std::llround(1000.0 * (double)r);
  const int64_t k = (rm * L + 500) / 1000;
  return (int32_t)std::min<int64_t>(std::max<int64_t>(k, std::min<int64_t>(4, L)), L);
}

kvop_status kvop_ea_select(kvop_pool* p, const float* scores, const int64_t* offsets, int32_t n, float r,
                           void* stream, int32_t* idx, int64_t* idx_offsets) {
  if (!p || n < 0 || (n > 0 && (!scores || !offsets || !idx || !idx_offsets))) return fail(KVOP_EINVAL, "bad arguments");
  if (!(r >= 0.f) || r > 1.f) return fail(KVOP_EINVAL, "r must lie in [0, 1]");
  if (n == 0) return KVOP_OK;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int64_t> doc_off(n + 1), out_off(n + 1);
  std::vector<int32_t> kc(n);
  out_off[0] = 0;
  for (int i = 0; i < n; i++) {
    const int64_t L = offsets[i + 1] - offsets[i];
    if (L < 1 || L >= kRopeMaxPos) return fail(KVOP_EINVAL, "document " + std::to_string(i) + ": bad length");
    doc_off[i] = offsets[i] - offsets[0];
    kc[i] = kvop_retained_count(r, L);
    out_off[i + 1] = out_off[i] + kc[i];
  }
  doc_off[n] = offsets[n] - offsets[0];
  kvop_model* m = p->m;
  CallOrder order(m, st);
  Mirror mir;
  size_t o_doc = mir.add((n + 1) * 8), o_out = mir.add((n + 1) * 8), o_k = mir.add(n * 4);
  if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess)
    return fail(KVOP_ENOMEM, "metadata staging");
  memcpy(m->stage.p + o_doc, doc_off.data(), (n + 1) * 8);
  memcpy(m->stage.p + o_out, out_off.data(), (n + 1) * 8);
  memcpy(m->stage.p + o_k, kc.data(), n * 4);
  char* md = (char*)m->meta.p;
  if (hipMemcpyAsync(md, m->stage.p, mir.size, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(m->stage.ev, st) != hipSuccess)
    return fail(KVOP_EDEVICE, "metadata upload");
  m->stage.pending = true;
  if (ea_select(scores + offsets[0], (const int64_t*)(md + o_doc), (const int32_t*)(md + o_k),
                (const int64_t*)(md + o_out), n, idx, st) != hipSuccess)
    return fail(KVOP_EDEVICE, "selection launch");
  memcpy(idx_offsets, out_off.data(), (n + 1) * 8);
  return KVOP_OK;
}

// ------------------------------------------------------------------ op_eval
// dbg_layer >= 0 (with dbg_out): stop every wave after that layer and copy its residual
// stream (all suffix rows of the wave's items, FP32) to dbg_out instead of evaluating the head
static kvop_status op_eval_impl(kvop_pool* p, const kvop_op* op, float r, const int32_t* idx, const int64_t* idx_off,
                                const kvop_handle* hs, int32_t n_items, const int32_t* select, int32_t n_select,
                                void* stream, float* logits, int8_t* decision, int32_t* tokens_out,
                                bool validate_only = false, int dbg_layer = -1, float* dbg_out = nullptr) {
  if (!p || !op || n_items < 0 || n_select < 0) return fail(KVOP_EINVAL, "bad arguments");
  if (n_items == 0 || (select && n_select == 0)) return KVOP_OK;
  kvop_model* m = p->m;
  const kvop_model_cfg& c = m->cfg;
  hipStream_t st = (hipStream_t)stream;
  const int kind = op->kind;
  if (kind != KVOP_FILTER && kind != KVOP_MAP && kind != KVOP_JOIN) return fail(KVOP_EINVAL, "bad op kind");
  if (!(r > 0.f && r <= 1.f)) return fail(KVOP_EINVAL, "retention must be in (0, 1]");
  const int S = op->suffix_len;
  if (S < 1 || !op->suffix_host) return fail(KVOP_EINVAL, "empty suffix");
  if (!idx || !idx_off || !hs || (!logits && dbg_layer < 0)) return fail(KVOP_EINVAL, "null buffer");
  if (dbg_layer >= 0 && (kind == KVOP_MAP || select || !dbg_out || dbg_layer >= m->cfg.n_layers))
    return fail(KVOP_EINVAL, "stage readout: filter or join items, a layer below n_layers and an output buffer");
  for (int j = 0; j < S; j++)
    if (op->suffix_host[j] < 0 || op->suffix_host[j] >= c.vocab) return fail(KVOP_EINVAL, "suffix id out of range");
  int n_gen = 1;
  if (kind == KVOP_MAP) {
    n_gen = op->n_gen;
    if (n_gen < 1 || op->label_n < 1 || op->label_lo < 0 || op->label_lo + op->label_n > c.vocab || !tokens_out)
      return fail(KVOP_EINVAL, "bad map fields");
  } else {
    if (op->yes_id < 0 || op->yes_id >= c.vocab || op->no_id < 0 || op->no_id >= c.vocab)
      return fail(KVOP_EINVAL, "bad answer ids");
  }
  const bool join = kind == KVOP_JOIN;
  const int per = join ? 2 : 1;
  if (select && kind == KVOP_MAP) return fail(KVOP_EINVAL, "item selection applies to filters and joins");
  const bool padded = (op->flags & KVOP_FLAG_PADDED) != 0;
  if (padded && !attention_is_dma(m->dt, p->kvdt, m->cfg.head_dim))
    return fail(KVOP_EINVAL, "padded batching needs the direct-load attention kernels (BF16 compute, BF16 or FP8 "
                             "cache, head_dim 64 or 128, attention variant >= 0)");
  // evaluated items (all, or the selection) and their lists: list lidx[i*per + j]
  const int n_eval = select ? n_select : n_items;
  std::vector<int32_t> ids(n_eval);
  for (int i = 0; i < n_eval; i++) {
    ids[i] = select ? select[i] : i;
    if (ids[i] < 0 || ids[i] >= n_items) return fail(KVOP_EINVAL, "selected item out of range");
  }
  const int n_lists = n_eval * per;
  std::vector<int64_t> lidx(n_lists);
  for (int i = 0; i < n_eval; i++)
    for (int j = 0; j < per; j++) lidx[i * per + j] = (int64_t)ids[i] * per + j;
  std::vector<const DocSlot*> docs(n_lists);
  std::vector<ListCheck> checks(n_lists);
  for (int i = 0; i < n_lists; i++) {
    const int64_t li = lidx[i];
    docs[i] = lookup(p, hs[li]);
    if (!docs[i]) return fail(KVOP_EBADHANDLE, "handle " + std::to_string(li) + " is not live in this pool");
    int64_t k = idx_off[li + 1] - idx_off[li];
    if (k < 1 || k > docs[i]->L) return fail(KVOP_EINVAL, "list " + std::to_string(li) + " has a bad length");
    if (!(op->flags & KVOP_FLAG_ANY_COUNT) && k != retained_count(r, docs[i]->L))
      return fail(KVOP_EINVAL, "list " + std::to_string(li) + " holds " + std::to_string(k) + " rows, k(r, L) = " +
                                   std::to_string(retained_count(r, docs[i]->L)));
    checks[i] = ListCheck{idx_off[li], (int32_t)k, docs[i]->L};
  }
  for (int i = 0; i < n_eval; i++) {
    int64_t top = join ? (int64_t)docs[2 * i]->L + docs[2 * i + 1]->L : docs[i]->L;
    if (top + S + n_gen >= kRopeMaxPos) return fail(KVOP_EINVAL, "positions exceed the rotary table");
  }
  CallOrder order(m, st);
  // device-side validation of the lists (sorted, in range), before any compute
  {
    Mirror mir;
    size_t o_chk = mir.add(checks.size() * sizeof(ListCheck));
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess)
      return fail(KVOP_ENOMEM, "metadata staging");
    memcpy(m->stage.p + o_chk, checks.data(), checks.size() * sizeof(ListCheck));
    HIPTRY(hipMemcpyAsync(m->meta.p, m->stage.p, mir.size, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemsetAsync(m->dflag, 0, 4, st));
    HIPTRY(validate_lists(idx, (const ListCheck*)m->meta.p, n_lists, m->dflag, st));
    HIPTRY(hipMemcpyAsync(m->hflag, m->dflag, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (m->hflag[0] != 0)
      return fail(KVOP_EINVAL, std::to_string(m->hflag[0]) + " index list(s) unsorted or out of range");
  }
  if (validate_only) return KVOP_OK;

  const int d = c.d_model, H = c.n_heads, Hkv = c.n_kv_heads, D = c.head_dim, G = H / Hkv, F = c.d_ffn;
  const int qc = m->qkv_cols();
  const int Pmax_s = std::max(1, std::min(S, 64 / G));       // query positions per work item
  const int wq = (S + Pmax_s - 1) / Pmax_s;                  // work items per operator item
  const int64_t max_rows = g_wave_rows;
  const int wave_items = (int)std::max<int64_t>(1, max_rows / S);
  const int rows_per_item = S + (kind == KVOP_MAP ? n_gen - 1 : 0);  // own rows kept for decoding
  const int e = m->esz();

  for (int w0 = 0; w0 < n_eval; w0 += wave_items) {
    const int B = std::min(wave_items, n_eval - w0);
    const int64_t rows = (int64_t)B * S;
    // per-row positions and (joins) rotation shifts; per-item work items
    std::vector<int32_t> pos(rows), shift(join ? rows : 0);
    std::vector<AttnWork> work, work_last;
    work.reserve((size_t)B * wq);
    work_last.reserve((size_t)B);
    std::vector<int32_t> pos_dec(kind == KVOP_MAP ? B : 0);
    for (int b = 0; b < B; b++) {
      int it = w0 + b;
      const DocSlot* A = docs[it * per];
      const DocSlot* Bd = join ? docs[it * per + 1] : nullptr;
      int pos0 = A->L + (join ? Bd->L : 0);
      for (int j = 0; j < S; j++) {
        pos[(int64_t)b * S + j] = pos0 + j;
        if (join) shift[(int64_t)b * S + j] = A->L;
      }
      for (int q0 = 0; q0 < S; q0 += Pmax_s) {
        AttnWork w{};
        const int64_t la = lidx[it * per];
        w.off_a = (int64_t)A->off;
        w.idx_a = idx_off[la];
        w.L_a = A->L;
        w.n_a = (int32_t)(idx_off[la + 1] - idx_off[la]);
        if (join) {
          const int64_t lb = lidx[it * per + 1];
          w.off_b = (int64_t)Bd->off;
          w.idx_b = idx_off[lb];
          w.L_b = Bd->L;
          w.n_b = (int32_t)(idx_off[lb + 1] - idx_off[lb]);
        } else {
          w.off_b = -1;
          w.idx_b = -1;
        }
        w.q_row0 = b * S + q0;
        w.q_pos0 = pos0 + q0;
        w.n_q = std::min(Pmax_s, S - q0);
        w.own_row0 = b * S;
        w.n_own = std::min(S, q0 + Pmax_s);
        w.own_pos0 = pos0;
        work.push_back(w);
        if (q0 + Pmax_s >= S) {
          // the last layer: the item's last row only, against all its own rows
          w.q_row0 = b * S + S - 1;
          w.q_pos0 = pos0 + S - 1;
          w.n_q = 1;
          w.n_own = S;
          work_last.push_back(w);
        }
      }
      if (kind == KVOP_MAP) pos_dec[b] = pos0 + S;
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const AttnWork& a, const AttnWork& b) { return a.n_a + a.n_b > b.n_a + b.n_b; });
    std::stable_sort(work_last.begin(), work_last.end(),
                     [](const AttnWork& a, const AttnWork& b) { return a.n_a + a.n_b > b.n_a + b.n_b; });
    if (padded) {
      // every item of the wave iterates over the wave's largest key count (padding of A)
      const int kmax = work.empty() ? 0 : work.front().n_a + work.front().n_b;
      for (AttnWork& w : work) w.pad_a = kmax - w.n_b;
      for (AttnWork& w : work_last) w.pad_a = kmax - w.n_b;
    }
    // map decode: work items with one query position against (retained rows + own rows)
    std::vector<AttnWork> dwork;
    std::vector<int32_t> own_src, own_dst;
    if (kind == KVOP_MAP) {
      for (int b = 0; b < B; b++) {
        int it = w0 + b;
        const DocSlot* A = docs[it];
        AttnWork w{};
        w.off_a = (int64_t)A->off;
        w.off_b = -1;
        w.idx_a = idx_off[lidx[it]];
        w.idx_b = -1;
        w.L_a = A->L;
        w.n_a = (int32_t)(idx_off[lidx[it] + 1] - idx_off[lidx[it]]);
        w.q_row0 = b;
        w.n_q = 1;
        w.own_row0 = b * rows_per_item;
        w.own_pos0 = A->L;
        dwork.push_back(w);
      }
      if (padded) {
        int kmax = 0;
        for (const AttnWork& w : dwork) kmax = std::max(kmax, w.n_a);
        for (AttnWork& w : dwork) w.pad_a = kmax;
      }
      // longest key lists first, so that no long item starts last (items are independent)
      std::stable_sort(dwork.begin(), dwork.end(), [](const AttnWork& a, const AttnWork& b) { return a.n_a > b.n_a; });
      own_src.resize(rows);
      own_dst.resize(rows);
      for (int b = 0; b < B; b++)
        for (int j = 0; j < S; j++) {
          own_src[(int64_t)b * S + j] = b * S + j;
          own_dst[(int64_t)b * S + j] = b * rows_per_item + j;
        }
    }
    std::vector<int32_t> suffix(op->suffix_host, op->suffix_host + S);
    std::vector<int32_t> out_rows(ids.begin() + w0, ids.begin() + w0 + B);
    Mirror mir;
    size_t o_out = mir.add(out_rows.size() * 4);
    size_t o_pos = mir.add(pos.size() * 4), o_shift = mir.add(shift.size() * 4),
           o_work = mir.add(work.size() * sizeof(AttnWork)), o_wlast = mir.add(work_last.size() * sizeof(AttnWork)),
           o_suf = mir.add(S * 4), o_dwork = mir.add(dwork.size() * sizeof(AttnWork)),
           o_os = mir.add(own_src.size() * 4),
           o_od = mir.add(own_dst.size() * 4), o_pdec = mir.add(pos_dec.size() * 4),
           o_ddst = mir.add(pos_dec.size() * 4), o_dsrc = mir.add(pos_dec.size() * 4),
           o_ntok = mir.add(pos_dec.size() * 4);
    // per-decode-step metadata, rewritten before each step (reserved now so that the device
    // buffer never moves while the wave's metadata is in use)
    size_t o_sp = mir.add(pos_dec.size() * 4), o_sd = mir.add(pos_dec.size() * 4),
           o_sw = mir.add(pos_dec.size() * sizeof(AttnWork));
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess)
      return fail(KVOP_ENOMEM, "metadata staging");
    char* hp = m->stage.p;
    memcpy(hp + o_out, out_rows.data(), out_rows.size() * 4);
    memcpy(hp + o_pos, pos.data(), pos.size() * 4);
    if (join) memcpy(hp + o_shift, shift.data(), shift.size() * 4);
    memcpy(hp + o_work, work.data(), work.size() * sizeof(AttnWork));
    memcpy(hp + o_wlast, work_last.data(), work_last.size() * sizeof(AttnWork));
    memcpy(hp + o_suf, suffix.data(), S * 4);
    if (kind == KVOP_MAP) {
      memcpy(hp + o_dwork, dwork.data(), dwork.size() * sizeof(AttnWork));
      memcpy(hp + o_os, own_src.data(), own_src.size() * 4);
      memcpy(hp + o_od, own_dst.data(), own_dst.size() * 4);
      memcpy(hp + o_pdec, pos_dec.data(), pos_dec.size() * 4);
      std::vector<int32_t> ddst(B), dsrc(B);
      for (int b = 0; b < B; b++) { ddst[b] = b * rows_per_item + S; dsrc[b] = b; }
      memcpy(hp + o_ddst, ddst.data(), B * 4);
      memcpy(hp + o_dsrc, dsrc.data(), B * 4);
    }
    char* md = (char*)m->meta.p;
    HIPTRY(hipMemcpyAsync(md, hp, o_ntok, hipMemcpyHostToDevice, st));
    HIPTRY(hipEventRecord(m->stage.ev, st));
    m->stage.pending = true;

    // workspace: activations (+ per-layer own rows for maps)
    size_t act = act_bytes(m, rows, join);
    size_t own_bytes = kind == KVOP_MAP ? (size_t)c.n_layers * B * rows_per_item * 2 * Hkv * D * e : 0;
    if (m->ws.reserve(act + align_up(own_bytes, kAlign), st) != hipSuccess)
      return fail(KVOP_ENOMEM, "activation workspace");
    LayerBufs bufs = carve(m, (char*)m->ws.p, rows, join);
    char* ownbuf = (char*)m->ws.p + act;
    const int64_t own_ld = 2LL * Hkv * D;

    {
      ProfScope ps(PC_EMBED, st);
      HIPTRY(embed_suffix(m->dt, m->embed, (const int32_t*)(md + o_suf), S, (int)rows, d, c.vocab, bufs.x, st));
    }
    LayerPlan lp{};
    lp.rows = (int)rows;
    lp.pos = (const int32_t*)(md + o_pos);
    lp.alt_shift = join ? (const int32_t*)(md + o_shift) : nullptr;
    lp.attn.work = (const AttnWork*)(md + o_work);
    lp.attn.n_work = (int)work.size();
    lp.attn.idx = idx;
    lp.attn.Pmax = Pmax_s;
    lp.own_from_qkv = true;
    for (int l = 0; l < c.n_layers; l++) {
      const bool last = l + 1 == c.n_layers;
      // layer 0: every item's rows are the suffix's embeddings
      lp.n_shared = l == 0 && B >= 2 ? 1 : 0;
      lp.shared[0] = LayerPlan::SharedBlock{0, (int)rows, S};
      if (last) lp.select_one(B, S, S - 1);  // only the last suffix row of every item feeds the head
      else lp.select_all();
      // the last layer: queries and attention for each item's last row only
      lp.q_last = last && S > 1 ? S : 0;
      lp.attn.work = (const AttnWork*)(md + (lp.q_last ? o_wlast : o_work));
      lp.attn.n_work = (int)(lp.q_last ? work_last.size() : work.size());
      lp.attn.Pmax = lp.q_last ? 1 : Pmax_s;
      kvop_status s = run_layer(m, l, bufs, lp, p->base, p->kvdt, nullptr, 0, st);
      if (s != KVOP_OK) return s;
      if (kind == KVOP_MAP) {
        HIPTRY(copy_kv_rows(m->dt, bufs.qkv, qc, H * D, 2 * Hkv * D, (const int32_t*)(md + o_os),
                            (const int32_t*)(md + o_od), (int)rows, ownbuf + (size_t)l * B * rows_per_item * own_ld * e,
                            own_ld, st));
      }
      if (l == dbg_layer) {
        HIPTRY(hipMemcpyAsync(dbg_out + (int64_t)w0 * S * d, bufs.x, (size_t)rows * d * 4, hipMemcpyDeviceToDevice,
                              st));
        break;
      }
    }
    if (dbg_layer >= 0) continue;
    const float* xlast = bufs.x + (int64_t)(S - 1) * d;
    if (kind != KVOP_MAP) {
      ProfScope ps(PC_HEAD, st);
      HIPTRY(head_filter(m->dt, xlast, (int64_t)S * d, B, d, m->final_norm, c.rms_eps, m->head, op->yes_id, op->no_id,
                         op->theta_pos, op->theta_neg, nullptr, (const int32_t*)(md + o_out), logits, decision, st));
      continue;
    }
    // ---- map: step 1 from the suffix's last row, then n_gen - 1 decode steps
    const int ln = op->label_n;
    int32_t* ntok = (int32_t*)(md + o_ntok);
    float* lg = logits;
    int32_t* tk = tokens_out;
    const int32_t* orow = (const int32_t*)(md + o_out);
    HIPTRY(head_map(m->dt, xlast, (int64_t)S * d, B, d, m->final_norm, c.rms_eps, m->head, op->label_lo, ln, nullptr, orow, lg,
                    (int64_t)n_gen * ln, tk, n_gen, ntok, false, st));
    for (int t = 1; t < n_gen; t++) {
        ProfScope decode_scope(PC_DECODE, st);
      // positions of the fed token: L + S + t - 1; it is own row S + t - 1 of its item
      std::vector<int32_t> pdec(B), ddst(B);
      for (int b = 0; b < B; b++) {
        pdec[b] = pos_dec[b] + t - 1;
        ddst[b] = b * rows_per_item + S + t - 1;
      }
      std::vector<AttnWork> dw = dwork;
      for (AttnWork& x : dw) {
        x.q_pos0 = pdec[x.q_row0];
        x.n_own = S + t;
      }
      if (m->stage.reserve(mir.size) != hipSuccess) return fail(KVOP_EDEVICE, "metadata staging");
      memcpy(m->stage.p + o_sp, pdec.data(), B * 4);
      memcpy(m->stage.p + o_sd, ddst.data(), B * 4);
      memcpy(m->stage.p + o_sw, dw.data(), dw.size() * sizeof(AttnWork));
      HIPTRY(hipMemcpyAsync(md + o_sp, m->stage.p + o_sp, mir.size - o_sp, hipMemcpyHostToDevice, st));
      HIPTRY(hipEventRecord(m->stage.ev, st));
      m->stage.pending = true;
      HIPTRY(embed_rows(m->dt, m->embed, ntok, B, d, c.vocab, bufs.x, st));
      LayerPlan dp{};
      dp.rows = B;
      dp.pos = (const int32_t*)(md + o_sp);
      dp.alt_shift = nullptr;
      dp.attn.work = (const AttnWork*)(md + o_sw);
      dp.attn.n_work = B;
      dp.attn.idx = idx;
      dp.attn.Pmax = 1;
      dp.attn.decode = 1;
      dp.own_from_qkv = false;
      dp.own_stride = own_ld;
      dp.own_kcol = 0;
      dp.own_vcol = Hkv * D;
      dp.select_all();
      for (int l = 0; l < c.n_layers; l++) {
        char* own_l = ownbuf + (size_t)l * B * rows_per_item * own_ld * e;
        dp.own = own_l;
        // the new token's k, v must be in the own rows before the attention reads them:
        // run the projection + rotation, append, then attention and the tail
        const kvop_model::Layer& W = m->layers[l];
        HIPTRY(rmsnorm_rows(m->dt, bufs.x, d, W.attn_norm, B, d, c.rms_eps, bufs.h, d, st));
        {
          GemmShape s{B, qc, d, d, d, qc};
          if (m->dt == DT_BF16 && gemm_rope_supported(D)) {
            const RopeEpi re{dp.pos, m->cos_tab, m->sin_tab, D, (H + Hkv) * D, H * D, nullptr, nullptr};
            HIPTRY(gemm(m->dt, m->dt, EPI_ROPE, gemm_pick_tile(m->dt, EPI_ROPE, s), bufs.h, W.wqkv, bufs.qkv, s, st,
                        &re));
          } else {
            HIPTRY(gemm(m->dt, m->dt, EPI_STORE, gemm_pick_tile(m->dt, EPI_STORE, s), bufs.h, W.wqkv, bufs.qkv, s, st));
            HIPTRY(rope_qk(m->dt, bufs.qkv, qc, B, H, Hkv, D, dp.pos, m->cos_tab, m->sin_tab, nullptr, nullptr, st));
          }
        }
        HIPTRY(copy_kv_rows(m->dt, bufs.qkv, qc, H * D, 2 * Hkv * D, (const int32_t*)(md + o_dsrc),
                            (const int32_t*)(md + o_sd), B, own_l, own_ld, st));
        AttnArgs a = dp.attn;
        a.q = bufs.qkv;
        a.q_alt = nullptr;
        a.q_stride = qc;
        a.own = own_l;
        a.own_stride = own_ld;
        a.own_kcol = 0;
        a.own_vcol = Hkv * D;
        a.out = bufs.attn;
        a.out_stride = H * D;
        a.layer = l;
        a.n_layers = c.n_layers;
        a.Hkv = Hkv;
        a.G = G;
        a.pool = p->base;
        a.scale_log2 = (float)(1.4426950408889634 / std::sqrt((double)D));
        HIPTRY(attention(m->dt, p->kvdt, D, a, st));
        {
          GemmShape s{B, d, H * D, H * D, H * D, d};
          HIPTRY(gemm(m->dt, DT_F32, EPI_ADD, gemm_pick_tile(m->dt, EPI_ADD, s), bufs.attn, W.wo, bufs.x, s, st));
        }
        HIPTRY(rmsnorm_rows(m->dt, bufs.x, d, W.ffn_norm, B, d, c.rms_eps, bufs.h, d, st));
        {
          GemmShape s{B, 2 * F, d, d, d, F};
          HIPTRY(gemm(m->dt, m->dt, EPI_SWIGLU, gemm_pick_tile(m->dt, EPI_SWIGLU, s), bufs.h, W.wgu, bufs.act, s, st));
        }
        {
          GemmShape s{B, d, F, F, F, d};
          HIPTRY(gemm(m->dt, DT_F32, EPI_ADD, gemm_pick_tile(m->dt, EPI_ADD, s), bufs.act, W.wdown, bufs.x, s, st));
        }
      }
      HIPTRY(head_map(m->dt, bufs.x, d, B, d, m->final_norm, c.rms_eps, m->head, op->label_lo, ln, nullptr, orow,
                      lg + (int64_t)t * ln, (int64_t)n_gen * ln, tk + t, n_gen, ntok, false, st));
    }
  }
  return KVOP_OK;
}

kvop_status kvop_op_eval(kvop_pool* p, const kvop_op* op, float r, const int32_t* idx, const int64_t* idx_off,
                         const kvop_handle* hs, int32_t n_items, void* stream, float* logits, int8_t* decision,
                         int32_t* tokens_out) {
  return op_eval_impl(p, op, r, idx, idx_off, hs, n_items, nullptr, 0, stream, logits, decision, tokens_out);
}

kvop_status kvop_debug_stage(kvop_pool* p, const kvop_op* op, float r, const int32_t* idx, const int64_t* idx_off,
                             const kvop_handle* hs, int32_t n_items, int32_t layer, void* stream, float* hidden_out) {
  if (layer < 0) return fail(KVOP_EINVAL, "stage readout: layer must be >= 0");
  return op_eval_impl(p, op, r, idx, idx_off, hs, n_items, nullptr, 0, stream, nullptr, nullptr, nullptr, false, layer,
                      hidden_out);
}

kvop_status kvop_op_eval_select(kvop_pool* p, const kvop_op* op, float r, const int32_t* idx,
                                const int64_t* idx_offsets, const kvop_handle* hs, int32_t n_items,
                                const int32_t* select_host, int32_t n_select, void* stream, float* logits,
                                int8_t* decision) {
  if (!select_host && n_select > 0) return fail(KVOP_EINVAL, "null selection");
  if (n_select == 0) return KVOP_OK;
  return op_eval_impl(p, op, r, idx, idx_offsets, hs, n_items, select_host, n_select, stream, logits, decision, nullptr);
}

kvop_status kvop_cascade_eval(kvop_pool* p, const kvop_op* op, const kvop_stage* stages, int32_t n_stages,
                              const kvop_handle* hs, int32_t n_items, void* stream, float* logits, int8_t* decision,
                              int8_t* stage_out, int32_t* processed) {
  if (!p || !op || !stages || n_stages < 1 || n_stages > 127 || n_items < 0 || !processed)
    return fail(KVOP_EINVAL, "bad arguments");
  if (op->kind != KVOP_FILTER && op->kind != KVOP_JOIN) return fail(KVOP_EINVAL, "a cascade runs filters or joins");
  if (n_items > 0 && (!hs || !logits || !decision || !stage_out)) return fail(KVOP_EINVAL, "null output");
  for (int i = 0; i < n_stages; i++) {
    processed[i] = 0;
    if (std::isnan(stages[i].theta_pos) || std::isnan(stages[i].theta_neg) || !stages[i].idx_offsets_host)
      return fail(KVOP_EINVAL, "bad stage");
  }
  if (n_items == 0) return KVOP_OK;
  hipStream_t st = (hipStream_t)stream;
  // every stage's arguments and lists are checked before any stage runs, so that an
  // argument error leaves the outputs untouched
  for (int i = 0; i < n_stages; i++) {
    kvop_op o = *op;
    o.theta_pos = stages[i].theta_pos;
    o.theta_neg = stages[i].theta_neg;
    kvop_status s = op_eval_impl(p, &o, stages[i].r, stages[i].idx_dev, stages[i].idx_offsets_host, hs, n_items,
                                 nullptr, 0, stream, logits, decision, nullptr, true);
    if (s != KVOP_OK) return s;
  }
  std::vector<int32_t> sel(n_items);
  for (int t = 0; t < n_items; t++) sel[t] = t;               // every item starts unsure
  std::vector<int8_t> dec(n_items, -1), stage_of(n_items, -1);
  for (int i = 0; i < n_stages && !sel.empty(); i++) {
    kvop_op o = *op;
    o.theta_pos = stages[i].theta_pos;
    o.theta_neg = stages[i].theta_neg;
    kvop_status s = op_eval_impl(p, &o, stages[i].r, stages[i].idx_dev, stages[i].idx_offsets_host, hs, n_items,
                                 sel.data(), (int32_t)sel.size(), stream, logits, decision, nullptr);
    if (s != KVOP_OK) return s;
    processed[i] = (int32_t)sel.size();
    for (int32_t t : sel) stage_of[t] = (int8_t)i;
    if (i + 1 == n_stages) break;
    if (hipMemcpyAsync(dec.data(), decision, n_items, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(KVOP_EDEVICE, "decision readback");
    std::vector<int32_t> next;
    for (int32_t t : sel)
      if (dec[t] == -1) next.push_back(t);                    // still unsure: on to the next stage
    sel.swap(next);
  }
  if (hipMemcpyAsync(stage_out, stage_of.data(), n_items, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(KVOP_EDEVICE, "stage upload");
  return KVOP_OK;
}

// ------------------------------------------------------------------ mixed operators (batching form)
namespace {

struct MixedWave {
  std::vector<std::vector<int>> items;  // per op: item ids of this wave
  int64_t rows = 0;
};

}  // namespace

kvop_status kvop_mixed_eval(kvop_pool* p, const kvop_mixed_op* ops, int32_t n_ops, float r, const int32_t* idx,
                            const int64_t* idx_off, const kvop_handle* hs, const int32_t* item_op,
                            const int64_t* item_list, int32_t n_items, uint32_t flags, void* stream) {
  if (!p || !ops || n_ops < 1 || n_items < 0 || (n_items > 0 && (!item_op || !item_list || !idx || !idx_off || !hs)))
    return fail(KVOP_EINVAL, "bad arguments");
  if (n_items == 0) return KVOP_OK;
  if (!(r > 0.f && r <= 1.f)) return fail(KVOP_EINVAL, "retention must be in (0, 1]");
  kvop_model* m = p->m;
  const kvop_model_cfg& c = m->cfg;
  hipStream_t st = (hipStream_t)stream;
  int map_op = -1;
  bool any_join = false;
  for (int k = 0; k < n_ops; k++) {
    const kvop_op& o = ops[k].op;
    if (o.kind != KVOP_FILTER && o.kind != KVOP_MAP && o.kind != KVOP_JOIN) return fail(KVOP_EINVAL, "bad op kind");
    if (o.suffix_len < 1 || !o.suffix_host) return fail(KVOP_EINVAL, "empty suffix");
    for (int j = 0; j < o.suffix_len; j++)
      if (o.suffix_host[j] < 0 || o.suffix_host[j] >= c.vocab) return fail(KVOP_EINVAL, "suffix id out of range");
    if (!ops[k].logits_out_dev) return fail(KVOP_EINVAL, "null output");
    if (o.kind == KVOP_MAP) {
      if (map_op >= 0) return fail(KVOP_EINVAL, "at most one map operator per mixed call");
      if (o.n_gen < 1 || o.label_n < 1 || o.label_lo < 0 || o.label_lo + o.label_n > c.vocab || !ops[k].tokens_out_dev)
        return fail(KVOP_EINVAL, "bad map fields");
      map_op = k;
    } else if (o.yes_id < 0 || o.yes_id >= c.vocab || o.no_id < 0 || o.no_id >= c.vocab) {
      return fail(KVOP_EINVAL, "bad answer ids");
    }
    if (o.kind == KVOP_JOIN) any_join = true;
  }
  // items per operator, output rank of every item, list checks
  std::vector<std::vector<int>> by_op(n_ops);
  std::vector<int32_t> rank(n_items);
  std::vector<const DocSlot*> docA(n_items), docB(n_items, nullptr);
  std::vector<ListCheck> checks;
  for (int i = 0; i < n_items; i++) {
    int k = item_op[i];
    if (k < 0 || k >= n_ops) return fail(KVOP_EINVAL, "item operator out of range");
    rank[i] = (int32_t)by_op[k].size();
    by_op[k].push_back(i);
    const kvop_op& o = ops[k].op;
    const int nl = o.kind == KVOP_JOIN ? 2 : 1;
    for (int j = 0; j < nl; j++) {
      const int64_t li = item_list[i] + j;
      if (li < 0) return fail(KVOP_EINVAL, "negative list index");
      const DocSlot* d = lookup(p, hs[li]);
      if (!d) return fail(KVOP_EBADHANDLE, "handle " + std::to_string(li) + " is not live in this pool");
      int64_t kk = idx_off[li + 1] - idx_off[li];
      if (kk < 1 || kk > d->L) return fail(KVOP_EINVAL, "list " + std::to_string(li) + " has a bad length");
      if (!(o.flags & KVOP_FLAG_ANY_COUNT) && kk != retained_count(r, d->L))
        return fail(KVOP_EINVAL, "list " + std::to_string(li) + " does not hold k(r, L) rows");
      checks.push_back(ListCheck{idx_off[li], (int32_t)kk, d->L});
      (j == 0 ? docA[i] : docB[i]) = d;
    }
    int64_t top = docA[i]->L + (docB[i] ? docB[i]->L : 0);
    if (top + o.suffix_len + (o.kind == KVOP_MAP ? o.n_gen : 1) >= kRopeMaxPos)
      return fail(KVOP_EINVAL, "positions exceed the rotary table");
  }
  CallOrder order(m, st);
  {
    Mirror mir;
    size_t o_chk = mir.add(checks.size() * sizeof(ListCheck));
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess)
      return fail(KVOP_ENOMEM, "metadata staging");
    memcpy(m->stage.p + o_chk, checks.data(), checks.size() * sizeof(ListCheck));
    HIPTRY(hipMemcpyAsync(m->meta.p, m->stage.p, mir.size, hipMemcpyHostToDevice, st));
    HIPTRY(fill_i32(m->dflag, 0, 1, st));
    HIPTRY(validate_lists(idx, (const ListCheck*)m->meta.p, (int)checks.size(), m->dflag, st));
    HIPTRY(hipMemcpyAsync(m->hflag, m->dflag, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (m->hflag[0] != 0)
      return fail(KVOP_EINVAL, std::to_string(m->hflag[0]) + " index list(s) unsorted or out of range");
  }

  const int d = c.d_model, H = c.n_heads, Hkv = c.n_kv_heads, D = c.head_dim, G = H / Hkv, F = c.d_ffn;
  const int qc = m->qkv_cols();
  const int e = m->esz();
  const int64_t own_ld = 2LL * Hkv * D;
  // map items by rank (call-wide map index), for the decode steps after the waves
  const std::vector<int> map_by_rank = map_op >= 0 ? by_op[map_op] : std::vector<int>();
  // Each operator's items enter the waves longest key list first, so that the long items share
  // the first waves instead of each stretching the attention launch of its own wave (an
  // item's outputs keep their rank: the order of appearance in the call)
  for (int k = 0; k < n_ops; k++) {
    const int nl = ops[k].op.kind == KVOP_JOIN ? 2 : 1;
    auto keys = [&](int it) { return idx_off[item_list[it] + nl] - idx_off[item_list[it]]; };
    std::stable_sort(by_op[k].begin(), by_op[k].end(), [&](int a, int b) { return keys(a) > keys(b); });
  }
  // waves with a fixed per-operator composition: c_k items of operator k per wave
  int64_t total_rows = 0;
  for (int k = 0; k < n_ops; k++) total_rows += (int64_t)by_op[k].size() * ops[k].op.suffix_len;
  const int64_t max_rows = g_wave_rows;
  const int W = (int)std::max<int64_t>(1, (total_rows + max_rows - 1) / max_rows);
  std::vector<int> per(n_ops);
  for (int k = 0; k < n_ops; k++) per[k] = (int)((by_op[k].size() + W - 1) / W);
  const bool use_graph = (flags & KVOP_MIXED_GRAPH) != 0;
  const bool persistent = (flags & KVOP_MIXED_PERSISTENT) != 0;
  int* counter = m->dflag + 16;
  int Pmax = 64;
  for (int k = 0; k < n_ops; k++) Pmax = std::min(Pmax, std::max(1, std::min(ops[k].op.suffix_len, 64 / G)));
  // map decoding runs once after all waves, over every map item of the call: each wave
  // stores its map items' suffix keys/values (all layers) and first token; the decode
  // steps then run with all map items as rows
  const int nm_all = map_op >= 0 ? (int)by_op[map_op].size() : 0;
  const int n_gen = map_op >= 0 ? ops[map_op].op.n_gen : 1;
  const int Sm = map_op >= 0 ? ops[map_op].op.suffix_len : 0;
  const int rpi = Sm + n_gen - 1;  // own rows per map item: suffix + generated
  int64_t wave_rows_max = 0;
  for (int k = 0; k < n_ops; k++) wave_rows_max += (int64_t)per[k] * ops[k].op.suffix_len;
  const size_t act_w = align_up(act_bytes(m, wave_rows_max, any_join), kAlign);
  const size_t own_layer = (size_t)nm_all * rpi * own_ld * e;       // one layer's own rows of all map items
  const size_t own_all = align_up((size_t)c.n_layers * own_layer, kAlign);
  const size_t ntok_bytes = align_up((size_t)std::max(nm_all, 1) * 4, kAlign);
  const size_t act_d = nm_all > 0 ? align_up(act_bytes(m, nm_all, false), kAlign) : 0;
  if (m->ws.reserve(act_w + own_all + ntok_bytes + act_d, st) != hipSuccess)
    return fail(KVOP_ENOMEM, "activation workspace");
  char* ws = (char*)m->ws.p;
  LayerBufs bufs = carve(m, ws, wave_rows_max, any_join);
  char* ownbuf = ws + act_w;
  int32_t* ntok_all = (int32_t*)(ws + act_w + own_all);
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  auto cleanup_graph = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  };
  size_t full_meta = 0;

  for (int w = 0; w < W; w++) {
    // ---- items of this wave, rows grouped by operator
    std::vector<int> blk_row(n_ops), blk_n(n_ops);
    int64_t rows = 0;
    bool full = true;
    for (int k = 0; k < n_ops; k++) {
      int a = std::min<int>((int)by_op[k].size(), w * per[k]), b = std::min<int>((int)by_op[k].size(), (w + 1) * per[k]);
      blk_row[k] = (int)rows;
      blk_n[k] = b - a;
      if (b - a != per[k]) full = false;
      rows += (int64_t)(b - a) * ops[k].op.suffix_len;
    }
    if (rows == 0) continue;
    auto item_at = [&](int k, int b) { return by_op[k][(size_t)w * per[k] + b]; };
    std::vector<int32_t> tok(rows), pos(rows), shift(any_join ? rows : 0, -1);
    std::vector<AttnWork> work;
    std::vector<std::vector<int32_t>> in_rows(n_ops), out_rows(n_ops);
    for (int k = 0; k < n_ops; k++) {
      const kvop_op& o = ops[k].op;
      const int S = o.suffix_len;
      for (int b = 0; b < blk_n[k]; b++) {
        const int it = item_at(k, b);
        const DocSlot* A = docA[it];
        const DocSlot* Bd = docB[it];
        const int64_t r0 = blk_row[k] + (int64_t)b * S;
        const int pos0 = A->L + (Bd ? Bd->L : 0);
        for (int j = 0; j < S; j++) {
          tok[r0 + j] = o.suffix_host[j];
          pos[r0 + j] = pos0 + j;
          if (any_join) shift[r0 + j] = Bd ? A->L : -1;
        }
        for (int q0 = 0; q0 < S; q0 += Pmax) {
          AttnWork wk{};
          const int64_t la = item_list[it];
          wk.off_a = (int64_t)A->off;
          wk.idx_a = idx_off[la];
          wk.L_a = A->L;
          wk.n_a = (int32_t)(idx_off[la + 1] - idx_off[la]);
          if (Bd) {
            wk.off_b = (int64_t)Bd->off;
            wk.idx_b = idx_off[la + 1];
            wk.L_b = Bd->L;
            wk.n_b = (int32_t)(idx_off[la + 2] - idx_off[la + 1]);
          } else {
            wk.off_b = -1;
            wk.idx_b = -1;
          }
          wk.q_row0 = (int32_t)(r0 + q0);
          wk.q_pos0 = pos0 + q0;
          wk.n_q = std::min(Pmax, S - q0);
          wk.own_row0 = (int32_t)r0;
          wk.n_own = std::min(S, q0 + Pmax);
          wk.own_pos0 = pos0;
          work.push_back(wk);
        }
        in_rows[k].push_back((int32_t)(r0 + S - 1));
        out_rows[k].push_back(rank[it]);
      }
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const AttnWork& a, const AttnWork& b) { return a.n_a + a.n_b > b.n_a + b.n_b; });
    // map items of this wave: suffix rows -> own rows of their call-wide index (= output row)
    const int nm = map_op >= 0 ? blk_n[map_op] : 0;
    std::vector<int32_t> own_src, own_dst;
    for (int b = 0; b < nm; b++) {
      const int g = rank[item_at(map_op, b)];
      for (int j = 0; j < Sm; j++) {
        own_src.push_back(blk_row[map_op] + b * Sm + j);
        own_dst.push_back(g * rpi + j);
      }
    }
    // ---- metadata layout (identical for every full wave)
    Mirror mir;
    const size_t o_tok = mir.add(rows * 4), o_pos = mir.add(rows * 4), o_shift = mir.add(shift.size() * 4),
                 o_work = mir.add(work.size() * sizeof(AttnWork));
    std::vector<size_t> o_in(n_ops), o_out(n_ops);
    for (int k = 0; k < n_ops; k++) {
      o_in[k] = mir.add(in_rows[k].size() * 4);
      o_out[k] = mir.add(out_rows[k].size() * 4);
    }
    const size_t o_os = mir.add(own_src.size() * 4), o_od = mir.add(own_dst.size() * 4);
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess) {
      cleanup_graph();
      return fail(KVOP_ENOMEM, "metadata staging");
    }
    char* hp = m->stage.p;
    auto put = [&](size_t o, const void* src, size_t n) { if (n) memcpy(hp + o, src, n); };
    put(o_tok, tok.data(), rows * 4);
    put(o_pos, pos.data(), rows * 4);
    put(o_shift, shift.data(), shift.size() * 4);
    put(o_work, work.data(), work.size() * sizeof(AttnWork));
    for (int k = 0; k < n_ops; k++) {
      put(o_in[k], in_rows[k].data(), in_rows[k].size() * 4);
      put(o_out[k], out_rows[k].data(), out_rows[k].size() * 4);
    }
    put(o_os, own_src.data(), own_src.size() * 4);
    put(o_od, own_dst.data(), own_dst.size() * 4);
    char* md = (char*)m->meta.p;
    if (hipMemcpyAsync(md, hp, mir.size, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(m->stage.ev, st) != hipSuccess) {
      (void)hipGetLastError();
      cleanup_graph();
      return fail(KVOP_EDEVICE, "metadata upload");
    }
    m->stage.pending = true;

    // ---- the wave's launch sequence (enqueued directly, or captured once and replayed)
    auto enqueue = [&](hipStream_t st) -> kvop_status {
      HIPTRY(embed_rows(m->dt, m->embed, (const int32_t*)(md + o_tok), (int)rows, d, c.vocab, bufs.x, st));
      LayerPlan lp{};
      lp.rows = (int)rows;
      lp.pos = (const int32_t*)(md + o_pos);
      lp.alt_shift = any_join ? (const int32_t*)(md + o_shift) : nullptr;
      lp.attn.work = (const AttnWork*)(md + o_work);
      lp.attn.n_work = (int)work.size();
      lp.attn.idx = idx;
      lp.attn.Pmax = Pmax;
      lp.attn.counter = persistent ? counter : nullptr;
      lp.attn.persistent_wgs = 2 * m->n_cu;
      lp.attn.n_cu = m->n_cu;
      lp.own_from_qkv = true;
      for (int l = 0; l < c.n_layers; l++) {
        // layer 0: the rows of each operator's block repeat that operator's suffix
        lp.n_shared = 0;
        if (l == 0 && n_ops <= kMaxSelGroups)
          for (int k = 0; k < n_ops; k++)
            if (blk_n[k] > 0)
              lp.shared[lp.n_shared++] =
                  LayerPlan::SharedBlock{blk_row[k], blk_n[k] * ops[k].op.suffix_len, ops[k].op.suffix_len};
        // the last layer continues with each operator's last suffix rows only (one strided
        // group per operator); with more operators than groups every row continues
        lp.select_all();
        if (l + 1 == c.n_layers && n_ops <= kMaxSelGroups) {
          lp.n_groups = 0;
          for (int k = 0; k < n_ops; k++) {
            if (blk_n[k] == 0) continue;
            const int S = ops[k].op.suffix_len;
            lp.sel[lp.n_groups++] = SelGroup{blk_n[k], S, blk_row[k] + S - 1};
          }
        }
        kvop_status s = run_layer(m, l, bufs, lp, p->base, p->kvdt, nullptr, 0, st);
        if (s != KVOP_OK) return s;
        if (nm > 0)
          HIPTRY(copy_kv_rows(m->dt, bufs.qkv, qc, H * D, 2 * Hkv * D, (const int32_t*)(md + o_os),
                              (const int32_t*)(md + o_od), nm * Sm, ownbuf + (size_t)l * own_layer, own_ld, st));
      }
      for (int k = 0; k < n_ops; k++) {
        const kvop_op& o = ops[k].op;
        if (blk_n[k] == 0) continue;
        if (o.kind == KVOP_MAP) {
          // first generated id of every map item: logits, token and the next input at its row
          HIPTRY(head_map(m->dt, bufs.x, d, blk_n[k], d, m->final_norm, c.rms_eps, m->head, o.label_lo, o.label_n,
                          (const int32_t*)(md + o_in[k]), (const int32_t*)(md + o_out[k]), ops[k].logits_out_dev,
                          (int64_t)o.n_gen * o.label_n, ops[k].tokens_out_dev, o.n_gen, ntok_all, true, st));
          continue;
        }
        HIPTRY(head_filter(m->dt, bufs.x, d, blk_n[k], d, m->final_norm, c.rms_eps, m->head, o.yes_id, o.no_id,
                           o.theta_pos, o.theta_neg, (const int32_t*)(md + o_in[k]), (const int32_t*)(md + o_out[k]),
                           ops[k].logits_out_dev, ops[k].decision_out_dev, st));
      }
      return KVOP_OK;
    };

    // the first wave always runs directly (it also sizes every buffer); later full waves
    // replay one captured graph when asked to
    const bool graph_wave = use_graph && full && w > 0;
    if (!graph_wave) {
      kvop_status s = enqueue(st);
      if (s != KVOP_OK) { cleanup_graph(); return s; }
      if (full) full_meta = mir.size;
      continue;
    }
    if (!gexec) {
      // capture on the library's own stream (capturing records, it does not execute), then
      // launch the instantiated graph on the caller's stream
      if (mir.size != full_meta) { cleanup_graph(); return fail(KVOP_EDEVICE, "wave layout changed"); }
      if (!m->cap_stream && hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        m->cap_stream = nullptr;
        return fail(KVOP_EDEVICE, "capture stream creation failed");
      }
      g_prof.capturing = true;
      hipError_t ce = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed);
      kvop_status s = KVOP_OK;
      hipError_t ee = hipSuccess;
      if (ce == hipSuccess) {
        s = enqueue(m->cap_stream);
        ee = hipStreamEndCapture(m->cap_stream, &graph);
      }
      g_prof.capturing = false;
      if (ce != hipSuccess || s != KVOP_OK || ee != hipSuccess) {
        (void)hipGetLastError();
        cleanup_graph();
        if (s != KVOP_OK) return s;
        return fail(KVOP_EDEVICE, ce != hipSuccess ? "hipStreamBeginCapture failed" : "hipStreamEndCapture failed");
      }
      if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        cleanup_graph();
        return fail(KVOP_EDEVICE, "hipGraphInstantiate failed");
      }
    }
    if (hipGraphLaunch(gexec, st) != hipSuccess) {
      (void)hipGetLastError();
      cleanup_graph();
      return fail(KVOP_EDEVICE, "hipGraphLaunch failed");
    }
  }
  if (gexec) {
    if (hipStreamSynchronize(st) != hipSuccess) { cleanup_graph(); return fail(KVOP_EDEVICE, "graph replay failed"); }
  }
  cleanup_graph();
  if (nm_all == 0 || n_gen < 2) return KVOP_OK;

  // ---- map decoding over all map items of the call (rows g = call-wide map index)
  {
    const kvop_op& o = ops[map_op].op;
    const int ln = o.label_n;
    std::vector<int32_t> ident(nm_all), pdec, ddst;
    std::vector<AttnWork> dwork;
    for (int g = 0; g < nm_all; g++) ident[g] = g;
    for (int t = 1; t < n_gen; t++)
      for (int g = 0; g < nm_all; g++) {
        const int it = map_by_rank[g];
        const DocSlot* A = docA[it];
        pdec.push_back(A->L + Sm + t - 1);
        ddst.push_back(g * rpi + Sm + t - 1);
        AttnWork wk{};
        wk.off_a = (int64_t)A->off;
        wk.off_b = -1;
        wk.idx_a = idx_off[item_list[it]];
        wk.idx_b = -1;
        wk.L_a = A->L;
        wk.n_a = (int32_t)(idx_off[item_list[it] + 1] - idx_off[item_list[it]]);
        wk.q_row0 = g;
        wk.q_pos0 = A->L + Sm + t - 1;
        wk.n_q = 1;
        wk.own_row0 = g * rpi;
        wk.n_own = Sm + t;
        wk.own_pos0 = A->L;
        dwork.push_back(wk);
      }
    // each step's items longest key list first, so that no long item starts last
    for (int t = 1; t < n_gen; t++)
      std::stable_sort(dwork.begin() + (size_t)(t - 1) * nm_all, dwork.begin() + (size_t)t * nm_all,
                       [](const AttnWork& a, const AttnWork& b) { return a.n_a > b.n_a; });
    Mirror mir;
    const size_t o_id = mir.add(ident.size() * 4), o_pd = mir.add(pdec.size() * 4), o_dd = mir.add(ddst.size() * 4),
                 o_dw = mir.add(dwork.size() * sizeof(AttnWork));
    if (m->stage.reserve(mir.size) != hipSuccess || m->meta.reserve(mir.size, st) != hipSuccess)
      return fail(KVOP_ENOMEM, "metadata staging");
    memcpy(m->stage.p + o_id, ident.data(), ident.size() * 4);
    memcpy(m->stage.p + o_pd, pdec.data(), pdec.size() * 4);
    memcpy(m->stage.p + o_dd, ddst.data(), ddst.size() * 4);
    memcpy(m->stage.p + o_dw, dwork.data(), dwork.size() * sizeof(AttnWork));
    char* md = (char*)m->meta.p;
    HIPTRY(hipMemcpyAsync(md, m->stage.p, mir.size, hipMemcpyHostToDevice, st));
    HIPTRY(hipEventRecord(m->stage.ev, st));
    m->stage.pending = true;
    LayerBufs db = carve(m, ws + act_w + own_all + ntok_bytes, nm_all, false);
    const int32_t* id = (const int32_t*)(md + o_id);
    for (int t = 1; t < n_gen; t++) {
      ProfScope decode_scope(PC_DECODE, st);
      const int32_t* pd = (const int32_t*)(md + o_pd) + (size_t)(t - 1) * nm_all;
      const int32_t* dd = (const int32_t*)(md + o_dd) + (size_t)(t - 1) * nm_all;
      const AttnWork* dw = (const AttnWork*)(md + o_dw) + (size_t)(t - 1) * nm_all;
      HIPTRY(embed_rows(m->dt, m->embed, ntok_all, nm_all, d, c.vocab, db.x, st));
      for (int l = 0; l < c.n_layers; l++) {
        char* own_l = ownbuf + (size_t)l * own_layer;
        const kvop_model::Layer& Wl = m->layers[l];
        HIPTRY(rmsnorm_rows(m->dt, db.x, d, Wl.attn_norm, nm_all, d, c.rms_eps, db.h, d, st));
        {
          GemmShape g{nm_all, qc, d, d, d, qc};
          if (m->dt == DT_BF16 && gemm_rope_supported(D)) {
            const RopeEpi re{pd, m->cos_tab, m->sin_tab, D, (H + Hkv) * D, H * D, nullptr, nullptr};
            HIPTRY(gemm(m->dt, m->dt, EPI_ROPE, gemm_pick_tile(m->dt, EPI_ROPE, g), db.h, Wl.wqkv, db.qkv, g, st, &re));
          } else {
            HIPTRY(gemm(m->dt, m->dt, EPI_STORE, gemm_pick_tile(m->dt, EPI_STORE, g), db.h, Wl.wqkv, db.qkv, g, st));
            HIPTRY(rope_qk(m->dt, db.qkv, qc, nm_all, H, Hkv, D, pd, m->cos_tab, m->sin_tab, nullptr, nullptr, st));
          }
        }
        HIPTRY(copy_kv_rows(m->dt, db.qkv, qc, H * D, 2 * Hkv * D, id, dd, nm_all, own_l, own_ld, st));
        AttnArgs a{};
        a.work = dw;
        a.n_work = nm_all;
        a.idx = idx;
        a.pool = p->base;
        a.q = db.qkv;
        a.q_stride = qc;
        a.own = own_l;
        a.own_stride = own_ld;
        a.own_kcol = 0;
        a.own_vcol = Hkv * D;
        a.out = db.attn;
        a.out_stride = H * D;
        a.layer = l;
        a.n_layers = c.n_layers;
        a.Hkv = Hkv;
        a.G = G;
        a.Pmax = 1;
        a.decode = 1;
        a.scale_log2 = (float)(1.4426950408889634 / std::sqrt((double)D));
        a.counter = persistent ? counter : nullptr;
        a.persistent_wgs = 2 * m->n_cu;
        a.n_cu = m->n_cu;
        if (a.counter) HIPTRY(fill_i32(a.counter, 0, 1, st));
        HIPTRY(attention(m->dt, p->kvdt, D, a, st));
        {
          GemmShape g{nm_all, d, H * D, H * D, H * D, d};
          HIPTRY(gemm(m->dt, DT_F32, EPI_ADD, gemm_pick_tile(m->dt, EPI_ADD, g), db.attn, Wl.wo, db.x, g, st));
        }
        HIPTRY(rmsnorm_rows(m->dt, db.x, d, Wl.ffn_norm, nm_all, d, c.rms_eps, db.h, d, st));
        {
          GemmShape g{nm_all, 2 * F, d, d, d, F};
          HIPTRY(gemm(m->dt, m->dt, EPI_SWIGLU, gemm_pick_tile(m->dt, EPI_SWIGLU, g), db.h, Wl.wgu, db.act, g, st));
        }
        {
          GemmShape g{nm_all, d, F, F, F, d};
          HIPTRY(gemm(m->dt, DT_F32, EPI_ADD, gemm_pick_tile(m->dt, EPI_ADD, g), db.act, Wl.wdown, db.x, g, st));
        }
      }
      HIPTRY(head_map(m->dt, db.x, d, nm_all, d, m->final_norm, c.rms_eps, m->head, o.label_lo, ln, nullptr, id,
                      ops[map_op].logits_out_dev + (int64_t)t * ln, (int64_t)n_gen * ln, ops[map_op].tokens_out_dev + t,
                      n_gen, ntok_all, false, st));
    }
  }
  return KVOP_OK;
}

// ------------------------------------------------------------------ autotuner
kvop_status kvop_autotune(kvop_model* m, int64_t rows, int32_t reps, void* stream, char* report, int32_t report_len) {
  if (!m || rows < 1 || rows > (1 << 30) || reps < 1) return fail(KVOP_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const kvop_model_cfg& c = m->cfg;
  const int dt = m->dt, e = m->esz();
  const int d = c.d_model, F = c.d_ffn, HD = c.n_heads * c.head_dim, qc = m->qkv_cols();
  struct Shp { int N, K, epi; const char* name; };
  const Shp shapes[] = {{qc, d, EPI_STORE, "qkv"}, {d, HD, EPI_ADD, "o"}, {2 * F, d, EPI_SWIGLU, "gate_up"},
                        {d, F, EPI_ADD, "down"}};
  const int M = (int)rows;
  int64_t maxK = std::max(std::max(d, HD), F), maxN = std::max(std::max(qc, d), 2 * F);
  void *A = nullptr, *B = nullptr, *Cb = nullptr;
  size_t a_b = (size_t)M * maxK * e, b_b = (size_t)maxN * maxK * e, c_b = (size_t)M * maxN * 4;
  if (hipMalloc(&A, a_b) != hipSuccess || hipMalloc(&B, b_b) != hipSuccess || hipMalloc(&Cb, c_b) != hipSuccess) {
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    (void)hipGetLastError();
    return fail(KVOP_ENOMEM, "autotune scratch");
  }
  std::string rep;
  kvop_status status = KVOP_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipMemsetAsync(A, 0x3c, a_b, st);
  (void)hipMemsetAsync(B, 0x3c, b_b, st);
  for (const Shp& sh : shapes) {
    GemmShape g{M, sh.N, sh.K, sh.K, sh.K, sh.epi == EPI_SWIGLU ? sh.N / 2 : sh.N};
    const int out_dt = sh.epi == EPI_ADD ? DT_F32 : dt;
    int best = -1;
    float best_ms = 1e30f;
    for (int t = 0; t < gemm_num_tiles(dt); t++) {
      if (!gemm_tile_ok(dt, t, g, sh.epi)) continue;
      if (gemm(dt, out_dt, sh.epi, t, A, B, Cb, g, st) != hipSuccess) { status = fail(KVOP_EDEVICE, "autotune launch"); break; }
      (void)hipEventRecord(e0, st);
      for (int i = 0; i < reps; i++) (void)gemm(dt, out_dt, sh.epi, t, A, B, Cb, g, st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) { status = fail(KVOP_EDEVICE, "autotune timing"); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      rep += std::string(sh.name) + " M=" + std::to_string(M) + " " + gemm_tile_name(dt, t) + " " + std::to_string(ms) +
             " ms\n";
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (status != KVOP_OK) break;
    if (best >= 0) {
      gemm_set_tuned(dt, sh.epi, sh.N, sh.K, gemm_mbucket(M), best);
      rep += std::string("best ") + sh.name + " M=" + std::to_string(M) + " " + gemm_tile_name(dt, best) + "\n";
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(A);
  (void)hipFree(B);
  (void)hipFree(Cb);
  if (report && report_len > 0) {
    size_t n = std::min<size_t>(rep.size(), (size_t)report_len - 1);
    memcpy(report, rep.data(), n);
    report[n] = 0;
  }
  return status;
}

int32_t kvop_tuning_export(char* buf, int32_t len) {
  std::string t = gemm_tuned_export();
  if (buf && len > 0) {
    size_t n = std::min<size_t>(t.size(), (size_t)len - 1);
    memcpy(buf, t.data(), n);
    buf[n] = 0;
  }
  return (int32_t)t.size();
}

kvop_status kvop_tuning_import(const char* text) {
  if (!text) return fail(KVOP_EINVAL, "null text");
  std::string s(text);
  size_t pos = 0;
  int n_bad = 0;
  while (pos < s.size()) {
    size_t nl = s.find('\n', pos);
    std::string line = s.substr(pos, nl == std::string::npos ? std::string::npos : nl - pos);
    pos = nl == std::string::npos ? s.size() : nl + 1;
    if (line.empty() || line[0] == '#') continue;
    int dt, epi, N, K, mb;
    char name[128];
    if (sscanf(line.c_str(), "%d %d %d %d %d %127s", &dt, &epi, &N, &K, &mb, name) != 6 ||
        !gemm_tuned_import_line(dt, epi, N, K, mb, name))
      n_bad++;
  }
  if (n_bad) return fail(KVOP_EINVAL, std::to_string(n_bad) + " tuning line(s) not understood");
  return KVOP_OK;
}

kvop_status kvop_set_attention_kernel(int32_t variant) {
  if (variant < -1 || variant > 2) return fail(KVOP_EINVAL, "attention kernel variant must be -1 .. 2");
  attention_set_impl(variant);
  return KVOP_OK;
}

int32_t kvop_get_attention_kernel(void) { return attention_get_impl(); }

kvop_status kvop_debug_fp8_to_bf16(const uint8_t* codes_dev, int32_t n, uint16_t* out_dev, void* stream) {
  if (!codes_dev || !out_dev || n <= 0 || n % 8) return fail(KVOP_EINVAL, "n must be a positive multiple of 8");
  HIPTRY(fp8_widen(codes_dev, out_dev, n, (hipStream_t)stream));
  return KVOP_OK;
}

kvop_status kvop_set_wave_rows(int64_t rows) {
  if (rows < 64) return fail(KVOP_EINVAL, "wave must hold at least 64 rows");
  g_wave_rows = rows;
  return KVOP_OK;
}

// ------------------------------------------------------------------ profiling
kvop_status kvop_profile_start(void) {
  g_prof.on = true;
  for (int i = 0; i < PC_COUNT; i++) { g_prof.ms[i] = 0; g_prof.cnt[i] = 0; g_prof.launches[i].clear(); }
  for (auto& pe : g_prof.pending) { g_prof.pool.push_back(pe.second.first); g_prof.pool.push_back(pe.second.second); }
  g_prof.pending.clear();
  return KVOP_OK;
}

kvop_status kvop_profile_stop(double* ms_out, int64_t* count_out, int32_t n) {
  g_prof.on = false;
  for (auto& pe : g_prof.pending) {
    HIPTRY(hipEventSynchronize(pe.second.second));
    float ms = 0.f;
    HIPTRY(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
    g_prof.ms[pe.first] += ms;
    g_prof.cnt[pe.first] += 1;
    g_prof.launches[pe.first].push_back(ms);
    g_prof.pool.push_back(pe.second.first);
    g_prof.pool.push_back(pe.second.second);
  }
  g_prof.pending.clear();
  for (int i = 0; i < n && i < PC_COUNT; i++) {
    if (ms_out) ms_out[i] = g_prof.ms[i];
    if (count_out) count_out[i] = g_prof.cnt[i];
  }
  return KVOP_OK;
}

int32_t kvop_profile_launches(int32_t cls, double* ms_out, int32_t n) {
  if (cls < 0 || cls >= PC_COUNT) return -1;
  const auto& v = g_prof.launches[cls];
  for (int32_t i = 0; i < n && i < (int32_t)v.size(); i++) if (ms_out) ms_out[i] = v[i];
  return (int32_t)v.size();
}

int32_t kvop_profile_num_classes(void) { return PC_COUNT; }
const char* kvop_profile_class_name(int32_t i) { return i >= 0 && i < PC_COUNT ? kProfNames[i] : ""; }

// ------------------------------------------------------------------ diagnostics / tuning
int32_t kvop_gemm_num_tiles(int32_t dtype) { return gemm_num_tiles(dtype == KVOP_F32 ? DT_F32 : DT_BF16); }

const char* kvop_gemm_tile_name(int32_t dtype, int32_t tile) {
  int dt = dtype == KVOP_F32 ? DT_F32 : DT_BF16;
  if (tile < 0 || tile >= gemm_num_tiles(dt)) return "";
  return gemm_tile_name(dt, tile);
}

kvop_status kvop_debug_gemm(int32_t dtype, int32_t out_dtype, int32_t epi, int32_t tile, const void* A, const void* B,
                            void* Cm, int32_t M, int32_t N, int32_t K, int64_t lda, int64_t ldb, int64_t ldc,
                            void* stream) {
  if (dtype != KVOP_F32 && dtype != KVOP_BF16) return fail(KVOP_EINVAL, "bad dtype");
  if (epi < 0 || epi > 2 || !A || !B || !Cm || M < 0 || N < 0 || K < 1) return fail(KVOP_EINVAL, "bad arguments");
  int dt = dtype == KVOP_F32 ? DT_F32 : DT_BF16;
  int odt = out_dtype == KVOP_F32 ? DT_F32 : DT_BF16;
  if (dt == DT_F32 && odt != DT_F32) return fail(KVOP_EINVAL, "f32 operands produce f32 results");
  GemmShape s{M, N, K, lda, ldb, ldc};
  if (tile < 0) tile = gemm_pick_tile(dt, epi, s);
  if (!gemm_tile_ok(dt, tile, s, epi)) return fail(KVOP_EINVAL, "tile cannot run this shape");
  HIPTRY(gemm(dt, odt, epi, tile, A, B, Cm, s, (hipStream_t)stream));
  return KVOP_OK;
}

kvop_status kvop_debug_gemm_rope(int32_t tile, const void* A, const void* B, void* Cm, int32_t M, int32_t N, int32_t K,
                                 int32_t head_dim, int32_t rot_cols, const int32_t* pos_dev, const float* cos_dev,
                                 const float* sin_dev, int32_t fused, void* stream) {
  if (!A || !B || !Cm || !pos_dev || !cos_dev || !sin_dev || M < 0 || N < 1 || K < 1 || rot_cols < 0 || rot_cols > N ||
      !gemm_rope_supported(head_dim) || N % head_dim || rot_cols % head_dim)
    return fail(KVOP_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  GemmShape s{M, N, K, K, K, N};
  const int epi = fused ? EPI_ROPE : EPI_STORE;
  if (tile < 0) tile = gemm_pick_tile(DT_BF16, epi, s);
  if (!gemm_tile_ok(DT_BF16, tile, s, epi)) return fail(KVOP_EINVAL, "tile cannot run this shape");
  if (fused) {
    const RopeEpi re{pos_dev, cos_dev, sin_dev, head_dim, rot_cols, 0, nullptr, nullptr, 1};
    HIPTRY(gemm(DT_BF16, DT_BF16, EPI_ROPE, tile, A, B, Cm, s, st, &re));
  } else {
    // the plain product, then the separate pass (each element read and written by one thread)
    HIPTRY(gemm(DT_BF16, DT_BF16, EPI_STORE, tile, A, B, Cm, s, st));
    HIPTRY(rope_broadcast(Cm, std::max(M, 1), Cm, N, M, N, rot_cols, 0, head_dim, pos_dev, cos_dev, sin_dev, nullptr,
                          nullptr, st));
  }
  return KVOP_OK;
}

kvop_status kvop_gemm_set_tile(int32_t dtype, int32_t epi, int32_t N, int32_t K, int32_t M, int32_t tile) {
  int dt = dtype == KVOP_F32 ? DT_F32 : DT_BF16;
  if (tile < 0 || tile >= gemm_num_tiles(dt) || M < 1) return fail(KVOP_EINVAL, "bad tile");
  int mb = 0;
  while ((1 << (mb + 1)) <= M && mb < 30) mb++;
  gemm_set_tuned(dt, epi, N, K, mb, tile);
  return KVOP_OK;
}

int32_t kvop_gemm_pick_tile(int32_t dtype, int32_t epi, int32_t M, int32_t N, int32_t K) {
  if ((dtype != KVOP_F32 && dtype != KVOP_BF16) || epi < 0 || epi > 3 || M < 1 || N < 1 || K < 1) return -1;
  const GemmShape s{M, N, K, K, K, N};
  return gemm_pick_tile(dtype == KVOP_F32 ? DT_F32 : DT_BF16, epi, s);
}

kvop_status kvop_debug_read_cache(kvop_pool* p, kvop_handle h, int32_t layer, int32_t kv_head, int32_t kv,
                                  float* out, void* stream) {
  if (!p || !out) return fail(KVOP_EINVAL, "null argument");
  const DocSlot* d = lookup(p, h);
  if (!d) return fail(KVOP_EBADHANDLE, "handle is not live in this pool");
  const kvop_model_cfg& c = p->m->cfg;
  if (layer < 0 || layer >= c.n_layers || kv_head < 0 || kv_head >= c.n_kv_heads || (kv != 0 && kv != 1))
    return fail(KVOP_EINVAL, "bad layer/head/kv");
  HIPTRY(read_cache(p->kvdt, p->base + d->off, d->L, c.head_dim, layer, c.n_layers, c.n_kv_heads, kv_head, kv, out,
                    (hipStream_t)stream));
  return KVOP_OK;
}

}  // extern "C"
