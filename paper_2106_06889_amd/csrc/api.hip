// api.hip -- host runtime of the gtadoc C ABI: contexts over a caller-owned
// device arena, grammar loading, query entry points, results and errors.
//
// The arena plays the role of the paper's self-maintained GPU memory pool
// (Section "Data Structures"): every device buffer the library needs --
// grammar copies, initialization-phase products, per-call scratch and
// variable-size results -- is carved out of one buffer the caller provides,
// so the library itself never calls hipMalloc.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(GTADOC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kAlign = 256;

struct Block {
  uint64_t off = 0, size = 0;
};

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
 public:
  void init(uint64_t cap) {
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
    in_use_ = peak_ = 0;
  }
  bool alloc(uint64_t bytes, Block* out) {
    const uint64_t need = std::max<uint64_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > need) free_[off + need] = sz - need;
      *out = Block{off, need};
      in_use_ += need;
      peak_ = std::max(peak_, in_use_);
      peak_mark_ = std::max(peak_mark_, in_use_);
      return true;
    }
    return false;
  }
  // Peak bytes in use above the level at the last mark() (query footprints).
  void mark() { mark_ = peak_mark_ = in_use_; }
  uint64_t peak_since_mark() const { return peak_mark_ - mark_; }
  void release(const Block& b) {
    if (b.size == 0) return;
    in_use_ -= b.size;
    auto it = free_.emplace(b.off, b.size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  uint64_t cap() const { return cap_; }

 private:
  uint64_t cap_ = 0, in_use_ = 0, peak_ = 0, mark_ = 0, peak_mark_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

// Scratch of the allocation-free word count (gtadoc_word_count_noalloc): the
// packed word entries of the bucketed reduction, at most kStaticEntries of
// them (128 MiB). Each device the library runs on holds its own copy for the
// life of the process. In host code `scratch` names a host-side stand-in, not
// device memory: kernels receive the device address found once per device by
// hipGetSymbolAddress (static_scratch_at).
constexpr int64_t kStaticEntries = 32ll << 20;
static __device__ __align__(256) uint32_t scratch[kStaticEntries];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint32_t* g_static_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up on the first call for that device. Returns hipSuccess or the
// lookup's error.
hipError_t static_scratch_at(int device, uint32_t** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[device]) {
    uint32_t* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[device] = p;
  }
  *out = g_static_ptr[device];
  return hipSuccess;
}

constexpr size_t kPinnedBytes = 64 * 1024;
constexpr size_t kPinnedLevelAt = 1024;  // byte offset of the level offsets read back at load
constexpr int64_t kPinnedLevels = 4096;   // level offsets read back with the load counters

}  // namespace

struct gtadoc_ctx_s {
  char* base = nullptr;
  Arena arena;
  int device = 0;
  hipEvent_t done = nullptr;     // after the most recent call's work (see Call)
  hipStream_t last = nullptr;    // stream of the most recent call
  bool has_done = false;         // there was such a call
  char* pinned = nullptr;        // small pinned host buffer for read-backs
  int64_t wc_chunk = 16 * 1024;  // word-count reduce chunk (tunable)
  int64_t batch_blocks_per_cu = 4;
  int64_t batch_graph = 0;
  int64_t param_epoch = 0;       // bumped on every parameter change (invalidates captured graphs)
  int64_t timing = 0;            // phases timed: 1 all, else bit (p + 1) for phase p
  int64_t level_wide = 262144;   // level walk: bucketed mode from this many rules per level (0: never)
  gt::LevelParams level;         // level walk launch shape
  struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;  // recorded, not yet read
    std::vector<hipEvent_t> spare;
    double ms = 0;
    int64_t n = 0;
  } timers[GTADOC_NUM_PHASES];
};

struct gtadoc_batch_s {
  gtadoc_ctx ctx = nullptr;
  std::vector<Block> blocks;
  gt::BatchDesc* host = nullptr;   // pinned staging
  gt::BatchDesc* dev = nullptr;    // in the arena
  uint32_t* entries = nullptr;     // scratch in the arena
  int max_items = 0;
  uint64_t max_entries = 0;
  hipEvent_t done = nullptr;
  bool launched = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;  // private stream the launch sequence is captured on
  int64_t graph_epoch = -1;
  // streams of the mixed batch's variable-size queries (created on first use)
  static constexpr int kStreams = 4;
  hipStream_t pool[kStreams] = {};
  hipEvent_t pool_done[kStreams] = {};
  hipEvent_t start = nullptr;
};

struct gtadoc_grammar_s {
  gtadoc_ctx ctx = nullptr;
  std::vector<Block> blocks;
  gt::DevGrammar d{};
  gtadoc_stats st{};
  std::vector<int32_t> level_off;  // host copy, level_off[d] for d = 1..D+1
  bool has_levels = false;         // level_rule / level_off / depth built (by the load or on first need)
  // head/tail/len buffers for sequences (first use of sequence count)
  uint64_t* seq_len = nullptr;
  int32_t* seq_head = nullptr;
  int32_t* seq_tail = nullptr;
  // head/tail/len buffers of up to 7 words for the wide-key sequence count
  uint64_t* seqw_len = nullptr;
  int32_t* seqw_head = nullptr;
  int32_t* seqw_tail = nullptr;
  std::map<int64_t, uint64_t> footprint;  // arena bytes of a query kind (gtadoc_query_bytes)
  int64_t edges = -1;                     // distinct (parent, child) pairs (gtadoc_grammar_edges)
};

struct gtadoc_result_s {
  gtadoc_ctx ctx = nullptr;
  std::vector<Block> blocks;
  struct Arr {
    void* p;
    int64_t n;
    int eb;
  } a[4]{};
  int na = 0;
  const gtadoc_grammar_s* tv_of = nullptr;  // set on a term vector result: its grammar
};

namespace {

// Orders a call after the previous call on the same context and owns the
// call's scratch, which goes back to the arena when the call returns (later
// calls are ordered after this one's work, so the reuse is safe). Calls on
// one stream are ordered by the stream; a call on another stream waits for
// an event recorded after the previous call. A call on a stream the caller
// created records that event when it ends (the stream may be destroyed
// afterwards); a call on the null stream, which cannot be destroyed, leaves
// it to the next call on another stream, so back-to-back calls on the null
// stream record no event (each would leave the GPU idle for a few
// microseconds).
class Call {
 public:
  Call(gtadoc_ctx ctx, void* stream) : ctx_(ctx), s_(static_cast<hipStream_t>(stream)) {}
  // A call inside a batch submit: the submit orders the stream after earlier
  // work and joins it afterwards; the scratch goes to `defer` and is released
  // by the submit once every query of the batch is queued (the queries run
  // concurrently on different streams, so one's scratch must not be handed
  // to another).
  Call(gtadoc_ctx ctx, hipStream_t stream, std::vector<Block>* defer) : ctx_(ctx), s_(stream), defer_(defer) {}
  int begin() {
    if (hipSetDevice(ctx_->device) != hipSuccess) return fail(GTADOC_ERR_HIP, "hipSetDevice failed");
    if (!defer_ && ctx_->has_done && ctx_->last != s_) {
      if (ctx_->last == nullptr) HIP_TRY(hipEventRecord(ctx_->done, nullptr));
      HIP_TRY(hipStreamWaitEvent(s_, ctx_->done, 0));
    }
    return GTADOC_OK;
  }
  ~Call() {
    if (defer_) {
      defer_->insert(defer_->end(), scratch_.begin(), scratch_.end());
      return;
    }
    for (const Block& b : scratch_) ctx_->arena.release(b);
    if (s_ != nullptr) (void)hipEventRecord(ctx_->done, s_);
    ctx_->last = s_;
    ctx_->has_done = true;
  }
  // Scratch for this call only.
  template <typename T>
  T* scratch(int64_t count) {
    Block b;
    if (!ctx_->arena.alloc((uint64_t)std::max<int64_t>(count, 1) * sizeof(T), &b)) return nullptr;
    scratch_.push_back(b);
    return reinterpret_cast<T*>(ctx_->base + b.off);
  }
  // Memory that outlives the call, recorded in `owner`.
  template <typename T>
  T* keep(int64_t count, std::vector<Block>& owner) {
    Block b;
    if (!ctx_->arena.alloc((uint64_t)std::max<int64_t>(count, 1) * sizeof(T), &b)) return nullptr;
    owner.push_back(b);
    return reinterpret_cast<T*>(ctx_->base + b.off);
  }
  hipStream_t stream() const { return s_; }

 private:
  gtadoc_ctx ctx_;
  hipStream_t s_;
  std::vector<Block>* defer_ = nullptr;
  std::vector<Block> scratch_;
};

// Reads the recorded event pairs of a phase into its totals (waits for them).
void fold_timer(gtadoc_ctx_s::Timer& t) {
  for (auto& pr : t.pending) {
    float ms = 0;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      t.ms += ms;
      ++t.n;
    }
    t.spare.push_back(pr.first);
    t.spare.push_back(pr.second);
  }
  t.pending.clear();
}

// HIP events around one phase of a call, on the call's stream, when the
// context's timing is on. end() records the closing event; a scope left
// without end() (an error path) records nothing.
class PhaseScope {
 public:
  PhaseScope(gtadoc_ctx ctx, int phase, hipStream_t s) : ctx_(ctx), ph_(phase), s_(s) {
    if (ctx_->timing == 1 || ((ctx_->timing >> (ph_ + 1)) & 1)) a_ = take();
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) give(a_), a_ = nullptr;
  }
  void end() {
    if (!a_) return;
    hipEvent_t b = take();
    if (b && hipEventRecord(b, s_) == hipSuccess) {
      auto& t = ctx_->timers[ph_];
      t.pending.emplace_back(a_, b);
      if (t.pending.size() > 4096) fold_timer(t);
    } else {
      give(a_);
      if (b) give(b);
    }
    a_ = nullptr;
  }
  ~PhaseScope() {
    if (a_) give(a_);
  }

 private:
  hipEvent_t take() {
    auto& sp = ctx_->timers[ph_].spare;
    hipEvent_t e = nullptr;
    if (!sp.empty()) {
      e = sp.back();
      sp.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  void give(hipEvent_t e) { ctx_->timers[ph_].spare.push_back(e); }
  gtadoc_ctx ctx_;
  int ph_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr;
};

int oom(const char* what, uint64_t bytes) {
  return fail(GTADOC_ERR_OOM, "arena exhausted allocating %s (%llu bytes)", what, (unsigned long long)bytes);
}

int bitlen(uint64_t x) {
  int b = 0;
  while (x) ++b, x >>= 1;
  return b;
}

void release_all(gtadoc_ctx ctx, std::vector<Block>& blocks) {
  for (const Block& b : blocks) ctx->arena.release(b);
  blocks.clear();
}

}  // namespace

extern "C" {

const char* gtadoc_last_error(void) { return g_err.c_str(); }

int gtadoc_ctx_create(void* arena, uint64_t arena_bytes, gtadoc_ctx* out) {
  if (!arena || !out) return fail(GTADOC_ERR_INVALID_ARG, "null arena or output");
  if (reinterpret_cast<uintptr_t>(arena) % kAlign != 0) return fail(GTADOC_ERR_INVALID_ARG, "arena not 256-byte aligned");
  if (arena_bytes < (1u << 16)) return fail(GTADOC_ERR_INVALID_ARG, "arena smaller than 64 KiB");
  auto* c = new (std::nothrow) gtadoc_ctx_s;
  if (!c) return fail(GTADOC_ERR_OOM, "host allocation failed");
  c->base = static_cast<char*>(arena);
  c->arena.init(arena_bytes);
  if (hipGetDevice(&c->device) != hipSuccess || hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->pinned), kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    if (c->done) (void)hipEventDestroy(c->done);
    delete c;
    return fail(GTADOC_ERR_HIP, "context setup failed");
  }
  uint32_t* sp = nullptr;
  const hipError_t se = static_scratch_at(c->device, &sp);
  if (se != hipSuccess) {
    (void)hipEventDestroy(c->done);
    (void)hipHostFree(c->pinned);
    delete c;
    return fail(GTADOC_ERR_HIP, "device address of the static scratch: %s", hipGetErrorString(se));
  }
  *out = c;
  return GTADOC_OK;
}

int gtadoc_ctx_destroy(gtadoc_ctx ctx) {
  if (!ctx) return fail(GTADOC_ERR_INVALID_ARG, "null context");
  // the last call's stream may be gone by now: wait for the whole device
  if (ctx->has_done) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
  }
  for (auto& t : ctx->timers) {
    fold_timer(t);
    for (hipEvent_t e : t.spare) (void)hipEventDestroy(e);
  }
  (void)hipEventDestroy(ctx->done);
  (void)hipHostFree(ctx->pinned);
  delete ctx;
  return GTADOC_OK;
}

int gtadoc_ctx_usage(gtadoc_ctx ctx, uint64_t* in_use, uint64_t* peak, uint64_t* capacity) {
  if (!ctx) return fail(GTADOC_ERR_INVALID_ARG, "null context");
  if (in_use) *in_use = ctx->arena.in_use();
  if (peak) *peak = ctx->arena.peak();
  if (capacity) *capacity = ctx->arena.cap();
  return GTADOC_OK;
}

namespace {
bool hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fail(GTADOC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return false;
  }
  return true;
}

// The in-degree pass of the initialization phase on `s`: symbol ranges and
// word totals (lc), the word-bucket offsets (d.wc_off), the reference-bucket
// offsets (d.rc_off, scratch), then one packed word per rule in d.w
// (frequency in the root << kPendBits | in-edges from other rules; the root
// holds weight 1). With `zeroed`, the offset histograms are zero already.
// Returns false with the error recorded.
bool run_degrees(Call& call, gt::DevGrammar& d, gt::LoadCounters* lc, uint32_t* sums, int64_t n_wc_off,
                 int64_t n_rc_off, hipStream_t s, bool zeroed = false) {
  // with `zeroed`, the packed words are zero too when the in-degrees are
  // reduced by bucket
  const bool atomic_degrees = d.rc_nb == 0;
  if ((atomic_degrees && !hip_ok(gt::launch_fill_u64(d.w, d.R, 0, s), "fill")) ||
      (!zeroed && n_wc_off &&
       !hip_ok(gt::launch_fill_i32(reinterpret_cast<int32_t*>(d.wc_off), n_wc_off, 0, s), "fill")) ||
      (!zeroed && n_rc_off &&
       !hip_ok(gt::launch_fill_i32(reinterpret_cast<int32_t*>(d.rc_off), n_rc_off, 0, s), "fill")) ||
      !hip_ok(gt::launch_scan_symbols(d, lc, s), "scan_symbols") ||
      !hip_ok(gt::launch_scan_offsets2(d.wc_off, n_wc_off, &lc->wc_entries, d.rc_off, n_rc_off, &lc->rc_entries, sums,
                                       s),
              "scan offsets") ||
      (atomic_degrees && !hip_ok(gt::launch_fill_u64(d.w, 1, 1, s), "fill")))
    return false;
  if (!atomic_degrees) {
    // one entry per rule reference: at most S of them (the exact count stays on the device)
    uint16_t* ref_entries = call.scratch<uint16_t>(d.S);
    if (!ref_entries) {
      oom("reference entries", 2 * (uint64_t)d.S);
      return false;
    }
    if (!hip_ok(gt::launch_in_degrees(d, ref_entries, &lc->rc_entries, lc, s, zeroed), "in_degrees")) return false;
  }
  return true;
}
}  // namespace

int gtadoc_load_grammar(gtadoc_ctx ctx, const int64_t* rule_off, int64_t R, const int32_t* sym, int64_t S,
                        const int64_t* file_off, int64_t F, int32_t V, uint32_t flags, void* stream,
                        gtadoc_grammar* out) {
  if (!ctx || !out || !rule_off || !file_off || (S > 0 && !sym))
    return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (R < 1 || R >= INT32_MAX || S < 0 || F < 1 || V <= 0)
    return fail(GTADOC_ERR_INVALID_ARG, "bad sizes (R=%lld S=%lld F=%lld V=%d)", (long long)R, (long long)S,
                (long long)F, V);
  const bool host = flags & GTADOC_IN_HOST, dev = flags & GTADOC_IN_DEVICE, borrow = flags & GTADOC_IN_BORROW;
  const bool want_levels = flags & GTADOC_LOAD_LEVELS;
  if (host == dev || (borrow && !dev) ||
      (flags & ~(GTADOC_IN_HOST | GTADOC_IN_DEVICE | GTADOC_IN_BORROW | GTADOC_LOAD_LEVELS)))
    return fail(GTADOC_ERR_INVALID_ARG, "flags must be IN_HOST or IN_DEVICE[|BORROW], optionally LOAD_LEVELS");
  if (borrow && reinterpret_cast<uintptr_t>(sym) % 16 != 0)
    return fail(GTADOC_ERR_INVALID_ARG, "borrowed sym must be 16-byte aligned");

  Call call(ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  auto* g = new (std::nothrow) gtadoc_grammar_s;
  if (!g) return fail(GTADOC_ERR_OOM, "host allocation failed");
  g->ctx = ctx;
  auto bail = [&](int code) {
    (void)hipStreamSynchronize(s);  // the freed memory may still be in use by queued work
    release_all(ctx, g->blocks);
    delete g;
    return code;
  };

  gt::DevGrammar& d = g->d;
  d.R = R;
  d.S = S;
  d.F = F;
  d.V = V;
  d.ntiles = (S + gt::kTileSyms - 1) / gt::kTileSyms;
  d.nblk = (S + gt::kBlockSyms - 1) / gt::kBlockSyms;
  d.nslot = gt::kXcds * ((d.nblk + gt::kXcds - 1) / gt::kXcds);
  d.wc_nb = ((int64_t)V <= (int64_t)gt::kWcBucket * gt::kWcMaxBuckets) ? (int32_t)((V + gt::kWcBucket - 1) / gt::kWcBucket) : 0;
  d.rc_nb = (R <= (int64_t)gt::kRcBucket * gt::kRcMaxBuckets) ? (int32_t)((R + gt::kRcBucket - 1) / gt::kRcBucket) : 0;
  if (borrow) {
    d.rule_off = rule_off;
    d.sym = sym;
    d.file_off = file_off;
  } else {
    int64_t* ro = call.keep<int64_t>(R + 1, g->blocks);
    int32_t* sy = call.keep<int32_t>(S, g->blocks);
    int64_t* fo = call.keep<int64_t>(F + 1, g->blocks);
    if (!ro || !sy || !fo) return bail(oom("grammar copy", 8 * (R + F + 2) + 4 * S));
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(ro, rule_off, 8 * (R + 1), kind, s) != hipSuccess ||
        (S > 0 && hipMemcpyAsync(sy, sym, 4 * S, kind, s) != hipSuccess) ||
        hipMemcpyAsync(fo, file_off, 8 * (F + 1), kind, s) != hipSuccess)
      return bail(fail(GTADOC_ERR_HIP, "grammar copy failed"));
    d.rule_off = ro;
    d.sym = sy;
    d.file_off = fo;
  }
  int32_t* tile_rule = call.keep<int32_t>(d.ntiles + 1, g->blocks);
  d.w = call.keep<uint64_t>(R, g->blocks);
  d.level_rule = call.keep<int32_t>(std::max<int64_t>(R - 1, 1), g->blocks);
  d.level_off = call.keep<int32_t>(R + 2, g->blocks);
  const int64_t n_wc_off = (int64_t)d.wc_nb * d.nslot;
  const int64_t n_rc_off = (int64_t)d.rc_nb * d.nslot;
  d.wc_off = d.wc_nb ? call.keep<uint32_t>(n_wc_off, g->blocks) : nullptr;
  d.rc_off = d.rc_nb ? call.scratch<uint32_t>(n_rc_off) : nullptr;
  // the level walk's per-level counts, or the dataflow walk's queue weights,
  // chunk descriptors and counters
  int32_t* level_cnt = want_levels ? call.scratch<int32_t>(R + 2) : nullptr;
  gt::FlowBufs flow{};
  gt::FlowState* fs = nullptr;
  if (!want_levels) {
    flow.qc = d.level_rule;
    flow.qw = call.scratch<uint64_t>(R);
    flow.desc = call.scratch<uint64_t>(R);
    flow.qcap = (uint32_t)std::max<int64_t>(R - 1, 1);
    flow.ndesc = (uint32_t)R;
    fs = call.scratch<gt::FlowState>(1);
  }
  auto* lc = call.scratch<gt::LoadCounters>(1);
  const int64_t nbR = (R + 4095) / 4096;
  uint32_t* sums = call.scratch<uint32_t>(std::max({gt::scan2_scratch_entries(n_wc_off, n_rc_off),
                                                    nbR + gt::scan_scratch_entries(nbR) + 2}));
  if (!tile_rule || !d.w || !d.level_rule || !d.level_off || !lc || !sums || (want_levels && !level_cnt) ||
      (!want_levels && (!flow.qw || !flow.desc || !fs)) || (d.wc_nb && !d.wc_off) || (d.rc_nb && !d.rc_off))
    return bail(oom("initialization-phase buffers", 28 * (uint64_t)R + 4 * (uint64_t)(n_wc_off + n_rc_off)));
  d.tile_rule = tile_rule;

  auto* pc = reinterpret_cast<gt::LoadCounters*>(ctx->pinned);
  auto bad_layout = [&]() {
    return bail(fail(GTADOC_ERR_BAD_GRAMMAR, "bad grammar: %s%s%s",
                     (pc->status & gt::ST_BAD_OFFSETS) ? "rule offsets not monotone in [0, S]; " : "",
                     (pc->status & gt::ST_EMPTY_BODY) ? "empty non-root rule body; " : "",
                     (pc->status & gt::ST_BAD_FILES) ? "file spans do not tile the root body" : ""));
  };
  // phase 1: offsets and file spans. The level walk's load reads them back
  // first (its scratch is sized by the root's length); the dataflow load
  // queues everything at once, and its passes that index by offsets leave
  // at once on a bad layout, which the final read-back then reports.
  if (!hip_ok(gt::launch_fill_i32(reinterpret_cast<int32_t*>(lc), sizeof(gt::LoadCounters) / 4, 0, s), "fill"))
    return bail(GTADOC_ERR_HIP);
  if (!want_levels) {
    // the checks, the histograms' zeros and the walk's counters in one launch
    gt::ZeroRanges z{};
    z.add(d.wc_off, n_wc_off);
    z.add(d.rc_off, n_rc_off);
    z.add(fs, sizeof(gt::FlowState) / 4);
    z.add(flow.desc, 2 * (int64_t)flow.ndesc);
    if (d.rc_nb) z.add(d.w, 2 * R);  // the packed words the in-degree reduce adds into
    if (!hip_ok(gt::launch_load_prologue(d.rule_off, R, S, d.file_off, F, tile_rule, d.ntiles, lc, z, s), "checks"))
      return bail(GTADOC_ERR_HIP);
  } else {
    if (!hip_ok(gt::launch_check_rules(d.rule_off, R, S, tile_rule, d.ntiles, lc, s), "check_rules") ||
        !hip_ok(gt::launch_check_files(d.file_off, F, d.rule_off, lc, s), "check_files"))
      return bail(GTADOC_ERR_HIP);
    if (!hip_ok(hipMemcpyAsync(pc, lc, sizeof(gt::LoadCounters), hipMemcpyDeviceToHost, s), "read status") ||
        !hip_ok(hipStreamSynchronize(s), "sync"))
      return bail(GTADOC_ERR_HIP);
    if (pc->status) return bad_layout();
  }
  // scratch of the level walk's bucketed mode (wide levels); without room
  // for it every level takes the atomic mode
  gt::WideBufs wide{};
  {
    int64_t nbk = 1;
    int32_t nbk_bits = 0;
    while (nbk * gt::kWideBucket < R) nbk <<= 1, ++nbk_bits;
    const int64_t nonroot = S - pc->root_syms;
    if (want_levels && ctx->level_wide > 0 && nbk <= gt::kWideMaxBuckets && nonroot > 0 && nonroot < (1ll << 32)) {
      wide.ew = call.scratch<uint64_t>(nonroot);
      wide.ec = call.scratch<uint16_t>(nonroot);
      wide.cur = call.scratch<uint32_t>(nbk);
      wide.seg_lo = call.scratch<uint32_t>(nbk);
      wide.nbk = (int32_t)nbk;
      wide.nbk_bits = nbk_bits;
      wide.slots = (int32_t)((R + nbk - 1) / nbk);
      wide.min_rules = (int32_t)std::min<int64_t>(ctx->level_wide, INT32_MAX);
      if (!wide.ew || !wide.ec || !wide.cur || !wide.seg_lo) wide = gt::WideBufs{};
    }
  }
  // phase 2: symbols, in-degrees, then the weight walk: the level walk
  // (levels and weights) or the dataflow walk (weights; levels on first need)
  PhaseScope t_load(ctx, GTADOC_PHASE_LOAD, s);
  if (want_levels && !hip_ok(gt::launch_fill_i32(level_cnt, R + 2, 0, s), "fill")) return bail(GTADOC_ERR_HIP);
  if (!run_degrees(call, d, lc, sums, n_wc_off, n_rc_off, s, /*zeroed=*/!want_levels)) return bail(GTADOC_ERR_HIP);
  if (!hip_ok(gt::launch_level_frontier(d, lc, sums, s, want_levels ? nullptr : flow.qw, fs), "levels"))
    return bail(GTADOC_ERR_HIP);
  if (want_levels && !hip_ok(gt::prepare_level_walk(d, lc, sums, wide, s), "levels"))
    return bail(GTADOC_ERR_HIP);
  PhaseScope t_levels(ctx, GTADOC_PHASE_LEVELS, s);  // the walk kernel alone
  if (!hip_ok(want_levels ? gt::launch_level_walk(d, level_cnt, lc, sums, wide, ctx->level, ctx->device, s)
                          : gt::launch_flow_walk(d, lc, fs, flow, ctx->level, ctx->device, s),
              "levels"))
    return bail(GTADOC_ERR_HIP);
  t_levels.end();
  if (!hip_ok(gt::launch_unpack_weights(d, s), "weights")) return bail(GTADOC_ERR_HIP);
  t_load.end();
  // the counters (and the first level offsets) come back with one wait
  static_assert(sizeof(gt::LoadCounters) <= kPinnedLevelAt, "counters overlap the level offsets");
  int32_t* plevel = reinterpret_cast<int32_t*>(ctx->pinned + kPinnedLevelAt);
  const int64_t nlev = want_levels ? std::min<int64_t>(R + 2, kPinnedLevels) : 0;
  if (!hip_ok(hipMemcpyAsync(pc, lc, sizeof(gt::LoadCounters), hipMemcpyDeviceToHost, s), "read counters") ||
      (nlev && !hip_ok(hipMemcpyAsync(plevel, d.level_off, sizeof(int32_t) * nlev, hipMemcpyDeviceToHost, s),
                       "read levels")) ||
      !hip_ok(hipStreamSynchronize(s), "sync"))
    return bail(GTADOC_ERR_HIP);
  if (pc->status & gt::kBadLayout) return bad_layout();
  if (pc->status & (gt::ST_BAD_WORD | gt::ST_BAD_REF))
    return bail(fail(GTADOC_ERR_BAD_GRAMMAR, "bad grammar: %s%s",
                     (pc->status & gt::ST_BAD_WORD) ? "word id >= vocab; " : "",
                     (pc->status & gt::ST_BAD_REF) ? "rule reference outside [1, R)" : ""));
  if (pc->status & gt::ST_PACK)
    return bail(fail(GTADOC_ERR_UNSUPPORTED, "a rule is used 2^40 or more times, or referenced 2^24 or more times by "
                                             "other rules (the load packs weight and pending in-edges in 64 bits)"));
  if (d.wc_nb && pc->wc_entries != (int64_t)pc->word_syms)
    return bail(fail(GTADOC_ERR_HIP, "internal: word bucket histogram %lld != word symbols %llu",
                     (long long)pc->wc_entries, (unsigned long long)pc->word_syms));
  if (pc->status & gt::ST_FLOW)
    return bail(fail(GTADOC_ERR_HIP, "internal: the dataflow walk ran out of queue room or waited past its bound"));
  if (pc->placed != R - 1)
    return bail(fail(GTADOC_ERR_CYCLE, "rule graph has a cycle (%lld of %lld rules ordered)", (long long)pc->placed,
                     (long long)(R - 1)));
  const int32_t D = want_levels ? pc->depth : -1;
  if (want_levels) {
    g->level_off.assign((size_t)D + 2, 0);
    if (D > 0 && D + 2 <= nlev) {
      std::copy(plevel, plevel + D + 2, g->level_off.begin());
    } else if (D > 0) {
      if (!hip_ok(hipMemcpyAsync(g->level_off.data(), d.level_off, sizeof(int32_t) * (D + 2), hipMemcpyDeviceToHost, s),
                  "read levels") ||
          !hip_ok(hipStreamSynchronize(s), "sync"))
        return bail(GTADOC_ERR_HIP);
    }
    g->has_levels = true;
  }
  gtadoc_stats& st = g->st;
  st.tokens = (int64_t)(pc->tokens + pc->root_words);
  st.symbols = S;
  st.rules = R;
  st.files = F;
  st.word_syms = (int64_t)pc->word_syms;
  st.root_syms = pc->root_syms;
  st.depth = D;
  st.vocab = V;
  uint64_t bytes = 0;
  for (const Block& b : g->blocks) bytes += b.size;
  st.arena_bytes = bytes;
  *out = g;
  return GTADOC_OK;
}

namespace {
// Builds the level structure of a grammar loaded without it: the in-degree
// pass again into scratch (the grammar's weights stay as they are), level 1,
// then the level walk, which writes level_rule and level_off; the depth and
// the level offsets come back to the host. Synchronizes the call's stream.
int ensure_levels(gtadoc_grammar g, void* stream) {
  if (g->has_levels) return GTADOC_OK;
  gtadoc_ctx ctx = g->ctx;
  Call call(ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  gt::DevGrammar d = g->d;  // a copy whose packed words and histograms are scratch
  const int64_t R = d.R;
  const int64_t n_wc_off = (int64_t)d.wc_nb * d.nslot;
  const int64_t n_rc_off = (int64_t)d.rc_nb * d.nslot;
  d.w = call.scratch<uint64_t>(R);
  d.wc_off = d.wc_nb ? call.scratch<uint32_t>(n_wc_off) : nullptr;
  d.rc_off = d.rc_nb ? call.scratch<uint32_t>(n_rc_off) : nullptr;
  int32_t* level_cnt = call.scratch<int32_t>(R + 2);
  auto* lc = call.scratch<gt::LoadCounters>(1);
  const int64_t nbR = (R + 4095) / 4096;
  uint32_t* sums = call.scratch<uint32_t>(std::max({gt::scan2_scratch_entries(n_wc_off, n_rc_off),
                                                    nbR + gt::scan_scratch_entries(nbR) + 2}));
  if (!d.w || !level_cnt || !lc || !sums || (d.wc_nb && !d.wc_off) || (d.rc_nb && !d.rc_off))
    return oom("level buffers", 16 * (uint64_t)R + 4 * (uint64_t)(n_wc_off + n_rc_off));
  if (!hip_ok(gt::launch_fill_i32(reinterpret_cast<int32_t*>(lc), sizeof(gt::LoadCounters) / 4, 0, s), "fill") ||
      !hip_ok(gt::launch_fill_i32(level_cnt, R + 2, 0, s), "fill"))
    return GTADOC_ERR_HIP;
  if (!run_degrees(call, d, lc, sums, n_wc_off, n_rc_off, s)) return GTADOC_ERR_HIP;
  const gt::WideBufs wide{};  // every level in the atomic mode
  PhaseScope t_levels(ctx, GTADOC_PHASE_LEVELS, s);
  if (!hip_ok(gt::launch_level_frontier(d, lc, sums, s), "levels") ||
      !hip_ok(gt::prepare_level_walk(d, lc, sums, wide, s), "levels") ||
      !hip_ok(gt::launch_level_walk(d, level_cnt, lc, sums, wide, ctx->level, ctx->device, s), "levels"))
    return GTADOC_ERR_HIP;
  t_levels.end();
  gt::LoadCounters host{};
  if (!hip_ok(hipMemcpyAsync(&host, lc, sizeof(gt::LoadCounters), hipMemcpyDeviceToHost, s), "read counters") ||
      !hip_ok(hipStreamSynchronize(s), "sync"))
    return GTADOC_ERR_HIP;
  if (host.status || host.placed != R - 1)  // the load has checked all of these
    return fail(GTADOC_ERR_HIP, "internal: level walk status %u, %d of %lld rules placed", host.status, host.placed,
                (long long)(R - 1));
  const int32_t D = host.depth;
  std::vector<int32_t> off((size_t)D + 2, 0);
  if (D > 0 && (!hip_ok(hipMemcpyAsync(off.data(), d.level_off, sizeof(int32_t) * (D + 2), hipMemcpyDeviceToHost, s),
                        "read levels") ||
                !hip_ok(hipStreamSynchronize(s), "sync")))
    return GTADOC_ERR_HIP;
  g->level_off.swap(off);
  g->st.depth = D;
  g->has_levels = true;
  return GTADOC_OK;
}
}  // namespace

int gtadoc_build_levels(gtadoc_grammar g, void* stream) {
  if (!g) return fail(GTADOC_ERR_INVALID_ARG, "null grammar");
  return ensure_levels(g, stream);
}

int gtadoc_grammar_stats(gtadoc_grammar g, gtadoc_stats* out) {
  if (!g || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  *out = g->st;
  return GTADOC_OK;
}

int gtadoc_free_grammar(gtadoc_grammar g) {
  if (!g) return fail(GTADOC_ERR_INVALID_ARG, "null grammar");
  release_all(g->ctx, g->blocks);
  delete g;
  return GTADOC_OK;
}

namespace {
// Word count into `counts` on the call's stream: the bucketed on-chip
// reduction when the vocabulary fits the bucket table and every weight fits
// the packed entry (weights never exceed the token count), else direct atomics.
int word_count_into(gtadoc_grammar g, Call& call, uint64_t* counts) {
  const gt::DevGrammar& d = g->d;
  const int64_t W = g->st.word_syms;
  hipStream_t s = call.stream();
  if (W == 0) {
    HIP_TRY(gt::launch_fill_u64(counts, d.V, 0, s));
    return GTADOC_OK;
  }
  if (d.wc_nb > 0) {
    uint32_t* entries = call.scratch<uint32_t>(W);
    if (!entries) return oom("word entries", 4ull * W);
    PhaseScope t(g->ctx, GTADOC_PHASE_WORD_COUNT, s);
    HIP_TRY(gt::launch_word_count_buckets(d, counts, entries, W, g->ctx->wc_chunk, s));
    t.end();
    return GTADOC_OK;
  }
  PhaseScope t(g->ctx, GTADOC_PHASE_WORD_COUNT, s);
  HIP_TRY(gt::launch_word_count(d, counts, s));
  t.end();
  return GTADOC_OK;
}
}  // namespace

int gtadoc_word_count(gtadoc_grammar g, uint64_t* counts, void* stream) {
  if (!g || !counts) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  return word_count_into(g, call, counts);
}

int gtadoc_word_count_noalloc(gtadoc_grammar g, uint64_t* counts, void* stream) {
  if (!g || !counts) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  const gt::DevGrammar& d = g->d;
  const int64_t W = g->st.word_syms;
  if (d.wc_nb > 0 && W > kStaticEntries)
    return fail(GTADOC_ERR_UNSUPPORTED,
                "allocation-free word count holds at most %lld word symbols in its static scratch; this grammar has %lld",
                (long long)kStaticEntries, (long long)W);
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  if (W == 0) {
    HIP_TRY(gt::launch_fill_u64(counts, d.V, 0, s));
    return GTADOC_OK;
  }
  if (d.wc_nb == 0) {  // direct atomics: no scratch at all
    HIP_TRY(gt::launch_word_count(d, counts, s));
    return GTADOC_OK;
  }
  uint32_t* entries = nullptr;
  HIP_TRY(static_scratch_at(g->ctx->device, &entries));
  HIP_TRY(gt::launch_word_count_buckets(d, counts, entries, W, g->ctx->wc_chunk, s));
  return GTADOC_OK;
}

int gtadoc_decompress(gtadoc_grammar g, int32_t* tokens, int64_t* file_off, void* stream) {
  if (!g || !file_off || (g->st.tokens > 0 && !tokens)) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (int rl = ensure_levels(g, stream)) return rl;
  const gt::DevGrammar& d = g->d;
  const int64_t T = g->st.tokens, R = d.R, nroot = g->st.root_syms;
  const int32_t D = (int32_t)g->st.depth;
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  auto* len = call.scratch<uint64_t>(R);
  auto* pos = call.scratch<uint64_t>(nroot);
  auto* sums = call.scratch<uint64_t>(gt::scan_scratch_entries(nroot));
  auto* cnt = call.scratch<unsigned long long>(D + 3);
  if (!len || !pos || !sums || !cnt) return oom("decompression lengths", 8ull * (R + 2 * nroot));
  PhaseScope t(g->ctx, GTADOC_PHASE_DECOMPRESS, s);
  HIP_TRY(gt::launch_fill_u64(reinterpret_cast<uint64_t*>(cnt), D + 3, 0, s));
  HIP_TRY(gt::launch_rule_lengths(d, g->level_off.data(), D, len, s));
  // rule occurrences in the derivation tree (sum of the non-root weights)
  // bound the items of one depth, as do the tokens (items of one depth
  // expand to disjoint, non-empty output ranges)
  HIP_TRY(gt::launch_sum_u64(d.w + 1, R - 1, cnt + D + 2, s));
  auto* pc = reinterpret_cast<unsigned long long*>(g->ctx->pinned);
  HIP_TRY(hipMemcpyAsync(pc, cnt + D + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t occ = (int64_t)*pc;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(T, occ));
  int32_t* rule_a = call.scratch<int32_t>(cap);
  int32_t* rule_b = call.scratch<int32_t>(cap);
  int64_t* off_a = call.scratch<int64_t>(cap);
  int64_t* off_b = call.scratch<int64_t>(cap);
  if (!rule_a || !rule_b || !off_a || !off_b) return oom("decompression items", 24ull * cap);
  HIP_TRY(gt::launch_root_positions(d, len, pos, nroot, (uint64_t)T, file_off, sums, s));
  HIP_TRY(gt::launch_expand_root(d, pos, nroot, tokens, rule_a, off_a, cnt, s));
  for (int32_t k = 1; k <= D; ++k) {
    HIP_TRY(gt::launch_expand_depth(d, len, rule_a, off_a, cnt + k - 1, cap, tokens, rule_b, off_b, cnt + k, s));
    std::swap(rule_a, rule_b);
    std::swap(off_a, off_b);
  }
  t.end();
  return GTADOC_OK;
}

int gtadoc_sort(gtadoc_grammar g, const uint64_t* word_counts, uint32_t* ids, uint64_t* counts, int64_t* num,
                void* stream) {
  if (!g || !ids || !counts || !num) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  const int32_t V = g->d.V;
  if (!word_counts) {
    uint64_t* wc = call.scratch<uint64_t>(V);
    if (!wc) return oom("word counts", 8ull * V);
    rc = word_count_into(g, call, wc);
    if (rc) return rc;
    word_counts = wc;
  }
  gt::SortScratch sc{};
  sc.key[0] = call.scratch<uint64_t>(V);
  sc.key[1] = call.scratch<uint64_t>(V);
  sc.val[0] = call.scratch<uint32_t>(V);
  sc.val[1] = call.scratch<uint32_t>(V);
  sc.hist = call.scratch<uint32_t>(gt::word_sort_hist_entries(V));
  if (!sc.key[0] || !sc.key[1] || !sc.val[0] || !sc.val[1] || !sc.hist) return oom("sort scratch", 24ull * V);
  const int key_bits = std::max(1, bitlen((uint64_t)g->st.tokens));  // no count exceeds the token total
  PhaseScope t_sort(g->ctx, GTADOC_PHASE_SORT, s);
  HIP_TRY(gt::launch_sort_by_count(word_counts, V, key_bits, sc, ids, counts, num, s));
  t_sort.end();
  return GTADOC_OK;
}

namespace {

// The bits of the packed n-gram keys that word ids < V can occupy:
// bitlen(V-1) bits at bits 0 and 32 (n = 2), 0, 21 and 42 (n = 3), or 0, 16,
// 32 and 48 (n = 4); all other bits are zero.
gt::KeyBits gram_key_bits(int n, int32_t V) {
  const int b = std::max(1, bitlen((uint64_t)(V - 1)));
  gt::KeyBits kb{};
  const int step = n == 2 ? 32 : (n == 3 ? 21 : 16);
  kb.nseg = n;
  for (int x = 0; x < n; ++x) kb.lo[x] = step * x, kb.len[x] = b;
  return kb;
}

gtadoc_result new_result(gtadoc_ctx ctx) {
  auto* r = new (std::nothrow) gtadoc_result_s;
  if (r) r->ctx = ctx;
  return r;
}

}  // namespace

namespace {

// Term vector into arrays owned by `owner` (a result's blocks, or call
// scratch for the inverted index): off[F+1], word[NNZ], cnt[NNZ].
struct TvArrays {
  int64_t* off = nullptr;
  uint32_t* word = nullptr;
  uint64_t* cnt = nullptr;
  int64_t nnz = 0;
};

int term_vector_into(gtadoc_grammar g, Call& call, std::vector<Block>* owner, TvArrays* out) {
  const gt::DevGrammar& d = g->d;
  hipStream_t s = call.stream();
  const int64_t R = d.R, F = d.F;
  if ((uint64_t)g->st.tokens >= (1ull << 32))
    return fail(GTADOC_ERR_UNSUPPORTED, "term vector: counts beyond 2^32 tokens are not supported");
  if (d.V > gt::kWcBucket * gt::kWcMaxBuckets)
    return fail(GTADOC_ERR_UNSUPPORTED, "term vector: vocabularies above 2^24 words are not supported");
  const int32_t nb = (int32_t)((d.V + gt::kWcBucket - 1) / gt::kWcBucket);
  const int32_t D = (int32_t)g->st.depth;
  // 1. bounds (bottom-up), table offsets by one scan (bump allocation); file units
  auto* len = call.scratch<uint64_t>(R);
  auto* bound = call.scratch<uint64_t>(R);
  auto* toff = call.scratch<uint64_t>(R);
  auto* tsize = call.scratch<uint32_t>(R);
  auto* unit_off = call.scratch<int64_t>(F + 1);
  auto* sums64 = call.scratch<uint64_t>(gt::scan_scratch_entries(std::max<int64_t>(R, F + 1)));
  auto* tot = call.scratch<int64_t>(4);  // [0] pool entries, [1] units, [2] entries, [3] nnz
  if (!len || !bound || !toff || !tsize || !unit_off || !sums64 || !tot) return oom("term vector scratch", 36ull * R);
  HIP_TRY(gt::launch_fill_u64(len, R, 0, s));
  HIP_TRY(gt::launch_fill_u64(bound, R, 0, s));
  HIP_TRY(gt::launch_fill_i32(reinterpret_cast<int32_t*>(tsize), R, 0, s));
  HIP_TRY(gt::launch_fill_u64(reinterpret_cast<uint64_t*>(unit_off), F + 1, 0, s));
  HIP_TRY(gt::launch_tv_bounds(d, g->level_off.data(), D, len, bound, s));
  HIP_TRY(hipMemcpyAsync(toff, bound, 8 * R, hipMemcpyDeviceToDevice, s));
  HIP_TRY(gt::launch_scan_u64_ext(toff, R, tot + 0, sums64, s));
  HIP_TRY(gt::launch_tv_units(d, unit_off, s));
  HIP_TRY(gt::launch_scan_u64_ext(reinterpret_cast<uint64_t*>(unit_off), F + 1, tot + 1, sums64, s));
  auto* pc = reinterpret_cast<int64_t*>(g->ctx->pinned);
  HIP_TRY(hipMemcpyAsync(pc, tot, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t P = pc[0], NU = pc[1];
  // 2. tables, children first
  auto* pw = call.scratch<uint32_t>(P);
  auto* pcnt = call.scratch<uint32_t>(P);
  if (!pw || !pcnt) return oom("rule tables", 8ull * P);
  int32_t width = 1;
  for (int32_t lv = 1; lv <= D; ++lv) width = std::max(width, g->level_off[lv + 1] - g->level_off[lv]);
  auto* lists = call.scratch<int32_t>(4 * (int64_t)width);
  auto* lcounts = call.scratch<int32_t>(4 * ((int64_t)D + 2));
  if (!lists || !lcounts) return oom("rule lists", 16ull * width);
  PhaseScope t_tables(g->ctx, GTADOC_PHASE_TV_TABLES, s);
  HIP_TRY(gt::launch_tv_tables(d, g->level_off.data(), D, toff, tsize, pw, pcnt, lists, lcounts, s));
  t_tables.end();
  // 3. group every file's inputs by (file, word bucket)
  gt::TvFiles t{};
  t.unit_off = unit_off;
  t.nunits = NU;
  t.nb = nb;
  t.toff = toff, t.tsize = tsize, t.pw = pw, t.pc = pcnt;
  const int64_t ntab = (int64_t)nb * NU;
  t.table = call.scratch<uint32_t>(ntab + 1);
  auto* sums32 = call.scratch<uint32_t>(gt::scan_scratch_entries(std::max<int64_t>(ntab, F * (int64_t)nb)));
  if (!t.table || !sums32) return oom("term vector table", 4ull * ntab);
  HIP_TRY(gt::launch_fill_i32(reinterpret_cast<int32_t*>(t.table), ntab + 1, 0, s));
  HIP_TRY(gt::launch_tv_count(d, t, s));
  HIP_TRY(gt::launch_scan_u32_ext(t.table, ntab, tot + 2, sums32, s));
  HIP_TRY(hipMemcpyAsync(pc, tot + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t E = pc[0];
  if (E >= (1ll << 32)) return fail(GTADOC_ERR_UNSUPPORTED, "term vector: more than 2^32 merge inputs");
  auto* entries = call.scratch<uint64_t>(E);
  auto* nnz = call.scratch<uint32_t>(F * (int64_t)nb + 1);
  if (!entries || !nnz) return oom("term vector entries", 8ull * E);
  PhaseScope t_reduce(g->ctx, GTADOC_PHASE_TV_REDUCE, s);
  HIP_TRY(gt::launch_tv_scatter(d, t, entries, s));
  // 4. dense LDS sums per group, then the CSR
  auto* glists = call.scratch<int32_t>(F * (int64_t)nb);
  auto* gcounts = call.scratch<int32_t>(1);
  if (!glists || !gcounts) return oom("term vector group lists", 4ull * F * nb);
  HIP_TRY(gt::launch_tv_reduce(d, t, entries, E, nnz, glists, gcounts, s));
  t_reduce.end();
  auto* noff = call.scratch<uint32_t>(F * (int64_t)nb + 1);
  if (!noff) return oom("term vector offsets", 4ull * F * nb);
  HIP_TRY(hipMemcpyAsync(noff, nnz, 4 * F * (int64_t)nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(gt::launch_scan_u32_ext(noff, F * (int64_t)nb, tot + 3, sums32, s));
  HIP_TRY(hipMemcpyAsync(pc, tot + 3, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t NNZ = pc[0];
  TvArrays a;
  a.nnz = NNZ;
  if (owner) {
    a.off = call.keep<int64_t>(F + 1, *owner);
    a.word = call.keep<uint32_t>(NNZ, *owner);
    a.cnt = call.keep<uint64_t>(NNZ, *owner);
  } else {
    a.off = call.scratch<int64_t>(F + 1);
    a.word = call.scratch<uint32_t>(NNZ);
    a.cnt = call.scratch<uint64_t>(NNZ);
  }
  if (!a.off || !a.word || !a.cnt) return oom("term vector result", 12ull * NNZ);
  HIP_TRY(gt::launch_tv_emit(d, t, entries, E, nnz, noff, a.word, a.cnt, a.off, s));
  HIP_TRY(gt::launch_fill_u64(reinterpret_cast<uint64_t*>(a.off + F), 1, (uint64_t)NNZ, s));
  *out = a;
  return GTADOC_OK;
}

}  // namespace

namespace {
// Term vector by the top-down traversal (few files): per group of kTdGroup
// files, per-file rule weights from the root's references down the levels,
// then one word-count pass per file with its weight column into a dense
// F x V count matrix, compacted into the rows.
int term_vector_topdown_into(gtadoc_grammar g, Call& call, std::vector<Block>* owner, TvArrays* out) {
  const gt::DevGrammar& d = g->d;
  hipStream_t s = call.stream();
  const int64_t R = d.R, F = d.F, V = d.V, W = g->st.word_syms;
  const int32_t D = (int32_t)g->st.depth;
  if (d.wc_nb == 0)
    return fail(GTADOC_ERR_UNSUPPORTED, "top-down term vector: vocabularies above 2^24 words are not supported");
  const int64_t n = F * V;
  const int64_t nb = (n + 4095) / 4096;
  auto* dense = call.scratch<uint64_t>(n);
  auto* wgrp = call.scratch<uint64_t>(R * gt::kTdGroup);
  auto* wcol = call.scratch<uint64_t>(R);
  auto* entries = call.scratch<uint32_t>(W);
  auto* blk = call.scratch<uint32_t>(nb + gt::scan_scratch_entries(nb));
  auto* tot = call.scratch<int64_t>(2);
  auto* sums64 = call.scratch<uint64_t>(gt::scan_scratch_entries(F + 1));
  if (!dense || !wgrp || !wcol || !entries || !blk || !tot || !sums64)
    return oom("top-down term vector scratch", 8ull * n + 80ull * R + 4ull * W);
  PhaseScope t(g->ctx, GTADOC_PHASE_TV_TOPDOWN, s);
  for (int64_t f0 = 0; f0 < F; f0 += gt::kTdGroup) {
    const int32_t nf = (int32_t)std::min<int64_t>(gt::kTdGroup, F - f0);
    HIP_TRY(gt::launch_fill_u64(wgrp, R * gt::kTdGroup, 0, s));
    HIP_TRY(gt::launch_td_root(d, f0, nf, wgrp, s));
    HIP_TRY(gt::launch_td_levels(d, g->level_off.data(), D, wgrp, s));
    for (int32_t j = 0; j < nf; ++j) {
      HIP_TRY(gt::launch_td_column(wgrp, R, j, wcol, s));
      gt::DevGrammar df = d;
      df.w = wcol;
      df.span_file = f0 + j;
      if (W > 0) {
        HIP_TRY(gt::launch_word_count_buckets(df, dense + (f0 + j) * V, entries, W, g->ctx->wc_chunk, s));
      } else {
        HIP_TRY(gt::launch_fill_u64(dense + (f0 + j) * V, V, 0, s));
      }
    }
  }
  HIP_TRY(gt::launch_td_compact_count(dense, n, blk, s));
  HIP_TRY(gt::launch_scan_u32_ext(blk, nb, tot, blk + nb, s));
  auto* pc = reinterpret_cast<int64_t*>(g->ctx->pinned);
  HIP_TRY(hipMemcpyAsync(pc, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t NNZ = pc[0];
  int64_t* off;
  uint32_t* word;
  uint64_t* cnt;
  if (owner) {
    off = call.keep<int64_t>(F + 1, *owner);
    word = call.keep<uint32_t>(NNZ, *owner);
    cnt = call.keep<uint64_t>(NNZ, *owner);
  } else {
    off = call.scratch<int64_t>(F + 1);
    word = call.scratch<uint32_t>(NNZ);
    cnt = call.scratch<uint64_t>(NNZ);
  }
  if (!off || !word || !cnt) return oom("term vector", 12ull * NNZ);
  HIP_TRY(gt::launch_td_compact_write(dense, n, (int32_t)V, blk, word, cnt, s));
  HIP_TRY(gt::launch_fill_u64(reinterpret_cast<uint64_t*>(off), F + 1, 0, s));
  HIP_TRY(gt::launch_td_row_off(dense, F, (int32_t)V, off, s));
  HIP_TRY(gt::launch_scan_u64_ext(reinterpret_cast<uint64_t*>(off), F + 1, nullptr, sums64, s));
  t.end();
  out->off = off;
  out->word = word;
  out->cnt = cnt;
  out->nnz = NNZ;
  return GTADOC_OK;
}

// The traversal the selector takes: top-down for few files whose dense
// counts are small, bottom-up otherwise.
constexpr int64_t kTdAutoMaxFiles = 16;
constexpr uint64_t kTdAutoMaxDense = 1ull << 30;
int tv_auto_strategy(gtadoc_grammar g) {
  const int64_t F = g->d.F, V = g->d.V;
  if (g->d.wc_nb > 0 && F <= kTdAutoMaxFiles && 8ull * (uint64_t)F * (uint64_t)V <= kTdAutoMaxDense)
    return GTADOC_TV_TOP_DOWN;
  return GTADOC_TV_BOTTOM_UP;
}

int term_vector_any_into(gtadoc_grammar g, int strategy, Call& call, std::vector<Block>* owner, TvArrays* out) {
  if (strategy == GTADOC_TV_AUTO) strategy = tv_auto_strategy(g);
  if (strategy == GTADOC_TV_TOP_DOWN) return term_vector_topdown_into(g, call, owner, out);
  return term_vector_into(g, call, owner, out);
}

int term_vector_run(gtadoc_grammar g, int strategy, Call& call, gtadoc_result* out) {
  int rc;
  gtadoc_result res = new_result(g->ctx);
  if (!res) return fail(GTADOC_ERR_OOM, "host allocation failed");
  TvArrays a;
  rc = term_vector_any_into(g, strategy, call, &res->blocks, &a);
  if (rc) {
    (void)hipStreamSynchronize(call.stream());
    release_all(g->ctx, res->blocks);
    delete res;
    return rc;
  }
  res->a[0] = {a.off, g->d.F + 1, 8};
  res->a[1] = {a.word, a.nnz, 4};
  res->a[2] = {a.cnt, a.nnz, 8};
  res->na = 3;
  res->tv_of = g;
  *out = res;
  return GTADOC_OK;
}

int term_vector_entry(gtadoc_grammar g, int strategy, gtadoc_result* out, void* stream) {
  if (!g || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (strategy != GTADOC_TV_AUTO && strategy != GTADOC_TV_BOTTOM_UP && strategy != GTADOC_TV_TOP_DOWN)
    return fail(GTADOC_ERR_INVALID_ARG, "unknown term vector strategy %d", strategy);
  if (int rl = ensure_levels(g, stream)) return rl;
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  return term_vector_run(g, strategy, call, out);
}
}  // namespace

int gtadoc_term_vector(gtadoc_grammar g, gtadoc_result* out, void* stream) {
  return term_vector_entry(g, GTADOC_TV_AUTO, out, stream);
}

int gtadoc_term_vector_ex(gtadoc_grammar g, int strategy, gtadoc_result* out, void* stream) {
  return term_vector_entry(g, strategy, out, stream);
}

int gtadoc_term_vector_strategy(gtadoc_grammar g, int* strategy) {
  if (!g || !strategy) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  *strategy = tv_auto_strategy(g);
  return GTADOC_OK;
}

namespace {
// Inverted index of g from its term vector `a`, into a new result.
int inverted_index_from(gtadoc_grammar g, Call& call, const TvArrays& a, bool ranked, gtadoc_result* out) {
  hipStream_t s = call.stream();
  const int64_t NNZ = a.nnz;
  const int32_t V = g->d.V;
  gtadoc_result res = new_result(g->ctx);
  if (!res) return fail(GTADOC_ERR_OOM, "host allocation failed");
  auto* ii_off = call.keep<int64_t>((int64_t)V + 1, res->blocks);
  auto* file = call.keep<uint32_t>(NNZ, res->blocks);
  auto* tf = ranked ? call.keep<uint64_t>(NNZ, res->blocks) : nullptr;
  auto* k0 = call.scratch<uint64_t>(NNZ);
  auto* k1 = call.scratch<uint64_t>(NNZ);
  auto* kout = call.scratch<uint64_t>(NNZ);
  auto* v0 = call.scratch<uint32_t>(NNZ);
  auto* v1 = call.scratch<uint32_t>(NNZ);
  auto* hist = call.scratch<uint32_t>(gt::sort_scratch_hist_entries(NNZ));
  auto* num = call.scratch<int64_t>(1);
  if (!ii_off || !file || (ranked && !tf) || !k0 || !k1 || !kout || !v0 || !v1 || !hist || !num) {
    (void)hipStreamSynchronize(s);
    release_all(g->ctx, res->blocks);
    delete res;
    return oom("inverted index", 48ull * NNZ);
  }
  hipError_t e = gt::launch_fill_u64(reinterpret_cast<uint64_t*>(num), 1, (uint64_t)NNZ, s);
  if (e == hipSuccess)
    e = gt::launch_ii(a.off, g->d.F, a.word, ranked ? a.cnt : nullptr, NNZ, V, k0, v0, k1, v1, kout, file, num, hist,
                      ii_off, tf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    release_all(g->ctx, res->blocks);
    delete res;
    return fail(GTADOC_ERR_HIP, "inverted index: %s", hipGetErrorString(e));
  }
  res->a[0] = {ii_off, (int64_t)V + 1, 8};
  res->a[1] = {file, NNZ, 4};
  res->na = 2;
  if (ranked) res->a[2] = {tf, NNZ, 8}, res->na = 3;
  *out = res;
  return GTADOC_OK;
}

int inverted_index_run(gtadoc_grammar g, bool ranked, Call& call, gtadoc_result* out) {
  TvArrays a;
  const int rc = term_vector_any_into(g, GTADOC_TV_AUTO, call, nullptr, &a);
  if (rc) return rc;
  return inverted_index_from(g, call, a, ranked, out);
}

int inverted_index_entry(gtadoc_grammar g, bool ranked, gtadoc_result* out, void* stream) {
  if (!g || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (int rl = ensure_levels(g, stream)) return rl;
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  return inverted_index_run(g, ranked, call, out);
}

int inverted_index_from_tv_entry(gtadoc_grammar g, gtadoc_result term_vector, bool ranked, gtadoc_result* out,
                                 void* stream) {
  if (!g || !term_vector || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (term_vector->tv_of != g) return fail(GTADOC_ERR_INVALID_ARG, "not a term vector result of this grammar");
  Call call(g->ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  TvArrays a;
  a.off = static_cast<int64_t*>(term_vector->a[0].p);
  a.word = static_cast<uint32_t*>(term_vector->a[1].p);
  a.cnt = static_cast<uint64_t*>(term_vector->a[2].p);
  a.nnz = term_vector->a[1].n;
  return inverted_index_from(g, call, a, ranked, out);
}
}  // namespace

int gtadoc_inverted_index(gtadoc_grammar g, gtadoc_result* out, void* stream) {
  return inverted_index_entry(g, false, out, stream);
}

int gtadoc_inverted_index_from_tv(gtadoc_grammar g, gtadoc_result term_vector, gtadoc_result* out, void* stream) {
  return inverted_index_from_tv_entry(g, term_vector, false, out, stream);
}

int gtadoc_ranked_inverted_index(gtadoc_grammar g, gtadoc_result* out, void* stream) {
  return inverted_index_entry(g, true, out, stream);
}

int gtadoc_ranked_inverted_index_from_tv(gtadoc_grammar g, gtadoc_result term_vector, gtadoc_result* out,
                                         void* stream) {
  return inverted_index_from_tv_entry(g, term_vector, true, out, stream);
}

namespace {
int sequence_args(gtadoc_grammar g, int n) {
  if (n < 2 || n > 4) return fail(GTADOC_ERR_INVALID_ARG, "n must be 2, 3 or 4");
  const gt::DevGrammar& d = g->d;
  if (n == 3 && d.V > (1 << 21)) return fail(GTADOC_ERR_UNSUPPORTED, "trigram keys need vocab <= 2^21");
  if (n == 4 && d.V > (1 << 16) - 1) return fail(GTADOC_ERR_UNSUPPORTED, "4-gram keys need vocab < 2^16");
  return GTADOC_OK;
}

// The head/tail/len buffers of sequence count (Section "Sequence Support",
// initialization phase), built children first on the first use and kept
// with the grammar.
int ensure_headtail(gtadoc_grammar g, Call& call) {
  if (g->seq_len) return GTADOC_OK;
  const gt::DevGrammar& d = g->d;
  hipStream_t s = call.stream();
  const int64_t R = d.R;
  {
    std::vector<Block> kept;
    auto* len = call.keep<uint64_t>(R, kept);
    auto* head = call.keep<int32_t>(4 * R, kept);  // first / last 3 words of every rule (n <= 4), 16 B rows
    auto* tail = call.keep<int32_t>(4 * R, kept);
    if (!len || !head || !tail) {
      release_all(g->ctx, kept);
      return oom("head/tail buffers", 24ull * R);
    }
    hipError_t e = gt::launch_headtail(d, g->level_off.data(), (int32_t)g->st.depth, len, head, tail, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      release_all(g->ctx, kept);
      return fail(GTADOC_ERR_HIP, "head/tail: %s", hipGetErrorString(e));
    }
    g->blocks.insert(g->blocks.end(), kept.begin(), kept.end());
    g->seq_len = len, g->seq_head = head, g->seq_tail = tail;
  }
  return GTADOC_OK;
}

int sequence_count_run(gtadoc_grammar g, int n, Call& call, gtadoc_result* out) {
  const gt::DevGrammar& d = g->d;
  hipStream_t s = call.stream();
  const int64_t S = d.S;
  int rc = ensure_headtail(g, call);
  if (rc) return rc;
  // graph traversal phase: owned windows into an exact table sized from the
  // per-rule bound (at most n-1 windows start at every body position): the
  // table holds at least as many slots as there can be distinct keys (the
  // load factor stays under 1; on text, distinct n-grams are far fewer than
  // windows, so it is about 0.5)
  const uint64_t bound = (uint64_t)(n - 1) * (uint64_t)S + 1;
  uint64_t cap = 1024;
  while (cap < bound) cap <<= 1;
  auto* table = call.scratch<uint64_t>(2 * (int64_t)cap);
  const int64_t nb = ((int64_t)cap + 4095) / 4096;
  auto* cnt = call.scratch<uint32_t>(nb + gt::scan_scratch_entries(nb));
  auto* flags = call.scratch<int64_t>(2);  // [0] distinct keys, [1] overflow flag
  if (!table || !cnt || !flags) return oom("sequence table", 16 * cap);
  HIP_TRY(gt::launch_fill_i32(reinterpret_cast<int32_t*>(flags), 4, 0, s));
  PhaseScope t_win(g->ctx, GTADOC_PHASE_SEQ_WINDOWS, s);
  HIP_TRY(gt::launch_seq_windows(d, n, g->seq_len, g->seq_head, g->seq_tail, table, cap,
                                 reinterpret_cast<uint32_t*>(flags + 1), s));
  t_win.end();
  HIP_TRY(gt::launch_occ_count(table, (int64_t)cap, cnt, flags, cnt + nb, s));
  auto* pc = reinterpret_cast<int64_t*>(g->ctx->pinned);
  HIP_TRY(hipMemcpyAsync(pc, flags, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (pc[1] & 0xffffffff) return fail(GTADOC_ERR_OVERFLOW, "sequence table full");
  const int64_t U = pc[0];
  gtadoc_result res = new_result(g->ctx);
  if (!res) return fail(GTADOC_ERR_OOM, "host allocation failed");
  auto* okey = call.keep<uint64_t>(U, res->blocks);
  auto* oval = call.keep<uint64_t>(U, res->blocks);
  auto* k0 = call.scratch<uint64_t>(U);
  auto* v0 = call.scratch<uint64_t>(U);
  auto* k1 = call.scratch<uint64_t>(U);
  auto* v1 = call.scratch<uint64_t>(U);
  auto* hist = call.scratch<uint32_t>(gt::key_sort_hist_entries(U));
  if (!okey || !oval || !k0 || !v0 || !k1 || !v1 || !hist) {
    release_all(g->ctx, res->blocks);
    delete res;
    return oom("sequence result", 48 * (uint64_t)U);
  }
  if (U > 0) {
    hipError_t e = gt::launch_occ_write(table, (int64_t)cap, cnt, k0, v0, s);
    if (e == hipSuccess)
      e = gt::launch_sort_key_bits(k0, v0, k1, v1, U, gram_key_bits(n, d.V), hist, okey, oval, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      release_all(g->ctx, res->blocks);
      delete res;
      return fail(GTADOC_ERR_HIP, "sequence sort: %s", hipGetErrorString(e));
    }
  }
  res->a[0] = {okey, U, 8};
  res->a[1] = {oval, U, 8};
  res->na = 2;
  *out = res;
  return GTADOC_OK;
}
}  // namespace

namespace {
// Byte mask covering bits [0, nbits) of a 64-bit key.
uint64_t low_bytes_mask(int nbits) {
  uint64_t m = 0;
  for (int x = 0; x * 8 < nbits && x < 8; ++x) m |= 1ull << x;
  return m;
}

int sequence_count_wide_run(gtadoc_grammar g, int n, Call& call, gtadoc_result* out) {
  const gt::DevGrammar& d = g->d;
  hipStream_t s = call.stream();
  const int64_t R = d.R, S = d.S;
  const int b = std::max(1, bitlen((uint64_t)(d.V - 1)));
  if (n * b > 126)
    return fail(GTADOC_ERR_UNSUPPORTED, "wide sequence keys hold 126 bits: n = %d words of %d bits do not fit", n, b);
  if (!g->seqw_len) {  // initialization phase: buffers of up to 7 words, children first
    std::vector<Block> kept;
    auto* len = call.keep<uint64_t>(R, kept);
    auto* head = call.keep<int32_t>(8 * R, kept);
    auto* tail = call.keep<int32_t>(8 * R, kept);
    if (!len || !head || !tail) {
      release_all(g->ctx, kept);
      return oom("wide head/tail buffers", 72ull * R);
    }
    hipError_t e = gt::launch_headtail_wide(d, g->level_off.data(), (int32_t)g->st.depth, len, head, tail, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      release_all(g->ctx, kept);
      return fail(GTADOC_ERR_HIP, "wide head/tail: %s", hipGetErrorString(e));
    }
    g->blocks.insert(g->blocks.end(), kept.begin(), kept.end());
    g->seqw_len = len, g->seqw_head = head, g->seqw_tail = tail;
  }
  // at most n-1 windows start at a body position: the table has more slots than distinct keys
  const uint64_t bound = (uint64_t)(n - 1) * (uint64_t)S + 1;
  uint64_t cap = 1024;
  while (cap < bound) cap <<= 1;
  auto* table = call.scratch<uint64_t>(4 * (int64_t)cap);
  const int64_t nb = ((int64_t)cap + 4095) / 4096;
  auto* cnt = call.scratch<uint32_t>(nb + gt::scan_scratch_entries(nb));
  auto* flags = call.scratch<int64_t>(2);  // [0] distinct keys, [1] overflow flag
  if (!table || !cnt || !flags) return oom("wide sequence table", 32 * cap);
  HIP_TRY(gt::launch_fill_i32(reinterpret_cast<int32_t*>(flags), 4, 0, s));
  PhaseScope t_win(g->ctx, GTADOC_PHASE_SEQ_WINDOWS, s);
  HIP_TRY(gt::launch_seq_windows_wide(d, n, g->seqw_len, g->seqw_head, g->seqw_tail, b, table, cap,
                                      reinterpret_cast<uint32_t*>(flags + 1), s));
  t_win.end();
  HIP_TRY(gt::launch_wocc_count(table, (int64_t)cap, cnt, flags, cnt + nb, s));
  auto* pc = reinterpret_cast<int64_t*>(g->ctx->pinned);
  HIP_TRY(hipMemcpyAsync(pc, flags, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (pc[1] & 0xffffffff) return fail(GTADOC_ERR_OVERFLOW, "wide sequence table full");
  const int64_t U = pc[0];
  gtadoc_result res = new_result(g->ctx);
  if (!res) return fail(GTADOC_ERR_OOM, "host allocation failed");
  auto* ohi = call.keep<uint64_t>(U, res->blocks);
  auto* olo = call.keep<uint64_t>(U, res->blocks);
  auto* ocnt = call.keep<uint64_t>(U, res->blocks);
  uint64_t* k[3] = {call.scratch<uint64_t>(U), call.scratch<uint64_t>(U), call.scratch<uint64_t>(U)};
  uint32_t* v[3] = {call.scratch<uint32_t>(U), call.scratch<uint32_t>(U), call.scratch<uint32_t>(U)};
  auto* hist = call.scratch<uint32_t>(gt::sort_scratch_hist_entries(U));
  if (!ohi || !olo || !ocnt || !k[0] || !k[1] || !k[2] || !v[0] || !v[1] || !v[2] || !hist) {
    release_all(g->ctx, res->blocks);
    delete res;
    return oom("wide sequence result", 60ull * U);
  }
  if (U > 0) {
    const int total_bits = n * b;
    const hipError_t e = gt::launch_wide_sort(table, (int64_t)cap, cnt, flags, U, low_bytes_mask(std::min(63, total_bits)),
                                              low_bytes_mask(std::max(0, total_bits - 63)), k, v, hist, ohi, olo, ocnt, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      release_all(g->ctx, res->blocks);
      delete res;
      return fail(GTADOC_ERR_HIP, "wide sequence sort: %s", hipGetErrorString(e));
    }
  }
  res->a[0] = {ohi, U, 8};
  res->a[1] = {olo, U, 8};
  res->a[2] = {ocnt, U, 8};
  res->na = 3;
  *out = res;
  return GTADOC_OK;
}
}  // namespace

int gtadoc_sequence_count_wide(gtadoc_grammar g, int n, gtadoc_result* out, void* stream) {
  if (!g || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (n < 2 || n > 8) return fail(GTADOC_ERR_INVALID_ARG, "n must be in 2..8");
  if (int rl = ensure_levels(g, stream)) return rl;
  Call call(g->ctx, stream);
  const int rc = call.begin();
  if (rc) return rc;
  return sequence_count_wide_run(g, n, call, out);
}

int gtadoc_sequence_count(gtadoc_grammar g, int n, gtadoc_result* out, void* stream) {
  if (!g || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  int rc = sequence_args(g, n);
  if (rc) return rc;
  if ((rc = ensure_levels(g, stream))) return rc;
  Call call(g->ctx, stream);
  rc = call.begin();
  if (rc) return rc;
  return sequence_count_run(g, n, call, out);
}

int gtadoc_ctx_set_param(gtadoc_ctx ctx, int param, int64_t value) {
  if (!ctx) return fail(GTADOC_ERR_INVALID_ARG, "null context");
  switch (param) {
    case GTADOC_PARAM_WC_CHUNK:
      if (value < 1024 || value > (1ll << 30)) return fail(GTADOC_ERR_INVALID_ARG, "chunk out of range");
      ctx->wc_chunk = value;
      break;
    case GTADOC_PARAM_BATCH_BLOCKS_PER_CU:
      if (value < 1 || value > 16) return fail(GTADOC_ERR_INVALID_ARG, "blocks per CU out of range");
      ctx->batch_blocks_per_cu = value;
      break;
    case GTADOC_PARAM_BATCH_GRAPH:
      ctx->batch_graph = value ? 1 : 0;
      break;
    case GTADOC_PARAM_TIMING:
      if (value < 0 || value >= (2ll << GTADOC_NUM_PHASES)) return fail(GTADOC_ERR_INVALID_ARG, "timing mask out of range");
      ctx->timing = value;
      return GTADOC_OK;  // changes no launch sequence
    case GTADOC_PARAM_LEVEL_WIDE:
      if (value < 0) return fail(GTADOC_ERR_INVALID_ARG, "level width threshold out of range");
      ctx->level_wide = value;
      return GTADOC_OK;  // read at load time only
    case GTADOC_PARAM_LEVEL_LONG_BODY:
      if (value < 1 || value > (1 << 20)) return fail(GTADOC_ERR_INVALID_ARG, "long-body threshold out of range");
      ctx->level.long_body = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_LEVEL_MID_RULES:
      if (value < 1 || value > INT32_MAX) return fail(GTADOC_ERR_INVALID_ARG, "mid-level threshold out of range");
      ctx->level.mid_rules = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_LEVEL_MID_BLOCKS:
      if (value < 1 || value > 256) return fail(GTADOC_ERR_INVALID_ARG, "mid-level workgroups out of range");
      ctx->level.mid_blocks = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_LEVEL_TAIL_RULES:
      if (value < 1 || value > INT32_MAX) return fail(GTADOC_ERR_INVALID_ARG, "tail-level threshold out of range");
      ctx->level.tail_rules = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_FLOW_KEEP:
      if (value < 0 || value > 7168) return fail(GTADOC_ERR_INVALID_ARG, "ring threshold out of range (0..7168)");
      ctx->level.flow_keep = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_FLOW_CHUNK:
      if (value < 1 || value > 65535) return fail(GTADOC_ERR_INVALID_ARG, "level-1 chunk out of range (1..65535)");
      ctx->level.flow_chunk = (int32_t)value;
      return GTADOC_OK;
    case GTADOC_PARAM_FLOW_GROUP:
      if (value != 512 && value != 1024) return fail(GTADOC_ERR_INVALID_ARG, "dataflow workgroup size must be 512 or 1024");
      ctx->level.flow_group = (int32_t)value;
      return GTADOC_OK;
    default:
      return fail(GTADOC_ERR_INVALID_ARG, "unknown parameter %d", param);
  }
  ++ctx->param_epoch;
  return GTADOC_OK;
}

int gtadoc_ctx_get_param(gtadoc_ctx ctx, int param, int64_t* value) {
  if (!ctx || !value) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  switch (param) {
    case GTADOC_PARAM_WC_CHUNK: *value = ctx->wc_chunk; break;
    case GTADOC_PARAM_BATCH_BLOCKS_PER_CU: *value = ctx->batch_blocks_per_cu; break;
    case GTADOC_PARAM_BATCH_GRAPH: *value = ctx->batch_graph; break;
    case GTADOC_PARAM_TIMING: *value = ctx->timing; break;
    case GTADOC_PARAM_LEVEL_WIDE: *value = ctx->level_wide; break;
    case GTADOC_PARAM_LEVEL_LONG_BODY: *value = ctx->level.long_body; break;
    case GTADOC_PARAM_LEVEL_MID_RULES: *value = ctx->level.mid_rules; break;
    case GTADOC_PARAM_LEVEL_MID_BLOCKS: *value = ctx->level.mid_blocks; break;
    case GTADOC_PARAM_LEVEL_TAIL_RULES: *value = ctx->level.tail_rules; break;
    case GTADOC_PARAM_FLOW_KEEP: *value = ctx->level.flow_keep; break;
    case GTADOC_PARAM_FLOW_GROUP: *value = ctx->level.flow_group; break;
    case GTADOC_PARAM_FLOW_CHUNK: *value = ctx->level.flow_chunk; break;
    default: return fail(GTADOC_ERR_INVALID_ARG, "unknown parameter %d", param);
  }
  return GTADOC_OK;
}

int gtadoc_ctx_phase_time(gtadoc_ctx ctx, int phase, double* total_ms, int64_t* count, int reset) {
  if (!ctx || phase < 0 || phase >= GTADOC_NUM_PHASES) return fail(GTADOC_ERR_INVALID_ARG, "bad context or phase");
  auto& t = ctx->timers[phase];
  fold_timer(t);
  if (total_ms) *total_ms = t.ms;
  if (count) *count = t.n;
  if (reset) t.ms = 0, t.n = 0;
  return GTADOC_OK;
}

int gtadoc_batch_create(gtadoc_ctx ctx, int max_items, uint64_t max_entries, gtadoc_batch* out) {
  if (!ctx || !out) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (max_items < 1 || max_items > gt::kBatchMax) return fail(GTADOC_ERR_INVALID_ARG, "max_items out of range");
  auto* b = new (std::nothrow) gtadoc_batch_s;
  if (!b) return fail(GTADOC_ERR_OOM, "host allocation failed");
  b->ctx = ctx;
  b->max_items = max_items;
  b->max_entries = max_entries;
  Block blk;
  if (!ctx->arena.alloc(sizeof(gt::BatchDesc), &blk)) {
    delete b;
    return oom("batch descriptors", sizeof(gt::BatchDesc));
  }
  b->blocks.push_back(blk);
  b->dev = reinterpret_cast<gt::BatchDesc*>(ctx->base + blk.off);
  if (!ctx->arena.alloc(std::max<uint64_t>(max_entries, 1) * 4, &blk)) {
    release_all(ctx, b->blocks);
    delete b;
    return oom("batch entries", 4 * max_entries);
  }
  b->blocks.push_back(blk);
  b->entries = reinterpret_cast<uint32_t*>(ctx->base + blk.off);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->host), sizeof(gt::BatchDesc), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    if (b->host) (void)hipHostFree(b->host);
    release_all(ctx, b->blocks);
    delete b;
    return fail(GTADOC_ERR_HIP, "batch setup failed");
  }
  std::memset(b->host, 0, sizeof(gt::BatchDesc));
  *out = b;
  return GTADOC_OK;
}

int gtadoc_batch_destroy(gtadoc_batch b) {
  if (!b) return fail(GTADOC_ERR_INVALID_ARG, "null batch");
  if (b->launched) (void)hipEventSynchronize(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  for (int k = 0; k < gtadoc_batch_s::kStreams; ++k) {
    if (b->pool[k]) (void)hipStreamSynchronize(b->pool[k]), (void)hipStreamDestroy(b->pool[k]);
    if (b->pool_done[k]) (void)hipEventDestroy(b->pool_done[k]);
  }
  if (b->start) (void)hipEventDestroy(b->start);
  (void)hipEventDestroy(b->done);
  (void)hipHostFree(b->host);
  release_all(b->ctx, b->blocks);
  delete b;
  return GTADOC_OK;
}

int gtadoc_batch_word_count(gtadoc_batch b, const gtadoc_grammar* gs, uint64_t* const* counts, int n, void* stream) {
  if (!b || (n > 0 && (!gs || !counts))) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (n < 0 || n > b->max_items) return fail(GTADOC_ERR_INVALID_ARG, "batch of %d exceeds the plan (%d)", n, b->max_items);
  gtadoc_ctx ctx = b->ctx;
  // descriptors are rewritten only after the plan's previous batch finished
  if (b->launched && hipEventSynchronize(b->done) != hipSuccess) return fail(GTADOC_ERR_HIP, "batch wait failed");
  gt::BatchDesc& h = *b->host;
  h.n = n;
  h.chunk = ctx->wc_chunk;
  h.fill_base[0] = h.scatter_base[0] = h.reduce_base[0] = 0;
  uint64_t used = 0;
  for (int i = 0; i < n; ++i) {
    const gtadoc_grammar g = gs[i];
    if (!g || g->ctx != ctx || !counts[i]) return fail(GTADOC_ERR_INVALID_ARG, "item %d: null or foreign grammar", i);
    if (g->d.wc_nb == 0)
      return fail(GTADOC_ERR_UNSUPPORTED, "item %d: grammar needs the direct word count", i);
    const int64_t W = g->st.word_syms;
    gt::BatchItem& it = h.items[i];
    it.g = g->d;
    it.out = counts[i];
    it.entries = b->entries + used;
    it.W = W;
    used += (uint64_t)W;
    h.fill_base[i + 1] = h.fill_base[i] + (g->d.V + gt::kWcBucket - 1) / gt::kWcBucket;
    h.scatter_base[i + 1] = h.scatter_base[i] + (W > 0 ? g->d.nblk : 0);
    h.reduce_base[i + 1] = h.reduce_base[i] + (W + h.chunk - 1) / h.chunk;
  }
  if (used > b->max_entries)
    return fail(GTADOC_ERR_INVALID_ARG, "batch needs %llu entries, plan holds %llu", (unsigned long long)used,
                (unsigned long long)b->max_entries);
  Call call(ctx, stream);
  int rc = call.begin();
  if (rc) return rc;
  hipStream_t s = call.stream();
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int grid_scatter = (int)(cus * ctx->batch_blocks_per_cu);
  const int grid_reduce = cus;
  // the launch sequence: descriptors to the device, then the persistent kernels
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    hipError_t e = hipMemcpyAsync(b->dev, b->host, sizeof(gt::BatchDesc), hipMemcpyHostToDevice, q);
    if (e != hipSuccess) return e;
    return gt::launch_word_count_batch(b->dev, grid_scatter, grid_reduce, gt::kWcMaxBuckets, q);
  };
  if (ctx->batch_graph) {
    // captured once on the plan's own stream (the caller's may be the null
    // stream, which cannot capture), replayed on the caller's stream; the
    // copy node reads the pinned descriptors at each replay
    if (!b->exec || b->graph_epoch != ctx->param_epoch) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec), b->exec = nullptr;
      if (b->graph) (void)hipGraphDestroy(b->graph), b->graph = nullptr;
      if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(b->capture);
      hipGraph_t graph = nullptr;
      const hipError_t e2 = hipStreamEndCapture(b->capture, &graph);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(GTADOC_ERR_HIP, "batch capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      }
      b->graph = graph;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_epoch = ctx->param_epoch;
    }
    HIP_TRY(hipGraphLaunch(b->exec, s));
  } else {
    HIP_TRY(enqueue(s));
  }
  HIP_TRY(hipEventRecord(b->done, s));
  b->launched = true;
  return GTADOC_OK;
}

int gtadoc_batch_submit(gtadoc_batch b, gtadoc_query* q, int nq, void* stream) {
  if (!b || nq < 0 || (nq > 0 && !q)) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  gtadoc_ctx ctx = b->ctx;
  std::vector<gtadoc_grammar> wc_g;
  std::vector<uint64_t*> wc_out;
  std::vector<int> other;
  for (int i = 0; i < nq; ++i) {
    gtadoc_query& x = q[i];
    if (!x.grammar || x.grammar->ctx != ctx) return fail(GTADOC_ERR_INVALID_ARG, "query %d: null or foreign grammar", i);
    switch (x.kind) {
      case GTADOC_QUERY_WORD_COUNT:
        if (!x.counts) return fail(GTADOC_ERR_INVALID_ARG, "query %d: null counts", i);
        wc_g.push_back(x.grammar);
        wc_out.push_back(x.counts);
        break;
      case GTADOC_QUERY_TERM_VECTOR:
        if (x.strategy != GTADOC_TV_AUTO && x.strategy != GTADOC_TV_BOTTOM_UP && x.strategy != GTADOC_TV_TOP_DOWN)
          return fail(GTADOC_ERR_INVALID_ARG, "query %d: unknown term vector strategy %d", i, x.strategy);
        other.push_back(i);
        break;
      case GTADOC_QUERY_SEQUENCE_COUNT:
        if (x.n < 2 || x.n > 4) return fail(GTADOC_ERR_INVALID_ARG, "query %d: n must be 2, 3 or 4", i);
        other.push_back(i);
        break;
      case GTADOC_QUERY_INVERTED_INDEX:
      case GTADOC_QUERY_RANKED_INVERTED_INDEX:
        other.push_back(i);
        break;
      default:
        return fail(GTADOC_ERR_INVALID_ARG, "query %d: unknown kind %d", i, x.kind);
    }
  }
  if ((int)wc_g.size() > b->max_items)
    return fail(GTADOC_ERR_INVALID_ARG, "%d word counts exceed the plan (%d)", (int)wc_g.size(), b->max_items);
  for (int i : other)  // grammars loaded without levels get them first (synchronizes once per grammar)
    if (int rl = ensure_levels(q[i].grammar, stream)) return rl;
  for (int i = 0; i < nq; ++i) q[i].status = GTADOC_OK, q[i].result = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the other queries start after the context's earlier work, not after this batch's word counts
  Call outer(ctx, stream);
  int rc = outer.begin();
  if (rc) return rc;
  if (!other.empty()) {
    if (!b->start) HIP_TRY(hipEventCreateWithFlags(&b->start, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(b->start, s));
  }
  if (!wc_g.empty()) {
    rc = gtadoc_batch_word_count(b, wc_g.data(), wc_out.data(), (int)wc_g.size(), stream);
    if (rc) {
      for (int i = 0; i < nq; ++i)
        if (q[i].kind == GTADOC_QUERY_WORD_COUNT) q[i].status = rc;
      if (rc == GTADOC_ERR_HIP) return rc;
    }
  }
  if (other.empty()) return GTADOC_OK;
  bool used[gtadoc_batch_s::kStreams] = {};
  std::vector<Block> deferred;
  int next = 0;
  for (int i : other) {
    gtadoc_query& x = q[i];
    // sequence counts of one grammar share a stream: the first builds the
    // grammar's head/tail buffers, the later ones read them
    const int k = x.kind == GTADOC_QUERY_SEQUENCE_COUNT
                      ? (int)((reinterpret_cast<uintptr_t>(x.grammar) >> 4) % gtadoc_batch_s::kStreams)
                      : next++ % gtadoc_batch_s::kStreams;
    if (!b->pool[k]) {
      HIP_TRY(hipStreamCreateWithFlags(&b->pool[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&b->pool_done[k], hipEventDisableTiming));
    }
    if (!used[k]) {
      HIP_TRY(hipStreamWaitEvent(b->pool[k], b->start, 0));
      used[k] = true;
    }
    Call qc(ctx, b->pool[k], &deferred);
    rc = qc.begin();
    if (!rc) {
      switch (x.kind) {
        case GTADOC_QUERY_TERM_VECTOR: rc = term_vector_run(x.grammar, x.strategy, qc, &x.result); break;
        case GTADOC_QUERY_SEQUENCE_COUNT:
          rc = sequence_args(x.grammar, x.n);
          if (!rc) rc = sequence_count_run(x.grammar, x.n, qc, &x.result);
          break;
        case GTADOC_QUERY_INVERTED_INDEX: rc = inverted_index_run(x.grammar, false, qc, &x.result); break;
        default: rc = inverted_index_run(x.grammar, true, qc, &x.result); break;
      }
    }
    if (rc) x.result = nullptr;
    x.status = rc;
  }
  // join the pool into the caller's stream; the queries' scratch goes back
  // to the arena now (later calls on the context wait for this stream)
  for (int k = 0; k < gtadoc_batch_s::kStreams; ++k) {
    if (!used[k]) continue;
    HIP_TRY(hipEventRecord(b->pool_done[k], b->pool[k]));
    HIP_TRY(hipStreamWaitEvent(s, b->pool_done[k], 0));
  }
  for (const Block& blk : deferred) ctx->arena.release(blk);
  return GTADOC_OK;
}

int gtadoc_query_bytes(gtadoc_grammar g, int kind, int n, int strategy, uint64_t* bytes, void* stream) {
  if (!g || !bytes) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (kind == GTADOC_QUERY_TERM_VECTOR || kind == GTADOC_QUERY_INVERTED_INDEX ||
      kind == GTADOC_QUERY_RANKED_INVERTED_INDEX) {
    if (strategy != GTADOC_TV_AUTO && strategy != GTADOC_TV_BOTTOM_UP && strategy != GTADOC_TV_TOP_DOWN)
      return fail(GTADOC_ERR_INVALID_ARG, "unknown term vector strategy %d", strategy);
    if (strategy == GTADOC_TV_AUTO || kind != GTADOC_QUERY_TERM_VECTOR) strategy = tv_auto_strategy(g);
  } else {
    strategy = 0;
  }
  if (kind == GTADOC_QUERY_SEQUENCE_COUNT) {
    const int rc = sequence_args(g, n);
    if (rc) return rc;
  } else if (kind >= GTADOC_QUERY_WORD_COUNT && kind <= GTADOC_QUERY_RANKED_INVERTED_INDEX) {
    n = 0;
  } else {
    return fail(GTADOC_ERR_INVALID_ARG, "unknown kind %d", kind);
  }
  const int64_t key = (int64_t)kind * 1000 + n * 10 + strategy;
  auto it = g->footprint.find(key);
  if (it != g->footprint.end()) {
    *bytes = it->second;
    return GTADOC_OK;
  }
  gtadoc_ctx ctx = g->ctx;
  // the level structure and sequence count's head/tail buffers belong to the
  // grammar, not the query
  if (kind != GTADOC_QUERY_WORD_COUNT)
    if (int rl = ensure_levels(g, stream)) return rl;
  if (kind == GTADOC_QUERY_SEQUENCE_COUNT && !g->seq_len) {
    Call call(ctx, stream);
    int rc = call.begin();
    if (!rc) rc = ensure_headtail(g, call);
    if (rc) return rc;
  }
  Block out_blk{};
  if (kind == GTADOC_QUERY_WORD_COUNT && !ctx->arena.alloc(8ull * g->d.V, &out_blk)) return oom("word counts", 8ull * g->d.V);
  gtadoc_result res = nullptr;
  int rc;
  {
    Call call(ctx, stream);
    rc = call.begin();
    ctx->arena.mark();
    if (!rc) {
      switch (kind) {
        case GTADOC_QUERY_WORD_COUNT:
          rc = word_count_into(g, call, reinterpret_cast<uint64_t*>(ctx->base + out_blk.off));
          break;
        case GTADOC_QUERY_TERM_VECTOR: rc = term_vector_run(g, strategy, call, &res); break;
        case GTADOC_QUERY_SEQUENCE_COUNT: rc = sequence_count_run(g, n, call, &res); break;
        case GTADOC_QUERY_INVERTED_INDEX: rc = inverted_index_run(g, false, call, &res); break;
        default: rc = inverted_index_run(g, true, call, &res); break;
      }
    }
  }
  const uint64_t peak = ctx->arena.peak_since_mark();
  (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (res) gtadoc_result_free(res);
  if (out_blk.size) ctx->arena.release(out_blk);
  if (rc) return rc;
  g->footprint[key] = peak;
  *bytes = peak;
  return GTADOC_OK;
}

int gtadoc_grammar_edges(gtadoc_grammar g, int64_t* edges, void* stream) {
  if (!g || !edges) return fail(GTADOC_ERR_INVALID_ARG, "null argument");
  if (g->edges < 0) {
    Call call(g->ctx, stream);
    int rc = call.begin();
    if (rc) return rc;
    hipStream_t s = call.stream();
    auto* flag = call.scratch<uint8_t>(g->d.R);
    auto* cnt = call.scratch<unsigned long long>(1);
    if (!flag || !cnt) return oom("edge count", (uint64_t)g->d.R);
    HIP_TRY(gt::launch_count_edges(g->d, g->st.root_syms, flag, cnt, s));
    auto* pc = reinterpret_cast<unsigned long long*>(g->ctx->pinned);
    HIP_TRY(hipMemcpyAsync(pc, cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->edges = (int64_t)*pc;
  }
  *edges = g->edges;
  return GTADOC_OK;
}

int gtadoc_result_array(gtadoc_result res, int index, void** dptr, int64_t* length, int* elem_bytes) {
  if (!res || index < 0 || index >= res->na) return fail(GTADOC_ERR_INVALID_ARG, "bad result or index");
  if (dptr) *dptr = res->a[index].p;
  if (length) *length = res->a[index].n;
  if (elem_bytes) *elem_bytes = res->a[index].eb;
  return GTADOC_OK;
}

int gtadoc_result_free(gtadoc_result res) {
  if (!res) return fail(GTADOC_ERR_INVALID_ARG, "null result");
  release_all(res->ctx, res->blocks);
  delete res;
  return GTADOC_OK;
}

}  // extern "C"
