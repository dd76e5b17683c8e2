// synth.cpp -- seeded synthetic corpora and a Sequitur grammar compressor.
//
// This module prepares inputs only. It produces token streams shaped like the
// paper's workloads (Zipf vocabularies, repeated spans, many files of uneven
// size, nested repeats) and compresses them into the grammar form the
// analytics consume (Background, "TADOC": dictionary-encoded words, a
// context-free grammar inferred by Sequitur, unique splitters between files).
// It computes no analytics result: no counts, no weights, no tables.
//
// Grammar output encoding (CSR):
//   rule_off[R+1]  body(r) = sym[rule_off[r] .. rule_off[r+1]); r = 0 is the root
//   sym[S]         s >= 0: word id (< vocab);  s < 0: reference to rule -s
//   file_off[F+1]  file f = root body [file_off[f], file_off[f+1])
// The splitters are removed from the root and become file_off.
//
// Rules are renumbered by first encounter in a left-to-right preorder walk
// from the root, so the output is a deterministic function of the input text.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Pseudo-random numbers: splitmix64 for seeding, xoshiro256** for the stream
// (both from Blackman and Vigna, "Scrambled linear pseudorandom number
// generators", 2018; written here from their published definitions).
// ---------------------------------------------------------------------------
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
};

struct Rng {
  uint64_t s[4];
  explicit Rng(uint64_t seed) {
    SplitMix64 sm{seed};
    for (auto& x : s) x = sm.next();
  }
  static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
  }
  // uniform double in [0, 1) from the top 53 bits
  double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
  // uniform integer in [0, n), n >= 1 (multiply-shift with rejection, Lemire 2019)
  uint64_t below(uint64_t n) {
    unsigned __int128 m = (unsigned __int128)next() * n;
    uint64_t lo = (uint64_t)m;
    if (lo < n) {
      const uint64_t thresh = (0 - n) % n;
      while (lo < thresh) {
        m = (unsigned __int128)next() * n;
        lo = (uint64_t)m;
      }
    }
    return (uint64_t)(m >> 64);
  }
  // uniform integer in [lo, hi]
  int64_t range(int64_t lo, int64_t hi) { return lo + (int64_t)below((uint64_t)(hi - lo + 1)); }
  // standard normal (Box-Muller)
  double normal() {
    double u1 = uniform();
    while (u1 <= 0.0) u1 = uniform();
    const double u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// ---------------------------------------------------------------------------
// Zipf(s) over ranks 1..V, sampled with Vose's alias method. Rank k maps to
// word id perm[k-1], a seeded Fisher-Yates permutation, so that frequent ids
// are scattered over [0, V) instead of clustered at 0.
// ---------------------------------------------------------------------------
struct Zipf {
  uint32_t V = 0;
  std::vector<double> prob;
  std::vector<uint32_t> alias;
  std::vector<int32_t> perm;

  Zipf(uint32_t vocab, double s, Rng& rng) : V(vocab), prob(vocab), alias(vocab), perm(vocab) {
    std::vector<double> p(V);
    double total = 0.0;
    for (uint32_t k = 0; k < V; ++k) total += (p[k] = std::pow(double(k + 1), -s));
    std::vector<uint32_t> small, large;
    small.reserve(V);
    large.reserve(V);
    for (uint32_t k = 0; k < V; ++k) {
      p[k] = p[k] * V / total;
      (p[k] < 1.0 ? small : large).push_back(k);
    }
    while (!small.empty() && !large.empty()) {
      const uint32_t a = small.back();
      small.pop_back();
      const uint32_t b = large.back();
      prob[a] = p[a];
      alias[a] = b;
      p[b] = (p[b] + p[a]) - 1.0;
      if (p[b] < 1.0) {
        large.pop_back();
        small.push_back(b);
      }
    }
    for (uint32_t k : large) prob[k] = 1.0, alias[k] = k;
    for (uint32_t k : small) prob[k] = 1.0, alias[k] = k;
    for (uint32_t k = 0; k < V; ++k) perm[k] = (int32_t)k;
    for (uint32_t k = V; k > 1; --k) std::swap(perm[k - 1], perm[rng.below(k)]);
  }
  int32_t sample(Rng& rng) const {
    const uint32_t k = (uint32_t)rng.below(V);
    const uint32_t r = rng.uniform() < prob[k] ? k : alias[k];
    return perm[r];
  }
};

// Append n tokens to out. With probability q per step, copy a span of
// L ~ U{lmin..lmax} tokens starting at a uniform position of the history
// out[hist_lo, hist_hi) (hist_hi < 0 means "everything written so far");
// otherwise emit one Zipf token. q = p / ((1-p) * Lbar + p) makes the expected
// copied fraction p.
void span_text(std::vector<int32_t>& out, int64_t n, const Zipf& z, double p, int lmin, int lmax,
               int64_t hist_lo, int64_t hist_hi, Rng& rng) {
  const double lbar = 0.5 * (lmin + lmax);
  const double q = (p <= 0.0) ? 0.0 : p / ((1.0 - p) * lbar + p);
  const int64_t end = (int64_t)out.size() + n;
  while ((int64_t)out.size() < end) {
    const int64_t hi = hist_hi < 0 ? (int64_t)out.size() : hist_hi;
    const int64_t hist = hi - hist_lo;
    if (q > 0.0 && hist >= lmin && rng.uniform() < q) {
      int64_t L = rng.range(lmin, lmax);
      L = std::min<int64_t>(L, std::min<int64_t>(hist, end - (int64_t)out.size()));
      const int64_t start = hist_lo + (int64_t)rng.below((uint64_t)(hist - L + 1));
      for (int64_t i = 0; i < L; ++i) out.push_back(out[start + i]);
    } else {
      out.push_back(z.sample(rng));
    }
  }
}

}  // namespace

// ===========================================================================
// Corpus generation (C ABI for the Python wrapper)
// ===========================================================================
extern "C" {

typedef struct {
  int32_t kind;            // 0: span-copy text (1..F files), 1: nested motif chains (1 file)
  int32_t files;           // kind 0: number of files (1 = single file, exact `tokens`)
  int64_t tokens;          // single file / kind 1: total tokens
  double lognorm_median;   // kind 0, files > 1: file sizes ~ LogNormal(ln median, sigma)
  double lognorm_sigma;
  int64_t file_min, file_max;  // clip of the lognormal file sizes
  int32_t vocab;
  double zipf_s;
  double copy_frac;        // expected fraction of tokens made by span copies
  int32_t span_min, span_max;
  int32_t cross_file;      // 1: files copy only from earlier files' tokens
  int32_t motif_chains, motif_levels, motif_min, motif_max, motif_ext_max, motif_min_inserts;
  uint64_t seed;
  int32_t normalize;       // kind 0, files > 1: scale the lognormal sizes to sum to `tokens`
} synth_params;

typedef struct {
  std::vector<int32_t> tok;
  std::vector<int64_t> file_off;
} synth_corpus;

static void gen_kind0(const synth_params& P, synth_corpus& C, Rng& rng, const Zipf& z) {
  const int F = std::max(1, P.files);
  std::vector<int64_t> sizes(F);
  if (F == 1) {
    sizes[0] = P.tokens;
  } else {
    const double mu = std::log(P.lognorm_median);
    for (int f = 0; f < F; ++f) {
      const double x = std::exp(mu + P.lognorm_sigma * rng.normal());
      int64_t t = (int64_t)std::llround(x);
      sizes[f] = std::min(std::max(t, P.file_min), P.file_max);
    }
  }
  int64_t total = 0;
  for (auto s : sizes) total += s;
  if (F > 1 && P.normalize && P.tokens > 0 && total > 0) {
    // keep the lognormal shape, rescale so the sizes sum to exactly `tokens`
    int64_t acc = 0;
    for (int f = 0; f < F; ++f) {
      const int64_t t = (int64_t)((double)sizes[f] * (double)P.tokens / (double)total);
      sizes[f] = std::max<int64_t>(1, t);
      acc += sizes[f];
    }
    sizes[F - 1] = std::max<int64_t>(1, sizes[F - 1] + (P.tokens - acc));
    total = 0;
    for (auto s : sizes) total += s;
  }
  C.tok.reserve((size_t)total);
  C.file_off.assign(1, 0);
  for (int f = 0; f < F; ++f) {
    const int64_t start = (int64_t)C.tok.size();
    if (P.cross_file)
      span_text(C.tok, sizes[f], z, P.copy_frac, P.span_min, P.span_max, 0, start, rng);
    else
      span_text(C.tok, sizes[f], z, P.copy_frac, P.span_min, P.span_max, start, -1, rng);
    C.file_off.push_back((int64_t)C.tok.size());
  }
}

// Nested repeats: `chains` chains of `levels` motifs; m0 is a fresh Zipf span
// of U{motif_min..motif_max} tokens and m(j+1) is m(j) extended on a random
// side by U{1..motif_ext_max} fresh tokens. Every motif is inserted at least
// motif_min_inserts times, extra insertions are drawn uniformly until the
// inserted tokens reach copy_frac of the text, and the insertions are
// interleaved at random with fresh Zipf tokens.
static void gen_kind1(const synth_params& P, synth_corpus& C, Rng& rng, const Zipf& z) {
  const int64_t T = P.tokens;
  const int nm = P.motif_chains * P.motif_levels;
  std::vector<std::vector<int32_t>> motif((size_t)nm);
  for (int c = 0; c < P.motif_chains; ++c) {
    std::vector<int32_t> m;
    const int64_t L0 = rng.range(P.motif_min, P.motif_max);
    for (int64_t i = 0; i < L0; ++i) m.push_back(z.sample(rng));
    for (int j = 0; j < P.motif_levels; ++j) {
      if (j > 0) {
        const int64_t e = rng.range(1, P.motif_ext_max);
        std::vector<int32_t> ext;
        for (int64_t i = 0; i < e; ++i) ext.push_back(z.sample(rng));
        if (rng.below(2)) m.insert(m.end(), ext.begin(), ext.end());
        else m.insert(m.begin(), ext.begin(), ext.end());
      }
      motif[(size_t)c * P.motif_levels + j] = m;
    }
  }
  std::vector<int32_t> events;  // motif index per insertion
  int64_t inserted = 0;
  for (int k = 0; k < nm; ++k)
    for (int r = 0; r < P.motif_min_inserts; ++r) events.push_back(k), inserted += (int64_t)motif[k].size();
  const int64_t target = (int64_t)(P.copy_frac * (double)T);
  while (inserted < target) {
    const int k = (int)rng.below((uint64_t)nm);
    events.push_back(k);
    inserted += (int64_t)motif[k].size();
  }
  for (size_t i = events.size(); i > 1; --i) std::swap(events[i - 1], events[rng.below(i)]);
  int64_t fresh = std::max<int64_t>(0, T - inserted);
  C.tok.reserve((size_t)(T + 1024));
  size_t next_event = 0;
  while ((int64_t)C.tok.size() < T) {
    const uint64_t remaining_items = (uint64_t)fresh + (events.size() - next_event);
    if (remaining_items == 0) break;
    if (next_event < events.size() && rng.below(remaining_items) < events.size() - next_event) {
      const auto& m = motif[(size_t)events[next_event++]];
      for (int32_t t : m) {
        if ((int64_t)C.tok.size() >= T) break;
        C.tok.push_back(t);
      }
    } else {
      C.tok.push_back(z.sample(rng));
      if (fresh > 0) --fresh;
    }
  }
  while ((int64_t)C.tok.size() < T) C.tok.push_back(z.sample(rng));
  C.file_off = {0, (int64_t)C.tok.size()};
}

void* synth_corpus_new(const synth_params* P) {
  if (!P || P->vocab <= 0) return nullptr;
  try {
    Rng rng(P->seed);
    Zipf z((uint32_t)P->vocab, P->zipf_s, rng);
    auto* C = new synth_corpus;
    if (P->kind == 1) gen_kind1(*P, *C, rng, z);
    else gen_kind0(*P, *C, rng, z);
    return C;
  } catch (...) {
    return nullptr;
  }
}
int64_t synth_corpus_tokens(const void* h) { return (int64_t)((const synth_corpus*)h)->tok.size(); }
int64_t synth_corpus_files(const void* h) { return (int64_t)((const synth_corpus*)h)->file_off.size() - 1; }
void synth_corpus_copy(const void* h, int32_t* tok, int64_t* file_off) {
  const auto* C = (const synth_corpus*)h;
  if (tok) std::memcpy(tok, C->tok.data(), C->tok.size() * sizeof(int32_t));
  if (file_off) std::memcpy(file_off, C->file_off.data(), C->file_off.size() * sizeof(int64_t));
}
void synth_corpus_free(void* h) { delete (synth_corpus*)h; }

}  // extern "C"

// ===========================================================================
// Sequitur (Nevill-Manning and Witten): grammar inference that keeps two
// properties while the text is read one symbol at a time:
//   digram uniqueness -- no pair of adjacent symbols occurs twice in the
//                        grammar (two overlapping occurrences inside a run
//                        such as "x x x" excepted);
//   rule utility      -- every rule other than the root is used at least twice.
// TADOC adds a unique splitter between files so that no rule spans a file
// boundary; digrams that contain a splitter are never indexed.
//
// Symbols live in doubly linked lists, one per rule, closed by a guard node.
// Pending digram checks go through an explicit work stack instead of
// recursion, so that cascades of replacements need no deep call stack. A
// pending node that has been deleted meanwhile is skipped; re-checking a
// live node is always harmless.
// ===========================================================================
namespace {

constexpr uint32_t NIL = 0xffffffffu;
constexpr int32_t GUARD_BASE = -(1 << 30);  // guard of rule r has value GUARD_BASE - r
constexpr int32_t DEAD = INT32_MIN;

struct DigramIndex {
  // open addressing, linear probing, deletion by backward shift
  struct Slot {
    uint64_t key;
    uint32_t node;  // NIL = empty
  };
  std::vector<Slot> t;
  uint64_t mask = 0, count = 0;

  static uint64_t mix(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
  }
  void init(uint64_t cap) {
    uint64_t c = 1;
    while (c < cap) c <<= 1;
    t.assign(c, Slot{0, NIL});
    mask = c - 1;
    count = 0;
  }
  uint32_t find(uint64_t key) const {
    for (uint64_t i = mix(key) & mask;; i = (i + 1) & mask) {
      if (t[i].node == NIL) return NIL;
      if (t[i].key == key) return t[i].node;
    }
  }
  void grow() {
    std::vector<Slot> old;
    old.swap(t);
    init((mask + 1) * 2);
    for (const Slot& s : old)
      if (s.node != NIL) put(s.key, s.node);
  }
  void put(uint64_t key, uint32_t node) {  // key must be absent
    if ((count + 1) * 10 > (mask + 1) * 6) grow();
    uint64_t i = mix(key) & mask;
    while (t[i].node != NIL) i = (i + 1) & mask;
    t[i] = Slot{key, node};
    ++count;
  }
  // remove key if it maps to `node`
  void erase_if(uint64_t key, uint32_t node) {
    uint64_t i = mix(key) & mask;
    for (;; i = (i + 1) & mask) {
      if (t[i].node == NIL) return;
      if (t[i].key == key) break;
    }
    if (t[i].node != node) return;
    // backward-shift deletion
    uint64_t hole = i;
    for (uint64_t j = (i + 1) & mask;; j = (j + 1) & mask) {
      if (t[j].node == NIL) break;
      const uint64_t home = mix(t[j].key) & mask;
      // move t[j] into the hole if its home is not cyclically in (hole, j]
      const bool in_range = (hole <= j) ? (home > hole && home <= j) : (home > hole || home <= j);
      if (!in_range) {
        t[hole] = t[j];
        hole = j;
      }
    }
    t[hole].node = NIL;
    --count;
  }
};

struct Sequitur {
  std::vector<int32_t> val;
  std::vector<uint32_t> prv, nxt;
  std::vector<uint32_t> free_nodes;
  std::vector<uint32_t> guard;   // per rule: guard node (NIL if freed)
  std::vector<uint32_t> refs;    // per rule: number of references
  std::vector<uint32_t> free_rules;
  std::vector<uint32_t> work;    // pending digram checks (node ids)
  DigramIndex index;
  int32_t sep_base;

  explicit Sequitur(int32_t separator_base, size_t expect) : sep_base(separator_base) {
    val.reserve(expect + 16);
    prv.reserve(expect + 16);
    nxt.reserve(expect + 16);
    index.init(std::max<uint64_t>(1024, expect));
    new_rule();  // the root
  }

  static bool is_guard(int32_t v) { return v <= GUARD_BASE && v != DEAD; }
  static bool is_ref(int32_t v) { return v < 0 && v > GUARD_BASE; }
  bool is_sep(int32_t v) const { return v >= sep_base; }
  static uint64_t key(int32_t a, int32_t b) { return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b; }

  uint32_t new_node(int32_t v) {
    uint32_t n;
    if (!free_nodes.empty()) {
      n = free_nodes.back();
      free_nodes.pop_back();
      val[n] = v;
    } else {
      n = (uint32_t)val.size();
      val.push_back(v);
      prv.push_back(NIL);
      nxt.push_back(NIL);
    }
    if (is_ref(v)) ++refs[(uint32_t)(-v)];
    return n;
  }
  void free_node(uint32_t n) {
    if (is_ref(val[n])) --refs[(uint32_t)(-val[n])];
    val[n] = DEAD;
    free_nodes.push_back(n);
  }
  void link(uint32_t a, uint32_t b) {
    nxt[a] = b;
    prv[b] = a;
  }
  uint32_t new_rule() {
    uint32_t r;
    if (!free_rules.empty()) {
      r = free_rules.back();
      free_rules.pop_back();
    } else {
      r = (uint32_t)guard.size();
      guard.push_back(NIL);
      refs.push_back(0);
    }
    const uint32_t g = new_node(GUARD_BASE - (int32_t)r);
    link(g, g);
    guard[r] = g;
    refs[r] = 0;
    return r;
  }

  // digram starting at n, if n and its successor are both ordinary symbols
  bool digram_at(uint32_t n, uint64_t& k) const {
    const int32_t a = val[n];
    if (a == DEAD || is_guard(a)) return false;
    const int32_t b = val[nxt[n]];
    if (is_guard(b)) return false;
    if (is_sep(a) || is_sep(b)) return false;
    k = key(a, b);
    return true;
  }
  // Forget the digram starting at n if the index points at this occurrence.
  // A run "x x x" indexes only one of its two overlapping occurrences; when
  // that one goes, its overlapping twin (if any) is re-queued for checking.
  void unindex(uint32_t n) {
    uint64_t k;
    if (!digram_at(n, k)) return;
    if (index.find(k) != n) return;
    index.erase_if(k, n);
    if (val[n] == val[nxt[n]]) {
      work.push_back(prv[n]);
      work.push_back(nxt[n]);
    }
  }

  // Replace the digram starting at s by a reference to rule r.
  void substitute(uint32_t s, uint32_t r) {
    const uint32_t q = prv[s], t = nxt[s], u = nxt[t];
    unindex(q);
    unindex(s);
    unindex(t);
    free_node(s);
    free_node(t);
    const uint32_t x = new_node(-(int32_t)r);
    link(q, x);
    link(x, u);
    work.push_back(x);  // digram (x, u), checked second
    work.push_back(q);  // digram (q, x), checked first
  }

  // Inline the body of the rule referenced at node x (its last use) and drop the rule.
  void expand(uint32_t x) {
    const uint32_t r = (uint32_t)(-val[x]);
    const uint32_t g = guard[r], f = nxt[g], l = prv[g];
    const uint32_t q = prv[x], u = nxt[x];
    unindex(q);
    unindex(x);
    link(q, f);
    link(l, u);
    free_node(x);
    val[g] = DEAD;
    free_nodes.push_back(g);
    guard[r] = NIL;
    refs[r] = 0;
    free_rules.push_back(r);
    work.push_back(l);  // junction (l, u)
    work.push_back(q);  // junction (q, f)
  }

  // The digram at n equals the one indexed at m (a different, non-overlapping occurrence).
  void match(uint32_t n, uint32_t m) {
    uint32_t r;
    const uint32_t gm = prv[m];
    if (is_guard(val[gm]) && is_guard(val[nxt[nxt[m]]])) {
      // m is the complete body of an existing rule: reuse it
      r = (uint32_t)(GUARD_BASE - val[gm]);
      substitute(n, r);
    } else {
      r = new_rule();
      const uint32_t g = guard[r];
      const uint32_t a = new_node(val[n]), b = new_node(val[nxt[n]]);
      link(g, a);
      link(a, b);
      link(b, g);
      substitute(m, r);
      substitute(n, r);
      index.put(key(val[a], val[b]), a);
    }
    // rule utility: a rule referenced from r's body that is now used only there is inlined
    const uint32_t g = guard[r];
    const uint32_t a = nxt[g], b = nxt[a];
    const int32_t va = val[a], vb = val[b];
    if (is_ref(va) && refs[(uint32_t)(-va)] == 1) expand(a);
    if (is_ref(vb) && vb != va && refs[(uint32_t)(-vb)] == 1) expand(b);
  }

  void check(uint32_t n) {
    uint64_t k;
    if (!digram_at(n, k)) return;
    const uint32_t m = index.find(k);
    if (m == NIL) {
      index.put(k, n);
      return;
    }
    if (m == n) return;
    if (nxt[m] == n || nxt[n] == m) return;  // overlapping occurrences inside a run
    match(n, m);
  }

  void drain() {
    while (!work.empty()) {
      const uint32_t n = work.back();
      work.pop_back();
      check(n);
    }
  }

  void append(int32_t v) {
    const uint32_t g = guard[0];
    const uint32_t last = prv[g];
    const uint32_t n = new_node(v);
    link(last, n);
    link(n, g);
    work.push_back(last);
    drain();
  }
};

struct Grammar {
  std::vector<int64_t> rule_off;
  std::vector<int32_t> sym;
  std::vector<int64_t> file_off;
};

}  // namespace

extern "C" {

// Compress files tok[file_off[f] .. file_off[f+1]) over words in [0, vocab).
// Returns a grammar handle, or null on invalid input.
void* synth_sequitur(const int32_t* tok, const int64_t* file_off, int64_t num_files, int32_t vocab) {
  if (!tok && num_files > 0 && file_off[num_files] > 0) return nullptr;
  if (num_files < 1 || vocab <= 0) return nullptr;
  try {
    const int64_t T = file_off[num_files];
    for (int64_t i = 0; i < T; ++i)
      if (tok[i] < 0 || tok[i] >= vocab) return nullptr;
    Sequitur sq(vocab, (size_t)(T + num_files));
    // large inputs report their progress on stderr (they take minutes)
    const int64_t every = T >= (int64_t(1) << 27) ? (int64_t(1) << 26) : INT64_MAX;
    int64_t next_report = every;
    for (int64_t f = 0; f < num_files; ++f) {
      if (f > 0) sq.append(vocab + (int32_t)(f - 1));  // unique splitter
      for (int64_t i = file_off[f]; i < file_off[f + 1]; ++i) {
        sq.append(tok[i]);
        if (i + 1 == next_report) {
          std::fprintf(stderr, "[synth] sequitur %lld / %lld tokens\n", (long long)(i + 1), (long long)T);
          std::fflush(stderr);
          next_report += every;
        }
      }
    }
    // renumber: root = 0, then first encounter in a left-to-right preorder walk
    const size_t nr = sq.guard.size();
    std::vector<int64_t> newid(nr, -1);
    std::vector<uint32_t> order;
    newid[0] = 0;
    order.push_back(0);
    {
      std::vector<uint32_t> stack;  // node cursors
      stack.push_back(sq.nxt[sq.guard[0]]);
      while (!stack.empty()) {
        uint32_t n = stack.back();
        const int32_t v = sq.val[n];
        if (Sequitur::is_guard(v)) {
          stack.pop_back();
          continue;
        }
        stack.back() = sq.nxt[n];
        if (Sequitur::is_ref(v)) {
          const uint32_t r = (uint32_t)(-v);
          if (newid[r] < 0) {
            newid[r] = (int64_t)order.size();
            order.push_back(r);
            stack.push_back(sq.nxt[sq.guard[r]]);
          }
        }
      }
    }
    auto* G = new Grammar;
    G->rule_off.reserve(order.size() + 1);
    G->rule_off.push_back(0);
    G->file_off.push_back(0);
    for (uint32_t r : order) {
      for (uint32_t n = sq.nxt[sq.guard[r]]; !Sequitur::is_guard(sq.val[n]); n = sq.nxt[n]) {
        const int32_t v = sq.val[n];
        if (v >= vocab) {  // splitter: closes a file span of the root
          G->file_off.push_back((int64_t)G->sym.size());
          continue;
        }
        G->sym.push_back(Sequitur::is_ref(v) ? -(int32_t)newid[(uint32_t)(-v)] : v);
      }
      G->rule_off.push_back((int64_t)G->sym.size());
      if (r == 0) G->file_off.push_back((int64_t)G->sym.size());
    }
    return G;
  } catch (const std::bad_alloc&) {
    return nullptr;
  }
}

int64_t synth_grammar_rules(const void* h) { return (int64_t)((const Grammar*)h)->rule_off.size() - 1; }
int64_t synth_grammar_syms(const void* h) { return (int64_t)((const Grammar*)h)->sym.size(); }
int64_t synth_grammar_files(const void* h) { return (int64_t)((const Grammar*)h)->file_off.size() - 1; }
void synth_grammar_copy(const void* h, int64_t* rule_off, int32_t* sym, int64_t* file_off) {
  const auto* G = (const Grammar*)h;
  std::memcpy(rule_off, G->rule_off.data(), G->rule_off.size() * sizeof(int64_t));
  std::memcpy(sym, G->sym.data(), G->sym.size() * sizeof(int32_t));
  std::memcpy(file_off, G->file_off.data(), G->file_off.size() * sizeof(int64_t));
}
void synth_grammar_free(void* h) { delete (Grammar*)h; }

}  // extern "C"
