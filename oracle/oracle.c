/* oracle.c -- plain, slow, obviously correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline of the benchmark call this code; the GPU library never does and
 * shares nothing with it.
 *
 * It computes the analytics of the paper in two independent ways:
 *   (A) brute force: expand the grammar back to text, then apply the plain
 *       definitions of the five analytics (word count, sort, term vector,
 *       inverted index, sequence count) to the text;
 *   (B) direct traversal of the rule DAG, in the order the paper describes
 *       (Background, "TADOC", the word-count walk-through; Section
 *       "Fine-Grained Thread-Level Execution Engine", top-down traversal;
 *       Section "Sequence Support", head and tail buffers).
 * It also checks a grammar's structure and the Sequitur properties.
 *
 * Everything is integer arithmetic on uint64 counts; nothing is approximate.
 *
 * Grammar encoding (CSR):
 *   rule_off[R+1]: body(r) = sym[rule_off[r] .. rule_off[r+1]); rule 0 is the root
 *   sym[S]:        s >= 0 is a word id (< V); s < 0 references rule -s
 *   file_off[F+1]: file f is the root body [file_off[f], file_off[f+1])
 *
 * Sequence keys pack an n-gram (w0 .. w(n-1)) so that ascending keys are
 * lexicographic n-gram order:
 *   n = 1: w0;  n = 2: w0 << 32 | w1;  n = 3: w0 << 42 | w1 << 21 | w2 (V <= 2^21);
 *   n = 4: w0 << 48 | w1 << 32 | w2 << 16 | w3 (V <= 2^16).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_RANGE (-1)   /* symbol or offset out of range */
#define OR_ERR_CYCLE (-2)   /* rule DAG has a cycle */
#define OR_ERR_NOMEM (-3)
#define OR_ERR_ARG (-4)

void or_free(void* p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Structure of a grammar                                                   */
/* ------------------------------------------------------------------------ */

/* Structural validity: offsets monotone and in range, every rule other than
 * the root has a non-empty body, word ids < V, rule references in [1, R),
 * file spans tile the root body. Returns OR_OK or OR_ERR_RANGE.
 * (Background, "TADOC": rules, words and splitters are all numbers; a rule
 * is a node of the DAG that stands for a non-empty run of symbols, and R0 is
 * its root.) */
int or_check_structure(const int64_t* rule_off, int64_t R, const int32_t* sym, int64_t S,
                       const int64_t* file_off, int64_t F, int32_t V) {
  if (R < 1 || F < 1 || V <= 0) return OR_ERR_ARG;
  if (rule_off[0] != 0 || rule_off[R] != S) return OR_ERR_RANGE;
  for (int64_t r = 0; r < R; ++r)
    if (rule_off[r + 1] < rule_off[r]) return OR_ERR_RANGE;
  for (int64_t r = 1; r < R; ++r)
    if (rule_off[r + 1] == rule_off[r]) return OR_ERR_RANGE; /* empty non-root body */
  for (int64_t i = 0; i < S; ++i) {
    int64_t s = sym[i];
    if (s >= 0 && s >= V) return OR_ERR_RANGE;
    if (s < 0 && (-s < 1 || -s >= R)) return OR_ERR_RANGE;
  }
  if (file_off[0] != 0 || file_off[F] != rule_off[1]) return OR_ERR_RANGE;
  for (int64_t f = 0; f < F; ++f)
    if (file_off[f + 1] < file_off[f]) return OR_ERR_RANGE;
  return OR_OK;
}

/* Depth-first postorder of the rules reachable from the root (children
 * before parents), iterative. Reversed, it is a topological order (parents
 * before children). Returns the number of rules written to `post`, or
 * OR_ERR_CYCLE. The rule DAG: Background, "TADOC" (the grammar organised as a
 * DAG for traversal). */
int64_t or_postorder(const int64_t* rule_off, int64_t R, const int32_t* sym, int32_t* post) {
  unsigned char* color = calloc((size_t)R, 1); /* 0 new, 1 on stack, 2 done */
  int64_t* cur = malloc(sizeof(int64_t) * (size_t)R);
  int32_t* stack = malloc(sizeof(int32_t) * (size_t)R);
  if (!color || !cur || !stack) {
    free(color), free(cur), free(stack);
    return OR_ERR_NOMEM;
  }
  int64_t top = 0, n = 0;
  stack[top++] = 0;
  color[0] = 1;
  cur[0] = rule_off[0];
  while (top > 0) {
    int32_t r = stack[top - 1];
    if (cur[r] == rule_off[r + 1]) {
      color[r] = 2;
      post[n++] = r;
      --top;
      continue;
    }
    int32_t s = sym[cur[r]++];
    if (s >= 0) continue;
    int32_t c = -s;
    if (color[c] == 1) {
      free(color), free(cur), free(stack);
      return OR_ERR_CYCLE;
    }
    if (color[c] == 0) {
      color[c] = 1;
      cur[c] = rule_off[c];
      stack[top++] = c;
    }
  }
  free(color), free(cur), free(stack);
  return n;
}

/* Number of words in the expansion of every rule (0 for unreachable ones
 * is never needed: every rule gets its length). len(r) = (words in body)
 * + sum over child references of len(child), computed children first. */
int or_rule_len(const int64_t* rule_off, int64_t R, const int32_t* sym, uint64_t* len) {
  /* every rule, reachable or not: repeat postorder from each unvisited rule */
  unsigned char* done = calloc((size_t)R, 1);
  int64_t* cur = malloc(sizeof(int64_t) * (size_t)R);
  int32_t* stack = malloc(sizeof(int32_t) * (size_t)R);
  unsigned char* onstack = calloc((size_t)R, 1);
  if (!done || !cur || !stack || !onstack) {
    free(done), free(cur), free(stack), free(onstack);
    return OR_ERR_NOMEM;
  }
  int rc = OR_OK;
  for (int64_t start = R - 1; start >= 0 && rc == OR_OK; --start) {
    if (done[start]) continue;
    int64_t top = 0;
    stack[top++] = (int32_t)start;
    cur[start] = rule_off[start];
    onstack[start] = 1;
    while (top > 0) {
      int32_t r = stack[top - 1];
      if (cur[r] == rule_off[r + 1]) {
        uint64_t L = 0;
        for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i) L += sym[i] >= 0 ? 1u : len[-sym[i]];
        len[r] = L;
        done[r] = 1;
        onstack[r] = 0;
        --top;
        continue;
      }
      int32_t s = sym[cur[r]++];
      if (s >= 0) continue;
      int32_t c = -s;
      if (onstack[c]) {
        rc = OR_ERR_CYCLE;
        break;
      }
      if (!done[c]) {
        onstack[c] = 1;
        cur[c] = rule_off[c];
        stack[top++] = c;
      }
    }
  }
  free(done), free(cur), free(stack), free(onstack);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* (A) Brute force: decompress, then apply the plain definitions             */
/* ------------------------------------------------------------------------ */

/* Expand every file span of the root back into words. out_tok must hold the
 * total length (sum of len over the root body); out_file_off gets F+1
 * offsets. Returns the number of words written. */
int64_t or_expand(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                  int64_t F, int32_t* out_tok, int64_t* out_file_off) {
  (void)R;
  /* explicit stack of body cursors: (position, end) */
  int64_t cap = 64, top = 0, n = 0;
  int64_t* pos = malloc(sizeof(int64_t) * (size_t)cap);
  int64_t* end = malloc(sizeof(int64_t) * (size_t)cap);
  if (!pos || !end) {
    free(pos), free(end);
    return OR_ERR_NOMEM;
  }
  out_file_off[0] = 0;
  for (int64_t f = 0; f < F; ++f) {
    top = 0;
    pos[top] = file_off[f];
    end[top] = file_off[f + 1];
    ++top;
    while (top > 0) {
      if (pos[top - 1] == end[top - 1]) {
        --top;
        continue;
      }
      int32_t s = sym[pos[top - 1]++];
      if (s >= 0) {
        out_tok[n++] = s;
        continue;
      }
      if (top == cap) {
        cap *= 2;
        int64_t* p2 = realloc(pos, sizeof(int64_t) * (size_t)cap);
        if (p2) pos = p2;
        int64_t* e2 = realloc(end, sizeof(int64_t) * (size_t)cap);
        if (e2) end = e2;
        if (!p2 || !e2) {
          free(pos), free(end);
          return OR_ERR_NOMEM;
        }
      }
      pos[top] = rule_off[-s];
      end[top] = rule_off[-s + 1];
      ++top;
    }
    out_file_off[f + 1] = n;
  }
  free(pos), free(end);
  return n;
}

/* Word count: wc[w] = number of occurrences of w in all files. */
void or_wc_text(const int32_t* tok, int64_t T, int32_t V, uint64_t* wc) {
  memset(wc, 0, sizeof(uint64_t) * (size_t)V);
  for (int64_t i = 0; i < T; ++i) wc[tok[i]] += 1;
}

/* Sort: words with a nonzero count, by count descending, then id ascending. */
static const uint64_t* g_sort_wc;
static int cmp_sort(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  if (g_sort_wc[x] != g_sort_wc[y]) return g_sort_wc[x] > g_sort_wc[y] ? -1 : 1;
  return x < y ? -1 : (x > y);
}
int64_t or_sort(const uint64_t* wc, int32_t V, uint32_t* id, uint64_t* cnt) {
  int64_t k = 0;
  for (int32_t w = 0; w < V; ++w)
    if (wc[w]) id[k++] = (uint32_t)w;
  g_sort_wc = wc;
  qsort(id, (size_t)k, sizeof(uint32_t), cmp_sort);
  for (int64_t i = 0; i < k; ++i) cnt[i] = wc[id[i]];
  return k;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : (x > y);
}

/* Term vector: for each file f, the (word, count) pairs with count > 0 in
 * ascending word order. Outputs are malloc'ed: *off has F+1 entries, *word and
 * *cnt have *off[F] entries. */
int or_tv_text(const int32_t* tok, const int64_t* file_off, int64_t F, int32_t V, int64_t** off_out,
               uint32_t** word_out, uint64_t** cnt_out) {
  int64_t T = file_off[F];
  uint64_t* c = calloc((size_t)V, sizeof(uint64_t));
  uint32_t* seen = malloc(sizeof(uint32_t) * (size_t)(T > 0 ? T : 1));
  int64_t* off = malloc(sizeof(int64_t) * (size_t)(F + 1));
  uint32_t* word = malloc(sizeof(uint32_t) * (size_t)(T > 0 ? T : 1));
  uint64_t* cnt = malloc(sizeof(uint64_t) * (size_t)(T > 0 ? T : 1));
  if (!c || !seen || !off || !word || !cnt) {
    free(c), free(seen), free(off), free(word), free(cnt);
    return OR_ERR_NOMEM;
  }
  int64_t nnz = 0;
  off[0] = 0;
  for (int64_t f = 0; f < F; ++f) {
    int64_t k = 0;
    for (int64_t i = file_off[f]; i < file_off[f + 1]; ++i) {
      if (c[tok[i]] == 0) seen[k++] = (uint32_t)tok[i];
      c[tok[i]] += 1;
    }
    qsort(seen, (size_t)k, sizeof(uint32_t), cmp_u32);
    for (int64_t j = 0; j < k; ++j) {
      word[nnz] = seen[j];
      cnt[nnz] = c[seen[j]];
      c[seen[j]] = 0;
      ++nnz;
    }
    off[f + 1] = nnz;
  }
  free(c), free(seen);
  *off_out = off, *word_out = word, *cnt_out = cnt;
  return OR_OK;
}

/* Inverted index: for each word, the ascending list of files whose term
 * vector holds it. Built by counting, then placing files in file order. */
int or_inverted_index(const int64_t* tv_off, const uint32_t* tv_word, int64_t F, int32_t V,
                      int64_t** off_out, uint32_t** file_out) {
  int64_t nnz = tv_off[F];
  int64_t* off = calloc((size_t)V + 1, sizeof(int64_t));
  uint32_t* file = malloc(sizeof(uint32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t* fill = malloc(sizeof(int64_t) * (size_t)V + 1);
  if (!off || !file || !fill) {
    free(off), free(file), free(fill);
    return OR_ERR_NOMEM;
  }
  for (int64_t i = 0; i < nnz; ++i) off[tv_word[i] + 1] += 1;
  for (int32_t w = 0; w < V; ++w) off[w + 1] += off[w];
  for (int32_t w = 0; w < V; ++w) fill[w] = off[w];
  for (int64_t f = 0; f < F; ++f)
    for (int64_t i = tv_off[f]; i < tv_off[f + 1]; ++i) file[fill[tv_word[i]]++] = (uint32_t)f;
  free(fill);
  *off_out = off, *file_out = file;
  return OR_OK;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y);
}

static uint64_t pack_key(const int32_t* g, int n) {
  if (n == 1) return (uint64_t)(uint32_t)g[0];
  if (n == 2) return (uint64_t)(uint32_t)g[0] << 32 | (uint32_t)g[1];
  if (n == 3) return (uint64_t)(uint32_t)g[0] << 42 | (uint64_t)(uint32_t)g[1] << 21 | (uint32_t)g[2];
  return (uint64_t)(uint32_t)g[0] << 48 | (uint64_t)(uint32_t)g[1] << 32 | (uint64_t)(uint32_t)g[2] << 16 |
         (uint32_t)g[3];
}

/* Collapse a list of keys (ascending after sorting) into (key, count) runs.
 * keys is sorted in place; outputs are malloc'ed. */
static int64_t runs_of(uint64_t* keys, int64_t m, uint64_t** key_out, uint64_t** cnt_out) {
  qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);
  uint64_t* k = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  uint64_t* c = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  if (!k || !c) {
    free(k), free(c);
    return OR_ERR_NOMEM;
  }
  int64_t u = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (u > 0 && k[u - 1] == keys[i]) {
      c[u - 1] += 1;
    } else {
      k[u] = keys[i];
      c[u] = 1;
      ++u;
    }
  }
  *key_out = k, *cnt_out = c;
  return u;
}

/* Sequence count: occurrences of every length-n window of words inside each
 * file (windows never cross files), as ascending (key, count) pairs.
 * Returns the number of distinct keys. Collect every window's key, sort,
 * count runs: no hashing. */
int64_t or_sc_text(const int32_t* tok, const int64_t* file_off, int64_t F, int n, int32_t V,
                   uint64_t** key_out, uint64_t** cnt_out) {
  if (n < 1 || n > 4 || (n == 3 && V > (1 << 21)) || (n == 4 && V > (1 << 16))) return OR_ERR_ARG;
  int64_t m = 0, T = file_off[F];
  uint64_t* keys = malloc(sizeof(uint64_t) * (size_t)(T > 0 ? T : 1));
  if (!keys) return OR_ERR_NOMEM;
  for (int64_t f = 0; f < F; ++f)
    for (int64_t i = file_off[f]; i + n <= file_off[f + 1]; ++i) keys[m++] = pack_key(tok + i, n);
  int64_t u = runs_of(keys, m, key_out, cnt_out);
  free(keys);
  return u;
}

/* ------------------------------------------------------------------------ */
/* (B) Direct traversal of the rule DAG                                      */
/* ------------------------------------------------------------------------ */

/* Rule weights (top-down traversal, Algorithm "Top-Down Traversal"): the
 * weight of a rule is the number of times it occurs in the full derivation of
 * the root. The root has weight 1; in topological order (parents first),
 * every occurrence of child c in the body of r adds weight(r) to weight(c).
 * Rules not reachable from the root keep weight 0. */
int or_weights(const int64_t* rule_off, int64_t R, const int32_t* sym, uint64_t* w) {
  int32_t* post = malloc(sizeof(int32_t) * (size_t)R);
  if (!post) return OR_ERR_NOMEM;
  int64_t n = or_postorder(rule_off, R, sym, post);
  if (n < 0) {
    free(post);
    return (int)n;
  }
  memset(w, 0, sizeof(uint64_t) * (size_t)R);
  w[0] = 1;
  for (int64_t k = n - 1; k >= 0; --k) {
    int32_t r = post[k];
    for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i)
      if (sym[i] < 0) w[-sym[i]] += w[r];
  }
  free(post);
  return OR_OK;
}

/* Word count by traversal (the word-count walk-through of Background,
 * "TADOC", and the reduction step of the top-down traversal):
 * wc[word] = sum over rules r of weight(r) * (occurrences of word in body(r)). */
int or_wc_traverse(const int64_t* rule_off, int64_t R, const int32_t* sym, int32_t V, uint64_t* wc) {
  uint64_t* w = malloc(sizeof(uint64_t) * (size_t)R);
  if (!w) return OR_ERR_NOMEM;
  int rc = or_weights(rule_off, R, sym, w);
  if (rc == OR_OK) {
    memset(wc, 0, sizeof(uint64_t) * (size_t)V);
    for (int64_t r = 0; r < R; ++r)
      for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i)
        if (sym[i] >= 0) wc[sym[i]] += w[r];
  }
  free(w);
  return rc;
}

/* The same word count with the accumulation spread over host threads, for
 * the CPU baseline on all cores (TADOC's coarse-grained CPU parallelism):
 * weights as in or_weights (one sequential topological pass), then the
 * rules are cut into `nthreads` ranges of about equal symbol count, each
 * thread sums weight(r) * (words in body(r)) into a private count array, and
 * the private arrays are added together. Same result as or_wc_traverse. */
int or_wc_traverse_par(const int64_t* rule_off, int64_t R, const int32_t* sym, int32_t V, uint64_t* wc,
                       int nthreads) {
  if (nthreads < 1) return OR_ERR_ARG;
  uint64_t* w = malloc(sizeof(uint64_t) * (size_t)R);
  uint64_t* priv = calloc((size_t)nthreads * (size_t)V, sizeof(uint64_t));
  int64_t* cut = malloc(sizeof(int64_t) * (size_t)(nthreads + 1));
  if (!w || !priv || !cut) {
    free(w), free(priv), free(cut);
    return OR_ERR_NOMEM;
  }
  int rc = or_weights(rule_off, R, sym, w);
  if (rc == OR_OK) {
    /* rule ranges [cut[t], cut[t+1]) of about S / nthreads symbols each */
    int64_t S = rule_off[R], r = 0;
    cut[0] = 0;
    for (int t = 1; t < nthreads; ++t) {
      int64_t target = S / nthreads * t;
      while (r < R && rule_off[r] < target) ++r;
      cut[t] = r;
    }
    cut[nthreads] = R;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
      uint64_t* mine = priv + (size_t)t * (size_t)V;
      for (int64_t q = cut[t]; q < cut[t + 1]; ++q)
        for (int64_t i = rule_off[q]; i < rule_off[q + 1]; ++i)
          if (sym[i] >= 0) mine[sym[i]] += w[q];
    }
    memset(wc, 0, sizeof(uint64_t) * (size_t)V);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t x = 0; x < V; ++x) {
      uint64_t sum = 0;
      for (int t = 0; t < nthreads; ++t) sum += priv[(size_t)t * (size_t)V + (size_t)x];
      wc[x] = sum;
    }
  }
  free(w), free(priv), free(cut);
  return rc;
}

/* Term vector by traversal: for each file, a top-down pass over the part of
 * the DAG reachable from the file's span of the root, with per-file weights
 * (the file's span counts once; each occurrence of c in body(r) adds
 * weight_f(r) to weight_f(c)), then word counts summed with those weights.
 * This is top-down on purpose: the GPU library builds term vectors bottom-up,
 * so the two methods are independent. Outputs as in or_tv_text. */
int or_tv_traverse(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                   int64_t F, int32_t V, int64_t** off_out, uint32_t** word_out, uint64_t** cnt_out) {
  int64_t* off = malloc(sizeof(int64_t) * (size_t)(F + 1));
  int32_t* stamp = malloc(sizeof(int32_t) * (size_t)R);
  int32_t* post = malloc(sizeof(int32_t) * (size_t)R);
  int32_t* stack = malloc(sizeof(int32_t) * (size_t)R);
  int64_t* cur = malloc(sizeof(int64_t) * (size_t)R);
  uint64_t* wf = calloc((size_t)R, sizeof(uint64_t));
  uint64_t* c = calloc((size_t)V, sizeof(uint64_t));
  uint32_t* seen = malloc(sizeof(uint32_t) * (size_t)V);
  int64_t cap = 1024, nnz = 0;
  uint32_t* word = malloc(sizeof(uint32_t) * (size_t)cap);
  uint64_t* cnt = malloc(sizeof(uint64_t) * (size_t)cap);
  int rc = OR_OK;
  if (!off || !stamp || !post || !stack || !cur || !wf || !c || !seen || !word || !cnt) {
    rc = OR_ERR_NOMEM;
    goto done;
  }
  for (int64_t r = 0; r < R; ++r) stamp[r] = -1;
  off[0] = 0;
  for (int64_t f = 0; f < F; ++f) {
    /* postorder of the sub-DAG reachable from span f */
    int64_t np = 0;
    for (int64_t i = file_off[f]; i < file_off[f + 1]; ++i) {
      if (sym[i] >= 0 || stamp[-sym[i]] == (int32_t)f) continue;
      int64_t top = 0;
      int32_t s0 = -sym[i];
      stamp[s0] = (int32_t)f;
      cur[s0] = rule_off[s0];
      stack[top++] = s0;
      while (top > 0) {
        int32_t r = stack[top - 1];
        if (cur[r] == rule_off[r + 1]) {
          post[np++] = r;
          --top;
          continue;
        }
        int32_t s = sym[cur[r]++];
        if (s < 0 && stamp[-s] != (int32_t)f) {
          stamp[-s] = (int32_t)f;
          cur[-s] = rule_off[-s];
          stack[top++] = -s;
        }
      }
    }
    /* per-file weights: span references count once each */
    for (int64_t i = file_off[f]; i < file_off[f + 1]; ++i)
      if (sym[i] < 0) wf[-sym[i]] += 1;
    for (int64_t k = np - 1; k >= 0; --k) {
      int32_t r = post[k];
      for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i)
        if (sym[i] < 0) wf[-sym[i]] += wf[r];
    }
    /* words: the span's own words, then every reached rule's words times its weight */
    int64_t k = 0;
    for (int64_t i = file_off[f]; i < file_off[f + 1]; ++i)
      if (sym[i] >= 0) {
        if (c[sym[i]] == 0) seen[k++] = (uint32_t)sym[i];
        c[sym[i]] += 1;
      }
    for (int64_t j = 0; j < np; ++j) {
      int32_t r = post[j];
      for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i)
        if (sym[i] >= 0) {
          if (c[sym[i]] == 0) seen[k++] = (uint32_t)sym[i];
          c[sym[i]] += wf[r];
        }
      wf[r] = 0;
    }
    qsort(seen, (size_t)k, sizeof(uint32_t), cmp_u32);
    if (nnz + k > cap) {
      while (nnz + k > cap) cap *= 2;
      uint32_t* w2 = realloc(word, sizeof(uint32_t) * (size_t)cap);
      if (w2) word = w2;
      uint64_t* c2 = realloc(cnt, sizeof(uint64_t) * (size_t)cap);
      if (c2) cnt = c2;
      if (!w2 || !c2) {
        rc = OR_ERR_NOMEM;
        goto done;
      }
    }
    for (int64_t j = 0; j < k; ++j) {
      word[nnz] = seen[j];
      cnt[nnz] = c[seen[j]];
      c[seen[j]] = 0;
      ++nnz;
    }
    off[f + 1] = nnz;
  }
done:
  free(stamp), free(post), free(stack), free(cur), free(wf), free(c), free(seen);
  if (rc != OR_OK) {
    free(off), free(word), free(cnt);
    return rc;
  }
  *off_out = off, *word_out = word, *cnt_out = cnt;
  return OR_OK;
}

/* Head and tail buffers (Section "Data Structures", head and tail; Section
 * "Sequence Support", initialization phase): head(r) holds the first
 * min(n-1, len(r)) words of the expansion of r and tail(r) the last ones.
 * They are filled children first: walking body(r) from the left, words are
 * taken as they are and a child contributes its own head, until n-1 words are
 * collected; the tail is the mirror image from the right. head and tail are
 * R x (n-1) arrays (row r valid for its first min(n-1, len(r)) entries). */
int or_head_tail(const int64_t* rule_off, int64_t R, const int32_t* sym, const uint64_t* len, int n,
                 int32_t* head, int32_t* tail) {
  int32_t* post = malloc(sizeof(int32_t) * (size_t)R);
  if (!post) return OR_ERR_NOMEM;
  const int m = n - 1;
  /* all rules, children first: postorder from every rule id */
  unsigned char* done = calloc((size_t)R, 1);
  int64_t* cur = malloc(sizeof(int64_t) * (size_t)R);
  int32_t* stack = malloc(sizeof(int32_t) * (size_t)R);
  if (!done || !cur || !stack) {
    free(post), free(done), free(cur), free(stack);
    return OR_ERR_NOMEM;
  }
  int64_t np = 0;
  for (int64_t s0 = 0; s0 < R; ++s0) {
    if (done[s0]) continue;
    int64_t top = 0;
    stack[top++] = (int32_t)s0;
    cur[s0] = rule_off[s0];
    done[s0] = 1;
    while (top > 0) {
      int32_t r = stack[top - 1];
      if (cur[r] == rule_off[r + 1]) {
        post[np++] = r;
        --top;
        continue;
      }
      int32_t s = sym[cur[r]++];
      if (s < 0 && !done[-s]) {
        done[-s] = 1;
        cur[-s] = rule_off[-s];
        stack[top++] = -s;
      }
    }
  }
  for (int64_t k = 0; k < np; ++k) {
    int32_t r = post[k];
    int32_t* h = head + (size_t)r * (size_t)m;
    int32_t* t = tail + (size_t)r * (size_t)m;
    int want = len[r] < (uint64_t)m ? (int)len[r] : m;
    int got = 0;
    for (int64_t i = rule_off[r]; i < rule_off[r + 1] && got < want; ++i) {
      int32_t s = sym[i];
      if (s >= 0) {
        h[got++] = s;
      } else {
        int take = len[-s] < (uint64_t)m ? (int)len[-s] : m;
        for (int j = 0; j < take && got < want; ++j) h[got++] = head[(size_t)(-s) * m + j];
      }
    }
    /* tail: collect from the right, filling t[want-1], t[want-2], ... */
    got = 0;
    for (int64_t i = rule_off[r + 1] - 1; i >= rule_off[r] && got < want; --i) {
      int32_t s = sym[i];
      if (s >= 0) {
        t[want - 1 - got++] = s;
      } else {
        int take = len[-s] < (uint64_t)m ? (int)len[-s] : m;
        const int32_t* ct = tail + (size_t)(-s) * m;
        for (int j = take - 1; j >= 0 && got < want; --j) t[want - 1 - got++] = ct[j];
      }
    }
  }
  free(post), free(done), free(cur), free(stack);
  return OR_OK;
}

/* Windows owned by one body segment body[lo, hi): every length-n window of
 * the segment's expansion that is not contained in the expansion of a single
 * child occurrence. The parent handles the sequences that cross rule
 * boundaries by looking only at the children's head and tail buffers (Section
 * "Data Structures", head and tail). The segment is reduced to words, where a
 * child contributes its whole expansion if it has at most 2(n-1) words (then
 * head and tail together are that expansion) and otherwise head, a gap and
 * tail. Each window of the reduced sequence that holds no gap and does not
 * lie inside one child's piece is emitted via emit(key, weight). Returns the
 * number of windows, or < 0 on error. */
typedef struct {
  uint64_t* key;
  uint64_t* key2; /* low half of a wide key (wide_b > 0), else unused */
  uint64_t* wt;
  int64_t m, cap;
  int wide_b;     /* 0: keys packed by pack_key; b > 0: wide keys, b bits per word */
} or_pairs;

static int push_pair2(or_pairs* p, uint64_t k, uint64_t k2, uint64_t w) {
  if (p->m == p->cap) {
    int64_t cap = p->cap ? p->cap * 2 : 1024;
    uint64_t* a = realloc(p->key, sizeof(uint64_t) * (size_t)cap);
    if (a) p->key = a;
    uint64_t* b = realloc(p->key2, sizeof(uint64_t) * (size_t)cap);
    if (b) p->key2 = b;
    uint64_t* c = realloc(p->wt, sizeof(uint64_t) * (size_t)cap);
    if (c) p->wt = c;
    if (!a || !b || !c) return OR_ERR_NOMEM;
    p->cap = cap;
  }
  p->key[p->m] = k;
  p->key2[p->m] = k2;
  p->wt[p->m] = w;
  ++p->m;
  return OR_OK;
}

static int push_pair(or_pairs* p, uint64_t k, uint64_t w) { return push_pair2(p, k, 0, w); }

/* Wide keys, for n-grams whose packed form does not fit 64 bits: the words
 * are packed big-endian with b bits each (b = bits of vocab - 1) into a
 * number of at most 126 bits, split into two 63-bit halves hi and lo, so
 * ascending (hi, lo) is lexicographic n-gram order. */
static void pack_wide(const int32_t* g, int n, int b, uint64_t* hi, uint64_t* lo) {
  const uint64_t m63 = (1ull << 63) - 1;
  uint64_t h = 0, l = 0;
  for (int i = 0; i < n; ++i) {
    h = ((h << b) | (l >> (63 - b))) & m63;
    l = ((l << b) | (uint32_t)g[i]) & m63;
  }
  *hi = h, *lo = l;
}

static int bits_of(int32_t V) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) < (int64_t)V) ++b;
  return b > 0 ? b : 1;
}

static int64_t owned_windows(const int64_t* rule_off, const int32_t* sym, const uint64_t* len,
                             const int32_t* head, const int32_t* tail, int n, int64_t lo, int64_t hi,
                             uint64_t weight, or_pairs* out) {
  (void)rule_off;
  const int m = n - 1;
  /* reduced sequence: word, or -1 for a gap; piece id per position (-1 for
   * the segment's own words, else the index of the child occurrence) */
  int64_t cap = 0;
  for (int64_t i = lo; i < hi; ++i) cap += sym[i] >= 0 ? 1 : (len[-sym[i]] <= (uint64_t)(2 * m) ? (int64_t)len[-sym[i]] : 2 * m + 1);
  int32_t* seq = malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  int64_t* piece = malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
  if (!seq || !piece) {
    free(seq), free(piece);
    return OR_ERR_NOMEM;
  }
  int64_t k = 0;
  for (int64_t i = lo; i < hi; ++i) {
    int32_t s = sym[i];
    if (s >= 0) {
      seq[k] = s, piece[k] = -1, ++k;
      continue;
    }
    int32_t c = -s;
    if (len[c] <= (uint64_t)(2 * m)) {
      /* whole expansion = head followed by the part of tail not in head */
      int L = (int)len[c];
      int hn = L < m ? L : m;
      for (int j = 0; j < hn; ++j) seq[k] = head[(size_t)c * m + j], piece[k] = i, ++k;
      int tn = L < m ? L : m;
      for (int j = tn - (L - hn); j < tn; ++j) seq[k] = tail[(size_t)c * m + j], piece[k] = i, ++k;
    } else {
      for (int j = 0; j < m; ++j) seq[k] = head[(size_t)c * m + j], piece[k] = i, ++k;
      seq[k] = -1, piece[k] = i, ++k;
      for (int j = 0; j < m; ++j) seq[k] = tail[(size_t)c * m + j], piece[k] = i, ++k;
    }
  }
  int64_t count = 0;
  for (int64_t a = 0; a + n <= k; ++a) {
    int gap = 0, inside = 1;
    for (int j = 0; j < n; ++j) {
      if (seq[a + j] < 0) gap = 1;
      if (piece[a + j] < 0 || piece[a + j] != piece[a]) inside = 0;
    }
    if (gap || inside) continue;
    int prc = OR_OK;
    if (out && out->wide_b > 0) {
      uint64_t hi, lo;
      pack_wide(seq + a, n, out->wide_b, &hi, &lo);
      prc = push_pair2(out, hi, lo, weight);
    } else if (out) {
      prc = push_pair(out, pack_key(seq + a, n), weight);
    }
    if (prc != OR_OK) {
      free(seq), free(piece);
      return OR_ERR_NOMEM;
    }
    ++count;
  }
  free(seq), free(piece);
  return count;
}

/* Owned-window count of every rule (root: sum over its file spans), for
 * comparison with the per-rule bound of the paper's equation for the memory
 * of sequence support. own must hold R entries. */
int or_owned_counts(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                    int64_t F, int n, uint64_t* own) {
  if (n < 1 || n > 4) return OR_ERR_ARG;
  size_t hs = (size_t)R * (size_t)(n > 1 ? n - 1 : 1);
  uint64_t* len = malloc(sizeof(uint64_t) * (size_t)R);
  int32_t* head = malloc(sizeof(int32_t) * hs);
  int32_t* tail = malloc(sizeof(int32_t) * hs);
  int rc = (!len || !head || !tail) ? OR_ERR_NOMEM : or_rule_len(rule_off, R, sym, len);
  if (rc == OR_OK) rc = or_head_tail(rule_off, R, sym, len, n, head, tail);
  for (int64_t r = 0; r < R && rc == OR_OK; ++r) {
    own[r] = 0;
    if (r == 0) {
      for (int64_t f = 0; f < F && rc == OR_OK; ++f) {
        int64_t c = owned_windows(rule_off, sym, len, head, tail, n, file_off[f], file_off[f + 1], 1, NULL);
        if (c < 0) rc = (int)c;
        else own[0] += (uint64_t)c;
      }
    } else {
      int64_t c = owned_windows(rule_off, sym, len, head, tail, n, rule_off[r], rule_off[r + 1], 1, NULL);
      if (c < 0) rc = (int)c;
      else own[r] = (uint64_t)c;
    }
  }
  free(len), free(head), free(tail);
  return rc;
}

static const uint64_t* g_pair_keys;
static int cmp_pair(const void* a, const void* b) {
  uint64_t x = g_pair_keys[*(const int64_t*)a], y = g_pair_keys[*(const int64_t*)b];
  return x < y ? -1 : (x > y);
}

/* Sequence count by traversal (Section "Sequence Support"): head and tail
 * buffers first (initialization phase), then every rule contributes its owned
 * windows, each counted weight(r) times (graph traversal phase); the root
 * contributes the owned windows of each file span once. The (key, weight)
 * pairs are merged by sorting, into ascending (key, count) pairs. */
int64_t or_sc_traverse(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                       int64_t F, int n, int32_t V, uint64_t** key_out, uint64_t** cnt_out) {
  if (n < 1 || n > 4 || (n == 3 && V > (1 << 21)) || (n == 4 && V > (1 << 16))) return OR_ERR_ARG;
  size_t hs = (size_t)R * (size_t)(n > 1 ? n - 1 : 1);
  uint64_t* len = malloc(sizeof(uint64_t) * (size_t)R);
  uint64_t* w = malloc(sizeof(uint64_t) * (size_t)R);
  int32_t* head = malloc(sizeof(int32_t) * hs);
  int32_t* tail = malloc(sizeof(int32_t) * hs);
  or_pairs P = {0, 0, 0, 0, 0, 0};
  int64_t rc = (!len || !w || !head || !tail) ? OR_ERR_NOMEM : or_rule_len(rule_off, R, sym, len);
  if (rc == OR_OK) rc = or_head_tail(rule_off, R, sym, len, n, head, tail);
  if (rc == OR_OK) rc = or_weights(rule_off, R, sym, w);
  for (int64_t f = 0; f < F && rc >= 0; ++f) {
    int64_t c = owned_windows(rule_off, sym, len, head, tail, n, file_off[f], file_off[f + 1], 1, &P);
    if (c < 0) rc = c;
  }
  for (int64_t r = 1; r < R && rc >= 0; ++r) {
    if (w[r] == 0) continue;
    int64_t c = owned_windows(rule_off, sym, len, head, tail, n, rule_off[r], rule_off[r + 1], w[r], &P);
    if (c < 0) rc = c;
  }
  int64_t u = 0;
  if (rc >= 0) {
    int64_t* idx = malloc(sizeof(int64_t) * (size_t)(P.m > 0 ? P.m : 1));
    uint64_t* k = malloc(sizeof(uint64_t) * (size_t)(P.m > 0 ? P.m : 1));
    uint64_t* c = malloc(sizeof(uint64_t) * (size_t)(P.m > 0 ? P.m : 1));
    if (!idx || !k || !c) {
      free(idx), free(k), free(c);
      rc = OR_ERR_NOMEM;
    } else {
      for (int64_t i = 0; i < P.m; ++i) idx[i] = i;
      g_pair_keys = P.key;
      qsort(idx, (size_t)P.m, sizeof(int64_t), cmp_pair);
      for (int64_t i = 0; i < P.m; ++i) {
        uint64_t key = P.key[idx[i]], wt = P.wt[idx[i]];
        if (u > 0 && k[u - 1] == key) c[u - 1] += wt;
        else k[u] = key, c[u] = wt, ++u;
      }
      free(idx);
      *key_out = k, *cnt_out = c;
    }
  }
  free(len), free(w), free(head), free(tail), free(P.key), free(P.key2), free(P.wt);
  return rc < 0 ? rc : u;
}

/* ---- wide keys (any n up to 8, n * bits(vocab - 1) <= 126) ---- */

static const uint64_t* g_wk_hi;
static const uint64_t* g_wk_lo;
static int cmp_wide(const void* a, const void* b) {
  int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
  if (g_wk_hi[i] != g_wk_hi[j]) return g_wk_hi[i] < g_wk_hi[j] ? -1 : 1;
  if (g_wk_lo[i] != g_wk_lo[j]) return g_wk_lo[i] < g_wk_lo[j] ? -1 : 1;
  return 0;
}

/* Merge weighted wide keys into ascending (hi, lo, count) by sorting. */
static int64_t wide_runs(const or_pairs* P, uint64_t** hi_out, uint64_t** lo_out, uint64_t** cnt_out) {
  int64_t m = P->m;
  int64_t* idx = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  uint64_t* h = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  uint64_t* l = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  uint64_t* c = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  if (!idx || !h || !l || !c) {
    free(idx), free(h), free(l), free(c);
    return OR_ERR_NOMEM;
  }
  for (int64_t i = 0; i < m; ++i) idx[i] = i;
  g_wk_hi = P->key, g_wk_lo = P->key2;
  qsort(idx, (size_t)m, sizeof(int64_t), cmp_wide);
  int64_t u = 0;
  for (int64_t i = 0; i < m; ++i) {
    uint64_t a = P->key[idx[i]], b = P->key2[idx[i]], w = P->wt[idx[i]];
    if (u > 0 && h[u - 1] == a && l[u - 1] == b) c[u - 1] += w;
    else h[u] = a, l[u] = b, c[u] = w, ++u;
  }
  free(idx);
  *hi_out = h, *lo_out = l, *cnt_out = c;
  return u;
}

static int wide_args(int n, int32_t V) { return n >= 1 && n <= 8 && V >= 1 && n * bits_of(V) <= 126; }

/* Sequence count with wide keys from the text: every window of every file. */
int64_t or_sc_text_wide(const int32_t* tok, const int64_t* file_off, int64_t F, int n, int32_t V,
                        uint64_t** hi_out, uint64_t** lo_out, uint64_t** cnt_out) {
  if (!wide_args(n, V)) return OR_ERR_ARG;
  or_pairs P = {0, 0, 0, 0, 0, bits_of(V)};
  int64_t rc = OR_OK;
  for (int64_t f = 0; f < F && rc == OR_OK; ++f)
    for (int64_t i = file_off[f]; i + n <= file_off[f + 1] && rc == OR_OK; ++i) {
      uint64_t hi, lo;
      pack_wide(tok + i, n, P.wide_b, &hi, &lo);
      rc = push_pair2(&P, hi, lo, 1);
    }
  int64_t u = rc == OR_OK ? wide_runs(&P, hi_out, lo_out, cnt_out) : rc;
  free(P.key), free(P.key2), free(P.wt);
  return u;
}

/* Sequence count with wide keys by traversal: head and tail buffers of n-1
 * words, then every rule's owned windows weighted by the rule's weight (the
 * root's per file span), as or_sc_traverse. */
int64_t or_sc_traverse_wide(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                            int64_t F, int n, int32_t V, uint64_t** hi_out, uint64_t** lo_out, uint64_t** cnt_out) {
  if (!wide_args(n, V)) return OR_ERR_ARG;
  size_t hs = (size_t)R * (size_t)(n > 1 ? n - 1 : 1);
  uint64_t* len = malloc(sizeof(uint64_t) * (size_t)R);
  uint64_t* w = malloc(sizeof(uint64_t) * (size_t)R);
  int32_t* head = malloc(sizeof(int32_t) * hs);
  int32_t* tail = malloc(sizeof(int32_t) * hs);
  or_pairs P = {0, 0, 0, 0, 0, bits_of(V)};
  int64_t rc = (!len || !w || !head || !tail) ? OR_ERR_NOMEM : or_rule_len(rule_off, R, sym, len);
  if (rc == OR_OK) rc = or_head_tail(rule_off, R, sym, len, n, head, tail);
  if (rc == OR_OK) rc = or_weights(rule_off, R, sym, w);
  for (int64_t f = 0; f < F && rc >= 0; ++f) {
    int64_t c = owned_windows(rule_off, sym, len, head, tail, n, file_off[f], file_off[f + 1], 1, &P);
    if (c < 0) rc = c;
  }
  for (int64_t r = 1; r < R && rc >= 0; ++r) {
    if (w[r] == 0) continue;
    int64_t c = owned_windows(rule_off, sym, len, head, tail, n, rule_off[r], rule_off[r + 1], w[r], &P);
    if (c < 0) rc = c;
  }
  int64_t u = rc >= 0 ? wide_runs(&P, hi_out, lo_out, cnt_out) : rc;
  free(len), free(w), free(head), free(tail), free(P.key), free(P.key2), free(P.wt);
  return u;
}

/* ------------------------------------------------------------------------ */
/* Sequitur properties of a grammar                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t key;
  int64_t rule, pos;
} or_digram;

static int cmp_digram(const void* a, const void* b) {
  const or_digram *x = a, *y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->rule != y->rule) return x->rule < y->rule ? -1 : 1;
  return x->pos < y->pos ? -1 : (x->pos > y->pos);
}

/* Sequitur's properties, as the grammar TADOC builds on (Background,
 * "TADOC"). Bit flags of what fails (0 = all hold):
 *   1  digram uniqueness: an ordered pair of adjacent symbols occurs twice
 *      (root pairs are taken inside one file span, as the splitters separate
 *      files), unless the two occurrences overlap inside a run x x x;
 *   2  rule utility: a rule other than the root is referenced fewer than 2 times;
 *   4  a rule other than the root has fewer than 2 symbols;
 *   8  a cycle, or a rule not reachable from the root. */
int or_check_sequitur(const int64_t* rule_off, int64_t R, const int32_t* sym, const int64_t* file_off,
                      int64_t F) {
  int flags = 0;
  int64_t S = rule_off[R];
  or_digram* d = malloc(sizeof(or_digram) * (size_t)(S > 0 ? S : 1));
  int64_t* refs = calloc((size_t)R, sizeof(int64_t));
  int32_t* post = malloc(sizeof(int32_t) * (size_t)R);
  if (!d || !refs || !post) {
    free(d), free(refs), free(post);
    return OR_ERR_NOMEM;
  }
  int64_t nd = 0;
  /* the root's pairs are taken inside one file span at a time; another
   * rule's pairs inside its body */
  for (int64_t r = 0; r < R; ++r) {
    int64_t nspan = r == 0 ? F : 1;
    for (int64_t f = 0; f < nspan; ++f) {
      int64_t lo = r == 0 ? file_off[f] : rule_off[r];
      int64_t hi = r == 0 ? file_off[f + 1] : rule_off[r + 1];
      for (int64_t i = lo; i + 1 < hi; ++i) {
        d[nd].key = (uint64_t)(uint32_t)sym[i] << 32 | (uint32_t)sym[i + 1];
        d[nd].rule = r;
        d[nd].pos = i;
        ++nd;
      }
    }
    for (int64_t i = rule_off[r]; i < rule_off[r + 1]; ++i)
      if (sym[i] < 0) refs[-sym[i]] += 1;
    if (r > 0 && rule_off[r + 1] - rule_off[r] < 2) flags |= 4;
  }
  qsort(d, (size_t)nd, sizeof(or_digram), cmp_digram);
  for (int64_t i = 0; i < nd;) {
    int64_t j = i;
    while (j < nd && d[j].key == d[i].key) ++j;
    if (j - i == 2) {
      /* allowed only as two overlapping occurrences in a run */
      int overlap = d[i].rule == d[i + 1].rule && d[i + 1].pos == d[i].pos + 1 &&
                    (uint32_t)(d[i].key >> 32) == (uint32_t)d[i].key;
      if (!overlap) flags |= 1;
    } else if (j - i > 2) {
      flags |= 1;
    }
    i = j;
  }
  for (int64_t r = 1; r < R; ++r)
    if (refs[r] < 2) flags |= 2;
  int64_t n = or_postorder(rule_off, R, sym, post);
  if (n < 0 || n != R) flags |= 8;
  free(d), free(refs), free(post);
  return flags;
}
