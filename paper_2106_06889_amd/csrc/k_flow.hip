// k_flow.hip -- top-down rule weights by a dataflow walk: a rule passes its
// weight to its sub-rules as soon as its last pending in-edge has arrived,
// with no barrier between levels.
//
// Paper: Algorithm "Top-Down Traversal" (a rule's weight is the sum, over its
// in-edges, of the referencing rule's weight; a rule is processed once all
// its in-edges have arrived, tracked by its mask of pending in-edges; the
// initial weights are the frequencies in the root).
//
// Differences from the paper's design (same weights): the paper runs rounds
// relaunched from the host until nothing changes, and the level walk in
// k_levels.hip runs them as levels with a grid barrier between them. Here
// readiness alone orders the work. A rule's weight and its pending in-edges
// share one 64-bit word (weight << kPendBits | pending); a parent's reference
// is one atomic add of (weight << kPendBits) - 1, and the thread whose add
// retires the last in-edge learns the rule's final weight from the value the
// atomic returns. It queues (rule, weight) in its workgroup's LDS ring and
// the workgroup walks that rule in a later round, so a chain of rules costs
// a few dependent memory round trips per link instead of a grid barrier plus
// a list round trip per level. Levels (longest path from the root) are not
// produced; queries that need them build them with the level walk.
//
// Rounds. Each workgroup runs rounds of at most kT rules (its thread count).
// A round's bodies are walked position-parallel: every thread loads one
// rule's offsets, a block scan of the body lengths places the round's
// symbols on one axis, and each thread takes symbols t, t + kT, ... (found
// back to their rule by binary search in LDS), 8 at a time, issuing all 8
// atomics before it looks at any result. A round costs about the same for a
// 2-symbol body and a 300-symbol one, and neighbouring threads read
// neighbouring symbols. At the end of the walk, where rounds hold a few
// rules of long chains of deep rules, a thread walks a short rule its atomic
// readied at once, and so down the chain, instead of a round per link.
//
// Work sharing. A round takes rules from the workgroup's LDS ring first,
// then from a held range of a global queue. The queue starts with level 1
// (the rules without pending in-edges, in rule-id order, in chunks of
// `chunk0` rules; see launch_flow_walk) and grows by
// chunks that workgroups publish when their ring holds more than `keep`
// rules (more than one round's worth while some workgroup waits idle), or
// when a round readies more rules than the ring holds. Tickets hand out the
// chunks in order: a workgroup takes the next one when its range is used up
// and its ring holds less than a round, and keeps working from its ring
// until a published chunk is there. A published chunk is a range of
// the queue's (rule, weight) arrays plus a descriptor, stored with release
// order after the entries; the ticket holder polls the descriptor and
// acquires. Termination: `live` counts the rules queued anywhere or being
// walked. A round adds (rules readied into its ring - rules taken) once,
// after its pushes; rules it publishes straight to the queue are added
// before they are published, since another workgroup may walk them (and
// subtract them) before the round ends. The rules a round has taken stay
// counted until it ends, so `live` is zero only when no work is left, and a
// workgroup waiting on a ticket leaves when it reads zero. Rules a thread
// walks in place are never counted: the round's own rules keep `live` above
// zero while it walks them. Every wait is bounded.
#include "device.h"

namespace gt {

constexpr uint32_t kFlowSpinLimit = 1u << 21;
// Rounds of at most kFlowContRound rules (the end of the walk, where the
// deepest rules form chains) let a thread walk a rule it readied at once:
// bodies of at most kFlowContBody symbols, at most kFlowContLinks links in a
// row; the rest goes to the ring.
constexpr int kFlowContRound = 32;
constexpr int64_t kFlowContBody = 16;
constexpr int kFlowContLinks = 256;

template <int kT>
struct FlowLds {
  static constexpr int kRing = 8 * kT;  // power of two
  int32_t rc[kRing];  // ring of ready rules and their final weights
  uint64_t rw[kRing];
  int64_t ra[kT];        // the round's rules: body start,
  uint64_t rwt[kT];      // weight,
  uint32_t roff[kT + 1];  // and first position on the round's symbol axis
  uint32_t scan[kT / 64 + 1];
  uint32_t head, tail;   // ring cursors: entries [head, tail), slot = cursor mod kRing
  uint32_t take_at;      // ring part of the round: [take_at, take_at + n - nglob)
  uint32_t gpos, gleft;  // held range of the global queue
  uint32_t gtake, nglob;  // global part of the round: [gtake, gtake + nglob)
  int64_t ticket;        // ticket whose chunk has not arrived (-1: none)
  int64_t n1;            // rules of level 1
  uint32_t n0;           // level-1 chunks
  int32_t chunk0;        // rules per level-1 chunk
  int32_t n;             // rules of the round (-1: leave)
  uint32_t pushed;       // rules readied into the ring in the round
  uint32_t sp_base, sp_n, sp_from;  // spill of the ring's excess at round end
  uint64_t part[kT / 64];
};

// Publishes queue entries [base, base + n) (already stored, with release
// order, by this wave or the workgroup) as one chunk.
__device__ __forceinline__ void flow_publish(FlowState* fs, const FlowBufs& fb, uint32_t* status, uint32_t base,
                                             uint32_t n) {
  const uint32_t j = atomicAdd(&fs->nspill, 1u);
  if (j >= fb.ndesc) {
    atomicOr(status, (uint32_t)ST_FLOW);
    return;
  }
  __hip_atomic_store(&fb.desc[j], ((uint64_t)base << 16) | n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Readied rules of one wave step: into the ring while it has room, the rest
// straight to the global queue as one chunk of this wave.
template <int kT>
__device__ __forceinline__ void flow_push(FlowLds<kT>& L, FlowState* fs, const FlowBufs& fb, uint32_t* status,
                                          bool ready, int32_t c, uint64_t w) {
  constexpr uint32_t kRing = FlowLds<kT>::kRing;
  const uint64_t mask = __ballot(ready);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  const uint32_t n = (uint32_t)__popcll(mask);
  uint32_t base = 0, room = 0;
  if (lane_id() == leader) {
    base = atomicAdd(&L.tail, n);
    const uint32_t lim = L.head + kRing;  // head does not move while rules are walked
    room = (int32_t)(lim - base) <= 0 ? 0u : (lim - base < n ? lim - base : n);
    if (room < n) atomicSub(&L.tail, n - room);  // only the wave that crosses the limit keeps a part
    if (room) atomicAdd(&L.pushed, room);          // counted in `live` at the end of the round
  }
  base = __shfl(base, leader);
  room = __shfl(room, leader);
  const uint32_t rank = (uint32_t)__popcll(mask & lanes_below());
  if (ready && rank < room) {
    const uint32_t slot = (base + rank) & (kRing - 1);
    L.rc[slot] = c;
    L.rw[slot] = w;
  }
  if (room == n) return;
  const uint32_t m = n - room;
  uint32_t qb = 0;
  if (lane_id() == leader) {
    // counted before anyone can take them: another workgroup may walk them
    // (and subtract them) before this round ends
    atomicAdd(reinterpret_cast<unsigned long long*>(&fs->live), (unsigned long long)m);
    qb = atomicAdd(&fs->space, m);
  }
  qb = __shfl(qb, leader);
  const bool ok = (uint64_t)qb + m <= fb.qcap;
  if (ready && rank >= room && ok) {
    fb.qc[qb + rank - room] = c;
    fb.qw[qb + rank - room] = w;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane_id() == leader) {
    if (ok) flow_publish(fs, fb, status, qb, m);
    else atomicOr(status, (uint32_t)ST_FLOW);
  }
}

// The round's rules, chosen by thread 0: ring entries first (the deeper
// rules, so chains of sub-rules move on as early as possible), then the held
// global range. When the range is used up and the ring holds less than a
// round, a ticket is taken; a level-1 chunk is there at once, a later one is
// picked up once its descriptor is published. With neither ring entries nor
// a range the workgroup waits for its chunk, or leaves when no work is left.
// A long wait polls more slowly, and reads the live count only every 8th
// time: polls of a counter queue with the atomics on its line, and at the
// end of the walk most workgroups wait while a few walk the deepest rules.
template <int kT>
__device__ __forceinline__ void flow_decide(FlowLds<kT>& L, FlowState* fs, const FlowBufs& fb, uint32_t* status) {
  const uint32_t n0 = L.n0;
  bool idle = false;
  for (uint32_t it = 0;; ++it) {
    if (L.gleft == 0) {
      if (L.ticket < 0 && L.tail - L.head < (uint32_t)kT) L.ticket = atomicAdd(&fs->ticket, 1u);
      if (L.ticket >= 0) {
        const uint32_t j = (uint32_t)L.ticket;
        if (j < n0) {
          const int64_t st = (int64_t)j * L.chunk0, left = L.n1 - st;
          L.gpos = (uint32_t)st;
          L.gleft = (uint32_t)(left < L.chunk0 ? left : L.chunk0);
          L.ticket = -1;
        } else if (j - n0 < fb.ndesc) {
          const uint64_t v = __hip_atomic_load(&fb.desc[j - n0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            L.gpos = (uint32_t)(v >> 16);
            L.gleft = (uint32_t)(v & 0xffffu);
            L.ticket = -1;
          }
        }
      }
    }
    if (L.tail != L.head || L.gleft) break;
    if (!idle) {  // counted idle while it waits, so that busy workgroups share
      idle = true;
      atomicAdd(&fs->idle, 1u);
    }
    // zero only once every rule has been walked: the chunk will never come
    if ((it < 16 || (it & 7) == 0) &&
        __hip_atomic_load(&fs->live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      L.n = -1;
      return;
    }
    if (it >= kFlowSpinLimit) {
      atomicOr(status, (uint32_t)ST_FLOW);
      L.n = -1;
      return;
    }
    if (it < 16) __builtin_amdgcn_s_sleep(2);
    else __builtin_amdgcn_s_sleep(16);
  }
  if (idle) atomicSub(&fs->idle, 1u);
  const uint32_t occ = L.tail - L.head;
  const uint32_t nr = occ < (uint32_t)kT ? occ : (uint32_t)kT;
  L.take_at = L.head;
  L.head += nr;
  const uint32_t ng = L.gleft < (uint32_t)kT - nr ? L.gleft : (uint32_t)kT - nr;
  L.gtake = L.gpos;
  L.gpos += ng;
  L.gleft -= ng;
  L.nglob = ng;
  L.n = (int32_t)(nr + ng);
}

// Exclusive scan of v over the workgroup; *total = the sum.
template <int kT>
__device__ __forceinline__ uint32_t flow_scan(uint32_t v, FlowLds<kT>& L, uint32_t* total) {
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane_id() >= d) x += y;
  }
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 63) L.scan[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int k = 0; k < kT / 64; ++k) {
      const uint32_t q = L.scan[k];
      L.scan[k] = s;
      s += q;
    }
    L.scan[kT / 64] = s;
  }
  __syncthreads();
  *total = L.scan[kT / 64];
  return L.scan[wv] + x - v;
}

// Retires one in-edge of rule c with weight w of the parent; returns the old
// packed word.
__device__ __forceinline__ uint64_t flow_retire(uint64_t* pw, int32_t c, uint64_t w) {
  return atomicAdd(reinterpret_cast<unsigned long long*>(&pw[c]), (unsigned long long)((w << kPendBits) - 1u));
}

template <int kT>
__global__ __launch_bounds__(kT) void k_flow(DevGrammar g, LoadCounters* lc, FlowState* fs, FlowBufs fb, int32_t keep,
                                             int32_t chunk0) {
  constexpr uint32_t kRing = FlowLds<kT>::kRing;
  __shared__ FlowLds<kT> L;
  uint32_t* status = &lc->status;
  if (lc->status & kBadLayout) return;  // set before this launch
  const int t = threadIdx.x;
  if (t == 0) {
    L.head = 0, L.tail = 0, L.pushed = 0, L.sp_n = 0, L.gleft = 0, L.gpos = 0, L.ticket = -1;
    L.n1 = fs->n1;
    L.chunk0 = chunk0;
    L.n0 = (uint32_t)((L.n1 + chunk0 - 1) / chunk0);
  }
  uint64_t tokens = 0;
  int64_t walked = 0;  // rules walked: the rounds' (thread 0) and the chains walked in place
  __syncthreads();
  for (;;) {
    if (t == 0) flow_decide(L, fs, fb, status);
    __syncthreads();
    const int32_t n = L.n;
    if (n < 0) break;
    const uint32_t nr = (uint32_t)n - L.nglob;
    int32_t c = -1;
    uint64_t w = 0;
    if ((uint32_t)t < nr) {
      const uint32_t slot = (L.take_at + (uint32_t)t) & (kRing - 1);
      c = L.rc[slot];
      w = L.rw[slot];
    } else if (t < n) {
      const uint32_t i = L.gtake + ((uint32_t)t - nr);
      c = fb.qc[i];
      w = fb.qw[i];
    }
    int64_t a = 0;
    uint32_t len = 0;
    if (c > 0 && c < g.R) {
      a = g.rule_off[c];
      len = (uint32_t)(g.rule_off[c + 1] - a);
    }
    uint32_t total;
    const uint32_t off = flow_scan(len, L, &total);  // its barriers also free the round's ring slots
    if (t < n) {
      L.ra[t] = a;
      L.rwt[t] = w;
      L.roff[t] = off;
    }
    if (t == 0) L.roff[n] = total;
    __syncthreads();
    // the round's symbols, 8 per thread at a time
    const bool tail = n <= kFlowContRound;
    bool has_cont = false;  // a rule this thread readied and walks itself (tail rounds)
    int32_t cc = 0;
    uint64_t cw = 0;
    int step = 1;
    while (step * 2 <= n) step *= 2;
    for (uint32_t p0 = 0; p0 < total; p0 += 8u * kT) {
      int32_t ri[8], v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) ri[k] = 0;
      for (int s2 = step; s2 >= 1; s2 >>= 1) {  // rule of each position: last roff <= p
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t p = p0 + (uint32_t)(k * kT + t);
          if (ri[k] + s2 < n && L.roff[ri[k] + s2] <= p) ri[k] += s2;
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t p = p0 + (uint32_t)(k * kT + t);
        v[k] = p < total ? g.sym[L.ra[ri[k]] + (p - L.roff[ri[k]])] : 0;
      }
      uint64_t old[8], wr[8];
      int32_t cs[8];
      bool ref[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {  // every atomic of the group is issued before any result is used
        const uint32_t p = p0 + (uint32_t)(k * kT + t);
        ref[k] = false;
        cs[k] = 0;
        old[k] = 0;
        wr[k] = 0;
        if (p >= total) continue;
        wr[k] = L.rwt[ri[k]];
        if (v[k] >= 0) {
          tokens += wr[k];
        } else if (-(int64_t)v[k] < g.R) {
          cs[k] = (int32_t)(-(int64_t)v[k]);
          ref[k] = true;
          old[k] = flow_retire(g.w, cs[k], wr[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (ref[k] && (old[k] >> kPendBits) + wr[k] >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
        const bool ready = ref[k] && (old[k] & kPendMask) == 1;
        const uint64_t wf = (old[k] >> kPendBits) + wr[k];
        const bool here = tail && ready && !has_cont;
        if (here) has_cont = true, cc = cs[k], cw = wf;
        flow_push(L, fs, fb, status, ready && !here, cs[k], wf);
      }
    }
    // Chains in place: the thread walks the rule it kept, then the first
    // rule that walk readies, and so on, a few memory round trips per link
    // instead of a round; every other readied rule goes to the ring.
    int links = 0;
    while (has_cont) {
      const int64_t a = g.rule_off[cc];
      const int64_t e = g.rule_off[cc + 1];
      if (e - a > kFlowContBody || links >= kFlowContLinks) {
        flow_push(L, fs, fb, status, true, cc, cw);
        break;
      }
      ++links;
      ++walked;
      bool nxt = false;
      int32_t nc = 0;
      uint64_t nw = 0;
      for (int64_t q0 = a; q0 < e; q0 += 8) {
        int32_t sv[8], ch[8];
        uint64_t o[8];
        bool rf[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sv[k] = q0 + k < e ? g.sym[q0 + k] : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {  // every atomic issued before any result is used
          rf[k] = false, ch[k] = 0, o[k] = 0;
          if (q0 + k >= e) continue;
          if (sv[k] >= 0) {
            tokens += cw;
          } else if (-(int64_t)sv[k] < g.R) {
            ch[k] = (int32_t)(-(int64_t)sv[k]);
            rf[k] = true;
            o[k] = flow_retire(g.w, ch[k], cw);
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (rf[k] && (o[k] >> kPendBits) + cw >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
          const bool ready = rf[k] && (o[k] & kPendMask) == 1;
          const uint64_t wf = (o[k] >> kPendBits) + cw;
          const bool here = ready && !nxt;
          if (here) nxt = true, nc = ch[k], nw = wf;
          flow_push(L, fs, fb, status, ready && !here, ch[k], wf);
        }
      }
      has_cont = nxt;
      cc = nc;
      cw = nw;
    }
    __syncthreads();
    if (t == 0) {
      // the round's ring pushes are done (published ones are counted already)
      const int64_t delta = (int64_t)L.pushed - (int64_t)n;
      if (delta) atomicAdd(reinterpret_cast<unsigned long long*>(&fs->live), (unsigned long long)delta);
      walked += n;
      L.pushed = 0;
      L.sp_n = 0;
      // share what is beyond `keep`; while other workgroups are idle, what is
      // beyond one round (the idle count is read only with such a backlog)
      const uint32_t occ = L.tail - L.head;
      uint32_t kp = (uint32_t)keep;
      if (occ > (uint32_t)kT && kp > (uint32_t)kT &&
          __hip_atomic_load(&fs->idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        kp = (uint32_t)kT;
      if (occ > kp) {
        const uint32_t sn = occ - kp < (uint32_t)kT ? occ - kp : (uint32_t)kT;
        const uint32_t base = atomicAdd(&fs->space, sn);
        if ((uint64_t)base + sn <= fb.qcap) {
          L.sp_base = base;
          L.sp_n = sn;
          L.sp_from = L.tail - sn;
        } else {
          atomicOr(status, (uint32_t)ST_FLOW);
        }
      }
    }
    __syncthreads();
    const uint32_t sn = L.sp_n;
    if (sn) {
      // the newest `sn` ring entries become a chunk of the global queue
      if ((uint32_t)t < sn) {
        const uint32_t slot = (L.sp_from + (uint32_t)t) & (kRing - 1);
        fb.qc[L.sp_base + t] = L.rc[slot];
        fb.qw[L.sp_base + t] = L.rw[slot];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the waves that stored
      }
      __syncthreads();
      if (t == 0) {
        flow_publish(fs, fb, status, L.sp_base, sn);
        L.tail -= sn;
      }
      // the next round's decision is thread 0's, after this
    }
  }
  // token and rule totals, one atomic each per workgroup
  tokens = wave_sum_u64(tokens);
  if (lane_id() == 0) L.part[t >> 6] = tokens;
  __syncthreads();
  if (t == 0) {
    uint64_t sum = 0;
    for (int k = 0; k < kT / 64; ++k) sum += L.part[k];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->tokens), (unsigned long long)sum);
  }
  __syncthreads();
  const uint64_t nw = wave_sum_u64((uint64_t)walked);
  if (lane_id() == 0) L.part[t >> 6] = nw;
  __syncthreads();
  if (t == 0) {
    uint64_t sum = 0;
    for (int k = 0; k < kT / 64; ++k) sum += L.part[k];
    if (sum) atomicAdd(&lc->placed, (int32_t)sum);
  }
}

template <int kT>
hipError_t launch_flow_kernel(const DevGrammar& g, LoadCounters* lc, FlowState* fs, const FlowBufs& fb, int32_t keep,
                              int32_t chunk0, int device, hipStream_t s) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  constexpr int kPerCu = 1024 / kT;  // workgroups that fit a CU together (LDS)
  const int64_t want = (g.R + kT - 1) / kT;
  const int64_t cap = (int64_t)(cus > 0 ? cus : 1) * kPerCu;
  const unsigned grid = (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
  const int32_t k = keep < 0 ? 0 : (keep > FlowLds<kT>::kRing - kT ? FlowLds<kT>::kRing - kT : keep);
  // no workgroup holds work while it waits, so the walk needs no co-residency
  k_flow<kT><<<grid, kT, 0, s>>>(g, lc, fs, fb, k, chunk0);
  return hipGetLastError();
}

hipError_t launch_flow_walk(const DevGrammar& g, LoadCounters* lc, FlowState* fs, const FlowBufs& fb,
                            const LevelParams& lp, int device, hipStream_t s) {
  // Level-1 chunks of ~128 rules: the first rules Sequitur made (low ids)
  // tend to head the deepest subtrees, and small chunks start more of them
  // at once (on the 10^8-token corpus: 479 us with 128, 536 with 1024, 917
  // with 4096; 64 is slower again, 514 us).
  const int32_t chunk0 = lp.flow_chunk < 1 ? 1 : (lp.flow_chunk > 65535 ? 65535 : lp.flow_chunk);
  if (lp.flow_group == 512)
    return launch_flow_kernel<512>(g, lc, fs, fb, lp.flow_keep * 512 / 1024, chunk0, device, s);
  return launch_flow_kernel<1024>(g, lc, fs, fb, lp.flow_keep, chunk0, device, s);
}

}  // namespace gt
