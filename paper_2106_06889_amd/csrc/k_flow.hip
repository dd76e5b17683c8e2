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
// Work sharing. Each workgroup runs rounds of at most kFlowThreads rules,
// one per thread (bodies longer than `long_body` symbols are walked by a
// whole wave, lanes across the body). A round takes its rules from the LDS
// ring; a workgroup whose ring is empty takes a ticket for one chunk of a
// global queue. The queue starts with level 1 (the rules without pending
// in-edges, in chunks of kFlowThreads) and grows by chunks that workgroups
// publish when their ring holds more than `keep` rules, or when a round
// readies more rules than the ring holds. A published chunk is a range of
// the queue's (rule, weight) arrays plus a descriptor, stored with release
// order after the entries; the ticket holder polls the descriptor and
// acquires. Termination: `live` counts the rules queued anywhere or being
// walked. A round adds (rules readied into its ring - rules taken) once,
// after its pushes; rules it publishes straight to the queue are added
// before they are published, since another workgroup may walk them (and
// subtract them) before the round ends. The rules a round has taken stay
// counted until it ends, so `live` is zero only when no work is left, and a
// workgroup waiting on a ticket leaves when it reads zero. Every wait is
// bounded.
#include "device.h"

namespace gt {

constexpr int kFlowThreads = 1024;
constexpr int kFlowRing = 8192;  // power of two
constexpr uint32_t kFlowSpinLimit = 1u << 21;

struct FlowLds {
  int32_t rc[kFlowRing];  // ring of ready rules and their final weights
  uint64_t rw[kFlowRing];
  int32_t lc[kFlowThreads];  // long bodies of the round
  uint64_t lw[kFlowThreads];
  uint32_t head, tail;  // ring cursors: entries [head, tail), slot = cursor mod kFlowRing
  uint32_t take_at;     // ring cursor of the round's first rule
  int32_t n;            // rules of the round (-1: leave)
  int32_t src;          // 0: ring, 1: global queue at gstart
  uint32_t gstart;
  uint32_t pushed;  // rules readied into the ring in the round
  int32_t nlong;
  uint32_t sp_base, sp_n, sp_from;  // spill of the ring's excess at round end
  uint64_t part[kFlowThreads / 64];
};

// Publishes queue entries [base, base + n) (already stored by this wave or,
// after a block barrier, by the workgroup) as one chunk.
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
__device__ __forceinline__ void flow_push(FlowLds& L, FlowState* fs, const FlowBufs& fb, uint32_t* status, bool ready,
                                          int32_t c, uint64_t w) {
  const uint64_t mask = __ballot(ready);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  const uint32_t n = (uint32_t)__popcll(mask);
  uint32_t base = 0, room = 0;
  if (lane_id() == leader) {
    base = atomicAdd(&L.tail, n);
    const uint32_t lim = L.head + kFlowRing;  // head does not move while rules are walked
    room = (int32_t)(lim - base) <= 0 ? 0u : (lim - base < n ? lim - base : n);
    if (room < n) atomicSub(&L.tail, n - room);  // only the wave that crosses the limit keeps a part
    if (room) atomicAdd(&L.pushed, room);          // counted in `live` at the end of the round
  }
  base = __shfl(base, leader);
  room = __shfl(room, leader);
  const uint32_t rank = (uint32_t)__popcll(mask & lanes_below());
  if (ready && rank < room) {
    const uint32_t slot = (base + rank) & (kFlowRing - 1);
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

// Retires one in-edge of rule c with weight w of the parent; returns the old
// packed word.
__device__ __forceinline__ uint64_t flow_retire(uint64_t* pw, int32_t c, uint64_t w) {
  return atomicAdd(reinterpret_cast<unsigned long long*>(&pw[c]), (unsigned long long)((w << kPendBits) - 1u));
}

// The round's source, chosen by thread 0: the ring, else a ticket of the
// global queue (waiting until its chunk is published or no work is left).
__device__ __forceinline__ void flow_decide(FlowLds& L, FlowState* fs, const FlowBufs& fb, uint32_t* status) {
  const uint32_t occ = L.tail - L.head;
  if (occ) {
    const uint32_t n = occ < (uint32_t)kFlowThreads ? occ : (uint32_t)kFlowThreads;
    L.take_at = L.head;
    L.head += n;
    L.n = (int32_t)n;
    L.src = 0;
    return;
  }
  const uint32_t j = atomicAdd(&fs->ticket, 1u);
  const uint32_t n0 = fs->nchunks0;
  if (j < n0) {
    const int64_t st = (int64_t)j * kFlowThreads;
    const int64_t left = fs->n1 - st;
    L.gstart = (uint32_t)st;
    L.n = (int32_t)(left < kFlowThreads ? left : kFlowThreads);
    L.src = 1;
    return;
  }
  const uint32_t k = j - n0;
  for (uint32_t it = 0;; ++it) {
    if (k < fb.ndesc) {
      const uint64_t v = __hip_atomic_load(&fb.desc[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        L.gstart = (uint32_t)(v >> 16);
        L.n = (int32_t)(v & 0xffffu);
        L.src = 1;
        return;
      }
    }
    // zero only once every rule has been walked: the chunk will never come
    if (__hip_atomic_load(&fs->live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      L.n = -1;
      return;
    }
    if (it >= kFlowSpinLimit) {
      atomicOr(status, (uint32_t)ST_FLOW);
      L.n = -1;
      return;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__global__ __launch_bounds__(kFlowThreads) void k_flow(DevGrammar g, LoadCounters* lc, FlowState* fs, FlowBufs fb,
                                                       int32_t long_body, int32_t keep) {
  __shared__ FlowLds L;
  uint32_t* status = &lc->status;
  const int t = threadIdx.x;
  if (t == 0) L.head = 0, L.tail = 0, L.pushed = 0, L.nlong = 0, L.sp_n = 0;
  uint64_t tokens = 0;
  int64_t walked = 0;  // thread 0
  __syncthreads();
  for (;;) {
    if (t == 0) flow_decide(L, fs, fb, status);
    __syncthreads();
    const int32_t n = L.n;
    if (n < 0) break;
    int32_t c = -1;
    uint64_t w = 0;
    if (t < n) {
      if (L.src == 0) {
        const uint32_t slot = (L.take_at + (uint32_t)t) & (kFlowRing - 1);
        c = L.rc[slot];
        w = L.rw[slot];
      } else {
        c = fb.qc[L.gstart + t];
        w = fb.qw[L.gstart + t];
      }
    }
    __syncthreads();  // the round's ring slots are read before pushes reuse them
    if (c > 0 && c < g.R) {
      const int64_t a = g.rule_off[c], e = g.rule_off[c + 1];
      if (e - a > long_body) {
        const int k = atomicAdd(&L.nlong, 1);
        L.lc[k] = c;
        L.lw[k] = w;
      } else {
        uint64_t words = 0;
        for (int64_t q0 = a; q0 < e; q0 += 8) {
          int32_t v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = q0 + k < e ? g.sym[q0 + k] : 0;
          uint64_t old[8];
          int32_t cs[8];
          bool ref[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {  // every atomic of the group is issued before any result is used
            ref[k] = false;
            cs[k] = 0;
            old[k] = 0;
            if (q0 + k >= e) continue;
            if (v[k] >= 0) {
              ++words;
            } else if (-(int64_t)v[k] < g.R) {
              cs[k] = (int32_t)(-(int64_t)v[k]);
              ref[k] = true;
              old[k] = flow_retire(g.w, cs[k], w);
            }
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (ref[k] && (old[k] >> kPendBits) + w >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
            flow_push(L, fs, fb, status, ref[k] && (old[k] & kPendMask) == 1, cs[k], (old[k] >> kPendBits) + w);
          }
        }
        tokens += words * w;
      }
    }
    __syncthreads();
    const int nl = L.nlong;
    for (int j = t >> 6; j < nl; j += kFlowThreads >> 6) {
      const int32_t p = L.lc[j];
      const uint64_t wp = L.lw[j];
      const int64_t e = g.rule_off[p + 1];
      int64_t q = g.rule_off[p] + lane_id();
      int32_t cur = q < e ? g.sym[q] : 0;
      uint64_t words = 0;
      for (; q < e; q += 64) {
        const int32_t nxt = q + 64 < e ? g.sym[q + 64] : 0;  // next load in flight while this one is used
        bool ready = false;
        int32_t cc = 0;
        uint64_t nw = 0;
        if (cur >= 0) {
          ++words;
        } else if (-(int64_t)cur < g.R) {
          cc = (int32_t)(-(int64_t)cur);
          const uint64_t old = flow_retire(g.w, cc, wp);
          if ((old >> kPendBits) + wp >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
          ready = (old & kPendMask) == 1;
          nw = (old >> kPendBits) + wp;
        }
        flow_push(L, fs, fb, status, ready, cc, nw);
        cur = nxt;
      }
      tokens += words * wp;
    }
    __syncthreads();
    if (t == 0) {
      // the round's ring pushes are done (published ones are counted already)
      const int64_t delta = (int64_t)L.pushed - (int64_t)n;
      if (delta) atomicAdd(reinterpret_cast<unsigned long long*>(&fs->live), (unsigned long long)delta);
      walked += n;
      L.pushed = 0;
      L.nlong = 0;
      L.sp_n = 0;
      const uint32_t occ = L.tail - L.head;
      if (occ > (uint32_t)keep) {
        const uint32_t sn = occ - (uint32_t)keep < (uint32_t)kFlowThreads ? occ - (uint32_t)keep : (uint32_t)kFlowThreads;
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
        const uint32_t slot = (L.sp_from + (uint32_t)t) & (kFlowRing - 1);
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
    for (int k = 0; k < kFlowThreads / 64; ++k) sum += L.part[k];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->tokens), (unsigned long long)sum);
    if (walked) atomicAdd(&lc->placed, (int32_t)walked);
  }
}

__global__ void k_flow_init(const LoadCounters* lc, FlowState* fs) {
  if (threadIdx.x != 0) return;
  const int64_t n1 = lc->frontier0;
  fs->n1 = n1;
  fs->nchunks0 = (uint32_t)((n1 + kFlowThreads - 1) / kFlowThreads);
  fs->live = n1;
  fs->space = (uint32_t)n1;
  fs->ticket = 0;
  fs->nspill = 0;
}

hipError_t launch_flow_walk(const DevGrammar& g, LoadCounters* lc, FlowState* fs, const FlowBufs& fb,
                            const LevelParams& lp, int device, hipStream_t s) {
  hipError_t e = launch_fill_u64(fb.desc, fb.ndesc, 0, s);
  if (e != hipSuccess) return e;
  k_flow_init<<<1, 64, 0, s>>>(lc, fs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  const int64_t want = (g.R + kFlowThreads - 1) / kFlowThreads;
  const int64_t cap = cus > 0 ? cus : 1;
  const unsigned grid = (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
  const int32_t keep = lp.flow_keep < 0 ? 0 : (lp.flow_keep > kFlowRing - kFlowThreads ? kFlowRing - kFlowThreads : lp.flow_keep);
  // no workgroup holds work while it waits, so the walk needs no co-residency
  k_flow<<<grid, kFlowThreads, 0, s>>>(g, lc, fs, fb, lp.long_body < 1 ? 1 : lp.long_body, keep);
  return hipGetLastError();
}

}  // namespace gt
