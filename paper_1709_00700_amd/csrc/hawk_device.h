// Device-side building blocks shared by the kernel files: column loads, the
// two hash functions, atomics (LDS and device scope, exact 128-bit sums),
// join-table probe/insert, per-row pipeline evaluation, aggregation-table
// slot lookup and updates.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "hawk_plan.h"

typedef long long v16i64 __attribute__((ext_vector_type(16)));

#define WAVE 64

// ------------------------------------------------------------------ small helpers
__device__ __forceinline__ int64_t load_col(const HkCol& c, int64_t row) {
  if (c.dtype == HK_T_I32) return static_cast<const int32_t*>(c.ptr)[row];
  if (c.dtype == HK_T_I64) return static_cast<const int64_t*>(c.ptr)[row];
  return static_cast<const int8_t*>(c.ptr)[row];
}

// A column value as loaded: the aligned 8-byte block that holds the element.
// Every element type then takes one branch-free 64-bit load, so all loads of
// a phase (or of several rows) can be in flight at once; the element is
// shifted out and sign-extended when it is first used. An element is
// naturally aligned (checked at registration), so its 8-aligned block lies
// in the element's own page: the load never touches an unmapped address.
struct HkRaw { uint64_t w; };
typedef const __attribute__((address_space(1))) uint64_t hk_global_u64;  // a global (not flat) load
__device__ __forceinline__ uint32_t col_lg(int32_t dtype) {
  return dtype == HK_T_I64 ? 3u : (dtype == HK_T_I32 ? 2u : 0u);
}
// A column whose type is a compile-time constant (kernels compiled for one
// plan) and 32 bits wide is loaded as 32 bits (one register in flight);
// otherwise the aligned 64-bit word that holds the value.
__device__ __forceinline__ bool narrow_i32(const HkCol& c) {
  return __builtin_constant_p(c.dtype) && c.dtype == HK_T_I32;
}
__device__ __forceinline__ void load_raw(const HkCol& c, int64_t row, HkRaw& v) {
  const uint64_t a = reinterpret_cast<uint64_t>(c.ptr) + (static_cast<uint64_t>(row) << col_lg(c.dtype));
  if (narrow_i32(c)) v.w = *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(a);
  else v.w = *reinterpret_cast<hk_global_u64*>(a & ~7ull);
}
__device__ __forceinline__ int64_t raw_value(const HkCol& c, int64_t row, const HkRaw& v) {
  if (narrow_i32(c)) return static_cast<int32_t>(static_cast<uint32_t>(v.w));
  const uint32_t lg = col_lg(c.dtype);
  const uint64_t a = reinterpret_cast<uint64_t>(c.ptr) + (static_cast<uint64_t>(row) << lg);
  const uint32_t sh = static_cast<uint32_t>(a & 7ull) * 8u;
  const uint32_t top = 64u - (8u << lg);
  return static_cast<int64_t>((v.w >> sh) << top) >> top;
}

// The row of a column's own table behind pipeline row v. With a CROSS_JOIN
// (kernels of a class that handles one), v runs over the product in
// row-major order: v / xinner on the looped table, v % xinner on the second
// (quotient by multiplication with the rounded-up reciprocal, exact for
// 32-bit v: Lemire, Kaser and Kurz, "Faster remainder by direct computation").
template <class S>
__device__ __forceinline__ int64_t xrow(const HkPlan& P, const HkCol& c, int64_t v) {
  if (!S::cross || P.xinner == 0 || c.side == 0) return v;
  const uint64_t q = P.xinner == 1 ? static_cast<uint64_t>(v) : __umul64hi(P.xmagic, static_cast<uint64_t>(v));
  return c.side == 1 ? static_cast<int64_t>(q) : v - static_cast<int64_t>(q) * P.xinner;
}

// Murmur3 64-bit finaliser (Appleby, public domain).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// slot of `key` under hash function with parameter a, table of 2^log2cap slots
template <int HASH>
__device__ __forceinline__ uint32_t hslot(uint64_t key, uint64_t a, uint32_t log2cap) {
  if (HASH == HK_MURMUR) return static_cast<uint32_t>(fmix64(key ^ a) & ((1ull << log2cap) - 1));
  // multiply-shift (Dietzfelbinger et al.): top log2cap bits of a*key mod 2^64, a odd
  return static_cast<uint32_t>((key * a) >> (64 - log2cap));
}

template <bool LDS>
__device__ __forceinline__ void at_add(uint64_t* p, uint64_t v) {
  if (LDS) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ uint64_t at_add_ret(uint64_t* p, uint64_t v) {
  if (LDS) return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ void at_min(uint64_t* p, int64_t v) {
  int64_t* q = reinterpret_cast<int64_t*>(p);
  if (LDS) __hip_atomic_fetch_min(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else __hip_atomic_fetch_min(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ void at_max(uint64_t* p, int64_t v) {
  int64_t* q = reinterpret_cast<int64_t*>(p);
  if (LDS) __hip_atomic_fetch_max(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else __hip_atomic_fetch_max(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ uint64_t at_cas(uint64_t* p, uint64_t expected, uint64_t desired) {
  if (LDS)
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found in memory
}
__device__ __forceinline__ uint64_t at_xchg(uint64_t* p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_err(int* err, int bit) {
  __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exact 128-bit accumulation without 128-bit atomics: the low word takes the
// value modulo 2^64; the high word takes the carry out of the low word minus
// the sign (a negative v is (uint64)v - 2^64).
template <bool LDS>
__device__ __forceinline__ void at_add128(uint64_t* lo, uint64_t* hi, int64_t v) {
  uint64_t u = static_cast<uint64_t>(v);
  uint64_t old = at_add_ret<LDS>(lo, u);
  int64_t d = static_cast<int64_t>(old + u < old) - static_cast<int64_t>(v < 0);
  if (d != 0) at_add<LDS>(hi, static_cast<uint64_t>(d));
}
// adds a 128-bit partial (l, h)
template <bool LDS>
__device__ __forceinline__ void at_add128_pair(uint64_t* lo, uint64_t* hi, uint64_t l, int64_t h) {
  uint64_t old = at_add_ret<LDS>(lo, l);
  int64_t d = h + static_cast<int64_t>(old + l < old);
  if (d != 0) at_add<LDS>(hi, static_cast<uint64_t>(d));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << __lane_id()) - 1ull;
}

// ------------------------------------------------------------------ join tables
// slot word: key (high 32 bits) | payload (low 32 bits); all-ones = empty;
// key -1 would look empty and lives in the side word (bit 32 = present)

// Robin-hood linear probing (the extension Section 7.5.1 names): an entry's
// displacement is its distance from its home slot; an insertion that meets
// an entry displaced less than itself takes that slot and carries the
// evicted entry on (atomic compare-exchange per step), so displacements stay
// even. side[1] records the largest displacement, which bounds a lookup.
template <int HASH>
__device__ __forceinline__ void robin_insert(const HkJoinTable& t, const HkHash& h, uint64_t w, int* err) {
  const uint32_t mask = (1u << t.log2cap) - 1u;
  const uint32_t key = static_cast<uint32_t>(w >> 32);
  uint64_t cur = w;
  uint32_t pos = hslot<HASH>(key, h.a[0], t.log2cap);
  uint32_t d = 0;
  while (d <= HK_ROBIN_MAX_DISP && d <= mask) {
    const uint64_t old = t.slots[pos];
    if (old == HK_EMPTY) {
      if (at_cas<false>(&t.slots[pos], HK_EMPTY, cur) == HK_EMPTY) {
        at_max<false>(t.side + 1, static_cast<int64_t>(d));
        return;
      }
      continue;  // taken meanwhile: look at the slot again
    }
    if (static_cast<uint32_t>(old >> 32) == static_cast<uint32_t>(cur >> 32)) {
      set_err(err, HK_ERR_DUPKEY);
      return;
    }
    const uint32_t dold = (pos - hslot<HASH>(static_cast<uint32_t>(old >> 32), h.a[0], t.log2cap)) & mask;
    if (dold < d) {
      if (at_cas<false>(&t.slots[pos], old, cur) != old) continue;  // changed meanwhile
      at_max<false>(t.side + 1, static_cast<int64_t>(d));
      cur = old;  // the richer entry moves on
      d = dold;
    }
    pos = (pos + 1) & mask;
    ++d;
  }
  set_err(err, HK_ERR_CAPACITY);
}

template <int HASH>
__device__ __forceinline__ bool robin_lookup(const HkJoinTable& t, const HkHash& h, uint32_t key, int32_t& pay) {
  const uint32_t mask = (1u << t.log2cap) - 1u;
  const uint32_t maxd = static_cast<uint32_t>(t.side[1]);
  uint32_t pos = hslot<HASH>(key, h.a[0], t.log2cap);
  for (uint32_t d = 0; d <= maxd; ++d) {
    const uint64_t w = t.slots[pos];
    if (w == HK_EMPTY) return false;
    if (static_cast<uint32_t>(w >> 32) == key) {
      pay = static_cast<int32_t>(static_cast<uint32_t>(w));
      return true;
    }
    pos = (pos + 1) & mask;
  }
  return false;
}

// Home slot of a join key under linear probing: the first slot of an
// aligned pair, the pair picked by the hash, so a lookup reads whole pairs
// (one 16-byte load each: a random gather costs the vector memory pipeline
// per lane and load, whatever the width up to 16 bytes).
template <int HASH>
__device__ __forceinline__ uint32_t join_group(uint64_t key, const HkHash& h, uint32_t log2cap) {
  return hslot<HASH>(key, h.a[0], log2cap - 1) << 1;
}

// linear probing from pair g on, pair by pair until the key or an empty slot
// (the key is never the all-ones key, so a key match is never an empty slot;
// in a built table a key sits before the first empty slot of its probe
// sequence, and a pair read that holds it holds it once)
__device__ __forceinline__ bool join_scan_from(const HkJoinTable& t, uint32_t k, uint32_t g, int32_t& pay) {
  const uint32_t mask = (1u << t.log2cap) - 1u;
  for (uint32_t i = 0; i <= mask; i += 2) {
    const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(t.slots + g);
    const bool f0 = static_cast<uint32_t>(x.x >> 32) == k, f1 = static_cast<uint32_t>(x.y >> 32) == k;
    if (f0 || f1) {
      pay = static_cast<int32_t>(static_cast<uint32_t>(f0 ? x.x : x.y));
      return true;
    }
    if (x.x == HK_EMPTY || x.y == HK_EMPTY) return false;
    g = (g + 2) & mask;
  }
  return false;
}

// Copies a join table's slots into LDS (all threads of the workgroup, 16
// bytes each per step) and points the table there: its lookups then read
// LDS. The caller synchronises the workgroup before the first lookup.
__device__ __forceinline__ void stage_join(HkJoinTable& t, uint64_t* dst, uint32_t log2cap) {
  const ulonglong2* s = reinterpret_cast<const ulonglong2*>(t.slots);
  ulonglong2* d = reinterpret_cast<ulonglong2*>(dst);
  const uint32_t n = (1u << log2cap) / 2;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
  t.slots = dst;
  t.log2cap = log2cap;
}

template <int HT, int HASH>
__device__ __forceinline__ bool join_lookup(const HkJoinTable& t, const HkHash& h, int32_t key, int32_t& pay) {
  if (key == -1) {
    uint64_t s = *t.side;
    pay = static_cast<int32_t>(static_cast<uint32_t>(s));
    return (s >> 32) != 0;
  }
  const uint64_t k64 = static_cast<uint32_t>(key);
  if (HT == HK_LIN && t.robin) return robin_lookup<HASH>(t, h, static_cast<uint32_t>(key), pay);
  if (HT == HK_LIN) return join_scan_from(t, static_cast<uint32_t>(key), join_group<HASH>(k64, h, t.log2cap), pay);
#pragma unroll
  for (int i = 0; i < HK_CUCKOO_D; ++i) {
    uint64_t w = t.slots[hslot<HASH>(k64, h.a[i], t.log2cap)];
    if (w != HK_EMPTY && static_cast<uint32_t>(w >> 32) == static_cast<uint32_t>(key)) {
      pay = static_cast<int32_t>(static_cast<uint32_t>(w));
      return true;
    }
  }
  return false;
}

template <int HT, int HASH>
__device__ __forceinline__ void join_insert(const HkJoinTable& t, const HkHash& h, int32_t key, int32_t pay,
                                            int* err) {
  if (key == -1) {
    uint64_t v = (1ull << 32) | static_cast<uint32_t>(pay);
    if (at_cas<false>(t.side, 0ull, v) != 0ull) set_err(err, HK_ERR_DUPKEY);
    return;
  }
  const uint64_t w = (static_cast<uint64_t>(static_cast<uint32_t>(key)) << 32) | static_cast<uint32_t>(pay);
  if (HT == HK_LIN && t.robin) {
    robin_insert<HASH>(t, h, w, err);
    return;
  }
  if (HT == HK_LIN) {
    const uint32_t mask = (1u << t.log2cap) - 1u;
    uint32_t s = join_group<HASH>(static_cast<uint32_t>(key), h, t.log2cap);
    for (uint32_t i = 0; i <= mask; ++i) {
      uint64_t cur = t.slots[s];
      if (cur == HK_EMPTY) {
        cur = at_cas<false>(&t.slots[s], HK_EMPTY, w);
        if (cur == HK_EMPTY) return;
      }
      if (static_cast<uint32_t>(cur >> 32) == static_cast<uint32_t>(key)) {
        set_err(err, HK_ERR_DUPKEY);
        return;
      }
      s = (s + 1) & mask;
    }
    set_err(err, HK_ERR_CAPACITY);
  } else {
    // cuckoo insert: exchange into the current choice, the evicted entry moves
    // on to its next choice; bounded chain
    uint64_t cur = w;
    int i = 0;
    for (int step = 0; step < HK_CUCKOO_MAX_EVICT; ++step) {
      const uint64_t k = cur >> 32;
      const uint32_t s = hslot<HASH>(k, h.a[i], t.log2cap);
      const uint64_t old = at_xchg(&t.slots[s], cur);
      if (old == HK_EMPTY) return;
      if ((old >> 32) == k) {  // another entry with the same key
        set_err(err, HK_ERR_DUPKEY);
        return;
      }
      cur = old;
      int j = 0;
#pragma unroll
      for (int jj = HK_CUCKOO_D - 1; jj >= 0; --jj)
        if (hslot<HASH>(old >> 32, h.a[jj], t.log2cap) == s) j = jj;
      i = (j + 1) % HK_CUCKOO_D;
    }
    set_err(err, HK_ERR_CUCKOO);
  }
}

// ------------------------------------------------------------------ row evaluation
// The first load phase of a row: the columns read before anything can drop
// the row (FILTER columns; probe keys when there is no filter; value columns
// when there is neither filter nor probe). Kernels that scan several rows
// per thread fetch this phase for all of them before evaluating any.
template <class S>
struct HkFirst {
  static constexpr int A = S::colA;
  static constexpr int B = S::filters == 0 ? S::colB : 0;
  static constexpr int C = (S::filters == 0 && S::probes == 0) ? S::colC : 0;
  HkRaw a[A > 0 ? A : 1], b[B > 0 ? B : 1], c[C > 0 ? C : 1];
};

// Issues the same number of loads whatever the plan (unused slots read the
// context's zero block at row 0), so the wait for a row's loads can leave
// the loads issued after them in flight.
template <class S>
__device__ __forceinline__ void fetch_first(const HkPlan& P, int64_t row, HkFirst<S>& f) {
#pragma unroll
  for (int c = 0; c < HkFirst<S>::A; ++c) load_raw(P.colA[c], xrow<S>(P, P.colA[c], c < P.ncolA ? row : 0), f.a[c]);
#pragma unroll
  for (int c = 0; c < HkFirst<S>::B; ++c) load_raw(P.colB[c], xrow<S>(P, P.colB[c], c < P.ncolB ? row : 0), f.b[c]);
#pragma unroll
  for (int c = 0; c < HkFirst<S>::C; ++c) load_raw(P.colC[c], xrow<S>(P, P.colC[c], c < P.ncolC ? row : 0), f.c[c]);
}

// Pushes one row through LOOP's loads, FILTER, HASH_PROBE and (if VALUES)
// ARITHMETIC. Branched: returns false as soon as the row is dropped.
// Predicated: evaluates everything and returns the result_increment.
// PRE: the first load phase comes from `f` (fetched earlier) instead of memory.
template <int PRED, int HT, int HASH, bool VALUES, class S, bool PRE>
__device__ __forceinline__ bool eval_row_f(const HkPlan& P, int64_t row, const HkFirst<S>& f, v16i64& r) {
  // every load of a phase is issued before any is widened, so their
  // latencies overlap
  {
    HkRaw la[S::colA > 0 ? S::colA : 1];
#pragma unroll
    for (int c = 0; c < S::colA; ++c)
      if (c < P.ncolA) {
        if (PRE) la[c] = f.a[c];
        else load_raw(P.colA[c], xrow<S>(P, P.colA[c], row), la[c]);
      }
#pragma unroll
    for (int c = 0; c < S::colA; ++c)
      if (c < P.ncolA) r[P.colA[c].reg] = raw_value(P.colA[c], xrow<S>(P, P.colA[c], row), la[c]);
  }
  bool pass = true;
#pragma unroll
  for (int f2 = 0; f2 < S::filters; ++f2) {
    if (f2 >= P.nfilters) break;
    const int64_t x = r[P.filters[f2].reg];
    pass = pass & (x >= P.filters[f2].lo) & (x <= P.filters[f2].hi);
  }
  if (PRED == HK_BR && !pass) return false;
  if (S::colB > 0) {
    HkRaw lb[S::colB > 0 ? S::colB : 1];
#pragma unroll
    for (int c = 0; c < S::colB; ++c)
      if (c < P.ncolB) {
        if (PRE && c < HkFirst<S>::B) lb[c] = f.b[c < HkFirst<S>::B ? c : 0];
        else load_raw(P.colB[c], xrow<S>(P, P.colB[c], row), lb[c]);
      }
#pragma unroll
    for (int c = 0; c < S::colB; ++c)
      if (c < P.ncolB) r[P.colB[c].reg] = raw_value(P.colB[c], xrow<S>(P, P.colB[c], row), lb[c]);
  }
#pragma unroll
  for (int p = 0; p < S::probes; ++p) {
    if (p >= P.nprobes) break;
    int32_t pay = 0;
    const bool found = join_lookup<HT, HASH>(P.probes[p].t, P.hash, static_cast<int32_t>(r[P.probes[p].fk_reg]), pay);
    if (PRED == HK_BR && !found) return false;
    pass = pass & found;
    r[P.probes[p].pay_reg] = pay;
  }
  if (!VALUES) return pass;
  {
    HkRaw lc[S::colC > 0 ? S::colC : 1];
#pragma unroll
    for (int c = 0; c < S::colC; ++c)
      if (c < P.ncolC) {
        if (PRE && c < HkFirst<S>::C) lc[c] = f.c[c < HkFirst<S>::C ? c : 0];
        else load_raw(P.colC[c], xrow<S>(P, P.colC[c], row), lc[c]);
      }
#pragma unroll
    for (int c = 0; c < S::colC; ++c)
      if (c < P.ncolC) r[P.colC[c].reg] = raw_value(P.colC[c], xrow<S>(P, P.colC[c], row), lc[c]);
  }
#pragma unroll
  for (int k = 0; k < S::arith; ++k) {
    if (k >= P.narith) break;
    const HkArith& A = P.arith[k];
    const uint64_t x = A.xc ? static_cast<uint64_t>(A.cx) : static_cast<uint64_t>(r[A.x]);
    const uint64_t y = A.yc ? static_cast<uint64_t>(A.cy) : static_cast<uint64_t>(r[A.y]);
    const uint64_t v = A.op == HK_ADD ? x + y : (A.op == HK_SUB ? x - y : x * y);
    r[A.dst] = static_cast<long long>(v);
  }
  return pass;
}

// Every column load of a row (all three phases), for rows already known to
// pass: a projection kernel gathers them one block ahead of their use.
template <class S>
struct HkAll {
  HkRaw a[S::colA > 0 ? S::colA : 1], b[S::colB > 0 ? S::colB : 1], c[S::colC > 0 ? S::colC : 1];
};

template <class S>
__device__ __forceinline__ void fetch_all(const HkPlan& P, int64_t row, HkAll<S>& f) {
  // a filter-only column reads row 0 (one line for the whole wave) instead
#pragma unroll
  for (int c = 0; c < S::colA; ++c) load_raw(P.colA[c], xrow<S>(P, P.colA[c], c < P.ncolA && ((P.liveA >> c) & 1u) ? row : 0), f.a[c]);
#pragma unroll
  for (int c = 0; c < S::colB; ++c) load_raw(P.colB[c], xrow<S>(P, P.colB[c], c < P.ncolB ? row : 0), f.b[c]);
#pragma unroll
  for (int c = 0; c < S::colC; ++c) load_raw(P.colC[c], xrow<S>(P, P.colC[c], c < P.ncolC ? row : 0), f.c[c]);
}

// A row known to pass (its filters held and its probes found their keys):
// the registers from the gathered columns, the probes' payloads and the
// arithmetic, without the filters and early exits of eval_row_f.
template <int HT, int HASH, class S>
__device__ __forceinline__ void eval_passing_row(const HkPlan& P, int64_t row, const HkAll<S>& f, v16i64& r) {
#pragma unroll
  for (int c = 0; c < S::colA; ++c)
    if (c < P.ncolA && ((P.liveA >> c) & 1u)) r[P.colA[c].reg] = raw_value(P.colA[c], xrow<S>(P, P.colA[c], row), f.a[c]);
#pragma unroll
  for (int c = 0; c < S::colB; ++c)
    if (c < P.ncolB) r[P.colB[c].reg] = raw_value(P.colB[c], xrow<S>(P, P.colB[c], row), f.b[c]);
#pragma unroll
  for (int p = 0; p < S::probes; ++p) {
    if (p >= P.nprobes) break;
    int32_t pay = 0;
    join_lookup<HT, HASH>(P.probes[p].t, P.hash, static_cast<int32_t>(r[P.probes[p].fk_reg]), pay);
    r[P.probes[p].pay_reg] = pay;
  }
#pragma unroll
  for (int c = 0; c < S::colC; ++c)
    if (c < P.ncolC) r[P.colC[c].reg] = raw_value(P.colC[c], xrow<S>(P, P.colC[c], row), f.c[c]);
#pragma unroll
  for (int k = 0; k < S::arith; ++k) {
    if (k >= P.narith) break;
    const HkArith& A = P.arith[k];
    const uint64_t x = A.xc ? static_cast<uint64_t>(A.cx) : static_cast<uint64_t>(r[A.x]);
    const uint64_t y = A.yc ? static_cast<uint64_t>(A.cy) : static_cast<uint64_t>(r[A.y]);
    const uint64_t v = A.op == HK_ADD ? x + y : (A.op == HK_SUB ? x - y : x * y);
    r[A.dst] = static_cast<long long>(v);
  }
}

template <int PRED, int HT, int HASH, bool VALUES, class S>
__device__ __forceinline__ bool eval_row(const HkPlan& P, int64_t row, v16i64& r) {
  const HkFirst<S> none{};
  return eval_row_f<PRED, HT, HASH, VALUES, S, false>(P, row, none, r);
}

// true when workgroup `wgid` (nwg workgroups of `bs` threads) owns no row of
// n under the row mapping of MEM (uniform over the workgroup: it may leave
// before any barrier)
template <int MEM>
__device__ __forceinline__ bool wg_without_rows(int64_t n, int64_t wgid, int64_t nwg, int64_t bs) {
  const int64_t first = wgid * bs;  // its first thread
  if (MEM == HK_COAL) return first >= n;
  const int64_t T = nwg * bs;
  const int64_t chunk = (n + T - 1) / T;
  return first * chunk >= n;
}

// A spilled row of a plan with one 32-bit group attribute and one input
// value takes 12 bytes: its buffers hold two arrays over their n entries,
// the keys (4 bytes each) and then, from the next 16-byte boundary, the
// values (8 bytes each). Other two-word plans store 16-byte entries
// (ulonglong2, key then value). SpillArr<E> reads and writes entries of
// either form at index i of a buffer (or of an LDS tile) of n entries.
struct HkE12 { uint32_t k; uint64_t v; };
__device__ __forceinline__ uint64_t spill_key(const ulonglong2& e) { return e.x; }
__device__ __forceinline__ uint64_t spill_key(const HkE12& e) { return e.k; }
__device__ __forceinline__ int64_t spill_value(const ulonglong2& e) { return static_cast<int64_t>(e.y); }
__device__ __forceinline__ int64_t spill_value(const HkE12& e) { return static_cast<int64_t>(e.v); }
// LDS bytes of a tile of te spill entries (te a multiple of 4)
template <class E> struct SpillEntryBytes { static constexpr int64_t value = 16; };
template <> struct SpillEntryBytes<HkE12> { static constexpr int64_t value = 12; };
template <class E>
__host__ __device__ constexpr int64_t spill_tile_bytes(int64_t te) {
  return te * SpillEntryBytes<E>::value;
}
template <class E> struct SpillArr;
template <>
struct SpillArr<ulonglong2> {
  ulonglong2* a;
  __device__ SpillArr(void* buf, int64_t, int64_t off) : a(static_cast<ulonglong2*>(buf) + off) {}
  __device__ ulonglong2 get(int64_t i) const { return a[i]; }
  __device__ void put(int64_t i, const ulonglong2& e) const { a[i] = e; }
};
template <>
struct SpillArr<HkE12> {
  uint32_t* k;
  uint64_t* v;
  __device__ SpillArr(void* buf, int64_t n, int64_t off)
      : k(static_cast<uint32_t*>(buf) + off),
        v(reinterpret_cast<uint64_t*>(static_cast<char*>(buf) + (n * 4 + 15) / 16 * 16) + off) {}
  __device__ HkE12 get(int64_t i) const {
    HkE12 e;
    e.k = k[i];
    e.v = v[i];
    return e;
  }
  __device__ void put(int64_t i, const HkE12& e) const {
    k[i] = e.k;
    v[i] = e.v;
  }
};

// first spill entry of workgroup w: the rows scanned by workgroups before it
// (closed form of the coalesced and the sequential row mapping), so regions
// hold exactly the scan's rows in all
__device__ __forceinline__ int64_t spill_region_start(const HkSpill& sp, int64_t nwg, int64_t w) {
  const int64_t bs = sp.bs, T = nwg * bs, n = sp.nrows;
  if (sp.coal) {
    const int64_t K = n / T, rem = n - K * T;
    return w * bs * K + (rem < w * bs ? rem : w * bs);
  }
  const int64_t chunk = (n + T - 1) / T;
  return w * bs * chunk < n ? w * bs * chunk : n;
}

// row range of thread `t` out of `T` for sequential access, chunks rounded to `align`
__device__ __forceinline__ void seq_range(int64_t n, int64_t t, int64_t T, int64_t align, int64_t& b, int64_t& e) {
  int64_t chunk = (n + T - 1) / T;
  chunk = (chunk + align - 1) / align * align;
  b = t * chunk;
  e = b + chunk < n ? b + chunk : n;
  if (b > n) b = n;
}

// ------------------------------------------------------------------ structs passed to kernels


template <class S>
__device__ __forceinline__ void write_proj(const HkPlan& P, const HkOut& O, int64_t pos, const v16i64& r) {
#pragma unroll
  for (int c = 0; c < S::proj; ++c)
    if (c < P.nproj) O.col[c][pos] = r[P.preg[c]];
}

// ------------------------------------------------------------------ aggregation (Section 4.2)
// Global table: AoS slots [key, count, aggregate words...], linear probing or
// cuckoo (keys inserted by k_agg_keys before aggregation). Local strategy:
// each workgroup owns an LDS table of the same word layout (SoA), merged into
// the global table at the end; a row whose key finds no LDS slot within the
// probe bound goes straight to the global table.

// WGS: the caller's workgroup owns the key's region for the whole kernel, so
// workgroup-scope atomics suffice (performed in this XCD's L2)
template <int HASH, bool WGS = false>
__device__ __forceinline__ uint64_t* gslot_linear(const HkAggTable& T, const HkHash& h, uint64_t key, int* err) {
  const int64_t W = T.slot_words;
  if (key == HK_EMPTY) return T.words + (static_cast<int64_t>(1) << T.log2cap) * W;  // side slot
  const uint32_t rmask = (1u << T.rlog2) - 1u;
  uint32_t s = hslot<HASH>(key, h.a[0], T.log2cap);
  const uint32_t base = s & ~rmask;
  for (uint32_t i = 0; i <= rmask; ++i) {
    uint64_t* p = T.words + static_cast<int64_t>(s) * W;
    uint64_t cur = *p;
    if (cur == key) return p;
    if (cur == HK_EMPTY) {
      cur = at_cas<WGS>(p, HK_EMPTY, key);
      if (cur == HK_EMPTY || cur == key) return p;
    }
    s = base | ((s + 1) & rmask);
  }
  set_err(err, HK_ERR_CAPACITY);
  return nullptr;
}

template <int HASH>
__device__ __forceinline__ uint64_t* gslot_cuckoo(const HkAggTable& T, const HkHash& h, uint64_t key, int* err) {
  const int64_t W = T.slot_words;
  if (key == HK_EMPTY) return T.words + (static_cast<int64_t>(1) << T.log2cap) * W;
#pragma unroll
  for (int i = 0; i < HK_CUCKOO_D; ++i) {
    uint64_t* p = T.words + static_cast<int64_t>(hslot<HASH>(key, h.a[i], T.log2cap)) * W;
    if (*p == key) return p;
  }
  set_err(err, HK_ERR_CUCKOO);
  return nullptr;
}

template <int HT, int HASH>
__device__ __forceinline__ uint64_t* gslot(const HkAggTable& T, const HkHash& h, uint64_t key, int* err) {
  if (HT == HK_LIN) return gslot_linear<HASH>(T, h, key, err);
  return gslot_cuckoo<HASH>(T, h, key, err);
}

// cuckoo phase 1: key insertion with evictions (no aggregates yet)
template <int HASH>
__device__ __forceinline__ void gkey_cuckoo_insert(const HkAggTable& T, const HkHash& h, uint64_t key, int* err) {
  if (key == HK_EMPTY) return;
  const int64_t W = T.slot_words;
#pragma unroll
  for (int i = 0; i < HK_CUCKOO_D; ++i)
    if (T.words[static_cast<int64_t>(hslot<HASH>(key, h.a[i], T.log2cap)) * W] == key) return;
  uint64_t cur = key;
  int i = 0;
  for (int step = 0; step < HK_CUCKOO_MAX_EVICT; ++step) {
    const uint32_t s = hslot<HASH>(cur, h.a[i], T.log2cap);
    const uint64_t old = at_xchg(T.words + static_cast<int64_t>(s) * W, cur);
    if (old == HK_EMPTY || old == cur) return;
    cur = old;
    int j = 0;
#pragma unroll
    for (int jj = HK_CUCKOO_D - 1; jj >= 0; --jj)
      if (hslot<HASH>(old, h.a[jj], T.log2cap) == s) j = jj;
    i = (j + 1) % HK_CUCKOO_D;
  }
  set_err(err, HK_ERR_CUCKOO);
}

// group key of the row: one or two 32-bit attributes packed into 64 bits
__device__ __forceinline__ uint64_t group_key(const HkPlan& P, const v16i64& r) {
  if (P.ngroup == 0) return 0ull;
  const uint64_t g0 = static_cast<uint32_t>(static_cast<int32_t>(r[P.greg[0]]));
  if (P.ngroup == 1) return g0;
  return (g0 << 32) | static_cast<uint32_t>(static_cast<int32_t>(r[P.greg[1]]));
}

// applies one row to the slot whose word j >= 1 (count, aggregates) lives at
// w1[(j - 1) * stride]
template <int PRED, bool LDS, class S>
__device__ __forceinline__ void agg_apply_w1(uint64_t* w1, int64_t stride, const HkPlan& P, const v16i64& r, bool pass) {
  at_add<LDS>(w1, PRED == HK_PRED ? static_cast<uint64_t>(pass) : 1ull);
#pragma unroll
  for (int a = 0; a < S::aggs; ++a) {
    if (a >= P.naggs) break;
    const HkAgg& A = P.aggs[a];
    if (A.fn == HK_COUNT) continue;
    const int64_t x = r[A.reg];
    uint64_t* w = w1 + (A.word - 1) * stride;
    if (A.fn == HK_SUM || A.fn == HK_AVG) {
      // software predication: a dropped row contributes 0 (x * result_increment)
      const int64_t v = PRED == HK_PRED ? (pass ? x : 0) : x;
      if (A.wide) at_add128<LDS>(w, w + stride, v);
      else at_add<LDS>(w, static_cast<uint64_t>(v));
    } else if (A.fn == HK_MIN) {
      at_min<LDS>(w, PRED == HK_PRED ? (pass ? x : INT64_MAX) : x);
    } else {
      at_max<LDS>(w, PRED == HK_PRED ? (pass ? x : INT64_MIN) : x);
    }
  }
}

// applies one row to the slot whose word j lives at base[j * stride]
template <int PRED, bool LDS, class S>
__device__ __forceinline__ void agg_apply(uint64_t* base, int64_t stride, const HkPlan& P, const v16i64& r, bool pass) {
  agg_apply_w1<PRED, LDS, S>(base + stride, stride, P, r, pass);
}

// folds the words j >= 1 of slot copy b (word j at b[(j - 1) * stride]) into
// copy a (same layout); both belong to the calling thread
template <class S>
__device__ __forceinline__ void agg_fold_w1(uint64_t* a, const uint64_t* b, int64_t stride, const HkPlan& P) {
  a[0] += b[0];
#pragma unroll
  for (int k = 0; k < S::aggs; ++k) {
    if (k >= P.naggs) break;
    const HkAgg& A = P.aggs[k];
    if (A.fn == HK_COUNT) continue;
    uint64_t* x = a + (A.word - 1) * stride;
    const uint64_t y = b[(A.word - 1) * stride];
    if (A.fn == HK_SUM || A.fn == HK_AVG) {
      if (A.wide) {
        const uint64_t lo = *x + y;
        x[stride] += b[A.word * stride] + static_cast<uint64_t>(lo < y);
        *x = lo;
      } else {
        *x += y;
      }
    } else if (A.fn == HK_MIN) {
      *x = static_cast<int64_t>(y) < static_cast<int64_t>(*x) ? y : *x;
    } else {
      *x = static_cast<int64_t>(y) > static_cast<int64_t>(*x) ? y : *x;
    }
  }
}

// merges a slot's count and aggregate words (word j >= 1 at l1[(j - 1) * stride])
// into slot d (word j at d[j * ds]); WGS: workgroup-scope atomics (LDS)
template <bool WGS, class S>
__device__ __forceinline__ void agg_merge_into(uint64_t* d, int64_t ds, const uint64_t* l1, int64_t stride,
                                               const HkPlan& P) {
  at_add<WGS>(d + ds, l1[0]);
#pragma unroll
  for (int a = 0; a < S::aggs; ++a) {
    if (a >= P.naggs) break;
    const HkAgg& A = P.aggs[a];
    if (A.fn == HK_COUNT) continue;
    const uint64_t x = l1[(A.word - 1) * stride];
    uint64_t* y = d + A.word * ds;
    if (A.fn == HK_SUM || A.fn == HK_AVG) {
      if (A.wide) at_add128_pair<WGS>(y, y + ds, x, static_cast<int64_t>(l1[A.word * stride]));
      else at_add<WGS>(y, x);
    } else if (A.fn == HK_MIN) {
      at_min<WGS>(y, static_cast<int64_t>(x));
    } else {
      at_max<WGS>(y, static_cast<int64_t>(x));
    }
  }
}

// merges an LDS slot (word j >= 1 at l1[(j - 1) * stride]) into a global slot g
template <class S>
__device__ __forceinline__ void agg_merge_w1(uint64_t* g, const uint64_t* l1, int64_t stride, const HkPlan& P) {
  agg_merge_into<false, S>(g, 1, l1, stride, P);
}

// exclusive prefix sum of a[0..n) (LDS) in place by the whole workgroup; the
// prefixes also go to out[0..n), the total to out[n]. wave_tot: LDS words,
// one per wave of the workgroup. Ends with a barrier.
__device__ __forceinline__ void wg_exclusive_scan(uint32_t* a, int n, uint32_t* out, uint32_t* wave_tot) {
  const int bs = blockDim.x, t = threadIdx.x;
  const int K = (n + bs - 1) / bs;
  const int b = t * K < n ? t * K : n;
  const int e = b + K < n ? b + K : n;
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += a[i];
  const int lane = __lane_id();
  uint32_t x = sum;  // inclusive scan of the chunk sums within the wave
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, WAVE);
    if (lane >= d) x += y;
  }
  const int wv = t / WAVE;
  if (lane == WAVE - 1 || t == bs - 1) wave_tot[wv] = x;
  __syncthreads();
  uint32_t run = x - sum;
  for (int j = 0; j < wv; ++j) run += wave_tot[j];
  for (int i = b; i < e; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    out[i] = run;
    run += v;
  }
  if (t == bs - 1) out[n] = run;  // the last thread's chunk ends at n
  __syncthreads();
}

// merges an LDS slot (word j at l[j * stride]) into a global slot g
template <class S>
__device__ __forceinline__ void agg_merge(uint64_t* g, const uint64_t* l, int64_t stride, const HkPlan& P) {
  agg_merge_w1<S>(g, l + stride, stride, P);
}

// Admission filter of the local table (`door`: 2^dl2 bits in LDS): a key
// that would take an empty slot enters only if its bit was already set, so a
// key seen once by the workgroup leaves the slots to keys seen again. Sets
// the bit; true when the key may enter.
template <int HASH>
__device__ __forceinline__ bool door_admits(uint32_t* door, uint32_t dl2, const HkHash& h, uint64_t key) {
  const uint32_t b = hslot<HASH>(key, h.a[1], dl2);
  const uint32_t m = 1u << (b & 31u);
  return (atomicOr(&door[b >> 5], m) & m) != 0u;
}

// LDS slot lookup/insert for the local strategy; -1 = no slot within bound
// (or, with a filter, a key not admitted yet).
// Linear probing reads the table four slots at a time: the hash picks an
// aligned group of four slots whose first is the key's home slot, probing
// goes on slot by slot from there into the next group, and one 32-byte read
// brings a whole group's keys. A slot only ever changes from empty to a key,
// so the first slot of a group read that holds the key is the key's slot,
// and an insertion takes the first empty slot in probe order by
// compare-and-swap (re-reading the group when another key took it first).
template <int HT, int HASH, bool ADMIT = false>
__device__ __forceinline__ int32_t lslot(uint64_t* lkeys, uint32_t llog2, const HkHash& h, uint64_t key,
                                         uint32_t* door = nullptr, uint32_t dl2 = 0) {
  if (HT == HK_LIN) {
    const uint32_t mask = (1u << llog2) - 1u;
    uint32_t g = hslot<HASH>(key, h.a[0], llog2 - 2) << 2;
    // admission decided at the first empty slot met, then kept
    int adm = (ADMIT && dl2 > 0) ? -1 : 1;
#pragma unroll
    for (int k = 0; k < HK_LOCAL_PROBES / 4; ++k) {
      for (int tries = 0; tries < 5; ++tries) {  // each failed compare-and-swap fills one slot of the group
        const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(lkeys + g);
        const ulonglong2 y = *reinterpret_cast<const ulonglong2*>(lkeys + g + 2);
        int hit = 4;
        hit = y.y == key ? 3 : hit;
        hit = y.x == key ? 2 : hit;
        hit = x.y == key ? 1 : hit;
        hit = x.x == key ? 0 : hit;
        if (hit < 4) return static_cast<int32_t>(g + hit);
        int e = 4;
        e = y.y == HK_EMPTY ? 3 : e;
        e = y.x == HK_EMPTY ? 2 : e;
        e = x.y == HK_EMPTY ? 1 : e;
        e = x.x == HK_EMPTY ? 0 : e;
        if (e == 4) break;  // a full group without the key: the next group
        if (adm < 0) adm = door_admits<HASH>(door, dl2, h, key) ? 1 : 0;
        if (!adm) return -1;
        const uint64_t cur = at_cas<true>(&lkeys[g + e], HK_EMPTY, key);
        if (cur == HK_EMPTY || cur == key) return static_cast<int32_t>(g + e);
      }
      g = (g + 4) & mask;
    }
    return -1;
  } else {
    // cuckoo placement without eviction: the first free or matching choice
#pragma unroll
    for (int i = 0; i < HK_CUCKOO_D; ++i) {
      const uint32_t s = hslot<HASH>(key, h.a[i], llog2);
      uint64_t cur = lkeys[s];
      if (cur == key) return static_cast<int32_t>(s);
      if (cur == HK_EMPTY) {
        cur = at_cas<true>(&lkeys[s], HK_EMPTY, key);
        if (cur == HK_EMPTY || cur == key) return static_cast<int32_t>(s);
      }
    }
    return -1;
  }
}


__device__ __forceinline__ double i128_to_f64(uint64_t lo, int64_t hi) {
  const int64_t slo = static_cast<int64_t>(lo);
  if ((hi == 0 && slo >= 0) || (hi == -1 && slo < 0)) return static_cast<double>(slo);
  return static_cast<double>(hi) * 18446744073709551616.0 + static_cast<double>(lo);
}


// writes the group row of slot words p (key, count, aggregates) at row pos of the result columns
// result row `pos` from a slot whose word j is at p[j * ws]
__device__ __forceinline__ void write_group_row_s(const HkPlan& P, const uint64_t* p, int64_t ws, int64_t pos,
                                                  const HkResOut& O) {
  const uint64_t key = p[0];  // the side slot keeps the all-ones key
  if (P.ngroup == 1) O.gcol[0][pos] = static_cast<int32_t>(static_cast<uint32_t>(key));
  if (P.ngroup == 2) {
    O.gcol[0][pos] = static_cast<int32_t>(static_cast<uint32_t>(key >> 32));
    O.gcol[1][pos] = static_cast<int32_t>(static_cast<uint32_t>(key));
  }
  const uint64_t cnt = p[ws];
  O.count[pos] = static_cast<int64_t>(cnt);
  for (int a = 0; a < P.naggs; ++a) {
    const HkAgg& A = P.aggs[a];
    if (A.fn == HK_COUNT) {
      static_cast<int64_t*>(O.acol[a])[pos] = static_cast<int64_t>(cnt);
    } else if (A.fn == HK_AVG) {
      const double sum = A.wide ? i128_to_f64(p[A.word * ws], static_cast<int64_t>(p[(A.word + 1) * ws]))
                                : static_cast<double>(static_cast<int64_t>(p[A.word * ws]));
      static_cast<double*>(O.acol[a])[pos] = sum / static_cast<double>(cnt);
    } else if (A.fn == HK_SUM && A.wide) {
      static_cast<uint64_t*>(O.acol[a])[2 * pos] = p[A.word * ws];
      static_cast<uint64_t*>(O.acol[a])[2 * pos + 1] = p[(A.word + 1) * ws];
    } else {
      static_cast<int64_t*>(O.acol[a])[pos] = static_cast<int64_t>(p[A.word * ws]);
    }
  }
}

__device__ __forceinline__ void write_group_row(const HkPlan& P, const uint64_t* p, int64_t pos, const HkResOut& O) {
  write_group_row_s(P, p, 1, pos, O);
}

// ------------------------------------------------------------------ host-side launch helpers
#ifndef __HIPCC_RTC__
#define DISPATCH2(v, NAME, ...) \
  do {                          \
    if (v) {                    \
      constexpr int NAME = 1;   \
      __VA_ARGS__;              \
    } else {                    \
      constexpr int NAME = 0;   \
      __VA_ARGS__;              \
    }                           \
  } while (0)

// grid of `nwg` workgroups: 1-D up to 65536, else 2-D (x = 65536); the kernel
// linearises blockIdx and lets workgroups past nwg leave at once
static inline dim3 hk_wg_grid(int64_t nwg) {
  if (nwg <= 65536) return dim3(static_cast<uint32_t>(nwg));
  return dim3(65536u, static_cast<uint32_t>((nwg + 65535) / 65536));
}

static inline int64_t hk_grid_for(int64_t work, int64_t block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  return g < cap ? g : cap;
}
#endif  // __HIPCC_RTC__
