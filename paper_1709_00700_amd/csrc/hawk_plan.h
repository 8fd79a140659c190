// Internal plan representation shared by the host dispatcher and the gfx950
// kernels. A validated pipeline program (Section 3.1) is lowered into a
// fixed-size, by-value kernel argument: column loads into a 16-entry register
// file of 64-bit values, filter predicates, probe descriptors, arithmetic
// steps and the sink (projection or aggregation). Every variant dimension of
// Section 9.2 is a template parameter of the kernels; everything the query
// itself decides is data in this struct.
#pragma once
#ifndef __HIPCC_RTC__
#include <stdint.h>
#else
// compiled at run time (hipRTC): fixed-width types come from the runtime's own header
typedef __hip_internal::int8_t int8_t;
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int16_t int16_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
#ifndef INT64_MAX
#define INT64_MAX 9223372036854775807LL
#define INT64_MIN (-INT64_MAX - 1)
#endif
#endif

#define HK_NREG 16
#define HK_MAX_COLS_A 6          // columns loaded before the filters
#define HK_MAX_COLS_B 4          // join-key columns loaded before the probes
#define HK_MAX_COLS_C 8          // value columns loaded before the arithmetic
#define HK_MAX_FILTERS 6
#define HK_MAX_PROBES 4
#define HK_MAX_ARITH 8
#define HK_MAX_AGGS 8
#define HK_MAX_PROJ 4
#define HK_CUCKOO_D 3            // number of hash functions of the cuckoo table
#define HK_CUCKOO_MAX_EVICT 64   // eviction chain bound before the insert fails
#define HK_LOCAL_PROBES 8        // LDS linear probing bound before a row overflows to the global table

#define HK_EMPTY 0xFFFFFFFFFFFFFFFFull

enum { HK_SEQ = 0, HK_COAL = 1 };
enum { HK_BR = 0, HK_PRED = 1 };
enum { HK_LIN = 0, HK_CUCKOO = 1 };
#define HK_ROBIN_MAX_DISP 4096   // displacement bound of a robin-hood insertion before it fails
enum { HK_MURMUR = 0, HK_MULSHIFT = 1 };
enum { HK_LOCAL = 0, HK_GLOBAL = 1 };

enum { HK_T_I8 = 1, HK_T_I32 = 2, HK_T_I64 = 3 };
enum { HK_ADD = 1, HK_SUB = 2, HK_MUL = 3 };
enum { HK_COUNT = 1, HK_SUM = 2, HK_MIN = 3, HK_MAX = 4, HK_AVG = 5 };

// error flag bits written by kernels
// (HK_ERR_TIMEOUT: a bounded wait for another workgroup's result gave up)
enum { HK_ERR_CAPACITY = 1, HK_ERR_DUPKEY = 2, HK_ERR_CUCKOO = 4, HK_ERR_TIMEOUT = 8 };

// a column load into register `reg`; side: 0 = the looped table's row,
// with a CROSS_JOIN 1 = its row of the looped table, 2 = its row of the second table
struct HkCol { const void* ptr; int16_t dtype; int16_t side; int32_t reg; };
struct HkFilter { int64_t lo, hi; int32_t reg; int32_t pad; };
// hash functions of one query: murmur xor keys or multiply-shift odd multipliers
struct HkHash { uint64_t a[HK_CUCKOO_D]; };
// a join hash table: 64-bit slots (key << 32 | payload), plus side words:
// side[0] holds key -1, side[1] (robin hood) the largest displacement of any
// entry; robin = 1: robin-hood linear probing (kernels instantiated for
// linear probing take this form at run time)
struct HkJoinTable { uint64_t* slots; uint64_t* side; uint32_t log2cap; int32_t robin; };
struct HkProbe { HkJoinTable t; int32_t fk_reg; int32_t pay_reg; };
struct HkArith { int64_t cx, cy; int8_t op, dst, x, y, xc, yc, pad0, pad1; };
struct HkAgg { int8_t fn, wide, reg, pad; int32_t word; };

struct HkPlan {
  int64_t nrows;
  HkHash hash;
  // column loads into registers: colA before the filters, colB (join keys)
  // before the probes, colC before the arithmetic
  int32_t ncolA, ncolB, ncolC, nfilters;
  HkCol colA[HK_MAX_COLS_A];
  HkCol colB[HK_MAX_COLS_B];
  HkCol colC[HK_MAX_COLS_C];
  HkFilter filters[HK_MAX_FILTERS];
  int32_t nprobes, narith, ngroup, naggs;
  HkProbe probes[HK_MAX_PROBES];
  HkArith arith[HK_MAX_ARITH];
  int32_t greg[2];
  HkAgg aggs[HK_MAX_AGGS];
  int32_t nproj;
  int32_t preg[HK_MAX_PROJ];
  // aggregation table: AoS slots of slot_words 64-bit words:
  // [key, count, aggregate words...]; wide sums take two words (lo, hi)
  int32_t slot_words;
  // bit c: colA[c] is read after the filters (a column that only a filter
  // reads is not loaded again for rows already known to pass)
  uint32_t liveA;
  // CROSS_JOIN (Table 1): xinner > 0 rows of a second table; nrows is then the
  // product and row v stands for row v / xinner of the looped table and row
  // v % xinner of the second (xmagic = 2^64 / xinner rounded up: the quotient
  // of a 32-bit v is the high word of xmagic * v)
  uint32_t xinner;
  uint64_t xmagic;
};

// a build pipeline (LOOP, FILTER, HASH_PUT): filter part, key and payload columns, target table
struct HkBuild {
  HkPlan p;              // LOOP + FILTER part (colA filter columns), nrows, hash functions
  HkCol key, payload;
  HkJoinTable t;
};

// Shape classes: compile-time bounds of the per-row loops. A kernel
// instantiated for a class touches only the plan fields that class can use,
// so those fields stay in scalar registers for the whole row loop. The
// dispatcher picks the smallest class that holds the plan (hk_shape_of).
template <int A, int F, int B, int PR, int C, int AR, int AG, int PJ, int X = 0>
struct HkShape {
  static constexpr int colA = A, filters = F, colB = B, probes = PR, colC = C, arith = AR, aggs = AG, proj = PJ;
  static constexpr int cross = X;  // 1: handles plans with a CROSS_JOIN
};
using HkShapeA = HkShape<0, 0, 0, 0, 2, 0, 4, 0>;   // group-aggregate of value columns (no filters, joins, arithmetic)
using HkShapeF = HkShape<2, 2, 0, 0, 3, 2, 4, 2>;   // filters, a little arithmetic, projection or aggregation
using HkShapeJ = HkShape<0, 0, 4, 4, 1, 0, 2, 2>;   // joins: up to 4 probes
using HkShapeW = HkShape<0, 0, 0, 0, 6, 4, 8, 2>;   // wide: many value columns, arithmetic steps, aggregates
using HkShapeG = HkShape<HK_MAX_COLS_A, HK_MAX_FILTERS, HK_MAX_COLS_B, HK_MAX_PROBES, HK_MAX_COLS_C, HK_MAX_ARITH,
                         HK_MAX_AGGS, HK_MAX_PROJ, 1>;   // anything the plan format allows, CROSS_JOIN included
enum { HK_SHAPE_A = 0, HK_SHAPE_F = 1, HK_SHAPE_J = 2, HK_SHAPE_W = 3, HK_SHAPE_G = 4 };

template <class S>
inline bool hk_fits(const HkPlan& P) {
  return P.ncolA <= S::colA && P.nfilters <= S::filters && P.ncolB <= S::colB && P.nprobes <= S::probes &&
         P.ncolC <= S::colC && P.narith <= S::arith && P.naggs <= S::aggs && P.nproj <= S::proj;
}
inline int hk_shape_of(const HkPlan& P) {
  if (P.xinner > 0) return HK_SHAPE_G;
  if (hk_fits<HkShapeA>(P)) return HK_SHAPE_A;
  if (hk_fits<HkShapeF>(P)) return HK_SHAPE_F;
  if (hk_fits<HkShapeJ>(P)) return HK_SHAPE_J;
  if (hk_fits<HkShapeW>(P)) return HK_SHAPE_W;
  return HK_SHAPE_G;
}

// identity words of an aggregation slot [key, count, aggregates...]
struct HkIdent { uint64_t w[2 + 2 * HK_MAX_AGGS]; int32_t nw; };
// projection outputs (int64 per projected attribute) and the dump slot
struct HkOut { int64_t* col[HK_MAX_PROJ]; int64_t dump; };
// aggregation result columns
struct HkResOut {
  int64_t* gcol[2];
  void* acol[HK_MAX_AGGS];
  int64_t* count;
  unsigned long long* nrows;
  int32_t keep_empty;  // AGGREGATE without groups keeps its single row
};

// an aggregation hash table in HBM (plus one side slot for the sentinel key);
// linear probing stays inside the aligned region of 2^rlog2 slots that holds
// the key's hash slot (rlog2 == log2cap: the whole table is one region)
struct HkAggTable { uint64_t* words; uint32_t log2cap; int32_t slot_words; uint32_t rlog2; int32_t pad; };

// Overflow partitioning of the local strategy. A row whose key finds no slot
// in its workgroup's LDS table is appended to the workgroup's spill region as
// an entry [key, input values...]; the entries are then regrouped by table
// region (partition = hash slot >> rlog2) and each region is aggregated by
// the one workgroup that owns it. The LDS tables themselves either reach the
// owners too, each workgroup writing its slots out as merge entries [key,
// count, aggregate words...] sorted by region (merge = 1: no slot touches the
// table with device-scope atomics), or merge into the table with device-scope
// atomics before the owners start from it (merge = 0).
struct HkSpill {
  uint64_t* buf;              // one region per workgroup, as many entries as rows it scans (nrows in all)
  int64_t nrows;              // rows of the scan
  int32_t bs;                 // threads per workgroup
  int32_t coal;               // row mapping: 1 coalesced (thread-strided), 0 sequential (chunks)
  uint32_t* hist;             // entry counts per (partition, workgroup), partition-major
  uint32_t* cnt;              // entries per workgroup
  int32_t nparts;             // table regions: 2^(log2cap - rlog2)
  int32_t ncols;              // input values per entry
  int32_t ew;                 // words per entry: 1 + ncols
  int32_t reg[HK_MAX_AGGS];   // register of each input value
  uint64_t* flush;            // merge entries: fcap slots of slot_words words per workgroup
  uint32_t* foffs;            // per workgroup nparts + 1 offsets of its merge entries by region
  int32_t fcap;               // merge entries per workgroup, at most (its LDS table's slots)
  int32_t merge;              // 1: LDS tables leave as merge entries; 0: they merge into the table with device-scope atomics
  int32_t door_log2;          // > 0: a key enters the LDS table at its second miss (a 2^door_log2-bit filter in LDS)
  int32_t e12;                // 1: 12-byte entries (32-bit key, one 64-bit value; ew == 2), else ew words
};
