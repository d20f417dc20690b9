// Work-balanced worst-case-optimal join kernels for gfx950.
//
// A rule version is joined attribute at a time (paper Sec. 2, "Join
// Processing"): the variables x_0..x_{m-1} are bound in a fixed order, and the
// candidates for x_L are the values of one source atom's column inside its
// current row range, each kept only if every other atom constraining x_L
// holds it too (a leapfrog-style seek by binary search inside that atom's
// range).  Binding a value narrows every constraining atom to the contiguous
// rows that share the bound prefix (Sec. 4, flat sorted columns).
//
// Work balance follows Sec. 5 (Alg. 1 and Alg. 2): the histogram kernel
// gives every distinct root key k its work W[k] (the number of level-1
// candidates under it; for cross-product plans the product of the fan-outs),
// an inclusive prefix sum C flattens all work into [0, T), and workgroup b
// owns units [b*ceil(T/p), (b+1)*ceil(T/p)).  A heavy key is thereby split
// across workgroups.  Inside a workgroup, the deeper levels are expanded
// breadth-first in chunks of 256 candidates held in LDS buffers (one per
// level) and drained depth-first, so each lane checks one candidate at a
// time whatever the fan-out of the item it came from; this is the
// wavefront-cooperative form of the inner intersection on this GPU.
//
// Count and materialize run the same traversal (Sec. 4, two-phase
// deterministic allocation): count writes one total per workgroup, an
// exclusive scan turns totals into offsets, and materialize writes every
// workgroup's rows at its offset in traversal order, so the output is
// deterministic and, in variable order, lexicographically sorted.

#include <algorithm>
#include <functional>

#include "wcdl_internal.h"

namespace wcdl {
namespace {

constexpr int WG = 256;
constexpr int LEAF_K = 2;  // leaf candidates per lane and step
static_assert(LEAF_K * WG == (int)EMIT_ROWS, "the planner sizes the survivor buffer");
constexpr int XP_RPT = 8;                         // cross-product rows per thread
constexpr u32 XP_ROWS = (u32)WG * XP_RPT;         // rows per cross-product workgroup
constexpr u32 XP_KEYS = 1024;                     // root keys cached per workgroup
constexpr u32 UMAX = 0xffffffffu;

// Reads of device columns through the global address space.  The column
// pointers come out of the plan structure, so the compiler would otherwise
// emit flat loads, which share the LDS wait counter: every LDS read would
// then also wait for all outstanding column reads.
typedef const u32 __attribute__((address_space(1))) gu32;
typedef const u64 __attribute__((address_space(1))) gu64;
__device__ inline u32 ldg(const u32* p) { return *(gu32*)p; }
__device__ inline u64 ldg(const u64* p) { return *(gu64*)p; }

// Wave-uniform copies of values the compiler cannot prove uniform (they come
// from LDS), so that plan fields indexed by them are read with scalar loads.
__device__ inline u32 uni(u32 x) { return (u32)__builtin_amdgcn_readfirstlane((int)x); }
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline u64 uni(u64 x) { return ((u64)uni((u32)(x >> 32)) << 32) | uni((u32)x); }

__device__ inline u32 lower_bound_u32(const u32* col, u32 lo, u32 hi, u32 v) {
  while (lo < hi) {
    u32 mid = lo + ((hi - lo) >> 1);
    if (ldg(col + mid) < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ inline u32 upper_bound_u32(const u32* col, u32 lo, u32 hi, u32 v) {
  while (lo < hi) {
    u32 mid = lo + ((hi - lo) >> 1);
    if (ldg(col + mid) <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First index >= lo in [lo, hi) with col > v, by galloping from lo (runs of
// equal values are usually short).
__device__ inline u32 gallop_past(const u32* col, u32 lo, u32 hi, u32 v) {
  u32 a = lo;
  u64 b = lo, step = 1;
  while (b < hi && ldg(col + b) <= v) {
    a = (u32)b + 1;
    b = (u64)a + step;
    step <<= 1;
  }
  return upper_bound_u32(col, a, b < hi ? (u32)b : hi, v);
}

// Eight values held in named registers.  A plain array indexed with a lane-
// varying index would be moved to scratch memory; selecting among named
// scalars keeps everything in VGPRs.
struct R8 {
  u32 x0, x1, x2, x3, x4, x5, x6, x7;
  __device__ void put(int s, u32 v) {  // s is a compile-time constant after unrolling
    switch (s) {
      case 0: x0 = v; break;
      case 1: x1 = v; break;
      case 2: x2 = v; break;
      case 3: x3 = v; break;
      case 4: x4 = v; break;
      case 5: x5 = v; break;
      case 6: x6 = v; break;
      default: x7 = v; break;
    }
  }
  __device__ u32 get(u32 i) const {
    // Bit masks rather than selects, so the choice stays arithmetic on
    // registers instead of becoming an address computation.
    return (x0 & (0u - (u32)(i == 0))) | (x1 & (0u - (u32)(i == 1))) |
           (x2 & (0u - (u32)(i == 2))) | (x3 & (0u - (u32)(i == 3))) |
           (x4 & (0u - (u32)(i == 4))) | (x5 & (0u - (u32)(i == 5))) |
           (x6 & (0u - (u32)(i == 6))) | (x7 & (0u - (u32)(i == 7)));
  }
};
static_assert(MAXS == 8, "R8 holds one value per source");

__device__ inline u64 shfl_up_u64(u64 x, int d) {
  u32 lo = __shfl_up((u32)x, d, 64);
  u32 hi = __shfl_up((u32)(x >> 32), d, 64);
  return ((u64)hi << 32) | lo;
}

__device__ inline u64 wave_incl_scan(u64 x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    u64 y = shfl_up_u64(x, d);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ inline u64 block_excl_scan(u64 x, u64* sh, u64* total) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  u64 inc = wave_incl_scan(x);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  u64 off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WG / 64; ++i) {
    u64 s = sh[i];
    if (i < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - x;
}

// View of the level buffers for one workgroup.
struct Bufs {
  u32* sm;
  const DPlan* P;
  const u32* rng0;  // [2*MAXN] in LDS
  __device__ u32 lo(int b, u32 a, u32 i) const {
    const u32 s = b < 0 ? NONE : P->atom_slot[b][a];
    return s == NONE ? rng0[2 * a] : sm[P->off_lo[b] + s * P->cap + i];
  }
  __device__ u32 hi(int b, u32 a, u32 i) const {
    const u32 s = b < 0 ? NONE : P->atom_slot[b][a];
    return s == NONE ? rng0[2 * a + 1] : sm[P->off_hi[b] + s * P->cap + i];
  }
  __device__ u32 val(int b, u32 k, u32 i) const { return sm[P->off_val[b] + k * P->cap + i]; }
};

// Value of an operand while binding level L from parent item i of buffer L-1.
__device__ inline u32 operand(const Bufs& B, const DOperand& o, int L, u32 i, u32 v) {
  if (!o.is_var) return o.v;
  if ((int)o.v == L) return v;
  return B.val(L - 1, o.v, i);
}

// Stratified negation: true if no row of the negated atom's relation equals
// its operands under the current binding (level L bound to v).  The copy is
// sorted in the atom's search order, so each bound column narrows a range.
__device__ inline bool neg_absent(const DNeg& ng, const Bufs& B, int L, u32 i, u32 v) {
  u32 lo = 0, hi = ng.n;
  for (u32 j = 0; j < ng.ncols; ++j) {
    const u32 x = operand(B, ng.val[j], L, i, v);
    const u32 l2 = lower_bound_u32(ng.col[j], lo, hi, x);
    hi = upper_bound_u32(ng.col[j], l2, hi, x);
    lo = l2;
  }
  return lo >= hi;
}

// Column of source s of a level (s varies per lane; the level does not).
// The pointers are read as wave-uniform values and selected in registers; a
// per-lane indexed read of the plan would put a dependent memory access in
// front of every column read.
__device__ inline const u32* source_col(const DLevel& lv, u32 s) {
  const u32 n = uni(lv.nsrc);
  const u32* c0 = (const u32*)uni((u64)lv.src[0].col);
  const u32* c1 = n > 1 ? (const u32*)uni((u64)lv.src[1].col) : c0;
  const u32* col = s == 1 ? c1 : c0;
  for (u32 t = 2; t < n; ++t) {
    const u32* c = (const u32*)uni((u64)lv.src[t].col);
    if (s == t) col = c;
  }
  return col;
}

// Run bitmaps of source s of a level (s varies per lane; the level does not),
// selected among the sources' wave-uniform fields.
__device__ inline void source_bitmaps(const DLevel& lv, u32 s, const u32** bm_at, const u32** bm,
                                      u32* words, u32* bmin) {
  const u32 n = uni(lv.nsrc);
  *bm_at = nullptr;
  *bm = nullptr;
  *words = 0;
  *bmin = 0;
  for (u32 t = 0; t < n; ++t) {
    const u32* a = (const u32*)uni((u64)lv.src[t].bm_at);
    const u32* b = (const u32*)uni((u64)lv.src[t].bm);
    const u32 w = uni(lv.src[t].bm_words), m = uni(lv.src[t].bm_min);
    if (s == t) {
      *bm_at = a;
      *bm = b;
      *words = w;
      *bmin = m;
    }
  }
}

// Item of a level buffer owning candidate g: the first i with pre[i] > g,
// pre being the inclusive prefix of the items' candidate counts (g < pre[n-1]).
// The number of steps depends on n only.
__device__ inline u32 owner_item(const u64* pre, u32 n, u64 g) {
  u32 base = 0;
  while (n > 1) {
    const u32 half = n >> 1;
    base = pre[base + half] <= g ? base + half : base;
    n -= half;
  }
  return base + (pre[base] <= g ? 1u : 0u);
}

// Candidate v for level L (from parent item i, or the root when L == 0):
// the driver source `drv` supplies it at row r (its run of equal values ends
// at dhi if known, else NONE); every other source of the level must contain
// v inside its current range.  On success slo/shi hold each source's
// narrowed range.
__device__ inline bool try_candidate(const DPlan* P, const Bufs& B, int L, u32 i, u32 v, u32 drv,
                                     u32 r, u32 dhi, R8& slo, R8& shi) {
  // A per-lane flag instead of early returns: a lane-divergent return inside
  // a loop whose trip count comes from the plan has been seen to be skipped
  // on this target, so every test below clears `ok` and later work is
  // guarded by it.
  const DLevel& lv = P->lvl[L];
  u32 ok = 1;
  for (u32 f = 0; f < lv.nne; ++f) ok &= v != operand(B, lv.ne[f], L, i, v) ? 1u : 0u;
  if (L == 0) {
    // An atom without matches under its constants empties the rule.
    for (u32 a = 0; a < P->natoms; ++a) ok &= B.rng0[2 * a] < B.rng0[2 * a + 1] ? 1u : 0u;
    // Level-0 values come straight from the root keys, so their bounds
    // (constants only) are checked here; deeper levels clip candidate
    // ranges to their bounds instead (prepare_item).
    for (u32 b = 0; b < lv.nbnd; ++b) {
      const u32 x = lv.bnd[b].o.v, adj = lv.bnd[b].adj;
      if (!lv.bnd[b].is_hi)
        ok &= (x <= UMAX - adj && v >= x + adj) ? 1u : 0u;
      else
        ok &= (x >= adj && v <= x - adj) ? 1u : 0u;
    }
  }
#pragma unroll
  for (int s = 0; s < MAXS; ++s) {
    if (s < (int)lv.nsrc && ok) {
      const DSource& src = lv.src[s];
      const u32* col = src.col;
      const u32 a = src.atom;
      const bool last = src.last != 0;
      u32 lo = 0, hi = 0;
      if ((u32)s == drv) {
        lo = B.lo(L - 1, a, i);
        // Only the first row of a run of equal values yields the candidate.
        if (!last && r > lo && ldg(col + r - 1) == v) {
          ok = 0;
        } else {
          hi = B.hi(L - 1, a, i);
          lo = r;
          if (last) hi = r + 1;
          else if (dhi != NONE) hi = dhi;
          else if (src.dir) hi = ldg(src.dir + v + 1);
          else hi = gallop_past(col, r + 1, hi, v);
        }
      } else if (src.alias != NONE) {
        // Same column and same range as an earlier source: same result.
        lo = slo.get(src.alias);
        hi = shi.get(src.alias);
      } else if (src.dir) {
        // Unnarrowed first column: the directory gives the run directly.
        if (v > src.dmax) {
          ok = 0;
        } else {
          lo = ldg(src.dir + v);
          hi = ldg(src.dir + v + 1);
          if (lo >= hi) ok = 0;
        }
      } else {
        lo = B.lo(L - 1, a, i);
        hi = B.hi(L - 1, a, i);
        const u32 p = lower_bound_u32(col, lo, hi, v);
        if (p >= hi || ldg(col + p) != v) {
          ok = 0;
        } else {
          lo = p;
          hi = last ? p + 1 : gallop_past(col, p + 1, hi, v);
        }
      }
      slo.put(s, lo);
      shi.put(s, hi);
    }
  }
  // Negated atoms whose last variable is bound here.
  if (ok && lv.nneg)
    for (u32 k = 0; k < P->nneg; ++k)
      if (P->neg[k].level == (u32)L) ok &= neg_absent(P->neg[k], B, L, i, v) ? 1u : 0u;
  return ok != 0;
}

// Range of atom a after binding level L (narrowed if the atom is a source).
__device__ inline void new_range(const DPlan* P, const Bufs& B, int L, u32 i, u32 a,
                                 const R8& slo, const R8& shi, u32* lo, u32* hi) {
  const u32 s = P->lvl[L].atom_src[a];
  if (s != NONE) {
    *lo = slo.get(s);
    *hi = shi.get(s);
  } else {
    *lo = B.lo(L - 1, a, i);
    *hi = B.hi(L - 1, a, i);
  }
}

// After binding level L: choose the driver of level L+1 -- the source whose
// range, clipped to the value bounds of level L+1, is smallest -- and yield
// its clipped candidate rows [clo, chi) for the new item.
__device__ inline bool prepare_item(const DPlan* P, const Bufs& B, int L, u32 i, u32 v,
                                    const R8& slo, const R8& shi, u32* drv, u32* clo, u32* chi) {
  // Per-lane flag, no early returns inside the plan-driven loops (see
  // try_candidate).
  const DLevel& nx = P->lvl[L + 1];
  u32 lov = 0, hiv = UMAX, ok = 1;
  for (u32 b = 0; b < nx.nbnd; ++b) {
    const u32 x = operand(B, nx.bnd[b].o, L, i, v);
    const u32 adj = nx.bnd[b].adj;
    if (!nx.bnd[b].is_hi) {
      ok &= x <= UMAX - adj ? 1u : 0u;
      const u32 t = x + adj;
      lov = t > lov ? t : lov;
    } else {
      ok &= x >= adj ? 1u : 0u;
      const u32 t = x - adj;
      hiv = t < hiv ? t : hiv;
    }
  }
  ok &= lov <= hiv ? 1u : 0u;
  const bool clip = lov != 0 || hiv != UMAX;
  u32 best = 0, bsz = UMAX, blo = 0, bhi = 0;
  for (u32 s = 0; s < nx.nsrc; ++s) {
    if (nx.src[s].alias != NONE || !ok) continue;  // aliases: same range as an earlier source
    u32 lo, hi;
    new_range(P, B, L, i, nx.src[s].atom, slo, shi, &lo, &hi);
    if (clip) {
      const DSource& src = nx.src[s];
      if (src.dir) {
        // Unnarrowed first column: clip through the directory.
        if (lov) lo = lov <= src.dmax ? ldg(src.dir + lov) : hi;
        if (hiv < src.dmax) hi = ldg(src.dir + hiv + 1);
      } else {
        if (lov) lo = lower_bound_u32(src.col, lo, hi, lov);
        if (hiv != UMAX) hi = upper_bound_u32(src.col, lo, hi, hiv);
      }
    }
    if (lo >= hi) {
      ok = 0;  // no value can satisfy this source
    } else if (hi - lo < bsz) {
      bsz = hi - lo;
      best = s;
      blo = lo;
      bhi = hi;
    }
  }
  *drv = best;
  *clo = blo;
  *chi = bhi;
  return ok != 0;
}

__device__ inline void store_item(const DPlan* P, const Bufs& B, int L, u32 i, u32 v, u32 pos,
                                  const R8& slo, const R8& shi, u32 drv, u32 clo,
                                  u32 chi) {
  const u32 cap = P->cap;
  u32* sm = B.sm;
  for (int k = 0; k < L; ++k) sm[P->off_val[L] + k * cap + pos] = B.val(L - 1, k, i);
  sm[P->off_val[L] + L * cap + pos] = v;
  for (u32 t = 0; t < P->nslot[L]; ++t) {
    u32 lo, hi;
    new_range(P, B, L, i, P->slot_atom[L][t], slo, shi, &lo, &hi);
    sm[P->off_lo[L] + t * cap + pos] = lo;
    sm[P->off_hi[L] + t * cap + pos] = hi;
  }
  sm[P->off_drv[L] + pos] = drv;
  sm[P->off_clo[L] + pos] = clo;
  sm[P->off_chi[L] + pos] = chi;
}

__device__ inline void emit_row(const DPlan* P, const Bufs& B, int L, u32 i, u32 v, u64 at) {
  if (at >= P->out_rows) {  // never happens when count and materialize agree
    atomicOr(P->err, 1u);
    return;
  }
  for (u32 h = 0; h < P->head_arity; ++h) P->out[h][at] = operand(B, P->head[h], L, i, v);
}

__device__ inline void stage_row(const DPlan* P, const Bufs& B, int L, u32 i, u32 v, u64 at) {
  for (u32 h = 0; h < P->head_arity; ++h) P->stage[h][at] = operand(B, P->head[h], L, i, v);
}

struct WgState {
  u32 n[MAXV];        // items in each level buffer
  u64 total[MAXV];    // candidates of each level buffer
  u64 cur[MAXV];      // candidates consumed
  u64 key_next;       // next root key to turn into a level-0 item
  u64 exam[MAXV];     // candidates examined by this workgroup, per level
  u32 rng0[2 * MAXN];
  u64 sh[WG / 64];
  u64 alloc;          // arena chunk just taken (broadcast to the workgroup)
  u32 stop;           // a memory bound was crossed (broadcast)
};

// Output state of a workgroup, held in registers by every thread (all
// threads see the same chunk totals, so they update it identically).
struct Emit {
  u64 out = 0;        // rows written / staged so far
  u64 covered = 0;    // staged rows for which arena chunks are held
  u64 chunk0 = 0, chunk1 = 0;  // arena chunks of even / odd 4096-row ranges
  u32 ovf = 0;        // staging arena exhausted for this workgroup
  // Memory-bound accounting of count passes, per lane: bytes of rows found
  // for instance acc_id (serving cap) and for the round (budget), added to
  // the global counters once they pass ACC_FLUSH or the instance changes,
  // and at the end of the pass.
  u32 acc_id = 0;
  u64 acc_inst = 0, acc_all = 0;
};

constexpr u64 ACC_FLUSH = 64u << 10;

// An instance over its cap is not a reason to stop the pass: workgroups that
// work for it alone stop (k_join polls its total), the rest finish, and the
// host drops every instance over its cap and counts again.
__device__ inline void flush_inst(const DPlan* P, Emit& em) {
  if (!em.acc_inst) return;
  atomicAdd(&P->inst_bytes[em.acc_id], (unsigned long long)em.acc_inst);
  em.acc_inst = 0;
}

__device__ inline void flush_all(const DPlan* P, Emit& em) {
  if (!em.acc_all) return;
  const u64 was = atomicAdd(P->bound_acc, (unsigned long long)em.acc_all);
  if (was + em.acc_all > uni(P->bound_limit)) atomicOr(P->abort, 1u);
  em.acc_all = 0;
}

// Account `rows` output rows of instance `id` (the level-0 value; ignored
// unless serving with a cap) against the per-instance and round bounds.
__device__ inline void account(const DPlan* P, Emit& em, u32 id, u64 rows) {
  if (!rows) return;
  const u64 bytes = rows * uni(P->row_bytes);
  if (P->inst_bytes && id < uni(P->inst_n)) {
    if (id != em.acc_id) flush_inst(P, em);
    em.acc_id = id;
    em.acc_inst += bytes;
    if (em.acc_inst >= ACC_FLUSH) flush_inst(P, em);
  }
  if (P->bound_acc) {
    em.acc_all += bytes;
    if (em.acc_all >= ACC_FLUSH) flush_all(P, em);
  }
}

// Inclusive prefix of candidate counts of buffer b; sets total, resets cursor.
__device__ void finalize_buffer(const DPlan* P, u32* sm, WgState& st, int b) {
  const u32 n = st.n[b];
  const u32 per = P->cap / WG;  // items per thread (1, 2 or 4)
  u64* pre = reinterpret_cast<u64*>(sm + P->off_pre[b]);
  u64 sum = 0;
  for (u32 t = 0; t < per; ++t) {
    u32 it = threadIdx.x * per + t;
    sum += it < n ? (u64)(sm[P->off_chi[b] + it] - sm[P->off_clo[b] + it]) : 0;
  }
  u64 tot;
  u64 run = block_excl_scan(sum, st.sh, &tot);
  for (u32 t = 0; t < per; ++t) {
    u32 it = threadIdx.x * per + t;
    if (it < n) {
      run += (u64)(sm[P->off_chi[b] + it] - sm[P->off_clo[b] + it]);
      pre[it] = run;
    }
  }
  if (threadIdx.x == 0) {
    st.total[b] = tot;
    st.cur[b] = 0;
    st.exam[b + 1] += tot;
  }
  __syncthreads();
}

// Rank the lanes whose `alive` is set; returns the lane's rank, *tot the count.
__device__ inline u64 rank_alive(bool alive, WgState& st, u64* tot) {
  return block_excl_scan(alive ? 1 : 0, st.sh, tot);
}

// One chunk of output candidates, called by every thread: count them
// (mode 0), write them at their final offsets (mode 1), or count them and
// stage them in arena chunks (mode 2).  Lane t holds candidates t*K + k of
// the chunk (k < K); rows keep that order, which is traversal order.  Only
// the rank scan synchronises the workgroup (plus one barrier when a new
// arena chunk is taken): the output state lives in every thread's registers.
template <int MODE, int K>
__device__ inline void emit_chunk(const DPlan* P, const Bufs& B, WgState& st, Emit& em, int L,
                                  const u32 (&i)[K], const u32 (&v)[K], const u32 (&alive)[K],
                                  u64 obase, u64 b, u64& my_count) {
  static_assert(K * WG <= STAGE_CHUNK, "one call stages at most one new arena chunk");
  u32 mine = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) mine += alive[k];
  if (MODE != 1 && P->inst_bytes) {
    // Per-instance memory bound (serving): the instance is the level-0 value.
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (alive[k]) account(P, em, L == 0 ? v[k] : B.val(L - 1, 0, i[k]), 1);
  } else if (MODE != 1 && P->bound_acc) {
    account(P, em, 0, mine);  // memory bound of the round
  }
  if (MODE == 0) {
    my_count += mine;
    return;
  }
  u64 tot;
  u64 rk = block_excl_scan(mine, st.sh, &tot);
  tot = uni(tot);
  // A new arena chunk when this chunk's rows pass the covered range
  // (tot <= K*WG <= STAGE_CHUNK: at most one per call).
  const bool take = MODE == 2 && !em.ovf && em.out + tot > em.covered;
  const u64 seq = em.covered / STAGE_CHUNK;
  if (take && threadIdx.x == 0) {
    const u64 c = atomicAdd(reinterpret_cast<unsigned long long*>(P->stage_next), 1ull);
    if (c < P->stage_chunks) P->chunk_tag[c] = (b << 32) | seq;
    st.alloc = c;
  }
  if (P->off_emit != NONE) {
    // Survivors in rank order in LDS (value, then parent item: items of a
    // level buffer are below 256), then every thread writes whole rows: the
    // row code runs once per row instead of once per candidate slot.
    u32* cv = B.sm + P->off_emit;
    uint8_t* ci = reinterpret_cast<uint8_t*>(cv + K * WG);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (alive[k]) {
        cv[rk] = v[k];
        ci[rk] = (uint8_t)i[k];
        ++rk;
      }
    }
    __syncthreads();
    if (take) {
      const u64 c = uni(st.alloc);
      if (c >= P->stage_chunks) {
        em.ovf = 1;
      } else {
        if (seq & 1) em.chunk1 = c; else em.chunk0 = c;
        em.covered += STAGE_CHUNK;
      }
    }
    if (MODE == 1 || !em.ovf) {
      for (u32 r = threadIdx.x; r < (u32)tot; r += WG) {
        const u32 ii = ci[r], vv = cv[r];
        const u64 row = em.out + r;
        if (MODE == 1) {
          emit_row(P, B, L, ii, vv, obase + row);
        } else {
          const u64 c = ((row / STAGE_CHUNK) & 1) ? em.chunk1 : em.chunk0;
          stage_row(P, B, L, ii, vv, c * STAGE_CHUNK + (row % STAGE_CHUNK));
        }
      }
    }
    // cv / ci are next written after the next call's rank scan, which every
    // thread reaches only after finishing these rows.
  } else {
    // Each lane writes its own survivors.
    if (take) {
      __syncthreads();
      const u64 c = uni(st.alloc);
      if (c >= P->stage_chunks) {
        em.ovf = 1;
      } else {
        if (seq & 1) em.chunk1 = c; else em.chunk0 = c;
        em.covered += STAGE_CHUNK;
      }
    }
    if (MODE == 1 || !em.ovf) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (alive[k]) {
          const u64 row = em.out + rk++;
          if (MODE == 1) {
            emit_row(P, B, L, i[k], v[k], obase + row);
          } else {
            const u64 c = ((row / STAGE_CHUNK) & 1) ? em.chunk1 : em.chunk0;
            stage_row(P, B, L, i[k], v[k], c * STAGE_CHUNK + (row % STAGE_CHUNK));
          }
        }
      }
    }
  }
  em.out += tot;
}

// Leaf candidates g0 + t*K + k (lane t, k < K) of buffer bl: the parent item,
// the value, and whether every source of the leaf level holds it.  A lane's
// candidates are consecutive, so one search finds the first one's item and
// the rest step forward (every item has at least one candidate).  At the
// leaf every source's column is its last, so only membership matters: no
// ranges are narrowed.
//
// The code is branch-free per candidate: lanes past the end work on the last
// candidate (every read stays in bounds) and are dropped at the end; reads
// that a lane does not need go to row 0 of the same column; the K membership
// searches of a lane advance in lockstep, in a loop that runs while any lane
// of the wave still searches.  Divergent branches would cost more scalar
// instructions (execution-mask bookkeeping) than the memory reads they skip.
template <int K>
__device__ inline void leaf_probe(const DPlan* P, const Bufs& B, int L, int bl, u32 nb, u64 g0,
                                  u64 total, u32 (&it)[K], u32 (&v)[K], u32 (&alive)[K]) {
  const DLevel& lv = P->lvl[L];
  const u32 nsrc = uni(lv.nsrc);
  const u64* pre = reinterpret_cast<const u64*>(B.sm + uni(P->off_pre[bl]));
  const u32* clo = B.sm + uni(P->off_clo[bl]);
  const u32* dsel = B.sm + uni(P->off_drv[bl]);
  const u64 last = total - 1;
  const u64 gl = g0 + (u64)threadIdx.x * K;
  u32 i = owner_item(pre, nb, gl < last ? gl : last);
  u64 pe = pre[i];
  u64 gb = i ? pre[i ? i - 1 : 0] : 0;
  u32 drv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const u64 gk = gl + k;
    alive[k] = gk <= last ? 1u : 0u;
    const u64 g = gk <= last ? gk : last;
    const u32 adv = g >= pe ? 1u : 0u;  // at most one item per step
    i += adv;
    gb = adv ? pe : gb;
    pe = pre[i];
    it[k] = i;
    drv[k] = dsel[i];
    v[k] = ldg(source_col(lv, drv[k]) + clo[i] + (u32)(g - gb));
  }
  const u32 nne = uni(lv.nne);
  for (u32 f = 0; f < nne; ++f) {
#pragma unroll
    for (int k = 0; k < K; ++k) alive[k] &= v[k] != operand(B, lv.ne[f], L, it[k], v[k]) ? 1u : 0u;
  }
  // Sources read through a directory (an unnarrowed first column): two reads.
  // Aliases repeat an earlier source's column and range and are skipped.
  u32 nsearch = 0;
  const u32* col0 = nullptr;  // column of the first searched source
  u32 dsr[K];                 // the candidate's driver is a searched source
#pragma unroll
  for (int k = 0; k < K; ++k) dsr[k] = 0;
  for (u32 s = 0; s < nsrc; ++s) {
    const DSource& src = lv.src[s];
    if (uni(src.alias) != NONE) continue;
    const u32* dir = (const u32*)uni((u64)src.dir);
    if (!dir) {
      if (!nsearch) col0 = (const u32*)uni((u64)src.col);
      ++nsearch;
#pragma unroll
      for (int k = 0; k < K; ++k) dsr[k] |= drv[k] == s ? 1u : 0u;
      continue;
    }
    const u32 dmax = uni(src.dmax);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const u32 act = alive[k] & (drv[k] != s ? 1u : 0u);
      const u32 x = v[k] < dmax ? v[k] : dmax;
      const u32 r0 = ldg(dir + x), r1 = ldg(dir + x + 1);
      const u32 ok = (v[k] <= dmax ? 1u : 0u) & (r0 < r1 ? 1u : 0u);
      alive[k] &= (act ^ 1u) | ok;
    }
  }
  // Searched sources, in rounds: in round j each lane searches the j-th
  // searched source other than its candidate's driver, so a wave whose items
  // have different drivers still makes one pass per round.
  // Candidates whose driver is searched need one round fewer; the last
  // round runs only if some live candidate of the wave has another driver.
  u32 drv_other = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) drv_other |= alive[k] & (dsr[k] ^ 1u);
  u32 rounds = nsearch;
  if (nsearch && __ballot(drv_other) == 0) rounds = nsearch - 1;
  const u32 cap = uni(P->cap);
  for (u32 j = 0; j < rounds; ++j) {
    const u32* tcol[K];
    u32 lo[K], hi[K], act[K], cnt[K], tsrc[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      tcol[k] = col0, lo[k] = 0, hi[k] = 0, act[k] = 0, cnt[k] = 0, tsrc[k] = 0;
    for (u32 s = 0; s < nsrc; ++s) {
      const DSource& src = lv.src[s];
      if (uni(src.alias) != NONE || uni((u64)src.dir) != 0) continue;
      const u32* col = (const u32*)uni((u64)src.col);
      const u32 a = uni(src.atom);
      const u32 slot = uni(P->atom_slot[L - 1][a]);
      const u32* slo = slot == NONE ? nullptr : B.sm + uni(P->off_lo[L - 1]) + slot * cap;
      const u32* shi = slot == NONE ? nullptr : B.sm + uni(P->off_hi[L - 1]) + slot * cap;
      const u32 r0lo = B.rng0[2 * a], r0hi = B.rng0[2 * a + 1];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const u32 other = drv[k] != s ? 1u : 0u;
        const bool pick = other && cnt[k] == j;
        const u32 l = slo ? slo[it[k]] : r0lo;
        const u32 h = shi ? shi[it[k]] : r0hi;
        tcol[k] = pick ? col : tcol[k];
        tsrc[k] = pick ? s : tsrc[k];
        lo[k] = pick ? l : lo[k];
        hi[k] = pick ? h : hi[k];
        act[k] |= pick ? 1u : 0u;
        cnt[k] += other;
      }
    }
    // Search [lo, hi) for v: base moves to the last row with value <= v while
    // the window length halves; xb is the value at base.  Lanes with nothing
    // to search get the window [0, 0) of a column that is not empty.
    //
    // A window that is a run with a bitmap (a run of at least bm_min rows
    // sharing all but the last column) is answered by one bit instead.
    u32 base[K], len[K], xb[K], hasb[K], fb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const u32 use = alive[k] & act[k] & (lo[k] < hi[k] ? 1u : 0u);
      const u32* bm_at;
      const u32* bm;
      u32 words, bmin;
      source_bitmaps(lv, tsrc[k], &bm_at, &bm, &words, &bmin);
      const bool try_bm = use && bmin && hi[k] - lo[k] >= bmin;
      // Reads that are not needed go to row 0 of the (non-empty) column.
      const u32 bid = ldg(try_bm ? bm_at + lo[k] : tcol[k]);
      const bool inr = (v[k] >> 5) < words;
      const bool hb = try_bm && bid != NONE;
      const u32 word = ldg((hb && inr) ? bm + (u64)bid * words + (v[k] >> 5) : tcol[k]);
      hasb[k] = hb ? 1u : 0u;
      fb[k] = (hb && inr && ((word >> (v[k] & 31u)) & 1u)) ? 1u : 0u;
      base[k] = (use && !hb) ? lo[k] : 0u;
      len[k] = (use && !hb) ? hi[k] - lo[k] : 0u;
      xb[k] = ldg(tcol[k] + base[k]);
    }
    for (;;) {
      u32 most = len[0];
#pragma unroll
      for (int k = 1; k < K; ++k) most = most > len[k] ? most : len[k];
      if (__ballot(most > 1) == 0) break;
      u32 mid[K], x[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        mid[k] = base[k] + (len[k] >> 1);
        x[k] = ldg(tcol[k] + mid[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool le = x[k] <= v[k];
        base[k] = le ? mid[k] : base[k];
        xb[k] = le ? x[k] : xb[k];
        len[k] -= len[k] >> 1;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const u32 found = hasb[k] ? fb[k] : (len[k] != 0 ? 1u : 0u) & (xb[k] == v[k] ? 1u : 0u);
      alive[k] &= (act[k] ^ 1u) | found;
    }
  }
  // Negated atoms tested at the leaf.
  if (uni(lv.nneg)) {
    const u32 nneg = uni(P->nneg);
    for (u32 n = 0; n < nneg; ++n) {
      if (uni(P->neg[n].level) != (u32)L) continue;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (alive[k]) alive[k] &= neg_absent(P->neg[n], B, L, it[k], v[k]) ? 1u : 0u;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(WG) void k_join(const DPlan* __restrict__ P, RootSpace rs,
                                             Partition part, u64* counts, const u64* offsets,
                                             u64 wg0, const u32* wg_list) {
  extern __shared__ __align__(16) u32 sm[];
  __shared__ WgState st;
  const u64 b = wg_list ? (u64)wg_list[blockIdx.x] : wg0 + blockIdx.x;
  const int m = (int)P->m;
  u64 us, ue;
  if (part.balance_off) {
    us = b ? ldg(rs.C + b - 1) : 0;
    ue = ldg(rs.C + b);
  } else {
    us = b * part.slice;
    ue = us + part.slice < rs.T ? us + part.slice : rs.T;
  }
  if (threadIdx.x < 2 * MAXN) st.rng0[threadIdx.x] = rs.rng0[threadIdx.x];
  if (us >= ue) {
    if (MODE != 1 && threadIdx.x == 0) counts[b] = 0;
    if (MODE == 2 && threadIdx.x == 0) P->ovf[b] = 0;
    return;
  }
  const u64 kfirst = owner_key(rs.C, 0, rs.K, us);
  const u64 klast = owner_key(rs.C, kfirst, rs.K, ue - 1);
  if (threadIdx.x == 0) {
    st.key_next = kfirst;
    for (int j = 0; j < MAXV; ++j) st.exam[j] = 0;
    st.exam[0] = klast - kfirst + 1;
    for (int j = 0; j < MAXV; ++j) st.n[j] = 0, st.total[j] = 0, st.cur[j] = 0;
  }
  __syncthreads();
  Bufs B{sm, P, st.rng0};
  const u64 obase = MODE == 1 ? offsets[b] : 0;
  u64 my_count = 0;  // leaf rows found by this lane (count mode)
  Emit em;
  int bl = -1;       // buffer being drained; -1 = root keys

  // Serving with a cap: a workgroup whose units all lie under one root key
  // works for one instance (the level-0 value) and stops once that
  // instance's counted bytes pass its cap.
  const u32 solo = MODE != 1 && P->inst_bytes && kfirst == klast ? ldg(rs.U + kfirst) : ~0u;
  u32 polls = 0;
  for (;;) {
    if (MODE != 1 && (P->abort || solo != ~0u)) {
      // A memory bound was crossed: stop (the round will be refused, or the
      // instance dropped and the round counted again).
      if (threadIdx.x == 0) {
        u32 stop = P->abort ? atomicOr(P->abort, 0u) : 0u;  // coherent read
        if (!stop && solo < P->inst_n && (++polls & 7u) == 0)
          stop = atomicAdd(&P->inst_bytes[solo], 0ull) > P->inst_cap ? 1u : 0u;
        st.stop = stop;
      }
      __syncthreads();
      if (uni(st.stop)) break;
    }
    bl = uni(bl);
    if (bl < 0) {
      if (uni(st.key_next) > klast) break;
      if (threadIdx.x == 0) st.n[0] = 0;
      __syncthreads();
      // Root keys -> level-0 items (or output rows when m == 1).
      while (uni(st.key_next) <= klast && (m == 1 || uni(st.n[0]) + WG <= P->cap)) {
        const u64 kk = uni(st.key_next) + threadIdx.x;
        bool alive = kk <= klast;
        u32 v = 0, drv = 0, clo = 0, chi = 0;
        R8 slo{}, shi{};
        if (alive) {
          v = ldg(rs.U + kk);
          alive = try_candidate(P, B, 0, 0, v, P->root_src, ldg(rs.S + kk), ldg(rs.S + kk + 1),
                                slo, shi);
        }
        const u64 cs = (alive && kk) ? ldg(rs.C + kk - 1) : 0;
        if (alive && m == 1) {
          alive = cs >= us && cs < ue;  // its single unit lies in this slice
        } else if (alive) {
          alive = prepare_item(P, B, 0, 0, v, slo, shi, &drv, &clo, &chi);
          if (alive) {
            const u64 ce = ldg(rs.C + kk);
            const u64 lo = cs > us ? cs : us, hi = ce < ue ? ce : ue;
            alive = lo < hi;
            const u32 c0 = clo;
            clo = c0 + (u32)(lo - cs);
            chi = c0 + (u32)(hi - cs);
          }
        }
        if (m == 1) {
          const u32 ia[1] = {0}, va[1] = {v}, aa[1] = {alive ? 1u : 0u};
          emit_chunk<MODE, 1>(P, B, st, em, 0, ia, va, aa, obase, b, my_count);
        } else {
          u64 tot;
          u64 rk = rank_alive(alive, st, &tot);
          if (alive) store_item(P, B, 0, 0, v, st.n[0] + (u32)rk, slo, shi, drv, clo, chi);
          __syncthreads();
          if (threadIdx.x == 0) st.n[0] += (u32)tot;
        }
        __syncthreads();
        if (threadIdx.x == 0) st.key_next += WG;
        __syncthreads();
      }
      if (m == 1) continue;
      finalize_buffer(P, sm, st, 0);
      bl = 0;
      continue;
    }

    if (uni(st.cur[bl]) >= uni(st.total[bl])) {  // buffer drained: go up
      bl -= 1;
      continue;
    }
    const int L = bl + 1;  // level whose variable the candidates bind
    const u64* pre = reinterpret_cast<const u64*>(sm + P->off_pre[bl]);
    const u32 nb = uni(st.n[bl]);

    if (L == m - 1) {
      // Leaf level: every surviving candidate is an output row.
      if (MODE == 0 && P->leaf_fast) {  // every candidate is a row: just add
        if (threadIdx.x == 0) my_count += st.total[bl] - st.cur[bl];
        if (P->inst_bytes || P->bound_acc) {
          // Each item's candidates left in [cur, total) count for its instance.
          const u64 c0 = uni(st.cur[bl]), c1 = uni(st.total[bl]);
          for (u32 it = threadIdx.x; it < nb; it += WG) {
            const u64 lo = it ? pre[it - 1] : 0, hi = pre[it];
            const u64 a = lo > c0 ? lo : c0, z = hi < c1 ? hi : c1;
            if (z > a) account(P, em, B.val(bl, 0, it), z - a);
          }
        }
        __syncthreads();
        if (threadIdx.x == 0) st.cur[bl] = st.total[bl];
        __syncthreads();
        continue;
      }
      const u64 total = uni(st.total[bl]);
      for (u64 g0 = uni(st.cur[bl]); g0 < total; g0 += LEAF_K * WG) {
        u32 i[LEAF_K], v[LEAF_K], alive[LEAF_K];
        leaf_probe<LEAF_K>(P, B, L, bl, nb, g0, total, i, v, alive);
        emit_chunk<MODE, LEAF_K>(P, B, st, em, L, i, v, alive, obase, b, my_count);
      }
      if (threadIdx.x == 0) st.cur[bl] = total;
      __syncthreads();
      continue;
    }

    // Inner level: expand candidates of buffer bl into buffer bl+1.
    if (threadIdx.x == 0) st.n[L] = 0;
    __syncthreads();
    while (uni(st.cur[bl]) < uni(st.total[bl]) && uni(st.n[L]) + WG <= P->cap) {
      const u64 total = uni(st.total[bl]);
      const u64 g = uni(st.cur[bl]) + threadIdx.x;
      bool alive = g < total;
      u32 i = 0, v = 0, drv2 = 0, clo = 0, chi = 0;
      R8 slo{}, shi{};
      if (alive) {
        i = owner_item(pre, nb, g);
        const u64 gb = i ? pre[i - 1] : 0;
        const u32 r = sm[P->off_clo[bl] + i] + (u32)(g - gb);
        const u32 drv = sm[P->off_drv[bl] + i];
        v = ldg(source_col(P->lvl[L], drv) + r);
        alive = try_candidate(P, B, L, i, v, drv, r, NONE, slo, shi) &&
                prepare_item(P, B, L, i, v, slo, shi, &drv2, &clo, &chi);
      }
      u64 tot;
      u64 rk = rank_alive(alive, st, &tot);
      if (alive) store_item(P, B, L, i, v, st.n[L] + (u32)rk, slo, shi, drv2, clo, chi);
      __syncthreads();
      if (threadIdx.x == 0) {
        st.n[L] += (u32)tot;
        st.cur[bl] = (g - threadIdx.x) + WG < total ? (g - threadIdx.x) + WG : total;
      }
      __syncthreads();
    }
    finalize_buffer(P, sm, st, L);
    bl = L;
  }

  if (MODE != 1) {
    if (P->inst_bytes) flush_inst(P, em);
    if (P->bound_acc) flush_all(P, em);
  }
  if (MODE == 0) {
    u64 tot;
    block_excl_scan(my_count, st.sh, &tot);
    if (threadIdx.x == 0) counts[b] = tot;
  } else if (MODE == 2) {
    if (threadIdx.x == 0) {
      counts[b] = em.out;
      P->ovf[b] = em.ovf;
    }
  }
  if (MODE != 0 && P->cand && threadIdx.x < P->m)
    atomicAdd(reinterpret_cast<unsigned long long*>(P->cand + threadIdx.x),
              (unsigned long long)st.exam[threadIdx.x]);
}

// Write pass for staged rows (one workgroup per arena chunk).
__global__ __launch_bounds__(WG) void k_stage_copy(const DPlan* __restrict__ P, const u64* counts,
                                                   const u64* offsets, u32 arity, u64 w0, u64 w1) {
  const u64 c = blockIdx.x;
  const u64 tag = P->chunk_tag[c];
  const u64 b = tag >> 32, seq = tag & 0xffffffffull;
  if (b < w0 || b >= w1) return;  // another range of workgroups
  if (P->ovf[b]) return;          // re-run by the materialize pass
  const u64 n = counts[b], start = seq * STAGE_CHUNK;
  if (start >= n) return;
  const u64 rows = n - start < STAGE_CHUNK ? n - start : STAGE_CHUNK;
  const u64 dst = offsets[b] + start;
  if (dst + rows > P->out_rows) {
    if (threadIdx.x == 0) atomicOr(P->err, 1u);
    return;
  }
  for (u32 h = 0; h < arity; ++h) {
    const u32* src = P->stage[h] + c * STAGE_CHUNK;
    u32* out = P->out[h] + dst;
    for (u64 t = threadIdx.x; t < rows; t += WG) out[t] = src[t];
  }
}

// Per root key: the level-0 binding, its surviving work W (Alg. 1 Phase 1).
__global__ __launch_bounds__(WG) void k_hist(const DPlan* __restrict__ P, RootSpace rs, u64* W,
                                             u32* klo, u32* kd, u32 xprod) {
  __shared__ u32 rng0[2 * MAXN];
  if (threadIdx.x < 2 * MAXN) rng0[threadIdx.x] = rs.rng0[threadIdx.x];
  __syncthreads();
  const u64 kk = (u64)blockIdx.x * WG + threadIdx.x;
  if (kk >= rs.K) return;
  Bufs B{nullptr, P, rng0};
  R8 slo{}, shi{};
  const u32 v = rs.U[kk];
  bool alive = try_candidate(P, B, 0, 0, v, P->root_src, rs.S[kk], rs.S[kk + 1], slo, shi);
  u64 w = 0;
  if (alive) {
    if (P->m == 1) {
      w = 1;
    } else if (xprod) {
      // Cross product of independent single-source levels: W = prod d_j.
      w = 1;
      for (u32 j = 1; j < P->m && w; ++j) {
        u32 lo, hi;
        new_range(P, B, 0, 0, P->lvl[j].src[0].atom, slo, shi, &lo, &hi);
        klo[(u64)j * rs.K + kk] = lo;
        kd[(u64)j * rs.K + kk] = hi - lo;
        w *= (u64)(hi - lo);
      }
    } else {
      u32 drv, clo, chi;
      if (prepare_item(P, B, 0, 0, v, slo, shi, &drv, &clo, &chi)) w = chi - clo;
    }
  }
  W[kk] = w;
}

// Each unit of a cross-product plan is one output row (the work-unit decode
// of Sec. 5): local = g - C[key-1], then mixed-radix digits over the levels.
__global__ __launch_bounds__(WG) void k_xprod(const DPlan* __restrict__ P, RootSpace rs,
                                              const u32* klo, const u32* kd, u64 g0, u64 g1) {
  // A workgroup writes XP_ROWS consecutive rows, XP_RPT per thread (strided
  // by WG, so every store instruction is coalesced).  The inclusive work
  // prefix of the root keys it covers is cached in LDS, so finding a row's
  // key is an LDS search; the rows of a thread are decoded level by level
  // together, so their loads are independent and in flight at once.  A head
  // column is written as soon as its level's value is known.
  __shared__ u64 kend[XP_KEYS];
  __shared__ u64 kr[3];
  const u64 ub = g0 + (u64)blockIdx.x * XP_ROWS;
  const u64 ue = ub + XP_ROWS < g1 ? ub + XP_ROWS : g1;
  if (threadIdx.x == 0) {
    const u64 k0 = owner_key(rs.C, 0, rs.K, ub);
    kr[0] = k0;
    kr[1] = owner_key(rs.C, k0, rs.K, ue - 1) + 1;
    kr[2] = k0 ? ldg(rs.C + k0 - 1) : 0;
  }
  __syncthreads();
  const u64 k0 = kr[0], k1 = kr[1], s0 = kr[2];
  const u32 nk = (u32)(k1 - k0);
  const bool cached = k1 - k0 <= XP_KEYS;
  if (cached)
    for (u32 i = threadIdx.x; i < nk; i += WG) kend[i] = ldg(rs.C + k0 + i);
  __syncthreads();
  const u32 m = uni(P->m), ha = uni(P->head_arity);
  const u64 K = rs.K;
  u64 g[XP_RPT], kk[XP_RPT], local[XP_RPT];
  u32 ok[XP_RPT];
  u32 bad = 0;
#pragma unroll
  for (int r = 0; r < XP_RPT; ++r) {
    const u64 gr = ub + (u64)r * WG + threadIdx.x;
    ok[r] = gr < ue ? 1u : 0u;
    bad |= ok[r] & (gr >= P->out_rows ? 1u : 0u);  // never when count and write agree
    ok[r] &= gr < P->out_rows ? 1u : 0u;
    g[r] = gr < ue ? gr : ue - 1;
    u64 start;
    if (cached) {
      // First i with kend[i] > g (kend[nk-1] >= ue > g).
      u32 lo = 0, n = nk;
      while (n > 1) {
        const u32 half = n >> 1;
        lo = kend[lo + half - 1] <= g[r] ? lo + half : lo;
        n -= half;
      }
      kk[r] = k0 + lo;
      start = lo ? kend[lo - 1] : s0;
    } else {
      kk[r] = owner_key(rs.C, k0, k1, g[r]);
      start = kk[r] ? ldg(rs.C + kk[r] - 1) : 0;
    }
    local[r] = g[r] - start;
  }
  if (bad) atomicOr(P->err, 1u);
  // Head columns that are constants or the root variable.
  for (u32 h = 0; h < ha; ++h) {
    const DOperand o = P->head[h];
    u32* out = P->out[h];
    if (o.is_var && o.v != 0) continue;
#pragma unroll
    for (int r = 0; r < XP_RPT; ++r) {
      const u32 x = o.is_var ? ldg(rs.U + kk[r]) : o.v;
      if (ok[r]) out[g[r]] = x;
    }
  }
  for (u32 j = m - 1; j >= 1; --j) {
    const u32* col = (const u32*)uni((u64)P->lvl[j].src[0].col);
    u32 x[XP_RPT];
#pragma unroll
    for (int r = 0; r < XP_RPT; ++r) {
      const u32 d = ldg(kd + (u64)j * K + kk[r]);
      const u32 base = ldg(klo + (u64)j * K + kk[r]);
      u32 ij;
      if (local[r] <= 0xffffffffull) {
        const u32 l32 = (u32)local[r];
        ij = l32 % d;
        local[r] = l32 / d;
      } else {
        ij = (u32)(local[r] % d);
        local[r] /= d;
      }
      x[r] = ldg(col + base + ij);
    }
    for (u32 h = 0; h < ha; ++h) {
      const DOperand o = P->head[h];
      if (!o.is_var || o.v != j) continue;
      u32* out = P->out[h];
#pragma unroll
      for (int r = 0; r < XP_RPT; ++r)
        if (ok[r]) out[g[r]] = x[r];
    }
  }
}

// Narrow every atom by its leading constant columns.
__global__ void k_init_ranges(const DPlan* __restrict__ P, u32* rng0) {
  const u32 a = threadIdx.x;
  if (a >= MAXN) return;
  if (a >= P->natoms) {
    rng0[2 * a] = 0;
    rng0[2 * a + 1] = 0;
    return;
  }
  u32 lo = 0, hi = P->atom_n[a];
  for (u32 c = 0; c < P->atom_nconst[a]; ++c) {
    const u32* col = P->atom_col[a][c];
    const u32 x = P->atom_const[a][c];
    u32 l2 = lower_bound_u32(col, lo, hi, x);
    hi = upper_bound_u32(col, l2, hi, x);
    lo = l2;
  }
  rng0[2 * a] = lo;
  rng0[2 * a + 1] = hi;
}

// Root keys: first rows of runs of equal values in [lo, hi) of `col`.
__global__ __launch_bounds__(WG) void k_key_flags(const u32* col, const u32* rng0, u32 atom, u32 n,
                                                  u32* flags) {
  const u64 r = (u64)blockIdx.x * WG + threadIdx.x;
  if (r >= n) return;
  const u32 lo = rng0[2 * atom], hi = rng0[2 * atom + 1];
  flags[r] = (r >= lo && r < hi && (r == lo || col[r] != col[r - 1])) ? 1u : 0u;
}

__global__ __launch_bounds__(WG) void k_key_compact(const u32* col, const u32* flags,
                                                    const u64* pos, u32 n, u32* U, u32* S) {
  const u64 r = (u64)blockIdx.x * WG + threadIdx.x;
  if (r >= n || !flags[r]) return;
  U[pos[r]] = col[r];
  S[pos[r]] = (u32)r;
}

__global__ void k_key_end(const u32* rng0, u32 atom, u64 K, u32* S) { S[K] = rng0[2 * atom + 1]; }

// dir[v] = first row with value >= v, one thread per entry v in [0, vmax+1]
// (a lower bound search; adjacent threads walk nearly the same path, so the
// upper levels of the search stay in cache).
__global__ __launch_bounds__(WG) void k_build_dir(const u32* col, u64 n, u32 vmax, u32* dir) {
  const u64 v = (u64)blockIdx.x * WG + threadIdx.x;
  if (v > (u64)vmax + 1) return;
  u64 lo = 0, hi = n;
  while (lo < hi) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if ((u64)col[mid] < v) lo = mid + 1; else hi = mid;
  }
  dir[v] = (u32)lo;
}

u32 grid1(u64 n) {
  u64 g = ceil_div(n, WG);
  if (g > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "grid too large");
  return (u32)(g ? g : 1);
}

// ---- run bitmaps ------------------------------------------------------------

struct Prefix { const u32* c[MAXA]; };

__device__ inline int prefix_cmp(const Prefix& p, u32 kp, u64 i, u64 j) {
  for (u32 c = 0; c < kp; ++c) {
    const u32 x = p.c[c][i], y = p.c[c][j];
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

// Long runs without reading every row: a run of at least 2*RUN_PROBE rows
// holds two probe rows j and j + RUN_PROBE (j a multiple of RUN_PROBE) with
// equal prefixes.  Such a probe finds the run's bounds by binary search and
// reports it once, from the first probe row inside it.
constexpr u32 RUN_PROBE = 256;

__global__ __launch_bounds__(WG) void k_run_probe(Prefix p, u32 kp, u64 n, u32 min_run,
                                                  u32* count, u32 cap, u32* rs, u32* re) {
  const u64 t = (u64)blockIdx.x * WG + threadIdx.x;
  const u64 j = t * RUN_PROBE;
  if (j + RUN_PROBE >= n || prefix_cmp(p, kp, j, j + RUN_PROBE) != 0) return;
  // First row of the run: lower bound of row j's prefix in [0, j].
  u64 lo = 0, hi = j;
  while (lo < hi) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if (prefix_cmp(p, kp, mid, j) < 0) lo = mid + 1; else hi = mid;
  }
  const u64 s = lo;
  if ((s + RUN_PROBE - 1) / RUN_PROBE * RUN_PROBE != j) return;  // not the run's first probe
  // End of the run: upper bound in [j + RUN_PROBE, n).
  lo = j + RUN_PROBE;
  hi = n;
  while (lo < hi) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if (prefix_cmp(p, kp, mid, j) <= 0) lo = mid + 1; else hi = mid;
  }
  if (lo - s < min_run) return;
  const u32 at = atomicAdd(count, 1u);
  if (at < cap) {
    rs[at] = (u32)s;
    re[at] = (u32)lo;
  }
}

// Bitmap ids for the runs kept (length >= thr, in list order).
__global__ __launch_bounds__(WG) void k_run_keep(const u32* rs, const u32* re, u32 nruns, u32 thr,
                                                 u32* keep) {
  const u32 r = blockIdx.x * WG + threadIdx.x;
  if (r < nruns) keep[r] = re[r] - rs[r] >= thr ? 1u : 0u;
}

__global__ __launch_bounds__(WG) void k_run_mark(const u32* rs, const u32* re, u32 nruns,
                                                 const u32* keep, const u64* ids, u32* bm_at,
                                                 u32* start, u32* len) {
  const u32 r = blockIdx.x * WG + threadIdx.x;
  if (r >= nruns || !keep[r]) return;
  const u64 id = ids[r];
  bm_at[rs[r]] = (u32)id;
  start[id] = rs[r];
  len[id] = re[r] - rs[r];
}

// One workgroup per selected run: set the bits of its last-column values.
__global__ __launch_bounds__(WG) void k_run_bits(const u32* last, const u32* start,
                                                 const u32* len, u32 words, u32* bm) {
  const u64 id = blockIdx.x;
  const u64 s0 = start[id], l = len[id];
  u32* b = bm + id * words;
  for (u64 t = threadIdx.x; t < l; t += WG) {
    const u32 v = last[s0 + t];
    atomicOr(&b[v >> 5], 1u << (v & 31u));
  }
}

}  // namespace

void join_init_ranges(Ctx c, const DPlan* d_plan, u32 natoms, u32* d_rng0) {
  (void)natoms;
  k_init_ranges<<<1, 64, 0, c.s>>>(d_plan, d_rng0);
  WCDL_HIP(hipGetLastError());
}

void join_root_flags(Ctx c, const u32* col, const u32* d_rng0, u32 atom, u32 n_rows, u32* flags,
                     u64* pos, u64* d_K) {
  if (n_rows == 0) {
    fill_u64(c, d_K, 1, 0);
    return;
  }
  k_key_flags<<<grid1(n_rows), WG, 0, c.s>>>(col, d_rng0, atom, n_rows, flags);
  WCDL_HIP(hipGetLastError());
  scan_u32_excl(c, flags, pos, n_rows, d_K);
}

void join_root_compact(Ctx c, const u32* col, const u32* d_rng0, u32 atom, u32 n_rows,
                       const u32* flags, const u64* pos, u64 K, u32* U, u32* S) {
  if (n_rows) {
    k_key_compact<<<grid1(n_rows), WG, 0, c.s>>>(col, flags, pos, n_rows, U, S);
    WCDL_HIP(hipGetLastError());
  }
  k_key_end<<<1, 1, 0, c.s>>>(d_rng0, atom, K, S);
  WCDL_HIP(hipGetLastError());
}

void build_directory(Ctx c, const u32* col, u64 n, u32 vmax, u32* dir) {
  if (n == 0) return;
  k_build_dir<<<grid1((u64)vmax + 2), WG, 0, c.s>>>(col, n, vmax, dir);
  WCDL_HIP(hipGetLastError());
}

u32 build_run_bitmaps(Ctx c, u32 k, const u32* const* cols, u64 n, u32 vmax, u32 min_run,
                      u64 max_bytes, DBuf<u32>* bm_at, DBuf<u32>* bm, u32* words) {
  if (k < 2 || k > (u32)MAXA || n < min_run || n >= 0xffffffffull) return 0;
  if (min_run < 2 * RUN_PROBE) min_run = 2 * RUN_PROBE;
  Prefix p{};
  for (u32 j = 0; j + 1 < k; ++j) p.c[j] = cols[j];
  // At most one run per probe row can be long enough.
  const u64 probes = n / RUN_PROBE + 1;
  const u32 cap = (u32)std::min<u64>(probes, 1u << 24);
  DBuf<u32> cnt(c.mem, 1), rs(c.mem, cap), re(c.mem, cap);
  fill_u32(c, cnt.get(), 1, 0);
  k_run_probe<<<grid1(probes), WG, 0, c.s>>>(p, k - 1, n, min_run, cnt.get(), cap, rs.get(),
                                              re.get());
  WCDL_HIP(hipGetLastError());
  u32 nr = 0;
  WCDL_HIP(hipMemcpyAsync(&nr, cnt.get(), sizeof(u32), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipStreamSynchronize(c.s));
  nr = std::min(nr, cap);
  if (nr == 0) return 0;
  // Keep the longest runs that fit the budget: threshold = a run length.
  std::vector<u32> hs(nr), he(nr);
  WCDL_HIP(hipMemcpyAsync(hs.data(), rs.get(), nr * sizeof(u32), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipMemcpyAsync(he.data(), re.get(), nr * sizeof(u32), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipStreamSynchronize(c.s));
  std::vector<u32> lens(nr);
  for (u32 r = 0; r < nr; ++r) lens[r] = he[r] - hs[r];
  std::sort(lens.begin(), lens.end(), std::greater<u32>());
  const u64 w = ((u64)vmax >> 5) + 1;
  if (n * 4 + w * 4 > max_bytes) return 0;
  const u64 fit = (max_bytes - n * 4) / (w * 4);
  // All runs if they fit, else those longer than the (fit+1)-th longest.
  const u32 thr = nr <= fit ? min_run : lens[fit] + 1;
  u64 nsel = 0;
  for (u32 r = 0; r < nr; ++r) nsel += lens[r] >= thr ? 1 : 0;
  if (nsel == 0) return 0;
  DBuf<u32> keep(c.mem, nr);
  DBuf<u64> ids(c.mem, nr);
  k_run_keep<<<grid1(nr), WG, 0, c.s>>>(rs.get(), re.get(), nr, thr, keep.get());
  WCDL_HIP(hipGetLastError());
  scan_u32_excl(c, keep.get(), ids.get(), nr, nullptr);
  *bm_at = DBuf<u32>(c.mem, n);
  *bm = DBuf<u32>(c.mem, nsel * w);
  fill_u32(c, bm_at->get(), n, NONE);
  fill_u32(c, bm->get(), nsel * w, 0);
  DBuf<u32> st(c.mem, nsel), ln(c.mem, nsel);
  k_run_mark<<<grid1(nr), WG, 0, c.s>>>(rs.get(), re.get(), nr, keep.get(), ids.get(),
                                        bm_at->get(), st.get(), ln.get());
  WCDL_HIP(hipGetLastError());
  k_run_bits<<<(u32)nsel, WG, 0, c.s>>>(cols[k - 1], st.get(), ln.get(), (u32)w, bm->get());
  WCDL_HIP(hipGetLastError());
  WCDL_HIP(hipStreamSynchronize(c.s));
  *words = (u32)w;
  return thr;
}

void join_histogram(Ctx c, const DPlan* d_plan, const RootSpace& rs, u64* W, u32* klo, u32* kd,
                    u32 m) {
  (void)m;
  if (rs.K == 0) return;
  k_hist<<<grid1(rs.K), WG, 0, c.s>>>(d_plan, rs, W, klo, kd, klo != nullptr);
  WCDL_HIP(hipGetLastError());
}

void join_run(Ctx c, const DPlan* d_plan, const RootSpace& rs, const Partition& part,
              u32 lds_bytes, int mode, u64* counts, const u64* offsets, u64 wg0, u64 nwg,
              const u32* wg_list) {
  if (nwg == 0) return;
  if (nwg > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "too many workgroups");
  if (lds_bytes > 60 * 1024) {
    // Deep plans: allow more than the default dynamic LDS (gfx950 has 160 KB per CU).
    WCDL_HIP(hipFuncSetAttribute((const void*)k_join<0>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    WCDL_HIP(hipFuncSetAttribute((const void*)k_join<1>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    WCDL_HIP(hipFuncSetAttribute((const void*)k_join<2>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
  }
  if (mode == 0)
    k_join<0><<<(u32)nwg, WG, lds_bytes, c.s>>>(d_plan, rs, part, counts, offsets, wg0, wg_list);
  else if (mode == 1)
    k_join<1><<<(u32)nwg, WG, lds_bytes, c.s>>>(d_plan, rs, part, counts, offsets, wg0, wg_list);
  else
    k_join<2><<<(u32)nwg, WG, lds_bytes, c.s>>>(d_plan, rs, part, counts, offsets, wg0, wg_list);
  WCDL_HIP(hipGetLastError());
}

void join_stage_copy(Ctx c, const DPlan* d_plan, u64 used_chunks, const u64* counts,
                     const u64* offsets, u32 arity, u64 w0, u64 w1) {
  if (used_chunks == 0) return;
  if (used_chunks > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "too many staged chunks");
  k_stage_copy<<<(u32)used_chunks, WG, 0, c.s>>>(d_plan, counts, offsets, arity, w0, w1);
  WCDL_HIP(hipGetLastError());
}

void join_xprod(Ctx c, const DPlan* d_plan, const RootSpace& rs, const u32* klo, const u32* kd,
                u32 m, u64 g0, u64 g1) {
  (void)m;
  if (g1 <= g0) return;
  const u64 nwg = ceil_div(g1 - g0, (u64)XP_ROWS);
  if (nwg > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "grid too large");
  k_xprod<<<(u32)nwg, WG, 0, c.s>>>(d_plan, rs, klo, kd, g0, g1);
  WCDL_HIP(hipGetLastError());
}

}  // namespace wcdl
