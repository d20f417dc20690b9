// Host side of the engine: rule parsing and validation, stratification,
// join planning, the relation store and the semi-naive driver, behind the C
// ABI declared in wcdl.h.  Every step of evaluation runs in the HIP kernels
// of prim.hip and wcoj.hip; this file only plans, allocates and launches.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <functional>
#include <limits>
#include <memory>
#include <numeric>
#include <set>

#include "wcdl_internal.h"

namespace wcdl {

// ===========================================================================
// Static scratch of the allocation-free live-instance listing
// ===========================================================================
//
// wcdl_serve_live_static lists the live instances of a serving engine without
// allocating: its kernels work in this fixed device array (one copy per GPU,
// held until the process ends).  Layout in 32-bit words: [0] ids listed,
// [1] set if some id is >= LIVE_MAX_IDS; from LIVE_BITMAP_AT one bit per
// instance id below LIVE_MAX_IDS; from LIVE_LIST_AT at most LIVE_MAX_LIST ids.
constexpr u32 LIVE_MAX_IDS = 1u << 22;
constexpr u32 LIVE_MAX_LIST = 1u << 20;
constexpr u32 LIVE_BITMAP_AT = 64;
constexpr u32 LIVE_LIST_AT = LIVE_BITMAP_AT + LIVE_MAX_IDS / 32;
constexpr u32 LIVE_SCRATCH_WORDS = LIVE_LIST_AT + LIVE_MAX_LIST;

static __device__ __align__(256) u32 scratch[LIVE_SCRATCH_WORDS];

// Device address of `scratch` on each GPU (the host-side name is not one);
// looked up once per device when an engine is created there.
constexpr int MAX_DEVICES = 64;
u32* scratch_at[MAX_DEVICES] = {};

void ensure_scratch_address(int device) {
  if (device < 0 || device >= MAX_DEVICES) throw Error(WCDL_E_INVALID, "device ordinal out of range");
  if (scratch_at[device]) return;
  void* p = nullptr;
  WCDL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  scratch_at[device] = static_cast<u32*>(p);
}

// Clear the counters and the bitmap (a kernel rather than a memset).
__global__ void k_live_clear(u32* sc) {
  for (u64 w = (u64)blockIdx.x * blockDim.x + threadIdx.x; w < LIVE_LIST_AT;
       w += (u64)gridDim.x * blockDim.x)
    sc[w] = 0;
}

// Set the bit of every distinct leading value of a sorted column.
__global__ void k_live_mark(const u32* col, u64 n, u32* sc) {
  const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (i > 0 && col[i] == col[i - 1])) return;
  const u32 v = col[i];
  if (v >= LIVE_MAX_IDS) {
    atomicOr(&sc[1], 1u);
    return;
  }
  atomicOr(&sc[LIVE_BITMAP_AT + (v >> 5)], 1u << (v & 31u));
}

// One workgroup of 1,024 threads lists the set bits in ascending order:
// thread t owns a contiguous stretch of bitmap words.
__global__ __launch_bounds__(1024) void k_live_list(u32* sc) {
  constexpr u32 T = 1024, W = LIVE_MAX_IDS / 32 / T;
  __shared__ u32 part[T];
  const u32 t = threadIdx.x;
  const u32* bm = sc + LIVE_BITMAP_AT + t * W;
  u32 c = 0;
  for (u32 w = 0; w < W; ++w) c += __popc(bm[w]);
  part[t] = c;
  __syncthreads();
  // Exclusive prefix over the threads (Hillis-Steele in LDS).
  for (u32 d = 1; d < T; d <<= 1) {
    const u32 x = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  u32 at = part[t] - c;
  if (t == T - 1) sc[0] = part[t];
  for (u32 w = 0; w < W; ++w) {
    u32 bits = bm[w];
    while (bits) {
      const u32 b = __ffs(bits) - 1;
      bits &= bits - 1;
      if (at < LIVE_MAX_LIST) sc[LIVE_LIST_AT + at] = (t * W + w) * 32 + b;
      ++at;
    }
  }
}

// ===========================================================================
// Device memory cache
// ===========================================================================

size_t DeviceMemory::size_class(size_t bytes) {
  if (bytes <= 256) return 256;
  if (bytes <= (1u << 20)) {  // powers of two up to 1 MiB
    size_t c = 512;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t q = 1u << 20;  // then whole MiB
  return (bytes + q - 1) / q * q;
}

void* DeviceMemory::raw_alloc(size_t bytes) {
  void* p = nullptr;
  if (user_.alloc) {
    p = user_.alloc(user_.ctx, bytes, (void*)stream_);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

void DeviceMemory::raw_free(void* p, size_t bytes) {
  if (user_.alloc) {
    if (user_.free) user_.free(user_.ctx, p, bytes, (void*)stream_);
  } else {
    (void)hipFree(p);
  }
}

void* DeviceMemory::get(size_t bytes) {
  const size_t c = size_class(bytes);
  // Reuse a cached block of this class or one up to 25 % larger.
  auto it = free_.lower_bound(c);
  if (it != free_.end() && it->first <= c + c / 4) {
    void* p = it->second;
    size_t sz = it->first;
    free_.erase(it);
    live_[p] = sz;
    live_bytes_ += sz;
    return p;
  }
  void* p = raw_alloc(c);
  if (!p) {
    // Give the cache back and retry once.
    WCDL_HIP(hipDeviceSynchronize());
    sync_point();
    release_cached();
    p = raw_alloc(c);
  }
  if (!p) throw Error(WCDL_E_NOMEM, "device allocation of " + std::to_string(c) + " bytes failed");
  live_[p] = c;
  live_bytes_ += c;
  return p;
}

void DeviceMemory::put(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  pending_.push_back({p, it->second});
  live_bytes_ -= it->second;
  live_.erase(it);
}

void DeviceMemory::sync_point() {
  for (auto& b : pending_) free_.insert({b.second, b.first});
  pending_.clear();
}

void DeviceMemory::release_cached() {
  for (auto& b : free_) raw_free(b.second, b.first);
  free_.clear();
}

DeviceMemory::~DeviceMemory() {
  (void)hipDeviceSynchronize();
  sync_point();
  release_cached();
  for (auto& b : live_) raw_free(b.first, b.second);
  live_.clear();
}

namespace {

// ===========================================================================
// Program representation
// ===========================================================================

struct Term {
  bool var = false;
  u32 v = 0;
};

struct Atom {
  u32 rel = 0;
  std::vector<Term> t;
};

enum { OP_LT = 0, OP_LE = 1, OP_NE = 2 };

struct Cmp {
  u32 op = OP_LT;  // a op b
  Term a, b;
};

struct Rule {
  Atom head;
  std::vector<Atom> body;
  std::vector<Cmp> cmps;
  std::vector<Atom> negs;  // negated atoms (stratified negation)
  u32 nvars = 0;
  std::vector<u32> var_order;  // optional user order (original variable ids)
  // Helper-relation splitting: the body as registered, and where each of its
  // atoms now sits in `body` (-1 once a split moved it into a helper).
  std::vector<Atom> orig;
  std::vector<int> orig_at;
};

struct Relation {
  std::string name;
  u32 arity = 0;        // stored columns (the instance column included in batched mode)
  u32 user_arity = 0;   // columns as declared
  Cols base;                                   // loaded facts, canonical order
  Cols full;                                   // current relation (the body), canonical order
  // Rows merged this stratum but not yet into `full` (Sec. 4, Merge): the
  // relation is full ∪ head, disjoint.  Only kept while no join of the
  // stratum reads the full relation; empty outside a stratum's rounds.
  Cols head;
  std::map<std::vector<u32>, Cols> full_ord;   // other column orders of full
  std::map<std::vector<u32>, Cols> delta_ord;  // current delta, by column order
  std::vector<u64> delta_sizes;
  bool derived = false;                        // head of some rule
};

std::vector<u32> canonical(u32 k) {
  std::vector<u32> o(k);
  std::iota(o.begin(), o.end(), 0u);
  return o;
}

// ===========================================================================
// Text syntax parser (independent of the C structures' validation below).
// ===========================================================================

struct Lexer {
  const std::string& s;
  size_t i = 0;
  explicit Lexer(const std::string& src) : s(src) {}
  void skip() {
    for (;;) {
      while (i < s.size() && isspace((unsigned char)s[i])) ++i;
      if (i < s.size() && s[i] == '%') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else if (i + 1 < s.size() && s[i] == '/' && s[i + 1] == '/') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else {
        return;
      }
    }
  }
  bool at_end() { skip(); return i >= s.size(); }
  bool lit(const char* t) {
    skip();
    size_t n = strlen(t);
    if (s.compare(i, n, t) == 0) { i += n; return true; }
    return false;
  }
  bool peek(const char* t) {
    skip();
    return s.compare(i, strlen(t), t) == 0;
  }
  bool ident(std::string& out) {
    skip();
    if (i < s.size() && (isalpha((unsigned char)s[i]) || s[i] == '_')) {
      size_t j = i + 1;
      while (j < s.size() && (isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
      out = s.substr(i, j - i);
      i = j;
      return true;
    }
    return false;
  }
  int number(u32& out) {  // 1 ok, 0 none, -1 overflow
    skip();
    if (i >= s.size() || !isdigit((unsigned char)s[i])) return 0;
    u64 v = 0;
    while (i < s.size() && isdigit((unsigned char)s[i])) {
      v = v * 10 + (u64)(s[i++] - '0');
      if (v > 0xffffffffull) return -1;
    }
    out = (u32)v;
    return 1;
  }
  [[noreturn]] void fail(const std::string& m) {
    throw Error(WCDL_E_PARSE, m + " at offset " + std::to_string(i));
  }
};

// ===========================================================================
// Engine
// ===========================================================================

struct Version;

}  // namespace
}  // namespace wcdl

struct wcdl_engine {
  wcdl_config cfg{};
  std::vector<hipStream_t> streams;
  bool own_streams = false;
  std::unique_ptr<wcdl::DeviceMemory> mem;
  std::vector<wcdl::Relation> rels;
  std::map<std::string, uint32_t> rel_ids;
  std::vector<wcdl::Rule> rules;
  std::string err;
  // Pinned host copies of rule-version plans, one per version of the
  // largest batch so far, kept for the engine's lifetime (a plan is staged
  // here before its asynchronous upload).
  std::vector<void*> plan_staging;
  uint32_t helper_count = 0;
  std::map<std::string, uint32_t> helper_keys;  // canonical helper definition -> relation
  wcdl_run_stats last{};
  // Rows produced per work unit by each rule version (rule, delta atom) the
  // last time it ran; sizes the count-pass staging arena.
  std::map<std::pair<uint32_t, int>, double> rows_per_unit;
  // Serving state: one version per rule and body atom; admitted facts.
  bool serving = false;
  std::vector<wcdl::Version> serve_versions;
  std::map<uint32_t, wcdl::Cols> pending;
  // Instances (batched engines): ids handed out so far.
  uint32_t next_instance = 0;
  // Serving: largest instance id admitted so far; instances rejected by the
  // per-instance memory cap.
  uint32_t max_instance = 0;
  std::set<uint32_t> rejected;
  // Cost planner: distinct values per column of each relation, with the row
  // count they were taken at (recomputed when it changes).
  std::map<uint32_t, std::pair<uint64_t, std::vector<uint64_t>>> col_stats;
  uint64_t device_total = 0;  // bytes of device memory (queried once)
};

// An instance of a batched engine's program: its rows carry `id` in the
// leading column of every relation.
struct wcdl_instance {
  wcdl_engine* e = nullptr;
  uint32_t id = 0;
};

namespace wcdl {
namespace {

using Engine = wcdl_engine;

Ctx ctx(Engine* e, size_t s = 0) { return Ctx{e->mem.get(), e->streams[s % e->streams.size()]}; }

void sync_all(Engine* e) {
  for (auto s : e->streams) WCDL_HIP(hipStreamSynchronize(s));
  e->mem->sync_point();
}

u32 bits_of(u32 orv) {
  u32 b = 0;
  while (b < 32 && (orv >> b)) ++b;
  return b;
}

// Sorted copy of k columns (pointers in the target order), deduplicated if
// `dedup`.  Returns a Cols holding `order`.
Cols sort_rows(Engine* e, size_t si, const std::vector<u32>& order,
               const std::vector<const u32*>& in, u64 n, bool dedup) {
  Ctx c = ctx(e, si);
  const u32 k = (u32)in.size();
  Cols out;
  out.order = order;
  if (n == 0) {
    for (u32 j = 0; j < k; ++j) out.col.emplace_back();
    out.n = 0;
    return out;
  }
  DBuf<u32> d_or(c.mem, k);
  column_or(c, k, in.data(), n, d_or.get());
  std::vector<u32> h_or(k);
  WCDL_HIP(hipMemcpyAsync(h_or.data(), d_or.get(), k * sizeof(u32), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipStreamSynchronize(c.s));
  std::vector<u32> bits(k);
  for (u32 j = 0; j < k; ++j) bits[j] = bits_of(h_or[j]);
  std::vector<DBuf<u32>> sorted;
  std::vector<u32*> sp;
  for (u32 j = 0; j < k; ++j) {
    sorted.emplace_back(c.mem, n);
    sp.push_back(sorted.back().get());
  }
  radix_sort_rows(c, k, in.data(), sp.data(), n, bits.data());
  if (!dedup) {
    out.col = std::move(sorted);
    out.n = n;
    return out;
  }
  std::vector<DBuf<u32>> uq;
  std::vector<u32*> up;
  for (u32 j = 0; j < k; ++j) {
    uq.emplace_back(c.mem, n);
    up.push_back(uq.back().get());
  }
  std::vector<const u32*> sc(sp.begin(), sp.end());
  out.n = unique_rows(c, k, sc.data(), n, up.data());
  out.col = std::move(uq);
  return out;
}

// A copy of `src` (any order) re-sorted into `order` (a permutation of the
// logical columns).
Cols reorder(Engine* e, size_t si, const Cols& src, const std::vector<u32>& order) {
  std::vector<const u32*> in;
  for (u32 j = 0; j < order.size(); ++j) {
    u32 logical = order[j];
    u32 pos = (u32)(std::find(src.order.begin(), src.order.end(), logical) - src.order.begin());
    in.push_back(src.col[pos].get());
  }
  return sort_rows(e, si, order, in, src.n, false);
}

Cols copy_cols(Engine* e, const Cols& src) {
  Cols out;
  out.order = src.order;
  out.n = src.n;
  for (auto& c : src.col) {
    out.col.emplace_back(e->mem.get(), src.n);
    if (src.n) copy_u32(ctx(e), out.col.back().get(), c.get(), src.n);
  }
  return out;
}

Cols empty_cols(u32 k, const std::vector<u32>& order) {
  Cols c;
  c.order = order;
  for (u32 j = 0; j < k; ++j) c.col.emplace_back();
  (void)k;
  return c;
}

// rows(a) \ rows(b), both sorted unique in the same order.
// a \ b \ b2 (b2 optional) for sorted-unique runs in the same order.
Cols difference(Engine* e, size_t si, const Cols& a, const Cols& b, const Cols* b2 = nullptr) {
  Cols out;
  out.order = a.order;
  const u32 k = a.arity();
  if (a.n == 0) {
    for (u32 j = 0; j < k; ++j) out.col.emplace_back();
    return out;
  }
  std::vector<u32*> op;
  for (u32 j = 0; j < k; ++j) {
    out.col.emplace_back(e->mem.get(), a.n);
    op.push_back(out.col.back().get());
  }
  auto ap = a.ptrs(), bp = b.ptrs();
  std::vector<const u32*> b2p;
  if (b2 && b2->n) b2p = b2->ptrs();
  out.n = set_difference(ctx(e, si), k, ap.data(), a.n, bp.data(), b.n, op.data(),
                         b2p.empty() ? nullptr : b2p.data(), b2p.empty() ? 0 : b2->n);
  return out;
}

// a U b for disjoint sorted-unique runs in the same order.
Cols merged(Engine* e, size_t si, const Cols& a, const Cols& b) {
  Cols out;
  out.order = a.order;
  const u32 k = a.arity();
  out.n = a.n + b.n;
  std::vector<u32*> op;
  for (u32 j = 0; j < k; ++j) {
    out.col.emplace_back(e->mem.get(), out.n);
    op.push_back(out.col.back().get());
  }
  if (out.n) {
    auto ap = a.ptrs(), bp = b.ptrs();
    merge_disjoint(ctx(e, si), k, ap.data(), a.n, bp.data(), b.n, op.data());
  }
  return out;
}

// ===========================================================================
// Planning
// ===========================================================================

// One body atom as a version reads it.
struct AtomUse {
  u32 rel = 0;
  bool delta = false;
  std::vector<u32> order;     // index order: logical column per position
  std::vector<int> pos_var;   // per position: variable id or -1 (constant)
  std::vector<u32> pos_const;
  u32 nconst = 0;
};

struct Version {
  u32 rule = 0;
  int delta_atom = -1;
  u32 head_rel = 0;
  bool dead = false;            // a comparison between constants fails
  std::vector<u32> level_var;   // variable id at each level
  std::vector<AtomUse> atoms;
  std::vector<AtomUse> negs;    // negated atoms, in the order of DPlan::neg
  std::vector<std::vector<u32>> src_pos;  // per level, per source: column position in its atom
  std::vector<std::vector<bool>> want_dir;  // per level, per source: unnarrowed first column
  DPlan plan{};                 // pointers filled at evaluation time
  bool sorted_output = false;   // rows come out sorted by head columns, unique
  // Leading head columns that are the first join levels in order: the rows
  // come out non-decreasing in them (with repeats if levels follow them).
  u32 sorted_prefix = 0;
  u32 lds_bytes = 0;
};

// A rule with repeated variables inside one atom rewritten: each repeat
// becomes a fresh variable constrained equal (<= both ways) to the first.
Rule normalize(const Rule& r0) {
  Rule r = r0;
  for (auto& a : r.body) {
    std::set<u32> seen;
    for (auto& t : a.t) {
      if (!t.var) continue;
      if (seen.count(t.v)) {
        u32 fresh = r.nvars++;
        Cmp c1, c2;
        c1.op = OP_LE; c1.a = {true, fresh}; c1.b = {true, t.v};
        c2.op = OP_LE; c2.a = {true, t.v}; c2.b = {true, fresh};
        r.cmps.push_back(c1);
        r.cmps.push_back(c2);
        t.v = fresh;
      } else {
        seen.insert(t.v);
      }
    }
  }
  return r;
}

std::vector<u32> choose_order(const Rule& r, int delta_atom) {
  // Body variables in order of first appearance.
  std::vector<u32> vars;
  std::vector<int> first(r.nvars, -1);
  for (auto& a : r.body)
    for (auto& t : a.t)
      if (t.var && first[t.v] < 0) {
        first[t.v] = (int)vars.size();
        vars.push_back(t.v);
      }
  if (!r.var_order.empty() && r.var_order.size() == vars.size()) {
    // A user order over the original variables; fresh variables (from
    // repeats) are not in it, so it is only used when the sizes agree.
    return r.var_order;
  }
  std::vector<u32> occ(r.nvars, 0);
  for (auto& a : r.body) {
    std::set<u32> in;
    for (auto& t : a.t)
      if (t.var) in.insert(t.v);
    for (u32 v : in) occ[v]++;
  }
  std::vector<int> head_pos(r.nvars, 1 << 20);
  for (size_t h = 0; h < r.head.t.size(); ++h)
    if (r.head.t[h].var && head_pos[r.head.t[h].v] == (1 << 20)) head_pos[r.head.t[h].v] = (int)h;

  std::vector<bool> bound(r.nvars, false);
  std::vector<u32> order;
  auto connected_count = [&](u32 v) {
    u32 c = 0;
    for (auto& a : r.body) {
      bool has_v = false, has_b = false;
      for (auto& t : a.t)
        if (t.var) {
          if (t.v == v) has_v = true;
          else if (bound[t.v]) has_b = true;
        }
      if (has_v && has_b) ++c;
    }
    return c;
  };
  // Without a delta atom, try the head's own variable order: if it covers
  // every body variable once and stays connected, the output comes out
  // sorted and unique.
  if (delta_atom < 0) {
    std::vector<u32> hv;
    std::set<u32> hs;
    bool ok = true;
    for (auto& t : r.head.t) {
      if (!t.var) continue;
      if (hs.count(t.v)) { ok = false; break; }
      hs.insert(t.v);
      hv.push_back(t.v);
    }
    if (ok && hv.size() == vars.size()) {
      for (size_t i = 0; i < hv.size() && ok; ++i) {
        if (i > 0 && connected_count(hv[i]) == 0) ok = false;
        bound[hv[i]] = true;
      }
      if (ok) return hv;
      std::fill(bound.begin(), bound.end(), false);
    }
  }
  // Root: a variable of the delta atom (delta-first), most shared first.
  auto better = [&](u32 a, u32 b, bool use_conn) {  // is a preferred over b
    if (use_conn) {
      u32 ca = connected_count(a), cb = connected_count(b);
      if (ca != cb) return ca > cb;
    }
    if (occ[a] != occ[b]) return occ[a] > occ[b];
    if (head_pos[a] != head_pos[b]) return head_pos[a] < head_pos[b];
    return first[a] < first[b];
  };
  std::vector<u32> cand;
  if (delta_atom >= 0) {
    for (auto& t : r.body[delta_atom].t)
      if (t.var && std::find(cand.begin(), cand.end(), t.v) == cand.end()) cand.push_back(t.v);
  } else {
    cand = vars;
  }
  // Delta-first with the head's leading variables: when the delta atom's
  // leading columns are the head's leading variables (all but at most its
  // last), taking them first reads the delta in its stored order and emits
  // rows grouped by all but the last head column, which the grouped sort
  // orders without the radix passes.
  if (delta_atom >= 0 && r.head.t.size() >= 2) {
    const auto& dt = r.body[delta_atom].t;
    std::vector<u32> pre;
    for (size_t j = 0; j < dt.size() && j < r.head.t.size(); ++j) {
      if (!dt[j].var || !r.head.t[j].var || dt[j].v != r.head.t[j].v) break;
      if (std::find(pre.begin(), pre.end(), dt[j].v) != pre.end()) break;
      pre.push_back(dt[j].v);
    }
    if (pre.size() + 1 >= r.head.t.size()) {
      for (u32 v : pre) {
        order.push_back(v);
        bound[v] = true;
      }
    }
  }
  if (order.empty()) {
    u32 root = cand[0];
    for (u32 v : cand)
      if (better(v, root, false)) root = v;
    order.push_back(root);
    bound[root] = true;
  }
  while (order.size() < vars.size()) {
    int best = -1;
    bool any_conn = false;
    for (u32 v : vars)
      if (!bound[v] && connected_count(v) > 0) any_conn = true;
    for (u32 v : vars) {
      if (bound[v]) continue;
      if (any_conn && connected_count(v) == 0) continue;
      if (best < 0 || better(v, (u32)best, true)) best = (int)v;
    }
    order.push_back((u32)best);
    bound[best] = true;
  }
  return order;
}

// ---------------------------------------------------------------------------
// Cost-model variable order (the paper's future work on variable orders,
// Sec. 9).  Statistics: rows and distinct values per column of every body
// relation (one sort per column, cached while the row count is unchanged).
// Estimate for an order, under independence: a level's candidates are the
// bindings of the level above times the smallest per-binding fan-out among
// the atoms holding its variable (the intersection's driver); the other
// atoms keep a fraction fan-out / domain of them, and a comparison between
// bound variables keeps half.  Cost = candidates over all levels weighted by
// the sources each candidate is probed in, plus the output rows times the
// cost of sorting them (none when emitted in order, less when grouped by
// all but the last head column).  Delta-first as in the heuristic (Sec.
// 7.3): the root is one of the delta atom's variables.
// ---------------------------------------------------------------------------

const std::vector<u64>& relation_ndv(Engine* e, u32 rel) {
  Relation& R = e->rels[rel];
  auto it = e->col_stats.find(rel);
  if (it != e->col_stats.end() && it->second.first == R.full.n) return it->second.second;
  std::vector<u64> ndv(R.arity, 0);
  for (u32 c = 0; c < R.arity && R.full.n; ++c) {
    const u32 pos = (u32)(std::find(R.full.order.begin(), R.full.order.end(), c) - R.full.order.begin());
    std::vector<const u32*> in{R.full.col[pos].get()};
    ndv[c] = sort_rows(e, 0, {0u}, in, R.full.n, true).n;
  }
  auto& slot = e->col_stats[rel];
  slot = {R.full.n, std::move(ndv)};
  return slot.second;
}

// Estimated (join work, output sort work) of an order.
std::pair<double, double> order_cost(const Rule& r, int delta_atom, const std::vector<u32>& order,
                                     const std::vector<std::vector<u64>>& ndv,
                                     const std::vector<double>& rows) {
  const u32 nv = r.nvars;
  std::vector<bool> bound(nv, false);
  // Domain estimate per variable: the most distinct values any atom has for it.
  std::vector<double> dom(nv, 1.0);
  for (size_t a = 0; a < r.body.size(); ++a)
    for (size_t c = 0; c < r.body[a].t.size(); ++c)
      if (r.body[a].t[c].var) dom[r.body[a].t[c].v] = std::max(dom[r.body[a].t[c].v], (double)ndv[a][c]);
  double n = 1.0, cost = 0.0;
  for (u32 v : order) {
    // Per-binding fan-out of v in every atom holding it.
    std::vector<double> fan;
    for (size_t a = 0; a < r.body.size(); ++a) {
      bool has = false;
      double sel = rows[a];
      for (size_t c = 0; c < r.body[a].t.size(); ++c) {
        const Term& t = r.body[a].t[c];
        if (t.var && t.v == v) has = true;
        else if (!t.var || bound[t.v]) sel /= std::max<double>(1.0, (double)ndv[a][c]);
      }
      if (!has) continue;
      double nd = 1.0;
      for (size_t c = 0; c < r.body[a].t.size(); ++c)
        if (r.body[a].t[c].var && r.body[a].t[c].v == v) nd = std::max(nd, (double)ndv[a][c]);
      fan.push_back(std::max(std::min(sel, nd), 1e-9));
    }
    std::sort(fan.begin(), fan.end());
    const double examined = n * fan[0];
    cost += examined * (double)fan.size();
    double keep = fan[0];
    for (size_t i = 1; i < fan.size(); ++i) keep *= std::min(1.0, fan[i] / dom[v]);
    bound[v] = true;
    for (auto& c : r.cmps)
      if (c.a.var && c.b.var && (c.a.v == v || c.b.v == v) && bound[c.a.v] && bound[c.b.v]) keep *= 0.5;
    n *= keep;
  }
  // Output order: rows in head order need no sort; grouped by all but the
  // last head column, a cheap one; else the radix passes.
  u32 prefix = 0;
  for (size_t h = 0; h < r.head.t.size() && h < order.size(); ++h) {
    if (!r.head.t[h].var || r.head.t[h].v != order[h]) break;
    ++prefix;
  }
  const size_t hk = r.head.t.size();
  const double sort_cost = delta_atom < 0 && prefix == hk && hk == order.size() ? 0.0
                           : prefix + 1 >= hk ? 1.0 : 6.0;
  return {cost, n * sort_cost};
}

// Lowest-cost connected order; the incumbent (the heuristic's order) is kept
// unless the estimate's total is lower and its join work below a quarter of
// the incumbent's: independence estimates miss skew (hub-heavy graphs), so
// only a large predicted gain overrides the structural choice.
std::vector<u32> cost_order(Engine* e, const Rule& r, int delta_atom,
                            const std::vector<u32>& incumbent) {
  std::vector<std::vector<u64>> ndv;
  std::vector<double> rows;
  for (size_t a = 0; a < r.body.size(); ++a) {
    const Relation& R = e->rels[r.body[a].rel];
    ndv.push_back(relation_ndv(e, r.body[a].rel));
    // A delta is estimated at the relation's size: the first round's delta
    // is the whole relation.
    rows.push_back(std::max<double>(1.0, (double)R.full.n));
  }
  std::vector<u32> vars;
  for (auto& a : r.body)
    for (auto& t : a.t)
      if (t.var && std::find(vars.begin(), vars.end(), t.v) == vars.end()) vars.push_back(t.v);
  std::vector<u32> roots;
  if (delta_atom >= 0) {
    for (auto& t : r.body[delta_atom].t)
      if (t.var && std::find(roots.begin(), roots.end(), t.v) == roots.end()) roots.push_back(t.v);
  } else {
    roots = vars;
  }
  std::vector<u32> best, cur;
  double best_cost = std::numeric_limits<double>::infinity(), best_join = 0;
  std::vector<bool> used(r.nvars, false);
  auto connected = [&](u32 w) {  // w shares an atom with a bound variable
    for (auto& a : r.body) {
      bool hw = false, hb = false;
      for (auto& t : a.t)
        if (t.var) {
          if (t.v == w) hw = true;
          else if (used[t.v]) hb = true;
        }
      if (hw && hb) return true;
    }
    return false;
  };
  std::function<void()> dfs = [&] {
    if (cur.size() == vars.size()) {
      const auto c = order_cost(r, delta_atom, cur, ndv, rows);
      if (c.first + c.second < best_cost) best_cost = c.first + c.second, best_join = c.first, best = cur;
      return;
    }
    for (u32 v : (cur.empty() ? roots : vars)) {
      if (used[v]) continue;
      if (!cur.empty()) {
        // Only variables that share an atom with a bound one, while any do.
        bool any = false;
        for (u32 w : vars)
          if (!used[w] && connected(w)) any = true;
        if (any && !connected(v)) continue;
      }
      used[v] = true;
      cur.push_back(v);
      dfs();
      cur.pop_back();
      used[v] = false;
    }
  };
  dfs();
  if (incumbent.size() == vars.size()) {
    const auto inc = order_cost(r, delta_atom, incumbent, ndv, rows);
    if (!(best_cost < inc.first + inc.second && best_join * 4.0 < inc.first)) return incumbent;
  }
  return best;
}

// Build a version of rule `ri` with atom `delta_atom` read from the delta (or
// -1 for none).  Pointers are filled later.
Version plan_version(Engine* e, u32 ri, int delta_atom, u32 flags) {
  const Rule r = normalize(e->rules[ri]);
  Version v;
  v.rule = ri;
  v.delta_atom = delta_atom;
  v.head_rel = r.head.rel;
  v.level_var = choose_order(r, delta_atom);
  if ((flags & WCDL_F_COST_PLANNER) && r.var_order.empty() && !(e->cfg.flags & WCDL_F_BATCHED) &&
      !e->serving) {
    std::vector<u32> o = cost_order(e, r, delta_atom, v.level_var);
    if (o.size() == v.level_var.size()) v.level_var = std::move(o);
  }
  const u32 m = (u32)v.level_var.size();
  if (m == 0) throw Error(WCDL_E_UNSUPPORTED, "rule without body variables");
  if (m > (u32)MAXV) throw Error(WCDL_E_UNSUPPORTED, "rule has more than 8 variables");
  if (r.body.size() > (size_t)MAXN) throw Error(WCDL_E_UNSUPPORTED, "rule has more than 8 body atoms");
  std::vector<int> level_of(r.nvars, -1);
  for (u32 L = 0; L < m; ++L) level_of[v.level_var[L]] = (int)L;

  DPlan& P = v.plan;
  memset(&P, 0, sizeof(P));
  P.m = m;
  P.natoms = (u32)r.body.size();
  // Atom index orders: constants first, then variables by level.
  for (size_t ai = 0; ai < r.body.size(); ++ai) {
    const Atom& a = r.body[ai];
    AtomUse u;
    u.rel = a.rel;
    u.delta = ((int)ai == delta_atom);
    std::vector<u32> cols(a.t.size());
    std::iota(cols.begin(), cols.end(), 0u);
    std::stable_sort(cols.begin(), cols.end(), [&](u32 x, u32 y) {
      int kx = a.t[x].var ? level_of[a.t[x].v] : -1;
      int ky = a.t[y].var ? level_of[a.t[y].v] : -1;
      return kx < ky;
    });
    for (u32 c : cols) {
      u.order.push_back(c);
      if (a.t[c].var) {
        u.pos_var.push_back((int)a.t[c].v);
        u.pos_const.push_back(0);
      } else {
        u.pos_var.push_back(-1);
        u.pos_const.push_back(a.t[c].v);
        u.nconst++;
      }
    }
    P.atom_nconst[ai] = u.nconst;
    for (u32 c = 0; c < u.nconst; ++c) P.atom_const[ai][c] = u.pos_const[c];
    v.atoms.push_back(u);
  }
  // Levels: sources, bounds, filters.
  v.src_pos.assign(m, {});
  for (u32 L = 0; L < m; ++L) {
    DLevel& lv = P.lvl[L];
    for (u32 a = 0; a < (u32)MAXN; ++a) lv.atom_src[a] = NONE;
    for (size_t ai = 0; ai < v.atoms.size(); ++ai) {
      const AtomUse& u = v.atoms[ai];
      for (size_t p = 0; p < u.pos_var.size(); ++p) {
        if (u.pos_var[p] == (int)v.level_var[L]) {
          DSource& s = lv.src[lv.nsrc];
          s.atom = (u32)ai;
          s.last = (p + 1 == u.pos_var.size()) ? 1u : 0u;
          v.src_pos[L].push_back((u32)p);
          lv.atom_src[ai] = lv.nsrc;
          lv.nsrc++;
        }
      }
    }
  }
  auto operand = [&](const Term& t) {
    DOperand o;
    o.is_var = t.var ? 1u : 0u;
    o.v = t.var ? (u32)level_of[t.v] : t.v;
    return o;
  };
  for (const Cmp& c : r.cmps) {
    int la = c.a.var ? level_of[c.a.v] : -1;
    int lb = c.b.var ? level_of[c.b.v] : -1;
    if (la < 0 && lb < 0) {
      bool ok = c.op == OP_LT ? c.a.v < c.b.v : c.op == OP_LE ? c.a.v <= c.b.v : c.a.v != c.b.v;
      if (!ok) v.dead = true;
      continue;
    }
    if (c.a.var && c.b.var && c.a.v == c.b.v) {
      if (c.op != OP_LE) v.dead = true;
      continue;
    }
    const int L = std::max(la, lb);
    DLevel& lv = P.lvl[L];
    const bool a_is_level = (la == L);
    const Term& other = a_is_level ? c.b : c.a;
    if (c.op == OP_NE) {
      if (lv.nne >= (u32)MAXF) throw Error(WCDL_E_UNSUPPORTED, "too many != filters on one variable");
      lv.ne[lv.nne++] = operand(other);
      continue;
    }
    if (lv.nbnd >= (u32)MAXB) throw Error(WCDL_E_UNSUPPORTED, "too many bounds on one variable");
    DBound& b = lv.bnd[lv.nbnd++];
    b.o = operand(other);
    b.adj = (c.op == OP_LT) ? 1u : 0u;
    b.is_hi = a_is_level ? 1u : 0u;  // x_L < other -> upper bound; other < x_L -> lower
  }
  // Range slots and aliases.  The range of an atom after binding levels
  // 0..b depends only on its sorted copy, its constants and the variables
  // bound in its leading columns; atoms agreeing on all three share a slot.
  auto range_key = [&](size_t ai, int b) {
    const AtomUse& u = v.atoms[ai];
    std::vector<u64> key{u.rel, u.delta ? 1ull : 0ull};
    for (u32 c : u.order) key.push_back(c);
    key.push_back(0xffffffffull);
    for (size_t p = 0; p < u.pos_var.size(); ++p) {
      if (u.pos_var[p] < 0) key.push_back(((u64)1 << 40) | u.pos_const[p]);
      else if (level_of[u.pos_var[p]] <= b) key.push_back(u.pos_var[p]);
    }
    return key;
  };
  auto consumed = [&](size_t ai, int b) {
    u32 c = 0;
    for (int pv : v.atoms[ai].pos_var)
      if (pv >= 0 && level_of[pv] <= b) ++c;
    return c;
  };
  auto nvarcols = [&](size_t ai) {
    u32 c = 0;
    for (int pv : v.atoms[ai].pos_var)
      if (pv >= 0) ++c;
    return c;
  };
  for (u32 b = 0; b < m; ++b) {
    std::vector<std::vector<u64>> keys;
    P.nslot[b] = 0;
    for (u32 ai = 0; ai < (u32)MAXN; ++ai) P.atom_slot[b][ai] = NONE, P.slot_atom[b][ai] = NONE;
    for (size_t ai = 0; ai < v.atoms.size(); ++ai) {
      const u32 cb = consumed(ai, (int)b);
      if (cb == 0 || cb == nvarcols(ai)) continue;  // unnarrowed, or closed
      auto key = range_key(ai, (int)b);
      size_t k = std::find(keys.begin(), keys.end(), key) - keys.begin();
      if (k == keys.size()) {
        keys.push_back(key);
        P.slot_atom[b][k] = (u32)ai;
        P.nslot[b]++;
      }
      P.atom_slot[b][ai] = (u32)k;
    }
  }
  for (u32 L = 0; L < m; ++L) {
    DLevel& lv = P.lvl[L];
    for (u32 s2 = 0; s2 < lv.nsrc; ++s2) {
      DSource& src = lv.src[s2];
      src.alias = NONE;
      src.dir = nullptr;
      src.dmax = 0;
      const size_t ai = src.atom;
      auto k2 = range_key(ai, (int)L - 1);
      for (u32 s1 = 0; s1 < s2 && src.alias == NONE; ++s1)
        if (range_key(lv.src[s1].atom, (int)L - 1) == k2) src.alias = s1;
    }
  }
  // Root: the delta atom's source at level 0 if it has one there, else the
  // first level-0 source.
  {
    const DLevel& l0 = P.lvl[0];
    P.root_src = 0;
    if (delta_atom >= 0 && l0.atom_src[delta_atom] != NONE) {
      P.root_src = l0.atom_src[delta_atom];
    } else if ((flags & WCDL_F_COST_PLANNER) && !(e->cfg.flags & WCDL_F_BATCHED) && !e->serving) {
      // Cost planner: enumerate the root from the source with the fewest
      // distinct values of the root variable.
      u64 best = ~0ull;
      for (u32 s2 = 0; s2 < l0.nsrc; ++s2) {
        const Atom& a = r.body[l0.src[s2].atom];
        const std::vector<u64>& nd = relation_ndv(e, a.rel);
        for (size_t c = 0; c < a.t.size(); ++c)
          if (a.t[c].var && a.t[c].v == v.level_var[0] && nd[c] < best) {
            best = nd[c];
            P.root_src = s2;
          }
      }
    }
  }
  // Sources read through a dense directory: the first column of a copy that
  // nothing has narrowed yet (no constants, no earlier variable).
  v.want_dir.assign(m, {});
  for (u32 L = 0; L < m; ++L) {
    const DLevel& lv = P.lvl[L];
    for (u32 s2 = 0; s2 < lv.nsrc; ++s2) {
      const DSource& src = lv.src[s2];
      bool want = v.src_pos[L][s2] == 0 && v.atoms[src.atom].nconst == 0 && src.alias == NONE &&
                  !(L == 0 && s2 == P.root_src);
      v.want_dir[L].push_back(want);
    }
  }
  // Head.
  P.head_arity = (u32)r.head.t.size();
  bool sorted = (P.head_arity == m);
  u32 prefix = 0;
  for (u32 h = 0; h < P.head_arity; ++h) {
    P.head[h] = operand(r.head.t[h]);
    if (!(P.head[h].is_var && P.head[h].v == h)) sorted = false;
    if (prefix == h && P.head[h].is_var && P.head[h].v == h) ++prefix;
  }
  v.sorted_output = sorted;
  v.sorted_prefix = prefix;
  // Fast paths.
  if (m >= 2) {
    const DLevel& leaf = P.lvl[m - 1];
    P.leaf_fast = (leaf.nsrc == 1 && leaf.src[0].last && leaf.nne == 0) ? 1u : 0u;
    bool xp = !(flags & WCDL_F_XPROD_OFF);
    for (u32 L = 1; L < m && xp; ++L) {
      const DLevel& lv = P.lvl[L];
      if (lv.nsrc != 1 || lv.nbnd || lv.nne || !lv.src[0].last) { xp = false; break; }
      // The atom may only hold x_0 and x_L.
      for (int pv : v.atoms[lv.src[0].atom].pos_var)
        if (pv >= 0 && level_of[pv] != 0 && level_of[pv] != (int)L) xp = false;
    }
    P.xprod = xp ? 1u : 0u;
  }
  // Negated atoms: searched in a copy ordered constants first, then
  // variables by level, at the level that binds their last variable.
  {
    struct NegPlan { u32 level; AtomUse u; };
    std::vector<NegPlan> np;
    for (const Atom& a : r.negs) {
      NegPlan x;
      x.u.rel = a.rel;
      std::vector<u32> cols(a.t.size());
      std::iota(cols.begin(), cols.end(), 0u);
      std::stable_sort(cols.begin(), cols.end(), [&](u32 c1, u32 c2) {
        int k1 = a.t[c1].var ? level_of[a.t[c1].v] : -1;
        int k2 = a.t[c2].var ? level_of[a.t[c2].v] : -1;
        return k1 < k2;
      });
      x.level = 0;
      for (u32 c : cols) {
        x.u.order.push_back(c);
        x.u.pos_var.push_back(a.t[c].var ? (int)a.t[c].v : -1);
        x.u.pos_const.push_back(a.t[c].var ? 0u : a.t[c].v);
        if (a.t[c].var) x.level = std::max<u32>(x.level, (u32)level_of[a.t[c].v]);
      }
      np.push_back(x);
    }
    std::stable_sort(np.begin(), np.end(), [](const NegPlan& a, const NegPlan& b) { return a.level < b.level; });
    P.nneg = (u32)np.size();
    for (u32 k = 0; k < np.size(); ++k) {
      DNeg& ng = P.neg[k];
      ng.ncols = (u32)np[k].u.order.size();
      ng.level = np[k].level;
      for (u32 j = 0; j < ng.ncols; ++j) {
        const int pv = np[k].u.pos_var[j];
        ng.val[j].is_var = pv >= 0 ? 1u : 0u;
        ng.val[j].v = pv >= 0 ? (u32)level_of[pv] : np[k].u.pos_const[j];
      }
      P.lvl[ng.level].nneg++;
      v.negs.push_back(np[k].u);
    }
    if (P.nneg) {
      P.xprod = 0;
      if (P.lvl[m - 1].nneg) P.leaf_fast = 0;
    }
  }
  // LDS layout of the level buffers 0..m-2.
  auto layout = [&](u32 cap) {
    u32 w = 0;
    for (u32 b = 0; b + 1 < m; ++b) {
      P.off_val[b] = w; w += (b + 1) * cap;
      P.off_lo[b] = w; w += P.nslot[b] * cap;
      P.off_hi[b] = w; w += P.nslot[b] * cap;
      P.off_drv[b] = w; w += cap;
      P.off_clo[b] = w; w += cap;
      P.off_chi[b] = w; w += cap;
      w = (w + 1) & ~1u;
      P.off_pre[b] = w; w += 2 * cap;
    }
    return w;
  };
  // One workgroup's worth of items per buffer: the join is bound by memory
  // latency, so LDS goes to more resident workgroups rather than to longer
  // buffers (measured on the triangle join: 17% faster than 512 items).
  const u32 cap = 256;
  u32 words = layout(cap);
  if (words * 4 > 150 * 1024) throw Error(WCDL_E_UNSUPPORTED, "join too deep for LDS; split the rule");
  // A survivor buffer lets every thread write whole rows; it is added only
  // where it costs no resident workgroup (160 KB of LDS per CU; each
  // workgroup's share, static state included, counted in whole KB, which is
  // what the 4-clique plan measures: 32.6 KB per workgroup left 4 resident,
  // not 5; more than 6 per CU do not fit the registers anyway).
  P.off_emit = NONE;
  {
    auto per_cu = [](u32 bytes) { return (160u * 1024u) / ((bytes + 1024u + 1023u) / 1024u * 1024u); };
    const u32 extra = EMIT_ROWS + EMIT_ROWS / 4;
    if (per_cu((words + extra) * 4) >= std::min(per_cu(words * 4), 6u)) {
      P.off_emit = words;
      words += extra;
    }
  }
  P.cap = cap;
  P.lds_words = words;
  v.lds_bytes = words * 4;
  return v;
}

// ===========================================================================
// Stratification (Tarjan, dependencies first)
// ===========================================================================

// Strongly connected components of the dependency graph (head -> every body
// and negated relation), dependencies first.
std::vector<std::vector<u32>> strata_of(u32 n, const std::vector<Rule>& rules) {
  std::vector<std::vector<u32>> dep(n);
  for (auto& r : rules) {
    for (auto& a : r.body) dep[r.head.rel].push_back(a.rel);
    for (auto& a : r.negs) dep[r.head.rel].push_back(a.rel);
  }
  std::vector<int> idx(n, -1), low(n, 0);
  std::vector<bool> on(n, false);
  std::vector<u32> st;
  std::vector<std::vector<u32>> out;
  int counter = 0;
  std::function<void(u32)> go = [&](u32 v) {
    idx[v] = low[v] = counter++;
    st.push_back(v);
    on[v] = true;
    for (u32 w : dep[v]) {
      if (idx[w] < 0) {
        go(w);
        low[v] = std::min(low[v], low[w]);
      } else if (on[w]) {
        low[v] = std::min(low[v], idx[w]);
      }
    }
    if (low[v] == idx[v]) {
      std::vector<u32> comp;
      for (;;) {
        u32 w = st.back();
        st.pop_back();
        on[w] = false;
        comp.push_back(w);
        if (w == v) break;
      }
      std::sort(comp.begin(), comp.end());
      out.push_back(comp);
    }
  };
  for (u32 v = 0; v < n; ++v)
    if (idx[v] < 0) go(v);
  return out;
}

std::vector<std::vector<u32>> strata(Engine* e) { return strata_of((u32)e->rels.size(), e->rules); }

// Stratified negation: no rule may negate a relation of its own head's
// component (the negated relation must be complete before the rule runs).
void check_stratified(u32 nrels, const std::vector<Rule>& rules) {
  std::vector<u32> comp(nrels, 0);
  const auto sc = strata_of(nrels, rules);
  for (u32 c = 0; c < sc.size(); ++c)
    for (u32 rel : sc[c]) comp[rel] = c;
  for (auto& r : rules)
    for (auto& a : r.negs)
      if (comp[a.rel] == comp[r.head.rel])
        throw Error(WCDL_E_UNSUPPORTED, "program not stratifiable: a rule negates a relation "
                                        "that depends on its head");
}

// ===========================================================================
// Evaluation of a batch of rule versions (phase-aligned across streams)
// ===========================================================================

struct Stats {
  double phase[WCDL_N_PHASES] = {0};
  u64 candidates = 0;
  u64 units = 0;
  double kernel_ms[4] = {0};
  u64 launches[4] = {0};
  u64 examined = 0;
  u64 exam_level[MAXV] = {0};
  u64 bound_bytes = 0;  // bytes of candidate rows counted by count passes
};

// Serving: instances whose count-pass rows exceed the per-instance cap.
struct Rejected : Error {
  std::vector<u32> ids;
  explicit Rejected(std::vector<u32> v)
      : Error(WCDL_E_BUDGET, "instances over the per-instance memory cap"), ids(std::move(v)) {}
};

// HIP events around one kernel launch on its stream; read after a sync.
struct KernelTimer {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = -1;
  void start(hipStream_t s, int k) {
    kind = k;
    WCDL_HIP(hipEventCreate(&a));
    WCDL_HIP(hipEventCreate(&b));
    WCDL_HIP(hipEventRecord(a, s));
  }
  void stop(hipStream_t s) { WCDL_HIP(hipEventRecord(b, s)); }
  void collect(Stats& st) {
    if (kind < 0) return;
    float ms = 0;
    WCDL_HIP(hipEventElapsedTime(&ms, a, b));
    st.kernel_ms[kind] += ms;
    st.launches[kind] += 1;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    kind = -1;
  }
  ~KernelTimer() {
    if (kind >= 0) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t).count();
}

// Dense directory over column 0 of a copy, when its values are dense enough
// (largest value at most 4 rows per row plus slack).  Built once per copy.
void ensure_directory(Engine* e, Cols& c) {
  if (c.dir_tried || c.n == 0) return;
  c.dir_tried = true;
  // The copy may still be being written on stream 0: read it there.
  u32 vmax = 0;
  WCDL_HIP(hipMemcpyAsync(&vmax, c.col[0].get() + (c.n - 1), sizeof(u32), hipMemcpyDeviceToHost,
                          e->streams[0]));
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  if ((u64)vmax > 4 * c.n + 4096) return;
  c.dir = DBuf<u32>(e->mem.get(), (u64)vmax + 2);
  c.dir_max = vmax;
  build_directory(ctx(e), c.col[0].get(), c.n, vmax, c.dir.get());
}

// Run bitmaps of a copy that leaf levels probe (see Cols).  Built once per
// copy; only for copies that stay unchanged while they are read.
u32 run_bitmap_min(const Engine* e) { return e->cfg.bitmap_min_run ? e->cfg.bitmap_min_run : 512u; }

void ensure_run_bitmaps(Engine* e, Cols& c) {
  if (c.bm_tried || c.n < run_bitmap_min(e) || c.arity() < 2) return;
  c.bm_tried = true;
  const u32 k = c.arity();
  // Upper bound of the last column: the OR of its values.
  DBuf<u32> d_or(e->mem.get(), 1);
  const u32* last = c.col[k - 1].get();
  column_or(ctx(e), 1, &last, c.n, d_or.get());
  u32 orv = 0;
  WCDL_HIP(hipMemcpyAsync(&orv, d_or.get(), sizeof(u32), hipMemcpyDeviceToHost, e->streams[0]));
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  const u32 vmax = orv == 0 ? 0 : (orv >= 0x80000000u ? 0xffffffffu : (2u << (31 - __builtin_clz(orv))) - 1);
  size_t free_b = 0, total_b = 0;
  WCDL_HIP(hipMemGetInfo(&free_b, &total_b));
  const u64 budget = std::min<u64>((u64)(total_b * 0.02), (u64)(free_b / 8));
  auto cp = c.ptrs();
  c.bm_min = build_run_bitmaps(ctx(e), k, cp.data(), c.n, vmax, run_bitmap_min(e), budget, &c.bm_at,
                               &c.bm, &c.bm_words);
}

void flush_head(Engine* e, u32 rel, Stats* st);

// The sorted copy of (relation, delta?, order) a version reads; built on
// demand from the canonical copy.
Cols& get_cols(Engine* e, u32 rel, bool delta, const std::vector<u32>& order) {
  Relation& R = e->rels[rel];
  const std::vector<u32> canon = canonical(R.arity);
  if (!delta) {
    if (R.head.n) flush_head(e, rel, nullptr);  // joins read one sorted run
    if (order == canon) return R.full;
    auto it = R.full_ord.find(order);
    if (it == R.full_ord.end()) it = R.full_ord.emplace(order, reorder(e, 0, R.full, order)).first;
    return it->second;
  }
  auto it = R.delta_ord.find(order);
  if (it == R.delta_ord.end()) {
    auto ct = R.delta_ord.find(canon);
    if (ct == R.delta_ord.end()) throw Error(WCDL_E_STATE, "delta not available");
    it = R.delta_ord.emplace(order, reorder(e, 0, ct->second, order)).first;
  }
  return it->second;
}

// Per-version evaluation state across the phases of one batch.
struct VRun {
  Version* v = nullptr;
  size_t si = 0;
  bool skip = false;
  DPlan* host_plan = nullptr;  // pinned staging copy
  DBuf<DPlan> d_plan;
  DBuf<u32> rng0;
  DBuf<u32> flags;
  DBuf<u64> pos;
  DBuf<u32> U, S;
  DBuf<u64> W, C;
  DBuf<u32> klo, kd;
  DBuf<u64> counts, offsets;
  DBuf<u64> cand;  // candidates examined per level (materialize)
  bool staged = false;
  std::vector<DBuf<u32>> stage;
  DBuf<u64> chunk_tag, stage_next;
  DBuf<u32> ovf;
  u64 stage_chunks = 0, used_chunks = 0;
  std::vector<u32> overflowed;
  DBuf<u32> d_overflowed;
  u64* scal = nullptr;  // [0] K, [1] T, [2] total, [3] materialize error flag
                        // (4 words of the batch's scalar array)
  u64 K = 0, T = 0, total = 0;
  u64 out_off = 0;
  RootSpace rs{};
  Partition part{};
  u32 root_atom = 0, root_pos = 0;
  KernelTimer t_hist, t_count, t_mat;
};

constexpr u64 NCU = 256;
constexpr u64 MAX_WORKGROUPS = 1ull << 22;

// All streams idle: blocks freed so far may be handed out again.
void recycle(Engine* e) { sync_all(e); }

// Chunked materialization needs every workgroup's rows to fit one chunk.  If
// one does not, split [0,T) into finer slices and count again (without
// staging), up to one unit per workgroup.
void repartition(Engine* e, VRun& R, u64 max_rows, Stats& st) {
  Ctx c = ctx(e, R.si);
  for (;;) {
    const u64 p = R.part.p;
    std::vector<u64> cnt(p);
    WCDL_HIP(hipMemcpy(cnt.data(), R.counts.get(), p * sizeof(u64), hipMemcpyDeviceToHost));
    const u64 worst = *std::max_element(cnt.begin(), cnt.end());
    if (worst <= max_rows) return;
    const u64 cap = std::min<u64>(R.T, MAX_WORKGROUPS);
    if (R.part.balance_off || p >= cap)
      throw Error(WCDL_E_BUDGET, "a single work slice produces " + std::to_string(worst) +
                                     " rows, beyond the chunk budget (consider wcdl_split_rule)");
    u64 np = std::min<u64>(cap, p * std::max<u64>(2, 2 * ceil_div(worst, max_rows)));
    const u64 slice = ceil_div(R.T, np);
    np = ceil_div(R.T, slice);
    R.part = Partition{np, slice, 0, 0};
    // Staged rows belong to the old partition: drop them.
    R.staged = false;
    R.stage.clear();
    R.chunk_tag.reset();
    R.ovf.reset();
    R.overflowed.clear();
    R.used_chunks = 0;
    DPlan& P = R.v->plan;
    P.cand = nullptr;
    *R.host_plan = P;
    WCDL_HIP(hipMemcpyAsync(R.d_plan.get(), R.host_plan, sizeof(DPlan), hipMemcpyHostToDevice, c.s));
    R.counts = DBuf<u64>(c.mem, np);
    R.offsets = DBuf<u64>(c.mem, np);
    auto t = Clock::now();
    join_run(c, R.d_plan.get(), R.rs, R.part, R.v->lds_bytes, 0, R.counts.get(), nullptr, 0, np);
    scan_u64_excl(c, R.counts.get(), R.offsets.get(), np, R.scal + 2);
    recycle(e);
    st.phase[WCDL_PH_COUNT] += ms_since(t);
  }
}

// Device bytes held by every stored copy of every relation (loaded facts,
// full relation and head run, other column orders, deltas).
u64 resident_bytes(const Engine* e) {
  u64 b = 0;
  for (const auto& R : e->rels) {
    u64 rows = R.base.n + R.full.n + R.head.n;
    for (const auto& kv : R.full_ord) rows += kv.second.n;
    for (const auto& kv : R.delta_ord) rows += kv.second.n;
    b += rows * R.arity * 4ull;
  }
  return b;
}

// Raw head rows of one chunk (canonical column order, unsorted unless
// `presorted`: sorted, unique, above every row of the head's earlier chunks,
// and from the head's only version).  `grouped`: the rows, all from one
// version, are non-decreasing in their first `grouped` columns (repeats are
// possible unless `presorted`).
using Sink = std::function<void(u32 rel, Cols&& rows, bool presorted, u32 grouped)>;

// Evaluate a set of rule versions over the current relations and hand every
// chunk of raw head rows to `sink`.
void eval_batch(Engine* e, std::vector<Version>& vs, Stats& st, const Sink& sink) {
  const bool seq = (e->cfg.flags & WCDL_F_STREAMS_OFF) != 0;
  const u32 flags = e->cfg.flags;
  std::vector<VRun> runs(vs.size());
  static_assert(sizeof(DPlan) < 16384, "plan size");
  // Pinned staging for plans (one slot per version), grown as needed; the
  // streams are idle first, so no upload of an earlier batch (one that ended
  // early by an error included) still reads a slot.
  sync_all(e);
  while (e->plan_staging.size() < vs.size()) {
    void* h = nullptr;
    WCDL_HIP(hipHostMalloc(&h, sizeof(DPlan), hipHostMallocDefault));
    e->plan_staging.push_back(h);
  }

  auto t_index = Clock::now();
  // ---- Inputs: every version's sorted copies.  Missing column orders are
  // built on stream 0 (Build Index); fence it before other streams read them.
  for (size_t i = 0; i < vs.size(); ++i) {
    VRun& R = runs[i];
    Version& v = vs[i];
    R.v = &v;
    R.si = seq ? 0 : i % e->streams.size();
    R.host_plan = static_cast<DPlan*>(e->plan_staging[i]);
    if (v.dead) { R.skip = true; continue; }
    DPlan& P = v.plan;
    for (size_t ai = 0; ai < v.atoms.size(); ++ai) {
      const AtomUse& u = v.atoms[ai];
      Cols& cc = get_cols(e, u.rel, u.delta, u.order);
      if (cc.n == 0) R.skip = true;
      if (cc.n >= 0xffffffffull) throw Error(WCDL_E_UNSUPPORTED, "join source exceeds 2^32-1 rows");
      P.atom_n[ai] = (u32)cc.n;
      for (size_t p = 0; p < u.order.size(); ++p) P.atom_col[ai][p] = cc.col[p].get();
    }
    // Negated atoms read complete relations of lower strata.
    for (size_t k = 0; k < v.negs.size() && !R.skip; ++k) {
      const AtomUse& u = v.negs[k];
      Cols& cc = get_cols(e, u.rel, false, u.order);
      if (cc.n >= 0xffffffffull) throw Error(WCDL_E_UNSUPPORTED, "negated relation exceeds 2^32-1 rows");
      P.neg[k].n = (u32)cc.n;
      for (size_t j = 0; j < u.order.size(); ++j) P.neg[k].col[j] = cc.n ? cc.col[j].get() : nullptr;
    }
    for (u32 L = 0; L < P.m && !R.skip; ++L)
      for (u32 s2 = 0; s2 < P.lvl[L].nsrc; ++s2) {
        DSource& src = P.lvl[L].src[s2];
        src.bm_at = src.bm = nullptr;
        src.bm_words = src.bm_min = 0;
        if (L + 1 == P.m && L > 0 && src.alias == NONE && !v.want_dir[L][s2] && !e->serving &&
            !(e->cfg.flags & WCDL_F_RUN_BITMAPS_OFF)) {
          // Leaf sources of copies that no version of this batch writes.
          const AtomUse& u = v.atoms[src.atom];
          bool stable = !u.delta;
          for (auto& w : vs) stable = stable && w.head_rel != u.rel;
          if (stable) {
            Cols& cc = get_cols(e, u.rel, false, u.order);
            ensure_run_bitmaps(e, cc);
            if (cc.bm_min) {
              src.bm_at = cc.bm_at.get();
              src.bm = cc.bm.get();
              src.bm_words = cc.bm_words;
              src.bm_min = cc.bm_min;
            }
          }
        }
        src.dir = nullptr;
        if (!v.want_dir[L][s2]) continue;
        const AtomUse& u = v.atoms[src.atom];
        Cols& cc = get_cols(e, u.rel, u.delta, u.order);
        ensure_directory(e, cc);
        if (cc.dir.get()) {
          src.dir = cc.dir.get();
          src.dmax = cc.dir_max;
        }
      }
  }
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  st.phase[WCDL_PH_INDEX] += ms_since(t_index);
  auto t_hist = Clock::now();
  // Serving with a per-instance cap: count passes add up each instance's
  // row bytes (indexed by instance id).
  const bool per_instance = e->serving && e->cfg.instance_cap_bytes;
  const bool bounded = e->cfg.mem_budget_bytes != 0;
  DBuf<u64> inst_bytes, bound_acc;
  DBuf<u32> abort_flag;
  const u64 inst_n = (u64)e->max_instance + 1;
  if (per_instance) {
    inst_bytes = DBuf<u64>(e->mem.get(), inst_n);
    fill_u64(ctx(e), inst_bytes.get(), inst_n, 0);
  }
  if (bounded) {
    bound_acc = DBuf<u64>(e->mem.get(), 1);
    fill_u64(ctx(e), bound_acc.get(), 1, 0);
  }
  if (bounded) {
    abort_flag = DBuf<u32>(e->mem.get(), 1);
    fill_u32(ctx(e), abort_flag.get(), 1, 0);
  }
  const u64 held0 = bounded ? resident_bytes(e) : 0;
  // Every version's scalars (K, T, total, error flag) in one array, read back
  // with one copy per phase instead of one per version.
  DBuf<u64> scal_all(e->mem.get(), 4 * runs.size());
  fill_u64(ctx(e), scal_all.get(), 4 * runs.size(), 0);
  std::vector<u64> hscal(4 * runs.size());
  auto read_scalars = [&] {
    WCDL_HIP(hipMemcpy(hscal.data(), scal_all.get(), hscal.size() * sizeof(u64), hipMemcpyDeviceToHost));
  };
  auto scalar_of = [&](const VRun& R, int k) { return hscal[(size_t)(R.scal - scal_all.get()) + k]; };
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  // ---- Phase A: plan upload, constant narrowing, root-key flags.
  for (size_t i = 0; i < vs.size(); ++i) {
    VRun& R = runs[i];
    Version& v = vs[i];
    if (R.skip) continue;
    DPlan& P = v.plan;
    P.inst_bytes = per_instance ? reinterpret_cast<unsigned long long*>(inst_bytes.get()) : nullptr;
    P.inst_n = (u32)inst_n;
    P.inst_cap = e->cfg.instance_cap_bytes;
    P.row_bytes = P.head_arity * 4;
    P.bound_acc = bounded ? reinterpret_cast<unsigned long long*>(bound_acc.get()) : nullptr;
    P.bound_limit = bounded && e->cfg.mem_budget_bytes > held0 ? e->cfg.mem_budget_bytes - held0 : 0;
    P.abort = bounded ? abort_flag.get() : nullptr;
    for (u32 L = 0; L < P.m; ++L)
      for (u32 s = 0; s < P.lvl[L].nsrc; ++s)
        P.lvl[L].src[s].col = P.atom_col[P.lvl[L].src[s].atom][v.src_pos[L][s]];
    R.root_atom = P.lvl[0].src[P.root_src].atom;
    R.root_pos = v.src_pos[0][P.root_src];
    Ctx c = ctx(e, R.si);
    *R.host_plan = P;
    R.d_plan = DBuf<DPlan>(c.mem, 1);
    WCDL_HIP(hipMemcpyAsync(R.d_plan.get(), R.host_plan, sizeof(DPlan), hipMemcpyHostToDevice, c.s));
    R.rng0 = DBuf<u32>(c.mem, 2 * MAXN);
    R.scal = scal_all.get() + 4 * i;
    join_init_ranges(c, R.d_plan.get(), P.natoms, R.rng0.get());
    const u32 n = P.atom_n[R.root_atom];
    R.flags = DBuf<u32>(c.mem, n);
    R.pos = DBuf<u64>(c.mem, n);
    join_root_flags(c, P.atom_col[R.root_atom][R.root_pos], R.rng0.get(), R.root_atom, n,
                    R.flags.get(), R.pos.get(), R.scal);
  }
  sync_all(e);
  read_scalars();
  // ---- Phase B: root keys, histogram, prefix sums.
  for (auto& R : runs) {
    if (R.skip) continue;
    Ctx c = ctx(e, R.si);
    R.K = scalar_of(R, 0);
    if (R.K == 0) { R.skip = true; continue; }
    const DPlan& P = R.v->plan;
    const u32 n = P.atom_n[R.root_atom];
    R.U = DBuf<u32>(c.mem, R.K);
    R.S = DBuf<u32>(c.mem, R.K + 1);
    join_root_compact(c, P.atom_col[R.root_atom][R.root_pos], R.rng0.get(), R.root_atom, n,
                      R.flags.get(), R.pos.get(), R.K, R.U.get(), R.S.get());
    R.W = DBuf<u64>(c.mem, R.K);
    R.C = DBuf<u64>(c.mem, R.K);
    if (P.xprod) {
      R.klo = DBuf<u32>(c.mem, (u64)P.m * R.K);
      R.kd = DBuf<u32>(c.mem, (u64)P.m * R.K);
    }
    R.rs = RootSpace{R.U.get(), R.S.get(), R.C.get(), R.K, 0, R.rng0.get()};
    R.t_hist.start(c.s, 2);
    join_histogram(c, R.d_plan.get(), R.rs, R.W.get(), P.xprod ? R.klo.get() : nullptr,
                   P.xprod ? R.kd.get() : nullptr, P.m);
    R.t_hist.stop(c.s);
    scan_u64_incl(c, R.W.get(), R.C.get(), R.K, R.scal + 1);
  }
  sync_all(e);
  read_scalars();
  st.phase[WCDL_PH_HISTOGRAM] += ms_since(t_hist);
  // ---- Phase C: count pass (Alg. 1 Phase 2) and offsets.
  auto t_count = Clock::now();
  // Staging arenas: each version that ran before asks for its expected rows
  // (x stage_pct); together they get at most a fifth of the device memory
  // (or a quarter of the memory budget), shared in proportion.
  std::map<VRun*, u64> stage_plan;
  if (!(flags & WCDL_F_STAGE_OFF)) {
    const double pct = e->cfg.stage_pct ? e->cfg.stage_pct : 125;
    u64 want_total = 0;
    for (auto& R : runs) {
      if (R.skip || R.v->plan.xprod) continue;
      R.T = scalar_of(R, 1);
      auto rit = e->rows_per_unit.find(std::make_pair(R.v->rule, R.v->delta_atom));
      if (R.T == 0 || rit == e->rows_per_unit.end()) continue;
      const u64 wpc = e->cfg.wg_per_cu ? e->cfg.wg_per_cu : 32;
      const u64 pguess = std::min<u64>(ceil_div(R.T, 64), NCU * wpc);
      const u64 rows = (u64)((double)R.T * rit->second * pct / 100.0) + STAGE_CHUNK * pguess;
      const u64 bytes = ceil_div(rows, STAGE_CHUNK) * STAGE_CHUNK * R.v->plan.head_arity * 4ull;
      stage_plan[&R] = bytes;
      want_total += bytes;
    }
    // With a memory budget the arena shares what the relations leave of it.
    const u64 held = resident_bytes(e), budget = e->cfg.mem_budget_bytes;
    const u64 limit = budget ? (budget > held ? (budget - held) / 2 : 0) : (u64)(e->device_total * 0.2);
    const double scale = want_total > limit ? (double)limit / (double)want_total : 1.0;
    for (auto& kv : stage_plan) {
      const u64 per_chunk = STAGE_CHUNK * kv.first->v->plan.head_arity * 4ull;
      kv.second = (u64)((double)kv.second * scale) / per_chunk;  // now in chunks
    }
  }
  for (auto& R : runs) {
    if (R.skip) continue;
    R.T = scalar_of(R, 1);
    if (R.T == 0) { R.skip = true; continue; }
    R.rs.T = R.T;
    st.units += R.T;
    const DPlan& P = R.v->plan;
    if (P.xprod) {
      R.total = R.T;
      continue;
    }
    Ctx c = ctx(e, R.si);
    u64 p;
    if (flags & WCDL_F_BALANCE_OFF) {
      p = R.K;  // one root key per workgroup (the unbalanced baseline)
      R.part = Partition{p, 0, 1, 0};
    } else {
      const u64 wpc = e->cfg.wg_per_cu ? e->cfg.wg_per_cu : 32;
      p = std::min<u64>(ceil_div(R.T, 64), NCU * wpc);
      if (p == 0) p = 1;
      const u64 slice = ceil_div(R.T, p);
      p = ceil_div(R.T, slice);
      R.part = Partition{p, slice, 0, 0};
    }
    R.counts = DBuf<u64>(c.mem, p);
    R.offsets = DBuf<u64>(c.mem, p);
    // Stage rows during the count pass when the previous run of this rule
    // version tells how many to expect (arena shares across the batch).
    u64 chunks = stage_plan.count(&R) ? stage_plan[&R] : 0;
    if (chunks) {
      const u32 k = P.head_arity;
      if (chunks > 0) {
        try {
          for (u32 h = 0; h < k; ++h) R.stage.emplace_back(c.mem, chunks * STAGE_CHUNK);
          R.chunk_tag = DBuf<u64>(c.mem, chunks);
          R.stage_next = DBuf<u64>(c.mem, 1);
          R.ovf = DBuf<u32>(c.mem, p);
          R.staged = true;
          R.stage_chunks = chunks;
        } catch (const Error& x) {
          if (x.code != WCDL_E_NOMEM) throw;
          R.stage.clear();  // not enough memory: plain two passes
        }
      }
    }
    if (R.staged) {
      DPlan& PM = R.v->plan;
      R.cand = DBuf<u64>(c.mem, MAXV);
      fill_u64(c, R.cand.get(), MAXV, 0);
      PM.cand = R.cand.get();  // the staged count pass does the full traversal
      for (u32 h = 0; h < PM.head_arity; ++h) PM.stage[h] = R.stage[h].get();
      PM.stage_chunks = R.stage_chunks;
      PM.stage_next = R.stage_next.get();
      PM.chunk_tag = R.chunk_tag.get();
      PM.ovf = R.ovf.get();
      fill_u64(c, R.stage_next.get(), 1, 0);
      *R.host_plan = PM;
      WCDL_HIP(hipMemcpyAsync(R.d_plan.get(), R.host_plan, sizeof(DPlan), hipMemcpyHostToDevice, c.s));
    }
    R.t_count.start(c.s, 0);
    join_run(c, R.d_plan.get(), R.rs, R.part, R.v->lds_bytes, R.staged ? 2 : 0, R.counts.get(),
             nullptr, 0, p);
    R.t_count.stop(c.s);
    scan_u64_excl(c, R.counts.get(), R.offsets.get(), p, R.scal + 2);
  }
  sync_all(e);
  read_scalars();
  for (auto& R : runs) {
    if (R.skip || R.v->plan.xprod) continue;
    R.total = scalar_of(R, 2);
    e->rows_per_unit[std::make_pair(R.v->rule, R.v->delta_atom)] = (double)R.total / (double)R.T;
    if (R.staged) {
      WCDL_HIP(hipMemcpy(&R.used_chunks, R.stage_next.get(), sizeof(u64), hipMemcpyDeviceToHost));
      R.used_chunks = std::min(R.used_chunks, R.stage_chunks);
      std::vector<u32> ovf(R.part.p);
      WCDL_HIP(hipMemcpy(ovf.data(), R.ovf.get(), R.part.p * sizeof(u32), hipMemcpyDeviceToHost));
      for (u32 b = 0; b < R.part.p; ++b)
        if (ovf[b]) R.overflowed.push_back(b);
    }
    if (R.total == 0) R.skip = true;
  }
  st.phase[WCDL_PH_COUNT] += ms_since(t_count);
  u32 aborted = 0;
  if (bounded)
    WCDL_HIP(hipMemcpy(&aborted, abort_flag.get(), sizeof(u32), hipMemcpyDeviceToHost));
  if (per_instance) {
    std::vector<u64> hb(inst_n);
    WCDL_HIP(hipMemcpy(hb.data(), inst_bytes.get(), inst_n * sizeof(u64), hipMemcpyDeviceToHost));
    std::vector<u32> over;
    for (u64 id = 0; id < inst_n; ++id)
      if (hb[id] > e->cfg.instance_cap_bytes) over.push_back((u32)id);
    if (!over.empty()) throw Rejected(std::move(over));
  }
  if (aborted)
    throw Error(WCDL_E_BUDGET, "the round's count passes crossed the memory budget of " +
                                   std::to_string(e->cfg.mem_budget_bytes) + " bytes beside " +
                                   std::to_string(held0) + " bytes of relations (stopped early)");
  // Recounts (finer partitions of chunked heads) are not accounted again.
  for (auto& R : runs) {
    R.v->plan.inst_bytes = nullptr;
    R.v->plan.bound_acc = nullptr;
    R.v->plan.abort = nullptr;
  }
  // Memory bound of the round: the counted rows must fit beside the
  // relations within the budget, else nothing of this round is written.
  u64 need = 0;
  for (auto& R : runs)
    if (!R.skip) need += R.total * R.v->plan.head_arity * 4ull;
  st.bound_bytes += need;
  if (e->cfg.mem_budget_bytes) {
    const u64 held = resident_bytes(e);
    if (held + need > e->cfg.mem_budget_bytes)
      throw Error(WCDL_E_BUDGET, "the round's count pass found " + std::to_string(need) +
                                     " bytes of rows beside " + std::to_string(held) +
                                     " bytes of relations, beyond the budget of " +
                                     std::to_string(e->cfg.mem_budget_bytes) + " bytes");
  }
  // ---- Resize: one candidate buffer per head relation.  A head whose rows
  // exceed the chunk budget is materialized in ranges of workgroups (or of
  // units, for cross-product plans) instead, each range deduplicated by the
  // sink before the next one is written (chunked materialization).
  std::map<u32, u64> rows;
  std::map<u32, int> nver;
  bool all_sorted = true;
  for (auto& R : runs) {
    if (R.skip) continue;
    R.out_off = rows[R.v->head_rel];
    rows[R.v->head_rel] += R.total;
    nver[R.v->head_rel]++;
  }
  size_t free_b = 0, total_b = 0;
  WCDL_HIP(hipMemGetInfo(&free_b, &total_b));
  const u64 chunk_bytes = e->cfg.chunk_bytes ? e->cfg.chunk_bytes : (u64)(total_b * 0.06);
  // A head written by one version whose rows come out sorted and unique,
  // into an empty relation, needs no scratch beyond its final size: it is
  // written whole unless that size itself is large against the memory.
  std::map<u32, bool> in_order;
  for (auto& R : runs)
    if (!R.skip) {
      auto it = in_order.find(R.v->head_rel);
      bool ok = nver[R.v->head_rel] == 1 && R.v->sorted_output &&
                e->rels[R.v->head_rel].full.n == 0;
      in_order[R.v->head_rel] = it == in_order.end() ? ok : it->second && ok;
    }
  const u64 direct_bytes = free_b / 2;
  std::set<u32> chunked;
  for (auto& kv : rows) {
    const u64 bytes = kv.second * e->rels[kv.first].arity * 4ull;
    if (bytes > chunk_bytes && !(in_order[kv.first] && bytes <= direct_bytes))
      chunked.insert(kv.first);
  }
  std::map<u32, Cols> whole;
  for (auto& kv : rows) {
    if (chunked.count(kv.first)) continue;
    const u32 k = e->rels[kv.first].arity;
    Cols c;
    c.order = canonical(k);
    c.n = kv.second;
    for (u32 j = 0; j < k; ++j) c.col.emplace_back(e->mem.get(), kv.second);
    whole.emplace(kv.first, std::move(c));
  }
  (void)all_sorted;
  auto set_output = [&](VRun& R, u32* const* base, u64 lo_row, u64 hi_row) {
    // Rows [lo_row, hi_row) of this version land at base[h][row - lo_row].
    DPlan& P = R.v->plan;
    for (u32 h = 0; h < P.head_arity; ++h) P.out[h] = base[h] - lo_row;
    P.out_rows = hi_row;
    P.err = reinterpret_cast<u32*>(R.scal + 3);
    if (R.staged) {
      P.cand = nullptr;  // counted in the staged count pass
    } else {
      if (!R.cand.get()) {
        R.cand = DBuf<u64>(e->mem.get(), MAXV);
        fill_u64(ctx(e, R.si), R.cand.get(), MAXV, 0);
      }
      P.cand = R.cand.get();
    }
    *R.host_plan = P;
    WCDL_HIP(hipMemcpyAsync(R.d_plan.get(), R.host_plan, sizeof(DPlan), hipMemcpyHostToDevice,
                            ctx(e, R.si).s));
  };
  // Write the rows of workgroups [w0, w1) (or units, for cross products).
  auto write_rows = [&](VRun& R, u64 w0, u64 w1) {
    Ctx c = ctx(e, R.si);
    DPlan& P = R.v->plan;
    if (P.xprod) {
      join_xprod(c, R.d_plan.get(), R.rs, R.klo.get(), R.kd.get(), P.m, w0, w1);
    } else if (R.staged) {
      // Staged rows: copy to their offsets; re-run only workgroups whose
      // rows did not all fit in the arena.
      join_stage_copy(c, R.d_plan.get(), R.used_chunks, R.counts.get(), R.offsets.get(),
                      P.head_arity, w0, w1);
      std::vector<u32> redo;
      for (u32 b : R.overflowed)
        if (b >= w0 && b < w1) redo.push_back(b);
      if (!redo.empty()) {
        DBuf<u32> d_redo(c.mem, redo.size());
        WCDL_HIP(hipMemcpyAsync(d_redo.get(), redo.data(), redo.size() * sizeof(u32),
                                hipMemcpyHostToDevice, c.s));
        join_run(c, R.d_plan.get(), R.rs, R.part, R.v->lds_bytes, 1, nullptr, R.offsets.get(), 0,
                 redo.size(), d_redo.get());
        WCDL_HIP(hipStreamSynchronize(c.s));  // `redo` is read by the copy above
      }
    } else {
      join_run(c, R.d_plan.get(), R.rs, R.part, R.v->lds_bytes, 1, nullptr, R.offsets.get(), w0,
               w1 - w0);
    }
  };
  auto check_flag = [&](VRun& R) {
    u64 flag = 0;
    WCDL_HIP(hipMemcpy(&flag, R.scal + 3, sizeof(u64), hipMemcpyDeviceToHost));
    if (flag) throw Error(WCDL_E_DEVICE, "internal error: materialize produced more rows than counted");
  };
  // ---- Phase D: materialize (Alg. 1 Phase 3), whole heads, phase-aligned.
  auto t_mat = Clock::now();
  for (auto& R : runs) {
    if (R.skip || chunked.count(R.v->head_rel)) continue;
    Cols& dst = whole.at(R.v->head_rel);
    std::vector<u32*> base;
    for (u32 h = 0; h < R.v->plan.head_arity; ++h) base.push_back(dst.col[h].get() + R.out_off);
    set_output(R, base.data(), 0, R.total);
    R.t_mat.start(ctx(e, R.si).s, 1);
    write_rows(R, 0, R.v->plan.xprod ? R.T : R.part.p);
    R.t_mat.stop(ctx(e, R.si).s);
    st.candidates += R.total;
  }
  sync_all(e);
  for (auto& R : runs)
    if (!R.skip && !chunked.count(R.v->head_rel)) check_flag(R);
  st.phase[WCDL_PH_MATERIALIZE] += ms_since(t_mat);
  // Rows of one version keep its emission order (Sec. 3.3: each slice's rows
  // at its scanned offset), so a version's sorted prefix holds for its head.
  auto grouped_of = [&](u32 rel) -> u32 {
    if (nver[rel] != 1 || e->serving) return 0;
    for (auto& R : runs)
      if (!R.skip && R.v->head_rel == rel) return R.v->sorted_prefix;
    return 0;
  };
  for (auto& kv : whole) {
    bool sorted = nver[kv.first] == 1;
    for (auto& R : runs)
      if (!R.skip && R.v->head_rel == kv.first) sorted = sorted && R.v->sorted_output;
    const u32 g = grouped_of(kv.first);
    sink(kv.first, std::move(kv.second), sorted, g);
  }
  whole.clear();
  // ---- Chunked heads: one version and one range at a time.
  for (auto& R : runs) {
    if (R.skip || !chunked.count(R.v->head_rel)) continue;
    const u32 k = e->rels[R.v->head_rel].arity;
    const u64 max_rows = std::max<u64>(1, chunk_bytes / (k * 4ull));
    // Ranges [w0, w1) of workgroups (units for cross products) and their rows.
    std::vector<std::pair<u64, u64>> ranges;
    std::vector<u64> offs;
    if (R.v->plan.xprod) {
      for (u64 u = 0; u < R.T; u += max_rows) ranges.push_back({u, std::min(R.T, u + max_rows)});
    } else {
      repartition(e, R, max_rows, st);
      const u64 p = R.part.p;
      offs.resize(p + 1);
      WCDL_HIP(hipMemcpy(offs.data(), R.offsets.get(), p * sizeof(u64), hipMemcpyDeviceToHost));
      offs[p] = R.total;
      u64 w0 = 0;
      while (w0 < p) {
        u64 w1 = w0 + 1;
        if (offs[w1] - offs[w0] > max_rows)
          throw Error(WCDL_E_BUDGET, "one workgroup's rows exceed the chunk budget");
        while (w1 < p && offs[w1 + 1] - offs[w0] <= max_rows) ++w1;
        ranges.push_back({w0, w1});
        w0 = w1;
      }
    }
    for (auto& rg : ranges) {
      auto t_chunk = Clock::now();
      const u64 r0 = R.v->plan.xprod ? rg.first : offs[rg.first];
      const u64 r1 = R.v->plan.xprod ? rg.second : offs[rg.second];
      if (r1 == r0) continue;
      Cols chunk;
      chunk.order = canonical(k);
      chunk.n = r1 - r0;
      std::vector<u32*> base;
      for (u32 j = 0; j < k; ++j) {
        chunk.col.emplace_back(e->mem.get(), chunk.n);
        base.push_back(chunk.col.back().get());
      }
      set_output(R, base.data(), r0, r1);
      KernelTimer t;
      t.start(ctx(e, R.si).s, 1);
      write_rows(R, rg.first, rg.second);
      t.stop(ctx(e, R.si).s);
      sync_all(e);
      check_flag(R);
      t.collect(st);
      st.candidates += chunk.n;
      st.phase[WCDL_PH_MATERIALIZE] += ms_since(t_chunk);
      // Ranges go in workgroup order, so a sorted head's chunks ascend.
      sink(R.v->head_rel, std::move(chunk), in_order[R.v->head_rel], grouped_of(R.v->head_rel));
      recycle(e);
    }
    // The staging arena of this version is no longer needed.
    R.stage.clear();
    R.chunk_tag.reset();
    recycle(e);
  }
  for (auto& R : runs) {
    if (R.skip) continue;
    u64 lv[MAXV];
    if (R.v->plan.xprod) {
      st.examined += R.total;
      st.exam_level[R.v->plan.m - 1] += R.total;
    } else if (R.cand.get()) {
      WCDL_HIP(hipMemcpy(lv, R.cand.get(), sizeof(lv), hipMemcpyDeviceToHost));
      for (int j = 0; j < MAXV; ++j) {
        st.examined += lv[j];
        st.exam_level[j] += lv[j];
      }
    }
  }
  for (auto& R : runs) {
    R.t_hist.collect(st);
    R.t_count.collect(st);
    R.t_mat.collect(st);
  }
}

// Sorted, deduplicated rows of a chunk whose first `grouped` columns are
// already non-decreasing: only repeats to drop when that is every column; a
// bitmap per group in LDS when it is all but the last and the last column's
// values are small against the rows per group; else the radix sort.
Cols sort_unique(Engine* e, Cols rows, u32 grouped) {
  const u32 k = (u32)rows.col.size();
  if (rows.n == 0 || (e->cfg.flags & WCDL_F_GROUPED_SORT_OFF)) grouped = 0;
  if (grouped >= k && k > 0) {
    // Sorted already; repeats remain where the join has levels past the head.
    Ctx c = ctx(e);
    Cols out;
    out.order = rows.order;
    std::vector<u32*> op;
    for (u32 j = 0; j < k; ++j) {
      out.col.emplace_back(c.mem, rows.n);
      op.push_back(out.col.back().get());
    }
    std::vector<const u32*> in(rows.ptrs());
    out.n = unique_rows(c, k, in.data(), rows.n, op.data());
    return out;
  }
  if (k >= 2 && grouped + 1 == k) {
    Ctx c = ctx(e);
    DBuf<u32> d_or(c.mem, 1);
    const u32* last = rows.col[k - 1].get();
    column_or(c, 1, &last, rows.n, d_or.get());
    u32 h_or = 0;
    WCDL_HIP(hipMemcpyAsync(&h_or, d_or.get(), sizeof(u32), hipMemcpyDeviceToHost, c.s));
    WCDL_HIP(hipStreamSynchronize(c.s));
    const u32 zbits = bits_of(h_or);
    if (zbits <= 18) {
      std::vector<const u32*> in(rows.ptrs());
      Cols out;
      out.order = rows.order;
      std::vector<u32*> op;
      for (u32 j = 0; j < k; ++j) {
        out.col.emplace_back(c.mem, rows.n);
        op.push_back(out.col.back().get());
      }
      if (sort_unique_grouped(c, k, in.data(), rows.n, zbits, op.data(), &out.n)) return out;
    }
  }
  if (rows.n >= (1u << 20) && k <= 4 && !(e->cfg.flags & WCDL_F_TILE_DEDUP_OFF)) {
    // Repeats emitted close together go before the radix passes.
    Ctx c = ctx(e);
    Cols fewer;
    fewer.order = rows.order;
    std::vector<u32*> op;
    for (u32 j = 0; j < k; ++j) {
      fewer.col.emplace_back(c.mem, rows.n);
      op.push_back(fewer.col.back().get());
    }
    std::vector<const u32*> in(rows.ptrs());
    fewer.n = drop_tile_repeats(c, k, in.data(), rows.n, op.data());
    rows = std::move(fewer);
  }
  Cols srt = sort_rows(e, 0, rows.order, std::vector<const u32*>(rows.ptrs()), rows.n, true);
  rows = Cols();
  return srt;
}

// Fold one chunk of raw rows of relation `rel` into `acc`, the rows new this
// round: acc += unique(rows) \ full \ acc (Compute Delta, Sec. 4).
void absorb_chunk(Engine* e, u32 rel, Cols&& rows, bool presorted, u32 grouped, Cols& acc,
                  Stats& st) {
  Relation& R = e->rels[rel];
  auto t = Clock::now();
  if (presorted && R.full.n == 0 && R.head.n == 0) {
    // Ascending disjoint chunks: nothing to sort or subtract.
    if (acc.n == 0) acc = std::move(rows);
    else if (rows.n) acc = merged(e, 0, acc, rows);
  } else {
    Cols srt = sort_unique(e, std::move(rows), grouped);
    recycle(e);
    Cols d = difference(e, 0, srt, R.full, &R.head);
    srt = Cols();
    recycle(e);
    if (acc.n == 0) {
      acc = std::move(d);
    } else if (d.n) {
      Cols d2 = difference(e, 0, d, acc);
      if (d2.n) acc = merged(e, 0, acc, d2);
    }
  }
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  st.phase[WCDL_PH_DELTA] += ms_since(t);
}

// Merge the head run into the body and into every other maintained column
// order of it.
void flush_head(Engine* e, u32 rel, Stats* st) {
  Relation& R = e->rels[rel];
  if (R.head.n == 0) return;
  auto t = Clock::now();
  Cols h = std::move(R.head);
  R.head = empty_cols(R.arity, canonical(R.arity));
  if (R.full.n == 0) {
    R.full = std::move(h);
    for (auto& kv : R.full_ord) kv.second = reorder(e, 0, R.full, kv.first);
  } else {
    R.full = merged(e, 0, R.full, h);
    for (auto& kv : R.full_ord) kv.second = merged(e, 0, kv.second, reorder(e, 0, h, kv.first));
  }
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  if (st) st->phase[WCDL_PH_MERGE] += ms_since(t);
}

// Head runs are flushed once they hold more than 1/ratio of the body.
u64 head_ratio(const Engine* e) { return e->cfg.head_ratio ? e->cfg.head_ratio : 8u; }
constexpr u64 HEAD_MIN_ROWS = 1u << 16;

// Merge the new rows into the relation (Merge, Sec. 4).  With `use_head`
// they go into the small head run, which is flushed into the body (and its
// other column orders) only past a share of the body's size, so a long tail
// of small deltas does not rewrite the body every round; otherwise straight
// into full and every other maintained column order of it.
// Checked mode (WCDL_F_CHECKED): relation invariants, verified on the device.
bool checked(const Engine* e) { return (e->cfg.flags & WCDL_F_CHECKED) != 0; }

void check_sorted(Engine* e, const Cols& c, const char* what, u32 rel) {
  if (c.n < 2) return;
  auto p = c.ptrs();
  const u64 bad = order_violations(ctx(e), c.arity(), p.data(), c.n);
  if (bad)
    throw Error(WCDL_E_CHECK, std::string(what) + " of relation " + e->rels[rel].name + " has " +
                                  std::to_string(bad) + " rows out of order or repeated");
}

// A delta about to be merged: sorted, unique, and disjoint from the relation.
void check_delta(Engine* e, u32 rel, const Cols& d) {
  Relation& R = e->rels[rel];
  check_sorted(e, d, "a delta", rel);
  if (d.n && (R.full.n || R.head.n)) {
    auto dp = d.ptrs(), fp = R.full.ptrs();
    std::vector<const u32*> hp;
    if (R.head.n) hp = R.head.ptrs();
    DBuf<u32> tmp[MAXA];
    std::vector<u32*> op;
    for (u32 j = 0; j < d.arity(); ++j) {
      tmp[j] = DBuf<u32>(e->mem.get(), d.n);
      op.push_back(tmp[j].get());
    }
    const u64 kept = set_difference(ctx(e), d.arity(), dp.data(), d.n, fp.data(), R.full.n,
                                    op.data(), hp.empty() ? nullptr : hp.data(), R.head.n);
    if (kept != d.n)
      throw Error(WCDL_E_CHECK, "a delta of relation " + R.name + " repeats " +
                                    std::to_string(d.n - kept) + " rows it already holds");
  }
}

void commit_delta(Engine* e, u32 rel, Cols& d, Stats& st, bool consume = false,
                  bool use_head = false) {
  Relation& R = e->rels[rel];
  if (checked(e)) check_delta(e, rel, d);
  auto t = Clock::now();
  if (d.n && use_head && R.full.n) {
    R.head = R.head.n == 0 ? copy_cols(e, d) : merged(e, 0, R.head, d);
    WCDL_HIP(hipStreamSynchronize(e->streams[0]));
    st.phase[WCDL_PH_MERGE] += ms_since(t);
    if (checked(e)) check_sorted(e, R.head, "the head run", rel);
    if (R.head.n > std::max<u64>(HEAD_MIN_ROWS, R.full.n / head_ratio(e))) flush_head(e, rel, &st);
    return;
  }
  if (d.n) {
    if (R.full.n == 0) {
      // `consume`: the caller no longer needs d, so it becomes full as is.
      R.full = consume ? std::move(d) : copy_cols(e, d);
    } else {
      R.full = merged(e, 0, R.full, d);
    }
    for (auto& kv : R.full_ord) {
      Cols ds = reorder(e, 0, R.full.n == d.n ? R.full : d, kv.first);
      kv.second = merged(e, 0, kv.second, ds);
    }
  }
  WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  st.phase[WCDL_PH_MERGE] += ms_since(t);
  if (checked(e)) {
    check_sorted(e, R.full, "the relation", rel);
    for (auto& kv : R.full_ord) check_sorted(e, kv.second, "a column order", rel);
  }
}

// Evaluate versions and return the rows new to each head relation.
std::map<u32, Cols> new_rows(Engine* e, std::vector<Version>& vs, Stats& st) {
  std::map<u32, Cols> acc;
  eval_batch(e, vs, st, [&](u32 rel, Cols&& rows, bool presorted, u32 grouped) {
    auto it = acc.find(rel);
    if (it == acc.end())
      it = acc.emplace(rel, empty_cols(e->rels[rel].arity, canonical(e->rels[rel].arity))).first;
    absorb_chunk(e, rel, std::move(rows), presorted, grouped, it->second, st);
  });
  return acc;
}

// Rows of `c` whose leading (instance) column is (keep) or is not (!keep) in
// the sorted id list.
Cols select_instances(Engine* e, const Cols& c, const DBuf<u32>& ids, u64 nids, bool keep) {
  Cols out;
  out.order = c.order;
  const u32 k = c.arity();
  if (c.n == 0) {
    for (u32 j = 0; j < k; ++j) out.col.emplace_back();
    return out;
  }
  const u32 pos0 = (u32)(std::find(c.order.begin(), c.order.end(), 0u) - c.order.begin());
  std::vector<u32*> op;
  for (u32 j = 0; j < k; ++j) {
    out.col.emplace_back(e->mem.get(), c.n);
    op.push_back(out.col.back().get());
  }
  auto ip = c.ptrs();
  out.n = select_leading(ctx(e), k, ip.data(), c.n, pos0, ids.get(), nids, keep, op.data());
  return out;
}

// Evaluate the program (Sec. 2 stratification, Sec. 4 loop).  `only`
// (batched engines): start from the loaded facts of these instances alone.
void run_program(Engine* e, wcdl_run_stats* stats_out, const std::vector<u32>* only = nullptr) {
  auto t0 = Clock::now();
  Stats st;
  DBuf<u32> d_only;
  if (only && !only->empty()) {
    d_only = DBuf<u32>(e->mem.get(), only->size());
    WCDL_HIP(hipMemcpy(d_only.get(), only->data(), only->size() * sizeof(u32), hipMemcpyHostToDevice));
  }
  for (auto& R : e->rels) {
    if (only)
      R.full = only->empty() ? empty_cols(R.arity, canonical(R.arity))
                             : select_instances(e, R.base, d_only, only->size(), true);
    else
      R.full = copy_cols(e, R.base);
    R.head = empty_cols(R.arity, canonical(R.arity));
    R.full_ord.clear();
    R.delta_ord.clear();
    R.delta_sizes.clear();
    R.derived = false;
  }
  for (auto& r : e->rules) e->rels[r.head.rel].derived = true;
  sync_all(e);
  u64 rounds = 0;
  for (const auto& comp : strata(e)) {
    std::set<u32> in(comp.begin(), comp.end());
    std::vector<u32> exit_rules, rec_rules;
    for (u32 ri = 0; ri < e->rules.size(); ++ri) {
      const Rule& r = e->rules[ri];
      if (!in.count(r.head.rel)) continue;
      bool rec = false;
      for (auto& a : r.body)
        if (in.count(a.rel)) rec = true;
      (rec ? rec_rules : exit_rules).push_back(ri);
    }
    if (exit_rules.empty() && rec_rules.empty()) continue;
    // Exit rules read finished relations only.
    if (!exit_rules.empty()) {
      std::vector<Version> vs;
      for (u32 ri : exit_rules) {
        vs.push_back(plan_version(e, ri, -1, e->cfg.flags));
        // Sorted output may replace an empty full relation only when nothing
        // else can add to it in this stratum.
        if (!rec_rules.empty()) vs.back().sorted_output = false;
      }
      auto fresh = new_rows(e, vs, st);
      for (auto& kv : fresh) commit_delta(e, kv.first, kv.second, st, true);
    }
    if (rec_rules.empty()) continue;
    // Semi-naive rounds: delta_0 is everything the stratum holds so far.
    for (u32 rel : comp) {
      Relation& R = e->rels[rel];
      R.delta_ord.clear();
      R.delta_ord.emplace(canonical(R.arity), copy_cols(e, R.full));
      R.delta_sizes.push_back(R.full.n);
    }
    sync_all(e);  // the copies are read from every stream
    std::vector<Version> vs;
    for (u32 ri : rec_rules) {
      const Rule& r = e->rules[ri];
      for (u32 j = 0; j < r.body.size(); ++j)
        if (in.count(r.body[j].rel)) vs.push_back(plan_version(e, ri, (int)j, e->cfg.flags));
    }
    for (auto& v : vs) v.sorted_output = false;
    // Relations of the stratum whose full copy no version joins get a head
    // run (their full copy only serves to tell new rows from known ones).
    std::set<u32> joined_full;
    for (auto& v : vs)
      for (auto& a : v.atoms)
        if (!a.delta && in.count(a.rel)) joined_full.insert(a.rel);
    const bool head_body = !(e->cfg.flags & WCDL_F_HEAD_BODY_OFF);
    for (;;) {
      auto fresh = new_rows(e, vs, st);
      std::map<u32, Cols> nd;
      bool any = false;
      for (u32 rel : comp) {
        auto it = fresh.find(rel);
        Cols d = it != fresh.end() ? std::move(it->second)
                                   : empty_cols(e->rels[rel].arity, canonical(e->rels[rel].arity));
        commit_delta(e, rel, d, st, false, head_body && !joined_full.count(rel));
        if (d.n) any = true;
        nd.emplace(rel, std::move(d));
      }
      for (u32 rel : comp) {
        Relation& R = e->rels[rel];
        R.delta_sizes.push_back(nd[rel].n);
        R.delta_ord.clear();
        R.delta_ord.emplace(canonical(R.arity), std::move(nd[rel]));
      }
      ++rounds;
      sync_all(e);
      if (!any) break;
    }
    for (u32 rel : comp) {
      e->rels[rel].delta_ord.clear();
      flush_head(e, rel, &st);
    }
  }
  sync_all(e);
  wcdl_run_stats s{};
  s.rounds = rounds;
  for (auto& R : e->rels)
    if (R.derived) s.derived_rows += R.full.n;
  s.candidate_rows = st.candidates;
  s.join_units = st.units;
  s.wall_ms = ms_since(t0);
  for (int i = 0; i < WCDL_N_PHASES; ++i) s.phase_ms[i] = st.phase[i];
  for (int i = 0; i < 4; ++i) {
    s.kernel_ms[i] = st.kernel_ms[i];
    s.kernel_launches[i] = st.launches[i];
  }
  s.candidates_checked = st.examined;
  for (int j = 0; j < MAXV; ++j) s.candidates_per_level[j] = st.exam_level[j];
  e->last = s;
  if (stats_out) *stats_out = s;
}

// ===========================================================================
// Rule construction and validation
// ===========================================================================

bool batched(const Engine* e) { return (e->cfg.flags & WCDL_F_BATCHED) != 0; }

// Batched mode: thread an instance variable through the head and every body
// atom, so each rule only ever combines facts of one instance.
void batch_rewrite(Rule& r) {
  const u32 inst = r.nvars++;
  r.head.t.insert(r.head.t.begin(), Term{true, inst});
  for (auto& a : r.body) a.t.insert(a.t.begin(), Term{true, inst});
  for (auto& a : r.negs) a.t.insert(a.t.begin(), Term{true, inst});
  if (!r.var_order.empty()) r.var_order.insert(r.var_order.begin(), inst);
}

void validate_rule(Engine* e, const Rule& r) {
  auto check_atom = [&](const Atom& a) {
    if (a.rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    if (a.t.size() != e->rels[a.rel].arity)
      throw Error(WCDL_E_ARITY, "atom of " + e->rels[a.rel].name + " has the wrong arity");
    for (auto& t : a.t)
      if (t.var && t.v >= r.nvars) throw Error(WCDL_E_INVALID, "variable id out of range");
  };
  check_atom(r.head);
  if (r.body.empty()) throw Error(WCDL_E_UNSAFE_RULE, "a rule needs at least one body atom");
  if (r.body.size() > (size_t)MAXN) throw Error(WCDL_E_UNSUPPORTED, "more than 8 body atoms");
  if (r.cmps.size() > (size_t)WCDL_MAX_CMPS) throw Error(WCDL_E_UNSUPPORTED, "more than 8 comparisons");
  std::vector<bool> bound(r.nvars, false);
  for (auto& a : r.body) {
    check_atom(a);
    for (auto& t : a.t)
      if (t.var) bound[t.v] = true;
  }
  if (r.negs.size() > (size_t)MAXNEG) throw Error(WCDL_E_UNSUPPORTED, "more than 4 negated atoms");
  for (auto& a : r.negs) {
    check_atom(a);
    for (auto& t : a.t)
      if (t.var && !bound[t.v])
        throw Error(WCDL_E_UNSAFE_RULE, "negated-atom variable not bound by a positive body atom");
  }
  for (auto& t : r.head.t)
    if (t.var && !bound[t.v]) throw Error(WCDL_E_UNSAFE_RULE, "head variable not bound by the body");
  for (auto& c : r.cmps)
    if ((c.a.var && !bound[c.a.v]) || (c.b.var && !bound[c.b.v]))
      throw Error(WCDL_E_UNSAFE_RULE, "comparison variable not bound by the body");
  // Variable count after the repeated-variable rewrite.
  Rule n = normalize(r);
  u32 used = 0;
  std::vector<bool> seen(n.nvars, false);
  for (auto& a : n.body)
    for (auto& t : a.t)
      if (t.var && !seen[t.v]) { seen[t.v] = true; ++used; }
  if (used > (u32)MAXV) throw Error(WCDL_E_UNSUPPORTED, "more than 8 join variables");
  if (!r.var_order.empty()) {
    std::vector<u32> vo = r.var_order, bv;
    for (u32 v = 0; v < r.nvars; ++v)
      if (bound[v]) bv.push_back(v);
    std::sort(vo.begin(), vo.end());
    if (vo != bv) throw Error(WCDL_E_INVALID, "var_order must list every body variable once");
  }
}

Rule from_c(const wcdl_rule* cr) {
  Rule r;
  u32 nv = cr->n_vars;
  auto term = [&](const wcdl_term& t) {
    Term x;
    x.var = t.kind == WCDL_VAR;
    if (t.kind != WCDL_VAR && t.kind != WCDL_CONST) throw Error(WCDL_E_INVALID, "bad term kind");
    x.v = t.value;
    if (x.var && t.value + 1 > nv) nv = t.value + 1;
    return x;
  };
  auto atom = [&](const wcdl_atom& a) {
    Atom x;
    x.rel = a.rel;
    if (a.arity && !a.terms) throw Error(WCDL_E_INVALID, "null terms");
    for (u32 j = 0; j < a.arity; ++j) x.t.push_back(term(a.terms[j]));
    return x;
  };
  r.head = atom(cr->head);
  if (cr->n_body && !cr->body) throw Error(WCDL_E_INVALID, "null body");
  for (u32 i = 0; i < cr->n_body; ++i) r.body.push_back(atom(cr->body[i]));
  if (cr->n_cmp && !cr->cmp) throw Error(WCDL_E_INVALID, "null comparisons");
  for (u32 i = 0; i < cr->n_cmp; ++i) {
    const wcdl_cmp& c = cr->cmp[i];
    Cmp x;
    Term a = term(c.lhs), b = term(c.rhs);
    switch (c.op) {
      case WCDL_LT: x.op = OP_LT; x.a = a; x.b = b; break;
      case WCDL_LE: x.op = OP_LE; x.a = a; x.b = b; break;
      case WCDL_NE: x.op = OP_NE; x.a = a; x.b = b; break;
      case WCDL_GT: x.op = OP_LT; x.a = b; x.b = a; break;
      case WCDL_GE: x.op = OP_LE; x.a = b; x.b = a; break;
      default: throw Error(WCDL_E_INVALID, "bad comparison operator");
    }
    r.cmps.push_back(x);
  }
  if (cr->n_neg && !cr->neg) throw Error(WCDL_E_INVALID, "null negated atoms");
  for (u32 i = 0; i < cr->n_neg; ++i) r.negs.push_back(atom(cr->neg[i]));
  r.nvars = nv;
  if (cr->var_order) r.var_order.assign(cr->var_order, cr->var_order + cr->n_vars);
  return r;
}

// Parse rules (and ground facts) from text.
void parse_rules(Engine* e, const std::string& text, std::vector<Rule>& rules,
                 std::vector<std::pair<u32, std::vector<u32>>>& facts) {
  Lexer lx(text);
  while (!lx.at_end()) {
    std::map<std::string, u32> vars;
    Rule r;
    auto var_id = [&](const std::string& name) {
      if (name == "_") return r.nvars++;
      auto it = vars.find(name);
      if (it == vars.end()) it = vars.emplace(name, r.nvars++).first;
      return it->second;
    };
    auto term = [&]() {
      Term t;
      u32 c;
      int rc = lx.number(c);
      if (rc < 0) lx.fail("constant does not fit in 32 bits");
      if (rc > 0) { t.var = false; t.v = c; return t; }
      std::string id;
      if (!lx.ident(id)) lx.fail("expected a variable or a constant");
      t.var = true;
      t.v = var_id(id);
      return t;
    };
    auto atom_args = [&](Atom& a, const std::string& name) {
      auto it = e->rel_ids.find(name);
      if (it == e->rel_ids.end()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation " + name);
      a.rel = it->second;
      if (!lx.lit("(")) lx.fail("expected '('");
      if (!lx.lit(")")) {
        for (;;) {
          a.t.push_back(term());
          if (lx.lit(")")) break;
          if (!lx.lit(",")) lx.fail("expected ',' or ')'");
        }
      }
      if (a.t.size() != e->rels[a.rel].user_arity)
        throw Error(WCDL_E_ARITY, "wrong number of arguments for " + name);
    };
    std::string name;
    if (!lx.ident(name)) lx.fail("expected a relation name");
    atom_args(r.head, name);
    if (lx.lit(".")) {
      if (batched(e)) throw Error(WCDL_E_UNSUPPORTED, "facts in rule text need an instance in batched mode");
      std::vector<u32> row;
      for (auto& t : r.head.t) {
        if (t.var) throw Error(WCDL_E_UNSAFE_RULE, "a fact must be ground");
        row.push_back(t.v);
      }
      facts.push_back({r.head.rel, row});
      continue;
    }
    if (!lx.lit(":-")) lx.fail("expected ':-' or '.'");
    for (;;) {
      if (lx.peek("!") && !lx.peek("!=")) {
        // A negated atom  !name(...)
        lx.lit("!");
        std::string nid;
        if (!lx.ident(nid) || !lx.peek("(")) lx.fail("expected an atom after '!'");
        Atom a;
        atom_args(a, nid);
        r.negs.push_back(a);
        if (lx.lit(".")) break;
        if (!lx.lit(",")) lx.fail("expected ',' or '.'");
        continue;
      }
      size_t save = lx.i;
      std::string id;
      bool is_atom = lx.ident(id) && lx.peek("(");
      if (is_atom) {
        Atom a;
        atom_args(a, id);
        r.body.push_back(a);
      } else {
        lx.i = save;
        Term a = term();
        Cmp c;
        bool swap = false;
        if (lx.lit("<=")) c.op = OP_LE;
        else if (lx.lit(">=")) { c.op = OP_LE; swap = true; }
        else if (lx.lit("!=")) c.op = OP_NE;
        else if (lx.lit("<")) c.op = OP_LT;
        else if (lx.lit(">")) { c.op = OP_LT; swap = true; }
        else lx.fail("expected a comparison operator");
        Term b = term();
        c.a = swap ? b : a;
        c.b = swap ? a : b;
        r.cmps.push_back(c);
      }
      if (lx.lit(".")) break;
      if (!lx.lit(",")) lx.fail("expected ',' or '.'");
    }
    if (batched(e)) batch_rewrite(r);
    validate_rule(e, r);
    rules.push_back(r);
  }
}

// Add facts (canonical-order device columns) to a relation's loaded set.
void add_facts(Engine* e, u32 rel, const std::vector<const u32*>& dcols, u64 n) {
  Relation& R = e->rels[rel];
  if (n == 0) return;
  Cols s = sort_rows(e, 0, canonical(R.arity), dcols, n, true);
  if (R.base.n == 0) {
    R.base = std::move(s);
  } else {
    Cols d = difference(e, 0, s, R.base);
    if (d.n) R.base = merged(e, 0, R.base, d);
  }
  sync_all(e);
}

template <class F>
wcdl_status guarded(wcdl_engine* e, F&& f) {
  if (!e) return WCDL_E_INVALID;
  try {
    e->err.clear();
    WCDL_HIP(hipSetDevice(e->cfg.device));
    f();
    return WCDL_OK;
  } catch (const Error& x) {
    e->err = x.what();
    return x.code;
  } catch (const std::bad_alloc&) {
    e->err = "host allocation failed";
    return WCDL_E_NOMEM;
  } catch (const std::exception& x) {
    e->err = x.what();
    return WCDL_E_INVALID;
  }
}

bool valid_name(const char* s) {
  if (!s || !*s) return false;
  if (!(isalpha((unsigned char)s[0]) || s[0] == '_')) return false;
  for (const char* p = s; *p; ++p)
    if (!(isalnum((unsigned char)*p) || *p == '_')) return false;
  return true;
}

u32 declare(Engine* e, const std::string& name, u32 arity, bool internal = false) {
  // `internal`: arity already counts the instance column (helper relations).
  if (!valid_name(name.c_str())) throw Error(WCDL_E_INVALID, "bad relation name");
  const u32 extra = (batched(e) && !internal) ? 1 : 0;
  if (arity == 0 || arity + extra > (u32)MAXA)
    throw Error(WCDL_E_UNSUPPORTED, extra ? "arity must be 1..5 in batched mode" : "arity must be 1..6");
  if (e->rel_ids.count(name)) throw Error(WCDL_E_INVALID, "relation " + name + " already declared");
  Relation R;
  R.name = name;
  R.user_arity = internal && batched(e) ? arity - 1 : arity;
  arity += extra;
  R.arity = arity;
  R.base = empty_cols(arity, canonical(arity));
  R.full = empty_cols(arity, canonical(arity));
  u32 id = (u32)e->rels.size();
  e->rels.push_back(std::move(R));
  e->rel_ids[name] = id;
  return id;
}

}  // namespace
}  // namespace wcdl

// ===========================================================================
// C ABI
// ===========================================================================

using namespace wcdl;

namespace wcdl {

// Canonical text of a helper rule: variables renamed by first occurrence
// (head, then body, then comparisons); comparisons sorted.  Two helpers with
// equal keys define the same relation.
// Tuner choices of this process: (program key, size bucket, points key) ->
// (chosen index, its run time).
std::map<std::string, std::pair<u32, double>>& tune_memo() {
  static std::map<std::string, std::pair<u32, double>> m;
  return m;
}

std::string helper_key(const Rule& h) {
  std::map<u32, u32> ren;
  auto term = [&](const Term& t) {
    if (!t.var) return "c" + std::to_string(t.v);
    auto it = ren.find(t.v);
    if (it == ren.end()) it = ren.emplace(t.v, (u32)ren.size()).first;
    return "v" + std::to_string(it->second);
  };
  std::string k = "h" + std::to_string(h.head.t.size()) + "(";
  for (auto& t : h.head.t) k += term(t) + ",";
  k += "):-";
  for (auto& a : h.body) {
    k += std::to_string(a.rel) + "(";
    for (auto& t : a.t) k += term(t) + ",";
    k += ")";
  }
  std::vector<std::string> cs;
  for (auto& c : h.cmps) cs.push_back(term(c.a) + "op" + std::to_string((int)c.op) + term(c.b));
  std::sort(cs.begin(), cs.end());
  for (auto& c : cs) k += ";" + c;
  return k;
}

void drop_instances(Engine* e, const std::vector<u32>& ids);

// One serving round: admitted facts not yet known join the deltas of their
// relations, then one semi-naive round of every rule version over them.
void serve_round(Engine* e, Stats& st, wcdl_step_stats& s) {
  for (auto& kv : e->pending) {
    Relation& R = e->rels[kv.first];
    Cols d = difference(e, 0, kv.second, R.full);
    const std::vector<u32> canon = canonical(R.arity);
    Cols cur = empty_cols(R.arity, canon);
    auto it = R.delta_ord.find(canon);
    if (it != R.delta_ord.end()) cur = std::move(it->second);
    commit_delta(e, kv.first, d, st);
    Cols next = cur.n == 0 ? std::move(d) : (d.n ? merged(e, 0, cur, d) : std::move(cur));
    R.delta_ord.clear();
    R.delta_ord.emplace(canon, std::move(next));
  }
  e->pending.clear();
  sync_all(e);
  bool any = false;
  for (auto& R : e->rels) {
    auto it = R.delta_ord.find(canonical(R.arity));
    if (it != R.delta_ord.end() && it->second.n) any = true;
  }
  if (any) {
    std::map<u32, Cols> fresh;
    for (;;) {
      try {
        fresh = new_rows(e, e->serve_versions, st);
        break;
      } catch (const Rejected& r) {
        // Over the per-instance cap: drop those instances, count them, and
        // run the round again without them.
        for (u32 id : r.ids) e->rejected.insert(id);
        s.rejected += r.ids.size();
        sync_all(e);
        drop_instances(e, r.ids);
        st.bound_bytes = 0;
      }
    }
    for (u32 rel = 0; rel < e->rels.size(); ++rel) {
      Relation& R = e->rels[rel];
      auto it = fresh.find(rel);
      Cols d = it != fresh.end() ? std::move(it->second) : empty_cols(R.arity, canonical(R.arity));
      commit_delta(e, rel, d, st);
      s.new_rows += d.n;
      R.delta_ord.clear();
      R.delta_ord.emplace(canonical(R.arity), std::move(d));
    }
    sync_all(e);
  }
  for (auto& R : e->rels) s.resident_rows += R.full.n;
  s.candidate_rows = st.candidates;
  s.bound_bytes = st.bound_bytes;
  s.resident_bytes = resident_bytes(e);
}

// Instance ids that still have work: rows in some delta or pending facts.
std::set<u32> live_instances(Engine* e) {
  std::set<u32> live;
  auto collect = [&](const Cols& c) {
    if (c.n == 0) return;
    const u32 pos0 = (u32)(std::find(c.order.begin(), c.order.end(), 0u) - c.order.begin());
    DBuf<u32> out(e->mem.get(), c.n);
    const u32* in = c.col[pos0].get();
    u32* op = out.get();
    // Distinct instance ids of a copy sorted with the instance column first.
    u64 nd = unique_rows(ctx(e), 1, &in, c.n, &op);
    std::vector<u32> h(nd);
    WCDL_HIP(hipMemcpy(h.data(), out.get(), nd * sizeof(u32), hipMemcpyDeviceToHost));
    live.insert(h.begin(), h.end());
  };
  for (auto& R : e->rels)
    for (auto& kv : R.delta_ord)
      if (!kv.first.empty() && kv.first[0] == 0) { collect(kv.second); break; }
  for (auto& kv : e->pending) collect(kv.second);
  return live;
}

// Sorted, deduplicated instance ids of handles that belong to `e`.
std::vector<u32> instance_ids(Engine* e, wcdl_instance* const* v, u32 n) {
  if (n && !v) throw Error(WCDL_E_INVALID, "null instance list");
  std::vector<u32> ids;
  for (u32 i = 0; i < n; ++i) {
    if (!v[i] || v[i]->e != e) throw Error(WCDL_E_INVALID, "instance of another engine");
    ids.push_back(v[i]->id);
  }
  std::sort(ids.begin(), ids.end());
  ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
  return ids;
}

// Drop every row of the listed instances (sorted ids) from every relation.
void drop_instances(Engine* e, const std::vector<u32>& ids) {
  if (ids.empty()) return;
  DBuf<u32> d_ids(e->mem.get(), ids.size());
  WCDL_HIP(hipMemcpy(d_ids.get(), ids.data(), ids.size() * sizeof(u32), hipMemcpyHostToDevice));
  auto drop = [&](Cols& c) {
    if (c.n) c = select_instances(e, c, d_ids, ids.size(), false);
  };
  for (auto& R : e->rels) {
    if (R.head.n) flush_head(e, (u32)(&R - e->rels.data()), nullptr);
    drop(R.full);
    drop(R.base);
    for (auto& kv : R.full_ord) drop(kv.second);
    for (auto& kv : R.delta_ord) drop(kv.second);
  }
  for (auto& kv : e->pending) drop(kv.second);
  sync_all(e);
}

// Device columns of an instance's rows: the instance id column, then the
// caller's columns (host or device).
std::vector<DBuf<u32>> instance_columns(Engine* e, u32 rel, u32 id, const u32* const* cols, u64 n,
                                        int on_device) {
  const u32 k = e->rels[rel].arity;
  if (!cols) throw Error(WCDL_E_INVALID, "null columns");
  std::vector<DBuf<u32>> tmp;
  tmp.emplace_back(e->mem.get(), n);
  fill_u32(ctx(e), tmp.back().get(), n, id);
  for (u32 j = 1; j < k; ++j) {
    if (!cols[j - 1]) throw Error(WCDL_E_INVALID, "null column pointer");
    tmp.emplace_back(e->mem.get(), n);
    WCDL_HIP(hipMemcpyAsync(tmp.back().get(), cols[j - 1], n * sizeof(u32),
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            e->streams[0]));
  }
  return tmp;
}

}  // namespace wcdl

extern "C" {

void wcdl_config_default(wcdl_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
}

wcdl_status wcdl_create(const wcdl_config* cfg, wcdl_engine** out) {
  if (!out) return WCDL_E_INVALID;
  *out = nullptr;
  auto* e = new (std::nothrow) wcdl_engine();
  if (!e) return WCDL_E_NOMEM;
  if (cfg) e->cfg = *cfg;
  wcdl_status st = guarded(e, [&] {
    if (e->cfg.n_streams && e->cfg.streams) {
      for (u32 i = 0; i < e->cfg.n_streams; ++i) e->streams.push_back((hipStream_t)e->cfg.streams[i]);
    } else {
      e->own_streams = true;
      for (int i = 0; i < 4; ++i) {
        hipStream_t s;
        WCDL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        e->streams.push_back(s);
      }
    }
    e->cfg.streams = nullptr;
    e->mem.reset(new DeviceMemory(e->cfg.alloc, e->streams[0]));
    ensure_scratch_address(e->cfg.device);
    size_t free_b = 0, total_b = 0;
    WCDL_HIP(hipMemGetInfo(&free_b, &total_b));
    e->device_total = total_b;
  });
  if (st != WCDL_OK) {
    std::fprintf(stderr, "wcdl_create: %s\n", e->err.c_str());
    delete e;
    return st;
  }
  *out = e;
  return WCDL_OK;
}

void wcdl_destroy(wcdl_engine* e) {
  if (!e) return;
  (void)hipSetDevice(e->cfg.device);
  for (auto s : e->streams) (void)hipStreamSynchronize(s);
  e->rels.clear();
  e->mem.reset();
  for (void* p : e->plan_staging) (void)hipHostFree(p);
  if (e->own_streams)
    for (auto s : e->streams) (void)hipStreamDestroy(s);
  delete e;
}

const char* wcdl_last_error(const wcdl_engine* e) { return e ? e->err.c_str() : "null engine"; }

wcdl_status wcdl_declare_relation(wcdl_engine* e, const char* name, uint32_t arity,
                                  uint32_t* rel_id) {
  return guarded(e, [&] {
    if (!name) throw Error(WCDL_E_INVALID, "null name");
    u32 id = declare(e, name, arity);
    if (rel_id) *rel_id = id;
  });
}

wcdl_status wcdl_relation_id(const wcdl_engine* ce, const char* name, uint32_t* rel_id) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (!name || !rel_id) throw Error(WCDL_E_INVALID, "null argument");
    auto it = e->rel_ids.find(name);
    if (it == e->rel_ids.end()) throw Error(WCDL_E_UNKNOWN_REL, std::string("unknown relation ") + name);
    *rel_id = it->second;
  });
}

wcdl_status wcdl_load_columns(wcdl_engine* e, uint32_t rel, const uint32_t* const* cols,
                              uint64_t n_rows, int on_device) {
  return guarded(e, [&] {
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    const u32 k = e->rels[rel].arity;
    if (n_rows == 0) return;
    if (!cols) throw Error(WCDL_E_INVALID, "null columns");
    for (u32 j = 0; j < k; ++j)
      if (!cols[j]) throw Error(WCDL_E_INVALID, "null column pointer");
    std::vector<DBuf<u32>> tmp;
    std::vector<const u32*> dp;
    for (u32 j = 0; j < k; ++j) {
      tmp.emplace_back(e->mem.get(), n_rows);
      WCDL_HIP(hipMemcpyAsync(tmp.back().get(), cols[j], n_rows * sizeof(u32),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              e->streams[0]));
      dp.push_back(tmp.back().get());
    }
    add_facts(e, rel, dp, n_rows);
  });
}

wcdl_status wcdl_clear_relation(wcdl_engine* e, uint32_t rel) {
  return guarded(e, [&] {
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    Relation& R = e->rels[rel];
    R.base = empty_cols(R.arity, canonical(R.arity));
    R.full = empty_cols(R.arity, canonical(R.arity));
    R.head = empty_cols(R.arity, canonical(R.arity));
    R.full_ord.clear();
    R.delta_ord.clear();
  });
}

wcdl_status wcdl_add_rule(wcdl_engine* e, const wcdl_rule* rule, uint32_t* rule_id) {
  return guarded(e, [&] {
    if (!rule) throw Error(WCDL_E_INVALID, "null rule");
    Rule r = from_c(rule);
    for (auto* a : {&r.head})
      if (a->rel < e->rels.size() && a->t.size() != e->rels[a->rel].user_arity)
        throw Error(WCDL_E_ARITY, "head arity differs from the declaration");
    for (auto& a : r.body)
      if (a.rel < e->rels.size() && a.t.size() != e->rels[a.rel].user_arity)
        throw Error(WCDL_E_ARITY, "atom arity differs from the declaration");
    for (auto& a : r.negs)
      if (a.rel < e->rels.size() && a.t.size() != e->rels[a.rel].user_arity)
        throw Error(WCDL_E_ARITY, "negated atom arity differs from the declaration");
    if (batched(e)) batch_rewrite(r);
    validate_rule(e, r);
    std::vector<Rule> all = e->rules;
    all.push_back(r);
    check_stratified((u32)e->rels.size(), all);
    e->rules.push_back(r);
    if (rule_id) *rule_id = (u32)e->rules.size() - 1;
  });
}

wcdl_status wcdl_add_rules_text(wcdl_engine* e, const char* text) {
  return guarded(e, [&] {
    if (!text) throw Error(WCDL_E_INVALID, "null text");
    std::vector<Rule> rules;
    std::vector<std::pair<u32, std::vector<u32>>> facts;
    parse_rules(e, text, rules, facts);
    std::vector<Rule> all = e->rules;
    all.insert(all.end(), rules.begin(), rules.end());
    check_stratified((u32)e->rels.size(), all);
    for (auto& r : rules) e->rules.push_back(r);
    // Ground facts: group by relation and load.
    std::map<u32, std::vector<std::vector<u32>>> by_rel;
    for (auto& f : facts) by_rel[f.first].push_back(f.second);
    for (auto& kv : by_rel) {
      const u32 k = e->rels[kv.first].arity;
      const u64 n = kv.second.size();
      std::vector<std::vector<u32>> colv(k, std::vector<u32>(n));
      for (u64 i = 0; i < n; ++i)
        for (u32 j = 0; j < k; ++j) colv[j][i] = kv.second[i][j];
      std::vector<DBuf<u32>> tmp;
      std::vector<const u32*> dp;
      for (u32 j = 0; j < k; ++j) {
        tmp.emplace_back(e->mem.get(), n);
        WCDL_HIP(hipMemcpy(tmp.back().get(), colv[j].data(), n * sizeof(u32), hipMemcpyHostToDevice));
        dp.push_back(tmp.back().get());
      }
      add_facts(e, kv.first, dp, n);
    }
  });
}

wcdl_status wcdl_rule_count(const wcdl_engine* ce, uint32_t* n) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (!n) throw Error(WCDL_E_INVALID, "null argument");
    *n = (u32)e->rules.size();
  });
}

wcdl_status wcdl_split_rule(wcdl_engine* e, uint32_t rule_id, const uint32_t* atom_idx, uint32_t n,
                            uint32_t* helper_rel) {
  return guarded(e, [&] {
    if (rule_id >= e->rules.size()) throw Error(WCDL_E_INVALID, "unknown rule id");
    if (!atom_idx || n == 0) throw Error(WCDL_E_INVALID, "no atoms selected");
    Rule r = e->rules[rule_id];
    if (r.orig.empty()) {
      r.orig = r.body;
      r.orig_at.resize(r.body.size());
      for (size_t k = 0; k < r.body.size(); ++k) r.orig_at[k] = (int)k;
    }
    std::set<u32> sel(atom_idx, atom_idx + n);  // indices into the registered body
    if (sel.size() != n) throw Error(WCDL_E_INVALID, "repeated atom index");
    for (u32 a : sel)
      if (a >= r.orig.size()) throw Error(WCDL_E_INVALID, "atom index out of range");
    std::set<u32> present;  // selected atoms still in the body (positions)
    for (u32 a : sel)
      if (r.orig_at[a] >= 0) present.insert((u32)r.orig_at[a]);
    if (present.empty()) throw Error(WCDL_E_INVALID, "every selected atom is already in a helper");
    if (sel.size() >= r.orig.size()) throw Error(WCDL_E_INVALID, "must keep at least one atom");
    std::set<u32> inner;  // variables of the selected atoms
    for (u32 a : sel)
      for (auto& t : r.orig[a].t)
        if (t.var) inner.insert(t.v);
    std::set<u32> outer;  // variables used elsewhere
    for (u32 a = 0; a < r.body.size(); ++a)
      if (!present.count(a))
        for (auto& t : r.body[a].t)
          if (t.var) outer.insert(t.v);
    for (auto& t : r.head.t)
      if (t.var) outer.insert(t.v);
    for (auto& a : r.negs)
      for (auto& t : a.t)
        if (t.var) outer.insert(t.v);
    std::vector<Cmp> helper_cmps, rest_cmps;
    for (auto& c : r.cmps) {
      bool in_a = !c.a.var || inner.count(c.a.v), in_b = !c.b.var || inner.count(c.b.v);
      bool only_inner = in_a && in_b && ((c.a.var && !outer.count(c.a.v)) || (c.b.var && !outer.count(c.b.v)));
      if (in_a && in_b && only_inner) helper_cmps.push_back(c);
      else {
        rest_cmps.push_back(c);
        if (c.a.var) outer.insert(c.a.v);
        if (c.b.var) outer.insert(c.b.v);
      }
    }
    // Orders implied by the rule's comparisons (transitive closure over
    // variable-variable < and <=) among the selected atoms' variables are
    // copied into the helper: every binding the rule uses satisfies them, so
    // the helper may drop rows that do not (the rule keeps its own copies).
    {
      const u32 nv = r.nvars;
      std::vector<std::vector<int>> ord(nv, std::vector<int>(nv, -1));  // -1 none, 0 <=, 1 <
      for (auto& c : r.cmps)
        if (c.a.var && c.b.var && c.op != OP_NE && c.a.v != c.b.v)
          ord[c.a.v][c.b.v] = std::max(ord[c.a.v][c.b.v], c.op == OP_LT ? 1 : 0);
      for (u32 k = 0; k < nv; ++k)
        for (u32 i = 0; i < nv; ++i)
          for (u32 j = 0; j < nv; ++j)
            if (ord[i][k] >= 0 && ord[k][j] >= 0 && i != j)
              ord[i][j] = std::max(ord[i][j], std::max(ord[i][k], ord[k][j]));
      for (u32 i : inner)
        for (u32 j : inner) {
          if (i == j || ord[i][j] < 0 || helper_cmps.size() >= (size_t)WCDL_MAX_CMPS) continue;
          Cmp c;
          c.op = ord[i][j] == 1 ? OP_LT : OP_LE;
          c.a = Term{true, i};
          c.b = Term{true, j};
          bool dup = false;
          for (auto& h : helper_cmps)
            if (h.op == c.op && h.a.var && h.b.var && h.a.v == i && h.b.v == j) dup = true;
          if (!dup) helper_cmps.push_back(c);
        }
    }
    std::vector<u32> shared;  // in order of first occurrence in the selected atoms
    for (u32 a : sel)
      for (auto& t : r.orig[a].t)
        if (t.var && outer.count(t.v) && std::find(shared.begin(), shared.end(), t.v) == shared.end())
          shared.push_back(t.v);
    if (shared.empty()) throw Error(WCDL_E_UNSUPPORTED, "selected atoms share no variable with the rule");
    if (shared.size() > (size_t)MAXA) throw Error(WCDL_E_UNSUPPORTED, "helper relation would exceed arity 6");
    Rule helper, consumer;
    helper.nvars = consumer.nvars = r.nvars;
    for (u32 v : shared) helper.head.t.push_back(Term{true, v});
    for (u32 a : sel) helper.body.push_back(r.orig[a]);
    helper.cmps = helper_cmps;
    const std::string key = helper_key(helper);
    auto known = e->helper_keys.find(key);
    const bool reuse = known != e->helper_keys.end();
    std::string hname;
    u32 hid;
    if (reuse) {
      hid = known->second;  // an earlier split defined this very relation
    } else {
      hname = e->rels[r.head.rel].name + "__h" + std::to_string(e->helper_count);
      while (e->rel_ids.count(hname)) hname += "_";
      hid = (u32)e->rels.size();
    }
    helper.head.rel = hid;
    consumer.head = r.head;
    consumer.orig = r.orig;
    consumer.orig_at.assign(r.orig.size(), -1);
    for (u32 a = 0; a < r.body.size(); ++a)
      if (!present.count(a)) {
        for (size_t k = 0; k < r.orig.size(); ++k)
          if (r.orig_at[k] == (int)a) consumer.orig_at[k] = (int)consumer.body.size();
        consumer.body.push_back(r.body[a]);
      }
    consumer.body.push_back(helper.head);
    consumer.cmps = rest_cmps;
    consumer.negs = r.negs;
    if (!reuse) declare(e, hname, (u32)shared.size(), true);
    try {
      if (!reuse) validate_rule(e, helper);
      validate_rule(e, consumer);
    } catch (...) {
      if (!reuse) {
        e->rel_ids.erase(hname);
        e->rels.pop_back();
      }
      throw;
    }
    e->rules[rule_id] = consumer;
    if (!reuse) {
      e->helper_count++;
      e->helper_keys.emplace(key, hid);
      e->rules.push_back(helper);
    }
    if (helper_rel) *helper_rel = hid;
  });
}

wcdl_status wcdl_binary_plan(wcdl_engine* e, uint32_t* n_helpers) {
  return guarded(e, [&] {
    if (e->serving) throw Error(WCDL_E_STATE, "serving");
    for (auto& r : e->rules)
      if (!r.orig.empty()) throw Error(WCDL_E_STATE, "a rule is already split");
    // All or nothing: on failure the rules and relations are put back.
    const std::vector<Rule> rules0 = e->rules;
    const size_t nrels0 = e->rels.size();
    const uint32_t count0 = e->helper_count;
    const auto keys0 = e->helper_keys;
    u32 made = 0;
    try {
      // Rules appended by the splits (the helpers) are visited in turn.
      for (u32 r = 0; r < e->rules.size(); ++r) {
        const u32 k = (u32)e->rules[r].body.size();
        if (k < 3 || !e->rules[r].orig.empty()) continue;
        std::vector<u32> idx(k - 1);
        for (u32 a = 0; a + 1 < k; ++a) idx[a] = a;
        const size_t before = e->rules.size();
        u32 h = 0;
        const wcdl_status st = wcdl_split_rule(e, r, idx.data(), k - 1, &h);
        if (st != WCDL_OK) throw Error(st, "binary plan of rule " + std::to_string(r) + ": " + e->err);
        made += e->rules.size() > before ? 1u : 0u;
      }
    } catch (...) {
      e->rules = rules0;
      while (e->rels.size() > nrels0) {
        e->rel_ids.erase(e->rels.back().name);
        e->rels.pop_back();
      }
      e->helper_count = count0;
      e->helper_keys = keys0;
      throw;
    }
    if (n_helpers) *n_helpers = made;
  });
}

wcdl_status wcdl_run(wcdl_engine* e, wcdl_run_stats* stats) {
  return guarded(e, [&] { run_program(e, stats); });
}

wcdl_status wcdl_relation_size(const wcdl_engine* ce, uint32_t rel, uint64_t* n_rows) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (rel < e->rels.size() && e->rels[rel].head.n) flush_head(e, rel, nullptr);
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    if (!n_rows) throw Error(WCDL_E_INVALID, "null argument");
    const Relation& R = e->rels[rel];
    *n_rows = R.full.n ? R.full.n : R.base.n;
  });
}

wcdl_status wcdl_read_columns(const wcdl_engine* ce, uint32_t rel, uint32_t* const* cols_out,
                              uint64_t capacity, uint64_t* n_written, int on_device) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (rel < e->rels.size() && e->rels[rel].head.n) flush_head(e, rel, nullptr);
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    const Relation& R = e->rels[rel];
    const Cols& src = R.full.n ? R.full : R.base;
    u64 n = std::min<u64>(src.n, capacity);
    if (n && !cols_out) throw Error(WCDL_E_INVALID, "null output columns");
    for (u32 j = 0; j < R.arity && n; ++j) {
      if (!cols_out[j]) throw Error(WCDL_E_INVALID, "null output column");
      WCDL_HIP(hipMemcpyAsync(cols_out[j], src.col[j].get(), n * sizeof(u32),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              e->streams[0]));
    }
    WCDL_HIP(hipStreamSynchronize(e->streams[0]));
    if (n_written) *n_written = n;
  });
}

wcdl_status wcdl_delta_sizes(const wcdl_engine* ce, uint32_t rel, uint64_t* out, uint64_t cap,
                             uint64_t* count) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    const auto& d = e->rels[rel].delta_sizes;
    for (u64 i = 0; i < d.size() && i < cap && out; ++i) out[i] = d[i];
    if (count) *count = d.size();
  });
}

wcdl_status wcdl_relation_range(const wcdl_engine* ce, uint32_t rel, uint32_t lead,
                                uint64_t* first, uint64_t* count) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (rel < e->rels.size() && e->rels[rel].head.n) flush_head(e, rel, nullptr);
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    const Relation& R = e->rels[rel];
    const Cols& src = R.full.n ? R.full : R.base;
    u64 lohi[2] = {0, 0};
    if (src.n) {
      DBuf<u64> d(e->mem.get(), 2);
      lead_range(ctx(e), src.col[0].get(), src.n, lead, d.get());
      WCDL_HIP(hipMemcpyAsync(lohi, d.get(), sizeof(lohi), hipMemcpyDeviceToHost, e->streams[0]));
      WCDL_HIP(hipStreamSynchronize(e->streams[0]));
    }
    if (first) *first = lohi[0];
    if (count) *count = lohi[1] - lohi[0];
  });
}

wcdl_status wcdl_read_rows(const wcdl_engine* ce, uint32_t rel, uint64_t first, uint64_t n,
                           uint32_t* const* cols_out, int on_device) {
  auto* e = const_cast<wcdl_engine*>(ce);
  return guarded(e, [&] {
    if (rel < e->rels.size() && e->rels[rel].head.n) flush_head(e, rel, nullptr);
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    const Relation& R = e->rels[rel];
    const Cols& src = R.full.n ? R.full : R.base;
    if (first > src.n || n > src.n - first) throw Error(WCDL_E_INVALID, "row range out of bounds");
    if (n && !cols_out) throw Error(WCDL_E_INVALID, "null output columns");
    for (u32 j = 0; j < R.arity && n; ++j) {
      if (!cols_out[j]) throw Error(WCDL_E_INVALID, "null output column");
      WCDL_HIP(hipMemcpyAsync(cols_out[j], src.col[j].get() + first, n * sizeof(u32),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              e->streams[0]));
    }
    WCDL_HIP(hipStreamSynchronize(e->streams[0]));
  });
}

wcdl_status wcdl_autotune(wcdl_engine* e, const uint32_t* wg_per_cu, uint32_t n, uint32_t* chosen,
                          double* best_ms) {
  return guarded(e, [&] {
    if (!wg_per_cu || n == 0) throw Error(WCDL_E_INVALID, "no candidates");
    u32 best = 0;
    double bt = 0;
    for (u32 i = 0; i < n; ++i) {
      if (wg_per_cu[i] == 0) throw Error(WCDL_E_INVALID, "candidate must be positive");
      e->cfg.wg_per_cu = wg_per_cu[i];
      wcdl_run_stats s{};
      run_program(e, &s);
      if (i == 0 || s.wall_ms < bt) {
        bt = s.wall_ms;
        best = wg_per_cu[i];
      }
    }
    e->cfg.wg_per_cu = best;
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = bt;
  });
}

wcdl_status wcdl_trim(wcdl_engine* e, uint64_t* released) {
  return guarded(e, [&] {
    sync_all(e);
    const u64 n = e->mem->cached_bytes();
    e->mem->release_cached();
    if (released) *released = n;
  });
}

wcdl_status wcdl_autotune_points(wcdl_engine* e, const wcdl_tune_point* points, uint32_t n,
                                 uint32_t* chosen, double* best_ms) {
  return guarded(e, [&] {
    if (!points || n == 0) throw Error(WCDL_E_INVALID, "no candidates");
    for (u32 i = 0; i < n; ++i) {
      if (points[i].wg_per_cu == 0) throw Error(WCDL_E_INVALID, "wg_per_cu must be positive");
      if (points[i].flags & ~(u32)WCDL_TUNE_FLAGS) throw Error(WCDL_E_INVALID, "flag outside WCDL_TUNE_FLAGS");
    }
    if (e->serving) throw Error(WCDL_E_STATE, "serving");
    std::string key;
    for (auto& r : e->rules) {
      for (auto& a : r.body) key += e->rels[a.rel].name + "/";
      key += e->rels[r.head.rel].name + "|" + helper_key(r) + "\n";
    }
    u64 facts = 0;
    for (auto& R : e->rels) facts += R.base.n;
    u32 bucket = 0;
    while ((facts >> bucket) > 1) ++bucket;
    key += "#" + std::to_string(bucket) + "#";
    for (u32 i = 0; i < n; ++i)
      key += std::to_string(points[i].wg_per_cu) + "," + std::to_string(points[i].stage_pct) + "," +
             std::to_string(points[i].flags) + "," + std::to_string(points[i].head_ratio) + "," +
             std::to_string(points[i].bitmap_min_run) + ";";
    const u32 keep = e->cfg.flags & ~(u32)WCDL_TUNE_FLAGS;
    auto apply = [&](const wcdl_tune_point& p) {
      e->cfg.wg_per_cu = p.wg_per_cu;
      e->cfg.stage_pct = p.stage_pct;
      e->cfg.flags = keep | p.flags;
      e->cfg.head_ratio = p.head_ratio;
      e->cfg.bitmap_min_run = p.bitmap_min_run;
    };
    auto hit = tune_memo().find(key);
    if (hit != tune_memo().end()) {
      apply(points[hit->second.first]);
      if (chosen) *chosen = hit->second.first;
      if (best_ms) *best_ms = hit->second.second;
      return;
    }
    const wcdl_config saved = e->cfg;
    u32 best = 0;
    double bt = 0;
    try {
      for (u32 i = 0; i < n; ++i) {
        apply(points[i]);
        wcdl_run_stats s{};
        run_program(e, &s);
        if (i == 0 || s.wall_ms < bt) bt = s.wall_ms, best = i;
      }
    } catch (...) {
      e->cfg = saved;
      throw;
    }
    apply(points[best]);
    tune_memo()[key] = {best, bt};
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = bt;
  });
}

wcdl_status wcdl_serve_begin(wcdl_engine* e) {
  return guarded(e, [&] {
    if (!batched(e)) throw Error(WCDL_E_STATE, "serving needs a batched engine");
    for (auto& r : e->rules)
      if (!r.negs.empty())
        throw Error(WCDL_E_UNSUPPORTED, "a program with negation cannot be served (its single "
                                        "semi-naive loop needs a positive program)");
    for (auto& R : e->rels) {
      R.full = copy_cols(e, R.base);
      R.full_ord.clear();
      R.delta_ord.clear();
      R.delta_ord.emplace(canonical(R.arity), empty_cols(R.arity, canonical(R.arity)));
      R.delta_sizes.clear();
    }
    e->serve_versions.clear();
    for (u32 ri = 0; ri < e->rules.size(); ++ri)
      for (u32 j = 0; j < e->rules[ri].body.size(); ++j) {
        e->serve_versions.push_back(plan_version(e, ri, (int)j, e->cfg.flags));
        Version& v = e->serve_versions.back();
        v.sorted_output = false;
        if (e->cfg.instance_cap_bytes) {
          // Per-instance row accounting runs in the count kernel (the
          // cross-product path has no count pass).
          v.plan.xprod = 0;
        }
      }
    e->pending.clear();
    e->rejected.clear();
    e->serving = true;
    sync_all(e);
  });
}

wcdl_status wcdl_serve_admit(wcdl_engine* e, uint32_t rel, const uint32_t* const* cols,
                             uint64_t n_rows, int on_device) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving");
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    if (n_rows == 0) return;
    if (!cols) throw Error(WCDL_E_INVALID, "null columns");
    const u32 k = e->rels[rel].arity;
    std::vector<DBuf<u32>> tmp;
    std::vector<const u32*> dp;
    for (u32 j = 0; j < k; ++j) {
      if (!cols[j]) throw Error(WCDL_E_INVALID, "null column pointer");
      tmp.emplace_back(e->mem.get(), n_rows);
      WCDL_HIP(hipMemcpyAsync(tmp.back().get(), cols[j], n_rows * sizeof(u32),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              e->streams[0]));
      dp.push_back(tmp.back().get());
    }
    Cols srt = sort_rows(e, 0, canonical(k), dp, n_rows, true);
    // Rows are sorted by instance: the last one holds the largest id.
    u32 top = 0;
    WCDL_HIP(hipMemcpy(&top, srt.col[0].get() + (srt.n - 1), sizeof(u32), hipMemcpyDeviceToHost));
    e->max_instance = std::max(e->max_instance, top);
    auto it = e->pending.find(rel);
    if (it == e->pending.end()) {
      e->pending.emplace(rel, std::move(srt));
    } else {
      Cols d = difference(e, 0, srt, it->second);
      if (d.n) it->second = merged(e, 0, it->second, d);
    }
    sync_all(e);
  });
}

wcdl_status wcdl_serve_step(wcdl_engine* e, wcdl_step_stats* out) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving");
    auto t0 = Clock::now();
    Stats st;
    wcdl_step_stats s{};
    serve_round(e, st, s);
    s.wall_ms = ms_since(t0);
    for (int i = 0; i < WCDL_N_PHASES; ++i) s.phase_ms[i] = st.phase[i];
    if (out) *out = s;
  });
}

wcdl_status wcdl_serve_live(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving");
    const std::set<u32> live = live_instances(e);
    u64 i = 0;
    for (u32 v : live) {
      if (ids && i < cap) ids[i] = v;
      ++i;
    }
    if (count) *count = live.size();
  });
}

wcdl_status wcdl_serve_live_static(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving");
    u32* sc = scratch_at[e->cfg.device];
    if (!sc) throw Error(WCDL_E_STATE, "static scratch not set up on this device");
    hipStream_t s = e->streams[0];
    // Work of every stream is done before the columns are read.
    for (auto st : e->streams) WCDL_HIP(hipStreamSynchronize(st));
    k_live_clear<<<128, 256, 0, s>>>(sc);
    WCDL_HIP(hipGetLastError());
    auto mark = [&](const Cols& c) {
      if (c.n == 0 || c.order.empty() || c.order[0] != 0) return;
      const u64 blocks = (c.n + 255) / 256;
      if (blocks > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "relation too large");
      k_live_mark<<<(u32)blocks, 256, 0, s>>>(c.col[0].get(), c.n, sc);
      WCDL_HIP(hipGetLastError());
    };
    for (auto& R : e->rels)
      for (auto& kv : R.delta_ord) mark(kv.second);
    for (auto& kv : e->pending) mark(kv.second);
    k_live_list<<<1, 1024, 0, s>>>(sc);
    WCDL_HIP(hipGetLastError());
    u32 head[2] = {0, 0};
    WCDL_HIP(hipMemcpyAsync(head, sc, sizeof(head), hipMemcpyDeviceToHost, s));
    WCDL_HIP(hipStreamSynchronize(s));
    if (head[1])
      throw Error(WCDL_E_UNSUPPORTED, "an instance id is >= " + std::to_string(LIVE_MAX_IDS) +
                                          ", beyond the static listing's bitmap");
    if (head[0] > LIVE_MAX_LIST)
      throw Error(WCDL_E_UNSUPPORTED, std::to_string(head[0]) + " live instances exceed the static "
                                      "list of " + std::to_string(LIVE_MAX_LIST));
    const u64 n = std::min<u64>(head[0], cap);
    if (n && !ids) throw Error(WCDL_E_INVALID, "null ids");
    if (n) {
      WCDL_HIP(hipMemcpyAsync(ids, sc + LIVE_LIST_AT, n * sizeof(u32), hipMemcpyDeviceToHost, s));
      WCDL_HIP(hipStreamSynchronize(s));
    }
    if (count) *count = head[0];
  });
}

wcdl_status wcdl_serve_release(wcdl_engine* e, const uint32_t* ids, uint64_t n) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving");
    if (n == 0) return;
    if (!ids) throw Error(WCDL_E_INVALID, "null ids");
    std::vector<u32> h(ids, ids + n);
    std::sort(h.begin(), h.end());
    h.erase(std::unique(h.begin(), h.end()), h.end());
    drop_instances(e, h);
  });
}

wcdl_status wcdl_serve_rejected(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count) {
  return guarded(e, [&] {
    u64 i = 0;
    for (u32 v : e->rejected) {
      if (ids && i < cap) ids[i] = v;
      ++i;
    }
    if (count) *count = e->rejected.size();
  });
}

wcdl_status wcdl_serve_end(wcdl_engine* e) {
  return guarded(e, [&] {
    e->serving = false;
    e->serve_versions.clear();
    e->pending.clear();
  });
}

wcdl_status wcdl_instance_create(wcdl_engine* e, wcdl_instance** out) {
  return guarded(e, [&] {
    if (!out) throw Error(WCDL_E_INVALID, "null output");
    *out = nullptr;
    if (!batched(e)) throw Error(WCDL_E_STATE, "instances need a batched engine");
    if (e->next_instance == NONE) throw Error(WCDL_E_UNSUPPORTED, "instance ids exhausted");
    auto* in = new wcdl_instance();
    in->e = e;
    in->id = e->next_instance++;
    *out = in;
  });
}

uint32_t wcdl_instance_id(const wcdl_instance* in) { return in ? in->id : NONE; }

wcdl_status wcdl_instance_load(wcdl_instance* in, uint32_t rel, const uint32_t* const* cols,
                               uint64_t n_rows, int on_device) {
  if (!in) return WCDL_E_INVALID;
  wcdl_engine* e = in->e;
  return guarded(e, [&] {
    if (rel >= e->rels.size()) throw Error(WCDL_E_UNKNOWN_REL, "unknown relation id");
    if (n_rows == 0) return;
    auto tmp = instance_columns(e, rel, in->id, cols, n_rows, on_device);
    std::vector<const u32*> dp;
    for (auto& t : tmp) dp.push_back(t.get());
    const u32 k = e->rels[rel].arity;
    if (!e->serving) {
      add_facts(e, rel, dp, n_rows);
      return;
    }
    Cols srt = sort_rows(e, 0, canonical(k), dp, n_rows, true);
    e->max_instance = std::max(e->max_instance, in->id);
    auto it = e->pending.find(rel);
    if (it == e->pending.end()) {
      e->pending.emplace(rel, std::move(srt));
    } else {
      Cols d = difference(e, 0, srt, it->second);
      if (d.n) it->second = merged(e, 0, it->second, d);
    }
    sync_all(e);
  });
}

wcdl_status wcdl_instance_size(const wcdl_instance* in, uint32_t rel, uint64_t* n_rows) {
  if (!in) return WCDL_E_INVALID;
  uint64_t first = 0;
  return wcdl_relation_range(in->e, rel, in->id, &first, n_rows);
}

wcdl_status wcdl_instance_read(const wcdl_instance* in, uint32_t rel, uint32_t* const* cols_out,
                               uint64_t capacity, uint64_t* n_written, int on_device) {
  if (!in) return WCDL_E_INVALID;
  wcdl_engine* e = in->e;
  uint64_t first = 0, count = 0;
  wcdl_status rc = wcdl_relation_range(e, rel, in->id, &first, &count);
  if (rc != WCDL_OK) return rc;
  return guarded(e, [&] {
    const Relation& R = e->rels[rel];
    const Cols& src = R.full.n ? R.full : R.base;
    const u64 n = std::min<u64>(count, capacity);
    if (n && !cols_out) throw Error(WCDL_E_INVALID, "null output columns");
    for (u32 j = 1; j < R.arity && n; ++j) {
      if (!cols_out[j - 1]) throw Error(WCDL_E_INVALID, "null output column");
      WCDL_HIP(hipMemcpyAsync(cols_out[j - 1], src.col[j].get() + first, n * sizeof(u32),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              e->streams[0]));
    }
    WCDL_HIP(hipStreamSynchronize(e->streams[0]));
    if (n_written) *n_written = n;
  });
}

void wcdl_instance_destroy(wcdl_instance* in) {
  if (!in) return;
  wcdl_engine* e = in->e;
  const std::vector<u32> ids{in->id};
  (void)guarded(e, [&] { drop_instances(e, ids); });
  delete in;
}

wcdl_status wcdl_run_batch(wcdl_engine* e, wcdl_instance* const* v, uint32_t n,
                           wcdl_run_stats* stats) {
  return guarded(e, [&] {
    if (!batched(e)) throw Error(WCDL_E_STATE, "wcdl_run_batch needs a batched engine");
    if (e->serving) throw Error(WCDL_E_STATE, "the engine is serving");
    const std::vector<u32> ids = instance_ids(e, v, n);
    run_program(e, stats, &ids);
  });
}

wcdl_status wcdl_step(wcdl_engine* e, wcdl_instance* const* active, uint32_t n, uint8_t* done,
                      uint64_t* next_bound_bytes) {
  return guarded(e, [&] {
    if (!e->serving) throw Error(WCDL_E_STATE, "not serving (wcdl_serve_begin first)");
    const std::vector<u32> ids = instance_ids(e, active, n);
    DBuf<u32> d_ids;
    if (!ids.empty()) {
      d_ids = DBuf<u32>(e->mem.get(), ids.size());
      WCDL_HIP(hipMemcpy(d_ids.get(), ids.data(), ids.size() * sizeof(u32), hipMemcpyHostToDevice));
    }
    // Work of instances outside the active set waits: their delta rows and
    // admitted facts are set aside for this round and put back after it.
    std::map<u32, Cols> held_delta, held_pending;
    for (u32 rel = 0; rel < e->rels.size(); ++rel) {
      Relation& R = e->rels[rel];
      const std::vector<u32> canon = canonical(R.arity);
      auto it = R.delta_ord.find(canon);
      if (it != R.delta_ord.end() && it->second.n) {
        Cols cur = std::move(it->second);
        R.delta_ord.clear();
        if (ids.empty()) {
          held_delta.emplace(rel, std::move(cur));
          R.delta_ord.emplace(canon, empty_cols(R.arity, canon));
        } else {
          held_delta.emplace(rel, select_instances(e, cur, d_ids, ids.size(), false));
          R.delta_ord.emplace(canon, select_instances(e, cur, d_ids, ids.size(), true));
        }
      }
    }
    for (auto& kv : e->pending) {
      Cols rest = ids.empty() ? std::move(kv.second)
                              : select_instances(e, kv.second, d_ids, ids.size(), false);
      if (!ids.empty()) kv.second = select_instances(e, kv.second, d_ids, ids.size(), true);
      else kv.second = empty_cols(rest.arity(), rest.order);
      if (rest.n) held_pending.emplace(kv.first, std::move(rest));
    }
    sync_all(e);
    Stats st;
    wcdl_step_stats s{};
    serve_round(e, st, s);
    for (auto& kv : held_delta) {
      if (kv.second.n == 0) continue;
      Relation& R = e->rels[kv.first];
      const std::vector<u32> canon = canonical(R.arity);
      auto it = R.delta_ord.find(canon);
      Cols cur = it != R.delta_ord.end() ? std::move(it->second) : empty_cols(R.arity, canon);
      R.delta_ord.clear();
      R.delta_ord.emplace(canon, cur.n ? merged(e, 0, cur, kv.second) : std::move(kv.second));
    }
    for (auto& kv : held_pending) e->pending.emplace(kv.first, std::move(kv.second));
    sync_all(e);
    if (done) {
      const std::set<u32> live = live_instances(e);
      for (u32 i = 0; i < n; ++i) done[i] = live.count(active[i]->id) ? 0 : 1;
    }
    if (next_bound_bytes) *next_bound_bytes = resident_bytes(e) + st.bound_bytes;
  });
}

void wcdl_work_slice(uint64_t T, uint64_t p, uint64_t b, uint64_t* b_s, uint64_t* b_e) {
  const uint64_t s = ceil_div(T, p);
  uint64_t lo = b * s;
  if (lo > T) lo = T;
  uint64_t hi = lo + s < T ? lo + s : T;
  if (b_s) *b_s = lo;
  if (b_e) *b_e = hi;
}

uint64_t wcdl_owner_key(const uint64_t* C, uint64_t K, uint64_t g) { return owner_key(C, 0, K, g); }

void wcdl_decode_unit(const uint64_t* C, uint64_t K, const uint32_t* d2, uint64_t g, uint64_t* key,
                      uint64_t* i1, uint64_t* i2) {
  const uint64_t k = owner_key(C, 0, K, g);
  const uint64_t local = g - (k ? C[k - 1] : 0);
  if (key) *key = k;
  if (k < K && d2[k]) {
    if (i1) *i1 = local / d2[k];
    if (i2) *i2 = local % d2[k];
  }
}

}  // extern "C"
