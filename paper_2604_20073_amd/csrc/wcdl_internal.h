// Internal declarations shared by the engine's host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "wcdl.h"

namespace wcdl {

using u32 = uint32_t;
using u64 = uint64_t;

constexpr int MAXA = WCDL_MAX_ARITY;  // columns per atom
constexpr int MAXN = WCDL_MAX_BODY;   // atoms per rule body
constexpr int MAXV = WCDL_MAX_VARS;   // variables (join levels) per rule
constexpr int MAXS = MAXN;            // sources per level (one per atom at most)
constexpr int MAXB = 8;               // value bounds per level
constexpr int MAXF = 4;               // inequality filters per level
constexpr int MAXNEG = WCDL_MAX_NEG;  // negated atoms per rule
constexpr u32 NONE = 0xffffffffu;

// ---------------------------------------------------------------------------
// Errors: thrown inside the library, turned into status codes at the C ABI.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define WCDL_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::wcdl::Error(WCDL_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory: blocks come from the caller's allocator (or hipMalloc) and
// are cached by size class.  A freed block becomes reusable only after the
// next device-wide synchronisation point, so a block still read by work on
// another stream is never handed out again too early.
// ---------------------------------------------------------------------------
class DeviceMemory {
 public:
  DeviceMemory(const wcdl_allocator& a, hipStream_t s) : user_(a), stream_(s) {}
  ~DeviceMemory();
  void* get(size_t bytes);
  void put(void* p);
  void sync_point();  // pending frees become reusable
  void release_cached();
  size_t live_bytes() const { return live_bytes_; }
  size_t cached_bytes() const {
    size_t n = 0;
    for (auto& b : free_) n += b.first;
    return n;
  }

 private:
  static size_t size_class(size_t bytes);
  void* raw_alloc(size_t bytes);
  void raw_free(void* p, size_t bytes);
  wcdl_allocator user_;
  hipStream_t stream_;
  std::multimap<size_t, void*> free_;
  std::vector<std::pair<void*, size_t>> pending_;
  std::map<void*, size_t> live_;
  size_t live_bytes_ = 0;
};

// Owning handle to a device array of T.
template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(DeviceMemory* m, u64 n) : mem_(m), n_(n) {
    if (n) p_ = static_cast<T*>(m->get(n * sizeof(T)));
  }
  ~DBuf() { reset(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : mem_(o.mem_), p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      mem_ = o.mem_; p_ = o.p_; n_ = o.n_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  void reset() {
    if (p_ && mem_) mem_->put(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  u64 size() const { return n_; }

 private:
  DeviceMemory* mem_ = nullptr;
  T* p_ = nullptr;
  u64 n_ = 0;
};

// A relation (or delta) stored as k sorted device columns.  order[j] is the
// column of the logical relation that this copy holds in position j; rows
// are sorted lexicographically by position 0, 1, ..., k-1 and unique.
struct Cols {
  std::vector<u32> order;
  std::vector<DBuf<u32>> col;
  u64 n = 0;
  DBuf<u32> dir;       // dense directory of column 0 (built on demand)
  u32 dir_max = 0;
  bool dir_tried = false;
  // Run bitmaps (built on demand): for every run of rows sharing all but the
  // last column that is at least bm_min rows long, a bitmap of the last
  // column's values; bm_at[start row of such a run] = its bitmap, else NONE.
  DBuf<u32> bm_at, bm;
  u32 bm_words = 0;    // 32-bit words per bitmap
  u32 bm_min = 0;      // shortest run with a bitmap (0: none built)
  bool bm_tried = false;
  u32 arity() const { return (u32)order.size(); }
  std::vector<const u32*> ptrs() const {
    std::vector<const u32*> v;
    for (auto& c : col) v.push_back(c.get());
    return v;
  }
  std::vector<u32*> mptrs() {
    std::vector<u32*> v;
    for (auto& c : col) v.push_back(c.get());
    return v;
  }
};

// ---------------------------------------------------------------------------
// Join plan as the kernels see it (one per rule version).  Levels are the
// join variables x_1..x_m in the chosen order (index 0-based here).  Each
// body atom is read through a sorted copy whose column order follows the
// variable order (constants first), so binding the variables level by level
// narrows each atom to a contiguous row range (Sec. 4: tuples sharing a
// prefix are contiguous; Sec. 2: attribute-at-a-time evaluation).
// ---------------------------------------------------------------------------
struct DOperand {
  u32 is_var;  // 1: value of the variable at level `v`; 0: constant `v`
  u32 v;
};

struct DSource {      // an atom constraining the level's variable
  const u32* col;     // the atom's column holding this variable
  const u32* dir;     // optional dense directory of col (first column of a copy
                      // read unnarrowed): rows of value v are [dir[v], dir[v+1])
  u32 dmax;           // largest value covered by dir
  u32 atom;           // atom index
  u32 last;           // 1 if no variable column of the atom follows
  u32 alias;          // earlier source at this level with the same column and
                      // the same current range (its result is reused), or NONE
  const u32* bm_at;   // optional run bitmaps of the copy (leaf sources): per
  const u32* bm;      //   row, the bitmap of the run starting there or NONE
  u32 bm_words;       // 32-bit words per bitmap
  u32 bm_min;         // runs shorter than this have no bitmap
};

struct DBound {       // x_level >= opnd + adj (lo) or x_level <= opnd - adj (hi)
  u32 is_hi;
  u32 adj;
  DOperand o;
};

// A negated atom (stratified negation): a filter over a relation of a lower
// stratum, tested at the level that binds its last variable.  Its sorted copy
// holds its columns in `col` in search order (constants first, then
// variables by level); a binding survives if no row equals the operands.
struct DNeg {
  const u32* col[MAXA];
  DOperand val[MAXA];
  u32 ncols;
  u32 n;                  // rows of the copy
  u32 level;              // level at which every variable of the atom is bound
  u32 pad_;
};

struct DLevel {
  u32 nsrc;
  u32 nbnd;
  u32 nne;
  u32 nneg;               // negated atoms tested at this level
  DSource src[MAXS];
  DBound bnd[MAXB];
  DOperand ne[MAXF];      // x_level != operand
  u32 atom_src[MAXN];     // per atom: its source index at this level, or NONE
};

struct DPlan {
  u32 m;                  // number of variables (join depth)
  u32 natoms;
  u32 root_src;           // source (at level 0) whose column supplies the root keys
  u32 head_arity;
  u32 leaf_fast;          // count pass may sum leaf candidate ranges (single
                          // distinct-valued source, no filter at the leaf)
  u32 xprod;              // levels >= 1 are independent single sources
  DOperand head[MAXA];
  u32* out[MAXA];         // output columns (materialize)
  u64 out_rows;           // rows reserved at out[] (writes beyond are refused)
  u32* err;               // device flag set if a write was refused
  u64* cand;              // optional: candidates examined per level (materialize)
  // Staging of the count pass (mode 2): rows go to an arena of chunks of
  // STAGE_CHUNK rows taken from a global counter; chunk_tag[c] = (workgroup
  // << 32) | sequence number of the chunk within that workgroup's rows.
  u32* stage[MAXA];
  u64 stage_chunks;       // arena capacity in chunks
  u64* stage_next;        // chunks handed out so far
  u64* chunk_tag;
  u32* ovf;               // per workgroup: 1 if its rows did not all fit
  // Serving: bytes of rows counted per instance (indexed by the instance id,
  // the value of level 0), inst_n entries; NULL when not counted.
  unsigned long long* inst_bytes;
  u32 inst_n;
  u32 row_bytes;          // head arity x 4
  u64 inst_cap;           // bytes an instance may count (inst_bytes set)
  // Memory-bounded count passes: bytes counted by every version of the
  // round so far (bound_acc, NULL when unbounded) against bound_limit.  When
  // a bound is crossed the count kernels set *abort and every workgroup stops
  // at its next step (the round is then refused, its counts discarded).
  unsigned long long* bound_acc;
  u64 bound_limit;
  u32* abort;
  DNeg neg[MAXNEG];       // negated atoms, ordered by level
  u32 nneg;
  u32 atom_n[MAXN];       // rows in each atom's sorted copy
  u32 atom_nconst[MAXN];  // leading constant columns of each atom
  u32 atom_const[MAXN][MAXA];
  const u32* atom_col[MAXN][MAXA];
  DLevel lvl[MAXV];
  // Range slots of the level buffers.  After binding level b, atoms whose
  // ranges are equal share a slot; atom_slot[b][a] is NONE for an atom not
  // narrowed yet (its range is its constant-narrowed initial range) or no
  // longer needed (all its columns bound).  slot_atom[b][s] is an atom whose
  // range the slot holds.
  u32 nslot[MAXV];
  u32 atom_slot[MAXV][MAXN];
  u32 slot_atom[MAXV][MAXN];
  // Shared-memory layout of the level buffers (offsets in 32-bit words).
  u32 cap;                // items per level buffer
  u32 off_val[MAXV], off_lo[MAXV], off_hi[MAXV], off_drv[MAXV], off_clo[MAXV],
      off_chi[MAXV], off_pre[MAXV];
  u32 off_emit;           // survivors of an emitted chunk (EMIT_ROWS values, then
                          // EMIT_ROWS item bytes), or NONE: lanes write their own
  u32 lds_words;
};

// Root-level work space (Alg. 1 Phase 1): K root keys U with row starts S
// (S[K] = end of range) in the root atom's sorted copy, inclusive prefix sums
// C of the per-key work W, total T.
struct RootSpace {
  const u32* U;
  const u32* S;
  const u64* C;
  u64 K;
  u64 T;
  const u32* rng0;        // per atom [lo, hi) after constant narrowing (2*MAXN)
};

// Work partition (Alg. 2): p workgroups; slice = ceil(T/p) units each, or
// with balance off one root key per workgroup.
struct Partition {
  u64 p;
  u64 slice;
  u32 balance_off;
  u32 pad_;
};

// ---------------------------------------------------------------------------
// Host-callable launchers (prim.hip, wcoj.hip).  All are asynchronous on
// `s` unless noted.
// ---------------------------------------------------------------------------
struct Ctx {
  DeviceMemory* mem;
  hipStream_t s;
};

// Exclusive scan of n values into out (u64); *d_total (device) = sum.
void scan_u32_excl(Ctx c, const u32* in, u64* out, u64 n, u64* d_total);
void scan_u64_excl(Ctx c, const u64* in, u64* out, u64 n, u64* d_total);
// Inclusive scan u64 -> u64.
void scan_u64_incl(Ctx c, const u64* in, u64* out, u64 n, u64* d_total);

// Radix sort of rows (LSD, 8-bit digits).  in_cols[j] / out_cols[j] are the
// key columns in significance order (column 0 most significant).  col_bits[j]
// = number of significant bits of column j (values must be < 2^bits).
void radix_sort_rows(Ctx c, u32 k, const u32* const* in_cols, u32* const* out_cols, u64 n,
                     const u32* col_bits);
// OR of all values of each column (device results in d_or[k]).
void column_or(Ctx c, u32 k, const u32* const* cols, u64 n, u32* d_or);

// Rows non-decreasing in columns 0..k-2 and unsorted, with repeats, in
// column k-1 (values below 2^zbits): sorted and deduplicated through one LDS
// bitmap per group of equal leading columns.  Returns false, having written
// nothing, where the bitmaps would cost more than the rows (zbits > 18, or
// more than two bitmap words per row); else *out_n = rows written
// (synchronises).
bool sort_unique_grouped(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32 zbits,
                         u32* const* out_cols, u64* out_n);
// Unique adjacent rows of a sorted input; returns the count (synchronises).
u64 unique_rows(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32* const* out_cols);
// One copy of every row repeated inside each tile of 2,048 consecutive rows,
// in order (rows repeated across tiles stay); returns the rows written
// (synchronises).  Arity at most 4.
u64 drop_tile_repeats(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32* const* out_cols);
// Rows of sorted-unique A absent from sorted-unique B and from the optional
// sorted-unique B2; returns count (syncs).
u64 set_difference(Ctx c, u32 k, const u32* const* a, u64 na, const u32* const* b, u64 nb,
                   u32* const* out, const u32* const* b2 = nullptr, u64 nb2 = 0);
// Merge two disjoint sorted-unique runs into out (na + nb rows).
void merge_disjoint(Ctx c, u32 k, const u32* const* a, u64 na, const u32* const* b, u64 nb,
                    u32* const* out);
// Rows of sorted column `col` equal to v: d_out[0] = first, d_out[1] = end.
void lead_range(Ctx c, const u32* col, u64 n, u32 v, u64* d_out);
// Keep the rows whose column `lead_col` is (keep_listed) or is not (else) in
// the sorted list ids[0..nids); returns the count kept (synchronises).
u64 select_leading(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32 lead_col, const u32* ids,
                   u64 nids, bool keep_listed, u32* const* out_cols);
// Adjacent row pairs of a k-column run that are not strictly ascending
// (lexicographically): 0 for a sorted, duplicate-free run (synchronises).
u64 order_violations(Ctx c, u32 k, const u32* const* cols, u64 n);
// Fill helpers.
void fill_u32(Ctx c, u32* p, u64 n, u32 v);
void fill_u64(Ctx c, u64* p, u64 n, u64 v);
void copy_u32(Ctx c, u32* dst, const u32* src, u64 n);

// WCOJ (wcoj.hip).
void join_init_ranges(Ctx c, const DPlan* d_plan, u32 natoms, u32* d_rng0);
// Root keys of column `col` in rows [rng0[2a], rng0[2a+1]) of atom a, in two
// asynchronous steps: flags + scan (count of keys into *d_K), then, once K
// is known on the host, compaction into U (K values) and S (K+1 row starts).
void join_root_flags(Ctx c, const u32* col, const u32* d_rng0, u32 atom, u32 n_rows, u32* flags,
                     u64* pos, u64* d_K);
void join_root_compact(Ctx c, const u32* col, const u32* d_rng0, u32 atom, u32 n_rows,
                       const u32* flags, const u64* pos, u64 K, u32* U, u32* S);
// Per-key work W (Alg. 1 Phase 1).  For cross-product plans also writes
// per-key (lo, size) of every level >= 1 into klo/kd ([m][K]).
void join_histogram(Ctx c, const DPlan* d_plan, const RootSpace& rs, u64* W, u32* klo, u32* kd,
                    u32 m);
// Candidates of one leaf chunk (leaf candidates per lane x workgroup size).
constexpr u32 EMIT_ROWS = 512;
constexpr u64 STAGE_CHUNK = 4096;
// Count (mode 0), materialize (mode 1) or count-and-stage (mode 2) over
// workgroups wg0 + [0, nwg), or over the listed workgroups if wg_list is set.
void join_run(Ctx c, const DPlan* d_plan, const RootSpace& rs, const Partition& part,
              u32 lds_bytes, int mode, u64* counts, const u64* offsets, u64 wg0, u64 nwg,
              const u32* wg_list = nullptr);
// Write pass for staged rows: chunk c of workgroup b goes to
// offsets[b] + seq * STAGE_CHUNK unless b overflowed.
void join_stage_copy(Ctx c, const DPlan* d_plan, u64 used_chunks, const u64* counts,
                     const u64* offsets, u32 arity, u64 w0, u64 w1);
// Dense directory of a sorted column with values <= vmax: dir[v] = first row
// with value >= v, for v in [0, vmax+1] (vmax + 2 entries).
// Run bitmaps of a sorted copy with k >= 2 columns (see Cols): runs of at
// least `min_run` rows sharing columns 0..k-2 get a bitmap of column k-1's
// values (vmax: an upper bound of those values), at most max_bytes in
// total (min_run is raised until they fit).  Returns the shortest run with
// a bitmap, 0 if none was built (synchronises).
u32 build_run_bitmaps(Ctx c, u32 k, const u32* const* cols, u64 n, u32 vmax, u32 min_run,
                      u64 max_bytes, DBuf<u32>* bm_at, DBuf<u32>* bm, u32* words);
void build_directory(Ctx c, const u32* col, u64 n, u32 vmax, u32* dir);
// Cross-product decode path: writes the rows of units [g0, g1) (row g = unit g).
void join_xprod(Ctx c, const DPlan* d_plan, const RootSpace& rs, const u32* klo, const u32* kd,
                u32 m, u64 g0, u64 g1);

}  // namespace wcdl

// Shared by host and device: the work-slice arithmetic of Alg. 2.
namespace wcdl {
__host__ __device__ inline u64 ceil_div(u64 a, u64 b) { return b ? (a + b - 1) / b : 0; }

// First index k in [lo, hi) with C[k] > g (C nondecreasing); hi if none.
__host__ __device__ inline u64 owner_key(const u64* C, u64 lo, u64 hi, u64 g) {
  while (lo < hi) {
    u64 mid = lo + ((hi - lo) >> 1);
    if (C[mid] <= g) lo = mid + 1; else hi = mid;
  }
  return lo;
}
}  // namespace wcdl
