// Data-parallel primitives of the relation store, written for gfx950
// (wave64, 160 KB LDS per CU): prefix scans, LSD radix sort of multi-column
// rows, adjacent-duplicate removal, sorted set difference and the merge of
// two disjoint sorted runs.  The paper's pipeline relies on a memory-bound
// radix sort for Build Index and a single-pass merge for Merge (Sec. 4);
// these are this engine's own versions of both.

#include <algorithm>

#include "wcdl_internal.h"

namespace wcdl {
namespace {

constexpr int WG = 256;        // threads per workgroup (4 waves of 64)
constexpr int SCAN_IPT = 8;    // items per thread in scans
constexpr int SCAN_TILE = WG * SCAN_IPT;
constexpr int RS_IPT = 16;     // keys per thread in radix passes
constexpr int RS_TILE = WG * RS_IPT;  // 4096 keys per tile
constexpr int SEARCH_IPT = 4;  // rows per thread in tiled searches
constexpr int SEARCH_TILE = WG * SEARCH_IPT;
constexpr u32 AF_WORDS = 8192;  // LDS words of splitters in set differences (32 KB)

struct ColsIn { const u32* c[MAXA]; };
struct ColsOut { u32* c[MAXA]; };

ColsIn cols_in(u32 k, const u32* const* p) {
  ColsIn a{};
  for (u32 j = 0; j < k; ++j) a.c[j] = p[j];
  return a;
}
ColsOut cols_out(u32 k, u32* const* p) {
  ColsOut a{};
  for (u32 j = 0; j < k; ++j) a.c[j] = p[j];
  return a;
}

u32 grid_for(u64 n, u64 per_block) {
  u64 g = ceil_div(n, per_block);
  if (g > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "grid too large");
  return (u32)(g ? g : 1);
}

// ---- wave / block scans ---------------------------------------------------

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

// Exclusive scan across the 256 threads; *total gets the block sum.
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

template <class T>
__global__ __launch_bounds__(WG) void k_scan_reduce(const T* in, u64 n, u64* bsum) {
  __shared__ u64 sh[WG / 64];
  u64 base = (u64)blockIdx.x * SCAN_TILE + (u64)threadIdx.x * SCAN_IPT;
  u64 s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i)
    if (base + i < n) s += (u64)in[base + i];
  u64 tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// out = exclusive (or inclusive) scan of in, offset by bpre[block].
template <class T>
__global__ __launch_bounds__(WG) void k_scan_down(const T* in, u64* out, u64 n, const u64* bpre,
                                                  int inclusive, u64* d_total) {
  __shared__ u64 sh[WG / 64];
  u64 base = (u64)blockIdx.x * SCAN_TILE + (u64)threadIdx.x * SCAN_IPT;
  u64 v[SCAN_IPT];
  u64 s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    v[i] = (base + i < n) ? (u64)in[base + i] : 0;
    s += v[i];
  }
  u64 tot;
  u64 run = block_excl_scan(s, sh, &tot) + (bpre ? bpre[blockIdx.x] : 0);
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    if (base + i < n) out[base + i] = inclusive ? run + v[i] : run;
    run += v[i];
  }
  if (d_total && !bpre && threadIdx.x == 0) *d_total = tot;
}

__global__ void k_set_total(const u64* bpre, const u64* bsum, u64 nb, u64* d_total) {
  *d_total = bpre[nb - 1] + bsum[nb - 1];
}

template <class T>
void scan_impl(Ctx c, const T* in, u64* out, u64 n, u64* d_total, int inclusive) {
  if (n == 0) {
    if (d_total) fill_u64(c, d_total, 1, 0);
    return;
  }
  u64 nb = ceil_div(n, SCAN_TILE);
  if (nb == 1) {
    k_scan_down<T><<<1, WG, 0, c.s>>>(in, out, n, nullptr, inclusive, d_total);
    WCDL_HIP(hipGetLastError());
    return;
  }
  DBuf<u64> bsum(c.mem, nb), bpre(c.mem, nb);
  k_scan_reduce<T><<<grid_for(nb, 1), WG, 0, c.s>>>(in, n, bsum.get());
  WCDL_HIP(hipGetLastError());
  scan_impl<u64>(c, bsum.get(), bpre.get(), nb, nullptr, 0);
  k_scan_down<T><<<grid_for(nb, 1), WG, 0, c.s>>>(in, out, n, bpre.get(), inclusive, nullptr);
  WCDL_HIP(hipGetLastError());
  if (d_total) {
    k_set_total<<<1, 1, 0, c.s>>>(bpre.get(), bsum.get(), nb, d_total);
    WCDL_HIP(hipGetLastError());
  }
}

// ---- fills ---------------------------------------------------------------

template <class T>
__global__ void k_fill(T* p, u64 n, T v) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  u64 stride = (u64)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_copy(u32* dst, const u32* src, u64 n) {
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  u64 stride = (u64)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

u32 stream_grid(u64 n) {
  u64 g = ceil_div(n, WG);
  return (u32)(g < 65536 ? (g ? g : 1) : 65536);
}

// ---- column OR (bit width of keys) ---------------------------------------

__global__ __launch_bounds__(WG) void k_col_or(ColsIn a, u32 k, u64 n, u32* d_or) {
  u64 stride = (u64)gridDim.x * WG;
  for (u32 j = 0; j < k; ++j) {
    u32 acc = 0;
    for (u64 i = (u64)blockIdx.x * WG + threadIdx.x; i < n; i += stride) acc |= a.c[j][i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc |= __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr(&d_or[j], acc);
  }
}

// ---- radix sort ------------------------------------------------------------
//
// One pass = (digit histogram per tile) -> (exclusive scan, digit-major over
// tiles) -> (stable scatter).  The scatter ranks keys inside a tile with
// 64-lane ballots: the lanes holding the same 8-bit digit are found with
// eight ballots, the lowest of them updates a per-wave digit counter, and
// the tile is then written through LDS in digit order so global writes form
// contiguous runs.

__device__ inline u64 lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Lanes (among `valid` ones) whose digit equals this lane's digit.
__device__ inline u64 match_digit(u32 d, bool valid) {
  u64 m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    bool bit = (d >> b) & 1u;
    u64 bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__global__ __launch_bounds__(WG) void k_rs_hist(const u32* key, u64 n, u32 shift, u32* counts,
                                                u32 ntiles) {
  __shared__ u32 wcnt[WG / 64][256];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < (WG / 64) * 256; i += WG) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const u64 base = (u64)blockIdx.x * RS_TILE + (u64)w * (64 * RS_IPT);
#pragma unroll 4
  for (int i = 0; i < RS_IPT; ++i) {
    u64 idx = base + (u64)i * 64 + lane;
    bool valid = idx < n;
    u32 d = valid ? (key[idx] >> shift) & 255u : 0u;
    u64 m = match_digit(d, valid);
    if (valid && (m & lanemask_lt()) == 0) wcnt[w][d] += (u32)__popcll(m);
  }
  __syncthreads();
  u32 t = threadIdx.x;
  u32 s = 0;
#pragma unroll
  for (int ww = 0; ww < WG / 64; ++ww) s += wcnt[ww][t];
  counts[(u64)t * ntiles + blockIdx.x] = s;
}

__global__ __launch_bounds__(WG) void k_rs_scatter(ColsIn in, ColsOut out, u32 k, const u32* key,
                                                   u64 n, u32 shift, const u64* offs, u32 ntiles) {
  __shared__ u32 wcnt[WG / 64][256];
  __shared__ u32 dstart[256];
  __shared__ u64 gofs[256];
  __shared__ u64 sh[WG / 64];
  __shared__ u32 tile[RS_TILE];
  __shared__ uint8_t tdig[RS_TILE];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < (WG / 64) * 256; i += WG) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const u64 tbase = (u64)blockIdx.x * RS_TILE;
  const u64 base = tbase + (u64)w * (64 * RS_IPT);
  u32 dig[RS_IPT];
  u32 pos[RS_IPT];
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    u64 idx = base + (u64)i * 64 + lane;
    bool valid = idx < n;
    u32 d = valid ? (key[idx] >> shift) & 255u : 0u;
    u64 m = match_digit(d, valid);
    u32 below = (u32)__popcll(m & lanemask_lt());
    u32 prev = valid ? wcnt[w][d] : 0u;
    if (valid && below == 0) wcnt[w][d] = prev + (u32)__popcll(m);
    dig[i] = valid ? d : 256u;
    pos[i] = prev + below;
  }
  __syncthreads();
  {
    u32 t = threadIdx.x;
    u32 c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
    wcnt[0][t] = 0;
    wcnt[1][t] = c0;
    wcnt[2][t] = c0 + c1;
    wcnt[3][t] = c0 + c1 + c2;
    u64 tot;
    u64 ds = block_excl_scan((u64)(c0 + c1 + c2 + c3), sh, &tot);
    dstart[t] = (u32)ds;
    gofs[t] = offs[(u64)t * ntiles + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    if (dig[i] < 256u) {
      pos[i] += dstart[dig[i]] + wcnt[w][dig[i]];
      tdig[pos[i]] = (uint8_t)dig[i];
    }
  }
  const u32 tn = (u32)((n - tbase) < (u64)RS_TILE ? (n - tbase) : (u64)RS_TILE);
  for (u32 j = 0; j < k; ++j) {
    const u32* src = in.c[j];
    u32* dst = out.c[j];
#pragma unroll
    for (int i = 0; i < RS_IPT; ++i)
      if (dig[i] < 256u) tile[pos[i]] = src[base + (u64)i * 64 + lane];
    __syncthreads();
    for (u32 t = threadIdx.x; t < tn; t += WG) {
      u32 d = tdig[t];
      dst[gofs[d] + (t - dstart[d])] = tile[t];
    }
    __syncthreads();
  }
}

// ---- grouped sort -----------------------------------------------------------
//
// Rows already non-decreasing in columns 0..k-2 (groups) and unsorted, with
// repeats, in column k-1 -- what a join emits when the head starts with the
// join's first variables -- whose last values are small (below 2^zbits):
// each group gets a bitmap of its last values in LDS, one bit set per row,
// and the set bits read back in order are the group's sorted unique rows.
// Two streaming passes over the last column (count, then write) replace the
// global radix passes over every column.

constexpr u32 GB_WORDS = 8192;   // bitmap words of one tile (32 KB of LDS)
constexpr u32 GB_GROUPS = 1024;  // most groups in one tile

// flags[i] = 1 where row i starts a group (differs from row i-1 in 0..kp-1).
__global__ __launch_bounds__(WG) void k_group_flags(ColsIn a, u32 kp, u64 n, u32* flags) {
  const u64 i = (u64)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  u32 f = i == 0 ? 1u : 0u;
  for (u32 j = 0; j < kp && !f; ++j) f = a.c[j][i] != a.c[j][i - 1] ? 1u : 0u;
  flags[i] = f;
}

// Tile t = groups [t*G, (t+1)*G), `wpg` bitmap words each.  EMIT = false:
// cnt[t] = the tile's unique rows.  EMIT = true: those rows, in order, from
// off[t] on -- leading columns from the group's first row, last column from
// the bit.  Dynamic LDS: G*wpg bitmap words, then G+1 group starts.
template <bool EMIT>
__global__ __launch_bounds__(WG) void k_group_bitmap(ColsIn a, u32 k, u64 n, const u64* gs,
                                                     u64 ng, u32 G, u32 wpg, u32* cnt,
                                                     const u64* off, ColsOut o) {
  extern __shared__ u32 lds[];
  __shared__ u64 sh[WG / 64];
  u32* bm = lds;
  u64* gsl = reinterpret_cast<u64*>(lds + ((G * wpg + 1u) & ~1u));
  const u64 g0 = (u64)blockIdx.x * G;
  const u32 ngl = (u32)((ng - g0) < G ? (ng - g0) : G);
  const u32 W = ngl * wpg;
  for (u32 w = threadIdx.x; w < W; w += WG) bm[w] = 0;
  for (u32 j = threadIdx.x; j <= ngl; j += WG) gsl[j] = g0 + j < ng ? gs[g0 + j] : n;
  __syncthreads();
  const u32* last = a.c[k - 1];
  const u64 r0 = gsl[0], r1 = gsl[ngl];
  for (u64 r = r0 + threadIdx.x; r < r1; r += WG) {
    u32 lo = 0, hi = ngl;  // gsl[lo] <= r < gsl[hi]
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (gsl[mid] <= r) lo = mid; else hi = mid;
    }
    const u32 z = last[r];
    atomicOr(&bm[lo * wpg + (z >> 5)], 1u << (z & 31));
  }
  __syncthreads();
  if (!EMIT) {
    u64 mine = 0;
    for (u32 w = threadIdx.x; w < W; w += WG) mine += (u64)__popc(bm[w]);
    u64 tot;
    block_excl_scan(mine, sh, &tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = (u32)tot;
    return;
  }
  // Rounds of WG consecutive words: one word per thread, positions by a
  // block scan, so a round's rows are written contiguously.
  u64 base = off[blockIdx.x];
  for (u32 w0 = 0; w0 < W; w0 += WG) {
    const u32 w = w0 + threadIdx.x;
    u32 bits = w < W ? bm[w] : 0u;
    u64 tot;
    u64 at = base + block_excl_scan((u64)__popc(bits), sh, &tot);
    if (bits) {
      const u32 g = w / wpg;
      const u32 zhi = (w - g * wpg) << 5;
      const u64 row = gsl[g];
      u32 pre[MAXA];
#pragma unroll
      for (u32 j = 0; j < (u32)MAXA; ++j)
        if (j + 1 < k) pre[j] = a.c[j][row];
      while (bits) {
        const u32 bit = (u32)__ffs(bits) - 1u;
        bits &= bits - 1u;
#pragma unroll
        for (u32 j = 0; j < (u32)MAXA; ++j)
          if (j + 1 < k) o.c[j][at] = pre[j];
        o.c[k - 1][at] = zhi | bit;
        ++at;
      }
    }
    base += tot;
  }
}

// ---- row comparisons and tiled searches ------------------------------------

__device__ inline void load_row(const ColsIn& a, u32 k, u64 i, u32 (&r)[MAXA]) {
#pragma unroll
  for (int j = 0; j < MAXA; ++j) r[j] = (j < (int)k) ? a.c[j][i] : 0u;
}

// Is row i of b lexicographically less than key?
__device__ inline bool row_less(const ColsIn& b, u32 k, u64 i, const u32 (&key)[MAXA]) {
#pragma unroll
  for (int j = 0; j < MAXA; ++j) {
    if (j < (int)k) {
      u32 x = b.c[j][i];
      if (x != key[j]) return x < key[j];
    }
  }
  return false;
}

__device__ inline bool row_equal(const ColsIn& b, u32 k, u64 i, const u32 (&key)[MAXA]) {
#pragma unroll
  for (int j = 0; j < MAXA; ++j)
    if (j < (int)k && b.c[j][i] != key[j]) return false;
  return true;
}

__device__ inline u64 row_lower_bound(const ColsIn& b, u32 k, u64 lo, u64 hi,
                                      const u32 (&key)[MAXA]) {
  while (lo < hi) {
    u64 mid = lo + ((hi - lo) >> 1);
    if (row_less(b, k, mid, key)) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// bounds[t] = lower bound in b of a's row t*SEARCH_TILE (t < ntiles),
// bounds[ntiles] = nb: the rows of a's tile t can only equal rows of b in
// [bounds[t], bounds[t+1]).  One thread per boundary, so the searches'
// dependent loads overlap across the whole grid.
__global__ __launch_bounds__(WG) void k_tile_bounds(ColsIn a, ColsIn b, u32 k, u64 nb, u64 ntiles,
                                                    u64* bounds) {
  const u64 t = (u64)blockIdx.x * WG + threadIdx.x;
  if (t > ntiles) return;
  if (t == ntiles || nb == 0) {
    bounds[t] = t == ntiles ? nb : 0;
    return;
  }
  u32 key[MAXA];
  load_row(a, k, t * SEARCH_TILE, key);
  bounds[t] = row_lower_bound(b, k, 0, nb, key);
}

__global__ __launch_bounds__(WG) void k_adjacent_flags(ColsIn a, u32 k, u64 n, u32* flags) {
  u64 i = (u64)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  u32 f = 1;
  if (i > 0) {
    f = 0;
    for (u32 j = 0; j < k; ++j)
      if (a.c[j][i] != a.c[j][i - 1]) { f = 1; break; }
  }
  flags[i] = f;
}

// Stream compaction in two passes over the flags, with no per-row positions:
// per-tile counts (tiles of SCAN_TILE rows), a scan of those, then each tile
// ranks its flagged rows itself.  Wave w of a tile owns rows
// [w*64*SCAN_IPT, (w+1)*64*SCAN_IPT) of it, 64 consecutive rows per step, so
// every load and store of a step is one contiguous run.
__global__ __launch_bounds__(WG) void k_flag_tiles(const u32* flags, u64 n, u32* tcnt) {
  __shared__ u64 sh[WG / 64];
  const u64 base = (u64)blockIdx.x * SCAN_TILE + threadIdx.x;
  u64 s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    const u64 r = base + (u64)i * WG;
    if (r < n) s += flags[r] ? 1u : 0u;
  }
  u64 tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) tcnt[blockIdx.x] = (u32)tot;
}

// Flagged rows of a (or, with idx, their row numbers) in order, from
// toff[tile] on.
__global__ __launch_bounds__(WG) void k_compact_tiles(ColsIn a, ColsOut o, u32 k, u64 n,
                                                      const u32* flags, const u64* toff,
                                                      u64* idx) {
  __shared__ u32 wc[WG / 64];
  const u32 wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const u64 wbase = (u64)blockIdx.x * SCAN_TILE + (u64)wave * (64 * SCAN_IPT) + lane;
  const u64 below = (1ull << lane) - 1ull;
  u32 f[SCAN_IPT];
  u32 cnt = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    const u64 r = wbase + (u64)i * 64;
    f[i] = (r < n && flags[r]) ? 1u : 0u;
    cnt += (u32)__popcll(__ballot(f[i]));
  }
  if (lane == 0) wc[wave] = cnt;
  __syncthreads();
  u64 at = toff[blockIdx.x];
  for (u32 w = 0; w < wave; ++w) at += wc[w];
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    const u64 mask = __ballot(f[i]);
    if (f[i]) {
      const u64 r = wbase + (u64)i * 64;
      const u64 p = at + (u64)__popcll(mask & below);
      if (idx) {
        idx[p] = r;
      } else {
        for (u32 j = 0; j < k; ++j) o.c[j][p] = a.c[j][r];
      }
    }
    at += (u64)__popcll(mask);
  }
}

// Splitters of a window [lo, hi) of b in LDS: row lo + j*stride for j < ns,
// column-major (sp[col * S + j]); stride 1 stages the window whole.
struct Splitters {
  u64 lo, hi, stride;
  u32 ns;
};

__device__ inline void stage_splitters(const ColsIn& b, u32 k, u64 lo, u64 hi, u32 S, u32* sp,
                                       Splitters* out) {
  const u64 w = hi - lo;
  const u64 stride = w <= S ? 1 : (w + S - 1) / S;
  const u32 ns = (u32)((w + stride - 1) / stride);
  for (u32 j = threadIdx.x; j < ns; j += WG)
    for (u32 col = 0; col < k; ++col) sp[col * S + j] = b.c[col][lo + (u64)j * stride];
  if (threadIdx.x == 0) *out = Splitters{lo, hi, stride, ns};
}

// Is `key` a row of b?  Lower bound among the splitters in LDS, then among
// the at most stride-1 rows of b between two splitters.
__device__ inline bool in_window(const ColsIn& b, u32 k, const Splitters& w, const u32* sp, u32 S,
                                 const u32 (&key)[MAXA]) {
  u32 lo = 0, hi = w.ns;  // first splitter >= key
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    bool less = false;
#pragma unroll
    for (int c = 0; c < MAXA; ++c) {
      if (c < (int)k) {
        const u32 v = sp[c * S + mid];
        if (v != key[c]) { less = v < key[c]; break; }
      }
    }
    if (less) lo = mid + 1; else hi = mid;
  }
  if (w.stride == 1) {
    if (lo >= w.ns) return false;
#pragma unroll
    for (int c = 0; c < MAXA; ++c)
      if (c < (int)k && sp[c * S + lo] != key[c]) return false;
    return true;
  }
  const u64 L = lo == 0 ? w.lo : w.lo + (u64)(lo - 1) * w.stride + 1;
  const u64 R = lo < w.ns ? w.lo + (u64)lo * w.stride : w.hi;
  const u64 p = row_lower_bound(b, k, L, R, key);
  return p < w.hi && row_equal(b, k, p, key);
}

// flags[i] = 1 if row i of `a` is in neither b nor c (c may be empty).  Each
// tile of a searches the windows of b and c its rows can fall in, through S
// splitters per window staged in LDS (2*S*k words of dynamic LDS).
__global__ __launch_bounds__(WG) void k_absent_flags(ColsIn a, ColsIn b, ColsIn c, u32 k, u64 na,
                                                     const u64* bb, const u64* bc, u32 S,
                                                     u32* flags) {
  extern __shared__ u32 sp[];
  __shared__ Splitters sw[2];
  const u64 t0 = (u64)blockIdx.x * SEARCH_TILE;
  const u64 t1 = (t0 + SEARCH_TILE < na) ? t0 + SEARCH_TILE : na;
  const u64 blo = bb[blockIdx.x], bhi = bb[blockIdx.x + 1];
  const u64 clo = bc[blockIdx.x], chi = bc[blockIdx.x + 1];
  u32* spb = sp;
  u32* spc = sp + (size_t)S * k;
  stage_splitters(b, k, blo, bhi, S, spb, &sw[0]);
  stage_splitters(c, k, clo, chi, S, spc, &sw[1]);
  __syncthreads();
  const Splitters wb = sw[0], wc = sw[1];
  for (u64 i = t0 + threadIdx.x; i < t1; i += WG) {
    u32 key[MAXA];
    load_row(a, k, i, key);
    const bool in_b = in_window(b, k, wb, spb, S, key);
    const bool in_c = in_window(c, k, wc, spc, S, key);
    flags[i] = (in_b || in_c) ? 0u : 1u;
  }
}

// ---- merge path --------------------------------------------------------------
//
// The merge of two disjoint sorted runs a, b is cut into output tiles of
// MP_TILE rows.  A first kernel finds, for every tile boundary d, how many of
// the first d merged rows come from a (a binary search along the diagonal
// i + j = d).  A workgroup then stages its tile's slices of a and b in LDS,
// each thread finds its own sub-diagonal there and merges MP_PT rows into a
// permutation, and the columns are written out coalesced.

constexpr u32 MP_PT = 8;
constexpr u32 MP_TILE = WG * MP_PT;  // 2048 output rows per workgroup

__device__ inline bool row_lt_ab(const ColsIn& a, u64 i, const ColsIn& b, u64 j, u32 k) {
#pragma unroll
  for (int c = 0; c < MAXA; ++c) {
    if (c < (int)k) {
      const u32 x = a.c[c][i], y = b.c[c][j];
      if (x != y) return x < y;
    }
  }
  return false;
}

// split[t] = rows of a among the first min(t*MP_TILE, na+nb) merged rows.
__global__ __launch_bounds__(WG) void k_merge_split(ColsIn a, ColsIn b, u32 k, u64 na, u64 nb,
                                                    u64 nsplit, u64* split) {
  const u64 t = (u64)blockIdx.x * WG + threadIdx.x;
  if (t >= nsplit) return;
  const u64 d = t * MP_TILE < na + nb ? t * MP_TILE : na + nb;
  u64 lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if (row_lt_ab(a, mid, b, d - 1 - mid, k)) lo = mid + 1; else hi = mid;
  }
  split[t] = lo;
}

__global__ __launch_bounds__(WG) void k_merge_tile(ColsIn a, ColsIn b, ColsOut o, u32 k, u64 na,
                                                   u64 nb, const u64* split) {
  extern __shared__ __align__(16) u32 msm[];  // k columns of MP_TILE rows, then the permutation
  u32* perm = msm + (u64)k * MP_TILE;
  const u64 t = blockIdx.x;
  const u64 d0 = t * MP_TILE, d1 = d0 + MP_TILE < na + nb ? d0 + MP_TILE : na + nb;
  const u64 i0 = split[t], i1 = split[t + 1];
  const u32 nA = (u32)(i1 - i0), n = (u32)(d1 - d0), nB = n - nA;
  const u64 j0 = d0 - i0;
  for (u32 c = 0; c < k; ++c) {
    u32* col = msm + (u64)c * MP_TILE;
    for (u32 r = threadIdx.x; r < n; r += WG) col[r] = r < nA ? a.c[c][i0 + r] : b.c[c][j0 + r - nA];
  }
  __syncthreads();
  // Row x of the tile's a-part vs row y of its b-part (y indexes the b-part).
  auto less_ab = [&](u32 x, u32 y) {
    for (u32 c = 0; c < k; ++c) {
      const u32 u = msm[(u64)c * MP_TILE + x], v = msm[(u64)c * MP_TILE + nA + y];
      if (u != v) return u < v;
    }
    return false;
  };
  const u32 ld = threadIdx.x * MP_PT < n ? threadIdx.x * MP_PT : n;
  u32 lo = ld > nB ? ld - nB : 0, hi = ld < nA ? ld : nA;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if (less_ab(mid, ld - 1 - mid)) lo = mid + 1; else hi = mid;
  }
  u32 ia = lo, ib = ld - lo;
  for (u32 e = 0; e < MP_PT && ld + e < n; ++e) {
    const bool take_a = ib >= nB || (ia < nA && less_ab(ia, ib));
    perm[ld + e] = take_a ? ia++ : nA + ib++;
  }
  __syncthreads();
  for (u32 c = 0; c < k; ++c) {
    const u32* col = msm + (u64)c * MP_TILE;
    u32* dst = o.c[c] + d0;
    for (u32 r = threadIdx.x; r < n; r += WG) dst[r] = col[perm[r]];
  }
}

__global__ __launch_bounds__(WG) void k_keep_flags(const u32* lead, u64 n, const u32* ids,
                                                   u64 nids, u32 keep_listed, u32* flags) {
  const u64 i = (u64)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const u32 v = lead[i];
  u64 lo = 0, hi = nids;
  while (lo < hi) {
    u64 mid = lo + ((hi - lo) >> 1);
    if (ids[mid] < v) lo = mid + 1; else hi = mid;
  }
  const u32 listed = (lo < nids && ids[lo] == v) ? 1u : 0u;
  flags[i] = listed == keep_listed ? 1u : 0u;
}

// Adjacent rows i-1, i with row i-1 >= row i (lexicographic): counted.
__global__ __launch_bounds__(WG) void k_order_violations(ColsIn a, u32 k, u64 n, u64* bad) {
  const u64 i = (u64)blockIdx.x * WG + threadIdx.x;
  if (i == 0 || i >= n) return;
  int cmp = 0;
  for (u32 j = 0; j < k && cmp == 0; ++j) {
    const u32 x = a.c[j][i - 1], y = a.c[j][i];
    cmp = x < y ? -1 : (x > y ? 1 : 0);
  }
  if (cmp >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(bad), 1ull);
}

__global__ void k_lead_range(const u32* col, u64 n, u32 v, u64* out) {
  u64 lo = 0, hi = n;
  while (lo < hi) {
    u64 mid = lo + ((hi - lo) >> 1);
    if (col[mid] < v) lo = mid + 1; else hi = mid;
  }
  u64 lo2 = lo, hi2 = n;
  while (lo2 < hi2) {
    u64 mid = lo2 + ((hi2 - lo2) >> 1);
    if (col[mid] <= v) lo2 = mid + 1; else hi2 = mid;
  }
  out[0] = lo;
  out[1] = lo2;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers

// Stream compaction by flags: count() scans the per-tile counts and returns
// the flagged rows' number (synchronises), so the caller can size the output
// exactly; write() puts the flagged rows of a in order into o (or their row
// numbers into idx).
struct FlagCompaction {
  Ctx c;
  const u32* flags;
  u64 n, ntiles;
  DBuf<u32> tcnt;
  DBuf<u64> toff;
  FlagCompaction(Ctx cx, const u32* f, u64 rows) : c(cx), flags(f), n(rows) {
    ntiles = ceil_div(n, (u64)SCAN_TILE);
    if (ntiles > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "compaction too large");
    tcnt = DBuf<u32>(c.mem, ntiles);
    toff = DBuf<u64>(c.mem, ntiles);
  }
  u64 count() {
    DBuf<u64> total(c.mem, 1);
    k_flag_tiles<<<(u32)ntiles, WG, 0, c.s>>>(flags, n, tcnt.get());
    WCDL_HIP(hipGetLastError());
    scan_u32_excl(c, tcnt.get(), toff.get(), ntiles, total.get());
    u64 h = 0;
    WCDL_HIP(hipMemcpyAsync(&h, total.get(), sizeof(u64), hipMemcpyDeviceToHost, c.s));
    WCDL_HIP(hipStreamSynchronize(c.s));
    return h;
  }
  void write(u32 k, const ColsIn& a, const ColsOut& o, u64* idx) {
    k_compact_tiles<<<(u32)ntiles, WG, 0, c.s>>>(a, o, k, n, flags, toff.get(), idx);
    WCDL_HIP(hipGetLastError());
  }
};

// Rows of a whose flag is set, in order, into o; returns their number once
// they are written (synchronises: callers read the result from any stream).
u64 compact_flagged(Ctx c, u32 k, const ColsIn& a, u64 n, const u32* flags, const ColsOut& o) {
  FlagCompaction fc(c, flags, n);
  const u64 h = fc.count();
  if (h) fc.write(k, a, o, nullptr);
  WCDL_HIP(hipStreamSynchronize(c.s));
  return h;
}

// ---- repeats inside tiles ----------------------------------------------------
//
// A join emits the repeats of a row close together when the same binding is
// reached through several values of a projected-away variable.  Ahead of a
// full sort, each workgroup keeps one copy of every row repeated inside its
// tile of TILE_DEDUP consecutive rows: the tile goes to LDS, each row claims
// a slot of an LDS hash set by compare-and-swap of its index (linear
// probing over twice as many slots as rows, so every probe ends), and a row
// that meets an equal row in the set is dropped.

constexpr u32 TILE_DEDUP = 2048;
constexpr u32 TILE_DEDUP_SLOTS = 2 * TILE_DEDUP;

__global__ __launch_bounds__(WG) void k_tile_first(ColsIn in, u32 k, u64 n, u32* keep) {
  extern __shared__ u32 lds[];
  u32* rows = lds;                          // k x TILE_DEDUP
  u32* table = lds + k * TILE_DEDUP;        // TILE_DEDUP_SLOTS row indices, ~0u = empty
  const u64 base = (u64)blockIdx.x * TILE_DEDUP;
  const u32 m = (u32)(n - base < TILE_DEDUP ? n - base : TILE_DEDUP);
  for (u32 j = 0; j < k; ++j)
    for (u32 i = threadIdx.x; i < m; i += WG) rows[j * TILE_DEDUP + i] = in.c[j][base + i];
  for (u32 t = threadIdx.x; t < TILE_DEDUP_SLOTS; t += WG) table[t] = ~0u;
  __syncthreads();
  for (u32 i = threadIdx.x; i < m; i += WG) {
    u32 h = 0x9e3779b9u;
    for (u32 j = 0; j < k; ++j) {
      h = (h ^ rows[j * TILE_DEDUP + i]) * 0x85ebca6bu;
      h ^= h >> 13;
    }
    u32 slot = h & (TILE_DEDUP_SLOTS - 1);
    u32 first = 1, open = 1;
    while (open) {
      const u32 prev = atomicCAS(&table[slot], ~0u, i);
      if (prev == ~0u) {
        open = 0;  // this row holds the slot
      } else {
        u32 same = 1;
        for (u32 j = 0; j < k; ++j) same &= rows[j * TILE_DEDUP + prev] == rows[j * TILE_DEDUP + i] ? 1u : 0u;
        if (same) {
          first = 0;
          open = 0;
        } else {
          slot = (slot + 1) & (TILE_DEDUP_SLOTS - 1);
        }
      }
    }
    keep[base + i] = first;
  }
}

u64 drop_tile_repeats(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32* const* out_cols) {
  if (k == 0 || k > 4) throw Error(WCDL_E_UNSUPPORTED, "tile deduplication arity");
  if (n == 0) return 0;
  DBuf<u32> keep(c.mem, n);
  const u64 tiles = ceil_div(n, (u64)TILE_DEDUP);
  const size_t lds = ((size_t)k * TILE_DEDUP + TILE_DEDUP_SLOTS) * sizeof(u32);
  const ColsIn a = cols_in(k, in_cols);
  k_tile_first<<<(u32)tiles, WG, lds, c.s>>>(a, k, n, keep.get());
  WCDL_HIP(hipGetLastError());
  return compact_flagged(c, k, a, n, keep.get(), cols_out(k, out_cols));
}

u64 select_leading(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32 lead_col, const u32* ids,
                   u64 nids, bool keep_listed, u32* const* out_cols) {
  if (n == 0) return 0;
  DBuf<u32> flags(c.mem, n);
  k_keep_flags<<<grid_for(n, WG), WG, 0, c.s>>>(in_cols[lead_col], n, ids, nids,
                                                 keep_listed ? 1u : 0u, flags.get());
  WCDL_HIP(hipGetLastError());
  return compact_flagged(c, k, cols_in(k, in_cols), n, flags.get(), cols_out(k, out_cols));
}

u64 order_violations(Ctx c, u32 k, const u32* const* cols, u64 n) {
  if (n < 2) return 0;
  DBuf<u64> bad(c.mem, 1);
  fill_u64(c, bad.get(), 1, 0);
  k_order_violations<<<grid_for(n, WG), WG, 0, c.s>>>(cols_in(k, cols), k, n, bad.get());
  WCDL_HIP(hipGetLastError());
  u64 h = 0;
  WCDL_HIP(hipMemcpyAsync(&h, bad.get(), sizeof(u64), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipStreamSynchronize(c.s));
  return h;
}

void lead_range(Ctx c, const u32* col, u64 n, u32 v, u64* d_out) {
  k_lead_range<<<1, 1, 0, c.s>>>(col, n, v, d_out);
  WCDL_HIP(hipGetLastError());
}
// ---------------------------------------------------------------------------

void scan_u32_excl(Ctx c, const u32* in, u64* out, u64 n, u64* d_total) {
  scan_impl<u32>(c, in, out, n, d_total, 0);
}
void scan_u64_excl(Ctx c, const u64* in, u64* out, u64 n, u64* d_total) {
  scan_impl<u64>(c, in, out, n, d_total, 0);
}
void scan_u64_incl(Ctx c, const u64* in, u64* out, u64 n, u64* d_total) {
  scan_impl<u64>(c, in, out, n, d_total, 1);
}

void fill_u32(Ctx c, u32* p, u64 n, u32 v) {
  if (!n) return;
  k_fill<u32><<<stream_grid(n), WG, 0, c.s>>>(p, n, v);
  WCDL_HIP(hipGetLastError());
}
void fill_u64(Ctx c, u64* p, u64 n, u64 v) {
  if (!n) return;
  k_fill<u64><<<stream_grid(n), WG, 0, c.s>>>(p, n, v);
  WCDL_HIP(hipGetLastError());
}
void copy_u32(Ctx c, u32* dst, const u32* src, u64 n) {
  if (!n) return;
  k_copy<<<stream_grid(n), WG, 0, c.s>>>(dst, src, n);
  WCDL_HIP(hipGetLastError());
}

void column_or(Ctx c, u32 k, const u32* const* cols, u64 n, u32* d_or) {
  fill_u32(c, d_or, k, 0);
  if (!n) return;
  u32 g = stream_grid(n);
  if (g > 4096) g = 4096;
  k_col_or<<<g, WG, 0, c.s>>>(cols_in(k, cols), k, n, d_or);
  WCDL_HIP(hipGetLastError());
}

// ---- small sorts -----------------------------------------------------------
//
// Up to SMALL_SORT rows are sorted by one workgroup in LDS: the columns are
// loaded once, a bitonic network orders row indices by (row, index), and the
// rows are written out in that order.  One launch instead of the radix
// passes' four per 8-bit digit, for the small deltas of long-tail rounds.

constexpr u32 SMALL_SORT = 2048;

__device__ inline bool row_less(const u32* keys, u32 k, uint16_t a, uint16_t b) {
  for (u32 j = 0; j < k; ++j) {
    const u32 x = keys[j * SMALL_SORT + a], y = keys[j * SMALL_SORT + b];
    if (x != y) return x < y;
  }
  return a < b;
}

__global__ __launch_bounds__(WG) void k_small_sort(ColsIn in, ColsOut out, u32 k, u32 n, u32 n2) {
  extern __shared__ u32 lds[];
  u32* keys = lds;                                             // k x SMALL_SORT
  uint16_t* idx = reinterpret_cast<uint16_t*>(lds + k * SMALL_SORT);  // n2 (power of two)
  for (u32 j = 0; j < k; ++j)
    for (u32 i = threadIdx.x; i < n2; i += WG) keys[j * SMALL_SORT + i] = i < n ? in.c[j][i] : ~0u;
  for (u32 i = threadIdx.x; i < n2; i += WG) idx[i] = (uint16_t)i;
  __syncthreads();
  for (u32 size = 2; size <= n2; size <<= 1)
    for (u32 stride = size >> 1; stride > 0; stride >>= 1) {
      for (u32 t = threadIdx.x; t < n2 / 2; t += WG) {
        const u32 i = 2 * stride * (t / stride) + t % stride, j = i + stride;
        const bool up = (i & size) == 0;
        const uint16_t a = idx[i], b = idx[j];
        if (row_less(keys, k, b, a) == up) {
          idx[i] = b;
          idx[j] = a;
        }
      }
      __syncthreads();
    }
  for (u32 j = 0; j < k; ++j)
    for (u32 i = threadIdx.x; i < n; i += WG) out.c[j][i] = keys[j * SMALL_SORT + idx[i]];
}

void radix_sort_rows(Ctx c, u32 k, const u32* const* in_cols, u32* const* out_cols, u64 n,
                     const u32* col_bits) {
  if (k == 0 || k > (u32)MAXA) throw Error(WCDL_E_UNSUPPORTED, "radix sort arity");
  if (n > 1 && n <= SMALL_SORT) {
    u32 n2 = 2;
    while (n2 < n) n2 <<= 1;
    const size_t lds = (size_t)k * SMALL_SORT * sizeof(u32) + (size_t)n2 * sizeof(uint16_t);
    k_small_sort<<<1, WG, lds, c.s>>>(cols_in(k, in_cols), cols_out(k, out_cols), k, (u32)n, n2);
    WCDL_HIP(hipGetLastError());
    return;
  }
  // Digit passes from the least significant digit of the last column up.
  std::vector<std::pair<u32, u32>> passes;  // (column, shift)
  for (int j = (int)k - 1; j >= 0; --j)
    for (u32 sh = 0; sh < col_bits[j]; sh += 8) passes.push_back({(u32)j, sh});
  if (n <= 1 || passes.empty()) {
    for (u32 j = 0; j < k; ++j)
      if (n) copy_u32(c, out_cols[j], in_cols[j], n);
    return;
  }
  const u32 ntiles = grid_for(n, RS_TILE);
  DBuf<u32> counts(c.mem, (u64)256 * ntiles);
  DBuf<u64> offs(c.mem, (u64)256 * ntiles);
  std::vector<DBuf<u32>> tmp;
  for (u32 j = 0; j < k; ++j) tmp.emplace_back(c.mem, n);
  const size_t P = passes.size();
  const u32* const* src = in_cols;
  std::vector<const u32*> src_v(k);
  std::vector<u32*> dst_v(k);
  for (size_t p = 0; p < P; ++p) {
    bool to_out = ((P - 1 - p) % 2) == 0;
    for (u32 j = 0; j < k; ++j) dst_v[j] = to_out ? out_cols[j] : tmp[j].get();
    const u32* key = src[passes[p].first];
    k_rs_hist<<<ntiles, WG, 0, c.s>>>(key, n, passes[p].second, counts.get(), ntiles);
    WCDL_HIP(hipGetLastError());
    scan_u32_excl(c, counts.get(), offs.get(), (u64)256 * ntiles, nullptr);
    k_rs_scatter<<<ntiles, WG, 0, c.s>>>(cols_in(k, src), cols_out(k, dst_v.data()), k, key, n,
                                         passes[p].second, offs.get(), ntiles);
    WCDL_HIP(hipGetLastError());
    for (u32 j = 0; j < k; ++j) src_v[j] = dst_v[j];
    src = src_v.data();
  }
}

bool sort_unique_grouped(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32 zbits,
                         u32* const* out_cols, u64* out_n) {
  if (k < 2 || k > (u32)MAXA || zbits > 18) return false;
  *out_n = 0;
  if (n == 0) return true;
  const ColsIn A = cols_in(k, in_cols);
  DBuf<u32> flags(c.mem, n);
  k_group_flags<<<grid_for(n, WG), WG, 0, c.s>>>(A, k - 1, n, flags.get());
  WCDL_HIP(hipGetLastError());
  u64 ng = 0;
  DBuf<u64> gs;
  const u32 wpg = zbits <= 5 ? 1u : 1u << (zbits - 5);
  {
    FlagCompaction fc(c, flags.get(), n);
    ng = fc.count();
    // Each pass scans every group's bitmap: worth it while that is at most
    // two words per row.
    if (ng * wpg > 2 * n) return false;
    gs = DBuf<u64>(c.mem, ng);  // group starts: row numbers of the flagged rows
    fc.write(k, A, ColsOut{}, gs.get());
  }
  flags = DBuf<u32>();
  const u32 G = std::min<u32>(GB_GROUPS, GB_WORDS / wpg);
  const u64 ntiles = ceil_div(ng, (u64)G);
  if (ntiles > 0x7fffffffull) return false;
  const size_t lds = (size_t)((G * wpg + 1u) & ~1u) * 4 + (size_t)(G + 1) * 8;
  DBuf<u32> cnt(c.mem, ntiles);
  DBuf<u64> off(c.mem, ntiles), total(c.mem, 1);
  const ColsOut O = cols_out(k, out_cols);
  k_group_bitmap<false><<<(u32)ntiles, WG, lds, c.s>>>(A, k, n, gs.get(), ng, G, wpg, cnt.get(),
                                                      nullptr, O);
  WCDL_HIP(hipGetLastError());
  scan_u32_excl(c, cnt.get(), off.get(), ntiles, total.get());
  k_group_bitmap<true><<<(u32)ntiles, WG, lds, c.s>>>(A, k, n, gs.get(), ng, G, wpg, cnt.get(),
                                                     off.get(), O);
  WCDL_HIP(hipGetLastError());
  WCDL_HIP(hipMemcpyAsync(out_n, total.get(), sizeof(u64), hipMemcpyDeviceToHost, c.s));
  WCDL_HIP(hipStreamSynchronize(c.s));
  return true;
}

u64 unique_rows(Ctx c, u32 k, const u32* const* in_cols, u64 n, u32* const* out_cols) {
  if (n == 0) return 0;
  DBuf<u32> flags(c.mem, n);
  ColsIn a = cols_in(k, in_cols);
  k_adjacent_flags<<<grid_for(n, WG), WG, 0, c.s>>>(a, k, n, flags.get());
  WCDL_HIP(hipGetLastError());
  return compact_flagged(c, k, a, n, flags.get(), cols_out(k, out_cols));
}

u64 set_difference(Ctx c, u32 k, const u32* const* a, u64 na, const u32* const* b, u64 nb,
                   u32* const* out, const u32* const* b2, u64 nb2) {
  if (na == 0) return 0;
  ColsIn A = cols_in(k, a);
  if (nb == 0 && nb2 == 0) {
    for (u32 j = 0; j < k; ++j) copy_u32(c, out[j], a[j], na);
    return na;
  }
  DBuf<u32> flags(c.mem, na);
  const ColsIn B = nb ? cols_in(k, b) : ColsIn{}, B2 = nb2 ? cols_in(k, b2) : ColsIn{};
  const u32 S = AF_WORDS / (2 * k);
  const u64 ntiles = ceil_div(na, (u64)SEARCH_TILE);
  DBuf<u64> bb(c.mem, ntiles + 1), bc(c.mem, ntiles + 1);
  k_tile_bounds<<<grid_for(ntiles + 1, WG), WG, 0, c.s>>>(A, B, k, nb, ntiles, bb.get());
  WCDL_HIP(hipGetLastError());
  k_tile_bounds<<<grid_for(ntiles + 1, WG), WG, 0, c.s>>>(A, B2, k, nb2, ntiles, bc.get());
  WCDL_HIP(hipGetLastError());
  k_absent_flags<<<(u32)ntiles, WG, (size_t)2 * S * k * sizeof(u32), c.s>>>(
      A, B, B2, k, na, bb.get(), bc.get(), S, flags.get());
  WCDL_HIP(hipGetLastError());
  bb = DBuf<u64>();
  bc = DBuf<u64>();
  return compact_flagged(c, k, A, na, flags.get(), cols_out(k, out));
}

void merge_disjoint(Ctx c, u32 k, const u32* const* a, u64 na, const u32* const* b, u64 nb,
                    u32* const* out) {
  if (na + nb == 0) return;
  ColsIn A = cols_in(k, a), B = cols_in(k, b);
  ColsOut O = cols_out(k, out);
  if (na == 0 || nb == 0) {
    for (u32 j = 0; j < k; ++j) copy_u32(c, out[j], na ? a[j] : b[j], na ? na : nb);
    return;
  }
  const u64 ntiles = ceil_div(na + nb, (u64)MP_TILE);
  if (ntiles > 0x7fffffffull) throw Error(WCDL_E_UNSUPPORTED, "merge too large");
  DBuf<u64> split(c.mem, ntiles + 1);
  k_merge_split<<<grid_for(ntiles + 1, WG), WG, 0, c.s>>>(A, B, k, na, nb, ntiles + 1, split.get());
  WCDL_HIP(hipGetLastError());
  const size_t lds = (size_t)(k + 1) * MP_TILE * sizeof(u32);
  WCDL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_merge_tile),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  k_merge_tile<<<(u32)ntiles, WG, lds, c.s>>>(A, B, O, k, na, nb, split.get());
  WCDL_HIP(hipGetLastError());
}

}  // namespace wcdl
