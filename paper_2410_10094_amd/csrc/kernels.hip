// HIP kernels for sparse-sparse tensor contraction on gfx950 (CDNA4).
//
// Pipeline of the global-hash path (see sptc.h for the method and its
// citations; grouped.hip holds the X-grouped path):
//   plan:    fill Y table -> key_count -> scan counts -> y_scatter -> x_probe -> scan products
//   execute: fill output hash -> expand_acc -> compact (count, scan, fill)
//
// Everything is wave64-native: reductions and scans use 64-lane shuffles and
// one LDS slot per wave; hash tables are open-addressing with linear probing
// and 64-bit CAS on the key; values accumulate with hardware FP64 atomics.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {


// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_empty(uint4* __restrict__ slots, int64_t n, DevStatus* st) {
  const uint4 e = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
  if (st && blockIdx.x == 0 && threadIdx.x == 0) st->err = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    slots[i] = e;
}

// A1: count entries per packed key (Y by contracting key; X by free key on
// the grouped path) in an open-addressing table with linear probing.
__global__ __launch_bounds__(256) void k_key_count(const int32_t* __restrict__ idx, int64_t nnz, KeyPack kc,
                                                   YSlot* __restrict__ tab, TabGeom g, uint64_t seed,
                                                   int32_t max_probe, DevStatus* st,
                                                   unsigned long long* distinct) {
  unsigned long long fresh = 0;  // keys this thread inserted (one atomic per wave at the end)
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = pack_key(idx, nnz, e, kc);
    ProbeSeq p = probe_seq(key, g, seed);
    int32_t probe = 0;
    for (;;) {
      const uint64_t s = p.slot();
      // a slot's key changes once, from empty: a key seen here is final, and
      // only an empty slot needs the compare-and-swap
      const unsigned long long seen = __atomic_load_n(&tab[s].key, __ATOMIC_RELAXED);
      const unsigned long long prev =
          seen == kEmpty ? atomicCAS(&tab[s].key, (unsigned long long)kEmpty, (unsigned long long)key) : seen;
      if (prev == kEmpty || prev == key) {
        atomicAdd(&tab[s].count, 1u);
        fresh += prev == kEmpty;
        break;
      }
      if (++probe >= max_probe) {
        record_error(st, kErrCapacity);
        break;
      }
      p.next();
    }
  }
  if (distinct) {
    for (int off = 32; off > 0; off >>= 1) fresh += __shfl_xor(fresh, off);
    if ((threadIdx.x & 63) == 0 && fresh) atomicAdd(distinct, fresh);
  }
}

// A2 op: count -> inclusive end offset of the group, kept in `start`.
// run_end: start = end of the run (placement takes and decrements), else
// start = its beginning (placement from per-chunk offsets).
struct YTableScanOp {
  YSlot* tab;
  bool run_end;
  __device__ unsigned long long get(int64_t i) const { return tab[i].count; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long v) const {
    if (v) tab[i].start = (unsigned)(run_end ? excl + v : excl);
  }
};

// A3: scatter Y into its groups (counting-sort placement: take the end of
// the group's run and decrement).
__global__ __launch_bounds__(256) void k_y_scatter(const int32_t* __restrict__ yidx, const double* __restrict__ yval,
                                                   int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                                                   YSlot* __restrict__ tab, TabGeom g, uint64_t seed,
                                                   int32_t max_probe, YEntry* __restrict__ yg,
                                                   unsigned long long* __restrict__ yset, uint64_t yset_mask,
                                                   int32_t bits_y, DevStatus* st) {
  bool bad = false;  // a value is Inf or NaN
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    if (b.check && !coords_ok(yidx, nnz, e, b)) record_error(st, kErrCoord);
    const uint64_t key = pack_key(yidx, nnz, e, kc);
    const int64_t s = find_slot(tab, key, g, seed, max_probe);
    if (s < 0) {
      record_error(st, kErrInternal);
      continue;
    }
    const unsigned pos = atomicSub(&tab[s].start, 1u) - 1u;
    if ((int64_t)pos >= nnz) {
      record_error(st, kErrInternal);
      continue;
    }
    YEntry ent;
    ent.phi = pack_key(yidx, nnz, e, kf);
    ent.v = yval[e];
    bad |= !isfinite(ent.v);
    yg[pos] = ent;
    if (yset) {  // a repeated full coordinate marks Y as having duplicates
      const unsigned long long full = full_y_key(key, ent.phi, bits_y);
      uint64_t h = fmix64(full ^ seed) & yset_mask;
      for (uint64_t probe = 0; probe <= yset_mask; ++probe) {
        const unsigned long long prev = atomicCAS(&yset[h], (unsigned long long)kEmpty, full);
        if (prev == kEmpty) break;
        if (prev == full) {
          st->ydup = 1u;
          break;
        }
        h = (h + 1) & yset_mask;
      }
    }
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}

__global__ void k_fill_keys(unsigned long long* __restrict__ keys, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = kEmpty;
}

// B1: each X entry finds its Y group: start and count (0 on a miss).
__global__ __launch_bounds__(256) void k_x_probe(const int32_t* __restrict__ xidx, const double* __restrict__ xval,
                                                 int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                                                 const YSlot* __restrict__ tab, TabGeom g, uint64_t seed,
                                                 int32_t max_probe, XEntry* __restrict__ xrec,
                                                 uint32_t* __restrict__ xg, uint32_t* __restrict__ xcnt,
                                                 DevStatus* st) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    if (b.check && !coords_ok(xidx, nnz, e, b)) record_error(st, kErrCoord);
    const uint64_t key = pack_key(xidx, nnz, e, kc);
    ProbeSeq p = probe_seq(key, g, seed);
    unsigned start = 0, count = 0;
    for (int32_t probe = 0; probe < max_probe; ++probe) {
      const YSlot slot = tab[p.slot()];
      if (slot.key == key) {
        start = slot.start;
        count = slot.count;
        break;
      }
      if (slot.key == kEmpty) break;
      p.next();
    }
    XEntry ent;
    ent.phi = pack_key(xidx, nnz, e, kf);
    ent.v = xval[e];
    xrec[e] = ent;
    xg[e] = start;
    xcnt[e] = count;
  }
}

// live_n (when given): the number of entries in use, counted on the device.
struct ProductScanOp {
  const uint32_t* xcnt;
  unsigned long long* poff;
  const unsigned long long* live_n;
  __device__ int64_t live(int64_t n) const { return live_n ? (int64_t)*live_n : n; }
  __device__ unsigned long long get(int64_t i) const { return xcnt[i]; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { poff[i] = excl; }
};

struct FinProducts {
  unsigned long long* poff;
  int64_t n;
  const unsigned long long* live_n;
  unsigned long long* total_out;
  __device__ void operator()(unsigned long long total) const {
    const int64_t m = live_n && (int64_t)*live_n < n ? (int64_t)*live_n : n;
    poff[m] = total;
    *total_out = total;
  }
};

// B2 + C1: expand products and accumulate them in the output hash.
//
// The product space [0, P) is cut into tiles of BLOCK*ITEMS products; a tile
// stages the slice of poff it overlaps in LDS and each lane finds its X entry
// by binary search there (load-balanced search), so work per lane does not
// depend on group sizes.  Lanes take consecutive products, hence consecutive
// entries of one Y group: the Yg loads coalesce.
constexpr int kExpBlock = 256;
constexpr int kExpItems = 8;
constexpr int kExpTile = kExpBlock * kExpItems;

__device__ __forceinline__ void hash_accumulate(ZSlot* __restrict__ tab, uint64_t mask, uint64_t seed,
                                                int32_t max_probe, uint64_t key, double v, DevStatus* st) {
  uint64_t s = fmix64(key ^ seed) & mask;
  int32_t probe = 0;
  for (;;) {
    // a slot's key changes once, from empty: a key read here is final, and
    // only an empty slot needs the compare-and-swap (most products meet
    // their output's key already in place)
    const unsigned long long seen = __atomic_load_n(&tab[s].key, __ATOMIC_RELAXED);
    const unsigned long long prev =
        seen == kEmpty ? atomicCAS(&tab[s].key, (unsigned long long)kEmpty, (unsigned long long)key) : seen;
    if (prev == kEmpty || prev == key) {
      unsafeAtomicAdd(&tab[s].val, v);
      return;
    }
    if (++probe >= max_probe) {
      record_error(st, kErrCapacity);
      return;
    }
    s = (s + 1) & mask;
  }
}

__global__ __launch_bounds__(kExpBlock) void k_expand_acc(const unsigned long long* __restrict__ poff, int64_t nx,
                                                          const XEntry* __restrict__ xrec,
                                                          const uint32_t* __restrict__ xg,
                                                          const YEntry* __restrict__ yg, int64_t ny, int32_t bits_y,
                                                          ZSlot* __restrict__ tab, uint64_t mask, uint64_t seed,
                                                          int32_t max_probe, uint64_t products, DevStatus* st,
                                                          const unsigned long long* dnx,
                                                          const unsigned long long* dprod) {
  __shared__ unsigned long long s_poff[kExpTile + 1];
  __shared__ int64_t s_range[2];
  if (dnx && (int64_t)*dnx < nx) nx = (int64_t)*dnx;  // counts read on the device (bounded by the host's)
  if (dprod) products = *dprod;
  const uint64_t ntiles = (products + kExpTile - 1) / kExpTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t p0 = t * kExpTile;
    const uint64_t p1 = (p0 + kExpTile < products) ? p0 + kExpTile : products;
    if (threadIdx.x == 0) s_range[0] = upper_bound_idx(poff, 0, nx + 1, p0) - 1;
    if (threadIdx.x == 64) s_range[1] = upper_bound_idx(poff, 0, nx + 1, p1 - 1) - 1;
    __syncthreads();
    const int64_t xlo = s_range[0], xhi = s_range[1];
    const int64_t nloc = xhi - xlo + 1;  // X entries overlapping the tile
    const bool staged = nloc <= kExpTile;
    if (staged)
      for (int64_t k = threadIdx.x; k <= nloc; k += kExpBlock) s_poff[k] = poff[xlo + k];
    __syncthreads();
#pragma unroll 2
    for (int it = 0; it < kExpItems; ++it) {
      const uint64_t p = p0 + (uint64_t)it * kExpBlock + threadIdx.x;
      if (p >= p1) break;
      int64_t x;
      unsigned long long px;
      if (staged) {
        int lo = 0, hi = (int)nloc - 1;  // largest k with s_poff[k] <= p
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_poff[mid] <= p)
            lo = mid;
          else
            hi = mid - 1;
        }
        x = xlo + lo;
        px = s_poff[lo];
      } else {
        x = upper_bound_idx(poff, xlo, xhi + 1, p) - 1;
        px = poff[x];
      }
      const XEntry xe = xrec[x];
      const uint64_t y = (uint64_t)xg[x] + (p - px);
      if (y >= (uint64_t)ny) {
        record_error(st, kErrInternal);
        continue;
      }
      const YEntry ye = yg[y];
      const uint64_t key = (xe.phi << bits_y) | ye.phi;
      const double v = __dmul_rn(xe.v, ye.v);
      hash_accumulate(tab, mask, seed, max_probe, key, v, st);
    }
    __syncthreads();
  }
}

// C2: compaction of the output hash.
struct OccupancyOp {
  const ZSlot* tab;
  KeyUnpack ku;
  int32_t* out_idx;
  double* out_val;
  int64_t out_cap;
  const unsigned long long* base;
  __device__ unsigned long long get(int64_t i) const { return tab[i].key != kEmpty ? 1ull : 0ull; }
  __device__ void put(int64_t i, unsigned long long rank, unsigned long long v) const {
    if (!v) return;
    const unsigned long long pos = rank + (base ? *base : 0ull);
    if ((int64_t)pos >= out_cap) return;
    const ZSlot z = tab[i];
#pragma unroll
    for (int m = 0; m < kMaxOutOrder; ++m)
      if (m < ku.n)
        __builtin_nontemporal_store(key_field(z.key, ku.field[m]),
                                    &out_idx[(int64_t)m * out_cap + (int64_t)pos]);
    __builtin_nontemporal_store(z.val, &out_val[pos]);
  }
};

struct FinCompact {
  int64_t* out_nnz;
  int64_t out_cap;
  const unsigned long long* base;
  DevStatus* st;
  __device__ void operator()(unsigned long long count) const {
    const unsigned long long total = count + (base ? *base : 0ull);
    uint32_t err = st->err;
    if ((int64_t)total > out_cap) {
      err |= kErrCapacity;
      atomicOr(&st->err, kErrCapacity);
    }
    *out_nnz = err ? -(int64_t)status_of(err) : (int64_t)total;
  }
};

// Grouped path, global class: table keys are (group id << bits_y) | Y free
// key, so the X free coordinates come from the group's record.  (The group id
// is the dense small id of the X free key; it keeps keys within 63 bits when
// the packed X free key and Y free key together would not fit.)
struct GroupedOccupancyOp {
  const ZSlot* tab;
  const GroupRec* groups;
  const uint32_t* glist;  // table key >> bits_y indexes this list of group ids
  KeyUnpack ux, uy;
  int32_t bits_y;
  int32_t* out_idx;
  double* out_val;
  int64_t out_cap;
  const unsigned long long* base;
  const BatchOut* bout;  // batch: outputs go to the contraction's region, in place order
  BatchSeg* bseg;
  int32_t bwx;
  DevStatus* st;
  __device__ unsigned long long get(int64_t i) const { return tab[i].key != kEmpty ? 1ull : 0ull; }
  __device__ void put(int64_t i, unsigned long long rank, unsigned long long v) const {
    if (!v) return;
    const ZSlot z = tab[i];
    const unsigned long long phix = groups[glist[z.key >> bits_y]].phi;
    const unsigned long long phiy = bits_y ? (z.key & (~0ull >> (64 - bits_y))) : 0ull;
    if (bout) {
      const uint32_t b = (uint32_t)(phix >> bwx);
      const unsigned long long place = wave_reserve(bseg, b);
      batch_store(bout, out_idx, out_val, bwx, b, place, phix, phiy, z.val, st);
      return;
    }
    const unsigned long long pos = rank + *base;
    if ((int64_t)pos >= out_cap) return;
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < ux.n)
        __builtin_nontemporal_store(key_field(phix, ux.field[m]),
                                    &out_idx[(int64_t)(ux.row0 + m) * out_cap + (int64_t)pos]);
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < uy.n)
        __builtin_nontemporal_store(key_field(phiy, uy.field[m]),
                                    &out_idx[(int64_t)(uy.row0 + m) * out_cap + (int64_t)pos]);
    __builtin_nontemporal_store(z.val, &out_val[pos]);
  }
};

// Inspection: occupied Y table slots -> (key coordinates, count, start).
struct YGroupsOp {
  const YSlot* tab;
  KeyUnpack ku;
  int32_t* key_coords;
  int64_t* counts;
  int64_t* starts;
  int64_t cap;
  __device__ unsigned long long get(int64_t i) const { return tab[i].key != kEmpty ? 1ull : 0ull; }
  __device__ void put(int64_t i, unsigned long long pos, unsigned long long v) const {
    if (!v || (int64_t)pos >= cap) return;
    const YSlot y = tab[i];
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < ku.n) key_coords[(int64_t)m * cap + (int64_t)pos] = key_field(y.key, ku.field[m]);
    counts[pos] = y.count;
    starts[pos] = y.start;
  }
};

struct FinCount {
  int64_t* out;
  __device__ void operator()(unsigned long long total) const { *out = (int64_t)total; }
};

__global__ void k_y_grouped(const YEntry* __restrict__ yg, int64_t nnz, KeyUnpack ku, int32_t* __restrict__ coords,
                            double* __restrict__ vals) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const YEntry y = yg[e];
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < ku.n) coords[(int64_t)m * nnz + e] = key_field(y.phi, ku.field[m]);
    vals[e] = y.v;
  }
}

__global__ void k_x_counts(const unsigned long long* __restrict__ poff, int64_t nx, int64_t* __restrict__ counts) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nx; e += (int64_t)gridDim.x * blockDim.x)
    counts[e] = (int64_t)(poff[e + 1] - poff[e]);
}


// ---------------------------------------------------------------------------
// Direct-addressed small-key tables, aggregated per workgroup in LDS
// ---------------------------------------------------------------------------

// Small key spaces, count: each workgroup histograms its chunk in LDS and
// writes the histogram as row `chunk` of hist (no global atomics).
__global__ __launch_bounds__(kAggBlock) void k_key_count_agg(const int32_t* __restrict__ idx, int64_t nnz, KeyPack kc,
                                                             unsigned nslots, unsigned* __restrict__ hist) {
  extern __shared__ unsigned s_cnt[];
  for (unsigned s = threadIdx.x; s < nslots; s += kAggBlock) s_cnt[s] = 0u;
  __syncthreads();
  const Bounds none{};
  for_chunk_batches(idx, nnz, kc, false, none, [&](const int64_t*, const uint64_t* keys, const bool* ok, const bool*) {
#pragma unroll
    for (int u = 0; u < kAggUnroll; ++u)
      if (ok[u]) atomicAdd(&s_cnt[(unsigned)keys[u]], 1u);
  });
  __syncthreads();
  unsigned* row = hist + (size_t)blockIdx.x * nslots;
  for (unsigned s = threadIdx.x; s < nslots; s += kAggBlock) row[s] = s_cnt[s];
}

// The chunk histograms, taken key-major (key s, then chunk w), become the
// first position of key s's entries of chunk w: the start of s's run plus
// the entries of s in earlier chunks.  Two coalesced passes instead of one
// scan in key-major order (whose reads stride across the rows):
//
// k_agg_colscan: one workgroup per kColSlots consecutive keys (a 128-byte
// segment of every row); its kColRows thread rows split the chunks, sum
// their share, scan those sums down each key's column in LDS and rewrite
// their chunks with the column's exclusive prefix.  Key s's total lands in
// row nchunks.
constexpr int kColSlots = 32;
constexpr int kColRows = kAggBlock / kColSlots;

__global__ __launch_bounds__(kAggBlock) void k_agg_colscan(unsigned* __restrict__ hist, unsigned nchunks,
                                                           unsigned nslots) {
  __shared__ unsigned s_part[kColRows][kColSlots + 1];
  const unsigned col = threadIdx.x % kColSlots, r = threadIdx.x / kColSlots;
  const unsigned s = blockIdx.x * kColSlots + col;
  const unsigned per = (nchunks + kColRows - 1) / kColRows;
  const unsigned c0 = r * per < nchunks ? r * per : nchunks;
  const unsigned c1 = c0 + per < nchunks ? c0 + per : nchunks;
  unsigned sum = 0;
  if (s < nslots) {
#pragma unroll 4
    for (unsigned c = c0; c < c1; ++c) sum += hist[(size_t)c * nslots + s];
  }
  s_part[r][col] = sum;
  __syncthreads();
  if (r == 0) {
    unsigned run = 0;
    for (int k = 0; k < kColRows; ++k) {
      const unsigned t = s_part[k][col];
      s_part[k][col] = run;
      run += t;
    }
    if (s < nslots) hist[(size_t)nchunks * nslots + s] = run;
  }
  __syncthreads();
  if (s < nslots) {
    unsigned run = s_part[r][col];
    for (unsigned c = c0; c < c1; ++c) {
      unsigned* cell = hist + (size_t)c * nslots + s;
      const unsigned v = *cell;
      *cell = run;
      run += v;
    }
  }
}

// k_agg_slotscan (one workgroup): an exclusive scan of the key totals in
// row nchunks turns them into run starts in place; every occurring key gets
// its table entry (count and run start), every other slot is set empty, and
// *total gets the entry count.
constexpr unsigned kSlotsPerThread = 8;
static_assert((1u << kAggBits) <= kAggBlock * kSlotsPerThread, "one workgroup scans every key");

__global__ __launch_bounds__(kAggBlock) void k_agg_slotscan(unsigned* __restrict__ hist, unsigned nchunks,
                                                            unsigned nslots, unsigned long long* __restrict__ total,
                                                            YSlot* __restrict__ tab,
                                                            unsigned long long* __restrict__ distinct) {
  __shared__ unsigned long long s_wave[kAggBlock / 64 + 1];
  unsigned* row = hist + (size_t)nchunks * nslots;
  const unsigned s0 = threadIdx.x * kSlotsPerThread;
  unsigned cnt[kSlotsPerThread];
  unsigned mine = 0, used = 0;
#pragma unroll
  for (unsigned k = 0; k < kSlotsPerThread; ++k) {
    cnt[k] = s0 + k < nslots ? row[s0 + k] : 0u;
    mine += cnt[k];
    used += cnt[k] != 0u;
  }
  unsigned long long all;
  unsigned long long run = block_excl_scan<kAggBlock>(mine, s_wave, &all);
#pragma unroll
  for (unsigned k = 0; k < kSlotsPerThread; ++k) {
    if (s0 + k >= nslots) break;
    row[s0 + k] = (unsigned)run;
    YSlot t;  // every slot is written: the table needs no fill beforehand
    t.key = cnt[k] ? (unsigned long long)(s0 + k) : kEmpty;
    t.count = cnt[k];
    t.start = cnt[k] ? (unsigned)run : 0u;
    tab[s0 + k] = t;
    run += cnt[k];
  }
  const unsigned long long nused = block_sum_t<kAggBlock>((unsigned long long)used, s_wave);
  if (threadIdx.x == 0) {
    *total = all;
    if (distinct) atomicAdd(distinct, nused);
  }
}

__global__ __launch_bounds__(kAggBlock) void k_y_scatter_agg(const int32_t* __restrict__ yidx,
                                                             const double* __restrict__ yval, int64_t nnz, KeyPack kc,
                                                             KeyPack kf, Bounds b, const YSlot* __restrict__ tab,
                                                             unsigned nslots, const unsigned* __restrict__ choff,
                                                             YEntry* __restrict__ yg,
                                                             unsigned long long* __restrict__ yset,
                                                             uint64_t yset_mask, uint64_t seed, int32_t bits_y,
                                                             DevStatus* st) {
  bool bad = false;  // a value is Inf or NaN
  extern __shared__ unsigned s_agg[];
  const bool check = b.check != 0;
  place_chunk(yidx, nnz, kc, check, b, nslots, choff, s_agg, s_agg + nslots,
              [&](const int64_t* e, const uint64_t* keys, const unsigned* pos, const bool* ok, const bool* inbc) {
                bool good[kAggUnroll], inb[kAggUnroll];
                unsigned long long full[kAggUnroll];
                uint64_t fk[kAggUnroll];
                double v[kAggUnroll];
                // every load of the batch in flight before any store; the
                // two packs read every mode once, and check it on the way
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) inb[u] = inbc[u];
                pack_keys<kAggUnroll>(yidx, nnz, e, ok, kf, fk, check, b, inb);
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) {
                  v[u] = ok[u] ? yval[e[u]] : 0.0;
                  bad |= !isfinite(v[u]);
                }
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) {
                  good[u] = ok[u];
                  full[u] = 0ull;
                  if (!ok[u]) continue;
                  if (check && !inb[u]) record_error(st, kErrCoord);
                  if ((int64_t)pos[u] >= nnz) {
                    record_error(st, kErrInternal);
                    good[u] = false;
                    continue;
                  }
                  YEntry ent;
                  ent.phi = fk[u];
                  ent.v = v[u];
                  yg[pos[u]] = ent;
                  full[u] = full_y_key(keys[u], fk[u], bits_y);
                }
                if (yset) {
                  bool seen[kAggUnroll];
                  set_insert_batch(yset, yset_mask, seed, full, good, seen);
#pragma unroll
                  for (int u = 0; u < kAggUnroll; ++u)
                    if (seen[u]) st->ydup = 1u;
                }
              });
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}
}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_fill_empty(void* slots16, int64_t nslots, DevStatus* st, hipStream_t stream) {
  int64_t g = (nslots + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  k_fill_empty<<<dim3((unsigned)g), dim3(256), 0, stream>>>(static_cast<uint4*>(slots16), nslots, st);
  return hipGetLastError();
}

hipError_t launch_key_count(const int32_t* idx, int64_t nnz, KeyPack kc, YSlot* tab, TabGeom g, uint64_t seed,
                            int32_t max_probe, DevStatus* st, unsigned long long* distinct, int num_cus,
                            hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  k_key_count<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(idx, nnz, kc, tab, g, seed, max_probe, st,
                                                                distinct);
  return hipGetLastError();
}

hipError_t launch_scan_y_table(YSlot* tab, int64_t nslots, bool run_end, unsigned long long* tile_sums,
                               hipStream_t stream) {
  return device_scan(YTableScanOp{tab, run_end}, nslots, tile_sums, FinNone{}, stream);
}

hipError_t launch_y_scatter(const int32_t* yidx, const double* yval, int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                            YSlot* tab, TabGeom g, uint64_t seed, int32_t max_probe, YEntry* yg,
                            unsigned long long* yset, uint64_t yset_mask, int32_t bits_y, DevStatus* st, int num_cus,
                            hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  k_y_scatter<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(yidx, yval, nnz, kc, kf, b, tab, g, seed,
                                                                max_probe, yg, yset, yset_mask, bits_y, st);
  return hipGetLastError();
}

hipError_t launch_key_count_agg(const int32_t* idx, int64_t nnz, KeyPack kc, YSlot* tab, unsigned nslots,
                                unsigned* hist, unsigned long long* total, unsigned long long* distinct,
                                hipStream_t stream) {
  if (nslots > (1u << kAggBits)) return hipErrorInvalidValue;
  // no entries: no slot scan runs, so the table is set empty here
  if (nnz <= 0) return launch_fill_empty(tab, nslots, nullptr, stream);
  const unsigned chunks = (unsigned)agg_chunks(nnz);
  k_key_count_agg<<<chunks, kAggBlock, (size_t)nslots * 4, stream>>>(idx, nnz, kc, nslots, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_agg_colscan<<<(nslots + kColSlots - 1) / kColSlots, kAggBlock, 0, stream>>>(hist, chunks, nslots);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_agg_slotscan<<<1, kAggBlock, 0, stream>>>(hist, chunks, nslots, total, tab, distinct);
  return hipGetLastError();
}

hipError_t launch_y_scatter_agg(const int32_t* yidx, const double* yval, int64_t nnz, KeyPack kc, KeyPack kf,
                                Bounds b, const YSlot* tab, unsigned nslots, const unsigned* choff, YEntry* yg,
                                unsigned long long* yset,
                                uint64_t yset_mask, uint64_t seed, int32_t bits_y, DevStatus* st,
                                hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  const unsigned grid = (unsigned)agg_chunks(nnz);
  k_y_scatter_agg<<<grid, kAggBlock, (size_t)nslots * 8, stream>>>(yidx, yval, nnz, kc, kf, b, tab, nslots, choff, yg,
                                                                    yset, yset_mask, seed, bits_y, st);
  return hipGetLastError();
}

hipError_t launch_fill_keys(unsigned long long* keys, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  k_fill_keys<<<dim3((unsigned)g), 256, 0, stream>>>(keys, n);
  return hipGetLastError();
}

hipError_t launch_x_probe(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                          const YSlot* tab, TabGeom g, uint64_t seed, int32_t max_probe, XEntry* xrec,
                          uint32_t* xg, uint32_t* xcnt, DevStatus* st, int num_cus, hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  k_x_probe<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(xidx, xval, nnz, kc, kf, b, tab, g, seed, max_probe,
                                                              xrec, xg, xcnt, st);
  return hipGetLastError();
}

hipError_t launch_scan_products(const uint32_t* xcnt, int64_t n, unsigned long long* poff,
                                unsigned long long* tile_sums, unsigned long long* total, hipStream_t stream,
                                const unsigned long long* live_n) {
  return device_scan(ProductScanOp{xcnt, poff, live_n}, n, tile_sums, FinProducts{poff, n, live_n, total}, stream);
}

hipError_t launch_expand_acc(const unsigned long long* poff, int64_t nx, const XEntry* xrec, const uint32_t* xg,
                             const YEntry* yg, int64_t ny, int32_t bits_y, ZSlot* tab, uint64_t mask, uint64_t seed,
                             int32_t max_probe, uint64_t products, DevStatus* st, int num_cus,
                             hipStream_t stream, const unsigned long long* dnx, const unsigned long long* dprod) {
  if (!dprod && products == 0) return hipSuccess;
  // with device counts the grid is the persistent one; tiles past the
  // device's product count are skipped
  const uint64_t tiles = dprod ? ~0ull : (products + kExpTile - 1) / kExpTile;
  uint64_t g = (uint64_t)num_cus * 8;
  if (g > tiles) g = tiles;
  k_expand_acc<<<dim3((unsigned)g), dim3(kExpBlock), 0, stream>>>(poff, nx, xrec, xg, yg, ny, bits_y, tab, mask,
                                                                   seed, max_probe, products, st, dnx, dprod);
  return hipGetLastError();
}

hipError_t launch_compact(const ZSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* out_idx, double* out_val,
                          int64_t out_cap, int64_t* out_nnz, const unsigned long long* base,
                          unsigned long long* tile_sums, DevStatus* st, hipStream_t stream) {
  return device_scan(OccupancyOp{tab, ku, out_idx, out_val, out_cap, base}, nslots, tile_sums,
                     FinCompact{out_nnz, out_cap, base, st}, stream);
}

hipError_t launch_compact_grouped(const ZSlot* tab, int64_t nslots, const GroupRec* groups, const uint32_t* glist,
                                  KeyUnpack ux, KeyUnpack uy, int32_t bits_y, int32_t* out_idx, double* out_val,
                                  int64_t out_cap, int64_t* out_nnz, const unsigned long long* base,
                                  unsigned long long* tile_sums, DevStatus* st, const BatchOut* bout, BatchSeg* bseg,
                                  int32_t bwx, hipStream_t stream) {
  return device_scan(GroupedOccupancyOp{tab, groups, glist, ux, uy, bits_y, out_idx, out_val, out_cap, base, bout,
                                        bseg, bwx, st},
                     nslots, tile_sums, FinCompact{out_nnz, out_cap, base, st}, stream);
}

hipError_t launch_y_groups(const YSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* key_coords, int64_t* counts,
                           int64_t* starts, int64_t cap, int64_t* ngroups_dev, unsigned long long* tile_sums,
                           DevStatus* st, hipStream_t stream) {
  (void)st;
  return device_scan(YGroupsOp{tab, ku, key_coords, counts, starts, cap}, nslots, tile_sums, FinCount{ngroups_dev},
                     stream);
}

hipError_t launch_y_grouped(const YEntry* yg, int64_t nnz, KeyUnpack ku, int32_t* free_coords, double* vals,
                            hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  int64_t g = (nnz + 255) / 256;
  if (g > 65536) g = 65536;
  k_y_grouped<<<dim3((unsigned)g), 256, 0, stream>>>(yg, nnz, ku, free_coords, vals);
  return hipGetLastError();
}

hipError_t launch_x_counts(const unsigned long long* poff, int64_t nx, int64_t* counts, hipStream_t stream) {
  if (nx <= 0) return hipSuccess;
  int64_t g = (nx + 255) / 256;
  if (g > 65536) g = 65536;
  k_x_counts<<<dim3((unsigned)g), 256, 0, stream>>>(poff, nx, counts);
  return hipGetLastError();
}

}  // namespace sptc
