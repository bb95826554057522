// Device primitives shared by the kernel translation units: hashing, key
// packing, wave64/block scans and a device-wide exclusive scan.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "../../include/sptc.h"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

// MurmurHash3 64-bit finalizer (Appleby, public domain): a bijective mixer
// so that consecutive packed keys spread over the table.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// An entry's coordinates are read kModeGroup modes at a time, every load of
// a group issued before any is used (modes past n re-read mode n - 1, a
// cache hit): an order-n key costs ceil(n / kModeGroup) memory round trips,
// not n.  The loops over the modes stay rolled.
constexpr int kModeGroup = 4;

__device__ __forceinline__ uint64_t pack_key(const int32_t* __restrict__ idx, int64_t nnz, int64_t e,
                                             const KeyPack& kp) {
  uint64_t k = 0;
  const int n = kp.n;
  for (int t0 = 0; t0 < n; t0 += kModeGroup) {
    uint32_t c[kModeGroup];
#pragma unroll
    for (int j = 0; j < kModeGroup; ++j) {
      const int t = t0 + j < n ? t0 + j : n - 1;
      c[j] = (uint32_t)idx[(int64_t)field_mode(kp.field[t]) * nnz + e];
    }
#pragma unroll
    for (int j = 0; j < kModeGroup; ++j) {
      if (t0 + j >= n) continue;
      const uint32_t f = kp.field[t0 + j];
      k |= (uint64_t)(c[j] & field_mask(field_bits(f))) << field_shift(f);
    }
  }
  return k;
}

// The keys of U entries at once (entry u is e[u], read only where ok[u]):
// two modes of all U entries in flight together.  With check, also clears
// inb[u] when a coordinate it reads is outside its mode length (b.dim).
template <int U>
__device__ __forceinline__ void pack_keys(const int32_t* __restrict__ idx, int64_t nnz, const int64_t* e,
                                          const bool* ok, const KeyPack& kp, uint64_t* keys, bool check,
                                          const Bounds& b, bool* inb) {
#pragma unroll
  for (int u = 0; u < U; ++u) keys[u] = 0ull;
  const int n = kp.n;
  for (int t0 = 0; t0 < n; t0 += 2) {
    uint32_t c[2][U];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int t = t0 + j < n ? t0 + j : n - 1;
      const int32_t* col = idx + (int64_t)field_mode(kp.field[t]) * nnz;
#pragma unroll
      for (int u = 0; u < U; ++u) c[j][u] = ok[u] ? (uint32_t)col[e[u]] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (t0 + j >= n) continue;
      const uint32_t f = kp.field[t0 + j];
      const uint32_t m = field_mask(field_bits(f));
      const unsigned sh = field_shift(f);
#pragma unroll
      for (int u = 0; u < U; ++u) keys[u] |= (uint64_t)(c[j][u] & m) << sh;
      if (check) {
        const uint32_t d = b.dim[field_mode(f)];
#pragma unroll
        for (int u = 0; u < U; ++u) inb[u] = inb[u] && c[j][u] < d;
      }
    }
  }
}

// Checks every coordinate of entry e against its mode length.
__device__ __forceinline__ bool coords_ok(const int32_t* __restrict__ idx, int64_t nnz, int64_t e, const Bounds& b) {
  bool ok = true;
  const int n = b.order;
  for (int t0 = 0; t0 < n; t0 += kModeGroup) {
    uint32_t c[kModeGroup];
#pragma unroll
    for (int j = 0; j < kModeGroup; ++j) {
      const int t = t0 + j < n ? t0 + j : n - 1;
      c[j] = (uint32_t)idx[(int64_t)t * nnz + e];
    }
#pragma unroll
    for (int j = 0; j < kModeGroup; ++j)
      if (t0 + j < n) ok &= c[j] < b.dim[t0 + j];
  }
  return ok;
}

__device__ __forceinline__ void record_error(DevStatus* st, uint32_t bits) { atomicOr(&st->err, bits); }

__device__ __forceinline__ int status_of(uint32_t err) {
  if (err & kErrCoord) return SPTC_ERR_INVALID_ARG;
  if (err & kErrCapacity) return SPTC_ERR_CAPACITY;
  if (err) return SPTC_ERR_INTERNAL;
  return SPTC_OK;
}

// ---------------------------------------------------------------------------
// wave64 / block primitives, for u64 values and for pairs of u64 counters
// ---------------------------------------------------------------------------

struct U128 {
  unsigned long long lo, hi;
};
__device__ __forceinline__ U128 operator+(U128 a, U128 b) { return U128{a.lo + b.lo, a.hi + b.hi}; }
__device__ __forceinline__ U128 operator-(U128 a, U128 b) { return U128{a.lo - b.lo, a.hi - b.hi}; }
__device__ __forceinline__ unsigned long long shfl_up_v(unsigned long long v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ U128 shfl_up_v(U128 v, int d) {
  return U128{__shfl_up(v.lo, d, 64), __shfl_up(v.hi, d, 64)};
}
__device__ __forceinline__ unsigned long long shfl_xor_v(unsigned long long v, int d) { return __shfl_xor(v, d, 64); }
__device__ __forceinline__ U128 shfl_xor_v(U128 v, int d) {
  return U128{__shfl_xor(v.lo, d, 64), __shfl_xor(v.hi, d, 64)};
}

template <class V>
__device__ __forceinline__ V wave_incl_scan_t(V v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const V t = shfl_up_v(v, d);
    if (lane >= d) v = v + t;
  }
  return v;
}

template <class V>
__device__ __forceinline__ V wave_sum_t(V v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = v + shfl_xor_v(v, d);
  return v;
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) { return wave_incl_scan_t(v); }
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) { return wave_sum_t(v); }

// Exclusive scan over the block; *total receives the block sum.  s_wave
// holds BLOCK/64 + 1 entries.  Ends with a barrier so s_wave can be reused.
template <int BLOCK, class V>
__device__ __forceinline__ V block_excl_scan_t(V v, V* s_wave, V* total) {
  constexpr int W = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const V incl = wave_incl_scan_t(v);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    V run{};
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const V t = s_wave[w];
      s_wave[w] = run;
      run = run + t;
    }
    s_wave[W] = run;
  }
  __syncthreads();
  const V excl = s_wave[wave] + incl - v;
  *total = s_wave[W];
  __syncthreads();
  return excl;
}

template <int BLOCK>
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v, unsigned long long* s_wave,
                                                             unsigned long long* total) {
  return block_excl_scan_t<BLOCK>(v, s_wave, total);
}

template <int BLOCK, class V>
__device__ __forceinline__ V block_sum_t(V v, V* s_wave) {
  constexpr int W = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_t(v);
  if (lane == 0) s_wave[wave] = v;
  __syncthreads();
  V t{};
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w) t = t + s_wave[w];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

template <int BLOCK>
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long* s_wave) {
  return block_sum_t<BLOCK>(v, s_wave);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan: reduce tiles, scan tile sums, rescan tiles.
// An Op supplies get(i) -> V (u64 or U128) and put(i, exclusive_prefix,
// value).  The tile-sum buffer holds scan_tiles(n) + 1 values of V.
// ---------------------------------------------------------------------------

// An Op may also supply live(n): how many leading elements of the n are in
// use, read on the device (a count an earlier kernel wrote); tiles past it
// skip their work.
template <class Op, class = void>
struct HasLive : std::false_type {};
template <class Op>
struct HasLive<Op, std::void_t<decltype(std::declval<const Op&>().live(int64_t{}))>> : std::true_type {};

template <class Op>
__device__ __forceinline__ int64_t live_count(const Op& op, int64_t n) {
  if constexpr (HasLive<Op>::value) {
    const int64_t m = op.live(n);
    return m < n ? m : n;
  } else {
    return n;
  }
}

template <class Op, class V>
__global__ __launch_bounds__(kScanBlock) void k_tile_reduce(Op op, int64_t n, V* tile_sums) {
  __shared__ V s_wave[kScanBlock / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  n = live_count(op, n);
  if (base >= n) {  // uniform across the block
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = V{};
    return;
  }
  V s{};
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s = s + op.get(i);
  }
  s = block_sum_t<kScanBlock>(s, s_wave);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = s;
}

constexpr int kTopBlock = 1024;
constexpr int kTopItems = 8;

// Single block: exclusive scan of tile sums in place; fin(total) runs on
// thread 0 at the end.
template <class Fin, class V>
__global__ __launch_bounds__(kTopBlock) void k_scan_tile_sums(V* sums, int64_t ntiles, Fin fin) {
  __shared__ V s_wave[kTopBlock / 64 + 1];
  V carry{};
  for (int64_t base = 0; base < ntiles; base += (int64_t)kTopBlock * kTopItems) {
    V v[kTopItems];
    V local{};
    const int64_t first = base + (int64_t)threadIdx.x * kTopItems;
#pragma unroll
    for (int k = 0; k < kTopItems; ++k) {
      v[k] = (first + k < ntiles) ? sums[first + k] : V{};
      local = local + v[k];
    }
    V total;
    V run = carry + block_excl_scan_t<kTopBlock>(local, s_wave, &total);
#pragma unroll
    for (int k = 0; k < kTopItems; ++k) {
      if (first + k < ntiles) sums[first + k] = run;
      run = run + v[k];
    }
    carry = carry + total;
  }
  if (threadIdx.x == 0) fin(carry);
}

template <class Op, class V>
__global__ __launch_bounds__(kScanBlock) void k_tile_scan(Op op, int64_t n, const V* tile_offsets) {
  __shared__ V s_wave[kScanBlock / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  n = live_count(op, n);
  V carry = tile_offsets[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t chunk = base + (int64_t)k * kScanBlock;
    if (chunk >= n) break;  // uniform across the block
    const int64_t i = chunk + threadIdx.x;
    const V v = i < n ? op.get(i) : V{};
    V total;
    const V excl = block_excl_scan_t<kScanBlock>(v, s_wave, &total);
    if (i < n) op.put(i, carry + excl, v);
    carry = carry + total;
  }
}

// A scan of at most one tile: the whole of it in one 1024-thread
// workgroup, fin(total) on thread 0 at the end (one launch instead of
// three).
constexpr int kSingleBlock = 1024;

template <class Op, class Fin, class V>
__global__ __launch_bounds__(kSingleBlock) void k_scan_single(Op op, int64_t n, Fin fin) {
  __shared__ V s_wave[kSingleBlock / 64 + 1];
  n = live_count(op, n);
  V carry{};
  for (int64_t chunk = 0; chunk < n; chunk += kSingleBlock) {  // uniform across the block
    const int64_t i = chunk + threadIdx.x;
    const V v = i < n ? op.get(i) : V{};
    V total;
    const V excl = block_excl_scan_t<kSingleBlock>(v, s_wave, &total);
    if (i < n) op.put(i, carry + excl, v);
    carry = carry + total;
  }
  if (threadIdx.x == 0) fin(carry);
}

struct FinNone {
  template <class V>
  __device__ void operator()(V) const {}
};

// tile_sums: device scratch of at least scan_tiles(n) + 1 values of the Op's
// value type (U128 needs twice the u64 count).
template <class Op, class Fin>
hipError_t device_scan(Op op, int64_t n, void* tile_sums, Fin fin, hipStream_t stream) {
  using V = decltype(op.get(0));
  V* ts = static_cast<V*>(tile_sums);
  const int64_t tiles = scan_tiles(n);
  if (tiles <= 1) {
    k_scan_single<Op, Fin, V><<<1, kSingleBlock, 0, stream>>>(op, n, fin);
    return hipGetLastError();
  }
  k_tile_reduce<Op, V><<<dim3((unsigned)tiles), dim3(kScanBlock), 0, stream>>>(op, n, ts);
  k_scan_tile_sums<Fin, V><<<1, kTopBlock, 0, stream>>>(ts, tiles, fin);
  k_tile_scan<Op, V><<<dim3((unsigned)tiles), dim3(kScanBlock), 0, stream>>>(op, n, ts);
  return hipGetLastError();
}

// Key of a whole Y coordinate for the repeated-coordinate check:
// (contracting key << bits_y) | free key when that fits 63 bits (bits_y >= 0);
// otherwise (bits_y < 0) a 64-bit mix of the two, where a collision can only
// report a repeat that is not there (which merely disables an optimisation).
__device__ __forceinline__ unsigned long long full_y_key(uint64_t ckey, uint64_t fkey, int32_t bits_y) {
  if (bits_y >= 0) return (ckey << bits_y) | fkey;
  unsigned long long h = fmix64(ckey * 0x9e3779b97f4a7c15ull ^ fmix64(fkey + 0x632be59bd9b4e019ull));
  return h == kEmpty ? h - 1 : h;
}

// Home slot of a key in a table keyed by kp's packing.
// Calls f(i) with i in a scalar register when every active lane of the wave
// holds the same i (the common case: lanes walk one contraction's entries),
// so that what f loads through i comes from scalar loads; else f(i) per lane.
template <class F>
__device__ __forceinline__ void with_uniform(uint32_t i, F&& f) {
  const uint32_t i0 = __builtin_amdgcn_readfirstlane(i);
  if (__ballot(i != i0) == 0ull)
    f(i0);
  else
    f(i);
}

// Linear probing inside a key's table or region: slot() = base + off.
struct ProbeSeq {
  uint64_t base, mask, off;
  __device__ __forceinline__ uint64_t slot() const { return base + off; }
  __device__ __forceinline__ void next() { off = (off + 1) & mask; }
};

__device__ __forceinline__ ProbeSeq probe_seq(uint64_t key, const TabGeom& g, uint64_t seed) {
  if (g.reg) {
    ProbeSeq p;
    with_uniform((uint32_t)(key >> g.pshift), [&](uint32_t b) {
      const Region r = g.reg[b];
      p = ProbeSeq{r.base, r.mask, (r.ident ? key : fmix64(key ^ seed)) & r.mask};
    });
    return p;
  }
  return ProbeSeq{0ull, g.mask, (g.ident ? key : fmix64(key ^ seed)) & g.mask};
}

// Finds `key` in a YSlot table; returns the slot or -1.
__device__ __forceinline__ int64_t find_slot(const YSlot* __restrict__ tab, uint64_t key, const TabGeom& g,
                                             uint64_t seed, int32_t max_probe) {
  ProbeSeq p = probe_seq(key, g, seed);
  for (int32_t probe = 0; probe < max_probe; ++probe) {
    const unsigned long long k = tab[p.slot()].key;
    if (k == key) return (int64_t)p.slot();
    if (k == kEmpty) return -1;
    p.next();
  }
  return -1;
}

// First index in [lo, hi) with a[i] > v (hi if none).
template <class T, class V>
__device__ __forceinline__ int64_t upper_bound_idx(const T* a, int64_t lo, int64_t hi, V v) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ unsigned wave_incl_scan_u32(unsigned v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Orders this wave's LDS accesses (an LDS table private to one wave).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Per-workgroup LDS aggregation over a chunk of entries (small key spaces)
// ---------------------------------------------------------------------------

constexpr int kAggBlock = 1024;
constexpr int kAggUnroll = 4;    // entries a thread handles at once (independent memory ops in flight)

// Walks this workgroup's chunk kAggUnroll entries per thread at a time: f
// receives the entry indices, their packed keys, which are in range and
// (with check) whether the coordinates packed so far are inside b.
template <class F>
__device__ __forceinline__ void for_chunk_batches(const int32_t* __restrict__ idx, int64_t nnz, const KeyPack& kp,
                                                  bool check, const Bounds& b, F f) {
  const int64_t c0 = (int64_t)blockIdx.x * kAggChunk;
  const int64_t c1 = c0 + kAggChunk < nnz ? c0 + kAggChunk : nnz;
  for (int64_t base = c0 + threadIdx.x; base < c1; base += (int64_t)kAggBlock * kAggUnroll) {
    int64_t e[kAggUnroll];
    uint64_t keys[kAggUnroll];
    bool ok[kAggUnroll], inb[kAggUnroll];
#pragma unroll
    for (int u = 0; u < kAggUnroll; ++u) {
      e[u] = base + (int64_t)u * kAggBlock;
      ok[u] = e[u] < c1;
      inb[u] = true;
    }
    pack_keys<kAggUnroll>(idx, nnz, e, ok, kp, keys, check, b, inb);
    f(e, keys, ok, inb);
  }
}

// Places this workgroup's chunk: key s's entries of this chunk start at
// choff[chunk][s] (the start of s's run plus s's entries in earlier chunks)
// and follow in chunk order; hands every batch of entries with their
// positions to place(e, key, pos, ok, inb) (inb: kc's coordinates inside b,
// with check).  No global atomics.
template <class F>
__device__ __forceinline__ void place_chunk(const int32_t* __restrict__ idx, int64_t nnz, const KeyPack& kc,
                                            bool check, const Bounds& b, unsigned nslots,
                                            const unsigned* __restrict__ choff, unsigned* s_cnt, unsigned* s_base,
                                            F place) {
  const unsigned* row = choff + (size_t)blockIdx.x * nslots;
  const unsigned* start = choff + (size_t)((nnz + kAggChunk - 1) / kAggChunk) * nslots;
  // nslots <= 2^kAggBits: all of a thread's loads in flight at once
  constexpr int kSlotIters = (1 << kAggBits) / kAggBlock;
  static_assert(kSlotIters * kAggBlock == (1 << kAggBits), "whole rounds of slots");
  unsigned sb[kSlotIters];
#pragma unroll
  for (int k = 0; k < kSlotIters; ++k) {
    const unsigned s = threadIdx.x + k * kAggBlock < nslots ? threadIdx.x + k * kAggBlock : nslots - 1;
    sb[k] = start[s] + row[s];  // unconditional (a clamped index), so no branch splits the loads
  }
#pragma unroll
  for (int k = 0; k < kSlotIters; ++k) {
    const unsigned s = threadIdx.x + k * kAggBlock;
    if (s < nslots) {
      s_cnt[s] = 0u;
      s_base[s] = sb[k];
    }
  }
  __syncthreads();
  for_chunk_batches(idx, nnz, kc, check, b, [&](const int64_t* e, const uint64_t* keys, const bool* ok,
                                                const bool* inb) {
    unsigned pos[kAggUnroll];
#pragma unroll
    for (int u = 0; u < kAggUnroll; ++u)
      pos[u] = ok[u] ? s_base[(unsigned)keys[u]] + atomicAdd(&s_cnt[(unsigned)keys[u]], 1u) : 0u;
    place(e, keys, pos, ok, inb);
  });
}

// Inserts kAggUnroll keys into a kEmpty-filled set of 8-byte slots (first
// probes issued together); returns, per key, whether it was already there.
__device__ __forceinline__ void set_insert_batch(unsigned long long* __restrict__ set, uint64_t mask, uint64_t seed,
                                                 const unsigned long long* keys, const bool* ok, bool* seen) {
  uint64_t h[kAggUnroll];
  unsigned long long prev[kAggUnroll];
#pragma unroll
  for (int u = 0; u < kAggUnroll; ++u) {
    h[u] = fmix64(keys[u] ^ seed) & mask;
    prev[u] = ok[u] ? atomicCAS(&set[h[u]], (unsigned long long)kEmpty, keys[u]) : (unsigned long long)kEmpty;
  }
#pragma unroll
  for (int u = 0; u < kAggUnroll; ++u) {
    seen[u] = ok[u] && prev[u] == keys[u];
    if (!ok[u] || prev[u] == kEmpty || prev[u] == keys[u]) continue;
    uint64_t s = h[u];
    for (uint64_t probe = 0; probe < mask; ++probe) {  // collision: continue probing
      s = (s + 1) & mask;
      const unsigned long long p = atomicCAS(&set[s], (unsigned long long)kEmpty, keys[u]);
      if (p == kEmpty) break;
      if (p == keys[u]) {
        seen[u] = true;
        break;
      }
    }
  }
}

// Output entry `pos`: X free coordinates from phix, Y free coordinates from
// phiy, value v.  Streaming stores: the COO is written once and never read
// here, so it should not displace Y and the tables from the caches.
__device__ __forceinline__ void write_output(const GroupArgs& a, unsigned long long pos, unsigned long long phix,
                                             unsigned long long phiy, double v) {
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m)
    if (m < a.ux.n)
      __builtin_nontemporal_store(key_field(phix, a.ux.field[m]),
                                  &a.out_idx[(int64_t)(a.ux.row0 + m) * a.out_cap + (int64_t)pos]);
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m)
    if (m < a.uy.n)
      __builtin_nontemporal_store(key_field(phiy, a.uy.field[m]),
                                  &a.out_idx[(int64_t)(a.uy.row0 + m) * a.out_cap + (int64_t)pos]);
  __builtin_nontemporal_store(v, &a.out_val[pos]);
}

__device__ __forceinline__ uint64_t low_mask(int bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull); }

// Output `pos` of contraction b of a batch, in b's COO region: X free
// coordinates from phix (b's index above bit bwx), Y free ones from phiy.
__device__ __forceinline__ void batch_store_at(const BatchOut* __restrict__ bout, int32_t* __restrict__ out_idx,
                                               double* __restrict__ out_val, int32_t bwx, uint32_t b,
                                               unsigned long long pos, uint64_t phix, uint64_t phiy, double v,
                                               DevStatus* st) {
  const BatchOut& d = bout[b];
  if ((int64_t)pos >= d.cap) {
    record_error(st, kErrCapacity);
    return;
  }
  const uint64_t fx = phix & low_mask(bwx);
  const int nx = d.ux.n, ny = d.uy.n;
  int32_t* row = out_idx + d.idx_off + (int64_t)pos;
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m)
    if (m < nx) __builtin_nontemporal_store(key_field(fx, d.ux.field[m]), row + (int64_t)(d.ux.row0 + m) * d.cap);
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m)
    if (m < ny)
      __builtin_nontemporal_store(key_field(phiy, d.uy.field[m]), row + (int64_t)(d.uy.row0 + m) * d.cap);
  __builtin_nontemporal_store(v, &out_val[d.val_off + (int64_t)pos]);
}

__device__ __forceinline__ void batch_store(const BatchOut* __restrict__ bout, int32_t* __restrict__ out_idx,
                                            double* __restrict__ out_val, int32_t bwx, uint32_t b,
                                            unsigned long long pos, uint64_t phix, uint64_t phiy, double v,
                                            DevStatus* st) {
  with_uniform(b, [&](uint32_t bu) { batch_store_at(bout, out_idx, out_val, bwx, bu, pos, phix, phiy, v, st); });
}

// Reserves one place per calling lane from seg[b].cursor: one atomic per
// distinct b among the wave's active lanes.
__device__ __forceinline__ unsigned long long wave_reserve(BatchSeg* seg, uint32_t b) {
  const unsigned lane = threadIdx.x & 63u;
  for (;;) {
    const uint32_t bl = __builtin_amdgcn_readfirstlane(b);
    const unsigned long long m = __ballot(b == bl);
    if (b == bl) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0ull;
      if ((int)lane == leader) base = atomicAdd(&seg[bl].cursor, (unsigned long long)__popcll(m));
      base = __shfl(base, leader, 64);
      return base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
    }
  }
}

inline unsigned grid_for(int64_t n, int block, int num_cus, int per_cu = 16) {
  int64_t g = (n + block - 1) / block;
  const int64_t cap = (int64_t)num_cus * per_cu;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace
}  // namespace sptc
