// X grouping by partition, for hashed X free keys of at most 31 bits (one
// contraction): the counting sort of section 4.1.1 in two levels, so that
// no step takes a device-scope atomic per entry (such atomics on a table
// in device memory go past the L2, a few per entry cost more than the
// entries' bytes).  Entries are first partitioned by the top bits of their
// key's hash into 2^bbits buckets of about 4,096 entries (per-tile LDS
// histograms, a scan of them bucket-major, a scatter with LDS cursors);
// then one workgroup per bucket groups its entries with an LDS table of
// keys and counts, numbers the bucket's groups in slot order from a base
// reserved with one atomic per bucket, and places each entry in its group's
// run.  Each entry's
// X record (its Y run and value) is formed in the scatter, while X streams
// in order.  The groups and records come out as the hashed X table's path
// makes them (groups in some order, each group's entries contiguous).
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"
#include "xpart.hpp"

namespace sptc {
namespace {

constexpr int kPBlock = 1024;  // partition workgroups: 16 entries of a tile per thread
constexpr int kPU = 4;
constexpr int kPGBlock = 1024;
constexpr unsigned kPSlots = 16384;  // LDS key table of a bucket: 128 KB

// Tiles of this workgroup: XCD x (workgroup b runs on XCD b mod 8) takes a
// contiguous eighth of the tiles, so that the scatter's writes of
// neighbouring tiles, which share the lines at each bucket's boundary
// between them, meet in one L2 and leave it as whole lines.
struct TileRange {
  int64_t first, end, step;
};

__device__ __forceinline__ TileRange xcd_tiles(int64_t ntiles) {
  constexpr unsigned kX = 8;
  if (gridDim.x % kX) return TileRange{(int64_t)blockIdx.x, ntiles, (int64_t)gridDim.x};
  const int64_t per = (ntiles + kX - 1) / kX, x = blockIdx.x % kX;
  const int64_t lo = x * per, hi = lo + per < ntiles ? lo + per : ntiles;
  return TileRange{lo + blockIdx.x / kX, hi, (int64_t)(gridDim.x / kX)};
}

__device__ __forceinline__ unsigned part_bucket(uint64_t key, uint64_t seed, int bbits) {
  return bbits ? (unsigned)(fmix64(key ^ seed) >> (64 - bbits)) : 0u;
}

__global__ __launch_bounds__(kPBlock) void k_xpart_hist(const int32_t* __restrict__ xidx, int64_t nnz, KeyPack kf,
                                                        uint64_t seed, int bbits, unsigned* __restrict__ hist,
                                                        int64_t ntiles) {
  extern __shared__ unsigned s_h[];
  const unsigned nbk = 1u << bbits;
  const TileRange tr = xcd_tiles(ntiles);
  for (int64_t t = tr.first; t < tr.end; t += tr.step) {
    for (unsigned b = threadIdx.x; b < nbk; b += kPBlock) s_h[b] = 0u;
    __syncthreads();
    const int64_t e0 = t * kPTile, e1 = e0 + kPTile < nnz ? e0 + kPTile : nnz;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kPBlock)
      atomicAdd(&s_h[part_bucket(pack_key(xidx, nnz, e, kf), seed, bbits)], 1u);
    __syncthreads();
    for (unsigned b = threadIdx.x; b < nbk; b += kPBlock) hist[(int64_t)b * ntiles + t] = s_h[b];
    __syncthreads();
  }
}

// Exclusive scan of the histogram in place, bucket-major: hist[b][t] becomes
// where tile t's entries of bucket b go.
struct PartScanOp {
  unsigned* hist;
  __device__ unsigned long long get(int64_t i) const { return hist[i]; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { hist[i] = (unsigned)excl; }
};

__global__ __launch_bounds__(kPBlock) void k_xpart_scatter(const int32_t* __restrict__ xidx,
                                                           const double* __restrict__ xval, int64_t nnz, KeyPack kf,
                                                           KeyPack kc, Bounds bnd, uint64_t seed, int bbits,
                                                           const unsigned* __restrict__ hist, int64_t ntiles,
                                                           const YSlot* __restrict__ ytab, TabGeom yg,
                                                           int32_t max_probe_y, unsigned* __restrict__ pkey,
                                                           XRec* __restrict__ prec, DevStatus* st) {
  extern __shared__ unsigned s_o[];
  const unsigned nbk = 1u << bbits;
  bool bad = false;  // a value is Inf or NaN
  const TileRange tr = xcd_tiles(ntiles);
  for (int64_t t = tr.first; t < tr.end; t += tr.step) {
    for (unsigned b = threadIdx.x; b < nbk; b += kPBlock) s_o[b] = hist[(int64_t)b * ntiles + t];
    __syncthreads();
    const int64_t e0 = t * kPTile, e1 = e0 + kPTile < nnz ? e0 + kPTile : nnz;
    // kPU entries per thread at a time, so that their loads and probes are
    // in flight together
    for (int64_t base = e0 + threadIdx.x; base < e1; base += (int64_t)kPBlock * kPU) {
      int64_t e[kPU];
      uint64_t key[kPU], ck[kPU];
      double v[kPU];
      unsigned pos[kPU];
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        e[u] = base + (int64_t)u * kPBlock;
        if (e[u] < e1) {
          key[u] = pack_key(xidx, nnz, e[u], kf);
          ck[u] = pack_key(xidx, nnz, e[u], kc);
          v[u] = xval[e[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        if (e[u] >= e1) continue;
        if (bnd.check && !coords_ok(xidx, nnz, e[u], bnd)) record_error(st, kErrCoord);
        bad |= !isfinite(v[u]);
        pos[u] = atomicAdd(&s_o[part_bucket(key[u], seed, bbits)], 1u);
      }
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        if (e[u] >= e1) continue;
        if ((int64_t)pos[u] >= nnz) {
          record_error(st, kErrInternal);
          continue;
        }
        XRec r;  // its Y run (count 0 when Y has no entry with its contracting key) and value
        r.ystart = 0;
        r.ycnt = 0;
        r.v = v[u];
        const int64_t ys = find_slot(ytab, ck[u], yg, seed, max_probe_y);
        if (ys >= 0) {
          r.ystart = ytab[ys].start;
          r.ycnt = ytab[ys].count;
        }
        pkey[pos[u]] = (unsigned)key[u];
        prec[pos[u]] = r;
      }
    }
    __syncthreads();
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}

// Bucket b's entries: [hist[b][0], hist[b + 1][0]) (the last: to nnz).
__device__ __forceinline__ void part_range(const unsigned* hist, unsigned b, unsigned nbk, int64_t ntiles,
                                           int64_t nnz, unsigned* lo, unsigned* hi) {
  *lo = hist[(int64_t)b * ntiles];
  *hi = b + 1 < nbk ? hist[(int64_t)(b + 1) * ntiles] : (unsigned)nnz;
}

// Slots of a bucket's LDS table: a power of two of at least twice its
// entries (so at most half full), from kPGBlock to tmax (the launch's table:
// twice the mean bucket, so that two workgroups share a CU; a bucket of
// many entries has few distinct keys, and only distinct keys take slots).
__device__ __forceinline__ unsigned part_slots(unsigned entries, unsigned tmax) {
  unsigned t = kPGBlock;
  while (t < 2u * entries && t < tmax) t <<= 1;
  return t;
}

// The bucket's keys into the LDS table of tsize slots (key << 32 | count);
// a key that finds no room is recorded as a capacity error.
__device__ __forceinline__ void part_table(unsigned long long* tab, unsigned tsize, const unsigned* __restrict__ pkey,
                                           unsigned lo, unsigned hi, uint64_t seed, DevStatus* st) {
  const unsigned tmask = tsize - 1u;
  for (unsigned s = threadIdx.x; s < tsize; s += kPGBlock) tab[s] = kEmpty;
  __syncthreads();
  for (unsigned i = lo + threadIdx.x; i < hi; i += kPGBlock) {
    const unsigned long long key = pkey[i];
    unsigned s = (unsigned)fmix64(key ^ seed) & tmask;
    bool done = false;
    for (unsigned probe = 0; probe < tsize && !done; ++probe, s = (s + 1u) & tmask) {
      const unsigned long long prev = atomicCAS(&tab[s], (unsigned long long)kEmpty, key << 32 | 1ull);
      if (prev == kEmpty) {
        done = true;
      } else if ((prev >> 32) == key) {
        atomicAdd(&tab[s], 1ull);
        done = true;
      }
    }
    if (!done) record_error(st, kErrCapacity);
  }
  __syncthreads();
}

// Each bucket's groups, numbered in slot order from a base that one atomic
// on the group count reserves (so buckets' groups come in no fixed order),
// and its entries placed in their groups' runs.
__global__ __launch_bounds__(kPGBlock) void k_xpart_place(const unsigned* __restrict__ pkey,
                                                          const XRec* __restrict__ prec,
                                                          const unsigned* __restrict__ hist, int bbits,
                                                          int64_t ntiles, int64_t nnz, uint64_t seed, unsigned tmax,
                                                          GroupRec* __restrict__ groups, XRec* __restrict__ xr,
                                                          DevStatus* st) {
  extern __shared__ unsigned long long s_tab[];
  __shared__ unsigned long long s_wave[kPGBlock / 64 + 1];
  const unsigned nbk = 1u << bbits;
  for (unsigned b = blockIdx.x; b < nbk; b += gridDim.x) {
    unsigned lo, hi;
    part_range(hist, b, nbk, ntiles, nnz, &lo, &hi);
    const unsigned tsize = part_slots(hi - lo, tmax), tmask = tsize - 1u;
    const unsigned kPer = tsize / kPGBlock;  // consecutive slots per thread
    part_table(s_tab, tsize, pkey, lo, hi, seed, st);
    // group ids and run starts in slot order: (entries << 32 | groups) scanned
    const unsigned s0 = threadIdx.x * kPer;
    unsigned long long mine = 0;
    for (unsigned k = 0; k < kPer; ++k) {
      const unsigned long long w = s_tab[s0 + k];
      if (w != kEmpty) mine += ((w & 0xffffffffull) << 32) | 1ull;
    }
    unsigned long long tot;
    unsigned long long run = block_excl_scan<kPGBlock>(mine, s_wave, &tot);
    // st->xgroups starts at zero (the plan clears the status) and ends as
    // the number of groups
    __shared__ unsigned long long s_gb;
    if (threadIdx.x == 0) s_gb = (tot & 0xffffffffull) ? atomicAdd(&st->xgroups, tot & 0xffffffffull) : 0ull;
    __syncthreads();
    const unsigned long long gb = s_gb;
    for (unsigned k = 0; k < kPer; ++k) {
      const unsigned long long w = s_tab[s0 + k];
      if (w == kEmpty) continue;
      const unsigned long long gi = gb + (run & 0xffffffffull);
      const unsigned long long start = (unsigned long long)lo + (run >> 32), count = w & 0xffffffffull;
      if ((int64_t)gi >= nnz || (int64_t)(start + count) > nnz) {
        record_error(st, kErrInternal);
      } else {
        GroupRec g;
        g.phi = w >> 32;
        g.start = (unsigned)start;
        g.count = (unsigned)count;
        groups[gi] = g;
      }
      s_tab[s0 + k] = (w & 0xffffffff00000000ull) | (run >> 32);  // the run's cursor, from its first place
      run += (count << 32) | 1ull;
    }
    __syncthreads();
    for (unsigned i = lo + threadIdx.x; i < hi; i += kPGBlock) {
      const unsigned long long key = pkey[i];
      unsigned s = (unsigned)fmix64(key ^ seed) & tmask;
      unsigned probe = 0;
      while (probe < tsize && (s_tab[s] >> 32) != key) {
        s = (s + 1u) & tmask;
        ++probe;
      }
      if (probe == tsize) {
        record_error(st, kErrInternal);
        continue;
      }
      const unsigned long long pos = (unsigned long long)lo + (atomicAdd(&s_tab[s], 1ull) & 0xffffffffull);
      if ((int64_t)pos >= nnz) {
        record_error(st, kErrInternal);
        continue;
      }
      xr[pos] = prec[i];
    }
    __syncthreads();
  }
}

}  // namespace

int part_bits(int64_t nnz) {
  int b = 0;
  while (b < kPartMaxBits && ((int64_t)kPTile / 4 << b) < nnz) ++b;  // about 4,096 entries per bucket
  return b;
}

int64_t part_tiles(int64_t nnz) { return (nnz + kPTile - 1) / kPTile; }

hipError_t prepare_x_partition() {
  {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xpart_place),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kPSlots * 8));
    if (e != hipSuccess) return e;
  }
  const void* hist[] = {reinterpret_cast<const void*>(&k_xpart_hist), reinterpret_cast<const void*>(&k_xpart_scatter)};
  for (const void* k : hist) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4u << kPartMaxBits));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_x_partition(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                              const YSlot* ytab, TabGeom yg, int32_t max_probe_y, uint64_t seed, const XPartBuffers& w,
                              GroupRec* groups, XRec* xr, DevStatus* st, int num_cus, hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  if (nnz > kPartMaxEntries) return hipErrorInvalidValue;
  const int bbits = part_bits(nnz);
  const int64_t ntiles = part_tiles(nnz);
  const unsigned nbk = 1u << bbits;
  unsigned grid = grid_for(ntiles, 1, num_cus, 4);
  if (grid >= 8) grid -= grid % 8;  // whole XCDs (xcd_tiles)
  k_xpart_hist<<<grid, kPBlock, nbk * 4, stream>>>(xidx, nnz, kf, seed, bbits, w.hist, ntiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_scan(PartScanOp{w.hist}, (int64_t)nbk * ntiles, w.scan, FinNone{}, stream);
  if (e != hipSuccess) return e;
  k_xpart_scatter<<<grid, kPBlock, nbk * 4, stream>>>(xidx, xval, nnz, kf, kc, b, seed, bbits, w.hist, ntiles, ytab,
                                                      yg, max_probe_y, w.pkey, w.prec, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned tmax = kPGBlock;
  while ((int64_t)tmax < 2 * ((nnz + nbk - 1) / nbk) && tmax < kPSlots) tmax <<= 1;
  const unsigned per_cu = tmax * 8 <= (64u << 10) ? 2u : 1u;  // 1,024-thread workgroups: two fill a CU
  const unsigned bgrid = nbk < per_cu * (unsigned)num_cus ? nbk : per_cu * (unsigned)num_cus;
  k_xpart_place<<<bgrid, kPGBlock, tmax * 8, stream>>>(w.pkey, w.prec, w.hist, bbits, ntiles, nnz, seed, tmax,
                                                       groups, xr, st);
  return hipGetLastError();
}

}  // namespace sptc
