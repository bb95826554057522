// Per-wave work items of the LDS accumulation classes (section 4.3: each X
// group accumulates its products in a table of its own, sized from the
// group's bound), shared by the kernels that run them.
//
//   wave class   one group per wave, a private LDS hash of at most
//                kWaveSlots slots; the outputs' positions come from a count
//                pass and a scan (a batch: one atomic per group on its
//                contraction's cursor);
//   dense block  one (group, slice) tile per wave: the group's row of the
//                dense Y free key space restricted to one of kSlices slices,
//                a dense LDS array; the wave counts the tile's outputs,
//                reserves them with one atomic on the output cursor and
//                writes them.
#pragma once

#include <hip/hip_runtime.h>

#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

// Power-of-two table size holding d keys at load <= 0.7; at least 64 slots.
__device__ __forceinline__ unsigned table_size_for(unsigned long long d, unsigned max_slots) {
  const unsigned long long need = (d * 10 + 6) / 7;
  unsigned t = 64;
  while (t < need && t < max_slots) t <<= 1;
  return t;
}

// Adds v at key in an LDS hash table (linear probing, 64-bit CAS).
__device__ __forceinline__ bool lds_accumulate(ZSlot* tab, unsigned tmask, unsigned long long key, double v,
                                               uint64_t seed) {
  unsigned s = (unsigned)fmix64(key ^ seed) & tmask;
  for (unsigned probe = 0; probe <= tmask; ++probe) {
    const unsigned long long prev = atomicCAS(&tab[s].key, (unsigned long long)kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(&tab[s].val, v);
      return true;
    }
    s = (s + 1) & tmask;
  }
  return false;
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// The output cursor a group's outputs are reserved on.
__device__ __forceinline__ unsigned long long* out_cursor(const GroupArgs& a, unsigned long long phi) {
  return a.bout ? &a.bseg[phi >> a.bwx].cursor : &a.st->out_base;
}

// Writes output `pos` of group phix (a batch: into its contraction's region).
__device__ __forceinline__ void put_output(const GroupArgs& a, unsigned long long pos, unsigned long long phix,
                                           unsigned long long phiy, double v) {
  if (a.bout)
    batch_store(a.bout, a.out_idx, a.out_val, a.bwx, (uint32_t)(phix >> a.bwx), pos, phix, phiy, v, a.st);
  else if ((int64_t)pos < a.out_cap)
    write_output(a, pos, phix, phiy, v);
}

// ---------------------------------------------------------------------------
// Wave class
// ---------------------------------------------------------------------------

struct WaveScratch {
  unsigned long long off[64];
  unsigned ys[64];
  double v[64];
};

constexpr size_t kWaveItemLds = (size_t)kWaveSlots * sizeof(ZSlot) + sizeof(WaveScratch);

// Inserts key in an LDS key set (linear probing); false when the table is full.
__device__ __forceinline__ bool lds_insert(unsigned long long* keys, unsigned tmask, unsigned long long key,
                                           uint64_t seed) {
  unsigned s = (unsigned)fmix64(key ^ seed) & tmask;
  for (unsigned probe = 0; probe <= tmask; ++probe) {
    const unsigned long long prev = atomicCAS(&keys[s], (unsigned long long)kEmpty, key);
    if (prev == kEmpty || prev == key) return true;
    s = (s + 1) & tmask;
  }
  return false;
}

// Table size of group G in the wave class (from its bound).
__device__ __forceinline__ unsigned wave_table_size(const GroupArgs& a, const GroupRec& G) {
  const unsigned long long b = a.eoff[G.start + G.count] - a.eoff[G.start];
  return table_size_for(b < a.ycells ? b : a.ycells, kWaveSlots);
}

// Group G's products spread over the wave's lanes, 64 X entries at a time
// (a search over the entries' product offsets in the scratch): with VALUES
// each product is added into the LDS hash tab (ZSlot), else only its Y free
// key is inserted into the LDS key set keys.  The table must be cleared.
template <bool VALUES>
__device__ __forceinline__ void wave_group_walk(const GroupArgs& a, const GroupRec& G, unsigned tmask, ZSlot* tab,
                                                unsigned long long* keys, WaveScratch& sc) {
  const unsigned lane = threadIdx.x & 63u;
  for (unsigned base = 0; base < G.count; base += 64) {
    const unsigned e = base + lane;
    unsigned long long c = 0;
    unsigned ys = 0;
    double v = 0.0;
    if (e < G.count) {
      const XRec r = a.xr[G.start + e];
      c = r.ycnt;
      ys = r.ystart;
      v = r.v;
    }
    const unsigned long long incl = wave_incl_scan(c);
    const unsigned long long tot = __shfl(incl, 63, 64);
    sc.off[lane] = incl - c;
    sc.ys[lane] = ys;
    if (VALUES) sc.v[lane] = v;
    wave_lds_fence();
    for (unsigned long long q = lane; q < tot; q += 64) {
      int lo = 0, hi = 63;  // the last entry whose run starts at or before q
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sc.off[mid] <= q)
          lo = mid;
        else
          hi = mid - 1;
      }
      const unsigned long long y = (unsigned long long)sc.ys[lo] + (q - sc.off[lo]);
      if (y >= (unsigned long long)a.ny) {
        record_error(a.st, kErrInternal);
        continue;
      }
      bool ok;
      if (VALUES) {
        const YEntry ye = a.yg[y];
        ok = lds_accumulate(tab, tmask, ye.phi, __dmul_rn(sc.v[lo], ye.v), a.seed);
      } else {
        ok = lds_insert(keys, tmask, a.yg[y].phi, a.seed);
      }
      if (!ok) record_error(a.st, kErrCapacity);
    }
    wave_lds_fence();
  }
}

// Distinct outputs of group g (the count pass): the group's Y free keys in
// the wave's LDS key set (kWaveSlots slots).  Wave-uniform result.
__device__ __forceinline__ unsigned wave_group_count(const GroupArgs& a, uint32_t g, unsigned long long* keys,
                                                     WaveScratch& sc) {
  const unsigned lane = threadIdx.x & 63u;
  const GroupRec G = a.groups[g];
  const unsigned tsize = wave_table_size(a, G);
  for (unsigned s = lane; s < tsize; s += 64) keys[s] = kEmpty;
  wave_lds_fence();
  wave_group_walk<false>(a, G, tsize - 1, nullptr, keys, sc);
  unsigned n = 0;
  for (unsigned s = lane; s < tsize; s += 64) n += keys[s] != kEmpty ? 1u : 0u;
  n = (unsigned)wave_sum((unsigned long long)n);
  wave_lds_fence();
  return n;
}

// Group g accumulated in the wave's LDS hash (tab, kWaveSlots slots) and its
// outputs written from position pos, in slot order; with RESERVE, pos is
// taken instead by one atomic on the group's output cursor.
template <bool RESERVE>
__device__ __forceinline__ void wave_group_fill(const GroupArgs& a, uint32_t g, unsigned long long pos, ZSlot* tab,
                                                WaveScratch& sc) {
  const unsigned lane = threadIdx.x & 63u;
  const GroupRec G = a.groups[g];
  const unsigned tsize = wave_table_size(a, G);
  for (unsigned s = lane; s < tsize; s += 64) {
    tab[s].key = kEmpty;
    tab[s].val = 0.0;
  }
  wave_lds_fence();
  wave_group_walk<true>(a, G, tsize - 1, tab, nullptr, sc);
  if (RESERVE) {
    unsigned n = 0;
    for (unsigned s = lane; s < tsize; s += 64) n += tab[s].key != kEmpty ? 1u : 0u;
    n = (unsigned)wave_sum((unsigned long long)n);
    if (!n) {
      wave_lds_fence();
      return;
    }
    if (lane == 0) pos = atomicAdd(out_cursor(a, G.phi), (unsigned long long)n);
    pos = __shfl(pos, 0);
  }
  for (unsigned s0 = 0; s0 < tsize; s0 += 64) {
    const ZSlot z = tab[s0 + lane];
    const bool occ = z.key != kEmpty;
    const unsigned long long m = __ballot(occ);
    if (occ) put_output(a, pos + lanes_below(m), G.phi, z.key, z.val);
    pos += (unsigned long long)__popcll(m);
  }
  wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Dense block class, sliced over the XCDs
// ---------------------------------------------------------------------------
//
// With a dense Y free key (at most kDenseBits bits) a group accumulates in a
// dense array indexed by the Y free key, which is exactly the group's output
// row.  The Y free keys that the mode lengths allow are cut into kSlices
// equal slices of wcells cells (a multiple of 64), and every Y run (the Y
// entries of one contracting key, section 4.2) is laid out slice by slice
// at plan time, with yso giving where each slice of each run begins.  A tile is (group, slice): one wave walks the group's X entries
// and, for each, the slice of its Y run, adding x * y into the slice's cells
// of the group's row in LDS.
//
// Slice s runs on XCD s (workgroup b sits on XCD b mod 8), so each XCD reads
// only the Y entries of its slice: one eighth of grouped Y, which stays in
// that XCD's L2 while every group walks it.  The X records are read once per
// slice, a small fraction of the products' Y reads.
//
// A cell is an output when some product reached it, whatever its value.  A
// product is added as x * y + 0.0, which turns -0.0 into +0.0 and leaves
// every other value as it is; cells start at -0.0, which any such addend
// changes for good (a sum that cancels is +0.0 under round to nearest), so a
// cell was reached exactly when it is no longer -0.0.

constexpr int kBufferWord3 = 0x00020000;  // buffer descriptor word 3 for gfx9-family (raw, untyped) loads

// An X record read past the L2 (streaming): every XCD reads all of the
// block class's X records once, and they must not evict the XCD's slice of
// grouped Y, which every group rereads.
__device__ __forceinline__ XRec load_xrec(const XRec* p) {
  const unsigned long long* w = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long w0 = __builtin_nontemporal_load(w), w1 = __builtin_nontemporal_load(w + 1);
  XRec r;
  r.ystart = (unsigned)w0;
  r.ycnt = (unsigned)(w0 >> 32);
  r.v = __longlong_as_double((long long)w1);
  return r;
}

__device__ __forceinline__ bool cell_reached(const double* acc, unsigned c) {
  return __double_as_longlong(acc[c]) != (long long)0x8000000000000000ull;
}

// Loads of the compact grouped Y (16-bit Y free keys, values): through
// buffer descriptors when both arrays fit 31-bit byte offsets (the
// per-load address is then a 32-bit offset, and constant steps fold into
// the instruction), else plain global loads.
template <bool BUF>
struct YReader {
  __amdgpu_buffer_rsrc_t rk, rv;
  const uint16_t* key;
  const double* val;
  __device__ YReader(const uint16_t* k, const double* v, int64_t n) : key(k), val(v) {
    if constexpr (BUF) {
      rk = __builtin_amdgcn_make_buffer_rsrc((void*)k, 0, (int)(n * 2), kBufferWord3);
      rv = __builtin_amdgcn_make_buffer_rsrc((void*)v, 0, (int)(n * 8), kBufferWord3);
    }
  }
  __device__ __forceinline__ unsigned cell(unsigned i) const {
    if constexpr (BUF)
      return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rk, (int)(i * 2u), 0, 0);
    else
      return key[i];
  }
  __device__ __forceinline__ double value(unsigned i) const {
    if constexpr (BUF)
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, (int)(i * 8u), 0, 0));
    else
      return val[i];
  }
};

// A tile's outputs: the reached cells of acc[wcells] (Y free keys c0 + c).
__device__ __forceinline__ unsigned tile_count(const double* acc, unsigned wcells) {
  const unsigned lane = threadIdx.x & 63u;
  unsigned cnt = 0;
  for (unsigned cw = 0; cw < wcells; cw += 64) cnt += (unsigned)__popcll(__ballot(cell_reached(acc, cw + lane)));
  return cnt;
}

// Writes them in cell order from position pos.
__device__ __forceinline__ void tile_write(const GroupArgs& a, const GroupRec& G, unsigned c0, const double* acc,
                                           unsigned wcells, unsigned long long pos) {
  const unsigned lane = threadIdx.x & 63u;
  for (unsigned cw = 0; cw < wcells; cw += 64) {
    const unsigned c = cw + lane;
    const bool occ = cell_reached(acc, c);
    const unsigned long long mask = __ballot(occ);
    if (occ) put_output(a, pos + lanes_below(mask), G.phi, c0 + c, acc[c]);
    pos += (unsigned long long)__popcll(mask);
  }
}

// Counts them, reserves them with one atomic on the output cursor and
// writes them.
__device__ __forceinline__ void tile_outputs(const GroupArgs& a, const GroupRec& G, unsigned c0, const double* acc,
                                             unsigned wcells) {
  const unsigned cnt = tile_count(acc, wcells);
  if (cnt) {
    unsigned long long pos = 0;
    if ((threadIdx.x & 63u) == 0) pos = atomicAdd(out_cursor(a, G.phi), (unsigned long long)cnt);
    tile_write(a, G, c0, acc, wcells, __shfl(pos, 0));
  }
}

// Tile (group G, slice) in the wave's dense accumulator: the group's X
// entries are staged up to 64 at a time, one per lane (each lane loading its
// entry's record and the bounds of the entry's slice of its Y run: two
// dependent loads, in parallel across the lanes), and the products of a
// stage are taken as one flat stream: each entry contributes its slice of
// its Y run, and lane q of window w takes product 64 w + q of the stream, so
// every lane has a product whatever the slices' lengths.
//
// A lane's entry is the number of entries whose last product comes before
// its own (entries with no product are dropped from the stage).  At stage
// time each entry sets the bit of its last product in its window's 64-bit
// mask; window w's mask sits in lane w, so a window reads it with two
// scalar lane reads, and a lane's entry is the running count of earlier
// windows' bits plus the mask's bits below the lane (one mbcnt pair).  A
// stage takes the longest prefix of its entries whose stream fits the 64
// windows (4096 products), or, when the first entry alone is longer, that
// entry on its own (all its products then belong to it).
//
// The tile is left accumulated in acc (its outputs are the reached cells).
// Per wave LDS: acc[wcells + 2], then the stage: (stream start, first Y
// entry) and x of each entry, and the window masks.  Cell wcells collects
// the products of a bad cell (a corrupt plan: reported), cell wcells + 1
// those of lanes past the stream's end; neither is an output.  K windows
// are loaded before any of their products is added, with no branch between
// the loads and the adds.
constexpr unsigned kFlatStageBytes = 64 * 8 + 64 * 8 + 64 * 8;

__host__ __device__ constexpr size_t flat_wave_lds(unsigned wcells) {
  return (size_t)(wcells + 2) * 8 + kFlatStageBytes;
}

template <int K, bool BUF>
__device__ __forceinline__ void flat_tile_accumulate(const GroupArgs& a, const GroupRec& G, unsigned slice, double* acc,
                                               unsigned wcells, const uint32_t* __restrict__ yso, int64_t yso_slots,
                                               const YReader<BUF>& yr) {
  uint2* sse = reinterpret_cast<uint2*>(acc + wcells + 2);  // (stream start, first Y entry) per entry
  double* sx = reinterpret_cast<double*>(sse + 64);
  unsigned long long* smask = reinterpret_cast<unsigned long long*>(sx + 64);
  const unsigned lane = threadIdx.x & 63u;
  const unsigned c0 = slice * wcells;  // first Y free key of the slice
  for (unsigned c = lane; c < wcells + 2; c += 64) acc[c] = -0.0;
  bool bad = false;
  for (unsigned e0 = 0, taken = 0; e0 < G.count; e0 += taken) {
    // stage: lane l's entry e0 + l: its slice (start, length) and value
    unsigned my_lo = 0u, my_n = 0u;
    double my_x = 0.0;
    if (e0 + lane < G.count) {
      const XRec r = load_xrec(a.xr + G.start + e0 + lane);
      if (r.ycnt && (int64_t)r.ystart < yso_slots) {  // r.ystart is the run's Y table slot here
        const uint32_t* b = yso + (size_t)r.ystart * (kSlices + 1) + slice;
        const unsigned l = b[0], h = b[1];
        if (h >= l && h - l <= r.ycnt && (int64_t)h <= a.ny) {
          my_lo = l;
          my_n = h - l;
          my_x = r.v;
        } else {
          bad = true;
        }
      } else if (r.ycnt) {
        bad = true;
      }
    }
    const unsigned long long incl64 = wave_incl_scan((unsigned long long)my_n);
    const unsigned nfit = (unsigned)__popcll(__ballot(incl64 <= 64ull * 64ull));  // a prefix of the lanes
    const bool single = nfit == 0;  // the first entry alone is longer than 64 windows
    taken = single ? 1u : nfit;
    const unsigned total = (unsigned)__builtin_amdgcn_readlane((unsigned)incl64, (int)taken - 1);
    if (lane >= taken) my_n = 0u;  // staged again next time
    const unsigned start = (unsigned)incl64 - my_n;
    const unsigned rank = lanes_below(__ballot(my_n != 0u));
    wave_lds_fence();  // the previous stage's readers are done
    if (my_n) {
      sse[rank] = make_uint2(start, my_lo);
      sx[rank] = my_x;
    }
    smask[lane] = 0ull;
    wave_lds_fence();
    if (my_n && !single) {
      const unsigned last = start + my_n - 1u;
      atomicOr(&smask[last >> 6], 1ull << (last & 63u));
    }
    wave_lds_fence();
    const unsigned long long vmask = smask[lane];  // window `lane`'s mask
    const unsigned nwin = (unsigned)(((unsigned long long)total + 63ull) >> 6);
    unsigned cnt = 0;  // uniform: entries whose last product lies in an earlier window
    for (unsigned w0 = 0; w0 < nwin; w0 += K) {
      unsigned idx[K], cell[K];
      double xv[K], yv[K];
      bool ok[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const unsigned w = w0 + k, p = w * 64u + lane;
        const int wl = (int)(w & 63u);  // (past the stage's windows: any lane; those lanes are past the end)
        // (readlane returns int: each half goes through unsigned, so the low
        // half is not sign-extended into the high one)
        const unsigned mlo = (unsigned)__builtin_amdgcn_readlane((unsigned)vmask, wl);
        const unsigned mhi = (unsigned)__builtin_amdgcn_readlane((unsigned)(vmask >> 32), wl);
        const unsigned long long m = ((unsigned long long)mhi << 32) | mlo;
        unsigned e = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, cnt));
        e = e < 63u ? e : 63u;
        cnt += (unsigned)__popcll(m);
        ok[k] = p < total;
        const uint2 se = sse[e];
        // past the end: Y entry 0 (a mask, not a select, so that the compiler
        // reads se for every lane instead of branching around the read)
        idx[k] = (se.y + (p - se.x)) & (ok[k] ? ~0u : 0u);
        xv[k] = sx[e];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        cell[k] = yr.cell(idx[k]);
        yv[k] = yr.value(idx[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const unsigned c = cell[k] - c0;
        const unsigned t = c < wcells ? c : wcells;
        atomicAdd(&acc[ok[k] ? t : wcells + 1u], __dmul_rn(xv[k], yv[k]) + 0.0);
      }
    }
  }
  wave_lds_fence();
  bad |= cell_reached(acc, wcells);
  if (__ballot(bad) && lane == 0) record_error(a.st, kErrInternal);
}

}  // namespace
}  // namespace sptc
