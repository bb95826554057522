// Per-wave work items of the LDS accumulation classes (section 4.3: each X
// group accumulates its products in a table of its own, sized from the
// group's bound), shared by the kernels that run them.
//
//   wave class   one group per wave, a private LDS hash of at most
//                kWaveSlots slots;
//   dense block  one (group, slice) tile per wave: the group's row of the
//                dense Y free key space restricted to one of kSlices slices,
//                a dense LDS array.
//
// Either way the wave counts the item's outputs, reserves them with one
// atomic on the output cursor (the contraction's own cursor in a batch) and
// writes them, so an item needs nothing from any other item.
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

// Group g in the wave's LDS hash (tab, kWaveSlots slots) and scratch: the
// group's X entries 64 at a time, their products spread over the lanes by a
// search over the entries' product offsets.
__device__ __forceinline__ void wave_group_item(const GroupArgs& a, uint32_t g, ZSlot* tab, WaveScratch& sc) {
  const unsigned lane = threadIdx.x & 63u;
  const GroupRec G = a.groups[g];
  const unsigned long long b = a.eoff[G.start + G.count] - a.eoff[G.start];
  const unsigned long long d = b < a.ycells ? b : a.ycells;
  const unsigned tsize = table_size_for(d, kWaveSlots);
  const unsigned tmask = tsize - 1;
  for (unsigned s = lane; s < tsize; s += 64) {
    tab[s].key = kEmpty;
    tab[s].val = 0.0;
  }
  wave_lds_fence();
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
    sc.v[lane] = v;
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
      const YEntry ye = a.yg[y];
      if (!lds_accumulate(tab, tmask, ye.phi, __dmul_rn(sc.v[lo], ye.v), a.seed)) record_error(a.st, kErrCapacity);
    }
    wave_lds_fence();
  }
  unsigned n = 0;
  for (unsigned s = lane; s < tsize; s += 64) n += tab[s].key != kEmpty ? 1u : 0u;
  n = (unsigned)wave_sum((unsigned long long)n);
  if (n) {
    unsigned long long pos = 0;
    if (lane == 0) pos = atomicAdd(out_cursor(a, G.phi), (unsigned long long)n);
    pos = __shfl(pos, 0);
    for (unsigned s0 = 0; s0 < tsize; s0 += 64) {
      const ZSlot z = tab[s0 + lane];
      const bool occ = z.key != kEmpty;
      const unsigned long long m = __ballot(occ);
      if (occ) put_output(a, pos + lanes_below(m), G.phi, z.key, z.val);
      pos += (unsigned long long)__popcll(m);
    }
  }
  wave_lds_fence();
}

// ---------------------------------------------------------------------------
// Dense block class, sliced over the XCDs
// ---------------------------------------------------------------------------
//
// With a dense Y free key (at most kDenseBits bits) a group accumulates in a
// dense array indexed by the Y free key, which is exactly the group's output
// row.  The Y free key space is cut into kSlices equal slices, and every Y
// run (the Y entries of one contracting key, section 4.2) is laid out slice
// by slice at plan time, with yso giving where each slice of each run
// begins.  A tile is (group, slice): one wave walks the group's X entries
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

// Tile (group G, slice) in the wave's dense accumulator acc[wcells]: the
// wave takes G's X entries 64 at a time, one per lane, each lane loading its
// entry's record and the bounds of the entry's slice of its Y run (two
// dependent loads, in parallel across the lanes).  Teams of LPE lanes then
// walk the staged entries, U per team at a time, loading F * LPE Y entries
// of each of its U slices before any of their products is added, so that a
// step's loads are all in flight together; longer slices take further steps.
template <int LPE, int U, int F, bool BUF>
__device__ __forceinline__ void sliced_tile_item(const GroupArgs& a, const GroupRec& G, unsigned slice,
                                                 double* acc, unsigned wcells, const uint32_t* __restrict__ yso,
                                                 int64_t yso_slots, const YReader<BUF>& yr) {
  constexpr unsigned kTeams = 64 / LPE;
  const unsigned lane = threadIdx.x & 63u, team = lane / LPE, tl = lane % LPE;
  const unsigned c0 = slice * wcells;  // first Y free key of the slice
  for (unsigned c = lane; c < wcells; c += 64) acc[c] = -0.0;
  wave_lds_fence();
  for (unsigned e0 = 0; e0 < G.count; e0 += 64) {
    // stage: lane l holds entry e0 + l's slice (start, length) and value
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
          record_error(a.st, kErrInternal);
        }
      } else if (r.ycnt) {
        record_error(a.st, kErrInternal);
      }
    }
    const unsigned staged = G.count - e0 < 64u ? G.count - e0 : 64u;
    for (unsigned s0 = 0; s0 < staged; s0 += U * kTeams) {
      unsigned lo[U], n[U];
      double xv[U];
      unsigned m = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // staged entry s0 + u * kTeams + team (past `staged`: a lane with n = 0)
        if constexpr (LPE == 64) {
          const int src = (int)(s0 + u) & 63;  // uniform: a scalar read of the lane
          lo[u] = __builtin_amdgcn_readlane(my_lo, src);
          n[u] = __builtin_amdgcn_readlane(my_n, src);
          const unsigned long long xb = (unsigned long long)__double_as_longlong(my_x);
          const unsigned xlo = __builtin_amdgcn_readlane((unsigned)xb, src);
          const unsigned xhi = __builtin_amdgcn_readlane((unsigned)(xb >> 32), src);
          xv[u] = __longlong_as_double((long long)(((unsigned long long)xhi << 32) | xlo));
        } else {
          const int src = (int)(s0 + u * kTeams + team) & 63;
          lo[u] = __shfl(my_lo, src);
          n[u] = __shfl(my_n, src);
          xv[u] = __shfl(my_x, src);
        }
        m = n[u] > m ? n[u] : m;
      }
      for (unsigned jb = 0; jb < m; jb += F * LPE) {
        unsigned cell[U][F];
        double yv[U][F];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const unsigned j = jb + f * LPE + tl;
            if (j < n[u]) {
              cell[u][f] = yr.cell(lo[u] + j);
              yv[u][f] = yr.value(lo[u] + j);
            }
          }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const unsigned j = jb + f * LPE + tl;
            if (j < n[u]) {
              const unsigned c = cell[u][f] - c0;
              if (c < wcells)
                atomicAdd(&acc[c], __dmul_rn(xv[u], yv[u][f]) + 0.0);
              else
                record_error(a.st, kErrInternal);
            }
          }
      }
    }
  }
  wave_lds_fence();

  // the tile's outputs: count, reserve with one atomic, write in cell order
  unsigned cnt = 0;
  for (unsigned cw = 0; cw < wcells; cw += 64) cnt += (unsigned)__popcll(__ballot(cell_reached(acc, cw + lane)));
  if (cnt) {
    unsigned long long pos = 0;
    if (lane == 0) pos = atomicAdd(out_cursor(a, G.phi), (unsigned long long)cnt);
    pos = __shfl(pos, 0);
    for (unsigned cw = 0; cw < wcells; cw += 64) {
      const unsigned c = cw + lane;
      const bool occ = cell_reached(acc, c);
      const unsigned long long mask = __ballot(occ);
      if (occ) put_output(a, pos + lanes_below(mask), G.phi, c0 + c, acc[c]);
      pos += (unsigned long long)__popcll(mask);
    }
  }
  wave_lds_fence();
}

}  // namespace
}  // namespace sptc
