// Dense block class, sliced over the XCDs.
//
// The block class holds the X groups with the most products (section 4.3:
// the group's bound picks its accumulation table); with a dense Y free key
// (at most kDenseBits bits) each group accumulates in a dense LDS array
// indexed by the Y free key, which is exactly the group's output row.  The
// Y free key space is cut into kSlices equal slices, and every Y run (the Y
// entries of one contracting key, section 4.2) is laid out slice by slice
// at plan time, with yso giving where each slice of each run begins.  A
// tile is (group, slice): one wave walks the group's X entries and, for
// each, the slice of its Y run, adding x * y into the slice's cells of the
// group's row in LDS; then it reserves the row slice's outputs with one
// atomic and writes them.
//
// Slice s runs on XCD s (workgroup b sits on XCD b mod 8), so each XCD reads
// only the Y entries of its slice: one eighth of grouped Y, which stays in
// that XCD's L2 while every group walks it.  The X records are read once
// per slice (eight times in all), a small fraction of the products' Y
// reads.
//
// A cell is an output when some product reached it, whatever its value:
// cells start at -0.0, which any nonzero product changes for good (x + -0.0
// = x, and a sum of nonzero terms that cancels is +0.0 under round to
// nearest), and a product equal to zero sets the cell's bit in a bitmap.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kSlBlock = 256;                  // 4 waves per workgroup, one tile each
constexpr int kSlWaves = kSlBlock / 64;
constexpr int kSlXcds = kSlices;               // MI355X: one slice per XCD
constexpr int kBufferWord3 = 0x00020000;       // buffer descriptor word 3 for gfx9-family (raw, untyped) loads

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

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Loads of the compact grouped Y (16-bit Y free keys, values): through
// buffer descriptors when both arrays fit 32-bit byte offsets (the
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

// One wave per tile.  The wave takes its group's X entries 64 at a time, one
// per lane: each lane loads its entry's record and the bounds of the entry's
// slice of its Y run (two dependent loads, in parallel across the lanes).
// The wave then walks the staged entries U at a time, loading F * 64 Y
// entries of each of the U slices before any of their products is added,
// so that a step's loads are all in flight together; longer slices take
// further steps.  A product is x * y + 0.0 (which turns -0.0 into +0.0 and
// leaves every other value as it is), so a cell that started at -0.0 is
// reached exactly when it is no longer -0.0.
template <int LPE, int U, int F, bool BUF>
__global__ __launch_bounds__(kSlBlock) void k_group_block_sliced(GroupArgs a, const uint32_t* __restrict__ blist,
                                                                 int64_t nb, const uint32_t* __restrict__ yso,
                                                                 int64_t yso_slots, unsigned wcells) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  constexpr unsigned kTeams = 64 / LPE;
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const unsigned team = lane / LPE, tl = lane % LPE;
  double* acc = reinterpret_cast<double*>(s_dyn) + (size_t)wave * wcells;
  const unsigned slice = blockIdx.x % kSlXcds;
  const unsigned c0 = slice * wcells;  // first Y free key of the slice
  const YReader<BUF> yr(a.ykey16, a.yval, a.ny);
  const int64_t rstride = (int64_t)(gridDim.x / kSlXcds) * kSlWaves;
  for (int64_t i = (int64_t)(blockIdx.x / kSlXcds) * kSlWaves + wave; i < nb; i += rstride) {
    const GroupRec G = a.groups[blist[i]];
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
    if (cnt == 0) continue;  // uniform
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.bout ? &a.bseg[G.phi >> a.bwx].cursor : &a.st->out_base, (unsigned long long)cnt);
    base = __shfl(base, 0);
    for (unsigned cw = 0; cw < wcells; cw += 64) {
      const unsigned c = cw + lane;
      const bool occ = cell_reached(acc, c);
      const unsigned long long mask = __ballot(occ);
      if (occ) {
        const unsigned long long pos = base + lanes_below(mask);
        if (a.bout)
          batch_store(a.bout, a.out_idx, a.out_val, a.bwx, (uint32_t)(G.phi >> a.bwx), pos, G.phi, c0 + c, acc[c],
                      a.st);
        else if ((int64_t)pos < a.out_cap)
          write_output(a, pos, G.phi, c0 + c, acc[c]);
      }
      base += (unsigned long long)__popcll(mask);
    }
  }
}

// Block-class X records: run start -> the run's Y table slot.
__global__ __launch_bounds__(256) void k_block_runslots(const GroupRec* __restrict__ groups,
                                                        const uint32_t* __restrict__ blist, int64_t nb,
                                                        XRec* __restrict__ xr, const uint32_t* __restrict__ runslot,
                                                        int64_t ny, DevStatus* st) {
  const unsigned lane = threadIdx.x & 63u;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < nb; i += nw) {
    const GroupRec G = groups[blist[i]];
    for (unsigned e = lane; e < G.count; e += 64) {
      XRec& r = xr[G.start + e];
      if (!r.ycnt) continue;
      if ((int64_t)r.ystart < ny)
        r.ystart = runslot[r.ystart];
      else
        record_error(st, kErrInternal);
    }
  }
}

}  // namespace

hipError_t launch_block_runslots(const GroupRec* groups, const uint32_t* blist, int64_t nb, XRec* xr,
                                 const uint32_t* runslot, int64_t ny, DevStatus* st, int num_cus,
                                 hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  k_block_runslots<<<grid_for(nb * 64, 256, num_cus, 8), 256, 0, stream>>>(groups, blist, nb, xr, runslot, ny, st);
  return hipGetLastError();
}

hipError_t launch_group_block_sliced(const GroupArgs& a, const uint32_t* blist, int64_t nb, const uint32_t* yso,
                                     int64_t yso_slots, unsigned cells, double mean_slice_run, int num_cus,
                                     hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  if (cells < 1024u || (cells & (cells - 1u)) || cells > (1u << kDenseBits)) return hipErrorInvalidValue;
  const unsigned wcells = cells / kSlices;
  const size_t lds = (size_t)kSlWaves * wcells * 8;
  // one tile per wave: (ceil(nb / 4) row sets) x (8 slices) workgroups, at most 8 per CU per slice round
  int64_t sets = (nb + kSlWaves - 1) / kSlWaves;
  const int64_t cap = (int64_t)(num_cus > 0 ? num_cus : 1) * 8;
  if (sets > cap) sets = cap;
  const dim3 grid((unsigned)(sets * kSlXcds));
  // buffer loads when the compact Y arrays fit 31-bit byte offsets
  const bool buf = a.ny < ((int64_t)1 << 28);
  // lanes per X entry from the mean length of a run's slice: short slices
  // share a wave between several entries
#define SL_LAUNCH(L, UU, FF)                                                                               \
  (buf ? (k_group_block_sliced<L, UU, FF, true><<<grid, kSlBlock, lds, stream>>>(a, blist, nb, yso, yso_slots, \
                                                                                  wcells), 0)               \
       : (k_group_block_sliced<L, UU, FF, false><<<grid, kSlBlock, lds, stream>>>(a, blist, nb, yso, yso_slots, \
                                                                                   wcells), 0))
  if (mean_slice_run <= 24.0)
    SL_LAUNCH(16, 2, 2);
  else if (mean_slice_run <= 48.0)
    SL_LAUNCH(32, 2, 2);
  else
    SL_LAUNCH(64, 2, 2);
#undef SL_LAUNCH
  return hipGetLastError();
}

}  // namespace sptc
