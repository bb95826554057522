// Persistent execution of the LDS accumulation classes (section 4.3: each X
// group accumulates its products in a table of its own).
//
// Persistent workgroups drain device-side work queues built from the plan's
// class lists: the dense block class's (group, slice) tiles and the wave
// class's groups (lds_items.hpp), one launch per kind present (each kind is
// its own instantiation of the kernel, so a launch carries only that kind's
// registers).  Every wave is a worker: it takes the next items with one
// atomic on its queue's counter, runs them in its own part of the
// workgroup's LDS, and takes more until the queue is drained, so items of
// uneven cost balance across the waves.  The item counts are read on the
// device (from the plan's class counts), so the launches do not depend on
// them.  A tile of slice s is taken only by waves on XCD s (workgroup b runs
// on XCD b mod 8, and each slice has its own queue), so every XCD reads only
// its slice of grouped Y.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "lds_items.hpp"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kQBlock = 256;  // 4 waves per workgroup, each an independent worker
constexpr int kQWaves = kQBlock / 64;
constexpr int kQXcds = kSlices;

// Next items of one queue for the whole wave: the first of `take`
// consecutive items, taken with one atomic.
__device__ __forceinline__ unsigned long long wave_pop(unsigned long long* ctr, unsigned take) {
  unsigned long long i = 0;
  if ((threadIdx.x & 63u) == 0) i = atomicAdd(ctr, (unsigned long long)take);
  return __shfl(i, 0);
}

constexpr unsigned kWaveTake = 4;  // wave-class groups taken per atomic

// KIND 0: the dense block class's (group, slice) tiles; KIND 1: the wave
// class's groups.  Each kind is its own instantiation, so that a launch
// holds only one kind's registers.
template <int KIND, int LPE, int U, int F, bool BUF>
__global__ __launch_bounds__(kQBlock) void k_lds_queue(GroupArgs a, const uint32_t* __restrict__ list,
                                                       const uint32_t* __restrict__ yso, int64_t yso_slots,
                                                       unsigned wcells, unsigned wave_lds, LdsQueue* q) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  unsigned char* mine = s_dyn + (size_t)(threadIdx.x >> 6) * wave_lds;
  if constexpr (KIND == 0) {
    const unsigned xcd = blockIdx.x % kQXcds;
    const YReader<BUF> yr(a.ykey16, a.yval, a.ny);
    const unsigned long long nb = a.st->n_block;
    for (;;) {
      const unsigned long long i = wave_pop(&q->next_tile[xcd], 1u);
      if (i >= nb) break;
      const GroupRec G = a.groups[list[i]];
      sliced_tile_item<LPE, U, F, BUF>(a, G, xcd, reinterpret_cast<double*>(mine), wcells, yso, yso_slots, yr);
    }
  } else {
    const unsigned long long nw = a.st->n_wave;
    ZSlot* tab = reinterpret_cast<ZSlot*>(mine);
    WaveScratch& sc = *reinterpret_cast<WaveScratch*>(mine + (size_t)kWaveSlots * sizeof(ZSlot));
    for (;;) {
      const unsigned long long i0 = wave_pop(&q->next_wave, kWaveTake);
      if (i0 >= nw) break;
      const unsigned long long i1 = i0 + kWaveTake < nw ? i0 + kWaveTake : nw;
      for (unsigned long long i = i0; i < i1; ++i) wave_group_item(a, list[i], tab, sc);
    }
  }
}

// Block-class X records: run start -> the run's Y table slot.
__global__ __launch_bounds__(256) void k_block_runslots(const GroupRec* __restrict__ groups,
                                                        const uint32_t* __restrict__ blist, int64_t nb,
                                                        XRec* __restrict__ xr, const uint32_t* __restrict__ runslot,
                                                        int64_t ny, DevStatus* st, const DevStatus* dc) {
  const unsigned lane = threadIdx.x & 63u;
  if (dc && (int64_t)dc->n_block < nb) nb = (int64_t)dc->n_block;  // the count read on the device
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
                                 hipStream_t stream, const DevStatus* dc) {
  if (nb <= 0) return hipSuccess;
  k_block_runslots<<<grid_for(nb * 64, 256, num_cus, 8), 256, 0, stream>>>(groups, blist, nb, xr, runslot, ny, st,
                                                                            dc);
  return hipGetLastError();
}

hipError_t prepare_lds_queue() {
  const int tile_lds = (int)(kQWaves * (size_t)((1u << kDenseBits) / kSlices) * 8);
#define SET_LDS(L, UU, FF)                                                                                    \
  do {                                                                                                        \
    hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_queue<0, L, UU, FF, true>),      \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, tile_lds);                \
    if (e_ == hipSuccess)                                                                                     \
      e_ = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_queue<0, L, UU, FF, false>),              \
                               hipFuncAttributeMaxDynamicSharedMemorySize, tile_lds);                         \
    if (e_ != hipSuccess) return e_;                                                                          \
  } while (0)
  SET_LDS(16, 2, 2);
  SET_LDS(32, 2, 2);
  SET_LDS(64, 2, 2);
#undef SET_LDS
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_queue<1, 64, 1, 1, false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kQWaves * kWaveItemLds));
}

namespace {

// Persistent grid: up to 8 workgroups of `lds` bytes per CU, a whole number
// per XCD.
unsigned queue_grid(size_t lds, int num_cus) {
  unsigned per_cu = 8;
  while (per_cu > 1 && per_cu * lds > (size_t)160 * 1024) --per_cu;
  const unsigned grid = (unsigned)(num_cus > 0 ? num_cus : 1) * per_cu;
  return (grid + kQXcds - 1) / kQXcds * kQXcds;
}

}  // namespace

hipError_t launch_lds_queue(const GroupArgs& a, const uint32_t* blist, const uint32_t* wlist, const uint32_t* yso,
                            int64_t yso_slots, unsigned cells, int tiles, int waves, double mean_slice_run,
                            LdsQueue* q, int num_cus, hipStream_t stream) {
  if (tiles) {
    if (cells < 1024u || (cells & (cells - 1u)) || cells > (1u << kDenseBits)) return hipErrorInvalidValue;
    const unsigned wcells = cells / kSlices, wave_lds = wcells * 8;
    const size_t lds = (size_t)kQWaves * wave_lds;
    const unsigned grid = queue_grid(lds, num_cus);
    // buffer loads when the compact Y arrays fit 31-bit byte offsets
    const bool buf = a.ny < ((int64_t)1 << 28);
#define Q_LAUNCH(L, UU, FF)                                                                                       \
  (buf ? (k_lds_queue<0, L, UU, FF, true><<<grid, kQBlock, lds, stream>>>(a, blist, yso, yso_slots, wcells,       \
                                                                           wave_lds, q), 0)                       \
       : (k_lds_queue<0, L, UU, FF, false><<<grid, kQBlock, lds, stream>>>(a, blist, yso, yso_slots, wcells,      \
                                                                            wave_lds, q), 0))
    // lanes per X entry from the mean length of a run's slice: short slices
    // share a wave between several entries
    if (mean_slice_run <= 24.0)
      Q_LAUNCH(16, 2, 2);
    else if (mean_slice_run <= 48.0)
      Q_LAUNCH(32, 2, 2);
    else
      Q_LAUNCH(64, 2, 2);
#undef Q_LAUNCH
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (waves) {
    const unsigned wave_lds = (unsigned)((kWaveItemLds + 15) & ~(size_t)15);
    const size_t lds = (size_t)kQWaves * wave_lds;
    k_lds_queue<1, 64, 1, 1, false><<<queue_grid(lds, num_cus), kQBlock, lds, stream>>>(a, wlist, yso, yso_slots, 0u,
                                                                                        wave_lds, q);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace sptc
