// Launches of the LDS accumulation classes (section 4.3: each X group
// accumulates its products in a table of its own).
//
// Dense block class: persistent workgroups drain per-XCD work queues of
// (group, slice) tiles (lds_items.hpp).  Every wave is a worker: it takes
// the next tile with one atomic on its XCD's queue counter, runs it in its
// own part of the workgroup's LDS, and takes more until the queue is
// drained, so tiles of uneven cost balance across the waves.  A tile of
// slice s is taken only by waves on XCD s (workgroup b runs on XCD b mod 8,
// and each slice has its own queue), so every XCD reads only its slice of
// grouped Y.  The tile count is read on the device (from the plan's class
// counts), so the launch does not depend on it.  With many small tiles the
// one-atomic-per-tile reservation (device-scope atomics on one address are
// serialised, about 12 ns each on MI355X) gives way to two launches: one
// counts each tile's outputs, a scan places them, the other accumulates
// again and writes.
//
// Wave class: one group per wave, the groups spread over the waves by a
// fixed stride.  The output positions come from a count pass (each group's
// distinct Y free keys in an LDS key set), a scan of the counts and a fill
// pass, so no two groups contend for one counter, which a class of tens of
// thousands of small groups would otherwise pay in full.  In a batch each
// contraction has its own cursor, and one pass reserves per group on it.
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

// The first of the next `take` items of one queue for the whole wave,
// taken with one atomic.
__device__ __forceinline__ unsigned long long wave_pop(QueueCounter* ctr, unsigned take) {
  unsigned long long i = 0;
  if ((threadIdx.x & 63u) == 0) i = atomicAdd(&ctr->v, (unsigned long long)take);
  return __shfl(i, 0);
}

constexpr unsigned kPopsPerWave = 8;  // chunks per wave when tiles are many: balance against pops

// The dense block class's (group, slice) tiles, per-XCD queues (the tile
// itself: flat_tile_accumulate).  MODE 0: each tile reserves its outputs
// with an atomic and writes them; MODE 1: each tile's output count goes to
// tcnt[t]; MODE 2: each tile writes from tile_base + toff[t].  t = 8 i + s
// for the group at place i of the list and slice s.  Four windows of 64
// products per load batch measured best (eight: slower, from the registers).
constexpr int kFlatK = 4;

template <bool BUF, int MODE>
__global__ __launch_bounds__(kQBlock) void k_lds_queue(GroupArgs a, const uint32_t* __restrict__ list,
                                                       const uint32_t* __restrict__ yso, int64_t yso_slots,
                                                       unsigned wcells, unsigned wave_lds, LdsQueue* q,
                                                       uint32_t* __restrict__ tcnt,
                                                       const unsigned long long* __restrict__ toff) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  double* mine = reinterpret_cast<double*>(s_dyn + (size_t)(threadIdx.x >> 6) * wave_lds);
  const unsigned xcd = blockIdx.x % kQXcds;
  const YReader<BUF> yr(a.ykey16, a.yval, a.ny);
  const unsigned long long nb = a.st->n_block;
  const unsigned long long base = MODE == 2 ? a.st->tile_base : 0ull;
  QueueCounter* ctr = MODE == 2 ? &q->next_fill[xcd] : &q->next_tile[xcd];
  // tiles per pop: one while tiles are few (balance), more when each of the
  // XCD's waves would otherwise pop many times
  const unsigned long long waves_per_xcd = (unsigned long long)(gridDim.x / kQXcds) * kQWaves;
  const unsigned long long want = nb / (waves_per_xcd * kPopsPerWave);
  const unsigned take = want > 1ull ? (want < 256ull ? (unsigned)want : 256u) : 1u;
  for (;;) {
    const unsigned long long i0 = wave_pop(ctr, take);
    if (i0 >= nb) break;
    const unsigned long long i1 = i0 + take < nb ? i0 + take : nb;
    for (unsigned long long i = i0; i < i1; ++i) {
      const GroupRec G = a.groups[list[i]];
      flat_tile_accumulate<kFlatK, BUF>(a, G, xcd, mine, wcells, yso, yso_slots, yr);
      const unsigned c0 = xcd * wcells;
      const unsigned long long t = i * kSlices + xcd;
      if constexpr (MODE == 0) {
        tile_outputs(a, G, c0, mine, wcells);
      } else if constexpr (MODE == 1) {
        const unsigned n = tile_count(mine, wcells);
        if ((threadIdx.x & 63u) == 0) tcnt[t] = n;
      } else {
        tile_write(a, G, c0, mine, wcells, base + toff[t]);
      }
      wave_lds_fence();
    }
  }
}

struct TileScanOp {
  const uint32_t* tcnt;
  unsigned long long* toff;
  const DevStatus* st;
  __device__ int64_t live(int64_t) const { return (int64_t)st->n_block * kSlices; }
  __device__ unsigned long long get(int64_t i) const { return tcnt[i]; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { toff[i] = excl; }
};

// The tiles' outputs follow those placed so far.
struct FinTiles {
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const {
    st->tile_base = st->out_base;
    st->out_base += total;
  }
};

// Wave class: MODE 0 counts each group's outputs into wcnt[i], MODE 1
// accumulates and writes them from direct_products + woff[i], MODE 2 (a
// batch) accumulates and reserves per group.  i is the group's place in the
// list; the list's length is read on the device (at most nw).
constexpr int kWBlock = 256;
constexpr int kWWaves = kWBlock / 64;

template <int MODE>
__global__ __launch_bounds__(kWBlock) void k_wave_class(GroupArgs a, const uint32_t* __restrict__ wlist, int64_t nw,
                                                        uint32_t* __restrict__ wcnt,
                                                        const unsigned long long* __restrict__ woff) {
  constexpr unsigned kTabBytes = kWaveSlots * (MODE == 0 ? sizeof(unsigned long long) : sizeof(ZSlot));
  __shared__ __align__(16) unsigned char s_tab[kWWaves][kTabBytes];
  __shared__ WaveScratch s_sc[kWWaves];
  const unsigned w = threadIdx.x >> 6;
  const int64_t live = (int64_t)a.st->n_wave;
  if (live < nw) nw = live;
  const unsigned long long base = MODE == 1 ? a.st->direct_products : 0ull;
  for (int64_t i = (int64_t)blockIdx.x * kWWaves + w; i < nw; i += (int64_t)gridDim.x * kWWaves) {
    if constexpr (MODE == 0) {
      const unsigned n = wave_group_count(a, wlist[i], reinterpret_cast<unsigned long long*>(s_tab[w]), s_sc[w]);
      if ((threadIdx.x & 63u) == 0) wcnt[i] = n;
    } else {
      wave_group_fill<MODE == 2>(a, wlist[i], MODE == 1 ? base + woff[i] : 0ull, reinterpret_cast<ZSlot*>(s_tab[w]),
                                 s_sc[w]);
    }
  }
}

struct WaveScanOp {
  const uint32_t* wcnt;
  unsigned long long* woff;
  const DevStatus* st;
  __device__ int64_t live(int64_t) const { return (int64_t)st->n_wave; }
  __device__ unsigned long long get(int64_t i) const { return wcnt[i]; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { woff[i] = excl; }
};

// The wave class's outputs follow the direct class's; the atomics of the
// later classes start after them.
struct FinWave {
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const { st->out_base = st->direct_products + total; }
};

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

// Longest first: the dense block class's list reordered by decreasing
// product count, so that each XCD's queue hands out its largest tiles first
// and the smallest ones fill in at the end.  The order is by 1,024 bins of
// the count (bin width: the largest count / 1,024), enough for the balance:
// one workgroup holds every group's count in registers, bins them in LDS,
// scans the bins and places each group at its bin's cursor.
constexpr unsigned kOrderBlock = 1024;
constexpr unsigned kOrderBins = 1024;
constexpr unsigned kOrderPer = kOrderMax / kOrderBlock;

__global__ __launch_bounds__(kOrderBlock) void k_order_blist(const GroupRec* __restrict__ groups,
                                                             const unsigned long long* __restrict__ eoff,
                                                             uint32_t* __restrict__ blist, unsigned nb) {
  __shared__ unsigned s_bin[kOrderBins];
  __shared__ unsigned long long s_wave[kOrderBlock / 64 + 1];
  if (nb < 2u || nb > kOrderMax) return;  // uniform across the block
  uint32_t g[kOrderPer];
  unsigned long long p[kOrderPer];
  unsigned long long pmax = 0;
#pragma unroll
  for (unsigned k = 0; k < kOrderPer; ++k) {
    const unsigned i = k * kOrderBlock + threadIdx.x;
    g[k] = 0u;
    p[k] = 0ull;
    if (i < nb) {
      g[k] = blist[i];
      const GroupRec G = groups[g[k]];
      p[k] = eoff[G.start + G.count] - eoff[G.start];
      pmax = p[k] > pmax ? p[k] : pmax;
    }
  }
  s_bin[threadIdx.x] = 0u;
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(pmax, o);
    pmax = t > pmax ? t : pmax;
  }
  if ((threadIdx.x & 63u) == 0) s_wave[threadIdx.x >> 6] = pmax;
  __syncthreads();
  pmax = 0;
  for (unsigned w = 0; w < kOrderBlock / 64; ++w) pmax = s_wave[w] > pmax ? s_wave[w] : pmax;
  // bin kOrderBins - 1 - floor(p * kOrderBins / (pmax + 1)): the largest counts first
  unsigned bin[kOrderPer];
#pragma unroll
  for (unsigned k = 0; k < kOrderPer; ++k) {
    const unsigned i = k * kOrderBlock + threadIdx.x;
    const double scaled = (double)p[k] * (double)kOrderBins / ((double)pmax + 1.0);  // in [0, kOrderBins)
    bin[k] = kOrderBins - 1u - (scaled < (double)(kOrderBins - 1u) ? (unsigned)scaled : kOrderBins - 1u);
    if (i < nb) atomicAdd(&s_bin[bin[k]], 1u);
  }
  __syncthreads();
  unsigned long long tot;
  const unsigned long long start = block_excl_scan<kOrderBlock>(s_bin[threadIdx.x], s_wave, &tot);
  s_bin[threadIdx.x] = (unsigned)start;  // the bin's cursor
  __syncthreads();
#pragma unroll
  for (unsigned k = 0; k < kOrderPer; ++k) {
    const unsigned i = k * kOrderBlock + threadIdx.x;
    if (i < nb) {
      const unsigned at = atomicAdd(&s_bin[bin[k]], 1u);
      if (at < nb) blist[at] = g[k];
    }
  }
}

}  // namespace

hipError_t launch_order_blist(const GroupRec* groups, const unsigned long long* eoff, uint32_t* blist, int64_t nb,
                              hipStream_t stream) {
  if (nb < 2 || nb > (int64_t)kOrderMax) return hipSuccess;
  k_order_blist<<<1, kOrderBlock, 0, stream>>>(groups, eoff, blist, (unsigned)nb);
  return hipGetLastError();
}

hipError_t launch_block_runslots(const GroupRec* groups, const uint32_t* blist, int64_t nb, XRec* xr,
                                 const uint32_t* runslot, int64_t ny, DevStatus* st, int num_cus,
                                 hipStream_t stream, const DevStatus* dc) {
  if (nb <= 0) return hipSuccess;
  k_block_runslots<<<grid_for(nb * 64, 256, num_cus, 8), 256, 0, stream>>>(groups, blist, nb, xr, runslot, ny, st,
                                                                            dc);
  return hipGetLastError();
}

hipError_t prepare_lds_queue() {
  const int lds = (int)(kQWaves * flat_wave_lds((1u << kDenseBits) / kSlices));
  const void* kernels[] = {reinterpret_cast<const void*>(&k_lds_queue<true, 0>),
                           reinterpret_cast<const void*>(&k_lds_queue<true, 1>),
                           reinterpret_cast<const void*>(&k_lds_queue<true, 2>),
                           reinterpret_cast<const void*>(&k_lds_queue<false, 0>),
                           reinterpret_cast<const void*>(&k_lds_queue<false, 1>),
                           reinterpret_cast<const void*>(&k_lds_queue<false, 2>)};
  for (const void* k : kernels) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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

hipError_t launch_lds_queue(const GroupArgs& a, const uint32_t* blist, int64_t nb, const uint32_t* yso,
                            int64_t yso_slots, unsigned cells, unsigned slice_cells, LdsQueue* q, uint32_t* tcnt,
                            unsigned long long* toff, void* tile_sums, int num_cus, hipStream_t stream) {
  if (cells < 1024u || (cells & (cells - 1u)) || cells > (1u << kDenseBits)) return hipErrorInvalidValue;
  if (slice_cells == 0u || slice_cells % 64u || slice_cells > cells / kSlices) return hipErrorInvalidValue;
  if (a.ny <= 0 || nb <= 0) return hipSuccess;  // no products: no tile has an output
  if ((tcnt == nullptr) != (toff == nullptr)) return hipErrorInvalidValue;
  const unsigned wcells = slice_cells;
  const unsigned wave_lds = (unsigned)flat_wave_lds(wcells);
  const size_t lds = (size_t)kQWaves * wave_lds;
  const unsigned grid = queue_grid(lds, num_cus);
  // buffer loads when the compact Y arrays fit 31-bit byte offsets
  const bool buf = a.ny < ((int64_t)1 << 28);
#define Q_LAUNCH(M)                                                                                            \
  do {                                                                                                         \
    if (buf)                                                                                                   \
      k_lds_queue<true, M><<<grid, kQBlock, lds, stream>>>(a, blist, yso, yso_slots, wcells, wave_lds, q, tcnt, \
                                                          toff);                                              \
    else                                                                                                       \
      k_lds_queue<false, M><<<grid, kQBlock, lds, stream>>>(a, blist, yso, yso_slots, wcells, wave_lds, q, tcnt, \
                                                           toff);                                             \
  } while (0)
  if (!tcnt) {
    Q_LAUNCH(0);
    return hipGetLastError();
  }
  Q_LAUNCH(1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_scan(TileScanOp{tcnt, toff, a.st}, nb * kSlices, tile_sums, FinTiles{a.st}, stream);
  if (e != hipSuccess) return e;
  Q_LAUNCH(2);
#undef Q_LAUNCH
  return hipGetLastError();
}

hipError_t launch_wave_class(const GroupArgs& a, const uint32_t* wlist, int64_t nw, uint32_t* wcnt,
                             unsigned long long* woff, void* tile_sums, int num_cus, hipStream_t stream) {
  if (nw <= 0) return hipSuccess;
  const unsigned grid = grid_for((nw + kWWaves - 1) / kWWaves, 1, num_cus, 8);
  if (a.bout) {
    k_wave_class<2><<<grid, kWBlock, 0, stream>>>(a, wlist, nw, nullptr, nullptr);
    return hipGetLastError();
  }
  if (!wcnt || !woff) return hipErrorInvalidValue;
  k_wave_class<0><<<grid, kWBlock, 0, stream>>>(a, wlist, nw, wcnt, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_scan(WaveScanOp{wcnt, woff, a.st}, nw, tile_sums, FinWave{a.st}, stream);
  if (e != hipSuccess) return e;
  k_wave_class<1><<<grid, kWBlock, 0, stream>>>(a, wlist, nw, nullptr, woff);
  return hipGetLastError();
}

}  // namespace sptc
