// Batched contraction: many independent contractions share every launch.
//
// Each contraction b's entries are rewritten as packed keys prefixed with b
// (contracting key (b, kappa), X free key (b, phiX); the Y free key as is),
// so entries of different contractions never match and never share an X
// group.  One pass of the grouped pipeline then serves the whole batch; its
// key tables are cut into per-contraction regions, so every list of groups
// is ordered by contraction and each output goes straight to its
// contraction's COO.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kPackBlock = 256;

// Writes a key of up to 62 bits as two int32 coordinates (high, low).
__device__ __forceinline__ void put_split(int32_t* idx, int64_t n, int row, int64_t g, uint64_t key, int lo) {
  idx[(int64_t)row * n + g] = (int32_t)(key >> lo);
  idx[(int64_t)(row + 1) * n + g] = (int32_t)(key & low_mask(lo));
}

__global__ __launch_bounds__(kPackBlock) void k_batch_pack(const BatchIn* __restrict__ in,
                                                           const PackTile* __restrict__ tiles, int64_t ntiles,
                                                           BatchWidths w, int32_t* __restrict__ px,
                                                           double* __restrict__ pxv, int64_t nx_total,
                                                           int32_t* __restrict__ py, double* __restrict__ pyv,
                                                           int64_t ny_total, unsigned* err) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const PackTile tile = tiles[t];
    const BatchIn& d = in[tile.b];
    const uint64_t bc = (uint64_t)tile.b << w.wc, bx = (uint64_t)tile.b << w.wx;
    for (int64_t e = tile.start + threadIdx.x; e < tile.end; e += kPackBlock) {
      if (tile.side == 0) {
        if (d.xb.check && !coords_ok(d.xidx, d.nx, e, d.xb)) atomicOr(err, kErrCoord);
        const int64_t g = d.xoff + e;
        put_split(px, nx_total, 0, g, bc | pack_key(d.xidx, d.nx, e, d.xc), w.lo_c);
        put_split(px, nx_total, 2, g, bx | pack_key(d.xidx, d.nx, e, d.xf), w.lo_x);
        pxv[g] = d.xval[e];
      } else {
        if (d.yb.check && !coords_ok(d.yidx, d.ny, e, d.yb)) atomicOr(err, kErrCoord);
        const int64_t g = d.yoff + e;
        put_split(py, ny_total, 0, g, bc | pack_key(d.yidx, d.ny, e, d.yc), w.lo_c);
        put_split(py, ny_total, 2, g, pack_key(d.yidx, d.ny, e, d.yf), w.lo_y);
        pyv[g] = d.yval[e];
      }
    }
  }
}

// Per-contraction product totals, histogrammed per workgroup in LDS.
constexpr int kHistBlock = 256;
constexpr int64_t kHistChunk = 16384;

__global__ __launch_bounds__(kHistBlock) void k_batch_products(const GroupRec* __restrict__ groups, int64_t ngroups,
                                                               const unsigned long long* __restrict__ eoff, int32_t wx,
                                                               int32_t count, unsigned long long* __restrict__ pb) {
  extern __shared__ unsigned long long s_hist[];
  for (int32_t b = threadIdx.x; b < count; b += kHistBlock) s_hist[b] = 0ull;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kHistChunk;
  const int64_t c1 = c0 + kHistChunk < ngroups ? c0 + kHistChunk : ngroups;
  for (int64_t g = c0 + threadIdx.x; g < c1; g += kHistBlock) {
    const GroupRec G = groups[g];
    const uint64_t b = G.phi >> wx;
    if (b < (uint64_t)count) atomicAdd(&s_hist[b], eoff[G.start + G.count] - eoff[G.start]);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < count; b += kHistBlock)
    if (s_hist[b]) atomicAdd(&pb[b], s_hist[b]);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// First place in `list` (ordered by contraction) whose group belongs to a
// contraction >= b.
__device__ __forceinline__ int64_t first_of(const GroupRec* __restrict__ groups, const uint32_t* __restrict__ list,
                                            int64_t n, int32_t wx, uint64_t b) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((groups[list[mid]].phi >> wx) < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_batch_segments(const GroupRec* __restrict__ groups, const uint32_t* __restrict__ dlist, int64_t nd,
                                 const unsigned long long* __restrict__ dpos, int32_t wx, int32_t count,
                                 BatchSeg* __restrict__ seg) {
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x) {
    const int64_t dlo = first_of(groups, dlist, nd, wx, (uint64_t)b);
    const int64_t dhi = first_of(groups, dlist, nd, wx, (uint64_t)b + 1);
    BatchSeg s;
    s.dshift = dlo < dhi ? dpos[dlo] : 0ull;
    s.dcount = dlo < dhi ? dpos[dhi] - dpos[dlo] : 0ull;
    s.cursor = s.dcount;
    seg[b] = s;
  }
}

__global__ void k_batch_reset(int32_t count, BatchSeg* __restrict__ seg) {
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x)
    seg[b].cursor = seg[b].dcount;
}

__global__ void k_batch_finalize(const DevStatus* __restrict__ st, const BatchSeg* __restrict__ seg,
                                 const BatchOut* __restrict__ outs, int32_t count, int64_t* __restrict__ out_nnz) {
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x) {
    const uint32_t err = st->err;
    const unsigned long long c = seg[b].cursor;
    out_nnz[b] = err ? -(int64_t)status_of(err)
                     : ((int64_t)c > outs[b].cap ? -(int64_t)SPTC_ERR_CAPACITY : (int64_t)c);
  }
}

}  // namespace

hipError_t launch_batch_pack(const BatchIn* in, const PackTile* tiles, int64_t ntiles, BatchWidths w, int32_t* px,
                             double* pxv, int64_t nx_total, int32_t* py, double* pyv, int64_t ny_total,
                             unsigned* err, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const unsigned grid = (unsigned)(ntiles < 65536 ? ntiles : 65536);
  k_batch_pack<<<grid, kPackBlock, 0, stream>>>(in, tiles, ntiles, w, px, pxv, nx_total, py, pyv, ny_total, err);
  return hipGetLastError();
}

hipError_t launch_batch_products(const GroupRec* groups, int64_t ngroups, const unsigned long long* eoff,
                                 int32_t wx, int32_t count, unsigned long long* pb, hipStream_t stream) {
  if (ngroups <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((ngroups + kHistChunk - 1) / kHistChunk);
  k_batch_products<<<grid, kHistBlock, (size_t)count * 8, stream>>>(groups, ngroups, eoff, wx, count, pb);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  k_zero_u64<<<dim3((unsigned)g), 256, 0, stream>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_batch_segments(const GroupRec* groups, const uint32_t* dlist, int64_t nd,
                                 const unsigned long long* dpos, int32_t wx, int32_t count, BatchSeg* seg,
                                 hipStream_t stream) {
  const int32_t g = (count + 255) / 256;
  k_batch_segments<<<g < 1 ? 1 : g, 256, 0, stream>>>(groups, dlist, nd, dpos, wx, count, seg);
  return hipGetLastError();
}

hipError_t launch_batch_reset(int32_t count, BatchSeg* seg, hipStream_t stream) {
  const int32_t g = (count + 255) / 256;
  k_batch_reset<<<g < 1 ? 1 : g, 256, 0, stream>>>(count, seg);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const DevStatus* st, const BatchSeg* seg, const BatchOut* outs, int32_t count,
                                 int64_t* out_nnz, hipStream_t stream) {
  const int32_t g = (count + 255) / 256;
  k_batch_finalize<<<g < 1 ? 1 : g, 256, 0, stream>>>(st, seg, outs, count, out_nnz);
  return hipGetLastError();
}

}  // namespace sptc
