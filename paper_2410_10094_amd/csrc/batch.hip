// Batched contraction: many independent contractions share every launch.
//
// Each contraction b's entries are rewritten as packed keys prefixed with b
// (contracting key (b, kappa), X free key (b, phiX); the Y free key as is),
// so entries of different contractions never match and never share an X
// group.  One pass of the grouped pipeline then serves the whole batch, and
// the outputs are sorted back into one COO per contraction.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kPackBlock = 256;

__device__ __forceinline__ uint64_t low_mask(int bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull); }

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

// Places every packed output in its contraction's COO: per workgroup chunk,
// count outputs per contraction in LDS, reserve one run per contraction with
// a single atomic on its cursor, then decode and write.
constexpr int kUnpackBlock = 256;
constexpr int64_t kUnpackChunk = 4096;

__global__ __launch_bounds__(kUnpackBlock) void k_batch_unpack(const int32_t* __restrict__ tidx,
                                                               const double* __restrict__ tval, int64_t tcap,
                                                               const int64_t* __restrict__ tnnz, BatchWidths w,
                                                               int32_t count, const BatchOut* __restrict__ outs,
                                                               int32_t* __restrict__ out_idx,
                                                               double* __restrict__ out_val,
                                                               unsigned long long* __restrict__ cursor) {
  extern __shared__ unsigned long long s_u[];
  unsigned long long* s_base = s_u;                            // [count]
  unsigned* s_cnt = reinterpret_cast<unsigned*>(s_u + count);  // [count]
  const int64_t n = *tnnz < tcap ? *tnnz : tcap;               // negative (an error): nothing to place
  const int64_t c0 = (int64_t)blockIdx.x * kUnpackChunk;
  if (c0 >= n) return;  // uniform across the block
  const int64_t c1 = c0 + kUnpackChunk < n ? c0 + kUnpackChunk : n;
  for (int32_t b = threadIdx.x; b < count; b += kUnpackBlock) s_cnt[b] = 0u;
  __syncthreads();
  auto batch_of = [&](int64_t o) -> uint32_t {
    const uint64_t phix = ((uint64_t)(uint32_t)tidx[o] << w.lo_x) | (uint32_t)tidx[tcap + o];
    return (uint32_t)(phix >> w.wx);
  };
  for (int64_t o = c0 + threadIdx.x; o < c1; o += kUnpackBlock) {
    const uint32_t b = batch_of(o);
    if (b < (uint32_t)count) atomicAdd(&s_cnt[b], 1u);
  }
  __syncthreads();
  for (int32_t b = threadIdx.x; b < count; b += kUnpackBlock) {
    const unsigned c = s_cnt[b];
    if (c) s_base[b] = atomicAdd(&cursor[b], (unsigned long long)c);
    s_cnt[b] = 0u;
  }
  __syncthreads();
  for (int64_t o = c0 + threadIdx.x; o < c1; o += kUnpackBlock) {
    const uint64_t phix = ((uint64_t)(uint32_t)tidx[o] << w.lo_x) | (uint32_t)tidx[tcap + o];
    const uint64_t phiy = ((uint64_t)(uint32_t)tidx[2 * tcap + o] << w.lo_y) | (uint32_t)tidx[3 * tcap + o];
    const uint32_t b = (uint32_t)(phix >> w.wx);
    if (b >= (uint32_t)count) continue;
    const unsigned long long pos = s_base[b] + atomicAdd(&s_cnt[b], 1u);
    const BatchOut& d = outs[b];
    if ((int64_t)pos >= d.cap) continue;
    const uint64_t fx = phix & low_mask(w.wx);
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < d.ux.n)
        __builtin_nontemporal_store((int32_t)((fx >> d.ux.shift[m]) & d.ux.mask[m]),
                                    &out_idx[d.idx_off + (int64_t)m * d.cap + (int64_t)pos]);
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < d.uy.n)
        __builtin_nontemporal_store((int32_t)((phiy >> d.uy.shift[m]) & d.uy.mask[m]),
                                    &out_idx[d.idx_off + (int64_t)(d.ux.n + m) * d.cap + (int64_t)pos]);
    __builtin_nontemporal_store(tval[o], &out_val[d.val_off + (int64_t)pos]);
  }
}

__global__ void k_batch_finalize(const int64_t* __restrict__ tnnz, const unsigned long long* __restrict__ cursor,
                                 const BatchOut* __restrict__ outs, int32_t count, int64_t* __restrict__ out_nnz) {
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x) {
    const int64_t t = *tnnz;
    const unsigned long long c = cursor[b];
    out_nnz[b] = t < 0 ? t : ((int64_t)c > outs[b].cap ? -(int64_t)SPTC_ERR_CAPACITY : (int64_t)c);
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

hipError_t launch_batch_unpack(const int32_t* tidx, const double* tval, int64_t tcap, const int64_t* tnnz,
                               BatchWidths w, int32_t count, const BatchOut* outs, int32_t* out_idx, double* out_val,
                               unsigned long long* cursor, hipStream_t stream) {
  if (tcap <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((tcap + kUnpackChunk - 1) / kUnpackChunk);
  k_batch_unpack<<<grid, kUnpackBlock, (size_t)count * 12, stream>>>(tidx, tval, tcap, tnnz, w, count, outs, out_idx,
                                                                      out_val, cursor);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const int64_t* tnnz, const unsigned long long* cursor, const BatchOut* outs,
                                 int32_t count, int64_t* out_nnz, hipStream_t stream) {
  const int32_t g = (count + 255) / 256;
  k_batch_finalize<<<g < 1 ? 1 : g, 256, 0, stream>>>(tnnz, cursor, outs, count, out_nnz);
  return hipGetLastError();
}

}  // namespace sptc
