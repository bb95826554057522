// Block class on the matrix cores.
//
// With a dense Y free key (at most kDenseBits bits) and one contraction, the
// block class is a product of two sparse matrices: rows are the block-class
// X groups (X free keys), the inner dimension the Y runs (contracting keys,
// section 4.1: X and Y are grouped by them), columns the Y free cells that
// occur.  Row g holds the X entries of group g at their runs, and run k holds
// the Y entries of contracting key k at their cells, so entry (g, c) of the
// product sums every matching x * y of the output coordinate (g's X free key,
// c) -- the contraction of Eq. 4 for those outputs.  When X and Y are dense
// enough that rows x columns x runs is within a small factor of the products
// this class would otherwise walk, the product is computed densely: each
// workgroup owns a kMfmaRows x kMfmaCols output tile, and for every step of
// kMfmaK runs scatters the tile's X and Y entries into zeroed LDS tiles and
// multiplies them with v_mfma_f64_16x16x4f64.  Which outputs exist is
// structural (some matching pair, whatever the values), so alongside the
// values each step ORs per-row and per-column bitmasks of the runs present:
// output (g, c) exists when the masks of g and c share a run in some step.
//
// The plan writes X and Y as dense panels laid out block by block in the
// order the tiles read them, with the run masks beside them, so that a step
// is two contiguous 16 KiB copies into LDS (loaded a step ahead into
// registers) followed by the MFMA; the work is that of a dense product over
// the padded rows, columns and runs, which the plan weighs against the
// products before it takes this class.
//
// Every product is an exact FP64 multiply whose sums are rounded in another
// order than the walk's (MFMA accumulates with fused multiply-adds), inside
// the reordering bound that both paths meet.  Zero padding contributes exact
// zeros, which is why the plan takes this class only when every value
// involved is finite (0 * Inf would be NaN).
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kMBlock = 256;               // 4 waves: wave w computes rows [16w, 16w + 16) of the tile
constexpr int kAStride = kMfmaK + 2;       // LDS row of the X block ([row][run]), in doubles: 16-byte
                                           // stores, and the 16 rows an MFMA operand reads in distinct banks
constexpr int kBStride = kMfmaCols + 16;   // LDS row of the Y block, in doubles (padded)
constexpr int kAPairs = kMfmaK * kMfmaRows / 2 / kMBlock;  // 16-byte loads per thread and step
constexpr int kBPairs = kMfmaK * kMfmaCols / 2 / kMBlock;
constexpr unsigned kXcdsM = 8;            // MI355X: 8 XCDs, each with its own L2
static_assert(kMfmaRows == 64 && kMfmaCols == 64 && kMfmaK == 32, "tile shape is fixed by the lane layout below");

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Plan time
// ---------------------------------------------------------------------------

// The Y free cells that occur (LDS bitmap per workgroup, ORed into colbits).
// Runs: the non-empty Y table slots in slot order, which is the order of
// their starts (the table scan placed the runs in slot order).
struct MfmaRunOp {
  const YSlot* tab;
  unsigned* run_start;
  unsigned* runid;  // [ny]: at each run's start, the run's index
  unsigned ny;
  __device__ unsigned long long get(int64_t i) const { return tab[i].count > 0u ? 1ull : 0ull; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long v) const {
    if (!v) return;
    const unsigned s = tab[i].start;
    run_start[excl] = s;
    if (s < ny) runid[s] = (unsigned)excl;
  }
};

struct FinRuns {
  unsigned* run_start;
  unsigned ny;
  unsigned long long expected;  // runs the plan counted (the Y groups)
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const {
    if (total != expected) record_error(st, kErrInternal);
    run_start[total] = ny;
  }
};

// Columns: occurring cells numbered in key order (one workgroup, 8 cells per thread).
__global__ __launch_bounds__(1024) void k_mfma_cols(const unsigned* __restrict__ colbits, uint16_t* __restrict__ colid,
                                                    uint16_t* __restrict__ cellof) {
  static_assert((1u << kDenseBits) == 8 * 1024, "8 cells per thread");
  __shared__ unsigned long long s_wave[1024 / 64 + 1];
  const unsigned t = threadIdx.x;
  const unsigned bits = (colbits[t >> 2] >> ((t & 3) * 8)) & 0xffu;
  unsigned long long total;
  unsigned long long col = block_excl_scan<1024>((unsigned long long)__popc(bits), s_wave, &total);
  for (unsigned b = 0; b < 8; ++b) {
    const unsigned cell = 8 * t + b;
    if ((bits >> b) & 1u) {
      colid[cell] = (uint16_t)col;
      cellof[col] = (uint16_t)cell;
      ++col;
    } else {
      colid[cell] = 0xffffu;
    }
  }
}

// X into its panel, one wave per row (block group i, or a padding row past
// nb): the row's entries are added into an LDS copy of a chunk of its panel
// row (kXChunk runs; repeated X coordinates add up), with a bit per run in
// the chunk's step masks, and the chunk is then written out whole (zeros
// included), so the panel needs no clearing and no global atomics.
constexpr unsigned kXChunk = 2560;  // runs per LDS chunk (80 steps)
constexpr unsigned kXWaves = 1;  // one-wave workgroups: LDS is taken per wave, so more rows fit a CU
constexpr unsigned kXUnroll = 4;  // entries per lane in flight
static_assert(kXChunk % kMfmaK == 0, "chunks of whole steps");

__global__ __launch_bounds__(64 * kXWaves) void k_mfma_x_panel(const GroupRec* __restrict__ groups,
                                                               const uint32_t* __restrict__ blist, int64_t nb,
                                                               const XRec* __restrict__ xr,
                                                               const unsigned* __restrict__ runid,
                                                               const unsigned* __restrict__ run_start,
                                                               unsigned nruns, unsigned nsteps,
                                                               double* __restrict__ a, unsigned* __restrict__ am,
                                                               DevStatus* st) {
  __shared__ double s_v[kXWaves][kXChunk];
  __shared__ unsigned s_m[kXWaves][kXChunk / kMfmaK];
  const unsigned lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* v = s_v[w];
  unsigned* msk = s_m[w];
  const int64_t rows = (nb + kMfmaRows - 1) / kMfmaRows * kMfmaRows;
  const size_t K = (size_t)nsteps * kMfmaK;
  const unsigned yend = run_start[nruns];
  const int64_t waves = (int64_t)gridDim.x * kXWaves;
  for (int64_t i = (int64_t)blockIdx.x * kXWaves + w; i < rows; i += waves) {
    const GroupRec G = i < nb ? groups[blist[i]] : GroupRec{0ull, 0u, 0u};
    for (size_t k0 = 0; k0 < K; k0 += kXChunk) {
      const unsigned nk = (unsigned)(K - k0 < kXChunk ? K - k0 : kXChunk);
      for (unsigned j = lane; j < nk; j += 64) v[j] = 0.0;
      for (unsigned j = lane; j < nk / kMfmaK; j += 64) msk[j] = 0u;
      wave_lds_fence();
      // kXUnroll entries per lane at a time: their record, run and run
      // start loads are in flight together
      for (unsigned e0 = 0; e0 < G.count; e0 += kXUnroll * 64) {
        XRec r[kXUnroll];
        unsigned k[kXUnroll], ks[kXUnroll];
#pragma unroll
        for (unsigned u = 0; u < kXUnroll; ++u) {
          const unsigned e = e0 + u * 64 + lane;
          r[u] = e < G.count ? xr[G.start + e] : XRec{0u, 0u, 0.0};
        }
#pragma unroll
        for (unsigned u = 0; u < kXUnroll; ++u)
          k[u] = r[u].ycnt && r[u].ystart < yend ? runid[r[u].ystart] : 0xffffffffu;
#pragma unroll
        for (unsigned u = 0; u < kXUnroll; ++u) ks[u] = k[u] < nruns ? run_start[k[u]] : 0xffffffffu;
#pragma unroll
        for (unsigned u = 0; u < kXUnroll; ++u) {
          if (!r[u].ycnt) continue;
          if (k[u] >= nruns || ks[u] != r[u].ystart) {
            if (k0 == 0) record_error(st, kErrInternal);
            continue;
          }
          if (k[u] < k0 || k[u] >= k0 + nk) continue;
          const unsigned kk = (unsigned)(k[u] - k0);
          atomicAdd(&v[kk], r[u].v);
          atomicOr(&msk[kk / kMfmaK], 1u << (kk % kMfmaK));
        }
      }
      wave_lds_fence();
      double* dst = a + (size_t)i * K + k0;  // 16-byte aligned: K and k0 are even
      for (unsigned j = 2 * lane; j < nk; j += 128)
        *reinterpret_cast<v2d*>(dst + j) = v2d{v[j], v[j + 1]};
      for (unsigned j = lane; j < nk / kMfmaK; j += 64) am[(size_t)i * nsteps + k0 / kMfmaK + j] = msk[j];
      wave_lds_fence();
    }
  }
}

// Y into its panel, one workgroup per step (its 32 runs), the column
// numbering staged in LDS: values are stored into the zeroed panel (added
// when Y repeats a coordinate).  A step's entries are split over `split`
// workgroups; each ORs its column masks in LDS and then its nonzero words
// into the zeroed mask panel.
constexpr unsigned kYBlock = 512;
__global__ __launch_bounds__(kYBlock) void k_mfma_y_panel(const unsigned* __restrict__ run_start, unsigned nruns,
                                                          int64_t ny, const uint16_t* __restrict__ ykey16,
                                                          const double* __restrict__ yval,
                                                          const uint16_t* __restrict__ colid, unsigned nsteps,
                                                          unsigned split, unsigned ncols, unsigned nct, int ydup,
                                                          double* __restrict__ b, unsigned* __restrict__ bm,
                                                          DevStatus* st) {
  constexpr unsigned kCells = 1u << kDenseBits;
  __shared__ uint16_t s_col[kCells];
  __shared__ unsigned s_mask[kCells + kMfmaCols];  // nct * 64 <= kCells + 63
  __shared__ unsigned s_run[kMfmaK + 1];
  for (unsigned q = threadIdx.x; q < kCells; q += kYBlock) s_col[q] = colid[q];
  const unsigned ncp = nct * kMfmaCols;
  const unsigned items = nsteps * split;
  for (unsigned w = blockIdx.x; w < items; w += gridDim.x) {
    const unsigned step = w / split, part = w % split;
    for (unsigned q = threadIdx.x; q < ncp; q += kYBlock) s_mask[q] = 0u;
    if (threadIdx.x <= kMfmaK) {
      const unsigned k = step * kMfmaK + threadIdx.x;
      s_run[threadIdx.x] = run_start[k < nruns ? k : nruns];
    }
    __syncthreads();
    // the step's entries: runs of the step are contiguous in grouped Y
    const unsigned lo = s_run[0], hi = s_run[kMfmaK];
    const bool bad = lo > hi || (int64_t)hi > ny;  // runs ascend inside [0, ny) by construction
    const unsigned len = bad ? 0u : hi - lo;
    const unsigned plo = lo + (unsigned)((unsigned long long)len * part / split);
    const unsigned phi = lo + (unsigned)((unsigned long long)len * (part + 1) / split);
    for (unsigned j = plo + threadIdx.x; j < phi; j += kYBlock) {
      unsigned kk = 0;  // run of j within the step
#pragma unroll
      for (unsigned half = kMfmaK / 2; half > 0; half >>= 1)
        if (s_run[kk + half] <= j) kk += half;
      const unsigned c = s_col[ykey16[j] & (kCells - 1u)];
      if (c >= ncols) {
        record_error(st, kErrInternal);
        continue;
      }
      const double v = yval[j];
      double* dst = &b[(((size_t)(c / kMfmaCols) * nsteps + step) * kMfmaK + kk) * kMfmaCols + c % kMfmaCols];
      if (ydup)
        atomicAdd(dst, v);
      else
        *dst = v;
      atomicOr(&s_mask[c], 1u << kk);
    }
    if (bad && part == 0 && threadIdx.x == 0) record_error(st, kErrInternal);
    __syncthreads();
    for (unsigned q = threadIdx.x; q < ncp; q += kYBlock)
      if (s_mask[q]) atomicOr(&bm[((size_t)(q / kMfmaCols) * nsteps + step) * kMfmaCols + q % kMfmaCols], s_mask[q]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Execute
// ---------------------------------------------------------------------------

// One thread's share of a step's blocks, 16 bytes per load, and for
// threads [0, kMfmaRows) a row mask, [kMfmaRows, + kMfmaCols) a column mask.
struct StepRegs {
  v2d a[kAPairs], b[kBPairs];
  unsigned mask;
};

// A step's X block: rows rt * 64 .. + 63 of the row-major X panel at runs
// step * 32 .. + 31, 16 threads per row (256 contiguous bytes); the Y block
// is the contiguous 32 x 64 block of its panel.
__device__ __forceinline__ void load_step(const MfmaPlan& m, const double* arow, size_t arow0, size_t K,
                                          unsigned step, size_t bblk, StepRegs& r) {
  const unsigned t = threadIdx.x;
  const v2d* b2 = reinterpret_cast<const v2d*>(m.b + bblk * (kMfmaK * kMfmaCols));
  // arow: this thread's first X row (t / 16) at its pair (t % 16); pair u is
  // 16 u rows further (kMBlock / 16 rows per u)
#pragma unroll
  for (int u = 0; u < kAPairs; ++u)
    r.a[u] = *reinterpret_cast<const v2d*>(arow + (size_t)u * (kMBlock / (kMfmaK / 2)) * K + (size_t)step * kMfmaK);
#pragma unroll
  for (int u = 0; u < kBPairs; ++u) r.b[u] = b2[t + u * kMBlock];
  r.mask = t < kMfmaRows ? m.am[(arow0 + t) * (K / kMfmaK) + step]
                         : (t < kMfmaRows + kMfmaCols ? m.bm[bblk * kMfmaCols + t - kMfmaRows] : 0u);
}

__device__ __forceinline__ void store_step(const StepRegs& r, double* s_at, double* s_b, unsigned* s_amask,
                                           unsigned* s_bmask) {
  const unsigned t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kAPairs; ++u) {  // [row][run], as the panel
    const unsigned p = t + u * kMBlock, row = p / (kMfmaK / 2), kp = p % (kMfmaK / 2);
    *reinterpret_cast<v2d*>(&s_at[row * kAStride + 2 * kp]) = r.a[u];
  }
#pragma unroll
  for (int u = 0; u < kBPairs; ++u) {
    const unsigned q = 2 * (t + u * kMBlock);
    *reinterpret_cast<v2d*>(&s_b[(q / kMfmaCols) * kBStride + q % kMfmaCols]) = r.b[u];
  }
  if (t < kMfmaRows)
    s_amask[t] = r.mask;
  else if (t < kMfmaRows + kMfmaCols)
    s_bmask[t - kMfmaRows] = r.mask;
}

__global__ __launch_bounds__(kMBlock, 3) void k_group_block_mfma(GroupArgs a, const uint32_t* __restrict__ blist,
                                                              int64_t nb, MfmaPlan m) {
  static_assert(kMfmaRows + kMfmaCols <= kMBlock, "one thread per row and column mask");
  __shared__ __align__(16) double s_at[kMfmaRows * kAStride];  // X block: [row][run]
  __shared__ __align__(16) double s_b[kMfmaK * kBStride];   // Y block: [run][column]
  __shared__ unsigned s_amask[kMfmaRows], s_bmask[kMfmaCols];
  __shared__ unsigned long long s_phi[kMfmaRows];
  __shared__ unsigned s_cell[kMfmaCols];
  __shared__ unsigned long long s_wave[kMBlock / 64 + 1];
  __shared__ unsigned long long s_base;

  const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned nrt = (unsigned)((nb + kMfmaRows - 1) / kMfmaRows), nct = m.nct, nsteps = m.nsteps;
  const int64_t tiles = (int64_t)nrt * nct;
  // XCD-aware order: workgroups go round-robin over the XCDs, and each XCD
  // takes a contiguous range of tiles, row tile major, so that the
  // workgroups running together on an XCD share X panels in its L2.
  const unsigned nxcd = gridDim.x % kXcdsM == 0 ? kXcdsM : 1u;
  const unsigned xcd = blockIdx.x % nxcd, per_xcd = gridDim.x / nxcd;
  const int64_t lo = tiles * xcd / nxcd, hi = tiles * (xcd + 1) / nxcd;

  for (int64_t tile = lo + blockIdx.x / nxcd; tile < hi; tile += per_xcd) {
    const unsigned rt = (unsigned)(tile / nct), ct = (unsigned)(tile % nct);
    if (tid < kMfmaRows) {
      const int64_t i = (int64_t)rt * kMfmaRows + tid;
      s_phi[tid] = i < nb ? a.groups[blist[i]].phi : 0ull;
    } else if (tid < kMfmaRows + kMfmaCols) {
      const unsigned c = ct * kMfmaCols + (tid - kMfmaRows);
      s_cell[tid - kMfmaRows] = c < m.ncols ? m.cellof[c] : 0u;
    }
    // the wave's 16 rows x 64 columns as 4 MFMA tiles
    v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
    // bit 4c + q: output (row 16 wave + (lane >> 4) + 4q, column 16c + (lane & 15)) exists
    unsigned sbits = 0u;
    const size_t arow0 = (size_t)rt * kMfmaRows, K = (size_t)nsteps * kMfmaK, bblk0 = (size_t)ct * nsteps;
    const double* arow = m.a + (arow0 + tid / (kMfmaK / 2)) * K + 2 * (tid % (kMfmaK / 2));
    const unsigned last = nsteps - 1;
    // software pipeline two steps deep: step s's blocks are loaded into
    // registers (buffers 0 / 1 alternate) while steps s - 2 and s - 1
    // multiply; loads past the last step reload it (unconditional loads keep
    // no branch between a load and its use)
    StepRegs r0, r1;
    load_step(m, arow, arow0, K, 0, bblk0, r0);
    load_step(m, arow, arow0, K, min(1u, last), bblk0 + min(1u, last), r1);
    auto step_body = [&](StepRegs& r, unsigned step) {
      __syncthreads();  // the previous step's MFMA has read the blocks
      store_step(r, s_at, s_b, s_amask, s_bmask);
      load_step(m, arow, arow0, K, min(step + 2, last), bblk0 + min(step + 2, last), r);
      __syncthreads();
      // the multiply phase at raised wave priority: a wave that has its blocks
      // issues its MFMAs ahead of waves still copying the next ones
      __builtin_amdgcn_s_setprio(1);
      // D (16 x 16) += A (16 x 4) B (4 x 16): lane holds A[lane & 15][lane >> 4],
      // B[lane >> 4][lane & 15], and D rows (lane >> 4) + 4q of column lane & 15.
#pragma unroll
      for (unsigned s4 = 0; s4 < (unsigned)kMfmaK / 4; ++s4) {
        const unsigned kr = 4 * s4 + (lane >> 4);
        const double av = s_at[(16 * wave + (lane & 15)) * kAStride + kr];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double bv = s_b[kr * kBStride + 16 * c + (lane & 15)];
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[c], 0, 0, 0);
        }
      }
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned bmk = s_bmask[16 * c + (lane & 15)];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (s_amask[16 * wave + (lane >> 4) + 4 * q] & bmk) sbits |= 1u << (4 * c + q);
      }
    };
    for (unsigned step = 0; step + 1 < nsteps; step += 2) {
      step_body(r0, step);
      step_body(r1, step + 1);
    }
    if (nsteps & 1u) step_body(r0, last);

    // outputs: one reservation per tile; inside a wave, the outputs of one
    // accumulator register go to consecutive positions in lane order, so
    // that each store instruction writes contiguous memory
    unsigned long long total;
    unsigned mine = (unsigned)__popc(sbits);
    // per-wave total, then the wave's base by a block scan over the waves
    unsigned wtotal = mine;
    for (int off = 32; off > 0; off >>= 1) wtotal += __shfl_xor(wtotal, off);
    unsigned long long wbase = block_excl_scan<kMBlock>(lane == 0 ? (unsigned long long)wtotal : 0ull, s_wave, &total);
    wbase = __shfl(wbase, 0);
    if (tid == 0) s_base = total ? atomicAdd(&a.st->out_base, total) : 0ull;
    __syncthreads();
    // position of each accumulator's output after the wave's base (~0u: no
    // output, or past the capacity)
    const unsigned long long base = s_base + wbase;
    const unsigned long long room = (int64_t)base < a.out_cap ? (unsigned long long)a.out_cap - base : 0ull;
    unsigned rel[4][4];
    unsigned run = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool has = (sbits >> (4 * c + q)) & 1u;
        const unsigned long long m = __ballot(has);
        const unsigned r = run + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
        rel[c][q] = has && r < room ? r : ~0u;
        run += (unsigned)__popcll(m);
      }
    // one output row (coordinate mode) at a time: the loops over modes stay
    // rolled, so the kernel's code stays small
    unsigned long long rphi[4];
    unsigned ccell[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rphi[q] = s_phi[16 * wave + (lane >> 4) + 4 * q];
#pragma unroll
    for (int c = 0; c < 4; ++c) ccell[c] = s_cell[16 * c + (lane & 15)];
    const int nx = a.ux.n, ny = a.uy.n;
    for (int d = 0; d < nx; ++d) {
      const uint32_t fd = a.ux.field[d];
      int32_t* dst = a.out_idx + (int64_t)(a.ux.row0 + d) * a.out_cap + (int64_t)base;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rel[c][q] != ~0u) __builtin_nontemporal_store(key_field(rphi[q], fd), dst + rel[c][q]);
    }
    for (int d = 0; d < ny; ++d) {
      const uint32_t fd = a.uy.field[d];
      int32_t* dst = a.out_idx + (int64_t)(a.uy.row0 + d) * a.out_cap + (int64_t)base;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rel[c][q] != ~0u) __builtin_nontemporal_store(key_field(ccell[c], fd), dst + rel[c][q]);
    }
    double* vdst = a.out_val + base;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (rel[c][q] != ~0u) __builtin_nontemporal_store(acc[c][q], vdst + rel[c][q]);
    __syncthreads();  // the next tile rewrites the row and column tables
  }
}

// Block survey: the block class's products, a thread per block group, one
// atomic per wave, and (workgroup 0) the number of Y free cells that occur.
// (The scatter kernels flag non-finite values.)
__global__ __launch_bounds__(256) void k_block_survey(const GroupRec* __restrict__ groups,
                                                      const uint32_t* __restrict__ blist,
                                                      const unsigned long long* __restrict__ eoff,
                                                      const unsigned* __restrict__ colbits, DevStatus* st) {
  if (blockIdx.x == 0) {
    __shared__ unsigned long long s_wave[256 / 64 + 1];
    unsigned long long n = 0;
    for (unsigned w = threadIdx.x; w < (unsigned)kCellWords; w += 256) n += (unsigned)__popc(colbits[w]);
    n = block_sum<256>(n, s_wave);
    if (threadIdx.x == 0) st->ycols = (unsigned)n;
  }
  const int64_t nb = (int64_t)st->class_hi;
  unsigned long long prod = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
    const GroupRec G = groups[blist[i]];
    prod += eoff[G.start + G.count] - eoff[G.start];
  }
  for (int off = 32; off > 0; off >>= 1) prod += __shfl_xor(prod, off);
  if ((threadIdx.x & 63) == 0 && prod) atomicAdd(&st->block_products, prod);
}

}  // namespace

hipError_t launch_block_survey(const GroupRec* groups, const uint32_t* blist, const unsigned long long* eoff,
                               const unsigned* colbits, DevStatus* st, int num_cus, hipStream_t stream) {
  k_block_survey<<<(unsigned)(2 * num_cus), 256, 0, stream>>>(groups, blist, eoff, colbits, st);
  return hipGetLastError();
}

hipError_t launch_mfma_runs(const YSlot* ytab, int64_t yslots, int64_t ny, unsigned* run_start, unsigned* runid,
                            int64_t nruns, DevStatus* st, void* tile_sums, hipStream_t stream) {
  return device_scan(MfmaRunOp{ytab, run_start, runid, (unsigned)ny}, yslots, tile_sums,
                     FinRuns{run_start, (unsigned)ny, (unsigned long long)nruns, st}, stream);
}

hipError_t launch_mfma_panels(const unsigned* colbits, const GroupRec* groups, const uint32_t* blist, int64_t nb,
                              const XRec* xr, const unsigned* run_start, const unsigned* runid, unsigned nruns,
                              const uint16_t* ykey16, const double* yval, int64_t ny, uint16_t* colid,
                              uint16_t* cellof, unsigned ncols, unsigned nsteps, int ydup, double* a, unsigned* am,
                              double* b, unsigned* bm, DevStatus* st, int num_cus, hipStream_t stream) {
  k_mfma_cols<<<1, 1024, 0, stream>>>(colbits, colid, cellof);
  const int64_t xrows = (nb + kMfmaRows - 1) / kMfmaRows * kMfmaRows;
  k_mfma_x_panel<<<grid_for(xrows * 64, 64 * kXWaves, num_cus, 16), 64 * kXWaves, 0, stream>>>(
      groups, blist, nb, xr, runid, run_start, nruns, nsteps, a, am, st);
  const unsigned nct = (ncols + kMfmaCols - 1) / kMfmaCols;
  if (nsteps == 0) return hipGetLastError();
  // about two workgroups per compute unit, each with at least a few
  // entries per thread
  const int64_t want = (2 * (int64_t)num_cus + nsteps - 1) / nsteps;
  const int64_t room = ny / ((int64_t)nsteps * 4 * kYBlock);
  const unsigned split = (unsigned)std::max<int64_t>(1, std::min(want, room));
  k_mfma_y_panel<<<nsteps * split, kYBlock, 0, stream>>>(run_start, nruns, ny, ykey16, yval, colid, nsteps, split,
                                                        ncols, nct, ydup, b, bm, st);
  return hipGetLastError();
}

hipError_t launch_group_block_mfma(const GroupArgs& a, const uint32_t* blist, int64_t nb, const MfmaPlan& m,
                                   int num_cus, hipStream_t stream) {
  if (nb <= 0 || m.nsteps == 0 || m.nct == 0) return hipSuccess;
  const int64_t tiles = ((nb + kMfmaRows - 1) / kMfmaRows) * (int64_t)m.nct;
  unsigned grid = grid_for(tiles * kMBlock, kMBlock, num_cus, 3);
  if (grid >= kXcdsM) grid -= grid % kXcdsM;  // whole rounds over the XCDs
  k_group_block_mfma<<<grid, kMBlock, 0, stream>>>(a, blist, nb, m);
  return hipGetLastError();
}

}  // namespace sptc
