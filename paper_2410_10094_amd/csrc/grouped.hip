// X-grouped path: X is grouped by its free key (paper section 4.1: hash each
// free key to a small id, then counting sort), and each group's products are
// accumulated in a table of its own, sized from the group's bound (section
// 4.3: the sum of the Y counts over the group's X entries).  Groups never
// share an output coordinate (the output key embeds the X free key), so no
// accumulation crosses groups.
//
// Groups are sorted into four classes; d = min(products, Y free cells) is the
// most distinct outputs a group can have:
//   direct  one X entry and no repeated coordinate in Y: every product is its
//           own output, written straight from a product-space gather;
//   wave    d <= kWaveCap and few products: one wave, a private LDS hash;
//   block   dense Y free key (<= kDenseBits bits): (group, slice) tiles of a
//           dense LDS accumulator, one wave each; or d <= kBlockCap: one
//           1024-thread workgroup with an LDS hash;
//           dense block tiles run in a persistent launch over per-XCD work
//           queues and reserve their outputs with one atomic each; wave
//           groups take their output positions from a count pass and a
//           scan (queue.hip);
//   global  everything else: the products go to the device-memory hash.
#include <hip/hip_runtime.h>

#include "../../include/sptc.h"
#include "lds_items.hpp"
#include "prim.hpp"
#include "sptc_internal.hpp"

namespace sptc {
namespace {

constexpr int kBBlock = 1024;                           // block-class workgroup (largest table), Y run sort
constexpr int kBMidBlock = 512;                         // block-class workgroup (4,096-slot table): two per CU
constexpr int kBSmallBlock = 256;                       // and for groups that fit the small table
constexpr int kBlockSmallSlots = 2048;
constexpr unsigned kXcds = 8;                          // MI355X: 8 XCDs, each with its own L2
constexpr unsigned long long kWaveMaxProducts = 16384;  // beyond this a group goes to a workgroup

// ---------------------------------------------------------------------------
// Plan: group X by free key
// ---------------------------------------------------------------------------

// X table -> dense group records, in table order (so group runs are in
// increasing storage order).  Scans count << 32 | occupied in one pass.
// Groups and their entries both fit `cap` (the number of X entries) unless
// the table holds stale or corrupt counts: then the op records an internal
// error and writes nothing out of bounds.
struct XTableScanOp {
  YSlot* tab;
  GroupRec* groups;
  bool run_end;  // start = end of run (placement takes and decrements), else its beginning
  unsigned long long cap;
  DevStatus* st;
  __device__ unsigned long long get(int64_t i) const {
    const YSlot s = tab[i];
    return s.key != kEmpty ? (((unsigned long long)s.count << 32) | 1ull) : 0ull;
  }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long v) const {
    if (!v) return;
    const unsigned count = (unsigned)(v >> 32);
    const unsigned long long gi = excl & 0xffffffffull, start = excl >> 32;
    if (gi >= cap || start + count > cap) {
      record_error(st, kErrInternal);
      return;
    }
    GroupRec g;
    g.phi = tab[i].key;
    g.start = (unsigned)start;
    g.count = count;
    groups[gi] = g;
    tab[i].start = run_end ? g.start + count : g.start;
  }
};

struct FinXGroups {
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const { st->xgroups = total & 0xffffffffull; }
};

// X entry e's record: its Y group (start, count; count 0 when Y has no entry
// with its contracting key) and its value.
__device__ __forceinline__ XRec probe_y(const int32_t* __restrict__ xidx, int64_t nnz, int64_t e, const KeyPack& kc,
                                        const YSlot* __restrict__ ytab, const TabGeom& yg, int32_t max_probe_y,
                                        uint64_t seed, double v) {
  const uint64_t ckey = pack_key(xidx, nnz, e, kc);
  ProbeSeq p = probe_seq(ckey, yg, seed);
  XRec r;
  r.ystart = 0;
  r.ycnt = 0;
  r.v = v;
  for (int32_t probe = 0; probe < max_probe_y; ++probe) {
    const YSlot slot = ytab[p.slot()];
    if (slot.key == ckey) {
      r.ystart = slot.start;
      r.ycnt = slot.count;
      break;
    }
    if (slot.key == kEmpty) break;
    p.next();
  }
  return r;
}

// Compact X table for hashed X free keys of at most 31 bits (single
// contraction): one 64-bit word per slot, key << 32 | count, kEmpty when
// free, so a table takes half the memory (and cache) of YSlot and a new key
// is claimed and counted by one compare-and-swap.  After the scan the low
// half holds the end of the key's run, which placement decrements, with
// kSingle set when the key has one entry: that entry is placed without an
// atomic (entry counts stay below 2^31).
constexpr unsigned long long kLow32 = 0xffffffffull;
constexpr unsigned long long kSingle = 1ull << 31;

__global__ __launch_bounds__(256) void k_key_count32(const int32_t* __restrict__ idx, int64_t nnz, KeyPack kc,
                                                     unsigned long long* __restrict__ tab, TabGeom g, uint64_t seed,
                                                     int32_t max_probe, DevStatus* st) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = pack_key(idx, nnz, e, kc);
    const unsigned long long want = (unsigned long long)key << 32 | 1ull;
    ProbeSeq p = probe_seq(key, g, seed);
    for (int32_t probe = 0;; p.next()) {
      const uint64_t s = p.slot();
      const unsigned long long prev = atomicCAS(&tab[s], kEmpty, want);
      if (prev == kEmpty) break;
      if ((prev >> 32) == key) {
        atomicAdd(&tab[s], 1ull);
        break;
      }
      if (++probe >= max_probe) {
        record_error(st, kErrCapacity);
        break;
      }
    }
  }
}

struct XTable32ScanOp {
  unsigned long long* tab;
  GroupRec* groups;
  unsigned long long cap;  // as in XTableScanOp
  DevStatus* st;
  __device__ unsigned long long get(int64_t i) const {
    const unsigned long long w = tab[i];
    return w != kEmpty ? ((w & kLow32) << 32 | 1ull) : 0ull;
  }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long v) const {
    if (!v) return;
    const unsigned long long key = tab[i] >> 32;
    const unsigned long long gi = excl & kLow32, start = excl >> 32;
    if (gi >= cap || start + (v >> 32) > cap) {
      record_error(st, kErrInternal);
      return;
    }
    GroupRec g;
    g.phi = key;
    g.start = (unsigned)start;
    g.count = (unsigned)(v >> 32);
    groups[gi] = g;
    tab[i] = key << 32 | (unsigned long long)(g.start + g.count) | (g.count == 1 ? kSingle : 0ull);
  }
};

__global__ __launch_bounds__(256) void k_x_scatter32(const int32_t* __restrict__ xidx, const double* __restrict__ xval,
                                                     int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                                                     unsigned long long* __restrict__ xtab, TabGeom xg,
                                                     int32_t max_probe_x, const YSlot* __restrict__ ytab, TabGeom yg,
                                                     int32_t max_probe_y, uint64_t seed, XRec* __restrict__ xr,
                                                     DevStatus* st) {
  bool bad = false;  // a value is Inf or NaN
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    if (b.check && !coords_ok(xidx, nnz, e, b)) record_error(st, kErrCoord);
    const uint64_t fkey = pack_key(xidx, nnz, e, kf);
    ProbeSeq p = probe_seq(fkey, xg, seed);
    int64_t s = -1;
    unsigned long long w = kEmpty;
    for (int32_t probe = 0; probe < max_probe_x; ++probe, p.next()) {
      w = xtab[p.slot()];  // the key half and kSingle never change once the scan set them
      if (w == kEmpty) break;
      if ((w >> 32) == fkey) {
        s = (int64_t)p.slot();
        break;
      }
    }
    if (s < 0) {
      record_error(st, kErrInternal);
      continue;
    }
    const unsigned pos = (w & kSingle) ? (unsigned)((w & (kSingle - 1ull)) - 1ull)
                                       : (unsigned)((atomicSub(&xtab[s], 1ull) - 1ull) & (kSingle - 1ull));
    if ((int64_t)pos >= nnz) {
      record_error(st, kErrInternal);
      continue;
    }
    const double v = xval[e];
    bad |= !isfinite(v);
    xr[pos] = probe_y(xidx, nnz, e, kc, ytab, yg, max_probe_y, seed, v);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}


// The rest of a probe of Y's table whose home slot held another key.
__device__ __noinline__ XRec probe_y_from(const YSlot* __restrict__ ytab, ProbeSeq p, int32_t max_probe_y,
                                          uint64_t ckey, double v) {
  XRec r;
  r.ystart = 0;
  r.ycnt = 0;
  r.v = v;
  for (int32_t probe = 1; probe < max_probe_y; ++probe) {
    p.next();
    const YSlot cur = ytab[p.slot()];
    if (cur.key == ckey) {
      r.ystart = cur.start;
      r.ycnt = cur.count;
      break;
    }
    if (cur.key == kEmpty) break;
  }
  return r;
}

// Places every X entry in its group's run and records its Y group.
__global__ __launch_bounds__(256) void k_x_scatter(const int32_t* __restrict__ xidx, const double* __restrict__ xval,
                                                   int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                                                   YSlot* __restrict__ xtab, TabGeom xg, int32_t max_probe_x,
                                                   const YSlot* __restrict__ ytab, TabGeom yg,
                                                   int32_t max_probe_y, uint64_t seed, XRec* __restrict__ xr,
                                                   DevStatus* st) {
  bool bad = false;  // a value is Inf or NaN
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    if (b.check && !coords_ok(xidx, nnz, e, b)) record_error(st, kErrCoord);
    const uint64_t fkey = pack_key(xidx, nnz, e, kf);
    const int64_t s = find_slot(xtab, fkey, xg, seed, max_probe_x);
    if (s < 0) {
      record_error(st, kErrInternal);
      continue;
    }
    const unsigned pos = atomicSub(&xtab[s].start, 1u) - 1u;
    if ((int64_t)pos >= nnz) {
      record_error(st, kErrInternal);
      continue;
    }
    const double v = xval[e];
    bad |= !isfinite(v);
    xr[pos] = probe_y(xidx, nnz, e, kc, ytab, yg, max_probe_y, seed, v);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}

// Aggregated variant for a direct-addressed X table (small X free keys).
__global__ __launch_bounds__(kAggBlock) void k_x_scatter_agg(const int32_t* __restrict__ xidx,
                                                             const double* __restrict__ xval, int64_t nnz, KeyPack kf,
                                                             KeyPack kc, Bounds b, const YSlot* __restrict__ xtab,
                                                             unsigned nslots, const unsigned* __restrict__ choff,
                                                             const YSlot* __restrict__ ytab,
                                                             TabGeom yg, int32_t max_probe_y, uint64_t seed,
                                                             XRec* __restrict__ xr, DevStatus* st) {
  bool bad = false;  // a value is Inf or NaN
  extern __shared__ unsigned s_agg[];
  const bool check = b.check != 0;
  place_chunk(xidx, nnz, kf, check, b, nslots, choff, s_agg, s_agg + nslots,
              [&](const int64_t* e, const uint64_t*, const unsigned* pos, const bool* ok, const bool* inbf) {
                uint64_t ckey[kAggUnroll];
                ProbeSeq ys[kAggUnroll];
                YSlot slot[kAggUnroll];
                double v[kAggUnroll];
                bool inb[kAggUnroll];  // the two packs read every mode once, and check it on the way
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) inb[u] = inbf[u];
                pack_keys<kAggUnroll>(xidx, nnz, e, ok, kc, ckey, check, b, inb);
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) ys[u] = probe_seq(ckey[u], yg, seed);
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) {  // first probes and values, all in flight together
                  if (!ok[u]) continue;
                  slot[u] = ytab[ys[u].slot()];
                  v[u] = xval[e[u]];
                  bad |= !isfinite(v[u]);
                }
#pragma unroll
                for (int u = 0; u < kAggUnroll; ++u) {
                  if (!ok[u]) continue;
                  if (check && !inb[u]) record_error(st, kErrCoord);
                  if ((int64_t)pos[u] >= nnz) {
                    record_error(st, kErrInternal);
                    continue;
                  }
                  XRec r;
                  r.ystart = 0;
                  r.ycnt = 0;
                  r.v = v[u];
                  if (slot[u].key == ckey[u]) {
                    r.ystart = slot[u].start;
                    r.ycnt = slot[u].count;
                  } else if (slot[u].key != kEmpty) {
                    r = probe_y_from(ytab, ys[u], max_probe_y, ckey[u], v[u]);
                  }
                  xr[pos[u]] = r;
                }
              });
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1u);
}

struct EntryScanOp {
  const XRec* xr;
  unsigned long long* eoff;
  __device__ unsigned long long get(int64_t i) const { return xr[i].ycnt; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { eoff[i] = excl; }
};

struct FinEntries {
  unsigned long long* eoff_end;
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const {
    *eoff_end = total;
    st->products = total;
  }
};

// Class codes (U128): direct {1, 0}, wave {1 << 32, 0}, block {0, 1},
// global {0, 0}.
struct ClassifyOp {
  const GroupRec* groups;
  const unsigned long long* eoff;
  const DevStatus* st;
  uint64_t ycells;
  int32_t dense;
  uint32_t* dlist;
  uint32_t* wlist;
  uint32_t* blist;
  uint32_t* glist;
  unsigned long long* dcnt;  // direct group k's products, at the k-th place (scanned in place into offsets)
  unsigned long long block_cap;  // most distinct outputs of a group in a workgroup's LDS hash
  const XRec* xr;                // grouped X records
  DRec* drec;                    // direct group k's staging record, at the k-th place
  __device__ U128 code(int64_t g) const {
    const GroupRec G = groups[g];
    const unsigned long long b = eoff[G.start + G.count] - eoff[G.start];
    const unsigned long long d = b < ycells ? b : ycells;
    if (G.count == 1 && !st->ydup) return U128{1ull, 0ull};
    if (d <= (unsigned long long)kWaveCap && b <= kWaveMaxProducts) return U128{1ull << 32, 0ull};
    if (dense || d <= block_cap) return U128{0ull, 1ull};
    return U128{0ull, 0ull};
  }
  __device__ int64_t live(int64_t) const { return (int64_t)st->xgroups; }
  __device__ U128 get(int64_t g) const { return (unsigned long long)g < st->xgroups ? code(g) : U128{0ull, 0ull}; }
  __device__ void put(int64_t g, U128 excl, U128 v) const {
    if ((unsigned long long)g >= st->xgroups) return;
    const unsigned long long nd = excl.lo & 0xffffffffull, nw = excl.lo >> 32, nb = excl.hi;
    if (v.lo == 1ull) {
      dlist[nd] = (uint32_t)g;
      const GroupRec G = groups[g];  // read by code(g) just before: a cache hit
      dcnt[nd] = eoff[G.start + G.count] - eoff[G.start];
      const XRec r = xr[G.start];
      drec[nd] = DRec{G.phi, r.v, r.ystart, 0u};
    } else if (v.lo)
      wlist[nw] = (uint32_t)g;
    else if (v.hi)
      blist[nb] = (uint32_t)g;
    else
      glist[(unsigned long long)g - nd - nw - nb] = (uint32_t)g;
  }
};

struct FinClassify {
  DevStatus* st;
  __device__ void operator()(U128 total) const {
    st->class_lo = total.lo;
    st->class_hi = total.hi;
    st->n_direct = total.lo & 0xffffffffull;
    st->n_wave = total.lo >> 32;
    st->n_block = total.hi;
    st->n_global = st->xgroups - st->n_direct - st->n_wave - st->n_block;
  }
};

// In place over dpos: the products of each direct group (written by the
// classification) become their offsets.  A thread reads element i before
// it writes it, and no other thread touches it.
struct DirectScanOp {
  unsigned long long* dpos;
  const DevStatus* st;
  __device__ bool valid(int64_t i) const { return (unsigned long long)i < (st->class_lo & 0xffffffffull); }
  __device__ int64_t live(int64_t) const { return (int64_t)(st->class_lo & 0xffffffffull); }
  __device__ unsigned long long get(int64_t i) const { return valid(i) ? dpos[i] : 0ull; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const {
    if (valid(i)) dpos[i] = excl;
  }
};

struct FinDirect {
  unsigned long long* dpos;
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const {
    dpos[st->class_lo & 0xffffffffull] = total;
    st->direct_products = total;
  }
};

struct GlobalEntryScanOp {
  const GroupRec* groups;
  const uint32_t* glist;
  unsigned long long* gl_eoff;
  const DevStatus* st;
  __device__ int64_t live(int64_t) const { return (int64_t)st->n_global; }
  __device__ unsigned long long get(int64_t i) const { return groups[glist[i]].count; }
  __device__ void put(int64_t i, unsigned long long excl, unsigned long long) const { gl_eoff[i] = excl; }
};

struct FinGlobalEntries {
  DevStatus* st;
  __device__ void operator()(unsigned long long total) const { st->global_entries = total; }
};

__global__ __launch_bounds__(256) void k_gather_global(const GroupRec* __restrict__ groups,
                                                       const uint32_t* __restrict__ glist, int64_t ngl,
                                                       const unsigned long long* __restrict__ gl_eoff,
                                                       const XRec* __restrict__ xr, XEntry* __restrict__ xrec,
                                                       uint32_t* __restrict__ xg, uint32_t* __restrict__ xcnt,
                                                       const DevStatus* dc) {
  const int lane = threadIdx.x & 63;
  if (dc && (int64_t)dc->n_global < ngl) ngl = (int64_t)dc->n_global;  // read on the device
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < ngl; i += nwaves) {
    const uint32_t g = glist[i];
    const GroupRec G = groups[g];
    const unsigned long long base = gl_eoff[i];
    for (unsigned e = lane; e < G.count; e += 64) {
      const XRec r = xr[G.start + e];
      XEntry x;
      x.phi = (unsigned long long)i;  // the group's place in glist stands for its X free key in the table key
      x.v = r.v;
      xrec[base + e] = x;
      xg[base + e] = r.ystart;
      xcnt[base + e] = r.ycnt;
    }
  }
}

// ---------------------------------------------------------------------------
// Execute: per-group accumulation in LDS
// ---------------------------------------------------------------------------

// Ascending bitonic sort of a[0, n) in LDS (n a power of two, n <= blockDim.x),
// one element per thread; every thread of the block must call it.
__device__ __forceinline__ void bitonic_sort_lds(unsigned long long* a, unsigned n) {
  const unsigned i = threadIdx.x;
  for (unsigned k = 2; k <= n; k <<= 1) {
    for (unsigned j = k >> 1; j > 0; j >>= 1) {
      const unsigned ixj = i ^ j;
      if (i < n && ixj > i) {
        const unsigned long long x = a[i], y = a[ixj];
        if ((x > y) == ((i & k) == 0)) {
          a[i] = y;
          a[ixj] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Block class, one workgroup of BLOCK threads per group.  KIND 0 and 1: a
// Y free key too wide for a dense accumulator, an LDS hash of up to SLOTS
// slots (keys, then values: 8-byte words at random slots spread over twice
// the LDS banks that 16-byte {key, value} slots would use).  KIND 0 (2,048
// slots, four workgroups to a CU) walks the class list; KIND 1 (4,096
// slots and 512 threads, two to a CU, or 8,192 and 1,024, one) walks
// in_list, *in_count entries.  Each
// takes the groups whose bound fits its table (at most 70% of its slots)
// and appends the others to out_list (count in *out_count) for the next
// table size, so that no instance walks another's groups.  KIND 2: a dense Y
// free key and small groups (a few (group, slice) tiles' worth of
// products): the group's whole output row as a dense LDS array of `cells`
// doubles, cells starting at -0.0 and products added as x * y + 0.0, so a
// cell is an output exactly when it is no longer -0.0 (see the sliced
// tiles).  When the group has enough X entries for every wave and they
// average many products, each wave walks whole Y runs (coalesced, no
// search); otherwise the products are spread over all threads by a search
// over the staged entry offsets.  Then each wave counts the outputs in its
// share of the table, one atomic on the output cursor reserves the group's,
// and each wave writes its share.  The next group's list entry, record and
// product count are loaded one step per phase of the current group, so
// that their chain of dependent loads is not on the critical path.
template <int BLOCK, int SLOTS, int KIND>
__global__ __launch_bounds__(BLOCK) void k_group_block(GroupArgs a, const uint32_t* __restrict__ blist, int64_t nb,
                                                       const DevStatus* dc, unsigned cells,
                                                       const uint32_t* __restrict__ in_list,
                                                       const QueueCounter* in_count, uint32_t* out_list,
                                                       QueueCounter* out_count) {
  constexpr int kBChunk = BLOCK / 2;  // X entries staged at a time (LDS: the table dominates)
  constexpr unsigned long long kCap = (unsigned long long)SLOTS * 7 / 10;  // KIND 0, 1: the bound it takes
  if (in_list)
    nb = (int64_t)in_count->v;  // the groups the smaller table passed on
  else if (dc)
    nb = (int64_t)dc->n_block;  // the count read on the device
  const uint32_t* __restrict__ list = in_list ? in_list : blist;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  __shared__ unsigned long long s_off[kBChunk];
  __shared__ unsigned s_ys[kBChunk];
  __shared__ double s_v[kBChunk];
  __shared__ unsigned long long s_wave[BLOCK / 64 + 1];
  __shared__ unsigned long long s_base;
  unsigned long long* tkey = reinterpret_cast<unsigned long long*>(s_dyn);  // KIND 0, 1: SLOTS keys
  double* tval = reinterpret_cast<double*>(s_dyn + (size_t)SLOTS * 8);       // then SLOTS values
  double* acc = reinterpret_cast<double*>(s_dyn);                            // KIND 2: the dense row
  const unsigned tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr unsigned kWaves = BLOCK / 64;

  // XCD-aware order: workgroups go to the XCDs round-robin, so workgroup w
  // runs on XCD w % kXcds.  Each XCD takes one contiguous range of the list
  // (neighbouring groups share most of their contracting keys, hence Y
  // runs), and its workgroups stride through that range, so the groups in
  // flight on an XCD read the same Y runs through its L2.
  const unsigned nxcd = gridDim.x % kXcds == 0 ? kXcds : 1u;
  const unsigned xcd = blockIdx.x % nxcd, per_xcd = gridDim.x / nxcd;
  const int64_t lo = nb * xcd / nxcd, hi = nb * (xcd + 1) / nxcd;
  int64_t i = lo + blockIdx.x / nxcd;
  uint32_t gn = 0;
  GroupRec Gn{};
  unsigned long long bn = 0;
  if (i < hi) {
    gn = list[i];
    Gn = a.groups[gn];
    bn = a.eoff[Gn.start + Gn.count] - a.eoff[Gn.start];
  }
  for (; i < hi; i += per_xcd) {
    const uint32_t g = gn;
    const GroupRec G = Gn;
    const unsigned long long b = bn;
    const int64_t inext = i + per_xcd;
    const bool more = inext < hi;
    uint32_t gq = 0;
    if (more) gq = list[inext];  // the next group: its list entry now
    const unsigned long long d = b < a.ycells ? b : a.ycells;
    if (KIND != 2 && d > kCap) {  // for a larger table (uniform)
      if (tid == 0) {
        if (out_list)
          out_list[atomicAdd(&out_count->v, 1ull)] = g;
        else
          record_error(a.st, kErrInternal);  // past the class's cap
      }
      if (more) {
        gn = gq;
        Gn = a.groups[gq];
        bn = a.eoff[Gn.start + Gn.count] - a.eoff[Gn.start];
      }
      continue;
    }
    const unsigned tsize =
        KIND == 2 ? cells : (table_size_for(d, SLOTS) < (unsigned)BLOCK ? (unsigned)BLOCK : table_size_for(d, SLOTS));
    const unsigned tmask = tsize - 1;
    for (unsigned s = tid; s < tsize; s += BLOCK) {
      if constexpr (KIND == 2) {
        acc[s] = -0.0;
      } else {
        tkey[s] = kEmpty;
        tval[s] = 0.0;
      }
    }
    __syncthreads();
    GroupRec Gq{};
    if (more) Gq = a.groups[gq];  // the next group: its record

    auto accumulate = [&](unsigned long long key, double pv) {
      if constexpr (KIND == 2) {
        if (key < tsize)
          atomicAdd(&acc[key], pv + 0.0);
        else
          record_error(a.st, kErrInternal);
      } else {
        unsigned s = (unsigned)fmix64(key ^ a.seed) & tmask;
        for (unsigned probe = 0; probe <= tmask; ++probe) {
          const unsigned long long prev = atomicCAS(&tkey[s], (unsigned long long)kEmpty, key);
          if (prev == kEmpty || prev == key) {
            atomicAdd(&tval[s], pv);
            return;
          }
          s = (s + 1) & tmask;
        }
        record_error(a.st, kErrCapacity);
      }
    };

    if (b >= 32ull * G.count && G.count >= 2u * kWaves) {
      // entry-parallel.  Entries come in chunks of kBChunk, sorted by the
      // start of their Y run: every workgroup walks Y in the same order, so
      // the groups running at once on an XCD read the same Y runs together
      // and share them through its L2.  Each wave takes kEU entries at a time
      // (kEU independent loads in flight per lane); the waves of a workgroup
      // stay within kWaves * kEU consecutive entries of the sorted order.
      constexpr unsigned kEU = 4;
      for (unsigned base = 0; base < G.count; base += kBChunk) {
        const unsigned n = G.count - base < (unsigned)kBChunk ? G.count - base : (unsigned)kBChunk;
        unsigned long long key = ~0ull;
        if (tid < n) {
          XRec r = a.xr[G.start + base + tid];
          if ((unsigned long long)r.ystart + r.ycnt > (unsigned long long)a.ny) {
            record_error(a.st, kErrInternal);
            r.ycnt = 0;
          }
          s_ys[tid] = r.ycnt;
          s_v[tid] = r.v;
          key = ((unsigned long long)r.ystart << 32) | tid;
        }
        if (tid < (unsigned)kBChunk) s_off[tid] = key;
        __syncthreads();
        unsigned nsort = 2;
        while (nsort < n) nsort <<= 1;
        bitonic_sort_lds(s_off, nsort);
        for (unsigned r0 = wave; r0 < n; r0 += kWaves * kEU) {
          unsigned ys[kEU], cnt[kEU];
          double xv[kEU];
          unsigned m = 0;
#pragma unroll
          for (unsigned u = 0; u < kEU; ++u) {
            const unsigned rank = r0 + u * kWaves;
            cnt[u] = 0;
            ys[u] = 0;
            xv[u] = 0.0;
            if (rank < n) {
              const unsigned long long k = s_off[rank];
              const unsigned li = (unsigned)(k & 0xffffffffull);
              ys[u] = (unsigned)(k >> 32);
              cnt[u] = s_ys[li];
              xv[u] = s_v[li];
            }
            m = cnt[u] > m ? cnt[u] : m;
          }
          for (unsigned j = lane; j < m; j += 64) {
            YEntry ye[kEU];
#pragma unroll
            for (unsigned u = 0; u < kEU; ++u)
              if (j < cnt[u]) ye[u] = a.yg[ys[u] + j];
#pragma unroll
            for (unsigned u = 0; u < kEU; ++u)
              if (j < cnt[u]) accumulate(ye[u].phi, __dmul_rn(xv[u], ye[u].v));
          }
        }
        __syncthreads();
      }
    } else {
      // product-parallel over chunks of kBChunk entries: product q of the
      // chunk belongs to the last staged entry whose offset is <= q, found
      // by a branch-free search over the chunk's n entries
      for (unsigned base = 0; base < G.count; base += kBChunk) {
        const unsigned e = base + tid;
        const unsigned n = G.count - base < (unsigned)kBChunk ? G.count - base : (unsigned)kBChunk;
        unsigned long long c = 0;
        unsigned ys = 0;
        double v = 0.0;
        if (tid < (unsigned)kBChunk && e < G.count) {
          const XRec r = a.xr[G.start + e];
          c = r.ycnt;
          ys = r.ystart;
          v = r.v;
        }
        unsigned long long tot;
        const unsigned long long excl = block_excl_scan<BLOCK>(c, s_wave, &tot);
        if (tid < (unsigned)kBChunk) {
          s_off[tid] = excl;
          s_ys[tid] = ys;
          s_v[tid] = v;
        }
        __syncthreads();
        const int top = n > 1 ? 1 << (31 - __clz((int)n - 1)) : 0;  // the largest power of two below n
        for (unsigned long long q = tid; q < tot; q += BLOCK) {
          int lo = 0;
          for (int step = top; step > 0; step >>= 1) {
            const int c2 = lo + step;
            if (c2 < (int)n && s_off[c2] <= q) lo = c2;
          }
          const unsigned long long y = (unsigned long long)s_ys[lo] + (q - s_off[lo]);
          if (y >= (unsigned long long)a.ny) {
            record_error(a.st, kErrInternal);
            continue;
          }
          const YEntry ye = a.yg[y];
          accumulate(ye.phi, __dmul_rn(s_v[lo], ye.v));
        }
        __syncthreads();
      }
    }
    __syncthreads();
    unsigned long long bq = 0;
    if (more) bq = a.eoff[Gq.start + Gq.count] - a.eoff[Gq.start];  // the next group: its product count

    // count, reserve, write: wave w takes slots [w R, (w + 1) R)
    const unsigned R = tsize / kWaves;  // tsize >= BLOCK: a multiple of 64
    auto occupied = [&](unsigned s) {
      if constexpr (KIND == 2)
        return __double_as_longlong(acc[s]) != (long long)0x8000000000000000ull;
      else
        return tkey[s] != kEmpty;
    };
    unsigned n = 0;
    for (unsigned s0 = wave * R; s0 < (wave + 1) * R; s0 += 64) n += (unsigned)__popcll(__ballot(occupied(s0 + lane)));
    if (lane == 0) s_wave[wave] = n;
    __syncthreads();
    if (tid == 0) {
      unsigned long long run = 0;
      for (unsigned w = 0; w < kWaves; ++w) {
        const unsigned long long t = s_wave[w];
        s_wave[w] = run;
        run += t;
      }
      s_base = run ? atomicAdd(a.bout ? &a.bseg[G.phi >> a.bwx].cursor : &a.st->out_base, run) : 0ull;
    }
    __syncthreads();
    unsigned long long pos = s_base + s_wave[wave];
    for (unsigned s0 = wave * R; s0 < (wave + 1) * R; s0 += 64) {
      const unsigned s = s0 + lane;
      const bool occ = occupied(s);
      const unsigned long long m = __ballot(occ);
      if (occ) {
        const unsigned long long key = KIND == 2 ? (unsigned long long)s : tkey[s];
        const double val = KIND == 2 ? acc[s] : tval[s];
        const unsigned long long at = pos + lanes_below(m);
        if (a.bout)
          batch_store(a.bout, a.out_idx, a.out_val, a.bwx, (uint32_t)(G.phi >> a.bwx), at, G.phi, key, val, a.st);
        else if ((int64_t)at < a.out_cap)
          write_output(a, at, G.phi, key, val);
      }
      pos += (unsigned long long)__popcll(m);
    }
    __syncthreads();
    gn = gq;
    Gn = Gq;
    bn = bq;
  }
}

// Direct class: output q is product q of the direct list.  A product-space
// tile finds the groups it overlaps, stages their offsets, X records and free
// keys in LDS, and each lane maps its products to groups by binary search
// there.  Lanes take consecutive products, so the Y loads and the COO stores
// coalesce; each lane keeps kDItems Y loads in flight.
constexpr int kDBlock = 256;
constexpr int kDItemsOne = 8;    // products in flight per lane, one contraction
constexpr int kDItemsBatch = 5;  // and in a batch (the per-contraction decode takes registers)
constexpr int kDItemsSmall = 4;  // with the 1024-product tile option
constexpr int kDGroups = 1024;  // groups staged per tile; more fall back to global loads

// First direct group of every product-space tile: tile k's first product
// (k * tile) lies in group tfirst[k], the nonempty group that holds it, and
// tfirst[ntiles] = nd.  A thread per group writes the tiles starting in it.
// With dc the group and product counts are read on the device, and tiles
// past max_tiles (what tfirst holds) are an error.
__global__ __launch_bounds__(256) void k_direct_tiles(const unsigned long long* __restrict__ dpos, int64_t nd,
                                                      uint64_t tile, uint64_t ntiles, uint32_t* __restrict__ tfirst,
                                                      DevStatus* dc, uint64_t max_tiles) {
  if (dc) {
    nd = (int64_t)dc->n_direct;
    ntiles = (dc->direct_products + tile - 1) / tile;
    if (ntiles > max_tiles) {
      if (blockIdx.x == 0 && threadIdx.x == 0) record_error(dc, kErrCapacity);
      ntiles = max_tiles;
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = dpos[i], hi = dpos[i + 1];
    for (uint64_t k = (lo + tile - 1) / tile; k < ntiles && k * tile < hi; ++k) tfirst[k] = (uint32_t)i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) tfirst[ntiles] = (uint32_t)nd;
}

template <bool BATCH, int kDItems>
__global__ __launch_bounds__(kDBlock) void k_group_direct(GroupArgs a, const DRec* __restrict__ drec,
                                                          const unsigned long long* __restrict__ dpos, int64_t nd,
                                                          uint64_t nprod, const uint32_t* __restrict__ tfirst,
                                                          const DevStatus* dc, uint64_t max_tiles) {
  constexpr int kDTile = kDBlock * kDItems;
  if (dc) {  // counts read on the device; tfirst holds max_tiles tiles
    nd = (int64_t)dc->n_direct;
    nprod = dc->direct_products;
    if (nprod > max_tiles * (uint64_t)kDTile) nprod = max_tiles * (uint64_t)kDTile;
  }
  if (nd <= 0) return;
  __shared__ unsigned long long s_pos[kDGroups + 1];
  __shared__ unsigned long long s_phi[kDGroups];
  __shared__ double s_v[kDGroups];
  __shared__ unsigned s_ys[kDGroups];
  __shared__ unsigned long long s_sh[kDGroups];  // batch: the group's contraction's direct shift
  const uint64_t ntiles = (nprod + kDTile - 1) / kDTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t p0 = t * kDTile;
    const uint64_t p1 = (p0 + kDTile < nprod) ? p0 + kDTile : nprod;
    // the tile's groups: from the one holding p0 to the one holding p1 (or
    // the last); groups past p1 - 1 start at or after p1, so no product of
    // the tile maps to them
    const int64_t f0 = tfirst[t], nxt = tfirst[t + 1];
    const int64_t ilo = f0 < nd ? f0 : nd - 1;  // (clamped: indices stay inside the list)
    const int64_t ihi = nxt < ilo ? ilo : (nxt < nd ? nxt : nd - 1);
    const int64_t nloc = ihi - ilo + 1;
    const bool staged = nloc <= kDGroups;
    if (staged) {
      for (int64_t k = threadIdx.x; k < nloc; k += kDBlock) {
        const DRec d = drec[ilo + k];
        s_pos[k] = dpos[ilo + k];
        s_phi[k] = d.phi;
        s_v[k] = d.v;
        s_ys[k] = d.ystart;
        if constexpr (BATCH) s_sh[k] = a.bseg[d.phi >> a.bwx].dshift;
      }
      if (threadIdx.x == 0) s_pos[nloc] = dpos[ihi + 1];
    }
    __syncthreads();
    unsigned long long ys[kDItems], phx[kDItems], dsh[BATCH ? kDItems : 1];
    double xv[kDItems];
    YEntry ye[kDItems];
    // staged: the last staged group starting at or before each item's
    // product, by a branch-free binary search of all items in step (their
    // LDS reads interleave); `top` is the largest power of two below nloc
    int sg[kDItems];
#pragma unroll
    for (int it = 0; it < kDItems; ++it) sg[it] = 0;
    if (staged && nloc > 1) {
      const int top = 1 << (31 - __clz((int)nloc - 1));
      for (int step = top; step > 0; step >>= 1) {
#pragma unroll
        for (int it = 0; it < kDItems; ++it) {
          const uint64_t q = p0 + (uint64_t)it * kDBlock + threadIdx.x;
          const int c = sg[it] + step;
          if (c < (int)nloc && s_pos[c] <= q) sg[it] = c;
        }
      }
    }
#pragma unroll
    for (int it = 0; it < kDItems; ++it) {
      const uint64_t q = p0 + (uint64_t)it * kDBlock + threadIdx.x;
      ys[it] = ~0ull;
      if (q >= p1) continue;
      if (staged) {
        const int lo = sg[it];
        ys[it] = (unsigned long long)s_ys[lo] + (q - s_pos[lo]);
        phx[it] = s_phi[lo];
        xv[it] = s_v[lo];
        if constexpr (BATCH) dsh[it] = s_sh[lo];
      } else {
        const int64_t li = upper_bound_idx(dpos, ilo, ihi + 1, q) - 1;
        const DRec d = drec[li];
        ys[it] = (unsigned long long)d.ystart + (q - dpos[li]);
        phx[it] = d.phi;
        xv[it] = d.v;
        if constexpr (BATCH) dsh[it] = a.bseg[d.phi >> a.bwx].dshift;
      }
      if (ys[it] >= (unsigned long long)a.ny) {
        record_error(a.st, kErrInternal);
        ys[it] = ~0ull;
      }
    }
#pragma unroll
    for (int it = 0; it < kDItems; ++it)
      if (ys[it] != ~0ull) ye[it] = a.yg[ys[it]];
    if constexpr (BATCH) {
      // Usually every item of the wave belongs to one contraction (the list
      // is ordered by contraction): its output layout is then read once and
      // each output row stored for all items, as for one contraction;
      // otherwise each item is stored on its own.
      uint32_t bi = ~0u;
      bool one = true;
#pragma unroll
      for (int it = 0; it < kDItems; ++it) {
        if (ys[it] == ~0ull) continue;
        const uint32_t b = (uint32_t)(phx[it] >> a.bwx);
        if (bi == ~0u) bi = b;
        one &= b == bi;
      }
      const uint32_t b0 = __builtin_amdgcn_readfirstlane(bi);
      if (b0 != ~0u && __ballot(!one || (bi != ~0u && bi != b0)) == 0ull) {
        const BatchOut& d = a.bout[b0];
        const uint64_t xmask = low_mask(a.bwx);
        bool put[kDItems];
        unsigned long long pos[kDItems];
#pragma unroll
        for (int it = 0; it < kDItems; ++it) {
          pos[it] = p0 + (uint64_t)it * kDBlock + threadIdx.x - dsh[it];
          put[it] = ys[it] != ~0ull;
          if (put[it] && (int64_t)pos[it] >= d.cap) {
            record_error(a.st, kErrCapacity);
            put[it] = false;
          }
        }
        int32_t* rows = a.out_idx + d.idx_off;
        for (int m = 0; m < d.ux.n; ++m) {
          const uint32_t fd = d.ux.field[m];
          int32_t* dst = rows + (int64_t)(d.ux.row0 + m) * d.cap;
#pragma unroll
          for (int it = 0; it < kDItems; ++it)
            if (put[it]) __builtin_nontemporal_store(key_field(phx[it] & xmask, fd), dst + pos[it]);
        }
        for (int m = 0; m < d.uy.n; ++m) {
          const uint32_t fd = d.uy.field[m];
          int32_t* dst = rows + (int64_t)(d.uy.row0 + m) * d.cap;
#pragma unroll
          for (int it = 0; it < kDItems; ++it)
            if (put[it]) __builtin_nontemporal_store(key_field(ye[it].phi, fd), dst + pos[it]);
        }
#pragma unroll
        for (int it = 0; it < kDItems; ++it)
          if (put[it]) __builtin_nontemporal_store(__dmul_rn(xv[it], ye[it].v), a.out_val + d.val_off + pos[it]);
      } else {
#pragma unroll
        for (int it = 0; it < kDItems; ++it) {
          const uint64_t q = p0 + (uint64_t)it * kDBlock + threadIdx.x;
          if (ys[it] == ~0ull) continue;
          batch_store(a.bout, a.out_idx, a.out_val, a.bwx, (uint32_t)(phx[it] >> a.bwx), q - dsh[it], phx[it],
                      ye[it].phi, __dmul_rn(xv[it], ye[it].v), a.st);
        }
      }
    } else {
      // one output row (coordinate mode) at a time over all items: the
      // loops over modes stay rolled, so the kernel's code stays small
      const uint64_t q0 = p0 + threadIdx.x;
      bool put[kDItems];
#pragma unroll
      for (int it = 0; it < kDItems; ++it)
        put[it] = ys[it] != ~0ull && (int64_t)(q0 + (uint64_t)it * kDBlock) < a.out_cap;
      const int nx = a.ux.n, ny = a.uy.n;
      for (int d = 0; d < nx; ++d) {
        const uint32_t fd = a.ux.field[d];
        int32_t* dst = a.out_idx + (int64_t)(a.ux.row0 + d) * a.out_cap + (int64_t)q0;
#pragma unroll
        for (int it = 0; it < kDItems; ++it)
          if (put[it]) __builtin_nontemporal_store(key_field(phx[it], fd), dst + it * kDBlock);
      }
      for (int d = 0; d < ny; ++d) {
        const uint32_t fd = a.uy.field[d];
        int32_t* dst = a.out_idx + (int64_t)(a.uy.row0 + d) * a.out_cap + (int64_t)q0;
#pragma unroll
        for (int it = 0; it < kDItems; ++it)
          if (put[it]) __builtin_nontemporal_store(key_field(ye[it].phi, fd), dst + it * kDBlock);
      }
#pragma unroll
      for (int it = 0; it < kDItems; ++it)
        if (put[it]) __builtin_nontemporal_store(__dmul_rn(xv[it], ye[it].v), a.out_val + q0 + it * kDBlock);
    }
    __syncthreads();
  }
}

// SORT: sorts each Y run (a Y group's entries in the grouped array) of
// 2..1024 entries by Y free key, one workgroup per Y table slot.  Order
// within a run is free (section 4.1.3); sorted runs let the lanes of a wave
// that walk a run hit consecutive dense accumulator cells, i.e. distinct LDS
// banks.  Either way (dense Y free keys only) it writes the compact copy of
// grouped Y and finds repeated Y coordinates (two entries of one run with
// the same free key) with a per-run bitmap of the 2^kDenseBits keys, which
// the direct class needs to know about.  Without SORT it serves small
// tables only (a few slots per workgroup); larger ones take k_y_compact and
// k_y_repeats.
// With yso, runs are sorted by counting over the keys 0 ..
// slice_cells * kSlices - 1 (those the slices cover), else by a bitonic
// sort.  With yso, the compact copy of every run is also cut into
// kSlices slices of the Y free key space (key / slice_cells, the last
// slice taking every larger key): a sorted run
// is cut where the slice changes, a longer run is placed slice by slice (in
// no order within a slice).  yso[slot * (kSlices + 1) + s] receives the
// position where slice s of the slot's run begins (entry kSlices: the run's
// end), and runslot[start of the run] the slot.
template <bool SORT>
__global__ __launch_bounds__(kBBlock) void k_sort_y_runs(const YSlot* __restrict__ ytab, int64_t nslots,
                                                         YEntry* __restrict__ yg, int64_t ny,
                                                         uint16_t* __restrict__ ykey16, double* __restrict__ yval,
                                                         unsigned* __restrict__ colbits, uint32_t* __restrict__ yso,
                                                         uint32_t* __restrict__ runslot, unsigned slice_cells,
                                                         unsigned key_cells, DevStatus* st) {
  __shared__ unsigned long long s_key[kBBlock];
  __shared__ YEntry s_ent[kBBlock];
  constexpr unsigned kSeenWords = (1u << kDenseBits) / 32;
  __shared__ unsigned s_seen[kSeenWords];
  __shared__ unsigned s_cells[kSeenWords];  // cells that occur in this workgroup's runs
  __shared__ unsigned s_slice[kSlices];     // entries per slice, then the slices' placement cursors
  for (unsigned w = threadIdx.x; w < kSeenWords; w += kBBlock) s_cells[w] = 0u;
  auto seen_before = [&](unsigned long long phi) {
    const unsigned c = (unsigned)phi & ((1u << kDenseBits) - 1u), bit = 1u << (c & 31);
    if (colbits) atomicOr(&s_cells[c >> 5], bit);
    return (atomicOr(&s_seen[c >> 5], bit) & bit) != 0u;
  };
  auto slice_of = [&](unsigned long long phi) {
    const unsigned q = (unsigned)phi / slice_cells;
    return q < (unsigned)kSlices - 1u ? q : (unsigned)kSlices - 1u;
  };
  for (int64_t slot = blockIdx.x; slot < nslots; slot += gridDim.x) {
    const YSlot t = ytab[slot];
    if (t.key == kEmpty || t.count == 0 || (unsigned long long)t.start + t.count > (unsigned long long)ny)
      continue;  // uniform across the block
    const unsigned n = t.count, tid = threadIdx.x;
    uint32_t* so = yso ? yso + (size_t)slot * (kSlices + 1) : nullptr;
    if (so && tid == 0) runslot[t.start] = (uint32_t)slot;
    for (unsigned w = tid; w < kSeenWords; w += kBBlock) s_seen[w] = 0u;
    if (tid < kSlices) s_slice[tid] = 0u;
    __syncthreads();
    if (!SORT || n > (unsigned)kBBlock) {  // too long to sort here: copied as is, or slice by slice
      if (so) {
        for (unsigned j = tid; j < n; j += kBBlock)
          atomicAdd(&s_slice[slice_of(yg[t.start + j].phi)], 1u);
        __syncthreads();
        if (tid == 0) {
          unsigned run = 0;
          for (unsigned q = 0; q < kSlices; ++q) {
            const unsigned c = s_slice[q];
            so[q] = t.start + run;
            s_slice[q] = run;
            run += c;
          }
          so[kSlices] = t.start + n;
        }
        __syncthreads();
      }
      for (unsigned j = tid; j < n; j += kBBlock) {
        const YEntry e = yg[t.start + j];
        if (seen_before(e.phi)) st->ydup = 1u;
        const unsigned at = so ? atomicAdd(&s_slice[slice_of(e.phi)], 1u) : j;
        ykey16[t.start + at] = (uint16_t)e.phi;
        yval[t.start + at] = e.v;
      }
      __syncthreads();
      continue;
    }
    if (key_cells) {
      // a counting sort over the keys 0..key_cells - 1 (a larger key, from
      // a coordinate past its mode's length, goes in the last bin): a
      // histogram, its scan, and each entry placed at its bin's cursor;
      // s_key[place] = (key << 11) | entry, as the bitonic sort leaves it
      __shared__ unsigned s_cnt[1u << kDenseBits];
      __shared__ unsigned long long s_wave[kBBlock / 64 + 1];
      for (unsigned c = tid; c < key_cells; c += kBBlock) s_cnt[c] = 0u;
      __syncthreads();
      unsigned bin = 0;
      if (tid < n) {
        s_ent[tid] = yg[t.start + tid];
        if (seen_before(s_ent[tid].phi)) st->ydup = 1u;
        bin = s_ent[tid].phi < key_cells ? (unsigned)s_ent[tid].phi : key_cells - 1u;
        atomicAdd(&s_cnt[bin], 1u);
      }
      __syncthreads();
      const unsigned per = (key_cells + kBBlock - 1u) / kBBlock, c0 = tid * per;
      const unsigned c1 = c0 + per < key_cells ? c0 + per : key_cells;
      unsigned long long mine = 0;
      for (unsigned c = c0; c < c1; ++c) mine += s_cnt[c];
      unsigned long long tot;
      unsigned long long run = block_excl_scan<kBBlock>(mine, s_wave, &tot);
      for (unsigned c = c0; c < c1; ++c) {
        const unsigned v = s_cnt[c];
        s_cnt[c] = (unsigned)run;
        run += v;
      }
      __syncthreads();
      if (tid < n) {
        const unsigned at = atomicAdd(&s_cnt[bin], 1u);
        if (at < n) s_key[at] = (s_ent[tid].phi << 11) | tid;
      }
      __syncthreads();
    } else {
      unsigned long long key = ~0ull;
      if (tid < n) {
        s_ent[tid] = yg[t.start + tid];
        if (seen_before(s_ent[tid].phi)) st->ydup = 1u;
        key = (s_ent[tid].phi << 11) | tid;  // phi has <= kDenseBits bits here; tid < 2048
      }
      s_key[tid] = key;
      __syncthreads();
      unsigned nsort = 2;
      while (nsort < n) nsort <<= 1;
      bitonic_sort_lds(s_key, nsort);
    }
    if (tid < n) {
      const YEntry e = s_ent[(unsigned)(s_key[tid] & 2047ull)];
      yg[t.start + tid] = e;
      ykey16[t.start + tid] = (uint16_t)e.phi;
      yval[t.start + tid] = e.v;
      if (so) {  // slice boundaries: where the (sorted) slice index changes
        const unsigned q = slice_of(e.phi);
        const unsigned qp = tid == 0 ? 0u : slice_of(s_key[tid - 1] >> 11);
        for (unsigned b = (tid == 0 ? 0u : qp + 1u); b <= q; ++b) so[b] = t.start + tid;
        if (tid == n - 1)
          for (unsigned b = q + 1u; b <= (unsigned)kSlices; ++b) so[b] = t.start + n;
      }
    }
    __syncthreads();
  }
  if (colbits) {
    __syncthreads();
    for (unsigned w = threadIdx.x; w < kSeenWords; w += kBBlock)
      if (s_cells[w]) atomicOr(&colbits[w], s_cells[w]);
  }
}



// Dense Y free keys, at plan time: the compact copy of grouped Y (16-bit
// free key, value), entry by entry, and the cells that occur (colbits,
// optional; each workgroup gathers its entries' cells in LDS first).
__global__ __launch_bounds__(256) void k_y_compact(const YEntry* __restrict__ yg, int64_t ny,
                                                   uint16_t* __restrict__ ykey16, double* __restrict__ yval,
                                                   unsigned* __restrict__ colbits, unsigned* __restrict__ nlong) {
  constexpr unsigned kWords = (1u << kDenseBits) / 32;
  __shared__ unsigned s_cells[kWords];
  if (blockIdx.x == 0 && threadIdx.x == 0) *nlong = 0u;  // the long-run list of the repeat check
  for (unsigned w = threadIdx.x; w < kWords; w += blockDim.x) s_cells[w] = 0u;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < ny; p += (int64_t)gridDim.x * blockDim.x) {
    const YEntry e = yg[p];
    ykey16[p] = (uint16_t)e.phi;
    yval[p] = e.v;
    if (colbits) {
      const unsigned c = (unsigned)e.phi & ((1u << kDenseBits) - 1u);
      atomicOr(&s_cells[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
  if (colbits)
    for (unsigned w = threadIdx.x; w < kWords; w += blockDim.x)
      if (s_cells[w]) atomicOr(&colbits[w], s_cells[w]);
}

// Dense Y free keys: repeated Y coordinates, i.e. two entries of one run (Y
// group) with the same free key, which the direct class must know about.
// Each wave reads 64 Y table slots at a time and checks their runs of two
// to kLongRun entries one after another against a bitmap of the
// 2^kDenseBits keys in its own LDS (cleared per run; one wave's LDS
// operations complete in order).  Runs of one entry cannot repeat and cost
// nothing but their slot's read; longer runs go to the list `lng` (count
// *nlong, room for cap) for k_y_repeats_long, a workgroup per run, so that
// a few long runs do not hold a few waves for long.
constexpr unsigned kLongRun = 512;

__global__ __launch_bounds__(256) void k_y_repeats(const YSlot* __restrict__ ytab, int64_t nslots,
                                                   const YEntry* __restrict__ yg, int64_t ny, DevStatus* st,
                                                   uint32_t* __restrict__ lng, unsigned cap,
                                                   unsigned* __restrict__ nlong) {
  constexpr unsigned kWords = (1u << kDenseBits) / 32;
  __shared__ unsigned s_seen[4][kWords];
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  unsigned* seen = s_seen[wave];
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  bool dup = false;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64; base < nslots; base += nwaves * 64) {
    const int64_t slot = base + lane;
    unsigned start = 0u, n = 0u;
    if (slot < nslots) {
      const YSlot t = ytab[slot];
      if (t.key != kEmpty && t.count >= 2u && (unsigned long long)t.start + t.count <= (unsigned long long)ny) {
        start = t.start;
        n = t.count;
      }
    }
    for (unsigned long long m = __ballot(n != 0u); m; m &= m - 1ull) {
      const int r = __ffsll((long long)m) - 1;
      const unsigned rs = (unsigned)__builtin_amdgcn_readlane((int)start, r);
      const unsigned rn = (unsigned)__builtin_amdgcn_readlane((int)n, r);
      if (rn > kLongRun) {
        if (lane == 0) {
          const unsigned k = atomicAdd(nlong, 1u);
          if (k < cap)
            lng[k] = (uint32_t)(base + r);
          else
            record_error(st, kErrInternal);  // more long runs than entries allow
        }
        continue;
      }
      for (unsigned w = lane; w < kWords; w += 64) seen[w] = 0u;
      wave_lds_fence();
      for (unsigned j = lane; j < rn; j += 64) {
        const unsigned c = (unsigned)yg[rs + j].phi & ((1u << kDenseBits) - 1u), bit = 1u << (c & 31);
        if (atomicOr(&seen[c >> 5], bit) & bit) dup = true;
      }
      wave_lds_fence();
    }
  }
  if (__ballot(dup) && lane == 0) st->ydup = 1u;
}

// The long runs of k_y_repeats, one workgroup per run, with the bitmap in
// the workgroup's LDS.
__global__ __launch_bounds__(256) void k_y_repeats_long(const YSlot* __restrict__ ytab, const YEntry* __restrict__ yg,
                                                        DevStatus* st, const uint32_t* __restrict__ lng,
                                                        const unsigned* __restrict__ nlong) {
  constexpr unsigned kWords = (1u << kDenseBits) / 32;
  __shared__ unsigned s_seen[kWords];
  const unsigned nl = *nlong;
  bool dup = false;
  for (unsigned i = blockIdx.x; i < nl; i += gridDim.x) {
    const YSlot t = ytab[lng[i]];  // a run k_y_repeats checked: start + count <= ny
    for (unsigned w = threadIdx.x; w < kWords; w += blockDim.x) s_seen[w] = 0u;
    __syncthreads();
    for (unsigned j = threadIdx.x; j < t.count; j += blockDim.x) {
      const unsigned c = (unsigned)yg[t.start + j].phi & ((1u << kDenseBits) - 1u), bit = 1u << (c & 31);
      if (atomicOr(&s_seen[c >> 5], bit) & bit) dup = true;
    }
    __syncthreads();
  }
  if (__ballot(dup) && (threadIdx.x & 63u) == 0) st->ydup = 1u;
}

__global__ void k_finalize(int64_t* out_nnz, int64_t out_cap, DevStatus* st) {
  const unsigned long long total = st->out_base;
  uint32_t err = st->err;
  if ((int64_t)total > out_cap) {
    err |= kErrCapacity;
    atomicOr(&st->err, kErrCapacity);
  }
  *out_nnz = err ? -(int64_t)status_of(err) : (int64_t)total;
}

// Start of an execution: no error yet; outputs placed by the output cursor
// follow the direct class's (which take [0, direct products)); the work
// queues start over.
__global__ void k_reset_status(DevStatus* st, LdsQueue* q) {
  st->err = 0u;
  st->out_base = st->direct_products;
  if (q) {
    for (int s = 0; s < kSlices; ++s) q->next_tile[s].v = q->next_fill[s].v = 0ull;
    q->n_defer.v = q->n_defer2.v = 0ull;
  }
}

// Inspection: X groups -> (free coordinates, entry count, product count).
__global__ void k_x_groups(const GroupRec* __restrict__ groups, int64_t ng, const unsigned long long* __restrict__ eoff,
                           KeyUnpack ku, int32_t* __restrict__ coords, int64_t* __restrict__ counts,
                           int64_t* __restrict__ products, int64_t cap) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng && g < cap;
       g += (int64_t)gridDim.x * blockDim.x) {
    const GroupRec G = groups[g];
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m)
      if (m < ku.n) coords[(int64_t)m * cap + g] = key_field(G.phi, ku.field[m]);
    counts[g] = G.count;
    products[g] = (int64_t)(eoff[G.start + G.count] - eoff[G.start]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_scan_x_table(YSlot* tab, int64_t nslots, GroupRec* groups, int64_t cap, bool run_end,
                               void* tile_sums, DevStatus* st, hipStream_t stream) {
  return device_scan(XTableScanOp{tab, groups, run_end, (unsigned long long)cap, st}, nslots, tile_sums,
                     FinXGroups{st}, stream);
}

hipError_t launch_x_table32(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                            unsigned long long* xtab, TabGeom xg, int32_t max_probe_x, GroupRec* groups,
                            const YSlot* ytab, TabGeom yg, int32_t max_probe_y, uint64_t seed, XRec* xr,
                            void* tile_sums, DevStatus* st, int num_cus, hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  if (xg.reg || xg.ident) return hipErrorInvalidValue;
  const int64_t nslots = (int64_t)xg.mask + 1;
  hipError_t e = launch_fill_keys(xtab, nslots, stream);
  if (e != hipSuccess) return e;
  k_key_count32<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(xidx, nnz, kf, xtab, xg, seed, max_probe_x, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_scan(XTable32ScanOp{xtab, groups, (unsigned long long)nnz, st}, nslots, tile_sums, FinXGroups{st},
                  stream);
  if (e != hipSuccess) return e;
  k_x_scatter32<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(xidx, xval, nnz, kf, kc, b, xtab, xg, max_probe_x,
                                                                  ytab, yg, max_probe_y, seed, xr, st);
  return hipGetLastError();
}

hipError_t launch_x_scatter(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                            YSlot* xtab, TabGeom xg, int32_t max_probe_x, const YSlot* ytab, TabGeom yg,
                            int32_t max_probe_y, uint64_t seed, XRec* xr, DevStatus* st, int num_cus,
                            hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  k_x_scatter<<<grid_for(nnz, 256, num_cus), 256, 0, stream>>>(xidx, xval, nnz, kf, kc, b, xtab, xg, max_probe_x,
                                                                ytab, yg, max_probe_y, seed, xr, st);
  return hipGetLastError();
}

hipError_t launch_x_scatter_agg(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc,
                                Bounds b, const YSlot* xtab, unsigned nslots, const unsigned* choff, const YSlot* ytab,
                                TabGeom yg, int32_t max_probe_y, uint64_t seed, XRec* xr, DevStatus* st,
                                hipStream_t stream) {
  if (nnz <= 0) return hipSuccess;
  const unsigned grid = (unsigned)agg_chunks(nnz);
  k_x_scatter_agg<<<grid, kAggBlock, (size_t)nslots * 8, stream>>>(xidx, xval, nnz, kf, kc, b, xtab, nslots, choff,
                                                                    ytab, yg, max_probe_y, seed, xr, st);
  return hipGetLastError();
}

hipError_t launch_scan_entries(const XRec* xr, int64_t n, unsigned long long* eoff, void* tile_sums, DevStatus* st,
                               hipStream_t stream) {
  return device_scan(EntryScanOp{xr, eoff}, n, tile_sums, FinEntries{eoff + n, st}, stream);
}

hipError_t launch_classify(const GroupRec* groups, int64_t max_groups, const unsigned long long* eoff,
                           uint64_t ycells, int32_t dense, uint32_t* dlist, uint32_t* wlist, uint32_t* blist,
                           uint32_t* glist, unsigned long long* dpos, void* tile_sums, DevStatus* st,
                           hipStream_t stream, int32_t block_cap, const XRec* xr, DRec* drec) {
  if (!xr || !drec) return hipErrorInvalidValue;
  const unsigned long long cap = block_cap > 0 && block_cap < kBlockCap ? (unsigned long long)block_cap : kBlockCap;
  return device_scan(ClassifyOp{groups, eoff, st, ycells, dense, dlist, wlist, blist, glist, dpos, cap, xr, drec},
                     max_groups, tile_sums, FinClassify{st}, stream);
}

hipError_t launch_scan_direct(int64_t max_groups, unsigned long long* dpos, void* tile_sums, DevStatus* st,
                              hipStream_t stream) {
  return device_scan(DirectScanOp{dpos, st}, max_groups, tile_sums, FinDirect{dpos, st}, stream);
}

hipError_t launch_scan_global_entries(const GroupRec* groups, const uint32_t* glist, int64_t ngl,
                                      unsigned long long* gl_eoff, void* tile_sums, DevStatus* st,
                                      hipStream_t stream) {
  return device_scan(GlobalEntryScanOp{groups, glist, gl_eoff, st}, ngl, tile_sums, FinGlobalEntries{st}, stream);
}

hipError_t launch_gather_global(const GroupRec* groups, const uint32_t* glist, int64_t ngl,
                                const unsigned long long* gl_eoff, const XRec* xr, XEntry* xrec, uint32_t* xg,
                                uint32_t* xcnt, int num_cus, hipStream_t stream, const DevStatus* dc) {
  if (ngl <= 0) return hipSuccess;
  k_gather_global<<<grid_for(ngl * 64, 256, num_cus), 256, 0, stream>>>(groups, glist, ngl, gl_eoff, xr, xrec, xg,
                                                                         xcnt, dc);
  return hipGetLastError();
}


// Dynamic LDS of the block class: a hash of 16-byte slots, or a dense row.
hipError_t prepare_group_block() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group_block<kBMidBlock, kBlockSlots, 1>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kBlockSlots * 16);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group_block<kBBlock, kBlockXlSlots, 1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kBlockXlSlots * 16);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group_block<kBSmallBlock, kBlockSmallSlots, 0>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kBlockSmallSlots * 16);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_group_block<kBSmallBlock, 0, 2>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (1 << kDenseBits) * 8);
  return e;
}

// Hashed: the small-table instance walks the list, four workgroups of 256
// threads per CU, and passes the groups its table cannot hold to the
// large-table instance, two workgroups of 512 per CU (LDS and registers
// both allow two), which passes its own misfits to the largest table, one
// workgroup of 1024 per CU; each reads its count on the device.  Dense (cells > 0): 256-thread workgroups
// with a row of cells.
hipError_t launch_group_block(const GroupArgs& a, const uint32_t* blist, int64_t nb, int num_cus,
                              hipStream_t stream, const DevStatus* dc, unsigned cells, uint32_t* defer, LdsQueue* q) {
  if (nb <= 0) return hipSuccess;
  if (cells) {
    if (cells < 64u || (cells & (cells - 1u)) || cells > (1u << kDenseBits)) return hipErrorInvalidValue;
    unsigned grid = grid_for(nb, 1, num_cus, std::min(8, std::max(1, (160 << 10) / (int)(cells * 8 + (8 << 10)))));
    if (grid >= kXcds) grid -= grid % kXcds;
    k_group_block<kBSmallBlock, 0, 2><<<grid, kBSmallBlock, cells * 8, stream>>>(a, blist, nb, dc, cells, nullptr,
                                                                                 nullptr, nullptr, nullptr);
    return hipGetLastError();
  }
  if (!defer || !q) return hipErrorInvalidValue;
  uint32_t* defer2 = defer + nb;
  unsigned grid = grid_for(nb, 1, num_cus, 4);
  if (grid >= kXcds) grid -= grid % kXcds;
  k_group_block<kBSmallBlock, kBlockSmallSlots, 0><<<grid, kBSmallBlock, kBlockSmallSlots * 16, stream>>>(
      a, blist, nb, dc, 0u, nullptr, nullptr, defer, &q->n_defer);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  grid = grid_for(nb, 1, num_cus, 2);
  if (grid >= kXcds) grid -= grid % kXcds;
  k_group_block<kBMidBlock, kBlockSlots, 1><<<grid, kBMidBlock, kBlockSlots * 16, stream>>>(
      a, blist, nb, dc, 0u, defer, &q->n_defer, defer2, &q->n_defer2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  grid = grid_for(nb, 1, num_cus, 1);
  if (grid >= kXcds) grid -= grid % kXcds;
  k_group_block<kBBlock, kBlockXlSlots, 1><<<grid, kBBlock, kBlockXlSlots * 16, stream>>>(
      a, blist, nb, dc, 0u, defer2, &q->n_defer2, nullptr, nullptr);
  return hipGetLastError();
}

int64_t direct_tile_bound(uint64_t nprod) {
  const uint64_t tile = (uint64_t)kDBlock * kDItemsSmall;  // the smallest tile
  return (int64_t)((nprod + tile - 1) / tile) + 1;
}

hipError_t launch_group_direct(const GroupArgs& a, const DRec* drec, const unsigned long long* dpos, int64_t nd,
                               uint64_t nprod, uint32_t* tfirst, int num_cus, hipStream_t stream, int tile_products,
                               DevStatus* dc, int64_t tfirst_slots) {
  if (nd <= 0 || nprod == 0) return hipSuccess;
  if (nd >= (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  const bool small = tile_products == (int)(kDBlock * kDItemsSmall);
  const int items = small ? kDItemsSmall : (a.bout ? kDItemsBatch : kDItemsOne);
  const uint64_t tile = (uint64_t)kDBlock * items, tiles = (nprod + tile - 1) / tile;
  const uint64_t max_tiles = dc ? (uint64_t)(tfirst_slots > 1 ? tfirst_slots - 1 : 0) : tiles;
  k_direct_tiles<<<grid_for(nd, 256, num_cus, 8), 256, 0, stream>>>(dpos, nd, tile, tiles, tfirst, dc, max_tiles);
  uint64_t g = (uint64_t)num_cus * 8;
  if (g > tiles) g = tiles;
#define D_LAUNCH(B, I) \
  k_group_direct<B, I><<<dim3((unsigned)g), kDBlock, 0, stream>>>(a, drec, dpos, nd, nprod, tfirst, dc, max_tiles)
  if (a.bout && small)
    D_LAUNCH(true, kDItemsSmall);
  else if (a.bout)
    D_LAUNCH(true, kDItemsBatch);
  else if (small)
    D_LAUNCH(false, kDItemsSmall);
  else
    D_LAUNCH(false, kDItemsOne);
#undef D_LAUNCH
  return hipGetLastError();
}


int64_t y_long_run_slots(int64_t ny) { return ny / kLongRun + 2; }

// Y tables of at most this many slots take the one-launch copy without
// sorting: with a workgroup per slot each workgroup visits a few slots,
// where the three launches of the larger tables' path would cost more.
constexpr int64_t kSmallYTable = 8192;

hipError_t launch_sort_y_runs(const YSlot* ytab, int64_t nslots, YEntry* yg, int64_t ny, uint16_t* ykey16,
                              double* yval, unsigned* colbits, DevStatus* st, bool sort, int num_cus,
                              hipStream_t stream, uint32_t* yso, uint32_t* runslot, unsigned slice_cells,
                              uint32_t* ylong) {
  if (nslots <= 0 || ny <= 0) return hipSuccess;
  if (yso && !sort) return hipErrorInvalidValue;
  if (yso && (slice_cells == 0u || slice_cells % 64u || slice_cells * kSlices > (1u << kDenseBits)))
    return hipErrorInvalidValue;
  const int64_t grid = nslots < (int64_t)num_cus * 2 ? nslots : (int64_t)num_cus * 2;
  if (sort) {
    k_sort_y_runs<true><<<dim3((unsigned)grid), kBBlock, 0, stream>>>(ytab, nslots, yg, ny, ykey16, yval, colbits,
                                                                       yso, runslot, yso ? slice_cells : 1u,
                                                                       yso ? slice_cells * kSlices : 0u, st);
    return hipGetLastError();
  }
  if (nslots <= kSmallYTable) {  // a few slots per workgroup: one launch
    k_sort_y_runs<false><<<dim3((unsigned)grid), kBBlock, 0, stream>>>(ytab, nslots, yg, ny, ykey16, yval, colbits,
                                                                        nullptr, nullptr, 1u, 0u, st);
    return hipGetLastError();
  }
  // a larger table, mostly short runs or empty slots: an elementwise copy,
  // and the repeat check by waves over the slots, long runs by workgroups
  if (!ylong) return hipErrorInvalidValue;
  const unsigned cap = (unsigned)(ny / kLongRun + 1);
  unsigned* nlong = ylong + cap;
  k_y_compact<<<grid_for(ny, 256, num_cus, 8), 256, 0, stream>>>(yg, ny, ykey16, yval, colbits, nlong);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_y_repeats<<<grid_for((nslots + 255) / 256, 1, num_cus, 8), 256, 0, stream>>>(ytab, nslots, yg, ny, st, ylong, cap,
                                                                                 nlong);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_y_repeats_long<<<grid_for(ny / kLongRun + 1, 1, num_cus, 4), 256, 0, stream>>>(ytab, yg, st, ylong, nlong);
  return hipGetLastError();
}

hipError_t launch_finalize(int64_t* out_nnz, int64_t out_cap, DevStatus* st, hipStream_t stream) {
  k_finalize<<<1, 1, 0, stream>>>(out_nnz, out_cap, st);
  return hipGetLastError();
}

hipError_t launch_reset_status(DevStatus* st, LdsQueue* q, hipStream_t stream) {
  k_reset_status<<<1, 1, 0, stream>>>(st, q);
  return hipGetLastError();
}

hipError_t launch_x_groups(const GroupRec* groups, int64_t ng, const unsigned long long* eoff, KeyUnpack ku,
                           int32_t* coords, int64_t* counts, int64_t* products, int64_t cap, hipStream_t stream) {
  if (ng <= 0) return hipSuccess;
  int64_t g = (ng + 255) / 256;
  if (g > 65536) g = 65536;
  k_x_groups<<<dim3((unsigned)g), 256, 0, stream>>>(groups, ng, eoff, ku, coords, counts, products, cap);
  return hipGetLastError();
}

}  // namespace sptc
