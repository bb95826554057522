// Host runtime of the C ABI in include/sptc.h: argument validation, key
// layout, table sizing, workspace management and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sptc.h"
#include "sptc_internal.hpp"
#include "xpart.hpp"

using namespace sptc;

namespace {

thread_local std::string g_last_error;
// The last failed plan on this thread gave up on a stalled stream (its
// callers then release memory in stream order without waiting).
thread_local bool g_stalled = false;

sptc_status fail(sptc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

sptc_status hip_fail(hipError_t e, const char* what) {
  return fail(SPTC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                             \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

int32_t bits_for(int64_t d) {
  if (d <= 1) return 0;
  return 64 - __builtin_clzll((unsigned long long)(d - 1));
}

// Saturating product of mode lengths.
int64_t sat_prod(const int64_t* d, const std::vector<int32_t>& modes) {
  const int64_t cap = (int64_t)1 << 62;
  int64_t p = 1;
  for (int32_t m : modes) {
    if (p > cap / std::max<int64_t>(d[m], 1)) return cap;
    p *= d[m];
  }
  return p;
}

int64_t pow2_at_least(double x) {
  int64_t c = 2;
  while ((double)c < x && c < ((int64_t)1 << 46)) c <<= 1;
  return c;
}

struct DeviceInfo {
  int num_cus = 0;
  bool pool_configured = false;
};

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

sptc_status device_info(int dev, DeviceInfo** out) {
  if (dev < 0 || dev >= 64) return fail(SPTC_ERR_HIP, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_dev_mu);
  DeviceInfo& d = g_dev[dev];
  if (d.num_cus == 0) {
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    d.num_cus = std::max(cus, 1);
  }
  *out = &d;
  return SPTC_OK;
}

sptc_status configure_pool(int dev, DeviceInfo* d) {
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if (d->pool_configured) return SPTC_OK;
  hipMemPool_t pool;
  HIP_TRY(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t threshold = ~0ull;  // keep freed blocks cached in the pool
  HIP_TRY(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold));
  d->pool_configured = true;
  return SPTC_OK;
}

// Slabs given back by released plans and batches, per device, kept for the
// next ones: after a warm-up, planning makes no pool call at all (growing
// the stream-ordered pool inside hipMallocAsync has stalled single calls for
// seconds, and each call costs microseconds).  A slab carries an event
// recorded on the releasing stream; a reuse on another stream waits for it.
struct CachedSlab {
  void* p;
  size_t bytes;
  hipEvent_t ready;
};
std::mutex g_cache_mu;
std::multimap<size_t, CachedSlab> g_cache[64];
size_t g_cached_bytes[64];

// A cached slab of at least `bytes` (and at most twice that), or p = NULL.
CachedSlab cache_take(int dev, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto& c = g_cache[dev];
  auto it = c.lower_bound(bytes);
  if (it == c.end() || it->first > 2 * bytes) return CachedSlab{nullptr, 0, nullptr};
  CachedSlab sl = it->second;
  c.erase(it);
  g_cached_bytes[dev] -= sl.bytes;
  return sl;
}

void cache_put(int dev, const CachedSlab& sl) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_cache[dev].emplace(sl.bytes, sl);
  g_cached_bytes[dev] += sl.bytes;
}

// Frees cached slabs of `dev` (largest first) until at most keep_bytes stay.
sptc_status cache_trim(int dev, size_t keep_bytes) {
  std::vector<CachedSlab> out;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto& c = g_cache[dev];
    while (!c.empty() && g_cached_bytes[dev] > keep_bytes) {
      auto it = std::prev(c.end());
      out.push_back(it->second);
      g_cached_bytes[dev] -= it->first;
      c.erase(it);
    }
  }
  for (const CachedSlab& sl : out) {
    if (sl.ready) {
      HIP_TRY(hipEventSynchronize(sl.ready));
      HIP_TRY(hipEventDestroy(sl.ready));
    }
    HIP_TRY(hipFreeAsync(sl.p, nullptr));  // back to the pool (the slab is idle)
  }
  return SPTC_OK;
}

}  // namespace

// Device memory owned by a plan or batch: through the caller's allocator
// (one call per buffer), or slabs from the device (the slab cache above,
// else the stream-ordered pool).  Buffers are carved out of the slabs -- a
// buffer above the current slab's room opens a new one of max(buffer,
// kSlabMin doubling up to kSlabMax) -- so a plan holds a handful of slabs,
// not one allocation per buffer.
struct Workspace {
  struct Buf {
    void* p;
    size_t bytes;
    hipEvent_t ready;  // slabs: the event they came with from the cache, if any
  };
  static constexpr size_t kSlabMin = (size_t)8 << 20;
  static constexpr size_t kSlabMax = (size_t)256 << 20;
  hipStream_t stream = nullptr;
  bool has_alloc = false;
  sptc_allocator alloc{};
  int slab_device = -1;
  std::vector<Buf> bufs;  // caller's buffers, or the slabs
  size_t slab_used = 0, slab_next = kSlabMin;
  int64_t workspace = 0;  // bytes held

  sptc_status allocate(size_t bytes, void** out) {
    bytes = std::max<size_t>(bytes, 16);
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (has_alloc) {
      p = alloc.alloc(bytes, stream, alloc.ctx);
      if (!p) return fail(SPTC_ERR_OUT_OF_MEMORY, "allocator returned NULL for %zu bytes", bytes);
      bufs.push_back({p, bytes, nullptr});
      workspace += (int64_t)bytes;
      *out = p;
      return SPTC_OK;
    }
    if (bufs.empty() || slab_used + bytes > bufs.back().bytes) {
      if (slab_device < 0) HIP_TRY(hipGetDevice(&slab_device));
      const size_t sz = std::max(bytes, slab_next);
      CachedSlab sl = cache_take(slab_device, sz);
      if (sl.p) {
        if (sl.ready) HIP_TRY(hipStreamWaitEvent(stream, sl.ready, 0));
      } else {
        hipError_t e = hipMallocAsync(&sl.p, sz, stream);
        if (e != hipSuccess || !sl.p) {
          (void)hipGetLastError();
          // memory held in the cache may be what is missing: give it back and retry once
          if (cache_trim(slab_device, 0) != SPTC_OK || hipMallocAsync(&sl.p, sz, stream) != hipSuccess || !sl.p) {
            (void)hipGetLastError();
            return fail(SPTC_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu bytes): %s", sz, hipGetErrorString(e));
          }
        }
        sl.bytes = sz;
        sl.ready = nullptr;
      }
      bufs.push_back({sl.p, sl.bytes, sl.ready});
      workspace += (int64_t)sl.bytes;
      slab_used = 0;
      slab_next = std::min(slab_next * 2, kSlabMax);
    }
    *out = static_cast<char*>(bufs.back().p) + slab_used;
    slab_used += bytes;
    return SPTC_OK;
  }

  template <class T>
  sptc_status allocate_n(int64_t n, T** out) {
    void* p = nullptr;
    sptc_status s = allocate(sizeof(T) * (size_t)std::max<int64_t>(n, 1), &p);
    *out = static_cast<T*>(p);
    return s;
  }

  void release_all() {
    for (auto it = bufs.rbegin(); it != bufs.rend(); ++it) {
      if (has_alloc) {
        if (alloc.release) alloc.release(it->p, it->bytes, stream, alloc.ctx);
        continue;
      }
      // back to the cache, ready once the stream's work so far is done
      hipEvent_t ev = it->ready;
      if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(it->p, stream);
        continue;
      }
      if (hipEventRecord(ev, stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(stream);
      }
      cache_put(slab_device, CachedSlab{it->p, it->bytes, ev});
    }
    bufs.clear();
    slab_used = 0;
    slab_next = kSlabMin;
    workspace = 0;
  }
};

struct sptc_plan_s : Workspace {
  int device = 0;
  sptc_options opt{};
  int num_cus = 1;

  int32_t ox = 0, oy = 0, nc = 0;
  int64_t nx = 0, ny = 0;
  int32_t out_order = 0;
  int64_t out_dims[SPTC_MAX_OUT_ORDER] = {};
  int32_t bits_c = 0, bits_fx = 0, bits_fy = 0;
  int32_t nfy = 0;

  KeyPack x_c{}, x_f{}, y_c{}, y_f{};
  Bounds xb{}, yb{};
  KeyUnpack out_unpack{}, ykey_unpack{}, yfree_unpack{};

  YSlot* ytab = nullptr;
  int64_t ytab_slots = 0;
  YEntry* yg = nullptr;
  XEntry* xrec = nullptr;
  uint32_t* xg = nullptr;
  uint32_t* xcnt = nullptr;
  unsigned long long* poff = nullptr;
  unsigned long long* tile_sums = nullptr;
  DevStatus* st = nullptr;
  int64_t* readback = nullptr;  // device counts read back by the inspection calls
  ZSlot* ztab = nullptr;
  int64_t ztab_slots = 0;
  unsigned long long* ztile_sums = nullptr;
  int64_t expand_nx = 0;         // X entries the global-hash expansion walks
  int64_t expand_products = 0;   // products it expands

  // grouped path
  YSlot* xtab = nullptr;
  int64_t xtab_slots = 0;
  int32_t max_probe_x = 0;
  GroupRec* groups = nullptr;
  XRec* xr = nullptr;
  unsigned long long* eoff = nullptr;
  uint32_t* dlist = nullptr;
  DRec* drec = nullptr;  // the direct groups' staging records, by list place
  uint32_t* dtfirst = nullptr;  // direct class: each product tile's first group
  uint32_t* wlist = nullptr;
  uint32_t* wcnt = nullptr;            // wave class: each group's output count (by list place)
  unsigned long long* woff = nullptr;  // and its first output's offset in the class
  uint32_t* tcnt = nullptr;            // dense block tiles placed by a scan: each tile's output count
  unsigned long long* toff = nullptr;  // and its offset
  unsigned long long* tsums = nullptr;  // scan scratch for them
  uint32_t* blist = nullptr;
  uint32_t* bdefer = nullptr;          // hashed block class: groups passed to the large-table launch
  uint32_t* glist = nullptr;
  uint32_t* yso = nullptr;    // dense block class: where each slice of each Y run begins, per Y table slot
  unsigned slice_cells = 0;   // and the width of a slice of the Y free key space
  int32_t block_mfma = 0;     // dense block class on the matrix cores
  unsigned* ycolbits = nullptr;  // dense Y free key: the cells that occur (bitmap)
  unsigned ycols = 0;            // and their number
  unsigned* run_start = nullptr;
  uint16_t* colid = nullptr;
  uint16_t* cellof = nullptr;
  MfmaPlan mplan{};
  bool in_batch = false;      // the packed plan of a batch
  bool stalled = false;       // a read-back timed out: the stream still holds the plan's work
  bool capture = false;       // no read-back (opt.capture_out_cap > 0): counts stay on the device
  bool swapped = false;       // X and Y traded places (operand order): Z's rows are put back
  bool dense_rows = false;    // dense block class of small groups: a whole dense row per workgroup
  int64_t dtfirst_slots = 0;  // entries of the direct class's tile table
  bool pageable_readback = false;  // read counts back through pageable memory (no pinned buffer)
  bool block_surveyed = false;  // the block survey ran (dense Y free key, one contraction)
  int32_t block_nonfinite = 0;  // an X or Y value is not finite (the matrix cores need finite values)
  int64_t block_products = 0;   // survey: products of the block class
  unsigned long long* dpos = nullptr;
  uint16_t* ykey16 = nullptr;  // dense Y free keys: compact copy of grouped Y
  uint32_t* ylong = nullptr;    // and the long runs of the repeat check (with their count)
  double* yval = nullptr;
  unsigned long long* yset = nullptr;
  int64_t yset_slots = 0;
  LdsQueue* queue = nullptr;   // work queue counters of the persistent launch (grouped mode)
  unsigned long long* gl_eoff = nullptr;
  int64_t x_groups = 0, nd = 0, nw = 0, nb = 0, ngl = 0;
  int64_t direct_products = 0;
  int32_t ydup = 0;
  int32_t dense = 0;
  int32_t y_agg = 0, x_agg = 0;  // small keys: LDS-aggregated count and scatter
  unsigned* yhist = nullptr;     // their per-chunk histograms, then (key, chunk) positions
  unsigned* xhist = nullptr;
  unsigned long long* agg_total = nullptr;
  uint64_t ycells = 0;
  KeyUnpack ux{}, uy{};

  int64_t products = 0, y_groups = 0, out_bound = 0;
  int32_t max_probe_y = 0, max_probe_z = 0;

  // key table geometry; a batch's packed problem has one region per contraction
  TabGeom ygeom{}, xgeom{};
  std::vector<Region> xreg_h;
  Region* xreg = nullptr;
};

// Per-contraction regions of the X free key table of a batch's packed
// problem (keys >> xshift give the contraction): the X groups, and so every
// list of groups, come out ordered by contraction.  Y's table stays one
// hashed array.
struct BatchRegions {
  std::vector<Region> x;
  int32_t xshift = 0;
};


// Key layout of one contraction: contracting key in cx/cy order, free keys
// in ascending mode order; the output is X free coordinates then Y free ones.
struct Layout {
  KeyPack x_c{}, y_c{}, x_f{}, y_f{};
  int32_t bits_c = 0, bits_fx = 0, bits_fy = 0, nfy = 0, out_order = 0;
  int64_t out_dims[SPTC_MAX_OUT_ORDER] = {};
  Bounds xb{}, yb{};
  KeyUnpack ux{}, uy{};
  uint64_t ycells = 1;
  int64_t c_cells = 1, fx_cells = 1;  // contracting / X free key spaces (saturating)
};

// A batch: the packed problem's plan plus each contraction's output layout.
struct sptc_batch_s : Workspace {
  int32_t count = 0;
  sptc_plan_s* inner = nullptr;  // plan of the packed problem
  BatchWidths w{};
  struct Item {
    Layout L;
    int64_t products = 0, bound = 0, idx_off = 0, val_off = 0;
  };
  std::vector<Item> items;
  BatchOut* outs = nullptr;  // device [count]
  BatchSeg* seg = nullptr;   // device [count]
  int64_t* tnnz = nullptr;   // the packed plan's own output count (unused)
  int64_t idx_elems = 0, val_elems = 0;
};

namespace {

sptc_status check_coo(const sptc_coo* T, const char* name) {
  if (!T) return fail(SPTC_ERR_INVALID_ARG, "%s is NULL", name);
  if (T->order < 0 || T->order > SPTC_MAX_ORDER)
    return fail(SPTC_ERR_INVALID_ARG, "%s: order %d outside 0..%d", name, T->order, SPTC_MAX_ORDER);
  if (T->order > 0 && !T->dims) return fail(SPTC_ERR_INVALID_ARG, "%s: dims is NULL", name);
  for (int32_t m = 0; m < T->order; ++m)
    if (T->dims[m] < 1 || T->dims[m] > ((int64_t)1 << 31))
      return fail(SPTC_ERR_INVALID_ARG, "%s: mode %d length %lld outside 1..2^31", name, m, (long long)T->dims[m]);
  if (T->nnz < 0 || T->nnz > (int64_t)0xfffffffeLL)
    return fail(SPTC_ERR_INVALID_ARG, "%s: nnz %lld outside 0..2^32-2", name, (long long)T->nnz);
  if (T->nnz > 0 && !T->val) return fail(SPTC_ERR_INVALID_ARG, "%s: val is NULL", name);
  if (T->nnz > 0 && T->order > 0 && !T->idx) return fail(SPTC_ERR_INVALID_ARG, "%s: idx is NULL", name);
  return SPTC_OK;
}

sptc_status check_options(const sptc_options& o) {
  if (!(o.load_factor > 0.0 && o.load_factor <= 0.95))
    return fail(SPTC_ERR_INVALID_ARG, "load_factor %g outside (0, 0.95]", o.load_factor);
  if (o.max_probe < 0) return fail(SPTC_ERR_INVALID_ARG, "max_probe %d < 0", o.max_probe);
  if (o.mode != SPTC_MODE_GROUPED && o.mode != SPTC_MODE_GLOBAL)
    return fail(SPTC_ERR_INVALID_ARG, "unknown mode %d", o.mode);
  if (o.block_mfma < -1 || o.block_mfma > 1) return fail(SPTC_ERR_INVALID_ARG, "block_mfma %d not in -1..1", o.block_mfma);
  if (o.out_table_slots != 0 && (o.out_table_slots < 2 || (o.out_table_slots & (o.out_table_slots - 1))))
    return fail(SPTC_ERR_INVALID_ARG, "out_table_slots %lld is not a power of two >= 2",
                (long long)o.out_table_slots);
  if (o.tile != 0 && o.tile != 1024 && o.tile != 2048)
    return fail(SPTC_ERR_INVALID_ARG, "tile %d is not 0, 1024 or 2048", o.tile);
  if (o.lds_max_keys != 0 && (o.lds_max_keys < 64 || o.lds_max_keys > kBlockCap))
    return fail(SPTC_ERR_INVALID_ARG, "lds_max_keys %d outside 64..%d", o.lds_max_keys, kBlockCap);
  if (o.capture_out_cap < 0) return fail(SPTC_ERR_INVALID_ARG, "capture_out_cap < 0");
  if (o.operand_order != 0 && o.operand_order != 1)
    return fail(SPTC_ERR_INVALID_ARG, "operand_order %d is not 0 or 1", o.operand_order);
  return SPTC_OK;
}

// Lays out `modes` of a tensor in a key, first listed mode most significant.
KeyPack make_pack(const int64_t* dims, const std::vector<int32_t>& modes, int32_t* total_bits) {
  KeyPack kp{};
  kp.n = (int32_t)modes.size();
  int32_t shift = 0;
  for (int32_t k = kp.n - 1; k >= 0; --k) {
    const int32_t b = bits_for(dims[modes[k]]);
    kp.field[k] = make_field((uint32_t)modes[k], (uint32_t)shift, (uint32_t)b);
    shift += b;
  }
  *total_bits = shift;
  return kp;
}

void add_unpack(KeyUnpack& ku, const KeyPack& kp, int32_t extra_shift) {
  for (int32_t k = 0; k < kp.n; ++k) {
    ku.field[ku.n] = make_field(0u, field_shift(kp.field[k]) + (uint32_t)extra_shift, field_bits(kp.field[k]));
    ku.n++;
  }
}

Bounds make_bounds(const sptc_coo* T, int32_t check) {
  Bounds b{};
  b.order = T->order;
  for (int32_t m = 0; m < T->order; ++m) b.dim[m] = (uint32_t)T->dims[m];
  b.check = check;
  return b;
}

// Records the stage's begin (0) or end (1) event when the caller asked for it.
hipError_t mark_events(void* const* events, hipStream_t s, int stage, int end) {
  if (!events) return hipSuccess;
  void* ev = events[2 * stage + end];
  return ev ? hipEventRecord(static_cast<hipEvent_t>(ev), s) : hipSuccess;
}

hipError_t mark(const sptc_plan_s* P, hipStream_t s, int stage, int end) {
  return mark_events(P->opt.stage_events, s, stage, end);
}

sptc_status status_from_bits(uint32_t err) {
  if (err & kErrCoord) return fail(SPTC_ERR_INVALID_ARG, "a coordinate is outside its mode length");
  if (err & kErrCapacity) return fail(SPTC_ERR_CAPACITY, "hash probe limit reached or output larger than out_cap");
  if (err) return fail(SPTC_ERR_INTERNAL, "internal consistency check failed on the device (bits 0x%x)", err);
  return SPTC_OK;
}

// Pinned landing buffer for status read-backs, one per thread and device (a
// read-back completes before its call returns), allocated on first use and
// kept for the life of the process.  NULL if it cannot be allocated.
DevStatus* pinned_status(int dev) {
  thread_local DevStatus* buf[64] = {};
  if (dev < 0 || dev >= 64) return nullptr;
  if (!buf[dev]) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    buf[dev] = static_cast<DevStatus*>(p);
  }
  return buf[dev];
}

// The plan's counts: copied into pinned memory and waited for by polling the
// stream (the plan needs them within microseconds of the last kernel; a
// blocking wait would add its wake-up latency to every plan).  The first
// polls spin; later ones yield the core between queries, and after
// kReadbackDeadline the plan gives up with SPTC_ERR_HIP (the work is still
// queued: the plan's memory then goes back in stream order, without a wait).
constexpr auto kReadbackDeadline = std::chrono::seconds(60);
constexpr unsigned kReadbackSpins = 1024;

sptc_status read_status(sptc_plan_s* P, DevStatus* host) {
  DevStatus* pin = P->pageable_readback ? nullptr : pinned_status(P->device);
  if (!pin) {
    HIP_TRY(hipMemcpyAsync(host, P->st, sizeof *host, hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    return status_from_bits(host->err);
  }
  HIP_TRY(hipMemcpyAsync(pin, P->st, sizeof *pin, hipMemcpyDeviceToHost, P->stream));
  hipError_t e;
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned polls = 0; (e = hipStreamQuery(P->stream)) == hipErrorNotReady; ++polls) {
    if (polls < kReadbackSpins) continue;
    std::this_thread::yield();
    if ((polls & 255) == 0 && std::chrono::steady_clock::now() - t0 > kReadbackDeadline) {
      P->stalled = true;
      return fail(SPTC_ERR_HIP, "plan read-back: the stream did not finish within %lld s",
                  (long long)std::chrono::duration_cast<std::chrono::seconds>(kReadbackDeadline).count());
    }
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamQuery");
  *host = *pin;
  return status_from_bits(host->err);
}

int64_t out_cells(const sptc_plan_s* P) {
  int64_t cells = 1;
  for (int32_t m = 0; m < P->out_order; ++m) {
    if (cells > ((int64_t)1 << 62) / P->out_dims[m]) return (int64_t)1 << 62;
    cells *= P->out_dims[m];
  }
  return cells;
}

// Output hash for the products that are accumulated in device memory.
sptc_status size_out_table(sptc_plan_s* P, int64_t products) {
  const int64_t bound = std::min<int64_t>(products, out_cells(P));
  if (P->opt.out_table_slots > 0)
    P->ztab_slots = P->opt.out_table_slots;
  else
    P->ztab_slots = pow2_at_least((double)bound / P->opt.load_factor);
  P->max_probe_z = P->opt.max_probe > 0 ? P->opt.max_probe : (int32_t)std::min<int64_t>(P->ztab_slots, 1 << 30);
  sptc_status st;
  if ((st = P->allocate_n(P->ztab_slots, &P->ztab))) return st;
  if ((st = P->allocate_n(scan_tiles(P->ztab_slots) + 1, &P->ztile_sums))) return st;
  return SPTC_OK;
}

// Dense block tiles are placed by a count pass and a scan instead of an
// atomic each when there are more than kTileScanTiles of them (the atomics
// alone would take 1.6 ms) and they average fewer than kTileScanProducts
// products (a second walk is cheap); with 20K tiles a second walk measured
// costlier than the atomics it saves.
constexpr int64_t kTileScanTiles = 131072;
constexpr int64_t kTileScanProducts = 4096;

// Dense block groups averaging fewer products than this run one workgroup
// per group with the whole dense row instead of (group, slice) tiles.
constexpr int64_t kDenseRowProducts = 16384;

// Cells of the dense LDS accumulator for a Y free key of bits_y bits.
unsigned dense_cells(int32_t bits_y) { return std::max(1u << bits_y, 1024u); }

// Width of one slice of the dense Y free key space for the sliced walk:
// the keys that Y's mode lengths allow, 0 to pack(dims - 1), cut into
// kSlices equal parts of whole 64-cell chunks.  Cutting the packed key
// space itself would leave the keys past the largest (a mode length that is
// not a power of two leaves the top of its field unused) whole slices with
// nothing in them, and their XCDs idle.  A batch's packed plan cuts the
// whole space.
unsigned slice_width(const sptc_plan_s* P, unsigned cells) {
  const unsigned full = cells / kSlices;
  if (P->in_batch) return full;
  uint64_t kmax = 0;
  for (int32_t k = 0; k < P->y_f.n; ++k) {
    const uint32_t f = P->y_f.field[k];
    const uint64_t d = P->yb.dim[field_mode(f)];
    if (d > 1) kmax |= (d - 1) << field_shift(f);
  }
  uint64_t w = (kmax + kSlices) / kSlices;  // ceil((kmax + 1) / kSlices)
  w = (w + 63) / 64 * 64;
  return (unsigned)std::min<uint64_t>(w, full);
}

// Shift of the Y free key in the repeated-coordinate check, or -1 when the
// whole coordinate does not fit 63 bits and the check hashes it instead.
int32_t yset_bits(const sptc_plan_s* P) { return P->bits_c + P->bits_fy <= 63 ? P->bits_fy : -1; }

// A1-A3: Y grouped by contracting key (both modes).
sptc_status plan_group_y(sptc_plan_s* P, const sptc_coo* Y) {
  const hipStream_t s = P->stream;
  const uint64_t seed = P->opt.hash_seed;
  sptc_status st;
  if (P->y_agg && (st = P->allocate_n((agg_chunks(P->ny) + 1) * P->ytab_slots, &P->yhist))) return st;
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_COUNT, 0));
  if (!P->y_agg) HIP_TRY(launch_fill_empty(P->ytab, P->ytab_slots, nullptr, s));  // the aggregated count writes every slot
  if (P->y_agg)
    HIP_TRY(launch_key_count_agg(Y->idx, P->ny, P->y_c, P->ytab, (unsigned)P->ytab_slots, P->yhist, P->agg_total,
                                 &P->st->groups, s));
  else
    HIP_TRY(launch_key_count(Y->idx, P->ny, P->y_c, P->ytab, P->ygeom, seed, P->max_probe_y, P->st,
                             &P->st->groups, P->num_cus, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_COUNT, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_SCAN, 0));
  if (!P->y_agg) HIP_TRY(launch_scan_y_table(P->ytab, P->ytab_slots, true, P->tile_sums, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_SCAN, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_SCATTER, 0));
  if (P->yset) HIP_TRY(launch_fill_keys(P->yset, P->yset_slots, s));
  if (P->y_agg)
    HIP_TRY(launch_y_scatter_agg(Y->idx, Y->val, P->ny, P->y_c, P->y_f, P->yb, P->ytab, (unsigned)P->ytab_slots,
                                 P->yhist, P->yg, P->yset, (uint64_t)P->yset_slots - 1, seed, yset_bits(P), P->st,
                                 s));
  else
    HIP_TRY(launch_y_scatter(Y->idx, Y->val, P->ny, P->y_c, P->y_f, P->yb, P->ytab, P->ygeom, seed, P->max_probe_y,
                             P->yg, P->yset, (uint64_t)P->yset_slots - 1, yset_bits(P), P->st, P->num_cus, s));
  if (P->opt.mode == SPTC_MODE_GROUPED && P->dense) {
    // the runs are sorted later, for the block walk only (plan_grouped)
    HIP_TRY(launch_sort_y_runs(P->ytab, P->ytab_slots, P->yg, P->ny, P->ykey16, P->yval, P->ycolbits, P->st, false,
                               P->num_cus, s, nullptr, nullptr, 0u, P->ylong));
  }
  HIP_TRY(mark(P, s, SPTC_STAGE_Y_SCATTER, 1));
  return SPTC_OK;
}

sptc_status plan_global(sptc_plan_s* P, const sptc_coo* X) {
  const hipStream_t s = P->stream;
  sptc_status st;
  if ((st = P->allocate_n(P->nx, &P->xrec))) return st;
  if ((st = P->allocate_n(P->nx, &P->xg))) return st;
  if ((st = P->allocate_n(P->nx, &P->xcnt))) return st;
  if ((st = P->allocate_n(P->nx + 1, &P->poff))) return st;
  HIP_TRY(mark(P, s, SPTC_STAGE_X_PROBE, 0));
  HIP_TRY(launch_x_probe(X->idx, X->val, P->nx, P->x_c, P->x_f, P->xb, P->ytab, P->ygeom, P->opt.hash_seed,
                         P->max_probe_y, P->xrec, P->xg, P->xcnt, P->st, P->num_cus, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_X_PROBE, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_P_SCAN, 0));
  HIP_TRY(launch_scan_products(P->xcnt, P->nx, P->poff, P->tile_sums, &P->st->products, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_P_SCAN, 1));
  P->expand_nx = P->nx;
  if (P->capture) {  // no read-back: the product count stays on the device
    P->products = P->y_groups = P->expand_products = -1;
    P->out_bound = std::min<int64_t>(P->opt.capture_out_cap, out_cells(P));
    return size_out_table(P, P->out_bound);
  }
  DevStatus host{};
  if ((st = read_status(P, &host))) return st;
  P->products = (int64_t)host.products;
  P->y_groups = (int64_t)host.groups;
  P->out_bound = std::min<int64_t>(P->products, out_cells(P));
  P->expand_products = P->products;
  return size_out_table(P, P->products);
}

// X grouped by free key (section 4.1), then its groups sorted into
// accumulation classes.  Groups too large for LDS are gathered for the
// device-memory output hash.
// Rows x columns x runs of the matrix-core block class (padded to whole
// tiles) may be this many times its products.  Measured on the block-sparse
// 48^4 workload (work 12.9x its products): the dense product takes 0.59 ms
// where the walk takes 1.33 ms, and the panels cost 0.18 ms of plan time
// where the walk's sorts cost 0.2 ms.  Per unit the walk spends about 30x
// what the dense product spends per multiply-add; the panels' cost, which
// grows with the padded rows and columns rather than the products, brings
// the break-even down to about 24x.
constexpr double kMfmaWorkRatio = 24.0;
// Largest dense X and Y panels the class builds (bytes); beyond, the walk.
constexpr int64_t kMfmaMaxPanelBytes = (int64_t)8 << 30;

// Rows x columns x runs of the matrix-core product, padded to whole tiles.
double mfma_work(int64_t rows, int64_t cols, int64_t runs) {
  const auto up = [](int64_t v, int64_t t) { return (double)((v + t - 1) / t * t); };
  return up(rows, kMfmaRows) * up(cols, kMfmaCols) * up(runs, kMfmaK);
}

// From what is read back with the class counts: every X and Y value finite
// (zero padding must add exact zeros), not ruled out by the option, and
// under the cost rule dense work within the ratio of the block class's
// products (block survey).
bool mfma_candidate(const sptc_plan_s* P) {
  if (!P->block_surveyed || P->block_nonfinite || P->ycols == 0) return false;
  if (P->opt.block_mfma > 0) return true;
  return mfma_work(P->nb, P->ycols, P->y_groups) <= kMfmaWorkRatio * (double)P->block_products;
}

// Dense block class on the matrix cores (the survey already decided): the
// panels are built from what the plan knows (rows, columns that occur, runs),
// with no read-back.
sptc_status plan_block_mfma(sptc_plan_s* P) {
  const hipStream_t s = P->stream;
  sptc_status st;
  const unsigned cells = P->ycols;
  const int64_t nruns = P->y_groups;
  if (cells == 0 || nruns <= 0) return SPTC_OK;
  const int64_t nsteps = (nruns + kMfmaK - 1) / kMfmaK, nrt = (P->nb + kMfmaRows - 1) / kMfmaRows,
                nct = (cells + kMfmaCols - 1) / kMfmaCols;
  const int64_t ablocks = nrt * nsteps, bblocks = nct * nsteps;
  const int64_t panel_bytes =
      ablocks * (kMfmaK * kMfmaRows * 8 + kMfmaRows * 4) + bblocks * (kMfmaK * kMfmaCols * 8 + kMfmaCols * 4);
  if (panel_bytes > kMfmaMaxPanelBytes) return SPTC_OK;
  const int64_t runs_cap = std::min<int64_t>(P->ytab_slots, P->ny) + 1;
  unsigned* runid = nullptr;
  double *pa = nullptr, *pb = nullptr;
  unsigned *am = nullptr, *bm = nullptr;
  if ((st = P->allocate_n(runs_cap, &P->run_start))) return st;
  if ((st = P->allocate_n(P->ny, &runid))) return st;
  if ((st = P->allocate_n((int64_t)1 << kDenseBits, &P->colid))) return st;
  if ((st = P->allocate_n(cells, &P->cellof))) return st;
  if ((st = P->allocate_n(ablocks * kMfmaK * kMfmaRows, &pa))) return st;
  if ((st = P->allocate_n(ablocks * kMfmaRows, &am))) return st;
  if ((st = P->allocate_n(bblocks * kMfmaK * kMfmaCols, &pb))) return st;
  if ((st = P->allocate_n(bblocks * kMfmaCols, &bm))) return st;
  HIP_TRY(hipMemsetAsync(pb, 0, sizeof(double) * bblocks * kMfmaK * kMfmaCols, s));
  HIP_TRY(hipMemsetAsync(bm, 0, sizeof(unsigned) * bblocks * kMfmaCols, s));
  HIP_TRY(launch_mfma_runs(P->ytab, P->ytab_slots, P->ny, P->run_start, runid, nruns, P->st, P->tile_sums, s));
  HIP_TRY(launch_mfma_panels(P->ycolbits, P->groups, P->blist, P->nb, P->xr, P->run_start, runid, (unsigned)nruns,
                             P->ykey16, P->yval, P->ny, P->colid, P->cellof, cells, (unsigned)nsteps, P->ydup, pa, am,
                             pb, bm, P->st, P->num_cus, s));
  P->mplan = MfmaPlan{pa, am, pb, bm, P->cellof, (unsigned)nsteps, cells, (unsigned)nct};
  P->block_mfma = 1;
  return SPTC_OK;
}

sptc_status plan_grouped(sptc_plan_s* P, const sptc_coo* X) {
  const hipStream_t s = P->stream;
  const uint64_t seed = P->opt.hash_seed;
  sptc_status st;
  // hashed X free keys of at most 31 bits: the compact table
  const bool x32 = !P->x_agg && !P->xgeom.reg && !P->xgeom.ident && P->bits_fx <= 31 && P->nx < ((int64_t)1 << 31);
  // ... grouped by partition (no device atomic per entry) up to kPartMaxEntries
  const bool xpart = x32 && P->nx <= kPartMaxEntries;
  unsigned long long* xtab32 = nullptr;
  XPartBuffers xw{};
  if (xpart) {
    const int64_t nbk = (int64_t)1 << part_bits(P->nx), nh = nbk * part_tiles(P->nx);
    unsigned long long* scan = nullptr;
    if ((st = P->allocate_n(P->nx, &xw.pkey)) || (st = P->allocate_n(P->nx, &xw.prec)) ||
        (st = P->allocate_n(nh, &xw.hist)) || (st = P->allocate_n(scan_tiles(nh) + 1, &scan)))
      return st;
    xw.scan = scan;
  } else if (x32) {
    if ((st = P->allocate_n(P->xtab_slots, &xtab32))) return st;
  } else if ((st = P->allocate_n(P->xtab_slots, &P->xtab))) {
    return st;
  }
  if ((st = P->allocate_n(P->nx, &P->groups))) return st;
  if ((st = P->allocate_n(P->nx, &P->xr))) return st;
  if ((st = P->allocate_n(P->nx + 1, &P->eoff))) return st;
  if ((st = P->allocate_n(P->nx, &P->dlist))) return st;
  if ((st = P->allocate_n(P->nx, &P->drec))) return st;
  if ((st = P->allocate_n(P->nx, &P->wlist))) return st;
  if ((st = P->allocate_n(P->nx, &P->blist))) return st;
  if ((st = P->allocate_n(P->nx, &P->glist))) return st;
  if ((st = P->allocate_n(P->nx + 1, &P->dpos))) return st;

  if (P->x_agg && (st = P->allocate_n((agg_chunks(P->nx) + 1) * P->xtab_slots, &P->xhist))) return st;

  HIP_TRY(mark(P, s, SPTC_STAGE_X_PROBE, 0));
  if (xpart) {
    HIP_TRY(prepare_x_partition());
    HIP_TRY(launch_x_partition(X->idx, X->val, P->nx, P->x_f, P->x_c, P->xb, P->ytab, P->ygeom, P->max_probe_y, seed,
                               xw, P->groups, P->xr, P->st, P->num_cus, s));
  } else if (x32) {
    HIP_TRY(launch_x_table32(X->idx, X->val, P->nx, P->x_f, P->x_c, P->xb, xtab32, P->xgeom, P->max_probe_x,
                             P->groups, P->ytab, P->ygeom, P->max_probe_y, seed, P->xr, P->tile_sums, P->st,
                             P->num_cus, s));
  } else {
    if (!P->x_agg) HIP_TRY(launch_fill_empty(P->xtab, P->xtab_slots, nullptr, s));  // (as for Y)
    if (P->x_agg)
      HIP_TRY(launch_key_count_agg(X->idx, P->nx, P->x_f, P->xtab, (unsigned)P->xtab_slots, P->xhist, P->agg_total,
                                   nullptr, s));
    else
      HIP_TRY(launch_key_count(X->idx, P->nx, P->x_f, P->xtab, P->xgeom, seed, P->max_probe_x, P->st, nullptr,
                               P->num_cus, s));
    HIP_TRY(launch_scan_x_table(P->xtab, P->xtab_slots, P->groups, P->nx, !P->x_agg, P->tile_sums, P->st, s));
    if (P->x_agg)
      HIP_TRY(launch_x_scatter_agg(X->idx, X->val, P->nx, P->x_f, P->x_c, P->xb, P->xtab, (unsigned)P->xtab_slots,
                                   P->xhist, P->ytab, P->ygeom, P->max_probe_y, seed, P->xr, P->st, s));
    else
      HIP_TRY(launch_x_scatter(X->idx, X->val, P->nx, P->x_f, P->x_c, P->xb, P->xtab, P->xgeom, P->max_probe_x,
                               P->ytab, P->ygeom, P->max_probe_y, seed, P->xr, P->st, P->num_cus, s));
  }
  HIP_TRY(mark(P, s, SPTC_STAGE_X_PROBE, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_P_SCAN, 0));
  HIP_TRY(launch_scan_entries(P->xr, P->nx, P->eoff, P->tile_sums, P->st, s));
  // at most one X group per occupied table slot: small tables make these
  // scans a single tile
  const int64_t max_groups = std::min<int64_t>(P->nx, P->xtab_slots);
  HIP_TRY(launch_classify(P->groups, max_groups, P->eoff, P->ycells, P->dense, P->dlist, P->wlist, P->blist,
                          P->glist, P->dpos, P->tile_sums, P->st, s, P->opt.lds_max_keys, P->xr, P->drec));
  HIP_TRY(launch_scan_direct(max_groups, P->dpos, P->tile_sums, P->st, s));
  // the block class's products and finiteness, read back with the counts
  // below, decide the matrix-core class with no read-back of its own
  P->block_surveyed = P->dense && !P->in_batch && P->opt.block_mfma != 0;
  if (P->block_surveyed)
    HIP_TRY(launch_block_survey(P->groups, P->blist, P->eoff, P->ycolbits, P->st, P->num_cus, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_P_SCAN, 1));

  DevStatus host{};
  if (P->capture) {
    // no read-back: every count stays on the device and the host keeps
    // upper bounds (each class at most every group, the direct class's
    // products at most the outputs); the launches read the counts
    P->products = P->y_groups = -1;
    P->out_bound = std::min<int64_t>(P->opt.capture_out_cap, out_cells(P));
    P->x_groups = P->nd = P->nw = P->nb = P->ngl = max_groups;
    P->direct_products = P->out_bound;
    P->ydup = 1;
    P->ycols = 0;
    P->block_products = 0;
    P->block_nonfinite = 1;
  } else {
    if ((st = read_status(P, &host))) return st;
    P->products = (int64_t)host.products;
    P->y_groups = (int64_t)host.groups;
    P->out_bound = std::min<int64_t>(P->products, out_cells(P));
    P->x_groups = (int64_t)host.xgroups;
    P->nd = (int64_t)(host.class_lo & 0xffffffffull);
    P->nw = (int64_t)(host.class_lo >> 32);
    P->nb = (int64_t)host.class_hi;
    P->ngl = P->x_groups - P->nd - P->nw - P->nb;
    P->direct_products = (int64_t)host.direct_products;
    P->ydup = host.ydup ? 1 : 0;
    P->ycols = host.ycols;
    P->block_products = (int64_t)host.block_products;
    P->block_nonfinite = host.nonfinite ? 1 : 0;
    if (P->ngl < 0) return fail(SPTC_ERR_INTERNAL, "group classes do not add up");
  }
  if (P->nw > 0 && !P->in_batch) {
    if ((st = P->allocate_n(P->nw, &P->wcnt))) return st;
    if ((st = P->allocate_n(P->nw, &P->woff))) return st;
  }
  if (P->nd > 0 && P->direct_products > 0) {
    P->dtfirst_slots = direct_tile_bound((uint64_t)P->direct_products);
    if ((st = P->allocate_n(P->dtfirst_slots, &P->dtfirst))) return st;
  }
  if (P->nb > 0) {
    HIP_TRY(prepare_group_block());
    if (P->dense) {
      HIP_TRY(mark(P, s, SPTC_STAGE_X_SORT, 0));
      if (mfma_candidate(P) && (st = plan_block_mfma(P))) return st;
      // small groups (a few tiles' worth of products each): a workgroup per
      // group with its whole dense row beats eight thin slice tiles
      P->dense_rows = !P->block_mfma && !P->capture && P->products < P->nb * kDenseRowProducts;
      if (!P->block_mfma && !P->dense_rows) {
        // the sliced walk: runs sorted by Y free key (consecutive
        // accumulator cells) and cut into the slices of the Y free key
        // space; block-class X records keyed by their run's table slot
        uint32_t* runslot = nullptr;
        if ((st = P->allocate_n(P->ytab_slots * (kSlices + 1), &P->yso))) return st;
        if ((st = P->allocate_n(P->ny, &runslot))) return st;
        P->slice_cells = slice_width(P, dense_cells(P->bits_fy));
        HIP_TRY(launch_sort_y_runs(P->ytab, P->ytab_slots, P->yg, P->ny, P->ykey16, P->yval, nullptr, P->st, true,
                                   P->num_cus, s, P->yso, runslot, P->slice_cells));
        HIP_TRY(launch_block_runslots(P->groups, P->blist, P->nb, P->xr, runslot, P->ny, P->st, P->num_cus, s,
                                      P->capture ? P->st : nullptr));
        // (the list's length is known here unless the plan is captured)
        if (!P->capture && !P->in_batch) HIP_TRY(launch_order_blist(P->groups, P->eoff, P->blist, P->nb, s));
      }
      HIP_TRY(mark(P, s, SPTC_STAGE_X_SORT, 1));
    }
  }
  if ((st = P->allocate_n(1, &P->queue))) return st;
  HIP_TRY(prepare_lds_queue());
  if (P->nb > 0 && !P->dense && (st = P->allocate_n(2 * P->nb, &P->bdefer))) return st;
  // Very many small dense tiles: each tile's atomic on the one output
  // cursor (serialised, about 12 ns each) would cost more than accumulating
  // the tiles twice, once to count their outputs and once to write them at
  // offsets from a scan.  The read-back's products stand in for the class's.
  if (P->dense && !P->block_mfma && !P->dense_rows && P->nb > 0 && !P->capture && !P->in_batch &&
      P->nb * kSlices > kTileScanTiles &&
      P->nb * kSlices > P->products / kTileScanProducts) {
    const int64_t nt = P->nb * kSlices;
    if ((st = P->allocate_n(nt, &P->tcnt))) return st;
    if ((st = P->allocate_n(nt, &P->toff))) return st;
    if ((st = P->allocate_n(2 * (scan_tiles(nt) + 1), &P->tsums))) return st;
  }
  if (P->ngl == 0) return SPTC_OK;

  // The global class keys its table by (place in glist << Y free bits) | Y free key.
  if (bits_for(P->ngl) + P->bits_fy > 63)
    return fail(SPTC_ERR_KEY_OVERFLOW, "%lld groups too large for LDS and a %d-bit Y free key do not fit a 63-bit key",
                (long long)P->ngl, P->bits_fy);
  if ((st = P->allocate_n(P->ngl, &P->gl_eoff))) return st;
  HIP_TRY(launch_scan_global_entries(P->groups, P->glist, P->ngl, P->gl_eoff, P->tile_sums, P->st, s));
  if (P->capture) {
    P->expand_nx = P->nx;  // the global class's entries, at most all of X
  } else {
    if ((st = read_status(P, &host))) return st;
    P->expand_nx = (int64_t)host.global_entries;
  }
  if ((st = P->allocate_n(P->expand_nx, &P->xrec))) return st;
  if ((st = P->allocate_n(P->expand_nx, &P->xg))) return st;
  if ((st = P->allocate_n(P->expand_nx, &P->xcnt))) return st;
  if ((st = P->allocate_n(P->expand_nx + 1, &P->poff))) return st;
  HIP_TRY(launch_gather_global(P->groups, P->glist, P->ngl, P->gl_eoff, P->xr, P->xrec, P->xg, P->xcnt, P->num_cus,
                               s, P->capture ? P->st : nullptr));
  HIP_TRY(launch_scan_products(P->xcnt, P->expand_nx, P->poff, P->tile_sums, &P->st->global_products, s,
                               P->capture ? &P->st->global_entries : nullptr));
  if (P->capture) {
    P->expand_products = -1;
    return size_out_table(P, P->out_bound);  // the class's distinct outputs are outputs
  }
  if ((st = read_status(P, &host))) return st;
  P->expand_products = (int64_t)host.global_products;
  return size_out_table(P, P->expand_products);
}

sptc_status plan_body(sptc_plan_s* P, const sptc_coo* X, const sptc_coo* Y, const int32_t* cx, const int32_t* cy,
                      const BatchRegions* br) {
  // Key tables sized from the number of distinct keys they can hold.
  std::vector<int32_t> cyv(cy, cy + P->nc), fx;
  for (int32_t m = 0; m < X->order; ++m)
    if (std::find(cx, cx + P->nc, m) == cx + P->nc) fx.push_back(m);
  const bool grouped = P->opt.mode == SPTC_MODE_GROUPED;
  const int64_t y_bound = std::min<int64_t>(P->ny, sat_prod(Y->dims, cyv));
  P->ytab_slots = P->y_c.ident ? std::max<int64_t>((int64_t)1 << P->bits_c, 2)
                               : pow2_at_least((double)y_bound / P->opt.load_factor);
  if (br) {  // one X region per contraction, laid out by the batch
    P->xreg_h = br->x;
    P->xtab_slots = (int64_t)(br->x.back().base + br->x.back().mask + 1);
  } else {
    if (grouped) {
      const int64_t x_bound = std::min<int64_t>(P->nx, sat_prod(X->dims, fx));
      P->xtab_slots = P->x_f.ident ? std::max<int64_t>((int64_t)1 << P->bits_fx, 2)
                                   : pow2_at_least((double)x_bound / P->opt.load_factor);
    }
  }
  P->max_probe_y = P->opt.max_probe > 0 ? P->opt.max_probe : (int32_t)std::min<int64_t>(P->ytab_slots, 1 << 30);
  if (grouped)
    P->max_probe_x = P->opt.max_probe > 0 ? P->opt.max_probe : (int32_t)std::min<int64_t>(P->xtab_slots, 1 << 30);
  P->ygeom = TabGeom{(uint64_t)P->ytab_slots - 1, nullptr, 0, P->y_c.ident};
  P->xgeom = TabGeom{(uint64_t)P->xtab_slots - 1, nullptr, 0, P->x_f.ident};

  sptc_status st;
  if (br) {
    if ((st = P->allocate_n((int64_t)br->x.size(), &P->xreg))) return st;
    HIP_TRY(hipMemcpyAsync(P->xreg, P->xreg_h.data(), sizeof(Region) * P->xreg_h.size(), hipMemcpyHostToDevice,
                           P->stream));
    P->xgeom = TabGeom{0, P->xreg, br->xshift, 0};
  }
  if ((st = P->allocate_n(P->ytab_slots, &P->ytab))) return st;
  if ((st = P->allocate_n(P->ny, &P->yg))) return st;
  if (grouped && P->dense) {
    if ((st = P->allocate_n(P->ny, &P->ykey16))) return st;
    if ((st = P->allocate_n(P->ny, &P->yval))) return st;
    if ((st = P->allocate_n(y_long_run_slots(P->ny), &P->ylong))) return st;
    if ((st = P->allocate_n(kCellWords, &P->ycolbits))) return st;
    HIP_TRY(launch_zero_u64(reinterpret_cast<unsigned long long*>(P->ycolbits), kCellWords / 2, P->stream));
  }
  const int64_t tiles = std::max<int64_t>({scan_tiles(P->ytab_slots), scan_tiles(P->xtab_slots), scan_tiles(P->nx)});
  if ((st = P->allocate_n(2 * (tiles + 1), &P->tile_sums))) return st;  // room for pair-valued scans
  // Y coordinate set (grouped mode): finds repeated Y coordinates, which the
  // direct class cannot have.  With a dense Y free key the run sort finds
  // them instead.
  const bool yset = grouped && !P->dense;
  if (yset) {
    P->yset_slots = pow2_at_least(4.0 * (double)std::max<int64_t>(P->ny, 1));  // sparse: short probes
    if ((st = P->allocate_n(P->yset_slots, &P->yset))) return st;
  }
  if ((st = P->allocate_n(1, &P->st))) return st;
  if ((st = P->allocate_n(1, &P->agg_total))) return st;
  if ((st = P->allocate_n(2, &P->readback))) return st;
  static_assert(sizeof(DevStatus) % 8 == 0, "DevStatus is cleared in 8-byte words");
  HIP_TRY(launch_zero_u64(reinterpret_cast<unsigned long long*>(P->st), sizeof(DevStatus) / 8, P->stream));
  if ((st = plan_group_y(P, Y))) return st;
  return grouped ? plan_grouped(P, X) : plan_global(P, X);
}

// Argument checks shared by single and batched plans (section 2.2: paired
// modes must have equal length).
sptc_status check_problem(const sptc_coo* X, const sptc_coo* Y, int32_t ncontract, const int32_t* cx,
                          const int32_t* cy) {
  sptc_status st;
  if ((st = check_coo(X, "X"))) return st;
  if ((st = check_coo(Y, "Y"))) return st;
  if (ncontract < 0 || ncontract > X->order || ncontract > Y->order)
    return fail(SPTC_ERR_INVALID_ARG, "ncontract %d outside 0..min(order_X, order_Y)", ncontract);
  if (ncontract > 0 && (!cx || !cy)) return fail(SPTC_ERR_INVALID_ARG, "cx or cy is NULL");
  for (int32_t t = 0; t < ncontract; ++t) {
    if (cx[t] < 0 || cx[t] >= X->order) return fail(SPTC_ERR_INVALID_ARG, "cx[%d] = %d out of range", t, cx[t]);
    if (cy[t] < 0 || cy[t] >= Y->order) return fail(SPTC_ERR_INVALID_ARG, "cy[%d] = %d out of range", t, cy[t]);
    for (int32_t u = 0; u < t; ++u)
      if (cx[u] == cx[t] || cy[u] == cy[t]) return fail(SPTC_ERR_INVALID_ARG, "a mode is contracted twice");
  }
  for (int32_t t = 0; t < ncontract; ++t)
    if (X->dims[cx[t]] != Y->dims[cy[t]])
      return fail(SPTC_ERR_DIM_MISMATCH, "X mode %d has length %lld but Y mode %d has length %lld", cx[t],
                  (long long)X->dims[cx[t]], cy[t], (long long)Y->dims[cy[t]]);
  return SPTC_OK;
}

// Cells of a tensor's free key space (saturating): the product of its
// uncontracted mode lengths.
int64_t free_cells(const sptc_coo* T, int32_t ncontract, const int32_t* c) {
  std::vector<int32_t> fm;
  for (int32_t m = 0; m < T->order; ++m)
    if (std::find(c, c + ncontract, m) == c + ncontract) fm.push_back(m);
  return sat_prod(T->dims, fm);
}

void make_layout(const sptc_coo* X, const sptc_coo* Y, int32_t ncontract, const int32_t* cx, const int32_t* cy,
                 int32_t validate, Layout* L) {
  std::vector<int32_t> cxv(cx, cx + ncontract), cyv(cy, cy + ncontract), fx, fy;
  for (int32_t m = 0; m < X->order; ++m)
    if (std::find(cxv.begin(), cxv.end(), m) == cxv.end()) fx.push_back(m);
  for (int32_t m = 0; m < Y->order; ++m)
    if (std::find(cyv.begin(), cyv.end(), m) == cyv.end()) fy.push_back(m);
  int32_t bits_cy = 0;
  L->x_c = make_pack(X->dims, cxv, &L->bits_c);
  L->y_c = make_pack(Y->dims, cyv, &bits_cy);
  L->x_f = make_pack(X->dims, fx, &L->bits_fx);
  L->y_f = make_pack(Y->dims, fy, &L->bits_fy);
  // Small keys index their tables directly; the contracting key's choice
  // holds for X's probes of Y's table too.
  L->y_c.ident = L->x_c.ident = L->bits_c <= kIdentBits ? 1 : 0;
  L->x_f.ident = L->bits_fx <= kIdentBits ? 1 : 0;
  L->y_f.ident = 0;
  L->nfy = (int32_t)fy.size();
  L->out_order = (int32_t)(fx.size() + fy.size());
  int32_t k = 0;
  for (int32_t m : fx) L->out_dims[k++] = X->dims[m];
  for (int32_t m : fy) L->out_dims[k++] = Y->dims[m];
  add_unpack(L->ux, L->x_f, 0);
  add_unpack(L->uy, L->y_f, 0);
  L->ux.row0 = 0;
  L->uy.row0 = L->ux.n;  // Z's modes: X's free modes, then Y's
  L->ycells = (uint64_t)sat_prod(Y->dims, fy);
  L->c_cells = sat_prod(X->dims, cxv);
  L->fx_cells = sat_prod(X->dims, fx);
  L->xb = make_bounds(X, validate);
  L->yb = make_bounds(Y, validate);
}

sptc_status check_key_widths(const Layout& L, int32_t mode) {
  if (L.bits_c > 63 || L.bits_fx > 63 || L.bits_fy > 63)
    return fail(SPTC_ERR_KEY_OVERFLOW, "packed keys need %d (contracting), %d (X free), %d (Y free) bits; at most 63",
                L.bits_c, L.bits_fx, L.bits_fy);
  if (mode == SPTC_MODE_GLOBAL && L.bits_fx + L.bits_fy > 63)
    return fail(SPTC_ERR_KEY_OVERFLOW, "output key needs %d bits (> 63); the grouped mode handles it",
                L.bits_fx + L.bits_fy);
  return SPTC_OK;
}

// sptc_plan, or (br != nullptr) the plan of a batch's packed problem, whose
// key tables are cut into the batch's per-contraction regions.
sptc_status plan_create(sptc_plan_t* plan, const sptc_coo* X, const sptc_coo* Y, int32_t ncontract, const int32_t* cx,
                        const int32_t* cy, const sptc_options* opt, const sptc_allocator* alloc, void* stream,
                        const BatchRegions* br, bool pageable_readback = false) {
  if (!plan) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  *plan = nullptr;
  sptc_status st;
  if ((st = check_problem(X, Y, ncontract, cx, cy))) return st;
  sptc_options o;
  sptc_default_options(&o);
  if (opt) o = *opt;
  if ((st = check_options(o))) return st;
  if (alloc && (!alloc->alloc || !alloc->release))
    return fail(SPTC_ERR_INVALID_ARG, "allocator must provide alloc and release");
  if (o.capture_out_cap > 0 && !alloc)
    return fail(SPTC_ERR_INVALID_ARG, "capture_out_cap needs a caller allocator (the plan must not allocate from "
                                      "the stream's pool inside a graph capture)");
  if (o.capture_out_cap > 0 && br) return fail(SPTC_ERR_INVALID_ARG, "capture_out_cap is not for batches");
  // Operand order (section 5.4): the grouped mode groups X by its free key
  // and indexes each group's table by Y's free key, so it groups whichever
  // operand has the larger free key space.  With Y's the larger, X and Y
  // trade places here, and Z's rows are put back in X-then-Y order below.
  const bool swap = !br && o.mode == SPTC_MODE_GROUPED && o.operand_order == 0 &&
                    free_cells(Y, ncontract, cy) > free_cells(X, ncontract, cx);
  if (swap) {
    std::swap(X, Y);
    std::swap(cx, cy);
  }
  Layout L;
  make_layout(X, Y, ncontract, cx, cy, o.validate, &L);
  if (swap) {
    // Z's modes stay the caller's X free modes, then Y's: the grouped
    // operand's free coordinates (the caller's Y) go after the others
    int64_t dims[SPTC_MAX_OUT_ORDER];
    const int32_t nfx = L.ux.n, nfy = L.uy.n;
    for (int32_t m = 0; m < nfy; ++m) dims[m] = L.out_dims[nfx + m];
    for (int32_t m = 0; m < nfx; ++m) dims[nfy + m] = L.out_dims[m];
    for (int32_t m = 0; m < nfx + nfy; ++m) L.out_dims[m] = dims[m];
    L.uy.row0 = 0;
    L.ux.row0 = nfy;
  }
  if ((st = check_key_widths(L, o.mode))) return st;
  if (br) {  // regions decide direct addressing of X free keys per contraction
    if (o.mode != SPTC_MODE_GROUPED) return fail(SPTC_ERR_INTERNAL, "table regions need the grouped mode");
    L.x_f.ident = 0;
  }

  sptc_plan_s* P = new (std::nothrow) sptc_plan_s();
  if (!P) return fail(SPTC_ERR_OUT_OF_MEMORY, "host allocation failed");
  P->opt = o;
  P->in_batch = br != nullptr;
  P->capture = o.capture_out_cap > 0;
  if (P->capture) P->opt.block_mfma = 0;
  P->pageable_readback = pageable_readback;
  P->stream = static_cast<hipStream_t>(stream);
  if (alloc) {
    P->has_alloc = true;
    P->alloc = *alloc;
  }
  P->ox = X->order;
  P->oy = Y->order;
  P->nc = ncontract;
  P->nx = X->nnz;
  P->ny = Y->nnz;
  P->x_c = L.x_c;
  P->y_c = L.y_c;
  P->x_f = L.x_f;
  P->y_f = L.y_f;
  P->bits_c = L.bits_c;
  P->bits_fx = L.bits_fx;
  P->bits_fy = L.bits_fy;
  P->nfy = L.nfy;
  P->out_order = L.out_order;
  for (int32_t m = 0; m < L.out_order; ++m) P->out_dims[m] = L.out_dims[m];
  if (L.bits_fx + L.bits_fy <= 63) {  // packed output key (global mode, global class), fields in Z's row order
    if (swap) {
      add_unpack(P->out_unpack, P->y_f, 0);
      add_unpack(P->out_unpack, P->x_f, P->bits_fy);
    } else {
      add_unpack(P->out_unpack, P->x_f, P->bits_fy);
      add_unpack(P->out_unpack, P->y_f, 0);
    }
  }
  P->swapped = swap;
  add_unpack(P->ykey_unpack, P->y_c, 0);
  add_unpack(P->yfree_unpack, P->y_f, 0);
  P->y_agg = P->bits_c <= kAggBits ? 1 : 0;
  P->x_agg = (!br && o.mode == SPTC_MODE_GROUPED && P->bits_fx <= kAggBits) ? 1 : 0;
  P->ux = L.ux;
  P->uy = L.uy;
  P->ycells = L.ycells;
  P->dense = P->bits_fy <= kDenseBits ? 1 : 0;
  P->xb = L.xb;
  P->yb = L.yb;

  DeviceInfo* di = nullptr;
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "hipGetDevice");
  }
  if ((st = device_info(P->device, &di)) || (!P->has_alloc && (st = configure_pool(P->device, di)))) {
    delete P;
    return st;
  }
  P->num_cus = di->num_cus;

  st = plan_body(P, X, Y, cx, cy, br);
  if (st != SPTC_OK) {
    std::string msg = g_last_error;
    g_stalled = P->stalled;
    if (!P->stalled) (void)hipStreamSynchronize(P->stream);
    P->release_all();
    delete P;
    g_last_error = msg;
    return st;
  }
  *plan = P;
  return SPTC_OK;
}

// Outputs of a batch's packed plan: per-contraction COO regions, positions
// and nnz (out_nnz of execute_plan then only receives the packed total).
struct BatchExec {
  const BatchOut* bout;
  BatchSeg* bseg;
  int32_t bwx;
  int32_t count;
  int64_t* out_nnz;
};

sptc_status execute_plan(sptc_plan_s* P, int32_t* out_idx, double* out_val, int64_t out_cap, int64_t* out_nnz,
                         hipStream_t s, const BatchExec* bx) {
  if (bx) out_cap = INT64_MAX;  // capacity is checked per contraction
  if (P->opt.mode == SPTC_MODE_GROUPED) {
    HIP_TRY(launch_reset_status(P->st, P->queue, s));
    if (bx) HIP_TRY(launch_batch_reset(bx->count, bx->bseg, s));
    GroupArgs a{};
    a.groups = P->groups;
    a.xr = P->xr;
    a.eoff = P->eoff;
    a.yg = P->yg;
    a.ykey16 = P->ykey16;
    a.yval = P->yval;
    a.ny = P->ny;
    a.ycells = P->ycells;
    a.seed = P->opt.hash_seed;
    a.bits_y = P->bits_fy;
    a.ux = P->ux;
    a.uy = P->uy;
    a.out_idx = out_idx;
    a.out_val = out_val;
    a.out_cap = out_cap;
    a.st = P->st;
    if (bx) {
      a.bout = bx->bout;
      a.bseg = bx->bseg;
      a.bwx = bx->bwx;
    }
    HIP_TRY(mark(P, s, SPTC_STAGE_DIRECT, 0));
    HIP_TRY(launch_group_direct(a, P->drec, P->dpos, P->nd, (uint64_t)P->direct_products, P->dtfirst, P->num_cus, s,
                                P->opt.tile, P->capture ? P->st : nullptr, P->dtfirst_slots));
    HIP_TRY(mark(P, s, SPTC_STAGE_DIRECT, 1));
    HIP_TRY(mark(P, s, SPTC_STAGE_BLOCK, 0));
    // the wave class first: its outputs' positions come from a scan and
    // follow the direct class's; the later classes reserve theirs by atomics
    HIP_TRY(launch_wave_class(a, P->wlist, P->nw, P->wcnt, P->woff, P->tile_sums, P->num_cus, s));
    if (P->dense_rows)
      HIP_TRY(launch_group_block(a, P->blist, P->nb, P->num_cus, s, nullptr, dense_cells(P->bits_fy)));
    else if (P->dense && !P->block_mfma && P->nb > 0)
      HIP_TRY(launch_lds_queue(a, P->blist, P->nb, P->yso, P->ytab_slots, dense_cells(P->bits_fy), P->slice_cells,
                               P->queue, P->tcnt, P->toff, P->tsums, P->num_cus, s));
    if (P->block_mfma)
      HIP_TRY(launch_group_block_mfma(a, P->blist, P->nb, P->mplan, P->num_cus, s));
    else if (!P->dense)
      HIP_TRY(launch_group_block(a, P->blist, P->nb, P->num_cus, s, P->capture ? P->st : nullptr, 0u, P->bdefer,
                                 P->queue));
    HIP_TRY(mark(P, s, SPTC_STAGE_BLOCK, 1));
    if (P->ngl == 0) {
      HIP_TRY(mark(P, s, SPTC_STAGE_COMPACT, 0));
      if (bx)
        HIP_TRY(launch_batch_finalize(P->st, bx->bseg, bx->bout, bx->count, bx->out_nnz, s));
      else
        HIP_TRY(launch_finalize(out_nnz, out_cap, P->st, s));
      HIP_TRY(mark(P, s, SPTC_STAGE_COMPACT, 1));
      return SPTC_OK;
    }
  }
  const bool grouped = P->opt.mode == SPTC_MODE_GROUPED;
  const uint64_t zmask = (uint64_t)P->ztab_slots - 1;
  HIP_TRY(mark(P, s, SPTC_STAGE_OUT_CLEAR, 0));
  HIP_TRY(launch_fill_empty(P->ztab, P->ztab_slots, grouped ? nullptr : P->st, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_OUT_CLEAR, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_EXPAND, 0));
  // without read-backs the entry and product counts are read on the device
  const unsigned long long* dnx = P->capture && grouped ? &P->st->global_entries : nullptr;
  const unsigned long long* dprod =
      P->capture ? (grouped ? &P->st->global_products : &P->st->products) : nullptr;
  HIP_TRY(launch_expand_acc(P->poff, P->expand_nx, P->xrec, P->xg, P->yg, P->ny, P->bits_fy, P->ztab, zmask,
                            P->opt.hash_seed, P->max_probe_z, (uint64_t)P->expand_products, P->st, P->num_cus, s,
                            dnx, dprod));
  HIP_TRY(mark(P, s, SPTC_STAGE_EXPAND, 1));
  HIP_TRY(mark(P, s, SPTC_STAGE_COMPACT, 0));
  if (grouped) {
    HIP_TRY(launch_compact_grouped(P->ztab, P->ztab_slots, P->groups, P->glist, P->ux, P->uy, P->bits_fy, out_idx,
                                   out_val, out_cap, out_nnz, &P->st->out_base, P->ztile_sums, P->st,
                                   bx ? bx->bout : nullptr, bx ? bx->bseg : nullptr, bx ? bx->bwx : 0, s));
    if (bx) HIP_TRY(launch_batch_finalize(P->st, bx->bseg, bx->bout, bx->count, bx->out_nnz, s));
  } else
    HIP_TRY(launch_compact(P->ztab, P->ztab_slots, P->out_unpack, out_idx, out_val, out_cap, out_nnz, nullptr,
                           P->ztile_sums, P->st, s));
  HIP_TRY(mark(P, s, SPTC_STAGE_COMPACT, 1));
  return SPTC_OK;
}

constexpr int32_t kBatchMax = 4096;  // k_batch_unpack keeps 12 bytes per contraction in LDS
constexpr int64_t kPackTile = 8192;

int64_t layout_cells(const Layout& L) {
  int64_t cells = 1;
  for (int32_t m = 0; m < L.out_order; ++m) {
    if (cells > ((int64_t)1 << 62) / L.out_dims[m]) return (int64_t)1 << 62;
    cells *= L.out_dims[m];
  }
  return cells;
}

// A contraction's region of a batch key table, for n keys of `bits` bits:
// directly addressed when that costs at most 4x the hashed size.
Region make_region(int32_t bits, int64_t n, double load_factor, uint64_t* next_base) {
  const int64_t hashed = pow2_at_least((double)std::max<int64_t>(n, 1) / load_factor);
  Region r{};
  r.base = *next_base;
  if (bits <= kIdentBits && ((int64_t)1 << bits) <= 4 * hashed) {
    r.mask = (uint32_t)(std::max<int64_t>((int64_t)1 << bits, 2) - 1);
    r.ident = 1;
  } else {
    r.mask = (uint32_t)(hashed - 1);
    r.ident = 0;
  }
  *next_base += (uint64_t)r.mask + 1;
  return r;
}

// Packs every contraction's entries with its index as key prefix, plans the
// packed problem, then sizes each contraction's output from its products.
sptc_status batch_body(sptc_batch_s* B, const sptc_coo* X, const sptc_coo* Y, const sptc_options& o) {
  const hipStream_t s = B->stream;
  const int32_t count = B->count;
  const int32_t wb = bits_for(count);
  int32_t wc = 0, wx = 0, wy = 0;
  int64_t nx = 0, ny = 0;
  for (const auto& it : B->items) {
    wc = std::max(wc, it.L.bits_c);
    wx = std::max(wx, it.L.bits_fx);
    wy = std::max(wy, it.L.bits_fy);
  }
  if (wb + wc > 62 || wb + wx > 62 || wy > 62)
    return fail(SPTC_ERR_KEY_OVERFLOW, "batch keys need %d (contracting), %d (X free), %d (Y free) bits; at most 62",
                wb + wc, wb + wx, wy);
  B->w.wc = wc;
  B->w.wx = wx;
  B->w.wy = wy;
  B->w.lo_c = std::min(wb + wc, 31);
  B->w.lo_x = std::min(wb + wx, 31);
  B->w.lo_y = std::min(wy, 31);

  std::vector<BatchIn> in(count);
  std::vector<PackTile> tiles;
  for (int32_t b = 0; b < count; ++b) {
    const Layout& L = B->items[b].L;
    BatchIn& d = in[b];
    d.xidx = X[b].idx;
    d.xval = X[b].val;
    d.yidx = Y[b].idx;
    d.yval = Y[b].val;
    d.nx = X[b].nnz;
    d.ny = Y[b].nnz;
    d.xoff = nx;
    d.yoff = ny;
    d.xc = L.x_c;
    d.yc = L.y_c;
    d.xf = L.x_f;
    d.yf = L.y_f;
    d.xb = L.xb;
    d.yb = L.yb;
    for (int64_t e = 0; e < d.nx; e += kPackTile) tiles.push_back({b, 0, e, std::min(d.nx, e + kPackTile)});
    for (int64_t e = 0; e < d.ny; e += kPackTile) tiles.push_back({b, 1, e, std::min(d.ny, e + kPackTile)});
    nx += d.nx;
    ny += d.ny;
  }
  if (nx > (int64_t)0xfffffffeLL || ny > (int64_t)0xfffffffeLL)
    return fail(SPTC_ERR_INVALID_ARG, "batch holds %lld X and %lld Y entries; at most 2^32-2 each", (long long)nx,
                (long long)ny);

  // Packed inputs live only until the packed plan has copied what it needs.
  Workspace pk;
  pk.stream = s;
  pk.has_alloc = B->has_alloc;
  pk.alloc = B->alloc;
  struct Release {
    Workspace& w;
    ~Release() { w.release_all(); }
  } release{pk};
  BatchIn* in_d = nullptr;
  PackTile* tiles_d = nullptr;
  int32_t *px = nullptr, *py = nullptr;
  double *pxv = nullptr, *pyv = nullptr;
  unsigned* err = nullptr;
  sptc_status st;
  if ((st = pk.allocate_n(count, &in_d))) return st;
  if ((st = pk.allocate_n((int64_t)tiles.size(), &tiles_d))) return st;
  if ((st = pk.allocate_n(4 * nx, &px))) return st;
  if ((st = pk.allocate_n(nx, &pxv))) return st;
  if ((st = pk.allocate_n(4 * ny, &py))) return st;
  if ((st = pk.allocate_n(ny, &pyv))) return st;
  if ((st = pk.allocate_n(1, &err))) return st;
  HIP_TRY(hipMemcpyAsync(in_d, in.data(), sizeof(BatchIn) * count, hipMemcpyHostToDevice, s));
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(tiles_d, tiles.data(), sizeof(PackTile) * tiles.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(unsigned), s));
  HIP_TRY(mark_events(o.stage_events, s, SPTC_STAGE_BATCH_PACK, 0));
  HIP_TRY(launch_batch_pack(in_d, tiles_d, (int64_t)tiles.size(), B->w, px, pxv, nx, py, pyv, ny, err, s));
  HIP_TRY(mark_events(o.stage_events, s, SPTC_STAGE_BATCH_PACK, 1));
  unsigned herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((st = status_from_bits(herr))) return st;

  const int32_t kc = wb + wc, kx = wb + wx;
  const int64_t xdims[4] = {(int64_t)1 << (kc - B->w.lo_c), (int64_t)1 << B->w.lo_c, (int64_t)1 << (kx - B->w.lo_x),
                            (int64_t)1 << B->w.lo_x};
  const int64_t ydims[4] = {xdims[0], xdims[1], (int64_t)1 << (wy - B->w.lo_y), (int64_t)1 << B->w.lo_y};
  const sptc_coo PX{4, xdims, nx, px, pxv}, PY{4, ydims, ny, py, pyv};
  const int32_t cmodes[2] = {0, 1};
  sptc_options io = o;
  io.validate = 0;  // packed coordinates are in range by construction; the pack checked the originals
  BatchRegions br;
  br.xshift = wx;
  uint64_t xbase = 0;
  for (int32_t b = 0; b < count; ++b) {
    const Layout& L = B->items[b].L;
    br.x.push_back(make_region(L.bits_fx, std::min<int64_t>(in[b].nx, L.fx_cells), o.load_factor, &xbase));
  }
  sptc_plan_t inner = nullptr;
  if ((st = plan_create(&inner, &PX, &PY, 2, cmodes, cmodes, &io, B->has_alloc ? &B->alloc : nullptr, s, &br)))
    return st;
  B->inner = inner;

  // Products per contraction, from the packed plan's X groups.
  unsigned long long* pb = nullptr;
  if ((st = pk.allocate_n(count, &pb))) return st;
  HIP_TRY(mark_events(o.stage_events, s, SPTC_STAGE_BATCH_SEGMENTS, 0));
  HIP_TRY(launch_zero_u64(pb, count, s));
  HIP_TRY(launch_batch_products(inner->groups, inner->x_groups, inner->eoff, wx, count, pb, s));
  std::vector<unsigned long long> hpb(count);
  HIP_TRY(hipMemcpyAsync(hpb.data(), pb, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t total = 0;
  std::vector<BatchOut> outs(count);
  for (int32_t b = 0; b < count; ++b) {
    auto& it = B->items[b];
    it.products = (int64_t)hpb[b];
    total += it.products;
    it.bound = std::min<int64_t>(it.products, layout_cells(it.L));
    it.idx_off = B->idx_elems;
    it.val_off = B->val_elems;
    B->idx_elems += (int64_t)it.L.out_order * it.bound;
    B->val_elems += it.bound;
    outs[b].ux = it.L.ux;
    outs[b].uy = it.L.uy;
    outs[b].idx_off = it.idx_off;
    outs[b].val_off = it.val_off;
    outs[b].cap = it.bound;
  }
  if (total != inner->products)
    return fail(SPTC_ERR_INTERNAL, "per-contraction products add up to %lld, not %lld", (long long)total,
                (long long)inner->products);
  if ((st = B->allocate_n(count, &B->outs))) return st;
  if ((st = B->allocate_n(count, &B->seg))) return st;
  if ((st = B->allocate_n(1, &B->tnnz))) return st;
  HIP_TRY(hipMemcpyAsync(B->outs, outs.data(), sizeof(BatchOut) * count, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_batch_segments(inner->groups, inner->dlist, inner->nd, inner->dpos, wx, count, B->seg, s));
  HIP_TRY(mark_events(o.stage_events, s, SPTC_STAGE_BATCH_SEGMENTS, 1));
  HIP_TRY(hipStreamSynchronize(s));  // host arrays above are copied before they go out of scope
  return SPTC_OK;
}

}  // namespace

namespace sptc {

// Bump allocation over a caller-given device range: buffers are carved in
// order and never given back one by one (the range is reused by the next
// call).  `need` keeps the bytes asked for, also past the end.
struct ScratchBump {
  char* base;
  size_t cap, used, need;
};

void* scratch_alloc(size_t bytes, void* /*stream*/, void* ctx) {
  ScratchBump* b = static_cast<ScratchBump*>(ctx);
  const size_t n = (bytes + 255) & ~(size_t)255;
  b->need += n;
  if (b->used + n > b->cap) return nullptr;
  void* p = b->base + b->used;
  b->used += n;
  return p;
}

void scratch_release(void*, size_t, void*, void*) {}

// One contraction planned, executed and released with every workspace
// buffer carved from [base, base + bytes) and the plan's count read-backs
// through pageable memory, so that nothing is allocated: the body of
// sptc_contract_noalloc.
sptc_status contract_in_scratch(void* base, size_t bytes, const sptc_coo* X, const sptc_coo* Y, int32_t ncontract,
                                const int32_t* cx, const int32_t* cy, const sptc_options* opt, int32_t* out_idx,
                                double* out_val, int64_t out_cap, int64_t* out_nnz, void* stream) {
  if (!out_nnz) return fail(SPTC_ERR_INVALID_ARG, "out_nnz is NULL");
  if (out_cap < 0) return fail(SPTC_ERR_INVALID_ARG, "out_cap < 0");
  ScratchBump bump{static_cast<char*>(base), bytes, 0, 0};
  const sptc_allocator al{scratch_alloc, scratch_release, &bump};
  sptc_plan_t plan = nullptr;
  sptc_status st = plan_create(&plan, X, Y, ncontract, cx, cy, opt, &al, stream, nullptr, true);
  if (st == SPTC_ERR_OUT_OF_MEMORY && bump.need > bump.cap)
    return fail(SPTC_ERR_CAPACITY, "the plan needs more workspace than the %zu bytes of static scratch (%zu bytes asked "
                "for when it stopped)", bump.cap, bump.need);
  if (st != SPTC_OK) return st;
  if (out_cap > 0 && !out_val) st = fail(SPTC_ERR_INVALID_ARG, "out_val is NULL");
  else if (out_cap > 0 && plan->out_order > 0 && !out_idx) st = fail(SPTC_ERR_INVALID_ARG, "out_idx is NULL");
  else st = execute_plan(plan, out_idx, out_val, out_cap, out_nnz, static_cast<hipStream_t>(stream), nullptr);
  sptc_free(plan);
  return st;
}

sptc_status report_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }

}  // namespace sptc

extern "C" {

void sptc_default_options(sptc_options* opt) {
  if (!opt) return;
  opt->load_factor = 1.0 / 1.3;
  opt->validate = 1;
  opt->max_probe = 0;
  opt->hash_seed = 0x9e3779b97f4a7c15ull;
  opt->out_table_slots = 0;
  opt->stage_events = nullptr;
  opt->mode = SPTC_MODE_GROUPED;
  opt->block_mfma = 0;
  opt->tile = 0;
  opt->lds_max_keys = 0;
  opt->capture_out_cap = 0;
  opt->operand_order = 0;
}

sptc_status sptc_plan(sptc_plan_t* plan, const sptc_coo* X, const sptc_coo* Y, int32_t ncontract, const int32_t* cx,
                      const int32_t* cy, const sptc_options* opt, const sptc_allocator* alloc, void* stream) {
  return plan_create(plan, X, Y, ncontract, cx, cy, opt, alloc, stream, nullptr);
}

sptc_status sptc_plan_info(sptc_plan_t P, sptc_info* info) {
  if (!P || !info) return fail(SPTC_ERR_INVALID_ARG, "plan or info is NULL");
  std::memset(info, 0, sizeof *info);
  info->out_order = P->out_order;
  for (int32_t m = 0; m < P->out_order; ++m) info->out_dims[m] = P->out_dims[m];
  info->products = P->products;
  info->out_nnz_bound = P->out_bound;
  info->y_groups = P->y_groups;
  info->y_table_slots = P->ytab_slots;
  info->out_table_slots = P->ztab_slots;
  info->workspace_bytes = P->workspace;
  info->key_bits_contract = P->bits_c;
  info->key_bits_x_free = P->bits_fx;
  info->key_bits_y_free = P->bits_fy;
  info->mode = P->opt.mode;
  info->x_groups = P->x_groups;
  info->direct_groups = P->nd;
  info->direct_products = P->direct_products;
  info->wave_groups = P->nw;
  info->block_groups = P->nb;
  info->global_groups = P->ngl;
  info->block_mfma = P->block_mfma;
  info->block_mfma_work = P->block_mfma ? (int64_t)mfma_work(P->nb, P->mplan.ncols, P->y_groups) : 0;
  info->block_tiles_scanned = P->tcnt != nullptr;
  info->operands_swapped = P->swapped ? 1 : 0;
  info->block_dense_rows = P->dense_rows ? 1 : 0;
  return SPTC_OK;
}

sptc_status sptc_execute(sptc_plan_t P, int32_t* out_idx, double* out_val, int64_t out_cap, int64_t* out_nnz,
                         void* stream) {
  if (!P) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  if (!out_nnz) return fail(SPTC_ERR_INVALID_ARG, "out_nnz is NULL");
  if (out_cap < 0) return fail(SPTC_ERR_INVALID_ARG, "out_cap < 0");
  if (out_cap > 0 && !out_val) return fail(SPTC_ERR_INVALID_ARG, "out_val is NULL");
  if (out_cap > 0 && P->out_order > 0 && !out_idx) return fail(SPTC_ERR_INVALID_ARG, "out_idx is NULL");
  return execute_plan(P, out_idx, out_val, out_cap, out_nnz, static_cast<hipStream_t>(stream), nullptr);
}

sptc_status sptc_plan_set_stage_events(sptc_plan_t P, void** events) {
  if (!P) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  P->opt.stage_events = events;
  return SPTC_OK;
}

sptc_status sptc_plan_status(sptc_plan_t P, void* stream) {
  if (!P) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  DevStatus host{};
  HIP_TRY(hipMemcpyAsync(&host, P->st, sizeof host, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return status_from_bits(host.err);
}

void sptc_free(sptc_plan_t P) {
  if (!P) return;
  P->release_all();
  delete P;
}

const char* sptc_status_string(sptc_status s) {
  switch (s) {
    case SPTC_OK: return "success";
    case SPTC_ERR_INVALID_ARG: return "invalid argument";
    case SPTC_ERR_DIM_MISMATCH: return "contracted modes have different lengths";
    case SPTC_ERR_KEY_OVERFLOW: return "packed key wider than 63 bits";
    case SPTC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SPTC_ERR_CAPACITY: return "hash table or output capacity exceeded";
    case SPTC_ERR_HIP: return "HIP runtime error";
    case SPTC_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* sptc_last_error(void) { return g_last_error.c_str(); }

sptc_status sptc_plan_y_groups(sptc_plan_t P, int32_t* key_coords, int64_t* counts, int64_t* starts, int64_t cap,
                               int64_t* ngroups, void* stream) {
  if (!P || !ngroups) return fail(SPTC_ERR_INVALID_ARG, "plan or ngroups is NULL");
  *ngroups = P->y_groups;
  if (P->y_groups > cap) return fail(SPTC_ERR_CAPACITY, "%lld groups exceed cap %lld", (long long)P->y_groups,
                                     (long long)cap);
  if (cap > 0 && (!counts || !starts || (P->nc > 0 && !key_coords)))
    return fail(SPTC_ERR_INVALID_ARG, "output pointer is NULL");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_y_groups(P->ytab, P->ytab_slots, P->ykey_unpack, key_coords, counts, starts, cap, P->readback,
                          P->tile_sums, P->st, s));
  int64_t n = 0;
  HIP_TRY(hipMemcpyAsync(&n, P->readback, sizeof n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (n != P->y_groups) return fail(SPTC_ERR_INTERNAL, "group count %lld != %lld", (long long)n,
                                    (long long)P->y_groups);
  return SPTC_OK;
}

sptc_status sptc_plan_y_grouped(sptc_plan_t P, int32_t* free_coords, double* vals, void* stream) {
  if (!P) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  if (P->ny > 0 && (!vals || (P->nfy > 0 && !free_coords))) return fail(SPTC_ERR_INVALID_ARG, "output is NULL");
  HIP_TRY(launch_y_grouped(P->yg, P->ny, P->yfree_unpack, free_coords, vals, static_cast<hipStream_t>(stream)));
  return SPTC_OK;
}

sptc_status sptc_plan_x_groups(sptc_plan_t P, int32_t* free_coords, int64_t* counts, int64_t* products, int64_t cap,
                               int64_t* ngroups, void* stream) {
  if (!P || !ngroups) return fail(SPTC_ERR_INVALID_ARG, "plan or ngroups is NULL");
  if (P->opt.mode != SPTC_MODE_GROUPED) return fail(SPTC_ERR_INVALID_ARG, "the plan does not group X");
  *ngroups = P->x_groups;
  if (P->x_groups > cap)
    return fail(SPTC_ERR_CAPACITY, "%lld groups exceed cap %lld", (long long)P->x_groups, (long long)cap);
  if (P->x_groups > 0 && (!counts || !products || (P->ux.n > 0 && !free_coords)))
    return fail(SPTC_ERR_INVALID_ARG, "output pointer is NULL");
  HIP_TRY(launch_x_groups(P->groups, P->x_groups, P->eoff, P->ux, free_coords, counts, products, cap,
                          static_cast<hipStream_t>(stream)));
  return SPTC_OK;
}

sptc_status sptc_plan_x_counts(sptc_plan_t P, int64_t* counts, void* stream) {
  if (!P) return fail(SPTC_ERR_INVALID_ARG, "plan is NULL");
  if (P->opt.mode != SPTC_MODE_GLOBAL) return fail(SPTC_ERR_INVALID_ARG, "per-X counts exist in global mode only");
  if (P->nx > 0 && !counts) return fail(SPTC_ERR_INVALID_ARG, "counts is NULL");
  HIP_TRY(launch_x_counts(P->poff, P->nx, counts, static_cast<hipStream_t>(stream)));
  return SPTC_OK;
}

sptc_status sptc_batch_plan(sptc_batch_t* batch, int32_t count, const sptc_coo* X, const sptc_coo* Y,
                            const int32_t* ncontract, const int32_t* const* cx, const int32_t* const* cy,
                            const sptc_options* opt, const sptc_allocator* alloc, void* stream) {
  if (!batch) return fail(SPTC_ERR_INVALID_ARG, "batch is NULL");
  *batch = nullptr;
  if (count < 1 || count > kBatchMax) return fail(SPTC_ERR_INVALID_ARG, "count %d outside 1..%d", count, kBatchMax);
  if (!X || !Y || !ncontract || !cx || !cy) return fail(SPTC_ERR_INVALID_ARG, "a batch array is NULL");
  sptc_options o;
  sptc_default_options(&o);
  if (opt) o = *opt;
  sptc_status st;
  if ((st = check_options(o))) return st;
  if (o.mode != SPTC_MODE_GROUPED) return fail(SPTC_ERR_INVALID_ARG, "batches run in the grouped mode only");
  if (alloc && (!alloc->alloc || !alloc->release))
    return fail(SPTC_ERR_INVALID_ARG, "allocator must provide alloc and release");
  sptc_batch_s* B = new (std::nothrow) sptc_batch_s();
  if (!B) return fail(SPTC_ERR_OUT_OF_MEMORY, "host allocation failed");
  B->count = count;
  B->items.resize(count);
  for (int32_t b = 0; b < count; ++b) {
    st = check_problem(&X[b], &Y[b], ncontract[b], cx[b], cy[b]);
    if (st == SPTC_OK) {
      make_layout(&X[b], &Y[b], ncontract[b], cx[b], cy[b], o.validate, &B->items[b].L);
      st = check_key_widths(B->items[b].L, o.mode);
    }
    if (st != SPTC_OK) {
      g_last_error = "contraction " + std::to_string(b) + ": " + g_last_error;
      delete B;
      return st;
    }
  }
  B->stream = static_cast<hipStream_t>(stream);
  if (alloc) {
    B->has_alloc = true;
    B->alloc = *alloc;
  }
  g_stalled = false;
  st = batch_body(B, X, Y, o);
  if (st != SPTC_OK) {
    std::string msg = g_last_error;
    if (!g_stalled) (void)hipStreamSynchronize(B->stream);
    if (B->inner) sptc_free(B->inner);
    B->release_all();
    delete B;
    g_last_error = msg;
    return st;
  }
  *batch = B;
  return SPTC_OK;
}

sptc_status sptc_batch_sizes(sptc_batch_t B, int64_t* idx_elems, int64_t* val_elems, int64_t* workspace_bytes) {
  if (!B) return fail(SPTC_ERR_INVALID_ARG, "batch is NULL");
  if (idx_elems) *idx_elems = B->idx_elems;
  if (val_elems) *val_elems = B->val_elems;
  if (workspace_bytes) *workspace_bytes = B->workspace + (B->inner ? B->inner->workspace : 0);
  return SPTC_OK;
}

sptc_status sptc_batch_info(sptc_batch_t B, int32_t b, sptc_info* info, int64_t* idx_offset, int64_t* val_offset) {
  if (!B) return fail(SPTC_ERR_INVALID_ARG, "batch is NULL");
  if (b < 0 || b >= B->count) return fail(SPTC_ERR_INVALID_ARG, "contraction %d outside 0..%d", b, B->count - 1);
  const auto& it = B->items[b];
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->out_order = it.L.out_order;
    for (int32_t m = 0; m < it.L.out_order; ++m) info->out_dims[m] = it.L.out_dims[m];
    info->products = it.products;
    info->out_nnz_bound = it.bound;
    info->key_bits_contract = it.L.bits_c;
    info->key_bits_x_free = it.L.bits_fx;
    info->key_bits_y_free = it.L.bits_fy;
  }
  if (idx_offset) *idx_offset = it.idx_off;
  if (val_offset) *val_offset = it.val_off;
  return SPTC_OK;
}

sptc_status sptc_batch_execute(sptc_batch_t B, int32_t* out_idx, double* out_val, int64_t* out_nnz, void* stream) {
  if (!B) return fail(SPTC_ERR_INVALID_ARG, "batch is NULL");
  if (!out_nnz) return fail(SPTC_ERR_INVALID_ARG, "out_nnz is NULL");
  if (B->val_elems > 0 && !out_val) return fail(SPTC_ERR_INVALID_ARG, "out_val is NULL");
  if (B->idx_elems > 0 && !out_idx) return fail(SPTC_ERR_INVALID_ARG, "out_idx is NULL");
  const BatchExec bx{B->outs, B->seg, B->w.wx, B->count, out_nnz};
  return execute_plan(B->inner, out_idx, out_val, 0, B->tnnz, static_cast<hipStream_t>(stream), &bx);
}

sptc_status sptc_pool_trim(size_t keep_bytes) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  sptc_status st = cache_trim(dev, keep_bytes);
  if (st != SPTC_OK) return st;
  hipMemPool_t pool;
  HIP_TRY(hipDeviceGetDefaultMemPool(&pool, dev));
  HIP_TRY(hipMemPoolTrimTo(pool, keep_bytes));
  return SPTC_OK;
}

void sptc_batch_free(sptc_batch_t B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->stream);
  if (B->inner) sptc_free(B->inner);
  B->release_all();
  delete B;
}

}  // extern "C"
