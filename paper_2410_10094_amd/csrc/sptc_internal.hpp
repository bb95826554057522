// Internal types shared by the host runtime (sptc.cpp) and the kernels
// (kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sptc {

constexpr uint64_t kEmpty = ~0ull;  // key of an unused hash slot; real keys use <= 63 bits
constexpr int kMaxOrder = 16;
constexpr int kMaxOutOrder = 32;

// Error bits recorded by kernels in the plan's status word.
enum : uint32_t {
  kErrCapacity = 1u,   // probe limit hit, or more outputs than out_cap
  kErrCoord = 2u,      // coordinate outside its mode length (validation on)
  kErrInternal = 4u,   // a key that must be present was not found
};

// Packs chosen modes of one COO tensor into a 64-bit key: coordinate of
// mode[k] lands at bit shift[k] (the first listed mode is most significant).
struct KeyPack {
  int32_t n;
  int32_t mode[kMaxOrder];
  int32_t shift[kMaxOrder];
  uint32_t mask[kMaxOrder];  // (1 << bits) - 1: keeps any coordinate inside its field
};

// Coordinate bounds of one tensor (validation).
struct Bounds {
  int32_t order;
  uint32_t dim[kMaxOrder];  // mode lengths (<= 2^31)
  int32_t check;            // nonzero: validate
};

// Decodes an output key into out_order coordinates.
struct KeyUnpack {
  int32_t n;
  int32_t shift[kMaxOutOrder];
  uint32_t mask[kMaxOutOrder];
};

// Slot of the Y contracting-key table: key, number of Y entries with that
// key, and (after the scan and scatter) the start of their run in Yg.
struct alignas(16) YSlot {
  unsigned long long key;
  unsigned int count;
  unsigned int start;
};

// Slot of the output hash: packed output key and accumulated value.
struct alignas(16) ZSlot {
  unsigned long long key;
  double val;
};

// A grouped Y entry: packed Y free coordinates and value.
struct alignas(16) YEntry {
  unsigned long long phi;
  double v;
};

// An X entry as the expansion reads it: packed X free coordinates and value.
struct alignas(16) XEntry {
  unsigned long long phi;
  double v;
};

// Device-side scalars of a plan.
struct alignas(16) DevStatus {
  unsigned long long products;  // P
  unsigned long long groups;    // distinct contracting keys of Y
  unsigned int err;             // kErr* bits
  unsigned int pad[3];
};

// ---- launchers (kernels.hip) ----
// Each returns the hipError_t of its launch(es); all work goes on `stream`.

// Sets every 16-byte slot to {key = kEmpty, 0}; clears st->err when st is given.
hipError_t launch_fill_empty(void* slots16, int64_t nslots, DevStatus* st, hipStream_t stream);

hipError_t launch_y_count(const int32_t* yidx, int64_t nnz, KeyPack kc, YSlot* tab, uint64_t mask,
                          uint64_t seed, int32_t max_probe, DevStatus* st, int num_cus, hipStream_t stream);

// Exclusive scan support: tile sums need ceil(n / kScanTile) u64 entries.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// Y table: count field -> inclusive end offset stored in `start`.
hipError_t launch_scan_y_table(YSlot* tab, int64_t nslots, unsigned long long* tile_sums, hipStream_t stream);

hipError_t launch_y_scatter(const int32_t* yidx, const double* yval, int64_t nnz, KeyPack kc, KeyPack kf,
                            Bounds b, YSlot* tab, uint64_t mask, uint64_t seed, int32_t max_probe, YEntry* yg,
                            DevStatus* st, int num_cus, hipStream_t stream);

hipError_t launch_x_probe(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                          const YSlot* tab, uint64_t mask, uint64_t seed, int32_t max_probe, XEntry* xrec,
                          uint32_t* xg, uint32_t* xcnt, DevStatus* st, int num_cus, hipStream_t stream);

// poff[i] = sum of xcnt[0..i), poff[n] = P, and P also into st->products.
hipError_t launch_scan_products(const uint32_t* xcnt, int64_t n, unsigned long long* poff,
                                unsigned long long* tile_sums, DevStatus* st, hipStream_t stream);

hipError_t launch_expand_acc(const unsigned long long* poff, int64_t nx, const XEntry* xrec, const uint32_t* xg,
                             const YEntry* yg, int64_t ny, int32_t bits_y, ZSlot* tab, uint64_t mask, uint64_t seed,
                             int32_t max_probe, uint64_t products, DevStatus* st, int num_cus,
                             hipStream_t stream);

// Two-pass compaction of the output hash to COO; writes nnz (or the negated
// status on error) to *out_nnz.
hipError_t launch_compact(const ZSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* out_idx, double* out_val,
                          int64_t out_cap, int64_t* out_nnz, unsigned long long* tile_sums, DevStatus* st,
                          hipStream_t stream);

// Inspection helpers.
hipError_t launch_y_groups(const YSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* key_coords, int64_t* counts,
                           int64_t* starts, int64_t cap, int64_t* ngroups_dev, unsigned long long* tile_sums,
                           DevStatus* st, hipStream_t stream);
hipError_t launch_y_grouped(const YEntry* yg, int64_t nnz, KeyUnpack ku, int32_t* free_coords, double* vals,
                            hipStream_t stream);
hipError_t launch_x_counts(const unsigned long long* poff, int64_t nx, int64_t* counts, hipStream_t stream);

}  // namespace sptc
