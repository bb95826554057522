// X grouping by partition (xpart.hip): declarations for the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sptc_internal.hpp"

namespace sptc {

constexpr int kPTile = 16384;                          // X entries per partition tile
constexpr int kPartMaxBits = 14;                       // at most 16,384 buckets
constexpr int64_t kPartMaxEntries = (int64_t)150 << 20;  // beyond: buckets could outgrow their LDS tables

// Workspace of launch_x_partition for nnz X entries (device, caller-owned):
// pkey[nnz] and prec[nnz] (the partitioned keys and X records),
// hist[2^part_bits(nnz) * part_tiles(nnz)], and scan scratch for the
// histogram's scan (scan_tiles(n) + 1 64-bit values).
struct XPartBuffers {
  unsigned* pkey;
  XRec* prec;
  unsigned* hist;
  void* scan;
};

int part_bits(int64_t nnz);
int64_t part_tiles(int64_t nnz);

// Raises the partition kernels' dynamic LDS limits on the current device.
hipError_t prepare_x_partition();

// X grouped by its free key (at most 31 bits, hashed, one contraction, nnz
// <= kPartMaxEntries): groups[0, xgroups) and the grouped X records xr[nnz],
// st->xgroups (counted up: zero on entry), and st->nonfinite when an X value
// is not finite; with b.check, coordinates out of range are recorded.
hipError_t launch_x_partition(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                              const YSlot* ytab, TabGeom yg, int32_t max_probe_y, uint64_t seed, const XPartBuffers& w,
                              GroupRec* groups, XRec* xr, DevStatus* st, int num_cus, hipStream_t stream);

}  // namespace sptc
