// Internal types shared by the host runtime (sptc.cpp) and the kernels
// (kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sptc {

constexpr uint64_t kEmpty = ~0ull;  // key of an unused hash slot; real keys use <= 63 bits
struct BatchOut;
struct BatchSeg;

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
// One word per field (mode < 16, shift < 64, width < 32 as bytes 0, 1, 2),
// so that a kernel's argument block stays small and a field with a uniform
// index is one scalar load.
struct KeyPack {
  int32_t n;
  int32_t ident;              // the table keyed by this pack is direct-addressed (slot = key)
  uint32_t field[kMaxOrder];  // make_field(mode, shift, width): a coordinate keeps its low `width` bits
};

__host__ __device__ inline uint32_t make_field(uint32_t mode, uint32_t shift, uint32_t bits) {
  return mode | shift << 8 | bits << 16;
}
__host__ __device__ inline uint32_t field_mode(uint32_t f) { return f & 0xffu; }
__host__ __device__ inline uint32_t field_shift(uint32_t f) { return (f >> 8) & 0xffu; }
__host__ __device__ inline uint32_t field_bits(uint32_t f) { return (f >> 16) & 0xffu; }

// Mask of a field `bits` wide (bits <= 31).
__host__ __device__ inline uint32_t field_mask(uint32_t bits) { return (1u << bits) - 1u; }

// Coordinate stored in field f of `key`.
__host__ __device__ inline int32_t key_field(uint64_t key, uint32_t f) {
  return (int32_t)((uint32_t)(key >> field_shift(f)) & field_mask(field_bits(f)));
}

// Keys of at most this many bits index their table directly (no hashing,
// no probing); of at most kAggBits bits, their counting and placement are
// also aggregated per workgroup in LDS before touching the table.
constexpr int kIdentBits = 16;
constexpr int kAggBits = 13;
constexpr int kAggChunk = 4096;  // entries per workgroup of the aggregated count and placement

inline int64_t agg_chunks(int64_t nnz) { return (nnz + kAggChunk - 1) / kAggChunk; }

// Coordinate bounds of one tensor (validation).
struct Bounds {
  int32_t order;
  uint32_t dim[kMaxOrder];  // mode lengths (<= 2^31)
  int32_t check;            // nonzero: validate
};

// Geometry of an open-addressing key table.  A single contraction's table
// is one power-of-two array (hashed, or directly addressed when `ident`).
// A batch's table is cut into one region per contraction: a key's region is
// reg[key >> pshift], and probing wraps inside the region.
struct Region {
  unsigned long long base;  // first slot
  uint32_t mask;            // slots - 1 (a power of two)
  int32_t ident;            // directly addressed by the key's low bits
};

struct TabGeom {
  uint64_t mask;      // whole table (reg == nullptr)
  const Region* reg;  // regions, or nullptr
  int32_t pshift;     // key >> pshift selects the region
  int32_t ident;      // whole table directly addressed (reg == nullptr)
};

// Decodes an output key into out_order coordinates.
struct KeyUnpack {
  int32_t n;
  int32_t row0;                  // output row (coordinate mode of Z) of field 0; field m goes to row0 + m
  uint32_t field[kMaxOutOrder];  // make_field(0, shift, width)
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

// A grouped X entry (X grouped by free key): its Y group (start, count) and value.
struct alignas(16) XRec {
  unsigned int ystart;
  unsigned int ycnt;
  double v;
};

// A direct-class group as the direct kernel stages it, written at its
// place in the direct list when the groups are classified: its X free key,
// its one X entry's value and the start of that entry's Y run.
struct DRec {
  unsigned long long phi;
  double v;
  uint32_t ystart;
  uint32_t pad;
};

// An X group: packed X free key, and its run [start, start + count) of XRec.
struct alignas(16) GroupRec {
  unsigned long long phi;
  unsigned int start;
  unsigned int count;
};

// Device-side scalars of a plan.
struct alignas(16) DevStatus {
  unsigned long long products;         // P
  unsigned long long groups;           // distinct contracting keys of Y
  unsigned long long xgroups;          // distinct free keys of X (grouped path)
  unsigned long long class_lo;         // direct-class groups (low 32 bits) | wave-class groups (high 32 bits)
  unsigned long long class_hi;         // block-class groups
  unsigned long long direct_products;  // products (= outputs) of the direct class
  unsigned long long global_entries;   // X entries of groups accumulated in the global hash
  unsigned long long global_products;  // their products
  unsigned long long out_base;         // output cursor: outputs placed so far
  unsigned long long block_products;   // products of the block class (block survey)
  unsigned long long n_direct, n_wave, n_block, n_global;  // groups per class (grouped path)
  unsigned long long tile_base;        // dense block tiles placed by a scan: their first output
  unsigned int err;                    // kErr* bits
  unsigned int ydup;                   // nonzero: Y holds a repeated coordinate
  unsigned int ycols;                  // dense Y free key: distinct Y free cells that occur
  unsigned int nonfinite;              // an X or Y value is Inf or NaN (set by the scatter kernels)
};

// Capacities of the LDS accumulators (distinct outputs per X group).
constexpr int kWaveSlots = 512;    // LDS hash slots per wave
constexpr int kWaveCap = 358;      // largest distinct-output bound a wave takes (load <= 0.7)
constexpr int kBlockSlots = 4096;    // LDS hash slots per workgroup (large table)
constexpr int kBlockXlSlots = 8192;  // and the largest table (128 KB: one workgroup per CU)
constexpr int kBlockCap = 5734;      // largest distinct-output bound a workgroup hash takes (70% of 8192)
constexpr int kDenseBits = 13;     // dense LDS accumulator when the Y free key has <= 13 bits

// Block class on the matrix cores (dense Y free keys, one contraction).
// The block groups are the rows, the Y runs (distinct contracting keys) the
// inner dimension and the Y free cells that occur in Y the columns of a
// product computed in FP64 MFMA tiles of kMfmaRows x kMfmaCols over inner
// steps of kMfmaK runs.
constexpr int kMfmaRows = 64;
constexpr int kMfmaCols = 64;
constexpr int kMfmaK = 32;

constexpr int kCellWords = (1 << kDenseBits) / 32;  // bitmap of the dense Y free cells

// What the matrix-core block kernel reads besides GroupArgs: X as a dense
// row-major panel over the padded rows and runs, a[row * (nsteps * kMfmaK)
// + run], with am[row * nsteps + step] the runs of each step the row holds
// an entry of (bit k); Y as dense blocks, one per (column tile, step),
// b[((ct * nsteps + s) * kMfmaK + k) * kMfmaCols + col], with
// bm[(ct * nsteps + s) * kMfmaCols + col] likewise.
struct MfmaPlan {
  const double* a;
  const unsigned* am;
  const double* b;
  const unsigned* bm;
  const uint16_t* cellof;  // [ncols]: Y free key of each column
  unsigned nsteps, ncols, nct;
};

// ---- launchers (kernels.hip) ----
// Each returns the hipError_t of its launch(es); all work goes on `stream`.

// Sets every 16-byte slot to {key = kEmpty, 0}; clears st->err when st is given.
hipError_t launch_fill_empty(void* slots16, int64_t nslots, DevStatus* st, hipStream_t stream);

// Counts entries per packed key (the modes in kc) in an open-addressing table;
// *distinct is incremented once per new key.
hipError_t launch_key_count(const int32_t* idx, int64_t nnz, KeyPack kc, YSlot* tab, TabGeom g, uint64_t seed,
                            int32_t max_probe, DevStatus* st, unsigned long long* distinct, int num_cus,
                            hipStream_t stream);

// The same for a direct-addressed table of nslots <= 2^kAggBits slots:
// each workgroup histograms a chunk of kAggChunk entries in LDS into row
// `chunk` of hist [agg_chunks(nnz) + 1][nslots]; column scans turn row w
// into the entries of each key in chunks before w, and the last row into
// each key's run start; the table gets every key's count and run start and
// every other slot is set empty (no fill needed first; no global
// atomics).  total: one device u64 (the entry count).
hipError_t launch_key_count_agg(const int32_t* idx, int64_t nnz, KeyPack kc, YSlot* tab, unsigned nslots,
                                unsigned* hist, unsigned long long* total, unsigned long long* distinct,
                                hipStream_t stream);

// Exclusive scan support: tile sums need ceil(n / kScanTile) u64 entries.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// Y table: count field -> offset of the key's run stored in `start`: its end
// (run_end, for placement that takes and decrements) or its beginning.
hipError_t launch_scan_y_table(YSlot* tab, int64_t nslots, bool run_end, unsigned long long* tile_sums,
                               hipStream_t stream);

// Also inserts every full Y coordinate ((contracting key << bits_y) | free
// key) into yset (kEmpty-filled, yset_mask + 1 slots) when yset is given, and
// sets st->ydup on a repeat.
hipError_t launch_y_scatter(const int32_t* yidx, const double* yval, int64_t nnz, KeyPack kc, KeyPack kf,
                            Bounds b, YSlot* tab, TabGeom g, uint64_t seed, int32_t max_probe, YEntry* yg,
                            unsigned long long* yset, uint64_t yset_mask, int32_t bits_y, DevStatus* st, int num_cus,
                            hipStream_t stream);

// Y scatter for a direct-addressed Y table of nslots <= 2^kAggBits slots:
// each workgroup places its chunk at the run starts plus the chunk offsets
// (choff: the hist left by launch_key_count_agg; a key's entries of chunk w
// start at the last row's entry plus row w's).
hipError_t launch_y_scatter_agg(const int32_t* yidx, const double* yval, int64_t nnz, KeyPack kc, KeyPack kf,
                                Bounds b, const YSlot* tab, unsigned nslots, const unsigned* choff, YEntry* yg,
                                unsigned long long* yset, uint64_t yset_mask, uint64_t seed, int32_t bits_y,
                                DevStatus* st, hipStream_t stream);

// Sets n 8-byte words to kEmpty.
hipError_t launch_fill_keys(unsigned long long* keys, int64_t n, hipStream_t stream);

hipError_t launch_x_probe(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kc, KeyPack kf, Bounds b,
                          const YSlot* tab, TabGeom g, uint64_t seed, int32_t max_probe, XEntry* xrec,
                          uint32_t* xg, uint32_t* xcnt, DevStatus* st, int num_cus, hipStream_t stream);

// poff[i] = sum of xcnt[0..i), poff[n] = total, and the total also into *total.
// live_n (device, optional): only the first *live_n <= n entries are in use.
hipError_t launch_scan_products(const uint32_t* xcnt, int64_t n, unsigned long long* poff,
                                unsigned long long* tile_sums, unsigned long long* total, hipStream_t stream,
                                const unsigned long long* live_n = nullptr);

// dnx, dprod (device, optional): the X entry and product counts, read on
// the device (nx then bounds the entries, the grid is sized without P).
hipError_t launch_expand_acc(const unsigned long long* poff, int64_t nx, const XEntry* xrec, const uint32_t* xg,
                             const YEntry* yg, int64_t ny, int32_t bits_y, ZSlot* tab, uint64_t mask, uint64_t seed,
                             int32_t max_probe, uint64_t products, DevStatus* st, int num_cus,
                             hipStream_t stream, const unsigned long long* dnx = nullptr,
                             const unsigned long long* dprod = nullptr);

// Two-pass compaction of the output hash to COO, written from position
// *base (0 when base is NULL); writes *base + nnz (or the negated status on
// error) to *out_nnz.
hipError_t launch_compact(const ZSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* out_idx, double* out_val,
                          int64_t out_cap, int64_t* out_nnz, const unsigned long long* base,
                          unsigned long long* tile_sums, DevStatus* st, hipStream_t stream);

// Grouped path, global class: compaction of a table keyed by
// (group id << bits_y) | Y free key, written from position *base.
hipError_t launch_compact_grouped(const ZSlot* tab, int64_t nslots, const GroupRec* groups, const uint32_t* glist,
                                  KeyUnpack ux, KeyUnpack uy, int32_t bits_y, int32_t* out_idx, double* out_val,
                                  int64_t out_cap, int64_t* out_nnz, const unsigned long long* base,
                                  unsigned long long* tile_sums, DevStatus* st, const BatchOut* bout, BatchSeg* bseg,
                                  int32_t bwx, hipStream_t stream);

// ---- grouped path (grouped.hip) ----

// X table (keyed by X free key) -> dense group records; the table's start
// field becomes each group's end (run_end) or start offset for the scatter.
hipError_t launch_scan_x_table(YSlot* tab, int64_t nslots, GroupRec* groups, int64_t cap, bool run_end, void* tile_sums,
                               DevStatus* st, hipStream_t stream);

// X scatter for a direct-addressed X table of nslots <= 2^kAggBits slots,
// aggregated per workgroup in LDS like the Y scatter.
hipError_t launch_x_scatter_agg(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc,
                                Bounds b, const YSlot* xtab, unsigned nslots, const unsigned* choff, const YSlot* ytab,
                                TabGeom yg, int32_t max_probe_y, uint64_t seed, XRec* xr, DevStatus* st,
                                hipStream_t stream);

// Scatter X into its groups, probing Y's table for every entry.
hipError_t launch_x_scatter(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                            YSlot* xtab, TabGeom xg, int32_t max_probe_x, const YSlot* ytab, TabGeom yg,
                            int32_t max_probe_y, uint64_t seed, XRec* xr, DevStatus* st, int num_cus,
                            hipStream_t stream);
// The X grouping with the compact table (hashed X free keys of at most 31
// bits, fewer than 2^31 entries, one contraction, a hashed geometry): fills xtab (mask + 1 64-bit
// slots), counts, scans into groups and places the records, as
// launch_key_count + launch_scan_x_table + launch_x_scatter do with YSlot.
hipError_t launch_x_table32(const int32_t* xidx, const double* xval, int64_t nnz, KeyPack kf, KeyPack kc, Bounds b,
                            unsigned long long* xtab, TabGeom xg, int32_t max_probe_x, GroupRec* groups,
                            const YSlot* ytab, TabGeom yg, int32_t max_probe_y, uint64_t seed, XRec* xr,
                            void* tile_sums, DevStatus* st, int num_cus, hipStream_t stream);

// eoff[i] = products of grouped X entries before i; eoff[n] = P.
hipError_t launch_scan_entries(const XRec* xr, int64_t n, unsigned long long* eoff, void* tile_sums, DevStatus* st,
                               hipStream_t stream);

// Sorts groups into direct / wave / block / global accumulation classes
// (lists of group ids); counts land in st->class_lo / class_hi, and each
// direct group's products in dpos at its place in the direct list, and its
// staging record (from the grouped X records xr) in drec at the same place.
// block_cap: most distinct outputs of a group in a workgroup's LDS hash
// (0: kBlockCap).
hipError_t launch_classify(const GroupRec* groups, int64_t max_groups, const unsigned long long* eoff,
                           uint64_t ycells, int32_t dense, uint32_t* dlist, uint32_t* wlist, uint32_t* blist,
                           uint32_t* glist, unsigned long long* dpos, void* tile_sums, DevStatus* st,
                           hipStream_t stream, int32_t block_cap, const XRec* xr, DRec* drec);

// In place after launch_classify: dpos[i] = products of direct-class groups
// before list entry i; dpos[nd] and st->direct_products = their total.
// Scans max_groups entries, bounded on the device by the direct count.
hipError_t launch_scan_direct(int64_t max_groups, unsigned long long* dpos, void* tile_sums, DevStatus* st,
                              hipStream_t stream);

// Entries of the global-class groups, gathered for the global hash; each
// gathered record carries its group id in place of the packed X free key.
hipError_t launch_scan_global_entries(const GroupRec* groups, const uint32_t* glist, int64_t ngl,
                                      unsigned long long* gl_eoff, void* tile_sums, DevStatus* st,
                                      hipStream_t stream);
// dc (optional): the global class's group count read on the device (ngl
// then bounds it).
hipError_t launch_gather_global(const GroupRec* groups, const uint32_t* glist, int64_t ngl,
                                const unsigned long long* gl_eoff, const XRec* xr, XEntry* xrec, uint32_t* xg,
                                uint32_t* xcnt, int num_cus, hipStream_t stream, const DevStatus* dc = nullptr);

// Per-group accumulation in LDS.  fill = 0: count each group's outputs into
// gn[g]; fill = 1: write them from goff[g].
struct GroupArgs {
  const GroupRec* groups;
  const XRec* xr;
  const unsigned long long* eoff;
  const YEntry* yg;
  const uint16_t* ykey16;  // dense Y free keys: the grouped Y keys as 16-bit cells (else NULL)
  const double* yval;      // and the grouped Y values
  int64_t ny;
  uint64_t ycells;
  uint64_t seed;
  int32_t bits_y;
  KeyUnpack ux;  // X free key -> X free coordinates (output rows 0..)
  KeyUnpack uy;  // Y free key -> Y free coordinates (following rows)
  int32_t* out_idx;
  double* out_val;
  int64_t out_cap;
  DevStatus* st;
  // Batch (bout != NULL): outputs go to each contraction's own COO region;
  // X free key >> bwx is the contraction.
  const BatchOut* bout;
  BatchSeg* bseg;
  int32_t bwx;
};

// Block class, single pass: each workgroup accumulates a group, reserves its
// outputs with one atomic on st->out_base and writes them.
// Raises the hashed block-class kernel's dynamic LDS limit on the current
// device; called once per plan so that execute issues kernel launches only.
hipError_t prepare_group_block();
// Hashed block class (Y free key wider than kDenseBits).
// dc (optional): the block-class count read on the device (nb sizes the grid).
// cells > 0: a dense Y free key and small groups, each accumulated in a
// dense LDS row of `cells` doubles (a power of two, 64..2^kDenseBits) by one
// workgroup, in place of the (group, slice) tiles.
// Hashed (cells == 0): defer (2 nb elements) and q are required; each of
// the three table sizes' launches passes the groups its table cannot hold
// on to the next through defer (counts q->n_defer, q->n_defer2, zeroed by
// launch_reset_status).
struct LdsQueue;
hipError_t launch_group_block(const GroupArgs& a, const uint32_t* blist, int64_t nb, int num_cus, hipStream_t stream,
                              const DevStatus* dc = nullptr, unsigned cells = 0, uint32_t* defer = nullptr,
                              LdsQueue* q = nullptr);

// Block survey, before the class counts are read back: the block class's
// products into st->block_products (zeroed first; the block list's length
// is read on the device, st->class_hi) and the number of occurring Y free
// cells (bits of colbits) into st->ycols.  The X and Y scatter kernels set
// st->nonfinite when a value is Inf or NaN.
hipError_t launch_block_survey(const GroupRec* groups, const uint32_t* blist, const unsigned long long* eoff,
                               const unsigned* colbits, DevStatus* st, int num_cus, hipStream_t stream);
// Matrix-core block class, plan time.  runs: the run list
// (run_start[0..nruns], the last entry ny; runid[ny] gets each run's index
// at its start; a count other than nruns records an internal error).
// panels: columns (colid [2^kDenseBits], cellof [ncols], from colbits) and
// the panels of MfmaPlan, which must be zeroed first (the Y blocks and their
// masks; the X panel is written whole).
hipError_t launch_mfma_runs(const YSlot* ytab, int64_t yslots, int64_t ny, unsigned* run_start, unsigned* runid,
                            int64_t nruns, DevStatus* st, void* tile_sums, hipStream_t stream);
hipError_t launch_mfma_panels(const unsigned* colbits, const GroupRec* groups, const uint32_t* blist, int64_t nb,
                              const XRec* xr, const unsigned* run_start, const unsigned* runid, unsigned nruns,
                              const uint16_t* ykey16, const double* yval, int64_t ny, uint16_t* colid,
                              uint16_t* cellof, unsigned ncols, unsigned nsteps, int ydup, double* a, unsigned* am,
                              double* b, unsigned* bm, DevStatus* st, int num_cus, hipStream_t stream);
// Execute: every block group's outputs (one atomic per tile on st->out_base).
hipError_t launch_group_block_mfma(const GroupArgs& a, const uint32_t* blist, int64_t nb, const MfmaPlan& m,
                                   int num_cus, hipStream_t stream);

// Direct class: single-entry groups against a Y without repeated coordinates
// have one output per product; writes output q for product q in [0, nprod).
// tfirst: scratch of direct_tile_bound(nprod) u32 (each product tile's first
// group, found first by a pass over the groups).
int64_t direct_tile_bound(uint64_t nprod);
// dc (optional): the direct class's group and product counts read on the
// device (nd and nprod then size the grids; tfirst holds tfirst_slots
// entries, and more tiles than that are a capacity error).
// tile_products: 1024 for the small tile, else the default (2048, or 1280
// in a batch).
hipError_t launch_group_direct(const GroupArgs& a, const DRec* drec, const unsigned long long* dpos, int64_t nd,
                               uint64_t nprod, uint32_t* tfirst, int num_cus, hipStream_t stream,
                               int tile_products = 0, DevStatus* dc = nullptr, int64_t tfirst_slots = 0);

// *out_nnz = st->out_base, or the negated status.
hipError_t launch_finalize(int64_t* out_nnz, int64_t out_cap, DevStatus* st, hipStream_t stream);

// Dense Y free keys: writes the compact copy of grouped Y (16-bit keys,
// values) the dense accumulators read and flags repeated Y coordinates;
// with sort, first sorts each run of 2..1024 entries by Y free key.  With
// colbits (kCellWords words, zeroed first), also ORs in a bit for every
// Y free cell that occurs.  With yso (sort only; [nslots][kSlices + 1]
// u32) and runslot ([ny] u32), also cuts every run into kSlices slices of
// the Y free key (key / slice_cells, a positive multiple of 64; the last
// slice also takes every larger key), slice by slice in the compact copy:
// yso[slot][s] is where slice s of the slot's run begins (yso[slot][kSlices]
// its end) and runslot[run start] = slot.  Without sort, ylong
// (y_long_run_slots(ny) u32) is required: the list of long runs whose
// repeats a workgroup each checks.
hipError_t launch_sort_y_runs(const YSlot* ytab, int64_t nslots, YEntry* yg, int64_t ny, uint16_t* ykey16,
                              double* yval, unsigned* colbits, DevStatus* st, bool sort, int num_cus,
                              hipStream_t stream, uint32_t* yso = nullptr, uint32_t* runslot = nullptr,
                              unsigned slice_cells = 0, uint32_t* ylong = nullptr);
int64_t y_long_run_slots(int64_t ny);

// ---- LDS classes: dense block tiles and the wave class (queue.hip) ----
// The dense Y free key space is cut into kSlices slices, one per XCD: a
// tile of the dense block class is (block-class group, slice), accumulated
// by one wave in LDS.
constexpr int kSlices = 8;

// Work queue counters of the persistent launch, zeroed by launch_reset_status.
// A queue counter on a cache line of its own: device-scope atomics on one
// line are serialised (about 12 ns each), so counters of different XCDs
// sharing a line would serialise every XCD's pops together.
struct alignas(128) QueueCounter {
  unsigned long long v;
};

struct LdsQueue {
  QueueCounter next_tile[kSlices];  // next block-class tile of each slice's queue
  QueueCounter next_fill[kSlices];  // the same for the fill pass of a two-pass launch
  QueueCounter n_defer;             // hashed block groups passed to the large-table launch
  QueueCounter n_defer2;            // and from it to the largest-table launch
};

// Plan time: block-class X records refer to their Y run by its table slot
// (runslot of their run start) instead of the run start.
// dc (optional): the block-class count read on the device (nb sizes the grid).
hipError_t launch_block_runslots(const GroupRec* groups, const uint32_t* blist, int64_t nb, XRec* xr,
                                 const uint32_t* runslot, int64_t ny, DevStatus* st, int num_cus,
                                 hipStream_t stream, const DevStatus* dc = nullptr);

// The dense block class's list (blist, nb groups; groups and eoff as the
// classification read them) reordered by decreasing product count, when
// 2 <= nb <= kOrderMax; otherwise left as it is.
constexpr unsigned kOrderMax = 8192;
hipError_t launch_order_blist(const GroupRec* groups, const unsigned long long* eoff, uint32_t* blist, int64_t nb,
                              hipStream_t stream);

// Raises the persistent kernel's dynamic LDS limit on the current device.
hipError_t prepare_lds_queue();

// The dense block class's (group, slice) tiles (blist, runs cut by yso),
// persistent launches over per-XCD queues; the tile count is read on the
// device from the plan's class counts.  cells: the dense accumulator size (a
// power of two of at least 1024 and at least 2^bits_y); slice_cells: the
// width of one slice, as the runs were cut (a positive multiple of 64, at
// most cells / kSlices).  With tcnt == NULL
// each tile reserves its outputs with one atomic on the output cursor (one
// launch).  Otherwise (tcnt, toff: 8 * nb elements; tile_sums: scan scratch
// for them) a count launch writes each tile's outputs to tcnt, a scan turns
// them into offsets after the outputs placed so far, and a fill launch
// accumulates again and writes: no atomic per tile, for many small tiles.
hipError_t launch_lds_queue(const GroupArgs& a, const uint32_t* blist, int64_t nb, const uint32_t* yso,
                            int64_t yso_slots, unsigned cells, unsigned slice_cells, LdsQueue* q, uint32_t* tcnt,
                            unsigned long long* toff, void* tile_sums, int num_cus, hipStream_t stream);

// The wave class (wlist, at most nw groups; the count is read on the
// device).  One contraction: a count pass into wcnt[nw], a scan into
// woff[nw] (tile_sums: scan scratch for nw elements) and a fill pass; the
// class's outputs take [direct products, + their count) and st->out_base
// moves past them.  A batch (a.bout): one pass, one atomic per group on its
// contraction's cursor (wcnt, woff unused).
hipError_t launch_wave_class(const GroupArgs& a, const uint32_t* wlist, int64_t nw, uint32_t* wcnt,
                             unsigned long long* woff, void* tile_sums, int num_cus, hipStream_t stream);

// Clears st->err and st->out_base.
hipError_t launch_reset_status(DevStatus* st, LdsQueue* q, hipStream_t stream);

// Inspection: group g's X free coordinates ([nfx][cap]), entry count and product count.
hipError_t launch_x_groups(const GroupRec* groups, int64_t ng, const unsigned long long* eoff, KeyUnpack ku,
                           int32_t* coords, int64_t* counts, int64_t* products, int64_t cap, hipStream_t stream);

// Inspection helpers.
hipError_t launch_y_groups(const YSlot* tab, int64_t nslots, KeyUnpack ku, int32_t* key_coords, int64_t* counts,
                           int64_t* starts, int64_t cap, int64_t* ngroups_dev, unsigned long long* tile_sums,
                           DevStatus* st, hipStream_t stream);
hipError_t launch_y_grouped(const YEntry* yg, int64_t nnz, KeyUnpack ku, int32_t* free_coords, double* vals,
                            hipStream_t stream);
hipError_t launch_x_counts(const unsigned long long* poff, int64_t nx, int64_t* counts, hipStream_t stream);

// ---- batched contraction (batch.hip) ----

// One contraction of a batch, as the pack kernel reads it.
struct BatchIn {
  const int32_t* xidx;
  const double* xval;
  const int32_t* yidx;
  const double* yval;
  int64_t nx, ny, xoff, yoff;  // nnz and place in the concatenation
  KeyPack xc, yc, xf, yf;      // contracting and free keys
  Bounds xb, yb;
};

// A run of one contraction's X (side 0) or Y (side 1) entries to pack.
struct PackTile {
  int32_t b;
  int32_t side;
  int64_t start, end;
};

// Where contraction b's output goes and how to decode it.
struct BatchOut {
  KeyUnpack ux, uy;
  int64_t idx_off, val_off, cap;
};

// Contraction b's output positions.  The grouped pipeline numbers direct
// outputs, then wave outputs, across the whole batch; with the batch's key
// tables cut into per-contraction regions, b's groups and so its direct and
// wave outputs are contiguous in that numbering.  b's COO takes its direct
// outputs first, its wave outputs next, then block and global class outputs
// from `cursor`, which ends as b's nnz.
// One cache line per contraction: device-scope atomics on one line are
// serialised, so contractions must not share their cursors' line.
struct alignas(128) BatchSeg {
  unsigned long long dshift;  // numbering of b's first direct output
  unsigned long long dcount;  // b's direct outputs
  unsigned long long cursor;  // b's next output place after its direct outputs
};

// Packed key widths: a key of w bits is stored as (key >> lo, key & (2^lo - 1)).
struct BatchWidths {
  int32_t wc, wx;        // contracting / X free key widths before the index prefix
  int32_t lo_c, lo_x, lo_y;
  int32_t wy;
};

hipError_t launch_batch_pack(const BatchIn* in, const PackTile* tiles, int64_t ntiles, BatchWidths w, int32_t* px,
                             double* pxv, int64_t nx_total, int32_t* py, double* pyv, int64_t ny_total,
                             unsigned* err, hipStream_t stream);

// Per contraction: the sum of its groups' product counts.
hipError_t launch_batch_products(const GroupRec* groups, int64_t ngroups, const unsigned long long* eoff,
                                 int32_t wx, int32_t count, unsigned long long* pb, hipStream_t stream);

// Zeroes n 8-byte words.
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t stream);

// Plan time: each contraction's direct outputs, from the contraction-ordered
// direct list.
hipError_t launch_batch_segments(const GroupRec* groups, const uint32_t* dlist, int64_t nd,
                                 const unsigned long long* dpos, int32_t wx, int32_t count, BatchSeg* seg,
                                 hipStream_t stream);

// Execute time, first: each contraction's output cursor starts after its
// direct outputs.
hipError_t launch_batch_reset(int32_t count, BatchSeg* seg, hipStream_t stream);

// out_nnz[b] = b's nnz, or the negated status when the pipeline or b's
// region reported an error.
hipError_t launch_batch_finalize(const DevStatus* st, const BatchSeg* seg, const BatchOut* outs, int32_t count,
                                 int64_t* out_nnz, hipStream_t stream);

}  // namespace sptc
