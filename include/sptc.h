/*
 * sptc.h -- sparse-sparse tensor contraction on AMD Instinct MI355X (gfx950).
 *
 * Computes, for COO tensors X and Y and paired contracted modes
 * cx[t] <-> cy[t] (t = 0..ncontract-1),
 *
 *     Z[fX, fY] = sum over c of X[fX, c] * Y[c, fY]
 *
 * the general contraction of the paper's section 2.2 (Eq. 1, Eq. 2).  The
 * contract lists pair up by position and paired modes must have equal length
 * (section 2.2).  The output coordinate is X's free coordinates (ascending X
 * mode order) followed by Y's free coordinates (ascending Y mode order), as
 * in Eq. 4 and the matrix product of Fig. 2.  Output entries with equal
 * coordinates are summed (section 2.4, accumulation); every coordinate reached
 * by at least one matching pair is emitted, even if its sum is exactly zero.
 * The output is COO (section 2.1, Fig. 1) in no particular order: the method
 * never sorts (section 4.1.3), and a sorted output is optional (section 1).
 *
 * Method (sections 4.1-4.3).  Y's nonzeros are grouped by their
 * contracting-mode key in a device open-addressing table (section 2.3.1; the
 * probing table for Y of section 4.2): counted, prefix-summed and placed in
 * a grouped array (the counting sort of section 4.1.1 and the array form of
 * Y of section 4.2).  X's nonzeros are grouped the same way by their free
 * key (section 4.1), and each X entry looks up the run of Y entries that
 * share its contracting key.  The product count of a group (the bound of
 * section 4.3) chooses how the group accumulates: single-entry groups write
 * every product as an output; small groups accumulate in a wave's LDS hash,
 * large ones in a workgroup's dense LDS array or LDS hash; groups too large
 * for LDS go to a device-memory hash (the footnote to section 4.4), compacted
 * by count, prefix sum and fill (writeback, section 2.5).  On request
 * (sptc_options.block_mfma, off by default), the large groups with a dense Y
 * free key may instead run as a dense FP64 product on the matrix cores when
 * X and Y are dense enough; the default path has no dense product.  The
 * GLOBAL mode sends every product to that device hash.
 *
 * Conventions
 *  - Modes and coordinates are 0-based; 0 <= i_k < I_k (section 2.1.1).
 *  - Tensor order 0..16 each; mode lengths 1..2^31; nnz < 2^32 - 1.
 *  - Index arrays are int32, mode-major: idx[m * nnz + e] is coordinate m of
 *    nonzero e.  Values are IEEE double.  Repeated coordinates are allowed and
 *    act as separate terms.
 *  - Coordinates are packed into 64-bit keys with ceil(log2 I_k) bits per
 *    mode.  The contracting key, the X free key and the Y free key must each
 *    fit 63 bits (else SPTC_ERR_KEY_OVERFLOW).  Their output key may be
 *    wider: the grouped mode never packs X free and Y free coordinates
 *    together except under the dense id of the X free key (its group,
 *    section 4.1.2).  The global mode packs them and needs both to fit 63
 *    bits together.
 *  - "device" pointers are HIP device memory (or memory the GPU can address,
 *    e.g. pinned host memory where stated); "host" pointers are read by the
 *    calling thread only during the call.
 *  - Streams are hipStream_t passed as void*; NULL is the default stream.
 *
 * Errors: every entry point returns an sptc_status; no C++ exception crosses
 * this interface.  sptc_last_error() gives a thread-local detail string for
 * the last failure on the calling thread.  Errors found by kernels (probe
 * length exhausted, coordinate out of range with validation on) are recorded
 * in the plan: sptc_plan() reports them itself; after sptc_execute() they
 * make *out_nnz negative (the negated status) and sptc_plan_status() returns
 * them.
 */
#ifndef SPTC_H_
#define SPTC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define SPTC_API __attribute__((visibility("default")))
#else
#define SPTC_API
#endif

#define SPTC_MAX_ORDER 16
#define SPTC_MAX_OUT_ORDER 32

typedef enum sptc_status {
  SPTC_OK = 0,
  SPTC_ERR_INVALID_ARG = 1,   /* null pointer, bad order/mode list, nnz, coordinate out of range */
  SPTC_ERR_DIM_MISMATCH = 2,  /* paired modes of different length (section 2.2) */
  SPTC_ERR_KEY_OVERFLOW = 3,  /* packed key wider than 63 bits */
  SPTC_ERR_OUT_OF_MEMORY = 4, /* allocator returned NULL */
  SPTC_ERR_CAPACITY = 5,      /* hash probe limit reached, or output larger than out_cap */
  SPTC_ERR_HIP = 6,           /* a HIP runtime call failed */
  SPTC_ERR_INTERNAL = 7
} sptc_status;

/* Optional device-memory allocator.  alloc returns device memory of `bytes`
 * usable in stream order on `stream` (NULL on failure); release frees it in
 * stream order.  When no allocator is given the library uses the device's
 * stream-ordered memory pool (hipMallocAsync / hipFreeAsync). */
typedef struct sptc_allocator {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*release)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} sptc_allocator;

/* A COO tensor (section 2.1, Fig. 1).  dims: host [order].  idx: device
 * int32 [order][nnz] mode-major.  val: device double [nnz].  Both device
 * arrays are borrowed: sptc_plan reads them (on its stream) before it
 * returns; a plan keeps its own copies and never reads them again. */
typedef struct sptc_coo {
  int32_t order;
  const int64_t* dims;
  int64_t nnz;
  const int32_t* idx;
  const double* val;
} sptc_coo;

/* Pipeline stages, for optional per-stage timing with HIP events. */
typedef enum sptc_stage {
  SPTC_STAGE_Y_COUNT = 0,    /* Y key table: clear, then count entries per contracting key */
  SPTC_STAGE_Y_SCAN = 1,     /* prefix sum of the counts: group boundaries */
  SPTC_STAGE_Y_SCATTER = 2,  /* grouped Y array */
  SPTC_STAGE_X_PROBE = 3,    /* per X nonzero: its Y group (grouped mode: with X grouped by its free key) */
  SPTC_STAGE_P_SCAN = 4,     /* prefix sum of products per X nonzero; P */
  SPTC_STAGE_OUT_CLEAR = 5,  /* output hash: mark every slot empty */
  SPTC_STAGE_EXPAND = 6,     /* expand products, accumulate in the output hash */
  SPTC_STAGE_COMPACT = 7,    /* output hash -> COO: count, prefix sum, fill */
  SPTC_STAGE_GROUP_COUNT = 8, /* (not marked: the wave class runs in stage BLOCK) */
  SPTC_STAGE_GROUP_FILL = 9,  /* (not marked, as GROUP_COUNT) */
  SPTC_STAGE_DIRECT = 10,     /* grouped path, single-entry groups: write every product as an output */
  SPTC_STAGE_BLOCK = 11,      /* grouped path, groups accumulated in LDS: the wave class (count, scan,
                                 fill), then the block class (dense (group, slice) tiles over per-XCD work
                                 queues, dense rows, hashed tables, or the matrix cores) */
  SPTC_STAGE_BATCH_PACK = 12,   /* batch plan: key every contraction's entries with its index */
  SPTC_STAGE_BATCH_SEGMENTS = 13, /* batch plan: products and output segments per contraction */
  SPTC_STAGE_X_SORT = 14,       /* grouped plan, dense block class: Y runs sorted and cut into slices for
                                   the tiles and the class list ordered largest group first (or the
                                   matrix-core panels built) */
  SPTC_NUM_STAGES = 15
} sptc_stage;

/* Accumulation strategy.
 * GROUPED (default): X is grouped by its free key too (section 4.1) and each
 *   group's products are accumulated in an LDS table of its own sized from
 *   the group's bound (section 4.3); only groups too large for LDS use the
 *   output hash in device memory.  Plan stage X_PROBE then covers grouping X,
 *   P_SCAN the product prefix sum and the classing of groups by size.
 * GLOBAL: X stays ungrouped and every product goes to one output hash in
 *   device memory (the footnote to section 4.4). */
typedef enum sptc_mode { SPTC_MODE_GROUPED = 0, SPTC_MODE_GLOBAL = 1 } sptc_mode;

typedef struct sptc_options {
  double load_factor;        /* hash fill target in (0, 0.95]; default 1/1.3 (section 2.3.1) */
  int32_t validate;          /* nonzero: check every coordinate is within its mode length */
  int32_t max_probe;         /* probe-length guard per insert; 0 = table capacity */
  uint64_t hash_seed;        /* xored into keys before hashing */
  int64_t out_table_slots;   /* 0 = sized from the product count; else a power of two (testing) */
  void** stage_events;       /* NULL, or 2*SPTC_NUM_STAGES hipEvent_t: entry 2s is recorded on the
                                stream before stage s and entry 2s+1 after it (NULL entries skipped);
                                the caller owns the events and keeps the array alive */
  int32_t mode;              /* sptc_mode; default SPTC_MODE_GROUPED */
  int32_t block_mfma;        /* grouped mode, dense Y free key, sptc_plan only: run the block class
                                as a dense product on the FP64 matrix cores instead of the LDS walk.
                                0 (default): never; 1: whenever eligible; -1: when eligible and
                                rows x columns x runs is at most 24x the class's products.
                                Eligible: every X and Y value finite, and dense X and Y panels of at
                                most 8 GiB.  sptc_info.block_mfma reports the choice. */
  int32_t tile;              /* products per workgroup tile of the single-entry (direct) class: 0 (default,
                                2048), 1024 or 2048 */
  int32_t lds_max_keys;      /* grouped mode: most distinct outputs a group with a hashed (wide) Y free key
                                may accumulate in a workgroup's LDS table before it goes to the output hash in
                                device memory: 0 (default, 5734) or 64..5734 */
  int64_t capture_out_cap;   /* 0 (default): sptc_plan reads its counts back.  > 0: sptc_plan makes no
                                read-back at all (so sptc_plan and sptc_execute can be captured together into
                                one HIP graph): every buffer is sized from the nonzero counts and from this
                                bound on nnz(Z), every launch reads its counts on the device, and the plan
                                needs a caller allocator.  Counts the plan would read back are then unknown
                                (sptc_plan_info reports products = -1 and out_nnz_bound = capture_out_cap);
                                errors, including nnz(Z) > capture_out_cap, show in sptc_execute's out_nnz.
                                The matrix-core block class is not used.  Not for batches. */
  int32_t operand_order;     /* grouped mode, sptc_plan only.  0 (default): group whichever operand's free
                                key space is larger, so that the other's (the one the per-group tables
                                are indexed by) is the smaller (section 5.4: the operand order matters);
                                with Y's free key space the larger, the plan groups Y and accumulates
                                over X's free keys.  Z is the same either way (its modes stay X's free
                                modes, then Y's); sptc_info.operands_swapped reports the choice, and the
                                inspection calls then describe the operands as swapped.  1: as given. */
} sptc_options;

/* Sizes fixed by sptc_plan. */
typedef struct sptc_info {
  int32_t out_order;                       /* (order_X - ncontract) + (order_Y - ncontract) */
  int64_t out_dims[SPTC_MAX_OUT_ORDER];    /* X free dims ascending, then Y free dims ascending */
  int64_t products;                        /* P: number of matching (x, y) pairs */
  int64_t out_nnz_bound;                   /* min(P, product of out_dims): enough out_cap */
  int64_t y_groups;                        /* distinct contracting keys among Y's nonzeros */
  int64_t y_table_slots;                   /* capacity of the Y key table */
  int64_t out_table_slots;                 /* capacity of the output hash */
  int64_t workspace_bytes;                 /* device memory the plan holds */
  int32_t key_bits_contract, key_bits_x_free, key_bits_y_free;
  int32_t mode;                            /* sptc_mode the plan runs */
  int64_t x_groups;                        /* grouped mode: distinct X free keys */
  int64_t wave_groups, block_groups, global_groups;  /* grouped mode: groups per accumulation class */
  int64_t direct_groups;                   /* grouped mode: single-entry groups written directly */
  int64_t direct_products;                 /* their products (= their outputs) */
  int32_t block_mfma;                      /* 1: the block class runs on the matrix cores */
  int64_t block_mfma_work;                 /* then: padded rows x columns x runs (multiply-adds) */
  int32_t block_tiles_scanned;             /* 1: the dense block class's tiles are counted, then placed by a
                                              scan (many small tiles); 0: each reserves its outputs */
  int32_t operands_swapped;                /* 1: the plan groups Y (sptc_options.operand_order); key widths,
                                              group counts and classes then refer to the swapped operands */
  int32_t block_dense_rows;                /* 1: the dense block class's groups are small, and each is
                                              accumulated whole (its dense output row) by one workgroup */
} sptc_info;

typedef struct sptc_plan_s* sptc_plan_t;

/* Fill *opt with the defaults. */
SPTC_API void sptc_default_options(sptc_options* opt);

/* Build a plan (sections 4.1-4.3): group Y by its contracting key (the
 * counting sort of section 4.1.1 into the array form of Y with its probing
 * table, section 4.2); in the grouped mode, group X by its free key the same
 * way, look up every X entry's Y run, and take each X group's product count
 * (the bound of section 4.3), which sums to P and picks the group's
 * accumulation class; size the output hash (in the global mode, for all P
 * products).  Enqueues work on `stream` and waits for it to read counts
 * back: once in the global mode, and in the grouped mode once, or three
 * times when some X group is too large for LDS (its entries and its
 * products are counted before the device-memory hash is sized).  opt and
 * alloc may be NULL.  On success *plan owns all workspace (released by
 * sptc_free).  On failure *plan is NULL and nothing stays allocated. */
SPTC_API sptc_status sptc_plan(sptc_plan_t* plan, const sptc_coo* X, const sptc_coo* Y, int32_t ncontract,
                      const int32_t* cx, const int32_t* cy, const sptc_options* opt,
                      const sptc_allocator* alloc, void* stream);

/* Copy the plan's sizes into *info (host): P, the number of matching (x, y)
 * pairs, which is the sum over X groups of the bound of section 4.3;
 * out_nnz_bound = min(P, product of out_dims), enough out_cap for
 * sptc_execute; class counts and workspace.  Does not synchronise. */
SPTC_API sptc_status sptc_plan_info(sptc_plan_t plan, sptc_info* info);

/* Contraction, accumulation and writeback (sections 2.4 and 2.5, with the
 * per-group accumulation tables of section 4.3): expand every product,
 * accumulate equal output coordinates (in the X group's LDS table, or in the
 * output hash) and write Z as COO: out_idx device int32 [out_order][out_cap]
 * (mode-major with row stride out_cap; may be NULL when out_order is 0),
 * out_val device double [out_cap], out_nnz a device or pinned-host int64
 * that receives nnz(Z), or the negated status when a kernel recorded an
 * error (including nnz(Z) > out_cap, in which case only the first out_cap
 * entries are written).  Never synchronises, allocates or copies to the
 * host, so it can be captured into a HIP graph; the plan may be executed
 * any number of times.  Executions of one plan must not overlap. */
SPTC_API sptc_status sptc_execute(sptc_plan_t plan, int32_t* out_idx, double* out_val, int64_t out_cap,
                         int64_t* out_nnz, void* stream);

/* Replace the stage events used by later sptc_execute calls (same layout as
 * sptc_options.stage_events; NULL turns timing off). */
SPTC_API sptc_status sptc_plan_set_stage_events(sptc_plan_t plan, void** events);

/* Synchronise `stream` and return the first error a kernel recorded for this
 * plan (SPTC_OK if none). */
SPTC_API sptc_status sptc_plan_status(sptc_plan_t plan, void* stream);

/* Release the plan's workspace in stream order on the plan's stream. */
SPTC_API void sptc_free(sptc_plan_t plan);

SPTC_API const char* sptc_status_string(sptc_status status);
SPTC_API const char* sptc_last_error(void);

/* ---- Inspection of the plan's intermediate structures (stage checks) ---- */

/* The Y groups (sections 4.1.1 and 4.2): for each distinct contracting key,
 * its coordinates (device int32 [ncontract][cap], mode-major, in cy order),
 * its number of entries and the start of its run in the grouped Y array
 * (device int64 [cap] each).  *ngroups (host) receives the group count; when
 * it exceeds cap nothing is written and SPTC_ERR_CAPACITY is returned.
 * Groups come in table order.  Synchronises `stream`. */
SPTC_API sptc_status sptc_plan_y_groups(sptc_plan_t plan, int32_t* key_coords, int64_t* counts, int64_t* starts,
                               int64_t cap, int64_t* ngroups, void* stream);

/* The grouped Y array (section 4.2): entry k's Y free coordinates (device
 * int32 [order_Y - ncontract][nnz_Y], mode-major, ascending Y mode order) and
 * value (device double [nnz_Y]).  Enqueued on `stream`. */
SPTC_API sptc_status sptc_plan_y_grouped(sptc_plan_t plan, int32_t* free_coords, double* vals, void* stream);

/* Global mode only: per X nonzero, the number of Y nonzeros sharing its
 * contracting key (device int64 [nnz_X]).  Enqueued on `stream`. */
SPTC_API sptc_status sptc_plan_x_counts(sptc_plan_t plan, int64_t* counts, void* stream);

/* Grouped mode only: the X groups (section 4.1): per group its X free
 * coordinates (device int32 [order_X - ncontract][cap], ascending X mode
 * order), its number of X entries and its number of products, the group's
 * bound of section 4.3 (device int64 [cap] each).  *ngroups (host) receives
 * the group count; when it exceeds cap nothing is written and
 * SPTC_ERR_CAPACITY is returned.  Enqueued on `stream`. */
SPTC_API sptc_status sptc_plan_x_groups(sptc_plan_t plan, int32_t* free_coords, int64_t* counts, int64_t* products,
                                        int64_t cap, int64_t* ngroups, void* stream);

/* ---- Batched contraction: many independent contractions in shared launches ----
 *
 * count contractions (X[b], Y[b], ncontract[b], cx[b], cy[b]) are planned and
 * executed together: every entry is keyed with its contraction's index, so
 * one pass of the grouped pipeline serves all of them, with the key tables
 * cut into one region per contraction.  1 <= count <= 4096.
 * Each contraction follows the rules of sptc_plan; the contraction index
 * plus its widest contracting key and its widest X free key must each fit
 * 62 bits.  Options apply to the whole batch (mode must be GROUPED). */
typedef struct sptc_batch_s* sptc_batch_t;

/* Plans the batch; synchronises `stream` a few times.  Arrays are host
 * arrays of `count` entries; cx[b] / cy[b] point to ncontract[b] modes. */
SPTC_API sptc_status sptc_batch_plan(sptc_batch_t* batch, int32_t count, const sptc_coo* X, const sptc_coo* Y,
                                     const int32_t* ncontract, const int32_t* const* cx, const int32_t* const* cy,
                                     const sptc_options* opt, const sptc_allocator* alloc, void* stream);

/* Output buffers the batch needs (host outputs): int32 elements for all
 * index rows and double elements for all values, both sized from pass 1's
 * product counts (section 4.3), and the bytes of device workspace the batch
 * holds.  Any pointer may be NULL. */
SPTC_API sptc_status sptc_batch_sizes(sptc_batch_t batch, int64_t* idx_elems, int64_t* val_elems,
                                      int64_t* workspace_bytes);

/* Contraction b's sizes (info: out_order, out_dims, products,
 * out_nnz_bound and key_bits_*; the plan-wide fields are zero) and where its
 * output sits: index row m at out_idx + idx_offset + m * info.out_nnz_bound,
 * values at out_val + val_offset. */
SPTC_API sptc_status sptc_batch_info(sptc_batch_t batch, int32_t b, sptc_info* info, int64_t* idx_offset,
                                     int64_t* val_offset);

/* Executes every contraction, writing each output straight into its
 * contraction's region.  out_idx / out_val: device buffers of the sizes
 * sptc_batch_sizes reports; out_nnz: device int64 [count] receiving each
 * contraction's nnz (or the negated status).  Like sptc_execute it never
 * synchronises, allocates or copies to the host. */
SPTC_API sptc_status sptc_batch_execute(sptc_batch_t batch, int32_t* out_idx, double* out_val, int64_t* out_nnz,
                                        void* stream);

SPTC_API void sptc_batch_free(sptc_batch_t batch);

/* ---- Memory ----
 *
 * Without a caller allocator, workspace comes in slabs from the current
 * device's stream-ordered pool.  Slabs of freed plans and batches are kept
 * by the library (per device, with an event recorded on the freeing stream
 * that a reuse on another stream waits for) and reused by later plans, so a
 * warmed-up caller makes no pool calls.  sptc_pool_trim gives cached slabs
 * above keep_bytes back to the pool and trims the pool to keep_bytes
 * (hipMemPoolTrimTo); memory of live plans is unaffected.  An allocation
 * that fails first releases the cache and retries. */
SPTC_API sptc_status sptc_pool_trim(size_t keep_bytes);

/* ---- One contraction without allocating ----
 *
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation):
 * sptc_plan + sptc_execute + sptc_free in one call, with every workspace
 * buffer carved from a static device array of SPTC_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends.
 * The call makes no device allocation, no pinned-host allocation and no
 * free; the caller passes the inputs (as for sptc_plan) and the outputs (as
 * for sptc_execute, so out_cap must be at least the contraction's
 * out_nnz_bound, known for instance from an earlier sptc_plan).  It waits
 * for `stream` to read the plan's counts back (as sptc_plan does), then
 * enqueues the execution and returns without waiting for it.
 * A contraction whose workspace does not fit the array returns
 * SPTC_ERR_CAPACITY (sptc_last_error() names the size) and writes nothing.
 * Every call on one device uses that device's one array, which keeps what
 * the last call left there (the plan clears what must start at zero):
 * calls on one stream run one after another, but calls that overlap on one
 * device (other streams, other threads) race and give wrong results. */
#define SPTC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

SPTC_API sptc_status sptc_contract_noalloc(const sptc_coo* X, const sptc_coo* Y, int32_t ncontract, const int32_t* cx,
                                           const int32_t* cy, const sptc_options* opt, int32_t* out_idx,
                                           double* out_val, int64_t out_cap, int64_t* out_nnz, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPTC_H_ */
