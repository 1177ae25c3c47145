/*
 * spg -- two-phase CSR sparse matrix-matrix multiply C = A*B on MI355X (gfx950).
 *
 * The operation is the one of the Kokkos Kernels paper, section 2.2: A is
 * m x n, B is n x k, C is m x k, all in compressed row storage (CRS, section
 * 2: row pointer, column indices, values).  C(i,:) is the sum over the
 * nonzeros j of A(i,:) of A(i,j) * B(j,:) (section 2.2.1, Eq. (1)).  The work
 * is split in the paper's two phases (section 2.2.1):
 *
 *   symbolic  -- the number of nonzeros of each row of C, scanned into the row
 *                pointer; its last entry is nnz(C).  The caller then allocates
 *                the column-index and value arrays of size nnz(C);
 *   numeric   -- the column indices (ascending within each row) and values.
 *
 * A symbolic result is reused by every later numeric call while the sparsity
 * patterns stay the same (section 2: the split of symbolic and numeric work),
 * so only values may change between numeric calls.  Runtime choices travel
 * in a handle (section 6, the handle passed to the dispatch layer).
 *
 * Conventions shared by every call:
 *   - indices and row pointers are int32; nnz(C) must stay below 2^31;
 *   - "device" pointers are HIP device memory of the handle's device, "host"
 *     pointers are ordinary host memory;
 *   - the caller owns every buffer it passes in; the library never returns
 *     memory.  Input structure arrays are borrowed: they must stay valid and
 *     unchanged from spg_set_matrices until the last spg_numeric;
 *   - input rows may be unsorted and may repeat a column (repeats add up);
 *     explicit zeros produced by cancellation are kept in C;
 *   - errors are reported as spg_status; no C++ exception crosses this ABI.
 *     spg_last_error returns a message for the last failing call on a handle;
 *   - all GPU work runs on the handle's stream, in order.  Only spg_symbolic
 *     waits for the device (it must return nnz(C) to the host; see there for
 *     when it waits twice).  One handle
 *     must not be used from two host threads at once.
 */
#ifndef SPG_H
#define SPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spg_handle_s* spg_handle;

typedef enum {
    SPG_OK = 0,
    SPG_ERR_ARG = 1,          /* null pointer, negative size, bad option value */
    SPG_ERR_SHAPE = 2,        /* inconsistent dimensions */
    SPG_ERR_STATE = 3,        /* call out of order, e.g. numeric before symbolic */
    SPG_ERR_INDEX = 4,        /* row pointer not monotone / not ending at nnz, or a
                                 column index out of range (always checked) */
    SPG_ERR_OVERFLOW = 5,     /* nnz(C) >= 2^31 */
    SPG_ERR_ALLOC = 6,        /* device or pinned-host allocation failed */
    SPG_ERR_HIP = 7,          /* a HIP runtime call failed */
    SPG_ERR_UNSUPPORTED = 8   /* feature not available on this device */
} spg_status;

typedef enum { SPG_F32 = 0, SPG_F64 = 1 } spg_dtype;

/* Options for spg_set_option. */
typedef enum {
    /* how symbolic sizes each row's accumulator (its occupied 32-column
       blocks): 0 = upper bound from the row's products, 1 = learned predictor
       set by spg_set_mlp, with overflow detection and an exact retry, 2 =
       upper bound from the compressed-B runs the row reads (tighter than 0,
       default), 3 = the exact count left by the previous spg_symbolic of the
       same matrices (the ideal estimate, which bounds what any predictor can
       gain; SPG_ERR_STATE without such a run); all are capped by the row's
       column range */
    SPG_OPT_BINNING = 0,
    /* HIP events on the handle's stream, read with spg_get_stats: 0 = none
       (default), 1 = around both phases, their stages and every class launch,
       2 = around the numeric class launches only (what a timed loop of
       products needs).  Setting it clears the summed numeric launch times. */
    SPG_OPT_TIMING = 1,
    /* force every row of both phases into one accumulator class (-1 = off);
       class = mode * 10 + tier with mode 0 direct, 1 hashed, 2 two-level
       and tier 0..8 LDS, 9 global memory.  Rows that do not fit the forced
       class are placed in the class they would get anyway. */
    SPG_OPT_FORCE_CLASS = 2,
    /* products per lane used to size the thread group of a row (default 16) */
    SPG_OPT_WORK_PER_LANE = 3,
    /* log2 safety margin added to the predictor's output, times 1000 (default 500) */
    SPG_OPT_MLP_MARGIN_MILLI = 4,
    /* largest number of occupied column blocks for which numeric may use a
       hashed block table (default 64) */
    SPG_OPT_HASH_MAX_BLOCKS = 6,
    /* LDS bytes per row at which the global-memory path takes over (power of
       two, 1024..65536, default 65536) */
    SPG_OPT_LDS_LIMIT = 7,
    /* keep each row's predictor features after symbolic even with upper-bound
       binning, so spg_export_rows can return them (default 0) */
    SPG_OPT_KEEP_FEATURES = 8,
    /* device memory, in MiB, for the rows' block lists that symbolic leaves
       for numeric (1..16383, default 8192).  Each row reserves 8 bytes per
       block it may occupy (the smaller of its compressed-B run count and
       its column range in 32-column blocks); rows past the limit, and rows
       of the symbolic global path, are computed by numeric on its global
       path instead.  When the bound m * (k/32 + 1) pairs is within both this
       limit and 256 MiB, that bound is reserved before the phase runs (so
       it waits once, see spg_symbolic). */
    SPG_OPT_LIST_LIMIT_MB = 9,
    /* run the rows of a class that has few rows in the next populated class
       of the same table mode with a larger tier (at most 4x the lanes per row,
       at least 8x the rows), saving a short launch (1 = default, 0 = off;
       off under SPG_OPT_FORCE_CLASS).  sym_rows / num_rows in spg_stats count
       rows by the class they ran in. */
    SPG_OPT_MERGE_CLASSES = 10,
    /* numeric rows of the global-memory path run tiled (1 = default): B's
       columns are cut into tiles of 4096 columns, each (row, tile) pair sums
       its products in a dense FP64 window (32 KB), so each product is
       visited once.  Applies when C has at most 128 tiles of columns; rows
       without a block list, and all rows when some B row's
       entries are not grouped by tile (rows in ascending column order always
       are), take the segment path (0 = always the segment path: the row's
       values summed one LDS segment of its ranks at a time) */
    SPG_OPT_TILED_GLOBAL = 11,
    /* accumulation method of both phases: 0 = this library's per-row classes
       (default); 1..3 = the paper's design (section 2.2.1), for comparison:
       one parallelisation method for the whole matrix (1 = chosen from the
       products per nonempty row: a 16-lane group per row below 256, else a
       256-lane team per row; 2 = always the group, 3 = always the team) with a
       two-level hash-map accumulator (LDS, then a global-memory level created
       when a row's LDS level fills).  With 1..3 the numeric phase leaves each
       row of C in hash order rather than ascending column order, and
       spg_numeric_jacobi is not available (SPG_ERR_UNSUPPORTED). */
    SPG_OPT_METHOD = 12
} spg_option;

#define SPG_NTIER 10
#define SPG_NCLASS 30

/* Statistics of the last symbolic and numeric calls (spg_get_stats). */
typedef struct {
    int32_t size;                       /* sizeof(spg_stats), set by the library */
    int32_t m, n, k;
    int64_t products;                   /* sum over rows of the B-row lengths touched = multiply-adds */
    int64_t nnz_c;
    int32_t sym_rows[SPG_NCLASS];       /* rows per symbolic accumulator class */
    int32_t num_rows[SPG_NCLASS];       /* rows per numeric accumulator class */
    int64_t num_a_nnz[SPG_NCLASS];      /* A nonzeros of the rows in each numeric class */
    int64_t num_c_nnz[SPG_NCLASS];      /* C nonzeros written by each numeric class */
    int64_t num_products[SPG_NCLASS];   /* multiply-adds of each numeric class */
    int32_t empty_rows;                 /* rows of C with no products */
    int32_t retried_rows;               /* learned binning: rows whose table overflowed */
    int32_t mispredicted_rows;          /* learned binning: predicted class != class of the true size */
    int32_t binning;                    /* SPG_OPT_BINNING of the last symbolic call */
    float sym_ms;                       /* GPU time of the last symbolic call (timing on) */
    float num_ms;                       /* GPU time of the last numeric call (timing on) */
    float sym_class_ms[SPG_NCLASS];     /* per symbolic class launch (timing on) */
    float num_class_ms[SPG_NCLASS];     /* per numeric class launch (timing on) */
    float analysis_ms;                  /* row analysis and binning (timing on) */
    float scan_ms;                      /* row-pointer scan (timing on) */
    float mlp_ms;                       /* predictor inference (timing on) */
    int64_t list_pairs;                 /* {block, mask} pairs reserved for the rows' lists */
    float num_class_ms_total[SPG_NCLASS];   /* timing on: summed GPU time of every numeric launch of each
                                               class since SPG_OPT_TIMING was last set */
    int32_t num_class_launches[SPG_NCLASS]; /* ... and the number of those launches */
    int32_t num_tiles;                  /* column tiles of the tiled global path (0: not used) */
    int32_t tile_fallback_rows;         /* global-path rows the last numeric call left to the segment path */
    int32_t sym_waits;                  /* host waits for the device in the last spg_symbolic: 1 when the
                                           buffers it fills could be sized before it ran (m x (k/32 + 1)
                                           list pairs within 256 MiB), else 2 (a read-back after the
                                           row analysis sizes them exactly) */
    int32_t reserved;
} spg_stats;

/* Human-readable name of a status code (static string). */
const char* spg_status_string(spg_status s);

/* Message describing the last error on h (valid until the next call on h). */
const char* spg_last_error(spg_handle h);

/* Creates a handle bound to the current HIP device and to `hip_stream`
   (a hipStream_t; NULL = the default stream).  *h receives the handle. */
spg_status spg_create(spg_handle* h, void* hip_stream);

/* Waits for the handle's stream, then releases every buffer the handle owns
   (back to the library's per-device memory pool, which keeps up to 2 GiB of
   freed memory for later handles until the process ends). Null is accepted. */
spg_status spg_destroy(spg_handle h);

/* Rebinds the handle to another stream (later calls run there).  Waits for
   the work already enqueued on the previous stream first: the handle's device
   buffers are allocated in that stream's order. */
spg_status spg_set_stream(spg_handle h, void* hip_stream);

/* Sets A (m x n) and B (n x k) structure, borrowed device arrays:
   a_row_ptr[m+1], a_col_idx[a_nnz], b_row_ptr[n+1], b_col_idx[b_nnz].
   `dt` is the value type later passed to spg_numeric.  Invalidates any
   previous symbolic result.  Index validity is checked by spg_symbolic. */
spg_status spg_set_matrices(spg_handle h, spg_dtype dt, int32_t m, int32_t n, int32_t k,
                            const int32_t* a_row_ptr, const int32_t* a_col_idx, int64_t a_nnz,
                            const int32_t* b_row_ptr, const int32_t* b_col_idx, int64_t b_nnz);

/* Symbolic phase (section 2.2.1): writes C's row pointer into the caller's
   device array c_row_ptr[m+1] (c_row_ptr[0] = 0) and nnz(C) into *nnz_c
   (host).  Waits for the device once, for nnz(C), when the buffers the phase
   fills fit bounds known before it runs (m * (k/32 + 1) list pairs within
   256 MiB and the list limit); a larger product also reads the row analysis
   back to size them exactly (two waits; spg_stats.sym_waits tells which).
   Malformed input stops every kernel after the analysis on the device and
   is reported after the wait.  c_row_ptr is borrowed by the handle and
   must stay valid and unchanged until the last spg_numeric.  The handle
   also keeps C's structure in compressed form (each row's occupied
   32-column blocks with their column bits, section 2.2.1's compressed
   representation), which every later spg_numeric reads instead of
   recomputing it (SPG_OPT_LIST_LIMIT_MB bounds its memory).  Returns
   SPG_ERR_INDEX for a malformed input, SPG_ERR_OVERFLOW if nnz(C) >= 2^31 and
   SPG_ERR_ALLOC if a device buffer cannot be allocated. */
spg_status spg_symbolic(spg_handle h, int32_t* c_row_ptr, int64_t* nnz_c);

/* Numeric phase (section 2.2.1): fills the caller's device arrays
   c_col_idx[nnz(C)] (ascending within each row) and c_vals[nnz(C)] from the
   device values a_vals[a_nnz] and b_vals[b_nnz] of the handle's dtype.
   Values may differ from call to call; the structure must not.  Asynchronous:
   returns once the work is queued.  SPG_ERR_STATE without a symbolic result. */
spg_status spg_numeric(spg_handle h, const void* a_vals, const void* b_vals,
                       int32_t* c_col_idx, void* c_vals);

/* Jacobi-fused numeric phase (section 2.2.2): C = (I - omega D^-1 A) B for
   a square A (m x m, every row storing its diagonal entry) and B (m x k),
   on the structure of the last spg_symbolic, which is the structure of A*B
   (A's diagonal puts B(i,:) inside it).  Row i of C is
       C(i,:) = B(i,:) - omega * dinv[i] * E(i,:),   E(i,:) = sum_j A(i,j) B(j,:),
   computed in one pass of the numeric kernels: E(i,:) is accumulated as in
   spg_numeric, scaled by -omega * dinv[i] once per row, and B(i,:)'s entries
   are added into the same accumulator before the row is written out.
   dinv: device, m values of the handle's dtype (D^-1, usually 1 / A(i,i);
   the caller's values are used as given).  Other arguments and ownership as
   spg_numeric; asynchronous.  SPG_ERR_SHAPE if A is not square or some row of
   A stores no diagonal entry (checked from the structure by spg_symbolic),
   SPG_ERR_STATE without a symbolic result. */
spg_status spg_numeric_jacobi(spg_handle h, double omega, const void* dinv, const void* a_vals, const void* b_vals,
                              int32_t* c_col_idx, void* c_vals);

/* Sets an spg_option (see above). */
spg_status spg_set_option(spg_handle h, int32_t opt, int64_t val);

/* Installs the learned row-size predictor: `nw` = 1217 host floats laid out
   as W1[32][3], b1[32], W2[32][32], b2[32], w3[32], b3 (row-major).  The
   network maps (log2(1+len), log2(1+ub), log2(1+mx)) of a row -- the length
   of A's row, the sum and the max of the B row lengths it touches -- to
   log2(1 + number of occupied 32-column blocks) of C's row. */
spg_status spg_set_mlp(spg_handle h, const float* w, int32_t nw);

/* Copies statistics of the last calls into *out (host); `size` = sizeof(spg_stats). */
spg_status spg_get_stats(spg_handle h, spg_stats* out, int32_t size);

/* After spg_symbolic: training rows for the predictor.  Writes, into the
   caller's device arrays, x[m*3] (FP32 features as in spg_set_mlp) and
   y[m] (FP32 log2(1 + occupied 32-column blocks)), and row_nnz[m] (int32,
   may be NULL).  Rows with no products get y = 0. */
spg_status spg_export_rows(spg_handle h, float* x, float* y, int32_t* row_nnz);

/* ---- learned predictor kernels (section-free: the paper has no network) ----
   All pointers are device pointers; `stream` is a hipStream_t (NULL = default).
   w: 1217 FP32 weights as in spg_set_mlp; x: rows x 3 features. */

/* y[rows] = network(x); if act != NULL also stores the activations needed by
   backward: act[rows * 64] = (z1[32], z2[32]) per row. */
spg_status spg_mlp_forward(void* stream, const float* w, const float* x, int32_t rows,
                           float* y, float* act);

/* dw[1217] = sum over rows of dy[r] * d y[r] / d w, from the activations of
   spg_mlp_forward.  dw is overwritten. */
spg_status spg_mlp_backward(void* stream, const float* w, const float* x, const float* act,
                            const float* dy, int32_t rows, float* dw);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving or training loops, harnesses that forbid
   hipMalloc): the same result as spg_mlp_backward, bit for bit, with no
   allocation and no allocating library call.  The per-workgroup partial
   gradients live in a fixed array of the library (256 x 1217 floats,
   1.19 MiB per device, held until the process ends); the backward grid never
   exceeds 256 workgroups whatever `rows` is, so every size fits (a grid
   beyond the array would return SPG_ERR_ARG).  The current HIP device must
   be the stream's device.  Every call on one device shares that device's
   array: calls that overlap in time on one device (two streams, two host
   threads) race and give wrong gradients; calls ordered on one stream are
   safe.  Asynchronous on `stream`. */
spg_status spg_mlp_backward_noalloc(void* stream, const float* w, const float* x, const float* act,
                                    const float* dy, int32_t rows, float* dw);

/* Trains w_inout (device, 1217 floats) in place with minibatch Adam
   (beta1 0.9, beta2 0.999, eps 1e-8), visiting x/y rows in the given order,
   `batch` rows per step, for `epochs` passes.  The loss per row is the
   squared error (y - net)^2 when quantile == 0, else the pinball loss of
   level `quantile` in (0, 1): quantile * d if d >= 0 else (quantile - 1) * d
   with d = y - net, whose minimiser is that quantile of y.  Each step
   minimises the batch mean.  loss_out (device, may be NULL) receives the
   mean loss of each epoch (`epochs` floats).  Asynchronous on `stream`. */
spg_status spg_mlp_train(void* stream, const float* x, const float* y, int32_t rows,
                         int32_t epochs, int32_t batch, float lr, float quantile,
                         float* w_inout, float* loss_out);

/* ---- batches: many independent products C_i = A_i * B_i ----------------
   The products run as one block-diagonal product, so rows of all products
   share the same accumulator launches; after planning, a whole run (both
   phases, or numeric alone) is one hipGraphLaunch of a graph captured on the
   first run with the given pointers.  This follows the paper's point that
   fusing work into fewer launches matters as per-launch work shrinks
   (section 2.2.2, Table t:jacobifusedspgemm discussion) and its functor-level
   batching of many small problems in one parallel dispatch (section 3). */
typedef struct spg_batch_s* spg_batch;

/* Creates a batch of `count` products over pooled device CSR arrays.  Host
   arrays m, n, k, a_nnz, b_nnz (length count) give each product's shape.
   Product i's A row pointer (m[i]+1 entries, from 0 to a_nnz[i]) starts at
   entry sum_{j<i}(m[j]+1) of a_row_ptr_pool and its columns at
   sum_{j<i} a_nnz[j] of a_col_pool; B likewise with n[i]+1 and b_nnz[i].
   Value pools (spg_batch_run) follow the column pools' layout.  The
   structure is packed once on the device (A copied, B's columns borrowed:
   b_col_pool must stay valid).  Every product's arrays are validated
   (SPG_ERR_INDEX).  `stream` NULL makes the batch create its own stream. */
spg_status spg_batch_create(spg_batch* b, void* stream, spg_dtype dt, int32_t count,
                            const int32_t* m, const int32_t* n, const int32_t* k,
                            const int64_t* a_nnz, const int64_t* b_nnz,
                            const int32_t* a_row_ptr_pool, const int32_t* a_col_pool,
                            const int32_t* b_row_ptr_pool, const int32_t* b_col_pool);

/* Releases the batch (null accepted). */
spg_status spg_batch_destroy(spg_batch b);

/* Message of the last failing call on b. */
const char* spg_batch_last_error(spg_batch b);

/* Same options as spg_set_option / spg_set_mlp, applied to every product;
   they invalidate the plan. */
spg_status spg_batch_set_option(spg_batch b, int32_t opt, int64_t val);
spg_status spg_batch_set_mlp(spg_batch b, const float* w, int32_t nw);

/* Plans the batch with one synchronised symbolic run: writes the total
   nnz over all C_i to *nnz_total and, when non-null, host arrays
   c_row_off[count+1] (first row of C_i in the pooled row pointer) and
   c_nnz_off[count+1] (first entry of C_i in the pooled column/value arrays). */
spg_status spg_batch_plan(spg_batch b, int64_t* nnz_total, int64_t* c_row_off, int64_t* c_nnz_off);

/* Runs all products as one graph launch on the batch's stream (asynchronous).
   a_val_pool / b_val_pool: device values in the column pools' layout.
   c_row_ptr: device int32[sum m + 1], the pooled row pointer (offsets into
   the C pools, so C_i's row pointer is its slice minus c_nnz_off[i]);
   c_col / c_val: device pools with capacity >= nnz_total entries.
   numeric_only = 0: both phases; 1: numeric alone on the planned structure
   (the planned row pointer is copied into c_row_ptr).  Allocates nothing;
   the graph is re-captured when a pointer or the mode changes. */
spg_status spg_batch_run(spg_batch b, const void* a_val_pool, const void* b_val_pool,
                         int32_t* c_row_ptr, int32_t* c_col, void* c_val, int64_t capacity,
                         int32_t numeric_only);

/* Autotuner: times every combination of products per lane {8,16,32},
   symbolic size bound (SPG_OPT_BINNING 2 or 0; a learned model is kept) and
   hashed-table block limit {32,64,128} on full runs of the batch (into the
   given output pools), keeps the fastest and re-plans.  chosen (host
   int32[3], may be NULL) receives the three settings in that order, best_ms
   (host, may be NULL) the best run time.  The trials replace the batch's
   plan and captured graph: if any trial fails, the call returns its status
   with the batch's options unchanged and the batch unplanned (spg_batch_run
   returns SPG_ERR_STATE until the next spg_batch_plan). */
spg_status spg_batch_tune(spg_batch b, const void* a_val_pool, const void* b_val_pool,
                          int32_t* c_row_ptr, int32_t* c_col, void* c_val, int64_t capacity,
                          int32_t* chosen, float* best_ms);

/* Both phases of every product in one persistent kernel over a device work
   queue, with no host work between the products (section 3: many small
   operations in one dispatch; section 2.2.2: launch latency).  Work items
   are (product, block of 128 rows, phase); a product's symbolic items
   compute its row sizes, the last of them to finish scans the product's
   row pointer (a segmented scan over the batch), takes the product's C
   space from a device bump allocator over the caller's pools and queues the
   product's numeric items.  Needs no spg_batch_plan; the first call runs
   one synchronised analysis of the batch (then the kernel is captured into
   a graph, replayed while the pointers and capacity stay the same) and
   returns SPG_ERR_UNSUPPORTED if a row of some C_i spans more than 4096
   columns (spg_batch_run has no such limit).  Asynchronous.
     c_row_ptr: device int32 pool of sum_i (m_i + 1) entries: C_i's row
       pointer at entry sum_{j<i} (m_j + 1), holding offsets into c_col and
       c_val (so C_i's entries are [c_row_ptr_i[0], c_row_ptr_i[m_i]));
     c_col, c_val: device pools of `capacity` entries, handed out to the
       products in the order their symbolic items finish;
     c_offsets: device int64[count]: C_i's first pool entry, or -1 if C_i
       did not fit in the pools (its numeric phase is skipped and its row
       pointer block left unwritten);
     stamps: device int64[2 * count] or NULL: per product the device clock
       (wall_clock64, 100 MHz) when its first work item started and when its
       last ended. */
spg_status spg_batch_run_queued(spg_batch b, const void* a_val_pool, const void* b_val_pool, int32_t* c_row_ptr,
                                int32_t* c_col, void* c_val, int64_t capacity, int64_t* c_offsets, int64_t* stamps);

/* Statistics of the batch's last planned or tuned symbolic run and of its
   numeric launches (per-class rows, products, times when timing is on). */
spg_status spg_batch_get_stats(spg_batch b, spg_stats* out, int32_t size);

/* ---- sparse matrix addition C = alpha*A + beta*B (section 2.3) ----------
   A and B are m x n CRS matrices; each row of C holds the union of the
   columns of A(i,:) and B(i,:), in ascending order, with every entry of one
   column (also repeats inside A's or B's row) added into one value; explicit
   zeros are kept.  Two phases as for the product: symbolic finds C's row
   pointer and, for every input entry, the position of its column in C's row
   (the paper's Apos and Bpos, kept in the handle); numeric scatters the
   scaled values there and may be called again with new values on the same
   structures.  Input rows may be unsorted; when both rows are in ascending
   column order the symbolic phase merges them (the merge network of a
   bitonic sort), otherwise it sorts them.  A row of A and B together may hold
   at most 16384 entries (SPG_ERR_UNSUPPORTED beyond). */
typedef struct spg_add_s* spg_add;

/* Creates an addition handle on `hip_stream` (hipStream_t; NULL = default). */
spg_status spg_add_create(spg_add* h, void* hip_stream);

/* Waits for the stream and frees the handle's device memory (null accepted). */
spg_status spg_add_destroy(spg_add h);

/* Message for the last failing call on h. */
const char* spg_add_last_error(spg_add h);

/* Symbolic phase: A and B structures (borrowed device arrays, which must stay
   valid and unchanged until the last spg_add_numeric), C's row pointer into
   the caller's device array c_row_ptr[m+1] (borrowed likewise), nnz(C) into
   *nnz_c (host).  Waits for the stream once.  SPG_ERR_INDEX for malformed
   input, SPG_ERR_OVERFLOW if nnz(C) >= 2^31, SPG_ERR_UNSUPPORTED for a row
   pair of more than 16384 entries, SPG_ERR_ALLOC if the handle's buffers
   (4 bytes per entry of A and B, 8 per row) cannot be allocated. */
spg_status spg_add_symbolic(spg_add h, int32_t m, int32_t n, const int32_t* a_row_ptr, const int32_t* a_col_idx,
                            int64_t a_nnz, const int32_t* b_row_ptr, const int32_t* b_col_idx, int64_t b_nnz,
                            int32_t* c_row_ptr, int64_t* nnz_c);

/* Numeric phase: c_col_idx[nnz(C)] and c_vals[nnz(C)] (caller's device
   arrays) from a_vals[a_nnz] and b_vals[b_nnz] (device, type dt); alpha and
   beta are converted to dt.  Each contribution is rounded once (alpha*a or
   beta*b) and added at its position, A's contributions before B's; repeats
   inside a row add in any order.  Asynchronous.  SPG_ERR_STATE without a
   symbolic result. */
spg_status spg_add_numeric(spg_add h, spg_dtype dt, double alpha, const void* a_vals, double beta,
                           const void* b_vals, int32_t* c_col_idx, void* c_vals);

#ifdef __cplusplus
}
#endif

#endif /* SPG_H */
