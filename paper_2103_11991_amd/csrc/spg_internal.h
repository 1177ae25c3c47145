// Internal declarations of the spg library (not part of the C ABI).
//
// Accumulator design.  Every row of C is accumulated in a table of 32-column
// blocks: a block id (column >> 5) carries a 32-bit mask of the columns seen
// so far.  The symbolic phase ORs masks in, as the paper's compressed
// accumulator does (section 2.2.1: columns represented by bits, bitwise OR as
// the accumulate operation); nnz(C(i,:)) is the sum of the masks' popcounts.
// It also stores each row's occupied blocks in ascending order as
// {block, mask} pairs (the row's list, C's structure in compressed form).
// The numeric phase reads the list back, turns it into ranks with a prefix
// sum of popcounts, and adds every product into a compact value array at
//     rank(c) = prefix[block(c)] + popcount(mask[block(c)] & ((1 << (c & 31)) - 1)),
// so the output comes out sorted without a sort of the columns themselves.
// A row's list has room for min(compressed-B runs its products read, words
// of its column range) pairs, a bound on its occupied blocks known before
// the symbolic phase; rows that the list memory cannot hold (and rows of the
// symbolic global path) take the numeric global path, which finds the masks
// from compressed B itself.
//
// The table is *direct* (indexed by block - first block of the row: the
// paper's dense accumulator restricted to the row's column range), *hashed*
// (the paper's HashmapAccumulator keyed by block id, open addressing with
// linear probing) or *two-level* (a bitmap of occupied blocks with running
// counts, then per occupied block its mask), whichever suits the row.  It
// lives in LDS for rows up to a per-row byte tier; longer rows take the
// global-memory path (section 2.2.1: second-level accumulator in slow global
// memory), where the mask table lives in LDS when it fits, else in a global
// slab, and values are summed in LDS segments of the rank space or, for the
// longest rows, straight into C's own storage with global atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spg.h"

namespace spg {

constexpr int NTIER = SPG_NTIER;     // tiers 0..8 in LDS, 9 = global memory
constexpr int NCLS = SPG_NCLASS;     // class = mode * NTIER + tier
constexpr int TIER_GLOBAL = 9;
constexpr int MODE_DIRECT = 0;
constexpr int MODE_HASHED = 1;
constexpr int MODE_TWOLEVEL = 2;
constexpr uint8_t CLS_EMPTY = 255;
constexpr int WIDE_THREADS = 1024;   // threads per row on the global path
constexpr int WIDE_WIN_BYTES = 2048;  // window table of the global path (K <= 8 windows x 16 waves)

// error flags in Control::err
constexpr int ERR_A_ROWPTR = 1;
constexpr int ERR_A_COL = 2;
constexpr int ERR_B_ROWPTR = 4;
constexpr int ERR_B_COL = 8;
constexpr int ERR_NNZ_OVERFLOW = 16;
// malformed input: kernels after the analysis exit at once when any is set
constexpr int ERR_INPUT = ERR_A_ROWPTR | ERR_A_COL | ERR_B_ROWPTR | ERR_B_COL;
constexpr int ERR_TABLE_OVERFLOW = 32;  // a bounded table overflowed (internal error)

// Per-tier geometry: LDS bytes per row, threads per row, rows per workgroup.
__host__ __device__ inline int tier_bytes(int t) { return 256 << t; }
__host__ __device__ inline int tier_threads(int t) {
    return t <= 2 ? (8 << t) : t <= 4 ? 64 : t == 5 ? 128 : t == 6 ? 256 : t == 7 ? 512 : 1024;
}
// rows per workgroup: groups of up to 64 lanes share a 256-lane workgroup
__host__ __device__ inline int tier_rows(int t) {
    int g = tier_threads(t);
    return g <= 64 ? 256 / g : 1;
}
// Flat product mapping of the row kernels: an A entry's B row is cut into
// groups of FLAT_VB consecutive entries (its compressed-B row into groups of
// FLAT_VC runs), each read with 16-byte loads; a batch gives every lane K
// slots, groups lane + G*k of the staged A chunk.
constexpr int FLAT_VB = 4;       // B entries per group
constexpr int FLAT_VC = 2;       // compressed-B runs per group (numeric global path)
constexpr int FLAT_VC_SYM = 1;   // compressed-B runs per group (symbolic)
constexpr int FLAT_KC = 5;       // run groups per lane and batch (symbolic; window table size)
constexpr int FLAT_KC_NUM = 3;   // numeric global path: run groups per lane and batch
constexpr int FLAT_KB_F64 = 3;   // B groups per lane and batch, FP64 values
constexpr int FLAT_KB_F32 = 4;   // B groups per lane and batch, FP32 values (window table size)
__host__ __device__ inline int group_waves(int g) { return g > 64 ? g / 64 : 1; }
// numeric staging of one row: per staged A entry its B {offset, end} pair
// and A's value (8 bytes each), then the window table (16 bytes per window
// and wavefront) of the batch in flight
__host__ __device__ inline int stage_bytes(int g) { return g * 16 + FLAT_KB_F32 * group_waves(g) * 16; }
// the symbolic phase stages no values and walks compressed B only
__host__ __device__ inline int sym_stage_bytes(int g) { return g * 8 + FLAT_KC * group_waves(g) * 16; }
// dynamic LDS of one workgroup of tier t: the rows' tables plus staging
__host__ __device__ inline int64_t tier_smem_bytes(int t) {
    return (int64_t)tier_rows(t) * (tier_bytes(t) + stage_bytes(tier_threads(t)));
}

__host__ __device__ inline int64_t pow2ceil64(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Runtime knobs of the class choice (copied into kernels by value).
struct ClassCfg {
    int32_t work_per_lane;    // products per lane that size a row's thread group
    int32_t hash_max_blocks;  // numeric hashed table only up to this many blocks
    int32_t lds_limit;        // LDS bytes per row beyond which rows go global
    int32_t force_class;      // -1 or a class id
    int32_t elem_bytes;       // 4 (FP32) or 8 (FP64)
    int32_t bound_est;        // symbolic tables sized from a guaranteed bound (1) or a prediction (0)
    int32_t pad[2];
};

// Row facts gathered by the analysis pass.
//   x = smallest column, y = largest column, z = products (capped at 2^31-1),
//   w = largest referenced B-row length
using RowInfo = int4;

// Table sizes, shared by the classifier and the kernels so both agree.
__host__ __device__ inline int64_t row_words(int32_t cmin, int32_t cmax) {
    return (int64_t)(cmax >> 5) - (int64_t)(cmin >> 5) + 1;
}
// Slots of a symbolic hashed table.  The table overflows (the row is retried
// on the global path) above three-quarter occupancy: a learned estimate gets
// 2x slots, a guaranteed upper bound 4/3x, enough never to reach that mark.
__host__ __device__ inline int64_t sym_hash_slots(int64_t est_blocks, bool bound = false) {
    const int64_t need = bound ? (est_blocks * 4 + 2) / 3 : est_blocks * 2;
    return pow2ceil64(need > 16 ? need : 16);
}
__host__ __device__ inline int64_t num_hash_slots(int64_t blocks) {
    return pow2ceil64(blocks * 2 > 16 ? blocks * 2 : 16);
}
__host__ __device__ inline int64_t align8(int64_t b) { return (b + 7) & ~(int64_t)7; }
__host__ __device__ inline int64_t num_direct_bytes(int64_t words, int64_t n, int eb) {
    return align8(words * 8) + n * eb;
}
// hashed numeric table: 16-byte slots {block, mask, prefix, -}
__host__ __device__ inline int64_t num_hashed_bytes(int64_t blocks, int64_t n, int eb) {
    return num_hash_slots(blocks) * 16 + n * eb;
}
// two-level numeric table: a {bits, first index} pair per 32 words of the
// row's block range (which blocks are occupied, and the list index of the
// first of them), then {mask, prefix} per occupied block
__host__ __device__ inline int64_t twolevel_words(int64_t words) { return (words + 31) / 32; }
__host__ __device__ inline int64_t num_twolevel_bytes(int64_t words, int64_t blocks, int64_t n, int eb) {
    return align8(twolevel_words(words) * 8 + blocks * 8) + n * eb;
}
// A row's list capacity: its compressed-B run count bounds its occupied
// blocks, and so does the width of its column range in words.
__host__ __device__ inline int32_t list_capacity(int64_t runs, int64_t words) {
    const int64_t c = runs < words ? runs : words;
    return c > INT32_MAX ? INT32_MAX : (int32_t)c;
}

// Smallest LDS tier that holds `bytes`, raised until its thread group gives
// at most work_per_lane products per lane; TIER_GLOBAL if it does not fit.
__host__ __device__ inline int pick_tier(int64_t bytes, int64_t work, const ClassCfg& c) {
    if (bytes > c.lds_limit) return TIER_GLOBAL;
    int t = 0;
    while (t < TIER_GLOBAL - 1 && tier_bytes(t) < bytes) ++t;
    if (tier_bytes(t) < bytes) return TIER_GLOBAL;
    while (t < TIER_GLOBAL - 1 && (int64_t)tier_threads(t) * c.work_per_lane < work &&
           tier_bytes(t + 1) <= c.lds_limit)
        ++t;
    return t;
}

// Bytes per occupied block of the symbolic two-level table: its mask and its
// id, kept as a 16-bit offset from the row's first block when the row's range
// spans at most 2^16 blocks.
__host__ __device__ inline int sym_block_bytes(int64_t words) { return words <= 65536 ? 6 : 8; }

// Symbolic class of a row from its products, column range and an estimate
// of its occupied blocks (an upper bound: the compressed-B runs its products
// read; or the learned prediction).
__host__ __device__ inline int sym_class(int64_t ub, int32_t cmin, int32_t cmax, int64_t est_blocks,
                                         const ClassCfg& c, bool bound = false) {
    if (ub <= 0) return CLS_EMPTY;
    int64_t words = row_words(cmin, cmax);
    int64_t est = est_blocks < words ? est_blocks : words;
    if (est < 1) est = 1;
    // direct: a mask per word; hashed: keys and masks; two-level: {bits,
    // prefix} per 32 words, a mask and the block id per (estimated) occupied block
    int64_t bd = words * 4, bh = sym_hash_slots(est, bound) * 8;
    int64_t b2 = align8(twolevel_words(words) * 8) + est * sym_block_bytes(words);
    if (c.force_class >= 0) {
        int fm = c.force_class / NTIER, ft = c.force_class % NTIER;
        if (ft == TIER_GLOBAL) return MODE_DIRECT * NTIER + TIER_GLOBAL;
        int64_t need = fm == MODE_DIRECT ? bd : fm == MODE_HASHED ? bh : b2;
        if (need <= tier_bytes(ft) && tier_bytes(ft) <= c.lds_limit) return c.force_class;
    }
    int mode = MODE_DIRECT;
    int64_t bytes = bd;
    if (b2 < bytes) mode = MODE_TWOLEVEL, bytes = b2;
    if (bh < bytes) mode = MODE_HASHED, bytes = bh;
    int t = pick_tier(bytes, ub, c);
    // a tier raised for the row's work may hold the direct table (one pass, no probing)
    if (t == TIER_GLOBAL || bd <= tier_bytes(t)) mode = MODE_DIRECT;
    return mode * NTIER + t;
}

// Numeric class of a row from its exact size n and occupied blocks: the
// direct table when the row's block range is about as small as its block
// count, else the two-level table; the hashed table for very wide, sparse
// rows with few blocks, when it is the smaller.
__host__ __device__ inline int num_class(int64_t ub, int32_t cmin, int32_t cmax, int64_t n, int64_t blocks,
                                         const ClassCfg& c) {
    if (n <= 0) return CLS_EMPTY;
    int64_t words = row_words(cmin, cmax);
    int eb = c.elem_bytes;
    int64_t bd = num_direct_bytes(words, n, eb), bh = num_hashed_bytes(blocks, n, eb);
    int64_t b2 = num_twolevel_bytes(words, blocks, n, eb);
    if (c.force_class >= 0) {
        int fm = c.force_class / NTIER, ft = c.force_class % NTIER;
        if (ft == TIER_GLOBAL) return MODE_DIRECT * NTIER + TIER_GLOBAL;
        int64_t need = fm == MODE_DIRECT ? bd : fm == MODE_HASHED ? bh : b2;
        if (need <= tier_bytes(ft) && tier_bytes(ft) <= c.lds_limit) return c.force_class;
    }
    int mode;
    int64_t bytes;
    if (words <= 2 * blocks + 8) mode = MODE_DIRECT, bytes = bd;
    else if (blocks <= c.hash_max_blocks && bh < b2) mode = MODE_HASHED, bytes = bh;
    else mode = MODE_TWOLEVEL, bytes = b2;
    int t = pick_tier(bytes, ub, c);
    // a tier raised for the row's work may hold the direct table (one lookup per product)
    if (t == TIER_GLOBAL || bd <= tier_bytes(t)) mode = MODE_DIRECT;
    return mode * NTIER + t;
}

// Launch classes: a class with few rows runs in the next populated class of
// the same mode and a larger LDS tier (up to 4x the lanes per row) when that
// class has at least 8x the rows.  The larger tier holds every table of the
// smaller one, so rows only change the launch they run in, and a short launch
// with its tail is saved.  Merges chain upwards.  remap gets the launch class
// of every class and merged the row counts per launch class.  The host and
// the grouping kernel both evaluate it on the same histogram.
__host__ __device__ inline void merge_classes(const int32_t* hist, uint8_t* remap, int32_t* merged, bool enable) {
    for (int c = 0; c < NCLS; ++c) remap[c] = (uint8_t)c, merged[c] = hist[c];
    if (!enable) return;
    for (int mode = 0; mode < 3; ++mode) {
        for (int t = 0; t < TIER_GLOBAL; ++t) {
            const int c = mode * NTIER + t;
            if (merged[c] == 0) continue;
            int u = t + 1;
            while (u < TIER_GLOBAL && merged[mode * NTIER + u] == 0) ++u;
            if (u >= TIER_GLOBAL || tier_threads(u) > 4 * tier_threads(t)) continue;
            const int d = mode * NTIER + u;
            if ((int64_t)merged[c] * 8 > merged[d]) continue;
            merged[d] += merged[c];
            merged[c] = 0;
            for (int e = 0; e < NCLS; ++e)
                if (remap[e] == c) remap[e] = (uint8_t)d;
        }
    }
}

// Device-side control block: counters and histograms the host reads back
// in one copy at each of symbolic's two synchronisation points.
struct Control {
    int32_t err;
    int32_t overflow_rows;        // learned binning: rows queued for retry
    int64_t products;             // sum of per-row products
    int64_t nnz_c;
    int32_t sym_hist[NCLS];
    int32_t num_hist[NCLS];
    int32_t empty_rows;
    int32_t mispredicted;
    int64_t max_words_sym_global; // widest row on the symbolic global path
    int64_t max_words_all;        // widest row overall (sizes retry slabs)
    int64_t max_words_num_global; // widest row on the numeric global path
    int64_t num_a_nnz[NCLS];
    int64_t num_c_nnz[NCLS];
    int64_t num_products[NCLS];
    int32_t tile_counter;         // dynamic tile id of the row-pointer scan
    int64_t bc_total;             // runs of compressed B
    int64_t list_total;           // list pairs reserved by the grouping of the symbolic rows
    int32_t tile_fallback;        // tiled global path: rows left to the segment path
    int32_t b_tile_unordered;     // tiled global path: a B row's entries are not grouped by tile
    int32_t tile_heavy;           // tiled global path: rows of more than TILE_G entries (one unit per tile)
    int32_t tile_light;           // tiled global path: rows of at most TILE_G entries (one unit per row)
    int32_t a_missing_diag;       // square A: rows without a stored diagonal entry
    int64_t max_products;         // most products of one row
    // symbolic grouping (tier-major: the three modes of a tier are adjacent):
    // rows and first slot of every launch class after the class merge
    int32_t sym_cnt[NCLS];
    int32_t sym_off[NCLS];
};

// ---- launch wrappers (spg_rows.hip) ----
void launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n);
void launch_fill_u8(hipStream_t s, void* p, uint8_t v, int64_t bytes);
// B rows in one pass: validation, binfo {length, smallest column, largest
// column, runs} and compressed B (section 2.2.1): per row its runs of entries
// sharing a 32-column block as {block, OR of the column bits}, stored from the
// row's own first entry on (bc holds b_nnz runs), and bhdr per row {first
// entry, length, first run, run count}.
void launch_b_rows(hipStream_t s, int32_t n, int32_t k, const int32_t* brp, const int32_t* bci, int64_t bnnz,
                   int4* binfo, int2* bc, int4* bhdr, Control* ctl);
void launch_a_rowinfo(hipStream_t s, int32_t m, int32_t n, const int32_t* arp, const int32_t* aci, int64_t annz,
                      const int4* binfo, RowInfo* rinfo, float* feats, ClassCfg cfg, int binning,
                      uint8_t* sym_cls, int32_t* row_nnz, int32_t* row_blocks, int32_t* lofs, Control* ctl);
void launch_mlp_classify(hipStream_t s, int32_t m, const float* feats, const float* w, const RowInfo* rinfo,
                         ClassCfg cfg, float margin, uint8_t* sym_cls, Control* ctl);
// groups rows by class; offsets come from the class histogram in device memory.
// perm gets the row ids, desc {row, arp[row], arp[row+1], crp ? crp[row] : 0}.
// With lofs (grouping of the symbolic rows): lofs holds each row's list
// capacity on entry and its list offset on exit (-1 for rows of the global
// path and rows past list_limit pairs), reserved from ctl->list_total; desc.w
// gets the same offset.
// With merge, rows are grouped by their launch class (merge_classes).
// Each class's rows come in ascending row order up to the order inside a
// chunk of 2048 rows.  state (scatter_state_bytes(m) bytes) is cleared here.
size_t scatter_state_bytes(int32_t m);
void launch_scatter(hipStream_t s, int32_t m, const uint8_t* cls, int merge, const int32_t* hist, int32_t* state,
                    int32_t* perm, const int32_t* arp, const int32_t* crp, int4* desc, int32_t* lofs = nullptr,
                    Control* ctl = nullptr, int64_t list_limit = 0);
void launch_scan(hipStream_t s, int32_t m, const int32_t* row_nnz, const int32_t* row_blocks, const RowInfo* rinfo,
                 const int32_t* arp, const uint8_t* sym_cls, const int32_t* lofs, int32_t* c_row_ptr,
                 uint64_t* tile_status, ClassCfg cfg, uint8_t* num_cls, Control* ctl);
void launch_export_rows(hipStream_t s, int32_t m, const float* feats, const int32_t* row_blocks,
                        const int32_t* row_nnz_in, float* x, float* y, int32_t* row_nnz_out);
int64_t scan_tiles(int32_t m);
// batched products: packs pooled per-product CSR arrays into one block-diagonal
// matrix; desc holds 7 int64 per product (see k_pack)
void launch_pack(hipStream_t s, int32_t count, const int64_t* desc, const int32_t* rp_pool, const int32_t* col_pool,
                 int32_t* rp_out, int32_t* col_out, int32_t* err);

// ---- accumulator kernels (spg_accum.hip) ----
struct SymArgs {
    const int32_t* perm;
    const int4* desc;             // per slot {row, A start, A end, list offset} (row kernels)
    int32_t count;
    int32_t tier;
    int32_t mode;
    const int32_t* arp;
    const int32_t* aci;
    const int32_t* brp;
    const int32_t* bci;
    const int2* bc;               // compressed B: {block, mask} runs (bhdr gives each row's)
    const int4* bhdr;             // per B row {start, length, run start, run count}
    int64_t bc_total;             // runs of compressed B (bound of the group loads)
    const RowInfo* rinfo;
    int32_t* row_nnz;
    int32_t* row_blocks;
    int32_t* ovf_list;            // rows whose hashed table overflowed
    Control* ctl;
    uint32_t* slab;               // global path: one mask table per workgroup
    int64_t slab_words;
    const int32_t* count_dev;     // global path: device-side row count (or null)
    const int32_t* off_dev;       // global path: device-side first slot in perm (or null)
    int32_t wide_lds;             // global path: LDS bytes per workgroup
    const int32_t* lofs;          // per row: first pair of its list, -1 if it has none
    int2* lists;                  // {block, mask} pairs of the rows' occupied blocks
};

struct NumArgs {
    const int32_t* perm;
    const int4* desc;             // per slot {row, A start, A end, C start} (row kernels)
    int32_t count;
    int32_t tier;
    int32_t mode;
    const int32_t* arp;
    const int32_t* aci;
    const void* av;
    const int32_t* brp;
    const int32_t* bci;
    const void* bv;
    const int2* bc;
    const int4* bhdr;             // per B row {start, length, run start, run count}
    int64_t bnnz;                 // entries of B and of compressed B (bounds of the
    int64_t bc_total;             // group loads near the arrays' ends)
    const int32_t* crp;
    const RowInfo* rinfo;
    const int32_t* row_blocks;
    int32_t* ccol;
    void* cval;
    uint32_t* slab;               // global path: masks and prefixes per workgroup
    int64_t slab_words;
    int32_t wide_lds;
    int32_t wide_vals;            // global path: values per LDS segment (0 = global atomics only)
    const int32_t* lofs;          // per row: first pair of its list, -1 if it has none
    const int2* lists;            // {block, mask} pairs in ascending block order
    const int32_t* count_dev;     // global path: device-side row count (or null)
    const void* dinv;             // Jacobi-fused product: D^-1 (m values), else null
    double omega;                 // Jacobi-fused product: the damping factor
};

// Tiled global path of the numeric phase (spg_accum.hip).  B's columns are
// cut into tiles of TILE_BYTES / 8 columns (the window sums in FP64 for
// either value type); a work item is one (row, tile) pair of a long row.
constexpr int TILE_BYTES = 32768;  // dense LDS window of one item
constexpr int TILE_G = 256;        // lanes per row
constexpr int TILE_MAX = 128;      // most tiles a matrix may have for this path
__host__ __device__ inline int tile_cols(int /*elem_bytes*/) { return TILE_BYTES / 8; }

struct TileArgs {
    int32_t n;                    // rows of B
    int32_t rows;                 // rows of the global class (R)
    int32_t ntiles;               // T
    int32_t log_cols;             // log2(columns per tile)
    const int32_t* perm;          // the class's rows (R entries)
    const int32_t* arp;
    const int32_t* aci;
    const void* av;
    const int32_t* brp;
    const int32_t* bci;
    const void* bv;
    int64_t bnnz;
    const int32_t* crp;
    const int32_t* lofs;
    const int32_t* row_blocks;
    const int2* lists;
    int32_t* toff;                // per B row, T + 1 tile offsets: first entry of each tile, then the row end
    int4* items;                  // [T][R]: {row, first list pair, end pair, rank of the first pair}
    int32_t* fallback;            // rows for the segment path (no list, or B rows not grouped by tile)
    int32_t* heavy;               // class slots of rows of more than TILE_G entries of A
    int32_t* light;               // class slots of the other rows
    Control* ctl;
    int32_t* ccol;
    void* cval;
    const void* dinv;             // Jacobi-fused product (see NumArgs)
    double omega;
};

// The paper's design (spg_paper.hip): one method for the whole matrix (a
// 16-lane group or a 256-lane team per row) with a two-level hash-map
// accumulator (LDS, then global memory created when a row needs it).
constexpr int PAPER_TEAM_PRODUCTS = 256;  // team method from this many products per nonempty row
struct PaperLaunch {
    int32_t m;
    int32_t team;
    int32_t grid;
    const int32_t* arp;
    const int32_t* aci;
    const void* av;
    const int32_t* brp;
    const int32_t* bci;
    const void* bv;
    const int2* bc;
    const int4* bhdr;
    const RowInfo* rinfo;
    int32_t* row_nnz;
    int32_t* row_blocks;
    const int32_t* crp;
    int32_t* ccol;
    void* cval;
    int32_t* slab;          // level-2 tables: grid * rows per workgroup of them
    int64_t slab_slots;     // slots of each
};
__host__ __device__ inline int paper_rows_per_wg(bool team) { return team ? 1 : 16; }
int launch_paper(hipStream_t s, const PaperLaunch& p, bool numeric, int elem_bytes, int n_cu);

// Batched products through one persistent kernel over a device work queue
// (spg_queue.hip).
struct QueueCtl {
    int64_t head;   // next queue slot to take
    int64_t tail;   // numeric slots appended so far
    int64_t used;   // entries of the C pools handed out (bump allocator)
    int64_t pad;    // nonzero if a numeric slot never filled (a wait gave up)
};
struct QueueArgs {
    int32_t count;              // products
    int32_t rb;                 // rows per work item
    int64_t n_items;            // symbolic items (as many numeric ones)
    const int64_t* item_off;    // count + 1: first symbolic item of each product
    const int64_t* row_off;     // count + 1: first packed row of each product
    const int64_t* crp_off;     // count: first entry of each product's row-pointer block (sum of m_q + 1)
    const int32_t* arp;
    const int32_t* aci;
    const void* av;
    const int32_t* brp;
    const int32_t* bci;
    const void* bv;
    const RowInfo* rinfo;
    int32_t* row_nnz;
    int32_t* c_row_ptr;
    int32_t* ccol;
    void* cval;
    int64_t cap;                // entries of the C pools
    int64_t* c_offsets;         // count: each product's first pool entry, -1 if it did not fit
    int64_t* stamps;            // 2 * count or null: first start, last end of each product's items
    QueueCtl* qc;
    int32_t* sym_left;          // count: symbolic items not yet done
    int64_t* queue;             // n_items numeric slots: (product << 32 | block) + 1, negated to skip, 0 = empty
    int32_t wmax;               // bitmap words of the widest row
    int32_t vmax;               // columns of the widest row's range
    uint32_t* qbm;              // each row's bitmap (wmax words per packed row) from the symbolic
                                // items for the numeric ones, or null (numeric ORs B again)
    const int2* bc;             // compressed B runs {block, mask} (symbolic), or null (entries)
    const int4* bhdr;           // per B row {start, length, run start, run count}
    int64_t bnnz;               // entries of B's pools
};
constexpr int QUEUE_MAX_WORDS = 128;  // widest row range the queued kernel holds (4096 columns)
size_t queue_lds_bytes(int wmax, int vmax, int elem_bytes);
void launch_queue(hipStream_t s, const QueueArgs& a, int elem_bytes, int grid);

// Tile offsets of B and the work items (once per symbolic result), then the
// tiled numeric launch; returns the grid used.
void launch_tile_build(hipStream_t s, const TileArgs& a);
int launch_num_tiled(hipStream_t s, const TileArgs& a, int elem_bytes, int n_cu);

// Launches one symbolic class; returns the grid size used.
int launch_sym_class(hipStream_t s, const SymArgs& a, int grid_cap);
// Launch offsets of the symbolic grouping: tier-major, so that the three
// table modes of one tier are adjacent (one persistent launch takes them).
__host__ __device__ inline void sym_class_offsets(const int32_t* rows, int32_t* off) {
    int32_t run = 0;
    for (int t = 0; t < NTIER; ++t)
        for (int md = 0; md < 3; ++md) {
            const int c = md * NTIER + t;
            off[c] = run, run += rows[c];
        }
}
// Symbolic rows of LDS tier a.tier (all three table modes), sized on the
// device: the kernel reads the tier's rows and first slot from the control
// block the grouping kernel wrote.  Persistent: the grid (a multiple of 8,
// at most what the device holds at once, at most one workgroup per row
// group of max_rows) walks the tier's row groups, each XCD a contiguous
// share of them.  Returns the grid.
int launch_sym_tier(hipStream_t s, const SymArgs& a, int64_t max_rows, int n_cu);
int launch_num_class(hipStream_t s, const NumArgs& a, int elem_bytes, int grid_cap);

}  // namespace spg
