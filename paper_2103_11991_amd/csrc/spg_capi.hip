// Handle, host runtime and the extern "C" boundary of the spg library.
//
// The call order follows the paper's statement of the two phases (section
// 2.2.1): the caller allocates C's row pointer, symbolic fills it and returns
// nnz(C), the caller allocates column indices and values, numeric fills them.
// The handle carries the runtime algorithm choices (section 6) and every
// intermediate buffer, so a repeated numeric call reuses the symbolic result
// (row classes, row permutation and C's row pointer) without recomputing it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "spg_internal.h"

using namespace spg;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool pooled = false;  // from the library's stream-ordered pool
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

enum EvId { EV_SYM0 = 0, EV_SYM1, EV_ANA1, EV_MLP0, EV_MLP1, EV_SCAN0, EV_SCAN1, EV_NUM0, EV_NUM1, EV_FIXED };
constexpr int EV_SYMCLS = EV_FIXED;                 // 2 per class
constexpr int EV_NUMCLS = EV_FIXED + 2 * NCLS;      // 2 per class, two alternating sets
constexpr int EV_TOTAL = EV_FIXED + 6 * NCLS;

}  // namespace

struct spg_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 256;
    int max_lds = 65536;
    std::string err;

    // inputs
    bool have_mats = false;
    spg_dtype dt = SPG_F64;
    int32_t m = 0, n = 0, k = 0;
    const int32_t *arp = nullptr, *aci = nullptr, *brp = nullptr, *bci = nullptr;
    int64_t annz = 0, bnnz = 0;

    // options
    int binning = 2;
    int timing = 0;
    int force_class = -1;
    int work_per_lane = 16;
    int hash_max_blocks = 64;
    int lds_limit = 65536;
    int mlp_margin_milli = 500;
    int keep_features = 0;
    int64_t list_limit_mb = 8192;
    int merge_classes = 1;
    int tiled_global = 1;
    int method = 0;            // 0: per-row classes; 1..3: the paper's design (auto, vector, team)
    bool have_mlp = false;

    // scratch
    DevBuf binfo, rinfo, feats, sym_cls, num_cls, perm_sym, perm_num, desc_sym, desc_num, row_nnz, row_blocks,
        tile_status, cursor,
        ovf_list, ctl, slab_sym, slab_retry, slab_num, mlp_w, bc, bhdr, lofs, lists, toff, titems, tfb, slab_paper;
    Control* hctl = nullptr;  // pinned host copy
    hipEvent_t ev_ctl = nullptr;  // marks the copy of the control block after the row-pointer scan

    // symbolic result
    bool have_sym = false;
    bool have_feats = false;
    bool blocks_valid = false;  // row_blocks holds the exact counts of the current matrices
    int32_t* crp = nullptr;
    int64_t nnz_c = 0;
    int32_t num_hist[NCLS] = {};
    int32_t num_off[NCLS] = {};
    int64_t slab_num_words = 0;
    int nslab_num = 0;
    // symbolic buffers reserved before the phase runs (host-known bounds)
    int64_t bc_runs = 0;          // compressed-B capacity in runs
    int64_t list_cap = 0;         // list pairs the grouping may hand out
    int64_t slab_sym_words = 0;   // per-workgroup slab of the symbolic global path (0: none)
    int sym_global_grid = 0;      // its workgroups (0: no row can take the global path)
    int64_t slab_retry_words = 0; // per-workgroup slab of the learned-size retry
    int retry_grid = 0;
    bool single_wait = false;     // this symbolic call waits for the device once
    int sym_waits = 0;            // host waits of the last symbolic call
    bool paper_team = false;   // the paper's design: team method (else vector method)
    int paper_grid = 0;
    int64_t paper_sym_slots = 0, paper_num_slots = 0;
    bool tiled = false;        // the numeric global class runs on the tiled path
    bool tiled_built = false;  // its tile offsets and items exist for this symbolic result
    int ntiles = 0;
    ClassCfg cfg{};
    Control geom{};  // control block after the analysis of the last symbolic run

    // stats and timing
    spg_stats stats{};
    hipEvent_t ev[EV_TOTAL] = {};
    bool ev_made = false;
    bool sym_timed = false, num_timed = false;
    bool sym_cls_timed[NCLS] = {}, num_cls_timed[NCLS] = {};
    // numeric class launches: two event sets used in turn; a set's previous
    // pair is read (long complete by then) when the set is reused or stats
    // are read, and summed per class
    int num_set = 0, num_last_set = 0;
    bool num_pending[2][NCLS] = {};
    double num_acc_ms[NCLS] = {};
    int32_t num_acc_n[NCLS] = {};
};

namespace {

spg_status fail(spg_handle h, spg_status s, const std::string& msg) {
    if (h) h->err = msg;
    return s;
}

spg_status hip_fail(spg_handle h, hipError_t e, const char* what) {
    return fail(h, SPG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, call)                                  \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

// Device memory of every handle comes from one stream-ordered pool per device
// that keeps up to 2 GiB of freed memory for reuse, so a handle created per
// product (a chain of small products) allocates without driver calls.  Null
// if the device has no pool support: plain hipMalloc then.
hipMemPool_t lib_pool(int device) {
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    static bool tried[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0 || device >= 64) return nullptr;
    if (!tried[device]) {
        tried[device] = true;
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        if (hipMemPoolCreate(&pools[device], &props) != hipSuccess) {
            pools[device] = nullptr;
            (void)hipGetLastError();
        } else {
            uint64_t keep = 2ull << 30;
            (void)hipMemPoolSetAttribute(pools[device], hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    return pools[device];
}

void release(DevBuf& b, hipStream_t s) {
    if (b.p) {
        if (b.pooled) (void)hipFreeAsync(b.p, s);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    b.pooled = false;
}

// Buffers (and pinned control blocks) of destroyed handles, kept per device
// for the handles created after them: a chain of products that creates a
// handle per product then allocates nothing after its first products (each
// allocation or free is a runtime call of several microseconds, and a
// handle has about twenty-five buffers).  A buffer enters only once its
// handle's stream has finished (spg_destroy waits for it first), so a new
// owner on another stream finds it idle.  At most 2 GiB are kept; a taken
// buffer is at most twice (plus 1 MiB) the size asked for.
struct CachedBuf {
    void* p;
    size_t cap;
    int device;
    bool pooled;
};
std::mutex g_cache_mu;
std::vector<CachedBuf> g_cache;
size_t g_cache_bytes = 0;
std::vector<Control*> g_pinned;
constexpr size_t CACHE_MAX_BYTES = (size_t)2 << 30;

bool cache_take(int device, size_t bytes, DevBuf& b) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache.size(); ++i) {
        const CachedBuf& c = g_cache[i];
        if (c.device != device || c.cap < bytes || c.cap > 2 * bytes + ((size_t)1 << 20)) continue;
        if (best < 0 || c.cap < g_cache[best].cap) best = i;
    }
    if (best < 0) return false;
    b.p = g_cache[best].p, b.cap = g_cache[best].cap, b.pooled = g_cache[best].pooled;
    g_cache_bytes -= b.cap;
    g_cache[best] = g_cache.back();
    g_cache.pop_back();
    return true;
}

// b's buffer into the cache (b idle), or freed when the cache is full.
void cache_put(int device, DevBuf& b) {
    if (!b.p) return;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        if (g_cache_bytes + b.cap <= CACHE_MAX_BYTES) {
            g_cache.push_back(CachedBuf{b.p, b.cap, device, b.pooled});
            g_cache_bytes += b.cap;
            b.p = nullptr, b.cap = 0, b.pooled = false;
            return;
        }
    }
    (void)hipFree(b.p);
    b.p = nullptr, b.cap = 0, b.pooled = false;
}

Control* pinned_take() {
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        if (!g_pinned.empty()) {
            Control* c = g_pinned.back();
            g_pinned.pop_back();
            return c;
        }
    }
    Control* c = nullptr;
    if (hipHostMalloc((void**)&c, sizeof(Control), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return c;
}

void pinned_put(Control* c) {
    if (!c) return;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        if (g_pinned.size() < 256) {
            g_pinned.push_back(c);
            return;
        }
    }
    (void)hipHostFree(c);
}

// Grows b to at least `bytes` on the handle's stream (contents not kept).
spg_status ensure(spg_handle h, DevBuf& b, size_t bytes) {
    if (bytes <= b.cap && b.p) return SPG_OK;
    release(b, h->stream);
    size_t want = std::max<size_t>(bytes, 256);
    if (cache_take(h->device, want, b)) return SPG_OK;
    hipMemPool_t pool = lib_pool(h->device);
    hipError_t e = pool ? hipMallocFromPoolAsync(&b.p, want, pool, h->stream) : hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(h, SPG_ERR_ALLOC, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.cap = want;
    b.pooled = pool != nullptr;
    return SPG_OK;
}

#define SPG_TRY(call)                 \
    do {                              \
        spg_status s_ = (call);       \
        if (s_ != SPG_OK) return s_;  \
    } while (0)

int num_ev(int set, int c) { return EV_NUMCLS + 2 * NCLS * set + 2 * c; }

float elapsed(spg_handle h, int a, int b);

// adds a numeric class launch's recorded time to the class's sum
void resolve_num(spg_handle h, int set, int c) {
    if (!h->num_pending[set][c]) return;
    h->num_pending[set][c] = false;
    const float ms = elapsed(h, num_ev(set, c), num_ev(set, c) + 1);
    if (ms >= 0.f) h->num_acc_ms[c] += ms, h->num_acc_n[c] += 1;
}

void reset_num_sums(spg_handle h) {
    for (int c = 0; c < NCLS; ++c) {
        h->num_pending[0][c] = h->num_pending[1][c] = false;
        h->num_acc_ms[c] = 0.0;
        h->num_acc_n[c] = 0;
    }
}

spg_status make_events(spg_handle h) {
    if (h->ev_made) return SPG_OK;
    for (int i = 0; i < EV_TOTAL; ++i) HIP_TRY(h, hipEventCreate(&h->ev[i]));
    h->ev_made = true;
    return SPG_OK;
}

// events of the phases and of every launch (timing 1)
void rec(spg_handle h, int id) {
    if (h->timing == 1) (void)hipEventRecord(h->ev[id], h->stream);
}

float elapsed(spg_handle h, int a, int b) {
    float ms = 0.f;
    if (hipEventSynchronize(h->ev[b]) != hipSuccess) return -1.f;
    if (hipEventElapsedTime(&ms, h->ev[a], h->ev[b]) != hipSuccess) return -1.f;
    return ms;
}


ClassCfg make_cfg(spg_handle h) {
    ClassCfg c{};
    c.work_per_lane = h->work_per_lane;
    c.hash_max_blocks = h->hash_max_blocks;
    c.lds_limit = h->lds_limit;
    c.force_class = h->force_class;
    c.elem_bytes = h->dt == SPG_F64 ? 8 : 4;
    c.bound_est = h->binning != 1;
    return c;
}

int wide_lds(spg_handle h) {
    // table LDS of a global-path workgroup: 64 KB, less if the device cannot
    // give it together with the 16 KB of staged A entries
    int v = 65536;
    while (v > 4096 && v + WIDE_THREADS * 16 + WIDE_WIN_BYTES + 1024 > h->max_lds) v >>= 1;
    return v;
}

// values per LDS segment of a global-path numeric workgroup: what the device
// leaves beside the mask table and the staged entries, 0 if under 4 KB
int wide_vals(spg_handle h, int eb) {
    const int64_t left = (int64_t)h->max_lds - wide_lds(h) - WIDE_THREADS * 16 - WIDE_WIN_BYTES - 1024;
    return left >= 4096 ? (int)((left & ~(int64_t)255) / eb) : 0;
}

// small classes run in larger ones unless a class is forced
int merging(spg_handle h) { return h->merge_classes && h->force_class < 0; }

// list pairs the list memory may hold (8 bytes each; offsets stay in int32)
int64_t list_limit_pairs(spg_handle h) { return h->list_limit_mb * (1 << 20) / 8; }

int clamp_lds_limit(spg_handle h, int v) {
    // largest tier whose workgroup (tables + staging) fits the device's LDS
    while (v > 1024) {
        int t = 0;
        while (tier_bytes(t) < v) ++t;
        if (tier_smem_bytes(t) + 1024 <= h->max_lds) break;
        v >>= 1;
    }
    return v;
}

spg_status sync_ctl(spg_handle h) {
    HIP_TRY(h, hipMemcpyAsync(h->hctl, h->ctl.p, sizeof(Control), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return SPG_OK;
}

spg_status check_input_errors(spg_handle h) {
    int e = h->hctl->err;
    if (e & (ERR_A_ROWPTR | ERR_B_ROWPTR))
        return fail(h, SPG_ERR_INDEX, std::string("malformed row pointer in ") + ((e & ERR_A_ROWPTR) ? "A" : "B"));
    if (e & (ERR_A_COL | ERR_B_COL))
        return fail(h, SPG_ERR_INDEX, std::string("column index out of range in ") + ((e & ERR_A_COL) ? "A" : "B"));
    return SPG_OK;
}


// ---- stages of the symbolic phase ----------------------------------------
// sym_prepare      buffers for the current matrices (may allocate)
// sym_stage_analysis  launches: control reset, B and A row analysis, learned classes,
//                  grouping by symbolic class with the rows' list offsets
// sym_stage_rows   launches: compressed B, accumulators, retry, scan, numeric grouping;
//                  launch geometry from h->geom (the control block read back after analysis)
// sym_finish       host bookkeeping from the control block read back after the scan
// A batch replays analysis + rows + numeric from a captured graph with the
// geometry of its first synchronised run (the structure is fixed).

spg_status reserve_symbolic(spg_handle h);

spg_status sym_prepare(spg_handle h) {
    const int32_t m = h->m;
    const bool learned = h->binning == 1;
    const bool want_feats = learned || h->keep_features;
    const size_t M = (size_t)std::max(m, 1);
    SPG_TRY(ensure(h, h->ctl, sizeof(Control)));
    SPG_TRY(ensure(h, h->binfo, (size_t)std::max(h->n, 1) * sizeof(int4)));
    SPG_TRY(ensure(h, h->rinfo, M * sizeof(RowInfo)));
    SPG_TRY(ensure(h, h->sym_cls, M));
    SPG_TRY(ensure(h, h->num_cls, M));
    SPG_TRY(ensure(h, h->perm_sym, M * 4));
    SPG_TRY(ensure(h, h->perm_num, M * 4));
    SPG_TRY(ensure(h, h->desc_sym, M * sizeof(int4)));
    SPG_TRY(ensure(h, h->desc_num, M * sizeof(int4)));
    SPG_TRY(ensure(h, h->row_nnz, M * 4));
    SPG_TRY(ensure(h, h->row_blocks, M * 4));
    SPG_TRY(ensure(h, h->tile_status, (size_t)(scan_tiles(std::max(m, h->n)) + 1) * 8));
    SPG_TRY(ensure(h, h->bhdr, (size_t)std::max(h->n, 1) * sizeof(int4)));
    SPG_TRY(ensure(h, h->cursor, scatter_state_bytes(m)));
    SPG_TRY(ensure(h, h->lofs, M * 4));
    if (learned) SPG_TRY(ensure(h, h->ovf_list, M * 4));
    if (want_feats) SPG_TRY(ensure(h, h->feats, M * 12));
    h->cfg = make_cfg(h);
    return reserve_symbolic(h);
}

// The symbolic phase waits for the device once (for the control block read
// back after the row-pointer scan) when the buffers it fills can be sized
// before it runs from what the host knows: compressed B holds at most one
// run per entry of B, a row's list at most one pair per word of its column
// range, a global-path slab the widest range a row can have.  Every launch
// then reads its rows from the control block the grouping kernel wrote.  The
// list bound m x (k/32 + 1) pairs is reserved for real, so this holds up to
// SINGLE_WAIT_PAIRS pairs (256 MiB): the small, latency-bound products.  A
// larger product reads the control block back after the analysis too (a
// second wait, about 12 us) and allocates the exact list, slab and launch
// sizes it finds there.
constexpr int64_t SINGLE_WAIT_PAIRS = (int64_t)32 << 20;

spg_status reserve_symbolic(spg_handle h) {
    const int64_t words_k = ((int64_t)h->k + 31) / 32 + 1;
    const int64_t list_bound = (int64_t)std::max(h->m, 1) * words_k;
    h->single_wait = !h->method && list_bound <= std::min(SINGLE_WAIT_PAIRS, list_limit_pairs(h));
    h->bc_runs = std::max<int64_t>(h->bnnz, 1);
    SPG_TRY(ensure(h, h->bc, (size_t)h->bc_runs * sizeof(int2)));
    h->slab_sym_words = 0;
    h->sym_global_grid = 0;
    h->slab_retry_words = 0;
    h->retry_grid = (int)std::min<int64_t>(64, std::max<int64_t>(h->m, 1));
    if (!h->single_wait) {
        h->list_cap = list_limit_pairs(h);  // the grouping's limit; the list is allocated after the analysis
        return SPG_OK;
    }
    SPG_TRY(ensure(h, h->lists, (size_t)list_bound * 8));
    h->list_cap = list_bound;
    const int wl = wide_lds(h);
    const int64_t slab_words = (words_k + 63) & ~(int64_t)63;
    const bool slab = words_k * 4 > wl;
    // the symbolic global path: rows whose smallest table exceeds the LDS
    // limit (impossible when a direct table of the widest range fits it),
    // and rows forced there
    const bool global = words_k * 4 > h->cfg.lds_limit || (h->force_class >= 0 && h->force_class % NTIER == TIER_GLOBAL);
    if (global) {
        h->sym_global_grid = (int)std::min<int64_t>(2 * h->n_cu, std::max<int64_t>(h->m, 1));
        if (slab) {
            SPG_TRY(ensure(h, h->slab_sym, (size_t)h->sym_global_grid * slab_words * 4));
            h->slab_sym_words = slab_words;
        }
    }
    if (h->binning == 1 && slab) {
        SPG_TRY(ensure(h, h->slab_retry, (size_t)h->retry_grid * slab_words * 4));
        h->slab_retry_words = slab_words;
    }
    return SPG_OK;
}

// The second-wait path: list, slabs and launch sizes from the analysis read
// back into h->geom.
spg_status size_from_analysis(spg_handle h) {
    const Control& hc = h->geom;
    const int wl = wide_lds(h);
    SPG_TRY(ensure(h, h->lists, (size_t)std::max<int64_t>(std::min(hc.list_total, list_limit_pairs(h)), 1) * 8));
    int32_t hist[NCLS];
    uint8_t remap[NCLS];
    merge_classes(hc.sym_hist, remap, hist, merging(h) != 0);
    const int gcls = MODE_DIRECT * NTIER + TIER_GLOBAL;
    h->sym_global_grid = std::min(hist[gcls], 2 * h->n_cu);
    h->slab_sym_words = 0;
    if (hist[gcls] > 0 && hc.max_words_sym_global * 4 > wl) {
        h->slab_sym_words = (hc.max_words_sym_global + 63) & ~(int64_t)63;
        SPG_TRY(ensure(h, h->slab_sym, (size_t)h->sym_global_grid * h->slab_sym_words * 4));
    }
    h->slab_retry_words = 0;
    if (h->binning == 1 && hc.max_words_all * 4 > wl) {
        h->slab_retry_words = (hc.max_words_all + 63) & ~(int64_t)63;
        SPG_TRY(ensure(h, h->slab_retry, (size_t)h->retry_grid * h->slab_retry_words * 4));
    }
    return SPG_OK;
}

void sym_stage_analysis(spg_handle h) {
    hipStream_t s = h->stream;
    const bool learned = h->binning == 1;
    const bool want_feats = learned || h->keep_features;
    Control* ctl = h->ctl.as<Control>();
    launch_fill_u8(s, ctl, 0, sizeof(Control));
    if (h->m == 0) return;
    launch_b_rows(s, h->n, h->k, h->brp, h->bci, h->bnnz, h->binfo.as<int4>(), h->bc.as<int2>(), h->bhdr.as<int4>(),
                  ctl);
    launch_a_rowinfo(s, h->m, h->n, h->arp, h->aci, h->annz, h->binfo.as<int4>(), h->rinfo.as<RowInfo>(),
                     want_feats ? h->feats.as<float>() : nullptr, h->cfg, h->binning, h->sym_cls.as<uint8_t>(),
                     h->row_nnz.as<int32_t>(), h->row_blocks.as<int32_t>(), h->lofs.as<int32_t>(), ctl);
    if (learned) {
        rec(h, EV_MLP0);
        launch_mlp_classify(s, h->m, h->feats.as<float>(), h->mlp_w.as<float>(), h->rinfo.as<RowInfo>(), h->cfg,
                            h->mlp_margin_milli / 1000.0f, h->sym_cls.as<uint8_t>(), ctl);
        rec(h, EV_MLP1);
    }
    // rows grouped by symbolic launch class (small classes merged); each
    // row's list placed (the total is read back)
    launch_scatter(s, h->m, h->sym_cls.as<uint8_t>(), merging(h), ctl->sym_hist, h->cursor.as<int32_t>(),
                   h->perm_sym.as<int32_t>(), h->arp, nullptr, h->desc_sym.as<int4>(), h->lofs.as<int32_t>(), ctl,
                   h->list_cap);
    rec(h, EV_ANA1);
}

// (with read_back, the control block is copied to the host right after the
// row-pointer scan and an event marks the copy: the host needs nothing the
// numeric grouping after it changes, and need not wait for it)
// (host_sized: launch per class from the histogram in h->geom even when the
// handle could size its launches on the device; a captured batch graph
// replays launches sized once by its planning run)
spg_status sym_stage_rows(spg_handle h, int32_t* c_row_ptr, bool read_back = false, bool host_sized = false) {
    hipStream_t s = h->stream;
    const int32_t m = h->m;
    const bool learned = h->binning == 1;
    Control* ctl = h->ctl.as<Control>();
    const int wl = wide_lds(h);
    SymArgs base{};
    base.arp = h->arp, base.aci = h->aci, base.brp = h->brp, base.bci = h->bci;
    base.bc = h->bc.as<int2>(), base.bhdr = h->bhdr.as<int4>();
    base.bc_total = h->bc_runs;
    base.rinfo = h->rinfo.as<RowInfo>();
    base.row_nnz = h->row_nnz.as<int32_t>();
    base.row_blocks = h->row_blocks.as<int32_t>();
    base.ctl = ctl;
    base.wide_lds = wl;
    base.lofs = h->lofs.as<int32_t>();
    base.lists = h->lists.as<int2>();
    base.ovf_list = learned ? h->ovf_list.as<int32_t>() : nullptr;  // learned sizes may overflow: retried
    if (h->method) {
        // the paper's design: one method for the whole matrix, two-level hash
        // maps; sized from the analysis read back before this stage
        const Control& hc = h->geom;
        const int64_t rows = std::max<int64_t>(1, (int64_t)m - hc.empty_rows);
        h->paper_team = h->method == 3 || (h->method == 1 && hc.products >= (int64_t)PAPER_TEAM_PRODUCTS * rows);
        const int rpw = paper_rows_per_wg(h->paper_team);
        // as many workgroups as the LDS of the chip holds at once (a team's
        // maps take ~37 KB, a group workgroup's ~25-49 KB)
        h->paper_grid = (int)std::min<int64_t>(((int64_t)m + rpw - 1) / rpw, (int64_t)h->n_cu * (h->paper_team ? 4 : 3));
        auto slots = [](int64_t bound) {
            int64_t s = 16;
            while (s < 2 * bound) s <<= 1;
            return s;
        };
        h->paper_sym_slots = slots(std::min<int64_t>(hc.max_products, hc.max_words_all));
        h->paper_num_slots = slots(std::min<int64_t>(hc.max_products, 32 * hc.max_words_all));
        // level-2 regions (symbolic: keys, masks, used; numeric: keys, used,
        // 8-byte values), zero when allocated and left zero by every row
        const int64_t per = std::max(3 * h->paper_sym_slots, 4 * h->paper_num_slots);
        const size_t bytes = (size_t)h->paper_grid * rpw * per * 4;
        const void* before = h->slab_paper.p;
        SPG_TRY(ensure(h, h->slab_paper, bytes));
        if (h->slab_paper.p != before) launch_fill_u8(s, h->slab_paper.p, 0, h->slab_paper.cap);
        PaperLaunch p{};
        p.m = m, p.team = h->paper_team, p.grid = h->paper_grid;
        p.arp = h->arp, p.aci = h->aci, p.brp = h->brp, p.bci = h->bci;
        p.bc = h->bc.as<int2>(), p.bhdr = h->bhdr.as<int4>(), p.rinfo = h->rinfo.as<RowInfo>();
        p.row_nnz = h->row_nnz.as<int32_t>(), p.row_blocks = h->row_blocks.as<int32_t>();
        p.slab = h->slab_paper.as<int32_t>(), p.slab_slots = h->paper_sym_slots;
        rec(h, EV_SYMCLS);
        launch_paper(s, p, false, h->dt == SPG_F64 ? 8 : 4, h->n_cu);
        rec(h, EV_SYMCLS + 1);
        h->sym_cls_timed[0] = h->timing == 1;
    } else if (h->single_wait && !host_sized) {
        // one persistent launch per LDS tier (its three table modes); each
        // reads its rows from the control block the grouping kernel wrote,
        // so no launch waits for the host.  Tiers above the LDS limit never
        // get rows.  Times are kept per tier (in the tier's direct class).
        for (int t = 0; t < TIER_GLOBAL; ++t) {
            if (tier_bytes(t) > h->cfg.lds_limit) continue;
            SymArgs a = base;
            a.perm = h->perm_sym.as<int32_t>();
            a.desc = h->desc_sym.as<int4>();
            a.tier = t;
            rec(h, EV_SYMCLS + 2 * t);
            launch_sym_tier(s, a, m, h->n_cu);
            rec(h, EV_SYMCLS + 2 * t + 1);
            h->sym_cls_timed[t] = h->timing == 1;
        }
        if (h->sym_global_grid > 0) {
            const int gcls = MODE_DIRECT * NTIER + TIER_GLOBAL;
            SymArgs a = base;
            a.perm = h->perm_sym.as<int32_t>();
            a.count_dev = &ctl->sym_cnt[gcls];
            a.off_dev = &ctl->sym_off[gcls];
            a.tier = TIER_GLOBAL;
            a.mode = MODE_DIRECT;
            a.slab = h->slab_sym_words ? h->slab_sym.as<uint32_t>() : nullptr;
            a.slab_words = h->slab_sym_words;
            rec(h, EV_SYMCLS + 2 * gcls);
            launch_sym_class(s, a, h->sym_global_grid);
            rec(h, EV_SYMCLS + 2 * gcls + 1);
            h->sym_cls_timed[gcls] = h->timing == 1;
        }
    } else {
        // one launch per populated class, sized from the analysis read back
        int32_t hist[NCLS], off[NCLS];
        uint8_t remap[NCLS];
        merge_classes(h->geom.sym_hist, remap, hist, merging(h) != 0);
        sym_class_offsets(hist, off);
        for (int c = 0; c < NCLS; ++c) {
            if (!hist[c]) continue;
            SymArgs a = base;
            a.perm = h->perm_sym.as<int32_t>() + off[c];
            a.desc = h->desc_sym.as<int4>() + off[c];
            a.count = hist[c];
            a.tier = c % NTIER;
            a.mode = c / NTIER;
            if (a.tier == TIER_GLOBAL) {
                a.slab = h->slab_sym_words ? h->slab_sym.as<uint32_t>() : nullptr;
                a.slab_words = h->slab_sym_words;
            }
            rec(h, EV_SYMCLS + 2 * c);
            launch_sym_class(s, a, 2 * h->n_cu);
            rec(h, EV_SYMCLS + 2 * c + 1);
            h->sym_cls_timed[c] = h->timing == 1;
        }
    }
    if (learned && !h->method) {
        // exact retry of overflowed rows on the global path (row count read on the device)
        SymArgs a = base;
        a.perm = h->ovf_list.as<int32_t>();
        a.count = 0;
        a.count_dev = &ctl->overflow_rows;
        a.tier = TIER_GLOBAL;
        a.mode = MODE_DIRECT;
        a.slab = h->slab_retry_words ? h->slab_retry.as<uint32_t>() : nullptr;
        a.slab_words = h->slab_retry_words;
        launch_sym_class(s, a, h->retry_grid);
    }
    // row pointer and numeric classes
    rec(h, EV_SCAN0);
    launch_fill_u8(s, h->tile_status.p, 0, (scan_tiles(m) + 1) * 8);
    launch_scan(s, m, h->row_nnz.as<int32_t>(), h->row_blocks.as<int32_t>(), h->rinfo.as<RowInfo>(), h->arp,
                h->sym_cls.as<uint8_t>(), h->lofs.as<int32_t>(), c_row_ptr, h->tile_status.as<uint64_t>(), h->cfg,
                h->num_cls.as<uint8_t>(), ctl);
    rec(h, EV_SCAN1);
    if (read_back) {
        if (!h->ev_ctl) HIP_TRY(h, hipEventCreateWithFlags(&h->ev_ctl, hipEventDisableTiming));
        HIP_TRY(h, hipMemcpyAsync(h->hctl, h->ctl.p, sizeof(Control), hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipEventRecord(h->ev_ctl, s));
    }
    launch_scatter(s, m, h->num_cls.as<uint8_t>(), merging(h), ctl->num_hist, h->cursor.as<int32_t>(),
                   h->perm_num.as<int32_t>(), h->arp, c_row_ptr, h->desc_num.as<int4>());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "symbolic launch");
    return SPG_OK;
}

spg_status sym_finish(spg_handle h, int32_t* c_row_ptr) {
    const Control& hc = h->geom;
    const Control hc2 = *h->hctl;
    if (hc2.err & ERR_NNZ_OVERFLOW)
        return fail(h, SPG_ERR_OVERFLOW, "nnz(C) = " + std::to_string(hc2.nnz_c) + " exceeds the int32 range");
    if (hc2.err & ERR_TABLE_OVERFLOW) return fail(h, SPG_ERR_HIP, "internal error: bounded symbolic table overflowed");
    h->nnz_c = hc2.nnz_c;
    uint8_t num_remap[NCLS];
    merge_classes(hc2.num_hist, num_remap, h->num_hist, merging(h) != 0);
    int32_t sym_hist[NCLS];
    uint8_t sym_remap[NCLS];
    merge_classes(hc.sym_hist, sym_remap, sym_hist, merging(h) != 0);
    int run = 0;
    for (int c = 0; c < NCLS; ++c) {
        h->num_off[c] = run;
        run += h->num_hist[c];
    }
    // global-path slabs for the numeric phase are sized now, not inside numeric
    const int gcls = MODE_DIRECT * NTIER + TIER_GLOBAL;
    const int grid_cap = 2 * h->n_cu;
    h->slab_num_words = 0;
    h->nslab_num = std::min(std::max(h->num_hist[gcls], 0), grid_cap);
    if (!h->method && h->num_hist[gcls] > 0 && hc2.max_words_num_global * 8 > wide_lds(h)) {
        h->slab_num_words = 2 * ((hc2.max_words_num_global + 63) & ~(int64_t)63);
        SPG_TRY(ensure(h, h->slab_num, (size_t)h->nslab_num * h->slab_num_words * 4));
    }
    // tiled global path: tile offsets of B and the (row, tile) items, built
    // by the first numeric call on this symbolic result
    h->tiled = false;
    h->tiled_built = false;
    if (h->tiled_global && !h->method && h->num_hist[gcls] > 0) {
        const int64_t w = tile_cols(h->dt == SPG_F64 ? 8 : 4);
        const int64_t T = (h->k + w - 1) / w;
        if (T >= 1 && T <= TILE_MAX) {
            const int64_t R = h->num_hist[gcls];
            SPG_TRY(ensure(h, h->toff, (size_t)h->n * (T + 1) * 4));
            SPG_TRY(ensure(h, h->titems, (size_t)(T * R) * sizeof(int4)));
            SPG_TRY(ensure(h, h->tfb, (size_t)R * 3 * 4));  // fallback rows, heavy and light slots
            h->tiled = true;
            h->ntiles = (int)T;
        }
    }
    spg_stats& st = h->stats;
    st.size = sizeof(spg_stats);
    st.m = h->m, st.n = h->n, st.k = h->k;
    st.products = hc2.products;
    st.nnz_c = hc2.nnz_c;
    // statistics per launch class
    for (int c = 0; c < NCLS; ++c) {
        st.sym_rows[c] = sym_hist[c];
        st.num_rows[c] = h->num_hist[c];
        st.num_a_nnz[c] = st.num_c_nnz[c] = st.num_products[c] = 0;
    }
    for (int c = 0; c < NCLS; ++c) {
        st.num_a_nnz[num_remap[c]] += hc2.num_a_nnz[c];
        st.num_c_nnz[num_remap[c]] += hc2.num_c_nnz[c];
        st.num_products[num_remap[c]] += hc2.num_products[c];
    }
    st.empty_rows = hc2.empty_rows;
    st.retried_rows = hc2.overflow_rows;
    st.mispredicted_rows = hc2.mispredicted;
    st.binning = h->binning;
    st.list_pairs = std::min(hc.list_total, h->list_cap);
    h->crp = c_row_ptr;
    h->have_sym = true;
    h->have_feats = h->binning == 1 || h->keep_features;
    h->blocks_valid = h->method == 0;  // the paper's design also counts them, but per its own hash maps
    return SPG_OK;
}

int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t)1 << (l + 1) <= v) ++l;
    return l;
}

// The numeric global class on the tiled path: tile offsets and items when
// this symbolic result has none yet (always when `build`), the (row, tile)
// items, then the rows left to the segment path.
void num_launch_tiled(spg_handle h, const NumArgs& g, bool build) {
    hipStream_t s = h->stream;
    const int eb = h->dt == SPG_F64 ? 8 : 4;
    Control* ctl = h->ctl.as<Control>();
    TileArgs t{};
    t.n = h->n;
    t.rows = g.count;
    t.ntiles = h->ntiles;
    t.log_cols = ilog2(tile_cols(eb));
    t.perm = g.perm;
    t.arp = h->arp, t.aci = h->aci, t.av = g.av;
    t.brp = h->brp, t.bci = h->bci, t.bv = g.bv, t.bnnz = h->bnnz;
    t.crp = h->crp;
    t.lofs = h->lofs.as<int32_t>();
    t.row_blocks = h->row_blocks.as<int32_t>();
    t.lists = h->lists.as<int2>();
    t.toff = h->toff.as<int32_t>();
    t.items = h->titems.as<int4>();
    t.fallback = h->tfb.as<int32_t>();
    t.heavy = t.fallback + g.count;
    t.light = t.heavy + g.count;
    t.ctl = ctl;
    t.ccol = g.ccol;
    t.cval = g.cval;
    t.dinv = g.dinv;
    t.omega = g.omega;
    if (build || !h->tiled_built) {
        launch_fill_u8(s, &ctl->tile_fallback, 0, 4 * sizeof(int32_t));
        launch_tile_build(s, t);
        h->tiled_built = true;
    }
    launch_num_tiled(s, t, eb, h->n_cu);
    NumArgs f = g;
    f.perm = h->tfb.as<int32_t>();
    f.count = 0;
    f.count_dev = &ctl->tile_fallback;
    launch_num_class(s, f, eb, std::max(h->nslab_num, 1));
}

// Numeric launches for the current symbolic result (no synchronisation).
// `build_tiles` rebuilds the tiled path's items even if they exist (a
// captured graph must hold the build).
spg_status num_launch_all(spg_handle h, const void* a_vals, const void* b_vals, int32_t* c_col_idx, void* c_vals,
                          bool build_tiles = false, const void* dinv = nullptr, double omega = 0.0) {
    hipStream_t s = h->stream;
    const int eb = h->dt == SPG_F64 ? 8 : 4;
    if (h->method) {
        if (dinv) return fail(h, SPG_ERR_UNSUPPORTED, "the Jacobi-fused product runs on the per-row classes only");
        PaperLaunch p{};
        p.m = h->m, p.team = h->paper_team, p.grid = h->paper_grid;
        p.arp = h->arp, p.aci = h->aci, p.av = a_vals, p.brp = h->brp, p.bci = h->bci, p.bv = b_vals;
        p.rinfo = h->rinfo.as<RowInfo>(), p.crp = h->crp, p.ccol = c_col_idx, p.cval = c_vals;
        p.slab = h->slab_paper.as<int32_t>(), p.slab_slots = h->paper_num_slots;
        const int set = h->num_set;
        if (h->timing) {
            resolve_num(h, set, 0);
            (void)hipEventRecord(h->ev[num_ev(set, 0)], s);
        }
        launch_paper(s, p, true, eb, h->n_cu);
        if (h->timing) {
            (void)hipEventRecord(h->ev[num_ev(set, 0) + 1], s);
            h->num_cls_timed[0] = true;
            h->num_pending[set][0] = true;
            h->num_last_set = h->num_set, h->num_set ^= 1;
        }
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? SPG_OK : hip_fail(h, e, "numeric launch");
    }
    for (int c = 0; c < NCLS; ++c) {
        if (!h->num_hist[c]) continue;
        NumArgs a{};
        a.perm = h->perm_num.as<int32_t>() + h->num_off[c];
        a.desc = h->desc_num.as<int4>() + h->num_off[c];
        a.count = h->num_hist[c];
        a.tier = c % NTIER;
        a.mode = c / NTIER;
        a.arp = h->arp, a.aci = h->aci, a.av = a_vals;
        a.brp = h->brp, a.bci = h->bci, a.bv = b_vals;
        a.bc = h->bc.as<int2>(), a.bhdr = h->bhdr.as<int4>();
        a.bc_total = h->bc_runs;
        a.bnnz = h->bnnz;
        a.crp = h->crp;
        a.rinfo = h->rinfo.as<RowInfo>();
        a.row_blocks = h->row_blocks.as<int32_t>();
        a.ccol = c_col_idx;
        a.cval = c_vals;
        a.slab = h->slab_num_words ? h->slab_num.as<uint32_t>() : nullptr;
        a.slab_words = h->slab_num_words;
        a.wide_lds = wide_lds(h);
        a.wide_vals = wide_vals(h, eb);
        a.lofs = h->lofs.as<int32_t>();
        a.lists = h->lists.as<int2>();
        a.dinv = dinv;
        a.omega = omega;
        const int set = h->num_set;
        if (h->timing) {
            resolve_num(h, set, c);
            (void)hipEventRecord(h->ev[num_ev(set, c)], s);
        }
        if (c == MODE_DIRECT * NTIER + TIER_GLOBAL && h->tiled) num_launch_tiled(h, a, build_tiles);
        else launch_num_class(s, a, eb, std::max(h->nslab_num, 1));
        if (h->timing) (void)hipEventRecord(h->ev[num_ev(set, c) + 1], s);
        h->num_cls_timed[c] = h->timing != 0;
        h->num_pending[set][c] = h->timing != 0;
    }
    if (h->timing) h->num_last_set = h->num_set, h->num_set ^= 1;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "numeric launch");
    return SPG_OK;
}

}  // namespace

extern "C" {

const char* spg_status_string(spg_status s) {
    switch (s) {
        case SPG_OK: return "SPG_OK";
        case SPG_ERR_ARG: return "SPG_ERR_ARG";
        case SPG_ERR_SHAPE: return "SPG_ERR_SHAPE";
        case SPG_ERR_STATE: return "SPG_ERR_STATE";
        case SPG_ERR_INDEX: return "SPG_ERR_INDEX";
        case SPG_ERR_OVERFLOW: return "SPG_ERR_OVERFLOW";
        case SPG_ERR_ALLOC: return "SPG_ERR_ALLOC";
        case SPG_ERR_HIP: return "SPG_ERR_HIP";
        case SPG_ERR_UNSUPPORTED: return "SPG_ERR_UNSUPPORTED";
    }
    return "SPG_ERR_UNKNOWN";
}

const char* spg_last_error(spg_handle h) { return h ? h->err.c_str() : "null handle"; }

spg_status spg_create(spg_handle* out, void* stream) {
    if (!out) return SPG_ERR_ARG;
    *out = nullptr;
    try {
        spg_handle h = new spg_handle_s();
        h->stream = static_cast<hipStream_t>(stream);
        hipError_t e = hipGetDevice(&h->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&h->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
        if (e == hipSuccess) {
            h->hctl = pinned_take();
            if (!h->hctl) e = hipErrorOutOfMemory;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return SPG_ERR_HIP;
        }
        h->lds_limit = clamp_lds_limit(h, h->lds_limit);
        *out = h;
        return SPG_OK;
    } catch (...) {
        return SPG_ERR_ALLOC;
    }
}

spg_status spg_destroy(spg_handle h) {
    if (!h) return SPG_OK;
    (void)hipStreamSynchronize(h->stream);  // no launch of this handle still reads its buffers
    DevBuf* bufs[] = {&h->binfo, &h->rinfo, &h->feats, &h->sym_cls, &h->num_cls, &h->perm_sym, &h->perm_num,
                      &h->desc_sym, &h->desc_num,
                      &h->row_nnz, &h->row_blocks, &h->tile_status, &h->cursor, &h->ovf_list, &h->ctl,
                      &h->slab_sym, &h->slab_retry, &h->slab_num, &h->mlp_w, &h->bc, &h->bhdr,
                      &h->lofs, &h->lists, &h->toff, &h->titems, &h->tfb, &h->slab_paper};
    for (DevBuf* b : bufs) cache_put(h->device, *b);  // idle: the stream has finished
    pinned_put(h->hctl);
    if (h->ev_made)
        for (auto& e : h->ev) (void)hipEventDestroy(e);
    if (h->ev_ctl) (void)hipEventDestroy(h->ev_ctl);
    delete h;
    return SPG_OK;
}

spg_status spg_set_stream(spg_handle h, void* stream) {
    if (!h) return SPG_ERR_ARG;
    // the handle's buffers are allocated in the old stream's order: let it finish
    if (hipStreamSynchronize(h->stream) != hipSuccess) return hip_fail(h, hipGetLastError(), "hipStreamSynchronize");
    h->stream = static_cast<hipStream_t>(stream);
    return SPG_OK;
}

spg_status spg_set_matrices(spg_handle h, spg_dtype dt, int32_t m, int32_t n, int32_t k, const int32_t* a_row_ptr,
                            const int32_t* a_col_idx, int64_t a_nnz, const int32_t* b_row_ptr,
                            const int32_t* b_col_idx, int64_t b_nnz) {
    if (!h) return SPG_ERR_ARG;
    try {
        h->have_mats = false;
        h->have_sym = false;
        h->blocks_valid = false;
        if (dt != SPG_F32 && dt != SPG_F64) return fail(h, SPG_ERR_ARG, "dtype must be SPG_F32 or SPG_F64");
        if (m < 0 || n < 0 || k < 0 || a_nnz < 0 || b_nnz < 0)
            return fail(h, SPG_ERR_ARG, "negative dimension or nnz");
        if (a_nnz > INT32_MAX || b_nnz > INT32_MAX) return fail(h, SPG_ERR_ARG, "nnz exceeds int32 range");
        if (!a_row_ptr || !b_row_ptr) return fail(h, SPG_ERR_ARG, "null row pointer");
        if ((a_nnz > 0 && !a_col_idx) || (b_nnz > 0 && !b_col_idx)) return fail(h, SPG_ERR_ARG, "null column index");
        if (n == 0 && a_nnz > 0) return fail(h, SPG_ERR_SHAPE, "A has entries but no columns");
        if (k == 0 && b_nnz > 0) return fail(h, SPG_ERR_SHAPE, "B has entries but no columns");
        h->dt = dt;
        h->m = m, h->n = n, h->k = k;
        h->arp = a_row_ptr, h->aci = a_col_idx, h->annz = a_nnz;
        h->brp = b_row_ptr, h->bci = b_col_idx, h->bnnz = b_nnz;
        h->have_mats = true;
        return SPG_OK;
    } catch (...) {
        return fail(h, SPG_ERR_ALLOC, "host exception");
    }
}

spg_status spg_symbolic(spg_handle h, int32_t* c_row_ptr, int64_t* nnz_c) {
    if (!h) return SPG_ERR_ARG;
    try {
        if (!h->have_mats) return fail(h, SPG_ERR_STATE, "spg_set_matrices must come first");
        if (!c_row_ptr || !nnz_c) return fail(h, SPG_ERR_ARG, "null output");
        if (h->binning == 1 && !h->have_mlp) return fail(h, SPG_ERR_STATE, "learned binning needs spg_set_mlp");
        if (h->binning == 3 && !h->blocks_valid)
            return fail(h, SPG_ERR_STATE, "the exact-count estimate needs a previous symbolic result of these matrices");
        h->have_sym = false;
        if (h->timing) SPG_TRY(make_events(h));
        h->sym_timed = h->timing == 1;
        std::fill(std::begin(h->sym_cls_timed), std::end(h->sym_cls_timed), false);
        SPG_TRY(sym_prepare(h));
        rec(h, EV_SYM0);
        sym_stage_analysis(h);
        if (h->m == 0) {
            launch_fill_i32(h->stream, c_row_ptr, 0, 1);
            SPG_TRY(sync_ctl(h));
            h->sym_waits = 1;
            rec(h, EV_SYM1);
            *nnz_c = 0;
            h->nnz_c = 0;
            h->crp = c_row_ptr;
            std::fill(std::begin(h->num_hist), std::end(h->num_hist), 0);
            h->nslab_num = 0;
            h->slab_num_words = 0;
            h->have_sym = true;
            h->have_feats = false;
            return SPG_OK;
        }
        h->sym_waits = 1;
        if (!h->single_wait) {
            // sizes from the analysis (a second wait; see reserve_symbolic)
            h->sym_waits = 2;
            SPG_TRY(sync_ctl(h));
            SPG_TRY(check_input_errors(h));
            h->geom = *h->hctl;
            if (!h->method) SPG_TRY(size_from_analysis(h));
        }
        SPG_TRY(sym_stage_rows(h, c_row_ptr, true));
        rec(h, EV_SYM1);
        // the one wait: the control block copied right after the row-pointer
        // scan gives nnz(C), input errors and the numeric launch geometry
        // (the numeric grouping may still run; numeric is ordered after it)
        HIP_TRY(h, hipEventSynchronize(h->ev_ctl));
        h->geom = *h->hctl;
        SPG_TRY(check_input_errors(h));
        SPG_TRY(sym_finish(h, c_row_ptr));
        *nnz_c = h->nnz_c;
        return SPG_OK;
    } catch (const std::bad_alloc&) {
        return fail(h, SPG_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(h, SPG_ERR_HIP, "unexpected host exception");
    }
}

spg_status spg_numeric(spg_handle h, const void* a_vals, const void* b_vals, int32_t* c_col_idx, void* c_vals) {
    if (!h) return SPG_ERR_ARG;
    try {
        if (!h->have_sym) return fail(h, SPG_ERR_STATE, "spg_symbolic must come first");
        if ((h->annz > 0 && !a_vals) || (h->bnnz > 0 && !b_vals)) return fail(h, SPG_ERR_ARG, "null input values");
        if (h->nnz_c > 0 && (!c_col_idx || !c_vals)) return fail(h, SPG_ERR_ARG, "null output");
        if (h->timing) SPG_TRY(make_events(h));
        h->num_timed = h->timing != 0;
        std::fill(std::begin(h->num_cls_timed), std::end(h->num_cls_timed), false);
        rec(h, EV_NUM0);
        SPG_TRY(num_launch_all(h, a_vals, b_vals, c_col_idx, c_vals));
        rec(h, EV_NUM1);
        return SPG_OK;
    } catch (...) {
        return fail(h, SPG_ERR_HIP, "unexpected host exception");
    }
}

spg_status spg_numeric_jacobi(spg_handle h, double omega, const void* dinv, const void* a_vals, const void* b_vals,
                              int32_t* c_col_idx, void* c_vals) {
    if (!h) return SPG_ERR_ARG;
    try {
        if (!h->have_sym) return fail(h, SPG_ERR_STATE, "spg_symbolic must come first");
        if (h->m != h->n) return fail(h, SPG_ERR_SHAPE, "the Jacobi-fused product needs a square A");
        if (h->geom.a_missing_diag > 0)
            return fail(h, SPG_ERR_SHAPE, std::to_string(h->geom.a_missing_diag) +
                                              " rows of A store no diagonal entry: C would leave the pattern of A*B");
        if (h->m > 0 && !dinv) return fail(h, SPG_ERR_ARG, "null D^-1");
        if ((h->annz > 0 && !a_vals) || (h->bnnz > 0 && !b_vals)) return fail(h, SPG_ERR_ARG, "null input values");
        if (h->nnz_c > 0 && (!c_col_idx || !c_vals)) return fail(h, SPG_ERR_ARG, "null output");
        if (h->timing) SPG_TRY(make_events(h));
        h->num_timed = h->timing != 0;
        std::fill(std::begin(h->num_cls_timed), std::end(h->num_cls_timed), false);
        rec(h, EV_NUM0);
        SPG_TRY(num_launch_all(h, a_vals, b_vals, c_col_idx, c_vals, false, dinv, omega));
        rec(h, EV_NUM1);
        return SPG_OK;
    } catch (...) {
        return fail(h, SPG_ERR_HIP, "unexpected host exception");
    }
}

spg_status spg_set_option(spg_handle h, int32_t opt, int64_t val) {
    if (!h) return SPG_ERR_ARG;
    switch (opt) {
        case SPG_OPT_BINNING:
            if (val < 0 || val > 3) return fail(h, SPG_ERR_ARG, "binning must be 0..3");
            h->binning = (int)val;
            break;
        case SPG_OPT_TIMING:
            if (val < 0 || val > 2) return fail(h, SPG_ERR_ARG, "timing must be 0, 1 or 2");
            h->timing = (int)val;
            reset_num_sums(h);
            break;
        case SPG_OPT_FORCE_CLASS:
            if (val < -1 || val >= NCLS) return fail(h, SPG_ERR_ARG, "class out of range");
            h->force_class = (int)val;
            break;
        case SPG_OPT_WORK_PER_LANE:
            if (val < 1 || val > 1 << 20) return fail(h, SPG_ERR_ARG, "work per lane out of range");
            h->work_per_lane = (int)val;
            break;
        case SPG_OPT_MLP_MARGIN_MILLI:
            if (val < -20000 || val > 20000) return fail(h, SPG_ERR_ARG, "margin out of range");
            h->mlp_margin_milli = (int)val;
            break;
        case SPG_OPT_HASH_MAX_BLOCKS:
            if (val < 0 || val > 4096) return fail(h, SPG_ERR_ARG, "hash block limit out of range");
            h->hash_max_blocks = (int)val;
            break;
        case SPG_OPT_LDS_LIMIT: {
            if (val < 1024 || val > 65536 || (val & (val - 1)))
                return fail(h, SPG_ERR_ARG, "LDS limit must be a power of two in [1024, 65536]");
            h->lds_limit = clamp_lds_limit(h, (int)val);
            break;
        }
        case SPG_OPT_KEEP_FEATURES: h->keep_features = val != 0; break;
        case SPG_OPT_MERGE_CLASSES: h->merge_classes = val != 0; break;
        case SPG_OPT_TILED_GLOBAL: h->tiled_global = val != 0; break;
        case SPG_OPT_METHOD:
            if (val < 0 || val > 3) return fail(h, SPG_ERR_ARG, "method must be 0..3");
            h->method = (int)val;
            break;
        case SPG_OPT_LIST_LIMIT_MB:
            if (val < 1 || val > 16383) return fail(h, SPG_ERR_ARG, "list memory limit must be 1..16383 MiB");
            h->list_limit_mb = val;
            break;
        default: return fail(h, SPG_ERR_ARG, "unknown option " + std::to_string(opt));
    }
    // options change how rows are binned: the symbolic result must be redone
    if (opt != SPG_OPT_TIMING) h->have_sym = false;
    return SPG_OK;
}

spg_status spg_set_mlp(spg_handle h, const float* w, int32_t nw) {
    if (!h) return SPG_ERR_ARG;
    if (!w || nw != 1217) return fail(h, SPG_ERR_ARG, "the predictor has exactly 1217 weights");
    SPG_TRY(ensure(h, h->mlp_w, 1217 * sizeof(float)));
    HIP_TRY(h, hipMemcpyAsync(h->mlp_w.p, w, 1217 * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->have_mlp = true;
    h->have_sym = false;
    return SPG_OK;
}

spg_status spg_get_stats(spg_handle h, spg_stats* out, int32_t size) {
    if (!h || !out) return SPG_ERR_ARG;
    if (size != (int32_t)sizeof(spg_stats)) return fail(h, SPG_ERR_ARG, "spg_stats size mismatch");
    spg_stats& st = h->stats;
    st.size = sizeof(spg_stats);
    if (h->ev_made) {
        if (h->sym_timed) {
            st.sym_ms = elapsed(h, EV_SYM0, EV_SYM1);
            st.analysis_ms = elapsed(h, EV_SYM0, EV_ANA1);
            st.scan_ms = elapsed(h, EV_SCAN0, EV_SCAN1);
            st.mlp_ms = st.binning == 1 ? elapsed(h, EV_MLP0, EV_MLP1) : 0.f;
            for (int c = 0; c < NCLS; ++c)
                st.sym_class_ms[c] = h->sym_cls_timed[c] ? elapsed(h, EV_SYMCLS + 2 * c, EV_SYMCLS + 2 * c + 1) : 0.f;
        }
        if (h->num_timed) {
            st.num_ms = h->timing == 1 ? elapsed(h, EV_NUM0, EV_NUM1) : 0.f;
            for (int c = 0; c < NCLS; ++c)
                st.num_class_ms[c] =
                    h->num_cls_timed[c] ? elapsed(h, num_ev(h->num_last_set, c), num_ev(h->num_last_set, c) + 1) : 0.f;
        }
        for (int set = 0; set < 2; ++set)
            for (int c = 0; c < NCLS; ++c) resolve_num(h, set, c);
    }
    for (int c = 0; c < NCLS; ++c) {
        st.num_class_ms_total[c] = (float)h->num_acc_ms[c];
        st.num_class_launches[c] = h->num_acc_n[c];
    }
    st.sym_waits = h->sym_waits;
    st.num_tiles = h->have_sym && h->tiled ? h->ntiles : 0;
    st.tile_fallback_rows = 0;
    if (st.num_tiles && h->tiled_built) {
        // written by the last numeric call's item build, on the handle's stream
        int32_t fb = 0;
        HIP_TRY(h, hipMemcpyAsync(&fb, &h->ctl.as<Control>()->tile_fallback, sizeof(fb), hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        st.tile_fallback_rows = fb;
    }
    *out = st;
    return SPG_OK;
}

spg_status spg_export_rows(spg_handle h, float* x, float* y, int32_t* row_nnz) {
    if (!h) return SPG_ERR_ARG;
    if (!h->have_sym || !h->have_feats)
        return fail(h, SPG_ERR_STATE, "needs a symbolic result computed with features (learned binning or keep-features)");
    if (h->m > 0 && (!x || !y)) return fail(h, SPG_ERR_ARG, "null output");
    launch_export_rows(h->stream, h->m, h->feats.as<float>(), h->row_blocks.as<int32_t>(), h->row_nnz.as<int32_t>(),
                       x, y, row_nnz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "export launch");
    return SPG_OK;
}

// ============================================================== batches
// Many independent products C_i = A_i * B_i run as one block-diagonal
// product (rows never mix across products), so every product's rows share
// the same class launches.  The launch sequence of a whole product
// (analysis, accumulators, scan, numeric) is captured once into a hipGraph
// with the geometry of a first synchronised run, and every later run is one
// hipGraphLaunch: no host round trip, no allocation.
}  // extern "C"

struct spg_batch_s {
    spg_handle h = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t count = 0;
    spg_dtype dt = SPG_F64;
    int64_t m_total = 0, n_total = 0, annz_total = 0, bnnz_total = 0;
    int32_t k_max = 0;
    std::vector<int64_t> row_off, c_nnz_off;
    DevBuf arp, aci, brp, desc, err, crp_plan;
    const int32_t* bci_pool = nullptr;
    bool planned = false;
    int64_t nnz_total = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* g_av = nullptr;
    const void* g_bv = nullptr;
    int32_t* g_crp = nullptr;
    int32_t* g_ccol = nullptr;
    void* g_cval = nullptr;
    int g_numeric_only = -1;
    std::string err_msg;
    // queued path: per-product tables (built once), the work queue, and its captured graph
    bool q_ready = false;
    int q_wmax = 0, q_vmax = 0, q_grid = 0;
    int64_t q_items = 0;
    DevBuf q_item_off, q_row_off, q_crp_off, q_ctl, q_left, q_queue, q_bm;
    hipGraph_t q_graph = nullptr;
    hipGraphExec_t q_exec = nullptr;
    const void* qg_key[7] = {};
    int64_t qg_cap = -1;
};

namespace {

spg_status bfail(spg_batch b, spg_status s, const std::string& msg) {
    if (b) b->err_msg = msg;
    return s;
}

void drop_graph(spg_batch b) {
    if (b->exec) (void)hipStreamSynchronize(b->stream);  // no replay still running
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_numeric_only = -1;
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

void drop_queue_graph(spg_batch b) {
    if (b->q_exec) (void)hipStreamSynchronize(b->stream);
    if (b->q_exec) (void)hipGraphExecDestroy(b->q_exec);
    if (b->q_graph) (void)hipGraphDestroy(b->q_graph);
    b->q_exec = nullptr;
    b->q_graph = nullptr;
}

constexpr int QUEUE_ROWS_PER_ITEM = 128;

// Once per batch: the row facts of the packed product (one synchronised
// analysis), the widest row's range (which sizes the kernel's LDS windows, or
// rules the queued path out), and the per-product item, row and row-pointer
// offsets.
spg_status queue_prepare(spg_batch b) {
    if (b->q_ready) return SPG_OK;
    spg_handle h = b->h;
    SPG_TRY(sym_prepare(h));
    sym_stage_analysis(h);
    SPG_TRY(sync_ctl(h));
    SPG_TRY(check_input_errors(h));
    const Control c = *h->hctl;
    if (c.max_words_all > QUEUE_MAX_WORDS)
        return bfail(b, SPG_ERR_UNSUPPORTED,
                     "a row of C spans " + std::to_string(c.max_words_all * 32) +
                         " columns; the queued kernel holds rows of up to " + std::to_string(QUEUE_MAX_WORDS * 32) +
                         " (use spg_batch_run)");
    // compressed B for the symbolic items: built by the analysis above
    b->q_wmax = (int)std::max<int64_t>(c.max_words_all, 1);
    b->q_vmax = 32 * b->q_wmax;
    const int32_t cnt = b->count;
    std::vector<int64_t> item_off((size_t)cnt + 1, 0), crp_off((size_t)std::max(cnt, 1), 0);
    int64_t crp = 0;
    for (int32_t p = 0; p < cnt; ++p) {
        const int64_t m = b->row_off[p + 1] - b->row_off[p];
        item_off[p + 1] = item_off[p] + (m + QUEUE_ROWS_PER_ITEM - 1) / QUEUE_ROWS_PER_ITEM;
        crp_off[p] = crp;
        crp += m + 1;
    }
    b->q_items = item_off[cnt];
    SPG_TRY(ensure(h, b->q_item_off, ((size_t)cnt + 1) * 8));
    SPG_TRY(ensure(h, b->q_row_off, ((size_t)cnt + 1) * 8));
    SPG_TRY(ensure(h, b->q_crp_off, (size_t)std::max(cnt, 1) * 8));
    SPG_TRY(ensure(h, b->q_ctl, sizeof(QueueCtl)));
    SPG_TRY(ensure(h, b->q_left, (size_t)std::max(cnt, 1) * 4));
    SPG_TRY(ensure(h, b->q_queue, (size_t)std::max<int64_t>(b->q_items, 1) * 8));
    // the rows' bitmaps from symbolic to numeric, when they take at most 4 GiB
    const int64_t bm_bytes = b->m_total * b->q_wmax * 4;
    if (bm_bytes <= (int64_t)4 << 30) SPG_TRY(ensure(h, b->q_bm, (size_t)std::max<int64_t>(bm_bytes, 4)));
    HIP_TRY(h, hipMemcpyAsync(b->q_item_off.p, item_off.data(), item_off.size() * 8, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(h, hipMemcpyAsync(b->q_row_off.p, b->row_off.data(), ((size_t)cnt + 1) * 8, hipMemcpyHostToDevice,
                              b->stream));
    HIP_TRY(h, hipMemcpyAsync(b->q_crp_off.p, crp_off.data(), crp_off.size() * 8, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(h, hipStreamSynchronize(b->stream));
    // as many workgroups as the compute units' LDS holds at once (at most 8 each)
    const size_t lds = queue_lds_bytes(b->q_wmax, b->q_vmax, b->dt == SPG_F64 ? 8 : 4);
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (size_t)h->max_lds / std::max<size_t>(lds, 1)));
    b->q_grid = h->n_cu * per_cu;
    b->q_ready = true;
    return SPG_OK;
}

// one synchronised symbolic run on the packed product: geometry, nnz, offsets
spg_status batch_replan(spg_batch b) {
    drop_graph(b);
    spg_handle h = b->h;
    int64_t nnz = 0;
    spg_status st = spg_symbolic(h, b->crp_plan.as<int32_t>(), &nnz);
    if (st != SPG_OK) return bfail(b, st, h->err);
    std::vector<int32_t> rp((size_t)b->m_total + 1);
    HIP_TRY(h, hipMemcpyAsync(rp.data(), b->crp_plan.p, rp.size() * 4, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(h, hipStreamSynchronize(b->stream));
    b->c_nnz_off.assign((size_t)b->count + 1, 0);
    for (int32_t p = 0; p <= b->count; ++p) b->c_nnz_off[p] = rp[(size_t)b->row_off[p]];
    b->nnz_total = nnz;
    b->planned = true;
    return SPG_OK;
}

}  // namespace

extern "C" {

spg_status spg_batch_create(spg_batch* out, void* stream, spg_dtype dt, int32_t count, const int32_t* m,
                            const int32_t* n, const int32_t* k, const int64_t* a_nnz, const int64_t* b_nnz,
                            const int32_t* a_row_ptr_pool, const int32_t* a_col_pool, const int32_t* b_row_ptr_pool,
                            const int32_t* b_col_pool) {
    if (!out) return SPG_ERR_ARG;
    *out = nullptr;
    if (count < 0 || (count > 0 && (!m || !n || !k || !a_nnz || !b_nnz || !a_row_ptr_pool || !b_row_ptr_pool)))
        return SPG_ERR_ARG;
    if (dt != SPG_F32 && dt != SPG_F64) return SPG_ERR_ARG;
    spg_batch b = nullptr;
    try {
        b = new spg_batch_s();
        b->count = count;
        b->dt = dt;
        b->row_off.assign((size_t)count + 1, 0);
        std::vector<int64_t> da(7 * (size_t)std::max(count, 1)), db(7 * (size_t)std::max(count, 1));
        int64_t rpa = 0, rpb = 0, na = 0, nb = 0, mrow = 0, nrow = 0;
        for (int32_t p = 0; p < count; ++p) {
            if (m[p] < 0 || n[p] < 0 || k[p] < 0 || a_nnz[p] < 0 || b_nnz[p] < 0) {
                delete b;
                return SPG_ERR_ARG;
            }
            int64_t* a = &da[7 * (size_t)p];
            a[0] = mrow, a[1] = rpa, a[2] = na, a[3] = m[p], a[4] = a_nnz[p], a[5] = nrow, a[6] = n[p];
            int64_t* c = &db[7 * (size_t)p];
            c[0] = nrow, c[1] = rpb, c[2] = nb, c[3] = n[p], c[4] = b_nnz[p], c[5] = 0, c[6] = k[p];
            b->row_off[p] = mrow;
            mrow += m[p], nrow += n[p], rpa += m[p] + 1, rpb += n[p] + 1, na += a_nnz[p], nb += b_nnz[p];
            b->k_max = std::max(b->k_max, k[p]);
        }
        b->row_off[count] = mrow;
        if (mrow >= INT32_MAX || nrow >= INT32_MAX || na >= INT32_MAX || nb >= INT32_MAX) {
            delete b;
            return SPG_ERR_OVERFLOW;
        }
        if ((na > 0 && !a_col_pool) || (nb > 0 && !b_col_pool)) {
            delete b;
            return SPG_ERR_ARG;
        }
        b->m_total = mrow, b->n_total = nrow, b->annz_total = na, b->bnnz_total = nb;
        b->bci_pool = b_col_pool;
        if (stream) {
            b->stream = static_cast<hipStream_t>(stream);
        } else {
            if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
                delete b;
                return SPG_ERR_HIP;
            }
            b->own_stream = true;
        }
        spg_status st = spg_create(&b->h, b->stream);
        if (st != SPG_OK) {
            spg_batch_destroy(b);
            return st;
        }
        spg_handle h = b->h;
        SPG_TRY(ensure(h, b->arp, (size_t)(mrow + 1) * 4));
        SPG_TRY(ensure(h, b->aci, (size_t)std::max<int64_t>(na, 1) * 4));
        SPG_TRY(ensure(h, b->brp, (size_t)(nrow + 1) * 4));
        SPG_TRY(ensure(h, b->desc, 2 * da.size() * 8));
        SPG_TRY(ensure(h, b->err, 16));
        SPG_TRY(ensure(h, b->crp_plan, (size_t)(mrow + 1) * 4));
        int64_t* ddesc = b->desc.as<int64_t>();
        HIP_TRY(h, hipMemcpyAsync(ddesc, da.data(), da.size() * 8, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(h, hipMemcpyAsync(ddesc + da.size(), db.data(), db.size() * 8, hipMemcpyHostToDevice, b->stream));
        launch_fill_i32(b->stream, b->err.as<int32_t>(), 0, 1);
        launch_pack(b->stream, count, ddesc, a_row_ptr_pool, a_col_pool, b->arp.as<int32_t>(), b->aci.as<int32_t>(),
                    b->err.as<int32_t>());
        launch_pack(b->stream, count, ddesc + da.size(), b_row_ptr_pool, b_col_pool, b->brp.as<int32_t>(), nullptr,
                    b->err.as<int32_t>());
        launch_fill_i32(b->stream, b->arp.as<int32_t>() + mrow, (int32_t)na, 1);
        launch_fill_i32(b->stream, b->brp.as<int32_t>() + nrow, (int32_t)nb, 1);
        int32_t herr = 0;
        HIP_TRY(h, hipMemcpyAsync(&herr, b->err.p, 4, hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(h, hipStreamSynchronize(b->stream));
        if (herr) {
            spg_batch_destroy(b);
            return SPG_ERR_INDEX;
        }
        st = spg_set_matrices(h, dt, (int32_t)mrow, (int32_t)nrow, b->k_max, b->arp.as<int32_t>(),
                              b->aci.as<int32_t>(), na, b->brp.as<int32_t>(), b_col_pool, nb);
        if (st != SPG_OK) {
            spg_batch_destroy(b);
            return st;
        }
        *out = b;
        return SPG_OK;
    } catch (...) {
        if (b) spg_batch_destroy(b);
        return SPG_ERR_ALLOC;
    }
}

spg_status spg_batch_destroy(spg_batch b) {
    if (!b) return SPG_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    drop_queue_graph(b);
    DevBuf* bufs[] = {&b->arp, &b->aci, &b->brp, &b->desc, &b->err, &b->crp_plan, &b->q_item_off, &b->q_row_off,
                      &b->q_crp_off, &b->q_ctl, &b->q_left, &b->q_queue, &b->q_bm};
    for (DevBuf* x : bufs) release(*x, b->stream);
    if (b->h) spg_destroy(b->h);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return SPG_OK;
}

const char* spg_batch_last_error(spg_batch b) {
    if (!b) return "null batch";
    return b->err_msg.empty() && b->h ? b->h->err.c_str() : b->err_msg.c_str();
}

spg_status spg_batch_set_option(spg_batch b, int32_t opt, int64_t val) {
    if (!b) return SPG_ERR_ARG;
    spg_status st = spg_set_option(b->h, opt, val);
    if (st != SPG_OK) return bfail(b, st, b->h->err);
    if (opt != SPG_OPT_TIMING) b->planned = false, drop_graph(b);
    return SPG_OK;
}

spg_status spg_batch_set_mlp(spg_batch b, const float* w, int32_t nw) {
    if (!b) return SPG_ERR_ARG;
    spg_status st = spg_set_mlp(b->h, w, nw);
    if (st != SPG_OK) return bfail(b, st, b->h->err);
    b->planned = false;
    drop_graph(b);
    return SPG_OK;
}

spg_status spg_batch_plan(spg_batch b, int64_t* nnz_total, int64_t* c_row_off, int64_t* c_nnz_off) {
    if (!b || !nnz_total) return SPG_ERR_ARG;
    try {
        SPG_TRY(batch_replan(b));
        *nnz_total = b->nnz_total;
        for (int32_t p = 0; p <= b->count; ++p) {
            if (c_row_off) c_row_off[p] = b->row_off[p];
            if (c_nnz_off) c_nnz_off[p] = b->c_nnz_off[p];
        }
        return SPG_OK;
    } catch (...) {
        return bfail(b, SPG_ERR_ALLOC, "host exception");
    }
}

spg_status spg_batch_run(spg_batch b, const void* a_val_pool, const void* b_val_pool, int32_t* c_row_ptr,
                         int32_t* c_col, void* c_val, int64_t capacity, int32_t numeric_only) {
    if (!b) return SPG_ERR_ARG;
    try {
        if (!b->planned) return bfail(b, SPG_ERR_STATE, "spg_batch_plan must come first");
        if (!c_row_ptr || (b->annz_total > 0 && !a_val_pool) || (b->bnnz_total > 0 && !b_val_pool))
            return bfail(b, SPG_ERR_ARG, "null pointer");
        if (capacity < b->nnz_total || (b->nnz_total > 0 && (!c_col || !c_val)))
            return bfail(b, SPG_ERR_ARG, "C pools smaller than the planned nnz");
        spg_handle h = b->h;
        const bool same = b->exec && b->g_av == a_val_pool && b->g_bv == b_val_pool && b->g_crp == c_row_ptr &&
                          b->g_ccol == c_col && b->g_cval == c_val && b->g_numeric_only == (numeric_only != 0);
        if (!same) {
            drop_graph(b);
            const int timing = h->timing;
            h->timing = 0;
            HIP_TRY(h, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            spg_status st = SPG_OK;
            if (!numeric_only) {
                sym_stage_analysis(h);
                st = sym_stage_rows(h, c_row_ptr, false, true);
                h->crp = c_row_ptr;
            } else {
                const int64_t n1 = b->m_total + 1;
                hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)std::min<int64_t>((n1 + 255) / 256, 4096)), dim3(256), 0,
                                   b->stream, b->crp_plan.as<int32_t>(), c_row_ptr, n1);
                h->crp = b->crp_plan.as<int32_t>();
            }
            if (st == SPG_OK) st = num_launch_all(h, a_val_pool, b_val_pool, c_col, c_val, true);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            h->timing = timing;
            if (st != SPG_OK) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(b, st, h->err);
            }
            if (e != hipSuccess) return bfail(b, SPG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return bfail(b, SPG_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            b->g_av = a_val_pool, b->g_bv = b_val_pool, b->g_crp = c_row_ptr, b->g_ccol = c_col, b->g_cval = c_val;
            b->g_numeric_only = numeric_only != 0;
        }
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return bfail(b, SPG_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
        return SPG_OK;
    } catch (...) {
        return bfail(b, SPG_ERR_HIP, "host exception");
    }
}

spg_status spg_batch_tune(spg_batch b, const void* a_val_pool, const void* b_val_pool, int32_t* c_row_ptr,
                          int32_t* c_col, void* c_val, int64_t capacity, int32_t* chosen, float* best_ms) {
    if (!b) return SPG_ERR_ARG;
    try {
        if (!b->planned) return bfail(b, SPG_ERR_STATE, "spg_batch_plan must come first");
        if (capacity < b->nnz_total) return bfail(b, SPG_ERR_ARG, "C pools smaller than the planned nnz");
        if (b->nnz_total > 0 && (!c_row_ptr || !c_col || !c_val)) return bfail(b, SPG_ERR_ARG, "null output pool");
        spg_handle h = b->h;
        // the trials rewrite the handle's structure state and may grow its
        // buffers: the captured graph and the plan are void from here on, and
        // a failure leaves the batch unplanned with its options as they were
        drop_graph(b);
        b->planned = false;
        struct Restore {
            spg_handle h;
            int w, v, hb;
            bool armed = true;
            ~Restore() {
                if (armed) h->work_per_lane = w, h->binning = v, h->hash_max_blocks = hb, h->have_sym = false;
            }
        } restore{h, h->work_per_lane, h->binning, h->hash_max_blocks};
        struct Events {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~Events() {
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
            }
        } ev;
        HIP_TRY(h, hipEventCreate(&ev.e0));
        HIP_TRY(h, hipEventCreate(&ev.e1));
        const int wpl[] = {8, 16, 32};
        const int bins[] = {2, 0};
        const int hmax[] = {32, 64, 128};
        float best = 1e30f;
        int bw = h->work_per_lane, bv = h->binning, bh = h->hash_max_blocks;
        const int learned = h->binning == 1;
        for (int w : wpl)
            for (int v : bins)
                for (int hb : hmax) {
                    if (learned && v != 2) continue;  // a learned model stays in charge of the sizing
                    h->work_per_lane = w, h->binning = learned ? 1 : v, h->hash_max_blocks = hb;
                    float t = 1e30f;
                    for (int it = 0; it < 2; ++it) {
                        int64_t nnz = 0;
                        HIP_TRY(h, hipEventRecord(ev.e0, b->stream));
                        spg_status st = spg_symbolic(h, c_row_ptr, &nnz);
                        if (st == SPG_OK) st = spg_numeric(h, a_val_pool, b_val_pool, c_col, c_val);
                        if (st != SPG_OK) return bfail(b, st, h->err);
                        HIP_TRY(h, hipEventRecord(ev.e1, b->stream));
                        HIP_TRY(h, hipEventSynchronize(ev.e1));
                        float ms = 0.f;
                        HIP_TRY(h, hipEventElapsedTime(&ms, ev.e0, ev.e1));
                        t = std::min(t, ms);
                    }
                    if (t < best) best = t, bw = w, bv = h->binning, bh = hb;
                }
        h->work_per_lane = bw, h->binning = bv, h->hash_max_blocks = bh;
        restore.armed = false;
        if (chosen) chosen[0] = bw, chosen[1] = bv, chosen[2] = bh;
        if (best_ms) *best_ms = best;
        return batch_replan(b);
    } catch (...) {
        return bfail(b, SPG_ERR_HIP, "host exception");
    }
}

spg_status spg_batch_run_queued(spg_batch b, const void* a_val_pool, const void* b_val_pool, int32_t* c_row_ptr,
                                int32_t* c_col, void* c_val, int64_t capacity, int64_t* c_offsets, int64_t* stamps) {
    if (!b) return SPG_ERR_ARG;
    try {
        if (!c_row_ptr || !c_offsets || capacity < 0 || (capacity > 0 && (!c_col || !c_val)) ||
            (b->annz_total > 0 && !a_val_pool) || (b->bnnz_total > 0 && !b_val_pool))
            return bfail(b, SPG_ERR_ARG, "null pointer or negative capacity");
        spg_handle h = b->h;
        SPG_TRY(queue_prepare(b));
        if (b->count == 0) return SPG_OK;
        const void* key[7] = {a_val_pool, b_val_pool, c_row_ptr, c_col, c_val, c_offsets, stamps};
        const bool same = b->q_exec && std::equal(std::begin(key), std::end(key), std::begin(b->qg_key)) &&
                          b->qg_cap == capacity;
        if (!same) {
            drop_queue_graph(b);
            QueueArgs a{};
            a.count = b->count;
            a.rb = QUEUE_ROWS_PER_ITEM;
            a.n_items = b->q_items;
            a.item_off = b->q_item_off.as<int64_t>();
            a.row_off = b->q_row_off.as<int64_t>();
            a.crp_off = b->q_crp_off.as<int64_t>();
            a.arp = b->arp.as<int32_t>(), a.aci = b->aci.as<int32_t>(), a.av = a_val_pool;
            a.brp = b->brp.as<int32_t>(), a.bci = b->bci_pool, a.bv = b_val_pool, a.bnnz = b->bnnz_total;
            a.rinfo = h->rinfo.as<RowInfo>();
            a.row_nnz = h->row_nnz.as<int32_t>();
            a.c_row_ptr = c_row_ptr, a.ccol = c_col, a.cval = c_val, a.cap = capacity;
            a.c_offsets = c_offsets, a.stamps = stamps;
            a.qc = b->q_ctl.as<QueueCtl>();
            a.sym_left = b->q_left.as<int32_t>();
            a.queue = b->q_queue.as<int64_t>();
            a.wmax = b->q_wmax, a.vmax = b->q_vmax;
            a.qbm = b->q_bm.p ? b->q_bm.as<uint32_t>() : nullptr;
            a.bc = h->bc.as<int2>(), a.bhdr = h->bhdr.as<int4>();
            HIP_TRY(h, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            launch_queue(b->stream, a, b->dt == SPG_F64 ? 8 : 4, b->q_grid);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess) return bfail(b, SPG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            b->q_graph = g;
            e = hipGraphInstantiate(&b->q_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_queue_graph(b);
                return bfail(b, SPG_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            std::copy(std::begin(key), std::end(key), std::begin(b->qg_key));
            b->qg_cap = capacity;
        }
        hipError_t e = hipGraphLaunch(b->q_exec, b->stream);
        if (e != hipSuccess) return bfail(b, SPG_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
        return SPG_OK;
    } catch (...) {
        return bfail(b, SPG_ERR_HIP, "host exception");
    }
}

spg_status spg_batch_get_stats(spg_batch b, spg_stats* out, int32_t size) {
    if (!b) return SPG_ERR_ARG;
    return spg_get_stats(b->h, out, size);
}

}  // extern "C"
