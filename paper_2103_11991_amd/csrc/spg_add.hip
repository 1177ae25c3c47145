// Sparse matrix addition C = alpha*A + beta*B on CRS matrices (section 2.3).
//
// Two phases like the product: symbolic finds, for every row, the union of
// the columns of A(i,:) and B(i,:) (entries of one column merged), its size
// (scanned into C's row pointer) and, for every input entry, the position of
// its column inside C's row (the paper's Apos and Bpos); numeric scatters
// alpha*A(i,j) and beta*B(i,j) to those positions and writes the columns, so
// a numeric call with new values needs no search at all.
//
// Per row, the entries' keys (column, then the entry's index inside the row:
// A's entries first) are ordered, and a key whose column differs from its
// predecessor's starts a new column of C.  When both rows are stored in
// ascending column order, A's keys followed by B's in reverse form a bitonic
// sequence, so the merge network of a bitonic sort alone orders them (log2 of
// the row's length steps, section 2.3); otherwise the full bitonic sort runs
// (section 5's team-level sort).  Rows of up to 64 entries sort in registers
// with cross-lane swaps (one wavefront per row), rows of up to 1024 in the
// wavefront's LDS, rows of up to 16384 on a 1024-lane workgroup with 128 KB
// of LDS; longer rows are refused (SPG_ERR_UNSUPPORTED).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>

#include "spg_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int MID_CAP = 1024;      // keys per wavefront in LDS
constexpr int LONG_CAP = 16384;    // keys per row on the long-row path
constexpr int LONG_THREADS = 1024;
constexpr int ROWS_PER_WG = 4;     // wavefronts (rows) per workgroup of the short/medium kernels
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr uint64_t ST_AGG = 1ull << 62, ST_PRE = 2ull << 62, ST_VAL = (1ull << 62) - 1;

// error flags
constexpr int AE_ROWPTR = 1, AE_COL = 2, AE_LONG = 4, AE_OVERFLOW = 8;

struct AddCtl {
    int32_t err;
    int32_t long_rows;      // rows queued for the long-row kernel
    int32_t tile_counter;   // dynamic tile id of the row-pointer scan
    int32_t pad;
    int64_t nnz_c;
};

// Orders a wavefront's own global-memory accesses (the C row it writes):
// workgroup scope is enough and writes nothing back from L2.
__device__ inline void wg_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, WAVE);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive sum over the wavefront.
__device__ inline int wave_scan(int x) {
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < WAVE; d <<= 1) {
        const int y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x;
}

// Key of entry t of the row (A's la entries, then B's): column, then t.
__device__ inline uint64_t make_key(int32_t col, int t) { return ((uint64_t)(uint32_t)col << 32) | (uint32_t)t; }

// Validity of the row's pointers and columns; the row's lengths.
__device__ inline bool row_range(const int32_t* rp, int64_t nnz, int32_t m, int64_t i, int& s, int& e) {
    s = rp[i], e = rp[i + 1];
    return !(s < 0 || e < s || (int64_t)e > nnz || (i == 0 && s != 0) || (i == m - 1 && (int64_t)e != nnz));
}

// The row's entries: t < la are A's, the others B's.
struct RowPair {
    const int32_t* ac;
    const int32_t* bc;
    int la, lb;
    __device__ inline int32_t col(int t) const { return t < la ? ac[t] : bc[t - la]; }
};

// Slot of entry t in the bitonic arrangement of P slots: A ascending in
// [0, la), B reversed at the end (descending), so the unused slots lie between.
__device__ inline int merge_slot(int t, int la, int lb, int P) { return t < la ? t : P - 1 - (t - la); }

// Writes each entry's position in C's row from the ordered keys (slot s
// holds key[s]) and returns the row's size.  Lanes of the group own P/G
// consecutive slots each.
template <int G>
__device__ inline int positions_from_sorted(const uint64_t* key, int P, int la, int32_t* apos, int32_t* bpos,
                                            int* red) {
    const int lane = threadIdx.x % G;
    const int per = P / G > 0 ? P / G : 1;
    const int s0 = lane * per;
    int local = 0;
    for (int s = s0; s < s0 + per && s < P; ++s) {
        const uint64_t k = key[s];
        if (k == ~0ull) break;
        local += s == 0 || (key[s - 1] >> 32) != (k >> 32);
    }
    int total, ex;
    if constexpr (G == WAVE) {
        const int incl = wave_scan(local);
        total = __shfl(incl, WAVE - 1, WAVE);
        ex = incl - local;
    } else {
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int incl = wave_scan(local);
        __syncthreads();
        if (wl == 63) red[wv] = incl;
        __syncthreads();
        int pre = 0;
        total = 0;
        for (int u = 0; u < G / WAVE; ++u) {
            if (u < wv) pre += red[u];
            total += red[u];
        }
        ex = pre + incl - local;
    }
    int pos = ex - 1;
    for (int s = s0; s < s0 + per && s < P; ++s) {
        const uint64_t k = key[s];
        if (k == ~0ull) break;
        pos += s == 0 || (key[s - 1] >> 32) != (k >> 32);
        const int t = (int)(uint32_t)k;
        if (t < la) apos[t] = pos;
        else bpos[t - la] = pos;
    }
    return total;
}

// Bitonic ordering of P (a power of two) keys in LDS by a group of G lanes:
// the merge network alone when the keys form a bitonic sequence, else the
// whole sort.  sync() orders the group's LDS accesses.
template <int G, typename Sync>
__device__ inline void lds_bitonic(uint64_t* key, int P, bool merge_only, Sync sync) {
    const int lane = threadIdx.x % G;
    for (int k = merge_only ? P : 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int x = lane; x < P / 2; x += G) {
                // the x-th pair of this step: lo has bit j clear
                const int lo = ((x & ~(j - 1)) << 1) | (x & (j - 1));
                const int hi = lo | j;
                const bool up = (lo & k) == 0;
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == up) key[lo] = b, key[hi] = a;
            }
            sync();
        }
    }
}

// Symbolic phase for rows of at most MID_CAP entries (longer rows are queued
// for k_add_sym_long).  One wavefront per row.
__global__ __launch_bounds__(WAVE * ROWS_PER_WG) void k_add_sym(int32_t m, int32_t n, const int32_t* __restrict__ arp,
                                                                const int32_t* __restrict__ aci, int64_t annz,
                                                                const int32_t* __restrict__ brp,
                                                                const int32_t* __restrict__ bci, int64_t bnnz,
                                                                int32_t* __restrict__ apos, int32_t* __restrict__ bpos,
                                                                int32_t* __restrict__ row_nnz,
                                                                int32_t* __restrict__ long_list, AddCtl* ctl) {
    __shared__ uint64_t keys[ROWS_PER_WG][MID_CAP];
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    uint64_t* key = keys[wv];
    for (int64_t i = (int64_t)blockIdx.x * ROWS_PER_WG + wv; i < m; i += (int64_t)gridDim.x * ROWS_PER_WG) {
        int as, ae, bs, be;
        const bool ok = row_range(arp, annz, m, i, as, ae) & row_range(brp, bnnz, m, i, bs, be);
        if (!ok) {
            if (lane == 0) atomicOr(&ctl->err, AE_ROWPTR), row_nnz[i] = 0;
            continue;
        }
        const RowPair rw{aci + as, bci + bs, ae - as, be - bs};
        const int L = rw.la + rw.lb;
        if (L > MID_CAP) {
            if (lane == 0) {
                long_list[atomicAdd(&ctl->long_rows, 1)] = (int32_t)i;
                row_nnz[i] = 0;
            }
            continue;
        }
        // columns in range, and whether each matrix row is ascending
        int bad = 0, unsorted = 0;
        for (int t = lane; t < L; t += WAVE) {
            const int32_t c = rw.col(t);
            bad |= c < 0 || c >= n;
            if (t != 0 && t != rw.la && rw.col(t - 1) > c) unsorted = 1;
        }
        if (__any(bad)) {
            if (lane == 0) atomicOr(&ctl->err, AE_COL), row_nnz[i] = 0;
            continue;
        }
        const bool merge_only = !__any(unsorted);
        int32_t* ap = apos + as;
        int32_t* bp = bpos + bs;
        if (L <= WAVE) {
            // one key per lane, the network in registers
            const int slot = lane;
            int P = 1;
            while (P < L) P <<= 1;
            // lane s holds slot s of the bitonic arrangement (or the whole input for a full sort)
            uint64_t v = ~0ull;
            if (merge_only) {
                const int t = slot < rw.la ? slot : (P - 1 - slot) < rw.lb ? rw.la + (P - 1 - slot) : -1;
                if (slot < P && t >= 0) v = make_key(rw.col(t), t);
            } else if (slot < L) {
                v = make_key(rw.col(slot), slot);
            }
            for (int k = merge_only ? P : 2; k <= P; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const uint64_t o = shfl_xor64(v, j);
                    const bool up = (slot & k) == 0;
                    const bool low = (slot & j) == 0;
                    // the lower slot of the pair keeps the smaller key when ascending
                    const bool take = low == up ? o < v : o > v;
                    if (slot < P && take) v = o;
                }
            // the previous slot's key (its column decides whether this one starts a column of C)
            const uint32_t plo = (uint32_t)__shfl_up((int)(uint32_t)v, 1, WAVE);
            const uint32_t phi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), 1, WAVE);
            const uint64_t pv = ((uint64_t)phi << 32) | plo;
            const bool valid = v != ~0ull;
            const int start = valid && (slot == 0 || (pv >> 32) != (v >> 32));
            const int incl = wave_scan(start);
            if (valid) {
                const int t = (int)(uint32_t)v;
                if (t < rw.la) ap[t] = incl - 1;
                else bp[t - rw.la] = incl - 1;
            }
            const int total = __shfl(incl, WAVE - 1, WAVE);
            if (lane == 0) row_nnz[i] = total;
            continue;
        }
        // keys in the wavefront's LDS
        int P = WAVE;
        while (P < L) P <<= 1;
        for (int s = lane; s < P; s += WAVE) key[s] = ~0ull;
        wave_sync();
        for (int t = lane; t < L; t += WAVE) {
            const int s = merge_only ? merge_slot(t, rw.la, rw.lb, P) : t;
            key[s] = make_key(rw.col(t), t);
        }
        wave_sync();
        lds_bitonic<WAVE>(key, P, merge_only, wave_sync);
        const int total = positions_from_sorted<WAVE>(key, P, rw.la, ap, bp, nullptr);
        if (lane == 0) row_nnz[i] = total;
        wave_sync();
    }
}

// Symbolic phase of the queued long rows (MID_CAP < entries <= LONG_CAP):
// one 1024-lane workgroup per row, keys in 128 KB of LDS.
__global__ __launch_bounds__(LONG_THREADS) void k_add_sym_long(int32_t n, const int32_t* __restrict__ arp,
                                                               const int32_t* __restrict__ aci,
                                                               const int32_t* __restrict__ brp,
                                                               const int32_t* __restrict__ bci,
                                                               int32_t* __restrict__ apos, int32_t* __restrict__ bpos,
                                                               int32_t* __restrict__ row_nnz,
                                                               const int32_t* __restrict__ long_list, AddCtl* ctl) {
    extern __shared__ uint64_t key[];
    __shared__ int red[LONG_THREADS / WAVE];
    __shared__ int flags[2];
    const int count = ctl->long_rows;
    const int tid = threadIdx.x;
    for (int r = blockIdx.x; r < count; r += gridDim.x) {
        const int i = long_list[r];
        const int as = arp[i], bs = brp[i];
        const RowPair rw{aci + as, bci + bs, arp[i + 1] - as, brp[i + 1] - bs};
        const int L = rw.la + rw.lb;
        if (tid == 0) flags[0] = flags[1] = 0;
        __syncthreads();
        if (L > LONG_CAP) {
            if (tid == 0) atomicOr(&ctl->err, AE_LONG);
            continue;
        }
        int bad = 0, unsorted = 0;
        for (int t = tid; t < L; t += LONG_THREADS) {
            const int32_t c = rw.col(t);
            bad |= c < 0 || c >= n;
            if (t != 0 && t != rw.la && rw.col(t - 1) > c) unsorted = 1;
        }
        if (bad) atomicOr(&flags[0], 1);
        if (unsorted) atomicOr(&flags[1], 1);
        __syncthreads();
        if (flags[0]) {
            if (tid == 0) atomicOr(&ctl->err, AE_COL), row_nnz[i] = 0;
            __syncthreads();
            continue;
        }
        const bool merge_only = flags[1] == 0;
        int P = LONG_THREADS;
        while (P < L) P <<= 1;
        for (int s = tid; s < P; s += LONG_THREADS) key[s] = ~0ull;
        __syncthreads();
        for (int t = tid; t < L; t += LONG_THREADS) {
            const int s = merge_only ? merge_slot(t, rw.la, rw.lb, P) : t;
            key[s] = make_key(rw.col(t), t);
        }
        __syncthreads();
        lds_bitonic<LONG_THREADS>(key, P, merge_only, [] { __syncthreads(); });
        const int total = positions_from_sorted<LONG_THREADS>(key, P, rw.la, apos + as, bpos + bs, red);
        if (tid == 0) row_nnz[i] = total;
        __syncthreads();
    }
}

// C's row pointer: exclusive scan of the row sizes in int64, single pass with
// decoupled look-back over tiles taken in order; flags nnz(C) >= 2^31.
__global__ __launch_bounds__(SCAN_THREADS) void k_add_scan(int32_t m, const int32_t* __restrict__ row_nnz,
                                                           int32_t* __restrict__ crp, uint64_t* tile_status,
                                                           AddCtl* ctl) {
    __shared__ int32_t tile_sh;
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    __shared__ int64_t tile_prefix;
    if (threadIdx.x == 0) tile_sh = atomicAdd(&ctl->tile_counter, 1);
    __syncthreads();
    const int tile = tile_sh;
    const int64_t r0 = (int64_t)tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        const int64_t r = r0 + t;
        run += r < m ? row_nnz[r] : 0;
        v[t] = run;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t x = run;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int64_t wpre = 0, agg = 0;
    for (int u = 0; u < SCAN_THREADS / 64; ++u) {
        if (u < wv) wpre += wsum[u];
        agg += wsum[u];
    }
    if (threadIdx.x == 0) {
        int64_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(&tile_status[0], ST_PRE | (uint64_t)agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&tile_status[tile], ST_AGG | (uint64_t)agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int t = tile - 1; t >= 0; --t) {
                uint64_t st;
                do {
                    st = __hip_atomic_load(&tile_status[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while ((st >> 62) == 0);
                prefix += (int64_t)(st & ST_VAL);
                if ((st >> 62) == 2) break;
            }
            __hip_atomic_store(&tile_status[tile], ST_PRE | (uint64_t)(prefix + agg), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        tile_prefix = prefix;
        const int64_t last_tile = ((int64_t)m + SCAN_TILE - 1) / SCAN_TILE - 1;
        if (tile == last_tile) {
            ctl->nnz_c = prefix + agg;
            if (prefix + agg > INT_MAX) atomicOr(&ctl->err, AE_OVERFLOW);
        }
    }
    __syncthreads();
    const int64_t base = tile_prefix + wpre + x - run;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        const int64_t r = r0 + t;
        if (r < m) crp[r + 1] = (int32_t)(base + v[t]);
    }
    if (tile == 0 && threadIdx.x == 0) crp[0] = 0;
}

// Numeric phase: per row, every entry adds alpha*a (A's first) or beta*b at
// its position; columns written by every contributor (the same value).  Rows
// of at most MID_CAP columns sum in the wavefront's LDS and copy out
// coalesced; longer rows sum in C's own storage.  Entries of A are added
// before those of B, so a column with one entry of each gets alpha*a + beta*b
// exactly as written.
template <typename T>
__global__ __launch_bounds__(WAVE * ROWS_PER_WG) void k_add_num(int32_t m, const int32_t* __restrict__ arp,
                                                                const int32_t* __restrict__ aci,
                                                                const T* __restrict__ av, const int32_t* __restrict__ brp,
                                                                const int32_t* __restrict__ bci,
                                                                const T* __restrict__ bv,
                                                                const int32_t* __restrict__ apos,
                                                                const int32_t* __restrict__ bpos,
                                                                const int32_t* __restrict__ crp, T alpha, T beta,
                                                                int32_t* __restrict__ ccol, T* __restrict__ cval) {
    __shared__ T acc[ROWS_PER_WG][MID_CAP];
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    T* s = acc[wv];
    for (int64_t i = (int64_t)blockIdx.x * ROWS_PER_WG + wv; i < m; i += (int64_t)gridDim.x * ROWS_PER_WG) {
        const int as = arp[i], ae = arp[i + 1], bs = brp[i], be = brp[i + 1];
        const int c0 = crp[i], nc = crp[i + 1] - c0;
        int32_t* cc = ccol + c0;
        T* cv = cval + c0;
        const bool in_lds = nc <= MID_CAP;
        T* dst = in_lds ? s : cv;
        for (int r = lane; r < nc; r += WAVE) dst[r] = T(0);
        if (!in_lds) wg_fence();
        wave_sync();
        for (int t = as + lane; t < ae; t += WAVE) {
            const int p = apos[t];
            cc[p] = aci[t];
            atomicAdd(&dst[p], alpha * av[t]);
        }
        if (!in_lds) wg_fence();
        wave_sync();
        for (int t = bs + lane; t < be; t += WAVE) {
            const int p = bpos[t];
            cc[p] = bci[t];
            atomicAdd(&dst[p], beta * bv[t]);
        }
        wave_sync();
        if (in_lds)
            for (int r = lane; r < nc; r += WAVE) cv[r] = s[r];
        wave_sync();
    }
}

int64_t add_scan_tiles(int32_t m) { return ((int64_t)m + SCAN_TILE - 1) / SCAN_TILE; }

}  // namespace

struct spg_add_s {
    hipStream_t stream = nullptr;
    int n_cu = 256;
    std::string err;
    spg_dtype dt = SPG_F64;
    int32_t m = 0, n = 0;
    const int32_t *arp = nullptr, *aci = nullptr, *brp = nullptr, *bci = nullptr;
    int64_t annz = 0, bnnz = 0;
    int32_t* crp = nullptr;
    int64_t nnz_c = 0;
    bool have_sym = false;
    void* buf = nullptr;     // apos | bpos | row_nnz | long list | tile status | control
    size_t cap = 0;
    AddCtl* hctl = nullptr;  // pinned copy of the control block
    int32_t *apos = nullptr, *bpos = nullptr, *row_nnz = nullptr, *long_list = nullptr;
    uint64_t* tiles = nullptr;
    AddCtl* ctl = nullptr;
};

namespace {

spg_status afail(spg_add h, spg_status s, const std::string& msg) {
    if (h) h->err = msg;
    return s;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

spg_status spg_add_create(spg_add* out, void* stream) {
    if (!out) return SPG_ERR_ARG;
    *out = nullptr;
    try {
        spg_add h = new spg_add_s();
        h->stream = static_cast<hipStream_t>(stream);
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipHostMalloc((void**)&h->hctl, sizeof(AddCtl), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return SPG_ERR_HIP;
        }
        *out = h;
        return SPG_OK;
    } catch (...) {
        return SPG_ERR_ALLOC;
    }
}

spg_status spg_add_destroy(spg_add h) {
    if (!h) return SPG_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->buf) (void)hipFree(h->buf);
    if (h->hctl) (void)hipHostFree(h->hctl);
    delete h;
    return SPG_OK;
}

const char* spg_add_last_error(spg_add h) { return h ? h->err.c_str() : "null handle"; }

spg_status spg_add_symbolic(spg_add h, int32_t m, int32_t n, const int32_t* a_row_ptr, const int32_t* a_col_idx,
                            int64_t a_nnz, const int32_t* b_row_ptr, const int32_t* b_col_idx, int64_t b_nnz,
                            int32_t* c_row_ptr, int64_t* nnz_c) {
    if (!h) return SPG_ERR_ARG;
    try {
        h->have_sym = false;
        if (m < 0 || n < 0 || a_nnz < 0 || b_nnz < 0) return afail(h, SPG_ERR_ARG, "negative dimension or nnz");
        if (a_nnz > INT32_MAX || b_nnz > INT32_MAX) return afail(h, SPG_ERR_ARG, "nnz exceeds int32 range");
        if (!a_row_ptr || !b_row_ptr || !c_row_ptr || !nnz_c) return afail(h, SPG_ERR_ARG, "null pointer");
        if ((a_nnz > 0 && !a_col_idx) || (b_nnz > 0 && !b_col_idx)) return afail(h, SPG_ERR_ARG, "null column index");
        if (n == 0 && (a_nnz > 0 || b_nnz > 0)) return afail(h, SPG_ERR_SHAPE, "entries but no columns");
        h->m = m, h->n = n;
        h->arp = a_row_ptr, h->aci = a_col_idx, h->annz = a_nnz;
        h->brp = b_row_ptr, h->bci = b_col_idx, h->bnnz = b_nnz;
        const size_t M = (size_t)std::max(m, 1);
        const size_t need = align256((size_t)std::max<int64_t>(a_nnz, 1) * 4) +
                            align256((size_t)std::max<int64_t>(b_nnz, 1) * 4) + 2 * align256(M * 4) +
                            align256((size_t)(add_scan_tiles(m) + 1) * 8) + align256(sizeof(AddCtl));
        if (need > h->cap) {
            if (h->buf) {
                if (hipStreamSynchronize(h->stream) != hipSuccess) return afail(h, SPG_ERR_HIP, "stream wait");
                (void)hipFree(h->buf);
                h->buf = nullptr, h->cap = 0;
            }
            if (hipMalloc(&h->buf, need) != hipSuccess) {
                (void)hipGetLastError();
                return afail(h, SPG_ERR_ALLOC, "device allocation of " + std::to_string(need) + " bytes failed");
            }
            h->cap = need;
        }
        uint8_t* p = static_cast<uint8_t*>(h->buf);
        h->apos = reinterpret_cast<int32_t*>(p), p += align256((size_t)std::max<int64_t>(a_nnz, 1) * 4);
        h->bpos = reinterpret_cast<int32_t*>(p), p += align256((size_t)std::max<int64_t>(b_nnz, 1) * 4);
        h->row_nnz = reinterpret_cast<int32_t*>(p), p += align256(M * 4);
        h->long_list = reinterpret_cast<int32_t*>(p), p += align256(M * 4);
        h->tiles = reinterpret_cast<uint64_t*>(p), p += align256((size_t)(add_scan_tiles(m) + 1) * 8);
        h->ctl = reinterpret_cast<AddCtl*>(p);
        hipStream_t s = h->stream;
        spg::launch_fill_u8(s, h->ctl, 0, sizeof(AddCtl));
        if (m > 0) {
            const int grid_rows = (int)std::min<int64_t>(((int64_t)m + ROWS_PER_WG - 1) / ROWS_PER_WG,
                                                         (int64_t)h->n_cu * 32);
            hipLaunchKernelGGL(k_add_sym, dim3(grid_rows), dim3(WAVE * ROWS_PER_WG), 0, s, m, n, a_row_ptr, a_col_idx,
                               a_nnz, b_row_ptr, b_col_idx, b_nnz, h->apos, h->bpos, h->row_nnz, h->long_list, h->ctl);
            hipLaunchKernelGGL(k_add_sym_long, dim3((unsigned)std::min(h->n_cu, m)), dim3(LONG_THREADS),
                               (size_t)LONG_CAP * 8, s, n, a_row_ptr, a_col_idx, b_row_ptr, b_col_idx, h->apos,
                               h->bpos, h->row_nnz, h->long_list, h->ctl);
            spg::launch_fill_u8(s, h->tiles, 0, (size_t)(add_scan_tiles(m) + 1) * 8);
            hipLaunchKernelGGL(k_add_scan, dim3((unsigned)add_scan_tiles(m)), dim3(SCAN_THREADS), 0, s, m, h->row_nnz,
                               c_row_ptr, h->tiles, h->ctl);
        } else {
            spg::launch_fill_i32(s, c_row_ptr, 0, 1);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return afail(h, SPG_ERR_HIP, std::string("symbolic launch: ") + hipGetErrorString(e));
        if (hipMemcpyAsync(h->hctl, h->ctl, sizeof(AddCtl), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return afail(h, SPG_ERR_HIP, "control block read-back");
        const AddCtl c = *h->hctl;
        if (c.err & AE_ROWPTR) return afail(h, SPG_ERR_INDEX, "malformed row pointer in A or B");
        if (c.err & AE_COL) return afail(h, SPG_ERR_INDEX, "column index out of range in A or B");
        if (c.err & AE_LONG)
            return afail(h, SPG_ERR_UNSUPPORTED, "a row of A and B together holds more than " +
                                                     std::to_string(LONG_CAP) + " entries");
        if (c.err & AE_OVERFLOW) return afail(h, SPG_ERR_OVERFLOW, "nnz(C) exceeds the int32 range");
        h->nnz_c = m > 0 ? c.nnz_c : 0;
        h->crp = c_row_ptr;
        h->have_sym = true;
        *nnz_c = h->nnz_c;
        return SPG_OK;
    } catch (...) {
        return afail(h, SPG_ERR_HIP, "unexpected host exception");
    }
}

spg_status spg_add_numeric(spg_add h, spg_dtype dt, double alpha, const void* a_vals, double beta,
                           const void* b_vals, int32_t* c_col_idx, void* c_vals) {
    if (!h) return SPG_ERR_ARG;
    try {
        if (!h->have_sym) return afail(h, SPG_ERR_STATE, "spg_add_symbolic must come first");
        if (dt != SPG_F32 && dt != SPG_F64) return afail(h, SPG_ERR_ARG, "dtype must be SPG_F32 or SPG_F64");
        if ((h->annz > 0 && !a_vals) || (h->bnnz > 0 && !b_vals)) return afail(h, SPG_ERR_ARG, "null input values");
        if (h->nnz_c > 0 && (!c_col_idx || !c_vals)) return afail(h, SPG_ERR_ARG, "null output");
        if (h->m == 0) return SPG_OK;
        const int grid = (int)std::min<int64_t>(((int64_t)h->m + ROWS_PER_WG - 1) / ROWS_PER_WG, (int64_t)h->n_cu * 32);
        if (dt == SPG_F64)
            hipLaunchKernelGGL(k_add_num<double>, dim3(grid), dim3(WAVE * ROWS_PER_WG), 0, h->stream, h->m, h->arp,
                               h->aci, static_cast<const double*>(a_vals), h->brp, h->bci,
                               static_cast<const double*>(b_vals), h->apos, h->bpos, h->crp, alpha, beta, c_col_idx,
                               static_cast<double*>(c_vals));
        else
            hipLaunchKernelGGL(k_add_num<float>, dim3(grid), dim3(WAVE * ROWS_PER_WG), 0, h->stream, h->m, h->arp,
                               h->aci, static_cast<const float*>(a_vals), h->brp, h->bci,
                               static_cast<const float*>(b_vals), h->apos, h->bpos, h->crp, (float)alpha,
                               (float)beta, c_col_idx, static_cast<float*>(c_vals));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return afail(h, SPG_ERR_HIP, std::string("numeric launch: ") + hipGetErrorString(e));
        return SPG_OK;
    } catch (...) {
        return afail(h, SPG_ERR_HIP, "unexpected host exception");
    }
}

}  // extern "C"
