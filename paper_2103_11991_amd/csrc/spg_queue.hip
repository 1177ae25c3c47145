// Batched products through one persistent kernel over a device work queue.
//
// Many independent products C_p = A_p * B_p (packed block-diagonally, see
// spg_batch_create) run as work items {product, block of rows, phase}.  The
// paper runs many small operations of one kind inside one parallel dispatch
// (section 3) and notes that launch latency matters as per-launch work
// shrinks (section 2.2.2); here one launch runs both phases of every product
// and nothing returns to the host in between:
//
//   symbolic items  (product, row block): each row's size, taken in product
//                   order by a global counter;
//   product finish  the workgroup that completes a product's last symbolic
//                   item scans the product's row sizes into its row pointer
//                   (the segmented scan), takes the product's C space from a
//                   device bump allocator over the caller's pools, and appends
//                   the product's numeric items to the queue;
//   numeric items   (product, row block): columns and values, written at the
//                   product's place in the pools.
//
// Workgroups take the queue's slots in order; a slot past the symbolic items
// is a numeric slot, which its workgroup waits for (every symbolic item was
// taken before it, by a running workgroup, and every product's numeric items
// are appended when its symbolic items end, so every wait ends).  Data one
// workgroup writes for another (row sizes, row pointers, queue entries) is
// stored and loaded at device scope; the queue entry is stored only after the
// writer has waited for its data stores to complete.
//
// A row is one group of RG = 32 lanes (two rows per wavefront): a bitmap of the
// row's column range in LDS (each product's B columns, or its compressed-B
// runs, are OR-ed in, lanes over the flattened (A entry, B entry) products),
// its popcount for the symbolic phase; in the numeric phase the bitmap's
// prefix of popcounts gives every column its rank, products are added at
// their ranks in an LDS value array (lanes over groups of four consecutive
// entries of each B row), and the row leaves sorted.  The LDS window of a
// group is sized for the batch's widest row (at most 128 words, 4096
// columns).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spg_internal.h"

namespace spg {

namespace {

constexpr int QWAVES = 4;  // wavefronts per workgroup
constexpr int RG = 32;     // lanes per row (two rows per wavefront)
constexpr int QGROUPS = QWAVES * 64 / RG;
constexpr int64_t QUEUE_SPIN_LIMIT = (int64_t)1 << 26;

__device__ inline void qwave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Inclusive sum over the lane's group of RG lanes.
__device__ inline int wscan_incl(int x) {
    const int lane = threadIdx.x & (RG - 1);
    for (int d = 1; d < RG; d <<= 1) {
        const int y = __shfl_up(x, d, RG);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline int wsum(int x) { return __shfl(wscan_incl(x), RG - 1, RG); }

// Inclusive sum over the whole wavefront (64 lanes, whatever RG is).
__device__ inline int wave_scan_incl(int x) {
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Position of set bit number k (from 0) of m, which has more than k bits set.
__device__ inline int nth_bit(uint32_t m, int k) {
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const int c = __popc(m & ((1u << w) - 1u));
        if (k >= c) k -= c, m >>= w, pos += w;
    }
    return pos;
}

template <typename T>
__device__ inline void st_dev(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ inline T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every vector memory access of this thread has completed (its device-scope
// stores are visible to other workgroups).
__device__ inline void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

// One wavefront's LDS window.
template <typename T>
struct Win_ {
    uint32_t* bm;   // bitmap words of the row's column range
    int* pf;        // exclusive prefix of their popcounts
    T* vals;        // the row's values, by rank
    int* pre;       // staged A entries: exclusive prefix of their B row lengths (groups)
    int* st;        // ... first B entry
    int* len;       // ... B row length
    T* av;          // ... A value
};

// OR of v over the run of consecutive lanes of the group with the same key
// that ends at this lane, returned by the run's last lane (others return 0).
// `full`: all RG lanes of the group are active (else each lane's run is
// itself alone).
__device__ inline uint32_t or_runs(uint32_t v, int key, int lane, bool full) {
    if (!full) return v;
    // segmented inclusive OR: a lane takes its left neighbour's partial while
    // the keys agree all the way (heads stop the propagation)
    const int prev = __shfl_up(key, 1, RG);
    bool head = lane == 0 || prev != key;
    for (int d = 1; d < RG; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)v, d, RG);
        const int hk = __shfl_up((int)head, d, RG);
        if (lane >= d && !head) v |= o;
        head = head || (lane >= d && hk);
    }
    const int next = __shfl_down(key, 1, RG);
    return (lane == RG - 1 || next != key) ? v : 0u;
}

// Products per lane whose loads are issued together in the walks below.
constexpr int QU = 2;

// The entry of the staged chunk that holds flattened product q (pre: the
// exclusive prefix of the entries' B row lengths, cnt entries).
__device__ inline int entry_of(const int* pre, int cnt, int q) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ORs the row's columns into bm (cleared by the caller).  Lanes walk the
// flattened products of chunks of RG A entries, QU slices of RG products at
// a time: every lane's QU loads go out together (a lane past the end loads
// the last product again and drops it), which keeps them from waiting on
// each other.
template <typename T>
__device__ inline void row_walk(const QueueArgs& a, int64_t r, int base, const Win_<T>& w) {
    const int lane = threadIdx.x & (RG - 1);
    const int a0 = a.arp[r], a1 = a.arp[r + 1];
    for (int e0 = a0; e0 < a1; e0 += RG) {
        // the chunk's entries: unconditional loads (index clamped into the row)
        const bool in_row = e0 + lane < a1;
        const int j = a.aci[min(e0 + lane, a1 - 1)];
        const int s0 = a.brp[j];
        const int len = in_row ? a.brp[j + 1] - s0 : 0;
        const int incl = wscan_incl(len);
        const int total = __shfl(incl, RG - 1, RG);
        const int cnt = min(RG, a1 - e0);
        w.pre[lane] = incl - len, w.st[lane] = s0;
        qwave_sync();
        for (int Q = 0; Q < total; Q += QU * RG) {
            int cc[QU];
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int q = min(Q + u * RG + lane, total - 1);
                const int lo = entry_of(w.pre, cnt, q);
                cc[u] = a.bci[w.st[lo] + (q - w.pre[lo])];
            }
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int qs = Q + u * RG;  // the slice's first product (uniform in the group)
                if (qs >= total) break;
                const bool ok = qs + lane < total;
                const int c = cc[u];
                const int wd = (c >> 5) - base;
                // neighbouring lanes mostly share a word (a B row's columns
                // are close): OR the bits of each run of lanes on one word
                // together, and only the run's last lane writes LDS
                const uint32_t bits = or_runs(1u << (c & 31), ok ? wd : -1, lane, qs + RG <= total);
                if (ok && bits) atomicOr(&w.bm[wd], bits);
            }
        }
        qwave_sync();
    }
}

// Four consecutive entries of B from index b (the first min(4, end - b) of
// them used), read with one 16-byte load per array unless the group would
// reach past the last entry of B's pools.
struct __attribute__((packed, aligned(4))) QI4 {
    int x, y, z, w;
};
struct __attribute__((packed, aligned(8))) QD2 {
    double x, y;
};
struct __attribute__((packed, aligned(4))) QF4 {
    float x, y, z, w;
};
template <typename T>
struct QGroup {
    int c[4];
    T y[4];
};
template <typename T>
__device__ inline QGroup<T> load_group(const int32_t* __restrict__ bci, const T* __restrict__ bv, int64_t bnnz,
                                       int b) {
    QGroup<T> g;
    if (b + 4 <= bnnz) {
        const QI4 c = *reinterpret_cast<const QI4*>(bci + b);
        g.c[0] = c.x, g.c[1] = c.y, g.c[2] = c.z, g.c[3] = c.w;
        if constexpr (sizeof(T) == 8) {
            const QD2 v0 = *reinterpret_cast<const QD2*>(bv + b);
            const QD2 v1 = *reinterpret_cast<const QD2*>(bv + b + 2);
            g.y[0] = v0.x, g.y[1] = v0.y, g.y[2] = v1.x, g.y[3] = v1.y;
        } else {
            const QF4 v = *reinterpret_cast<const QF4*>(bv + b);
            g.y[0] = v.x, g.y[1] = v.y, g.y[2] = v.z, g.y[3] = v.w;
        }
    } else {
        // the pools' last group: every index clamped to the last entry
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t q = min<int64_t>(b + j, bnnz - 1);
            g.c[j] = bci[q];
            g.y[j] = bv[q];
        }
    }
    return g;
}

// The numeric phase's walk: products added at their ranks (bm and pf hold
// the row's columns and their prefix), lanes over groups of four
// consecutive entries of each staged B row, so that a lane's entries come
// with three 16-byte loads and one search for their A entry.
template <typename T>
__device__ inline void row_walk_num(const QueueArgs& a, int64_t r, int base, const Win_<T>& w) {
    const int lane = threadIdx.x & (RG - 1);
    const int a0 = a.arp[r], a1 = a.arp[r + 1];
    const T* av = reinterpret_cast<const T*>(a.av);
    const T* bv = reinterpret_cast<const T*>(a.bv);
    for (int e0 = a0; e0 < a1; e0 += RG) {
        const bool in_row = e0 + lane < a1;
        const int e = min(e0 + lane, a1 - 1);
        const int j = a.aci[e];
        const T x = av[e];
        const int s0 = a.brp[j];
        const int len = in_row ? a.brp[j + 1] - s0 : 0;
        const int ng = (len + 3) >> 2;
        const int incl = wscan_incl(ng);
        const int total = __shfl(incl, RG - 1, RG);
        const int cnt = min(RG, a1 - e0);
        w.pre[lane] = incl - ng, w.st[lane] = s0, w.len[lane] = len;
        w.av[lane] = x;
        qwave_sync();
        for (int q0 = 0; q0 < total; q0 += RG) {
            const int q = min(q0 + lane, total - 1);  // a lane past the end loads the last group again
            const int lo = entry_of(w.pre, cnt, q);
            const int k = (q - w.pre[lo]) * 4;  // the group's first entry within its B row
            const QGroup<T> g = load_group<T>(a.bci, bv, a.bnnz, w.st[lo] + k);
            if (q0 + lane < total) {
                const int n = min(4, w.len[lo] - k);
                const T xa = w.av[lo];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (jj < n) {
                        const int c = g.c[jj];
                        const int wd = (c >> 5) - base;
                        const int rank = w.pf[wd] + __popc(w.bm[wd] & ((1u << (c & 31)) - 1u));
                        atomicAdd(&w.vals[rank], xa * g.y[jj]);
                    }
                }
            }
        }
        qwave_sync();
    }
}

// The row's compressed-B runs {block, mask} OR-ed into bm (cleared by the
// caller): the symbolic phase's walk, over a B row's runs instead of its
// entries (section 2.2.1, compressed B), with the loads issued as above.
template <typename T>
__device__ inline void row_walk_runs(const QueueArgs& a, int64_t r, int base, const Win_<T>& w) {
    const int lane = threadIdx.x & (RG - 1);
    const int a0 = a.arp[r], a1 = a.arp[r + 1];
    for (int e0 = a0; e0 < a1; e0 += RG) {
        const bool in_row = e0 + lane < a1;
        const int4 h = a.bhdr[a.aci[min(e0 + lane, a1 - 1)]];
        const int s0 = h.z, len = in_row ? h.w : 0;
        const int incl = wscan_incl(len);
        const int total = __shfl(incl, RG - 1, RG);
        const int cnt = min(RG, a1 - e0);
        w.pre[lane] = incl - len, w.st[lane] = s0;
        qwave_sync();
        for (int Q = 0; Q < total; Q += QU * RG) {
            int2 run[QU];
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int q = min(Q + u * RG + lane, total - 1);
                const int lo = entry_of(w.pre, cnt, q);
                run[u] = a.bc[w.st[lo] + (q - w.pre[lo])];
            }
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int qs = Q + u * RG;
                if (qs >= total) break;
                const bool ok = qs + lane < total;
                const int wd = run[u].x - base;
                const uint32_t bits = or_runs((uint32_t)run[u].y, ok ? wd : -1, lane, qs + RG <= total);
                if (ok && bits) atomicOr(&w.bm[wd], bits);
            }
        }
        qwave_sync();
    }
}

// Symbolic phase of packed row r: its size into row_nnz (device scope).
template <typename T>
__device__ inline void sym_row(const QueueArgs& a, int64_t r, const Win_<T>& w) {
    const int lane = threadIdx.x & (RG - 1);
    const RowInfo ri = a.rinfo[r];
    if (ri.z == 0) {
        if (lane == 0) st_dev(&a.row_nnz[r], 0);
        return;
    }
    const int base = ri.x >> 5, words = (ri.y >> 5) - base + 1;
    for (int t = lane; t < words; t += RG) w.bm[t] = 0;
    qwave_sync();
    if (a.bc) row_walk_runs<T>(a, r, base, w);
    else row_walk<T>(a, r, base, w);
    int c = 0;
    for (int t = lane; t < words; t += RG) {
        const uint32_t mk = w.bm[t];
        c += __popc(mk);
        if (a.qbm) st_dev(&a.qbm[r * a.wmax + t], mk);  // kept for the numeric phase
    }
    c = wsum(c);
    if (lane == 0) st_dev(&a.row_nnz[r], c);
    qwave_sync();
}

// Numeric phase of packed row r into C at `off` (its row pointer's entry).
template <typename T>
__device__ inline void num_row(const QueueArgs& a, int64_t r, int64_t off, int n, const Win_<T>& w) {
    const int lane = threadIdx.x & (RG - 1);
    const RowInfo ri = a.rinfo[r];
    if (ri.z == 0 || n == 0) return;
    const int base = ri.x >> 5, words = (ri.y >> 5) - base + 1;
    for (int t = lane; t < n; t += RG) w.vals[t] = T(0);
    if (a.qbm) {
        // the row's columns as the symbolic phase left them
        for (int t = lane; t < words; t += RG) w.bm[t] = ld_dev(&a.qbm[r * a.wmax + t]);
        qwave_sync();
    } else {
        for (int t = lane; t < words; t += RG) w.bm[t] = 0;
        qwave_sync();
        row_walk<T>(a, r, base, w);
    }
    // ranks: exclusive prefix of the words' popcounts (each lane a run of words)
    const int per = (words + RG - 1) / RG;
    const int t0 = min(lane * per, words), t1 = min(t0 + per, words);
    int loc = 0;
    for (int t = t0; t < t1; ++t) loc += __popc(w.bm[t]);
    int ex = wscan_incl(loc) - loc;
    for (int t = t0; t < t1; ++t) {
        w.pf[t] = ex;
        ex += __popc(w.bm[t]);
    }
    qwave_sync();
    // the row's columns, ascending, one rank per lane (coalesced): the word
    // holding rank k by binary search over the prefix, then its bit
    for (int k = lane; k < n; k += RG) {
        int lo = 0, hi = words - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (w.pf[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        a.ccol[off + k] = ((base + lo) << 5) + nth_bit(w.bm[lo], k - w.pf[lo]);
    }
    qwave_sync();
    row_walk_num<T>(a, r, base, w);
    T* cv = reinterpret_cast<T*>(a.cval) + off;
    for (int t = lane; t < n; t += RG) cv[t] = w.vals[t];
    qwave_sync();
}

__device__ inline int64_t clock_now() { return (int64_t)wall_clock64(); }

// The product's row pointer from its rows' sizes, its C space from the bump
// allocator, and its numeric items onto the queue.  Run by one workgroup.
template <typename T>
__device__ void finish_product(const QueueArgs& a, int p, int64_t* red64, int* flag) {
    const int tid = threadIdx.x;
    const int64_t r0 = a.row_off[p], m = a.row_off[p + 1] - r0;
    int32_t* crp = a.c_row_ptr + a.crp_off[p];
    // total, then the allocation, then the scan written with the offset
    int64_t s = 0;
    for (int64_t i = tid; i < m; i += blockDim.x) s += ld_dev(&a.row_nnz[r0 + i]);
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((tid & 63) == 0) red64[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t tot = 0;
        for (int u = 0; u < QWAVES; ++u) tot += red64[u];
        const int64_t off = atomicAdd((unsigned long long*)&a.qc->used, (unsigned long long)tot);
        const bool ok = off + tot <= a.cap && off + tot <= INT32_MAX;
        red64[QWAVES] = ok ? off : -1;
        st_dev(&a.c_offsets[p], ok ? off : (int64_t)-1);
    }
    __syncthreads();
    const int64_t off = red64[QWAVES];
    if (off >= 0) {
        // segmented scan of the product's rows, 256 rows per pass
        int64_t run = off;
        for (int64_t b0 = 0; b0 < m; b0 += blockDim.x) {
            const int64_t i = b0 + tid;
            const int v = i < m ? ld_dev(&a.row_nnz[r0 + i]) : 0;
            const int incl = wave_scan_incl(v);
            __syncthreads();
            if ((tid & 63) == 63) red64[tid >> 6] = incl;
            __syncthreads();
            int64_t pre = 0, tot = 0;
            for (int u = 0; u < QWAVES; ++u) {
                if (u < (tid >> 6)) pre += red64[u];
                tot += red64[u];
            }
            if (i < m) st_dev(&crp[i], (int32_t)(run + pre + incl - v));
            run += tot;
        }
        if (tid == 0) st_dev(&crp[m], (int32_t)run);
    }
    wait_mem();
    __syncthreads();
    // numeric items of the product (marked to be skipped if it did not fit)
    const int64_t nb = a.item_off[p + 1] - a.item_off[p];
    if (tid == 0) red64[0] = (int64_t)atomicAdd((unsigned long long*)&a.qc->tail, (unsigned long long)nb);
    __syncthreads();
    const int64_t slot = red64[0];
    for (int64_t b = tid; b < nb; b += blockDim.x) {
        const int64_t e = (((int64_t)p << 32) | b) + 1;
        st_dev(&a.queue[slot + b], off >= 0 ? e : -e);
    }
    wait_mem();
    __syncthreads();
    (void)flag;
}

// (6 waves per SIMD: the grouped numeric walk would otherwise take 83 VGPRs
// and 5 waves; measured on 1024 banded products, 12.7 against 14.0 ms)
template <typename T>
__global__ __launch_bounds__(64 * QWAVES) __attribute__((amdgpu_waves_per_eu(6))) void k_queue(QueueArgs a) {
    extern __shared__ __align__(16) uint8_t qsm[];
    __shared__ int64_t s_k, s_e;
    __shared__ int64_t red64[QWAVES + 1];
    __shared__ int s_last, s_flag;
    const int tid = threadIdx.x, gi = tid / RG;
    // this row group's window
    const size_t per_group = (size_t)a.wmax * 8 + (size_t)a.vmax * sizeof(T) + RG * (12 + sizeof(T));
    uint8_t* mine = qsm + per_group * gi;
    Win_<T> w;
    w.bm = reinterpret_cast<uint32_t*>(mine);
    w.pf = reinterpret_cast<int*>(mine + (size_t)a.wmax * 4);
    w.vals = reinterpret_cast<T*>(mine + (size_t)a.wmax * 8);
    w.av = reinterpret_cast<T*>(mine + (size_t)a.wmax * 8 + (size_t)a.vmax * sizeof(T));
    w.pre = reinterpret_cast<int*>(reinterpret_cast<uint8_t*>(w.av) + RG * sizeof(T));
    w.st = w.pre + RG;
    w.len = w.st + RG;
    const int64_t n = a.n_items;
    while (true) {
        if (tid == 0) s_k = (int64_t)atomicAdd((unsigned long long*)&a.qc->head, 1ull);
        __syncthreads();
        const int64_t k = s_k;
        if (k >= 2 * n) break;
        int p;
        int64_t blk;
        bool skip = false;
        const bool symbolic = k < n;
        if (symbolic) {
            int lo = 0, hi = a.count - 1;  // product of symbolic item k
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.item_off[mid] <= k) lo = mid;
                else hi = mid - 1;
            }
            p = lo;
            blk = k - a.item_off[p];
        } else {
            if (tid == 0) {
                // bounded wait (seconds of sleeps): a slot that never fills
                // (which the item counts rule out) ends as a skipped item and
                // raises the queue's failure flag, which ends every other wait
                int64_t e;
                int64_t spins = 0;
                while ((e = ld_dev(&a.queue[k - n])) == 0 && spins < QUEUE_SPIN_LIMIT) {
                    __builtin_amdgcn_s_sleep(2);
                    if ((++spins & 1023) == 0 && ld_dev(&a.qc->pad)) break;  // another wait gave up: so does this one
                }
                if (e == 0) {
                    atomicOr((unsigned long long*)&a.qc->pad, 1ull);
                    e = -1;  // product 0, block 0, skipped
                }
                s_e = e;
            }
            __syncthreads();
            int64_t e = s_e;
            skip = e < 0;
            e = (skip ? -e : e) - 1;
            p = (int)(e >> 32);
            blk = e & 0xffffffff;
        }
        if (tid == 0 && a.stamps) atomicMin((unsigned long long*)&a.stamps[2 * p], (unsigned long long)clock_now());
        const int64_t r0 = a.row_off[p], m = a.row_off[p + 1] - r0;
        const int64_t i0 = blk * a.rb, i1 = min<int64_t>(m, i0 + a.rb);
        if (symbolic) {
            for (int64_t i = i0 + gi; i < i1; i += QGROUPS) sym_row<T>(a, r0 + i, w);
        } else if (!skip) {
            const int32_t* crp = a.c_row_ptr + a.crp_off[p];
            for (int64_t i = i0 + gi; i < i1; i += QGROUPS) {
                const int32_t c0 = ld_dev(&crp[i]), c1 = ld_dev(&crp[i + 1]);
                num_row<T>(a, r0 + i, c0, c1 - c0, w);
            }
        }
        if (symbolic) wait_mem();  // the row sizes and bitmaps are out before the product's count drops
        __syncthreads();
        if (tid == 0) {
            s_last = 0;
            if (symbolic && atomicSub(&a.sym_left[p], 1) == 1) s_last = 1;
        }
        __syncthreads();
        if (s_last) finish_product<T>(a, p, red64, &s_flag);
        if (tid == 0 && a.stamps) atomicMax((unsigned long long*)&a.stamps[2 * p + 1], (unsigned long long)clock_now());
        __syncthreads();
    }
}

// Per run: counters, the products' symbolic item counts, the queue and the
// time stamps reset; products without rows finished at once.
__global__ void k_queue_init(QueueArgs a) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    if (g == 0) a.qc->head = 0, a.qc->tail = 0, a.qc->used = 0;
    for (int64_t q = g; q < a.n_items; q += stride) a.queue[q] = 0;
    for (int64_t p = g; p < a.count; p += stride) {
        a.sym_left[p] = (int32_t)(a.item_off[p + 1] - a.item_off[p]);
        if (a.stamps) a.stamps[2 * p] = INT64_MAX, a.stamps[2 * p + 1] = 0;
        if (a.row_off[p + 1] == a.row_off[p]) {
            a.c_offsets[p] = 0;
            a.c_row_ptr[a.crp_off[p]] = 0;
        }
    }
}

}  // namespace

size_t queue_lds_bytes(int wmax, int vmax, int elem_bytes) {
    return (size_t)QGROUPS * ((size_t)wmax * 8 + (size_t)vmax * elem_bytes + RG * (12 + elem_bytes));
}

void launch_queue(hipStream_t s, const QueueArgs& a, int elem_bytes, int grid) {
    hipLaunchKernelGGL(k_queue_init, dim3(256), dim3(256), 0, s, a);
    const size_t lds = queue_lds_bytes(a.wmax, a.vmax, elem_bytes);
    if (elem_bytes == 8) hipLaunchKernelGGL(k_queue<double>, dim3(grid), dim3(64 * QWAVES), lds, s, a);
    else hipLaunchKernelGGL(k_queue<float>, dim3(grid), dim3(64 * QWAVES), lds, s, a);
}

}  // namespace spg
