// Row accumulators of the symbolic and numeric phases (section 2.2.1).
//
// One group of G lanes owns one row of C.  Groups of up to 64 lanes live
// inside one wavefront (several rows per 256-lane workgroup, no workgroup
// barriers); groups of 128 and more lanes own a whole workgroup; the global
// path gives a row 1024 lanes.
//
// Work distribution (the flat product mapping, below): a chunk of up to G
// nonzeros of A's row is staged in LDS; their B rows are cut into groups of
// consecutive entries (their compressed-B rows into groups of runs) that
// are numbered in A order, and lane l takes groups l, l + G, ...: every lane
// busy, B read in coalesced 16-byte loads, all loads of a batch in flight
// together.  This is the paper's vector-parallel inner loop over a B row
// (section 2.2.1) flattened across the row's B rows.
//
// Tables (spg_internal.h): 32-column block masks, direct, hashed or two-level.
//   symbolic: OR each compressed-B run into the row's table; the value the
//             atomic OR returns says whether bits (and the block) are new, so
//             the row size and its occupied blocks are counted on the fly
//             (two-level: blocks are marked first, masks OR-ed in a second
//             pass); the occupied blocks then go out in ascending order as
//             the row's {block, mask} list;
//   numeric:  the list is read back, an exclusive prefix sum of its
//             popcounts places every block with its prefix (and writes the
//             row's columns), then every product is added with an LDS atomic
//             at its column's rank; the row leaves sorted, with coalesced
//             stores.
// Long rows use the global path: 1024 lanes per row, the mask table in LDS
// when it fits else in a per-workgroup global slab, values summed in LDS
// segments (or, for the longest rows, with global atomics straight into C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "spg_internal.h"

namespace spg {

namespace {

__device__ inline int hash_slot(int key, int logT) {
    return (int)(((uint32_t)key * 2654435761u) >> (32 - logT));
}

// Insert-or-find of a block id (open addressing, linear probing).  Returns the
// slot, or -1 when all T slots were probed without success.
__device__ inline int hash_insert(int32_t* keys, int T, int logT, int key, bool& inserted) {
    int h = hash_slot(key, logT);
    inserted = false;
    for (int probe = 0; probe < T; ++probe) {
        int cur = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == key) return h;
        if (cur == -1) {
            int old = atomicCAS(&keys[h], -1, key);
            if (old == -1) {
                inserted = true;
                return h;
            }
            if (old == key) return h;
        }
        h = (h + 1) & (T - 1);
    }
    return -1;
}

__device__ inline int hash_find(const int32_t* keys, int T, int logT, int key) {
    int h = hash_slot(key, logT);
    for (int probe = 0; probe < T; ++probe) {
        if (keys[h] == key) return h;
        h = (h + 1) & (T - 1);
    }
    return -1;
}

// Orders a workgroup's own global-memory accesses (its slab rows, the rows
// of C it writes): they stay within one compute unit, so workgroup scope is
// enough, and unlike an agent-scope fence it writes nothing back from L2.
__device__ inline void wg_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// bits below bit b of a 32-bit mask
__device__ inline uint32_t below(int b) { return (1u << b) - 1u; }

template <int G>
constexpr int rows_per_wg() {
    return G <= 64 ? 256 / G : 1;
}

// Orders LDS accesses among the lanes of one group.
template <int G>
__device__ inline void group_sync() {
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

// Inclusive sum over each aligned group of min(G, 64) lanes of a wavefront:
// DPP row shifts inside rows of 16 lanes, then broadcasts of lanes 15 and 31
// into the following rows.  No LDS traffic.
template <int G>
__device__ inline int wave_incl_scan(int x) {
    constexpr int S = G < 64 ? G : 64;
    const int l = threadIdx.x & (S - 1);
    if constexpr (S >= 2) {
        const int y = __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
        x += (S >= 16 || l >= 1) ? y : 0;
    }
    if constexpr (S >= 4) {
        const int y = __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
        x += (S >= 16 || l >= 2) ? y : 0;
    }
    if constexpr (S >= 8) {
        const int y = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
        x += (S >= 16 || l >= 4) ? y : 0;
    }
    if constexpr (S >= 16) x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    if constexpr (S >= 32) x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    if constexpr (S >= 64) x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Value held by the last lane of the lane's group of G <= 64 lanes.
template <int G>
__device__ inline int group_last(int x) {
    if constexpr (G >= 64) {
        return __builtin_amdgcn_readlane(x, 63);
    } else {
        const int g = (threadIdx.x & 63) / G;
        int r = 0;
#pragma unroll
        for (int t = 0; t < 64 / G; ++t) {
            const int v = __builtin_amdgcn_readlane(x, t * G + G - 1);
            r = g == t ? v : r;
        }
        return r;
    }
}

template <int G>
__device__ inline int group_sum(int v, int* red) {
    if constexpr (G <= 64) {
        return group_last<G>(wave_incl_scan<G>(v));
    } else {
        constexpr int W = G / 64;
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int t = __builtin_amdgcn_readlane(wave_incl_scan<64>(v), 63);
        __syncthreads();
        if (wl == 0) red[wv] = t;
        __syncthreads();
        int s = 0;
        for (int u = 0; u < W; ++u) s += red[u];
        return s;
    }
}

// Exclusive prefix sum over the G lanes of a group; total gets the sum.
template <int G>
__device__ inline int group_excl_scan(int v, int& total, int* red) {
    const int x = wave_incl_scan<G>(v);
    if constexpr (G <= 64) {
        total = group_last<G>(x);
        return x - v;
    } else {
        constexpr int W = G / 64;
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (wl == 63) red[wv] = x;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int u = 0; u < W; ++u) {
            int t = red[u];
            if (u < wv) pre += t;
            tot += t;
        }
        total = tot;
        return pre + x - v;
    }
}

// ------------------------------------------------------- flat product mapping
// The row kernels stage a chunk of up to G nonzeros of A's row and number
// the products of the chunk 0..P-1 in A order (entry e's B row takes products
// pb_e .. pb_e + len_e - 1).  A batch hands lane l the products
// P0 + l + G*k, k < K: every lane busy, consecutive lanes on consecutive
// entries of one B row (coalesced), and all K loads of a lane issued at once.
// The entry owning product p comes from a window table: per window of G
// products (and per wavefront of the group) a mask of the positions where a
// staged entry's products begin and the number of entries begun earlier, so
//     entry(p) = cum + popcount(mask & lanes_at_or_below) - 1.
// Compressed-B runs are numbered and handed out the same way.

struct Win {
    unsigned long long mask;
    int cum;
    int pad;
};

template <int G>
constexpr int waves_of() {
    return G > 64 ? G / 64 : 1;
}

// Workgroups are dispatched in order, round-robin over the 8 XCDs; renumber
// them so that each XCD takes runs of `span` consecutive slots (its L2 then
// holds the B rows that neighbouring rows share) while the 8 XCDs work on
// neighbouring runs at any time: rows are grouped in ascending row order,
// and where row sizes drift along it (R-MAT's heavy rows have low indices)
// one contiguous share per XCD would leave the first XCD with the heaviest
// rows and the others waiting.  Workgroups of 256 lanes or more hold one
// long row each: they keep the dispatch order (span 1), which balances
// best; shorter rows take runs of 64 workgroups (measured: 27-point
// stencil numeric 1.06 ms against 1.10 with span 1 and 1.13 with one share
// per XCD; R-MAT's 1024-lane symbolic rows 4.5 ms with span 1, 4.9 with 64,
// 9.3 with one share per XCD).  A bijection of [0, nblk): whole rounds of 8
// runs are renumbered, the remainder is left in dispatch order.
template <int G>
__device__ inline int xcd_block(int b, int nblk) {
    constexpr int NXCD = 8;
    constexpr int span = G >= 256 ? 1 : 64;
    if constexpr (span == 1) return b;
    const int full = nblk / (NXCD * span) * (NXCD * span);
    if (b >= full) return b;
    const int x = b % NXCD, k = b / NXCD;
    return ((k / span) * NXCD + x) * span + k % span;
}

template <int G>
__device__ inline int3 group_excl_scan3(int3 v, int3& total, int* red) {
    const int3 x = make_int3(wave_incl_scan<G>(v.x), wave_incl_scan<G>(v.y), wave_incl_scan<G>(v.z));
    if constexpr (G <= 64) {
        total = make_int3(group_last<G>(x.x), group_last<G>(x.y), group_last<G>(x.z));
        return make_int3(x.x - v.x, x.y - v.y, x.z - v.z);
    } else {
        constexpr int W = G / 64;
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (wl == 63) red[3 * wv] = x.x, red[3 * wv + 1] = x.y, red[3 * wv + 2] = x.z;
        __syncthreads();
        int3 pre = make_int3(0, 0, 0), tot = make_int3(0, 0, 0);
        for (int u = 0; u < W; ++u) {
            const int3 t = make_int3(red[3 * u], red[3 * u + 1], red[3 * u + 2]);
            if (u < wv) pre.x += t.x, pre.y += t.y, pre.z += t.z;
            tot.x += t.x, tot.y += t.y, tot.z += t.z;
        }
        total = tot;
        return make_int3(pre.x + x.x - v.x, pre.y + x.y - v.y, pre.z + x.z - v.z);
    }
}

template <int G>
__device__ inline int2 group_excl_scan2(int2 v, int2& total, int* red) {
    const int2 x = make_int2(wave_incl_scan<G>(v.x), wave_incl_scan<G>(v.y));
    if constexpr (G <= 64) {
        total = make_int2(group_last<G>(x.x), group_last<G>(x.y));
        return make_int2(x.x - v.x, x.y - v.y);
    } else {
        constexpr int W = G / 64;
        const int wl = threadIdx.x & 63, wv = threadIdx.x >> 6;
        __syncthreads();
        if (wl == 63) red[2 * wv] = x.x, red[2 * wv + 1] = x.y;
        __syncthreads();
        int2 pre = make_int2(0, 0), tot = make_int2(0, 0);
        for (int u = 0; u < W; ++u) {
            const int2 t = make_int2(red[2 * u], red[2 * u + 1]);
            if (u < wv) pre.x += t.x, pre.y += t.y;
            tot.x += t.x, tot.y += t.y;
        }
        total = tot;
        return make_int2(pre.x + x.x - v.x, pre.y + x.y - v.y);
    }
}

// Sets the start bit of a staged entry whose first product p0 falls in the
// batch [P0, P0 + K*G).
template <int G, int K>
__device__ inline void win_mark(Win* win, bool ne, int p0, int P0) {
    constexpr int W = waves_of<G>();
    const int d = p0 - P0;
    if (ne && d >= 0 && d < K * G) {
        const int dl = d % G;
        atomicOr(&win[(d / G) * W + (dl >> 6)].mask, 1ull << (dl & 63));
    }
}

// Fills the cum fields of two window tables (KA and KB windows) from their
// masks: exclusive prefix of popcounts in order, plus the entries begun
// before each batch (before_a, before_b).  Both counts stay below 2^16.
template <int G, int KA, int KB>
__device__ inline void win_scan(Win* wa, Win* wb, int before_a, int before_b, int lane, int* red) {
    constexpr int W = waves_of<G>();
    constexpr int NA = KA * W, NB = KB * W;
    constexpr int CA = (NA + G - 1) / G, CB = (NB + G - 1) / G;
    if constexpr (G > 64 && NB == 0 && NA <= 256) {
        // a few window entries per lane of one wavefront: the group's first
        // wavefront scans them (no workgroup barrier; the caller synchronises
        // after)
        constexpr int C1 = (NA + 63) / 64;
        if (threadIdx.x < 64) {
            int local = 0;
#pragma unroll
            for (int t = 0; t < C1; ++t)
                if (lane * C1 + t < NA) local += __popcll(wa[lane * C1 + t].mask);
            int ca = before_a + wave_incl_scan<64>(local) - local;
#pragma unroll
            for (int t = 0; t < C1; ++t)
                if (lane * C1 + t < NA) {
                    wa[lane * C1 + t].cum = ca;
                    ca += __popcll(wa[lane * C1 + t].mask);
                }
        }
        return;
    }
    int local = 0;
#pragma unroll
    for (int t = 0; t < CA; ++t)
        if (lane * CA + t < NA) local += __popcll(wa[lane * CA + t].mask);
#pragma unroll
    for (int t = 0; t < CB; ++t)
        if (lane * CB + t < NB) local += __popcll(wb[lane * CB + t].mask) << 16;
    int total;
    const int ex = group_excl_scan<G>(local, total, red);
    int ca = before_a + (ex & 0xffff), cb = before_b + (ex >> 16);
#pragma unroll
    for (int t = 0; t < CA; ++t)
        if (lane * CA + t < NA) {
            wa[lane * CA + t].cum = ca;
            ca += __popcll(wa[lane * CA + t].mask);
        }
#pragma unroll
    for (int t = 0; t < CB; ++t)
        if (lane * CB + t < NB) {
            wb[lane * CB + t].cum = cb;
            cb += __popcll(wb[lane * CB + t].mask);
        }
}

template <int G, int K>
__device__ inline void win_clear(Win* win, int lane) {
    constexpr int NW = K * waves_of<G>();
    for (int t = lane; t < NW; t += G) win[t] = Win{0ull, 0, 0};
}

// Staged entry of the lane's product in window k of the batch.  Groups of
// 64 lanes or more read a batch's window words once (lane t of a wavefront
// holds window t of its column) and broadcast them with readlane, so a slot
// costs no LDS access; smaller groups read the word from LDS.
template <int G, int K>
struct WinView {
    unsigned long long m;
    int c;
    const Win* win;
    __device__ inline void load(const Win* w, int wv) {
        win = w;
        if constexpr (G >= 64) {
            const int t = threadIdx.x & 63;
            m = 0, c = 0;
            if (t < K) {
                const Win x = w[t * waves_of<G>() + wv];
                m = x.mask, c = x.cum;
            }
        }
    }
    __device__ inline int entry(int k, int wv, unsigned long long le) const {
        if constexpr (G >= 64) {
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)m, k);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(m >> 32), k);
            const int cum = __builtin_amdgcn_readlane(c, k);
            return cum + __popcll((((unsigned long long)hi << 32) | lo) & le) - 1;
        } else {
            const Win w = win[k];
            return w.cum + __popcll(w.mask & le) - 1;
        }
    }
};

// Groups: V consecutive entries of one B row (or runs of one compressed-B
// row) from index q, the first n = min(V, end - q) of them valid, read with
// one 16-byte load per array (dword-aligned: 16-byte loads need only that on
// this target) unless the group would reach past the array's end.
struct __attribute__((packed, aligned(4))) U4 {
    int x, y, z, w;
};
struct __attribute__((packed, aligned(8))) D2 {
    double x, y;
};
struct __attribute__((packed, aligned(4))) F4 {
    float x, y, z, w;
};

template <typename T>
struct ColVal {
    int c;
    T y;
};

template <int V_>
struct RunGroup {  // V = 1 or 2
    static constexpr int V = V_;
    int2 r[V];
    int n;
    __device__ inline int2 at(int j) const { return r[j]; }
};

template <typename T>
struct BGroup {  // FLAT_VB == 4
    static constexpr int V = 4;
    int c[4];
    T y[4];
    int n;
    __device__ inline ColVal<T> at(int j) const { return ColVal<T>{c[j], y[j]}; }
};

template <int V>
__device__ inline RunGroup<V> load_runs(const int2* __restrict__ bc, int64_t total, int q, int end) {
    RunGroup<V> g;
    g.n = min(V, end - q);
    if constexpr (V == 1) {
        g.r[0] = bc[q];
    } else if (q + 2 <= total) {
        const U4 v = *reinterpret_cast<const U4*>(bc + q);
        g.r[0] = make_int2(v.x, v.y);
        g.r[1] = make_int2(v.z, v.w);
    } else {  // the array's last run: n == 1
        g.r[0] = bc[q];
        g.r[1] = make_int2(0, 0);
    }
    return g;
}

template <typename T>
__device__ inline BGroup<T> load_b(const int32_t* __restrict__ bci, const T* __restrict__ bv, int64_t total, int q,
                                   int end) {
    BGroup<T> g;
    g.n = min(4, end - q);
    if (q + 4 <= total) {
        const U4 c = *reinterpret_cast<const U4*>(bci + q);
        g.c[0] = c.x, g.c[1] = c.y, g.c[2] = c.z, g.c[3] = c.w;
        if constexpr (sizeof(T) == 8) {
            const D2 v0 = *reinterpret_cast<const D2*>(bv + q);
            const D2 v1 = *reinterpret_cast<const D2*>(bv + q + 2);
            g.y[0] = v0.x, g.y[1] = v0.y, g.y[2] = v1.x, g.y[3] = v1.y;
        } else {
            const F4 v = *reinterpret_cast<const F4*>(bv + q);
            g.y[0] = v.x, g.y[1] = v.y, g.y[2] = v.z, g.y[3] = v.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            g.c[j] = 0, g.y[j] = T(0);
            if (j < g.n) g.c[j] = bci[q + j], g.y[j] = bv[q + j];
        }
    }
    return g;
}

// One batch: issue the K group loads of the lane (slot k holds group
// P0 + lane + G*k when below P; off[e] = {start - V * first group, end} of
// staged entry e turns it into an index), then hand each group to
// apply(group, entry).
template <int G, int K, int V, typename Load>
struct Batch {
    using R = decltype(std::declval<Load>()(0, 0));
    R v[K];
    WinView<G, K> view;
    // Every staged offset is read before the first load goes out, and no
    // load of an earlier batch is still in flight here (the caller consumed
    // it): the explicit wait tells the compiler so, which otherwise orders
    // the K loads one after another behind waits for registers that the
    // previous batch's loads wrote.
    __device__ inline void issue(const int2* off, const Win* win, int P0, int P, int lane, int wv,
                                 unsigned long long le, Load& load) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        view.load(win, wv);
        int2 o[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            o[k] = make_int2(0, 0);
            if (P0 + k * G + lane < P) o[k] = off[view.entry(k, wv, le)];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int g = P0 + k * G + lane;
            if (g < P) v[k] = load(o[k].x + V * g, o[k].y);
        }
    }
    // the entry is found again here rather than held in a register across the
    // wait (the window table is unchanged until then)
    template <typename Apply>
    __device__ inline void consume(int P0, int P, int lane, int wv, unsigned long long le, Apply&& apply) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (P0 + k * G + lane < P) apply(v[k], view.entry(k, wv, le));
    }
    // every lane, with whether its slot holds a group (for cross-lane work)
    template <typename F>
    __device__ inline void consume_all(int P0, int P, int lane, F&& f) {
#pragma unroll
        for (int k = 0; k < K; ++k) f(v[k], P0 + k * G + lane < P);
    }
};

// ORs `bits` into l1[key].x; lanes next to each other in one group that hold
// the same key are OR-ed together first (a segmented OR over each aligned
// run of 16 lanes with DPP row shifts; segments also start at every group's
// first lane), and one lane per segment does the LDS atomic, which saves the
// atomics' serialisation on one address.  key < 0: nothing.
template <int G>
__device__ inline void or_word_merged(uint2* l1, int key, uint32_t bits) {
    const int l16 = threadIdx.x & 15, lg = threadIdx.x % G;
    const int kp = __builtin_amdgcn_mov_dpp(key, 0x111, 0xf, 0xf, false);  // row_shr:1
    const int kn = __builtin_amdgcn_mov_dpp(key, 0x101, 0xf, 0xf, false);  // row_shl:1
    int f = l16 == 0 || lg == 0 || kp != key;
    uint32_t m = bits;
    const auto step = [&](uint32_t mu, int fu, int d) {
        if (l16 >= d && !f) {
            m |= mu;
            f = fu;
        }
    };
    step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x111, 0xf, 0xf, false),
         __builtin_amdgcn_mov_dpp(f, 0x111, 0xf, 0xf, false), 1);  // row_shr:1
    step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x112, 0xf, 0xf, false),
         __builtin_amdgcn_mov_dpp(f, 0x112, 0xf, 0xf, false), 2);  // row_shr:2
    step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x114, 0xf, 0xf, false),
         __builtin_amdgcn_mov_dpp(f, 0x114, 0xf, 0xf, false), 4);  // row_shr:4
    step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x118, 0xf, 0xf, false),
         __builtin_amdgcn_mov_dpp(f, 0x118, 0xf, 0xf, false), 8);  // row_shr:8
    const bool last = l16 == 15 || lg == G - 1 || kn != key;
    if (last && key >= 0) atomicOr(&l1[key].x, m);
}

// Turns apply(element, entry) into apply(group, entry) over the valid elements.
template <typename F>
__device__ inline auto each(F& f) {
    return [&f](const auto& g, int e) {
#pragma unroll
        for (int j = 0; j < std::decay_t<decltype(g)>::V; ++j)
            if (j < g.n) f(g.at(j), e);
    };
}

// Walks the B groups (RUNS false) or compressed-B run groups (RUNS true) of
// A's row [a0, a1) in the flat mapping, for any row length: chunks of G staged
// entries (off[e] = {start - V * first group, end}, and A's value in ava when
// walking B), batches of K groups per lane.  apply(group, entry) sees every
// group once.  Used by the global path, whose rows are long.
// hdr(j) gives the {first entry, length} of the piece of B row (or
// compressed-B row) j that the walk covers.
// One staged chunk of the walk: the lane's entry (if `has`) covers the piece
// {first, length} = h of a B row with A value v.  The caller has cleared the
// window table and synchronised the group.
// extra: a value of the caller's scanned in the same pass, its exclusive
// prefix and total returned in *extra_scan.
template <int G, int K, int V, bool RUNS, typename T, typename Load, typename Apply>
__device__ inline void walk_chunk(int2 h, T v, int2* off, T* ava, Win* win, int* red, Load& load, Apply&& apply,
                                  int extra = 0, int2* extra_scan = nullptr) {
    const int lane = threadIdx.x % G, wv = lane >> 6;
    const unsigned long long le = (2ull << (lane & 63)) - 1;
    const int start = h.x, len = h.y;
    const bool ne = len > 0;
    int3 tot;
    const int3 ex = group_excl_scan3<G>(make_int3(ne, (len + V - 1) / V, extra), tot, red);
    if (extra_scan) *extra_scan = make_int2(ex.z, tot.z);
    const int P = tot.y;
    if (ne) {
        off[ex.x] = make_int2(start - V * ex.y, start + len);
        if constexpr (!RUNS) ava[ex.x] = v;
    }
    group_sync<G>();
    for (int P0 = 0; P0 < P; P0 += K * G) {
        if (P0 > 0) {
            group_sync<G>();
            win_clear<G, K>(win, lane);
            group_sync<G>();
        }
        win_mark<G, K>(win, ne, ex.y, P0);
        const int before = P0 > 0 ? group_sum<G>(ne && ex.y < P0, red) : 0;
        group_sync<G>();
        win_scan<G, K, 0>(win, nullptr, before, 0, lane, red);
        group_sync<G>();
        Batch<G, K, V, Load> bt;
        bt.issue(off, win, P0, P, lane, wv, le, load);
        bt.consume(P0, P, lane, wv, le, apply);
    }
}

// hdr(j) gives the {first entry, length} of the piece of B row (or
// compressed-B row) j that the walk covers.
template <int G, int K, int V, bool RUNS, typename T, typename Hdr, typename Load, typename Apply>
__device__ void flat_walk_hdr(const int32_t* __restrict__ aci, Hdr&& hdr, const T* __restrict__ av, int a0, int a1,
                              int2* off, T* ava, Win* win, int* red, Load& load, Apply&& apply) {
    const int lane = threadIdx.x % G;
    for (int e0 = a0; e0 < a1; e0 += G) {
        group_sync<G>();  // the previous chunk's readers are done
        win_clear<G, K>(win, lane);
        int2 h = make_int2(0, 0);
        T v = T(0);
        if (lane < a1 - e0) {
            h = hdr(aci[e0 + lane]);
            if constexpr (!RUNS) v = av[e0 + lane];
        }
        walk_chunk<G, K, V, RUNS, T>(h, v, off, ava, win, red, load, apply);
    }
    group_sync<G>();
}

// The walk over whole B rows (RUNS false) or compressed-B rows (RUNS true).
template <int G, int K, int V, bool RUNS, typename T, typename Load, typename Apply>
__device__ void flat_walk(const int32_t* __restrict__ aci, const int4* __restrict__ bhdr, const T* __restrict__ av,
                          int a0, int a1, int2* off, T* ava, Win* win, int* red, Load& load, Apply&& apply) {
    auto hdr = [&](int j) {
        const int4 h = bhdr[j];
        return RUNS ? make_int2(h.z, h.w) : make_int2(h.x, h.y);
    };
    flat_walk_hdr<G, K, V, RUNS, T>(aci, hdr, av, a0, a1, off, ava, win, red, load, static_cast<Apply&&>(apply));
}

// ------------------------------------------------------------------ symbolic
// Every entry of compressed B is a {block, mask} run: the row's table gets
// the mask OR-ed in, and the bits that were not yet set (and blocks that were
// empty) are counted from the value the atomic OR returns.

// One row of the symbolic phase in a table of MODE in the row's LDS share
// (d = the slot's descriptor {row, A start, A end, list offset}).
template <int G, int MODE>
__device__ __forceinline__ void sym_row(const SymArgs& a, const int4 d, const int sub, uint32_t* smem, int* red,
                                        int* occ, int* ovf) {
    constexpr int KC = FLAT_KC;
    constexpr int VC = FLAT_VC_SYM;
    const int bytes = tier_bytes(a.tier);
    const int per_row = bytes + sym_stage_bytes(G);
    const int lane = threadIdx.x % G, wv = lane >> 6;
    const unsigned long long le = (2ull << (lane & 63)) - 1;
    const int i = d.x, a0 = d.y, a1 = d.z;
    // the first chunk's B headers are gathered before the table is cleared
    int4 h0 = make_int4(0, 0, 0, 0);
    if (lane < a1 - a0) h0 = a.bhdr[a.aci[a0 + lane]];
    uint8_t* row_lds = reinterpret_cast<uint8_t*>(smem) + (size_t)sub * per_row;
    uint32_t* tab = reinterpret_cast<uint32_t*>(row_lds);
    int2* cq = reinterpret_cast<int2*>(row_lds + bytes);   // staged run {offset, end}
    Win* win = reinterpret_cast<Win*>(row_lds + bytes + 8 * G);
    // direct: a mask per word of the row's range.  hashed: keys, then masks.
    // two-level: {bits, prefix} per 32 words, then per occupied block a mask,
    // then per occupied block its id (for the row's list; 16-bit offsets from
    // the first block when the range allows).
    int base = 0, ncell = 0, T = 0, logT = 0, w1 = 0, cap = 0;
    int32_t* keys = reinterpret_cast<int32_t*>(tab);
    uint32_t* masks = tab;
    uint2* l1 = reinterpret_cast<uint2*>(tab);
    uint32_t* cm = tab;
    int32_t* cb = nullptr;
    uint16_t* cb16 = nullptr;
    bool short_ids = false;
    if constexpr (MODE != MODE_HASHED) {
        const RowInfo ri = a.rinfo[i];
        base = ri.x >> 5;
        ncell = (ri.y >> 5) - base + 1;
    }
    if constexpr (MODE == MODE_HASHED) {
        T = 1 << (31 - __clz(bytes / 8));
        logT = 31 - __clz(T);
        masks = tab + T;
        ncell = T;
    } else if constexpr (MODE == MODE_TWOLEVEL) {
        w1 = (ncell + 31) >> 5;
        cm = reinterpret_cast<uint32_t*>(l1 + w1);
        cap = (bytes - w1 * 8) / sym_block_bytes(ncell);
        short_ids = sym_block_bytes(ncell) == 6;
        cb = reinterpret_cast<int32_t*>(cm + cap);
        cb16 = reinterpret_cast<uint16_t*>(cm + cap);
    }
    // 16-byte clears (tables start 256-byte aligned and tiers are multiples of 16 bytes)
    if constexpr (MODE == MODE_DIRECT) {
        for (int c = 4 * lane; c < ncell; c += 4 * G) *reinterpret_cast<uint4*>(&masks[c]) = make_uint4(0, 0, 0, 0);
    } else if constexpr (MODE == MODE_HASHED) {
        for (int c = 4 * lane; c < ncell; c += 4 * G) {
            *reinterpret_cast<int4*>(&keys[c]) = make_int4(-1, -1, -1, -1);
            *reinterpret_cast<uint4*>(&masks[c]) = make_uint4(0, 0, 0, 0);
        }
    } else {
        for (int c = lane; c < w1; c += G) l1[c] = make_uint2(0u, 0u);
    }
    win_clear<G, KC>(win, lane);
    if (lane == 0) occ[sub] = 0, ovf[sub] = 0;
    group_sync<G>();

    // ---- staging: chunks of G entries of A's row, one window table of run groups
    int pc = 0, PC = 0;
    bool ne = false;
    int staged = -1, wc0 = 0;
    // h: the lane's B header in chunk e0 (window table cleared and
    // synchronised by the caller)
    auto stage = [&](int e0, int4 h) {
        ne = h.w > 0;
        int3 tot;
        const int3 ex = group_excl_scan3<G>(make_int3(ne, (h.w + VC - 1) / VC, 0), tot, red);
        pc = ex.y, PC = tot.y;
        if (ne) cq[ex.x] = make_int2(h.z - VC * ex.y, h.z + h.w);
        win_mark<G, KC>(win, ne, pc, 0);
        group_sync<G>();
        win_scan<G, KC, 0>(win, nullptr, 0, 0, lane, red);
        group_sync<G>();
        staged = e0, wc0 = 0;
    };
    auto restage = [&](int e0) {
        if (staged == e0) return;
        int4 h = make_int4(0, 0, 0, 0);
        if (lane < a1 - e0) h = a.bhdr[a.aci[e0 + lane]];
        group_sync<G>();
        win_clear<G, KC>(win, lane);
        group_sync<G>();
        stage(e0, h);
    };
    auto rewin = [&](int P0) {
        if (wc0 == P0) return;
        group_sync<G>();
        win_clear<G, KC>(win, lane);
        group_sync<G>();
        win_mark<G, KC>(win, ne, pc, P0);
        const int before = group_sum<G>(ne && pc < P0, red);
        group_sync<G>();
        win_scan<G, KC, 0>(win, nullptr, before, 0, lane, red);
        group_sync<G>();
        wc0 = P0;
    };
    auto load_run = [&](int q, int end) { return load_runs<VC>(a.bc, a.bc_total, q, end); };
    auto walk_runs = [&](auto&& apply) {
        for (int e0 = a0; e0 < a1; e0 += G) {
            restage(e0);
            for (int P0 = 0; P0 < PC; P0 += KC * G) {
                rewin(P0);
                Batch<G, KC, VC, decltype(load_run)> bt;
                bt.issue(cq, win, P0, PC, lane, wv, le, load_run);
                bt.consume(P0, PC, lane, wv, le, apply);
            }
        }
    };
    auto walk_runs_all = [&](auto&& f) {
        for (int e0 = a0; e0 < a1; e0 += G) {
            restage(e0);
            for (int P0 = 0; P0 < PC; P0 += KC * G) {
                rewin(P0);
                Batch<G, KC, VC, decltype(load_run)> bt;
                bt.issue(cq, win, P0, PC, lane, wv, le, load_run);
                bt.consume_all(P0, PC, lane, f);
            }
        }
    };

    int cnt = 0, nb = 0;
    // runs(apply): apply(run, entry) on every run; runs_all(f): f(group,
    // valid) on every lane of every batch
    auto finish = [&](auto&& runs, auto&& runs_all) {
        if constexpr (MODE == MODE_TWOLEVEL) {
            // pass A: occupied blocks; their count and compact indices from a
            // prefix of popcounts; pass B: masks OR-ed in at the compact index.
            // Neighbouring lanes mostly mark blocks of one word (a B row's runs
            // in one plane of a stencil): their bits are merged first.
            auto mark = [&](const auto& g, bool valid) {
                const int w = g.r[0].x - base;
                or_word_merged<G>(l1, valid ? w >> 5 : -1, valid ? 1u << (w & 31) : 0u);
            };
            runs_all(mark);
            group_sync<G>();
            {
                const int chunk = (w1 + G - 1) / G;
                const int beg = lane * chunk;
                const int end = min(beg + chunk, w1);
                int local = 0;
                for (int t = beg; t < end; ++t) local += __popc(l1[t].x);
                int total;
                int ex = group_excl_scan<G>(local, total, red);
                for (int t = beg; t < end; ++t) {
                    l1[t].y = (uint32_t)ex;
                    ex += __popc(l1[t].x);
                }
                nb = total;
            }
            if (nb > cap) {  // (only under a learned estimate) the row is retried exactly
                if (lane == 0) ovf[sub] = 1;
                return;
            }
            for (int c = lane; c < nb; c += G) cm[c] = 0u;
            group_sync<G>();
            auto orc = [&](int2 run, int) {
                const int w = run.x - base;
                const uint2 L = l1[w >> 5];
                const uint32_t bits = (uint32_t)run.y;
                const int ci = (int)L.y + __popc(L.x & below(w & 31));
                atomicOr(&cm[ci], bits);  // the row size is counted from the final masks
                // every run of the block stores the same id
                if (short_ids) cb16[ci] = (uint16_t)w;
                else cb[ci] = run.x;
            };
            runs(each(orc));
        } else {
            const int occ_max = (T * 3) / 4;
            auto apply = [&](int2 run, int) {
                const uint32_t bits = (uint32_t)run.y;
                int cell;
                if constexpr (MODE == MODE_DIRECT) {
                    cell = run.x - base;
                } else {
                    if (*(volatile int*)&ovf[sub]) return;
                    bool ins;
                    cell = hash_insert(keys, T, logT, run.x, ins);
                    if (cell < 0) {
                        ovf[sub] = 1;
                        return;
                    }
                    if (ins && atomicAdd(&occ[sub], 1) >= occ_max) ovf[sub] = 1;
                }
                const uint32_t old = atomicOr(&masks[cell], bits);
                cnt += __popc(bits & ~old);
                nb += old == 0;
            };
            runs(each(apply));
        }
    };

    stage(a0, h0);
    if (a1 - a0 <= G && PC <= KC * G) {
        // the whole row in one batch: its runs stay in registers for every pass
        Batch<G, KC, VC, decltype(load_run)> br;
        br.issue(cq, win, 0, PC, lane, wv, le, load_run);
        finish([&](auto&& apply) { br.consume(0, PC, lane, wv, le, apply); },
               [&](auto&& f) { br.consume_all(0, PC, lane, f); });
    } else {
        finish(walk_runs, walk_runs_all);
    }
    if constexpr (MODE != MODE_TWOLEVEL) {
        cnt = group_sum<G>(cnt, red);
        nb = group_sum<G>(nb, red);
    }
    group_sync<G>();
    // the row's list: its occupied blocks in ascending order with their masks
    const int lo = d.w;
    const bool overflowed = MODE != MODE_DIRECT && ovf[sub];
    if constexpr (MODE == MODE_TWOLEVEL) {
        // the row size from the final masks; compact indices are in block
        // order, so the list is one coalesced store per block
        if (!overflowed) {
            for (int t = lane; t < nb; t += G) {
                const uint32_t mk = cm[t];
                cnt += __popc(mk);
                if (lo >= 0) a.lists[lo + t] = make_int2(short_ids ? base + (int)cb16[t] : cb[t], (int)mk);
            }
        }
        cnt = group_sum<G>(cnt, red);
    }
    if (MODE != MODE_TWOLEVEL && lo >= 0 && !overflowed) {
        int2* out = a.lists + lo;
        if constexpr (MODE == MODE_DIRECT) {
            const int chunk = (ncell + G - 1) / G;
            const int beg = min(lane * chunk, ncell);
            const int end = min(beg + chunk, ncell);
            int local = 0;
            for (int t = beg; t < end; ++t) local += masks[t] != 0;
            int total;
            int pos = group_excl_scan<G>(local, total, red);
            for (int t = beg; t < end; ++t) {
                const uint32_t mk = masks[t];
                if (mk) out[pos++] = make_int2(base + t, (int)mk);
            }
        } else {
            // position of an occupied slot = occupied slots with a smaller block
            // id (empty slots hold -1, the largest unsigned key)
            const int4* k4 = reinterpret_cast<const int4*>(keys);
            for (int c = lane; c < T; c += G) {
                const int key = keys[c];
                if (key < 0) continue;
                int r = 0;
                for (int f = 0; f < T / 4; ++f) {
                    const int4 q = k4[f];
                    r += ((uint32_t)q.x < (uint32_t)key) + ((uint32_t)q.y < (uint32_t)key) +
                         ((uint32_t)q.z < (uint32_t)key) + ((uint32_t)q.w < (uint32_t)key);
                }
                out[r] = make_int2(key, (int)masks[c]);
            }
        }
    }
    if (lane == 0) {
        if (MODE != MODE_DIRECT && ovf[sub]) {
            // queued for the exact retry; a table sized from an upper bound
            // (no retry list) cannot overflow, so that would be an internal error
            if (a.ovf_list) {
                const int pos = atomicAdd(&a.ctl->overflow_rows, 1);
                a.ovf_list[pos] = i;
            } else {
                atomicOr(&a.ctl->err, ERR_TABLE_OVERFLOW);
            }
        } else {
            a.row_nnz[i] = cnt;
            a.row_blocks[i] = nb;
        }
    }
}

// The symbolic rows of one LDS tier, all three table modes (the grouping
// kernel placed them tier-major, one range of slots per mode; its control
// block gives the ranges).  Persistent: each mode's row groups of RPW slots
// are cut into 8 contiguous shares, one per XCD (workgroups are dispatched
// round-robin over the XCDs, so workgroup b runs on XCD b % 8), and the
// workgroups of an XCD take its share's groups in turn; neighbouring rows
// share most of their B rows, which then stay in that XCD's L2.  The modes
// run one after another, each in a loop of its own, so that each keeps the
// register budget of its own table code.
template <int G, int MODE>
__device__ __forceinline__ void sym_tier_mode(const SymArgs& a, const int first, const int total, const int sub,
                                              uint32_t* smem, int* red, int* occ, int* ovf) {
    constexpr int RPW = rows_per_wg<G>();
    constexpr int NXCD = 8;
    const int groups = (total + RPW - 1) / RPW;
    const int per = (groups + NXCD - 1) / NXCD;
    const int x = blockIdx.x % NXCD, nw = gridDim.x / NXCD;
    const int hi = min(groups, (x + 1) * per);
    for (int g = x * per + (int)blockIdx.x / NXCD; g < hi; g += nw) {
        const int k = g * RPW + sub;
        if (k >= total) break;  // uniform in the group (in the workgroup when G >= 128)
        group_sync<G>();        // the previous row's readers are done with the table
        sym_row<G, MODE>(a, a.desc[first + k], sub, smem, red, occ, ovf);
    }
}

template <int G>
// (up to 128 lanes per row the symbolic kernel fits 64 VGPRs: full occupancy)
__global__ __launch_bounds__(G * rows_per_wg<G>()) __attribute__((amdgpu_waves_per_eu(G <= 128 ? 8 : 4)))
void k_sym_tier(SymArgs a) {
    constexpr int RPW = rows_per_wg<G>();
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[48];
    __shared__ int occ[RPW];
    __shared__ int ovf[RPW];
    if (a.ctl->err & ERR_INPUT) return;
    const int t = a.tier;
    // a group of 64 or more lanes owns whole wavefronts: its row is wave-uniform
    const int sub = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
    const int c0 = MODE_DIRECT * NTIER + t, c1 = MODE_HASHED * NTIER + t, c2 = MODE_TWOLEVEL * NTIER + t;
    if (a.ctl->sym_cnt[c0]) sym_tier_mode<G, MODE_DIRECT>(a, a.ctl->sym_off[c0], a.ctl->sym_cnt[c0], sub, smem, red, occ, ovf);
    if (a.ctl->sym_cnt[c1]) {
        group_sync<G>();
        sym_tier_mode<G, MODE_HASHED>(a, a.ctl->sym_off[c1], a.ctl->sym_cnt[c1], sub, smem, red, occ, ovf);
    }
    if (a.ctl->sym_cnt[c2]) {
        group_sync<G>();
        sym_tier_mode<G, MODE_TWOLEVEL>(a, a.ctl->sym_off[c2], a.ctl->sym_cnt[c2], sub, smem, red, occ, ovf);
    }
}

// One launch per symbolic class, sized on the host from the class histogram
// (a.desc and a.count are the class's range): a workgroup per RPW rows.
template <int G, int MODE>
// (up to 128 lanes per row the symbolic kernel fits 64 VGPRs: full occupancy)
__global__ __launch_bounds__(G * rows_per_wg<G>()) __attribute__((amdgpu_waves_per_eu(G <= 128 ? 8 : 4)))
void k_sym(SymArgs a) {
    constexpr int RPW = rows_per_wg<G>();
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[48];
    __shared__ int occ[RPW];
    __shared__ int ovf[RPW];
    // a group of 64 or more lanes owns whole wavefronts: its row is wave-uniform
    const int sub = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
    const int slot = xcd_block<G>(blockIdx.x, gridDim.x) * RPW + sub;
    if (slot >= a.count) return;  // uniform in the group (in the workgroup when G >= 128)
    sym_row<G, MODE>(a, a.desc[slot], sub, smem, red, occ, ovf);
}

template <bool IN_LDS>
__device__ inline uint32_t ld_tab(const uint32_t* p) {
    if constexpr (IN_LDS) return *p;
    else return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool IN_LDS>
__device__ void wide_sym_row(const SymArgs& a, int i, uint32_t* masks, int2* off, Win* win, int* red) {
    constexpr int G = WIDE_THREADS;
    const int tid = threadIdx.x;
    const RowInfo ri = a.rinfo[i];
    const int base = ri.x >> 5;
    const int words = (ri.y >> 5) - base + 1;
    for (int c = tid; c < words; c += G) masks[c] = 0;
    if (!IN_LDS) wg_fence();
    __syncthreads();
    int cnt = 0, nb = 0;
    auto load_run = [&](int q, int end) { return load_runs<FLAT_VC_SYM>(a.bc, a.bc_total, q, end); };
    auto orb = [&](int2 run, int) {
        const uint32_t old = atomicOr(&masks[run.x - base], (uint32_t)run.y);
        cnt += __popc((uint32_t)run.y & ~old);
        nb += old == 0;
    };
    flat_walk<G, FLAT_KC, FLAT_VC_SYM, true, int>(a.aci, a.bhdr, nullptr, a.arp[i], a.arp[i + 1], off, nullptr, win,
                                                  red, load_run, each(orb));
    cnt = group_sum<G>(cnt, red);
    nb = group_sum<G>(nb, red);
    if (tid == 0) {
        a.row_nnz[i] = cnt;
        a.row_blocks[i] = nb;
    }
    const int lo = a.lofs[i];
    if (lo >= 0) {  // the row's list, from the masks in word order
        if (!IN_LDS) wg_fence();
        __syncthreads();
        int2* out = a.lists + lo;
        const int chunk = (words + G - 1) / G;
        const int beg = min(tid * chunk, words);
        const int end = min(beg + chunk, words);
        int local = 0;
        for (int t = beg; t < end; ++t) local += ld_tab<IN_LDS>(&masks[t]) != 0;
        int total;
        int pos = group_excl_scan<G>(local, total, red);
        for (int t = beg; t < end; ++t) {
            const uint32_t mk = ld_tab<IN_LDS>(&masks[t]);
            if (mk) out[pos++] = make_int2(base + t, (int)mk);
        }
    }
    __syncthreads();
}

// Global path of the symbolic phase: long rows, and the exact retry of rows
// whose learned-size table overflowed.  Persistent: each workgroup walks the
// row list with stride gridDim.x (the count may be read on the device).
__global__ __launch_bounds__(WIDE_THREADS) void k_sym_wide(SymArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[48];
    if (a.ctl->err & ERR_INPUT) return;
    const int count = a.count_dev ? *a.count_dev : a.count;
    const int32_t* perm = a.off_dev ? a.perm + *a.off_dev : a.perm;
    uint32_t* slab = a.slab ? a.slab + (int64_t)blockIdx.x * a.slab_words : nullptr;
    uint8_t* stage = reinterpret_cast<uint8_t*>(smem) + a.wide_lds;
    int2* off = reinterpret_cast<int2*>(stage);
    Win* win = reinterpret_cast<Win*>(stage + WIDE_THREADS * 16);
    for (int r = blockIdx.x; r < count; r += gridDim.x) {
        const int i = perm[r];
        const RowInfo ri = a.rinfo[i];
        const int64_t words = row_words(ri.x, ri.y);
        if (words * 4 <= a.wide_lds) wide_sym_row<true>(a, i, smem, off, win, red);
        else wide_sym_row<false>(a, i, slab, off, win, red);
    }
}

// ------------------------------------------------------------------- numeric
// The row's list (its occupied blocks in ascending order, from the symbolic
// phase) and a prefix sum of its popcounts give every column its rank; the
// walk over B adds each product at its column's rank.
//   direct:    one {mask, prefix} pair per 32-column word of the row's range;
//   two-level: a {bits, first} pair per 32 blocks marks occupied blocks and
//              holds the list index of the first of them, so a block's list
//              index is first + a popcount; per listed block {mask, prefix};
//   hashed:    {block, mask, prefix} slots keyed by block id.

// Hashed numeric slot {block id, mask, prefix, -}: insert-or-find by block id.
__device__ inline int slot_insert(int4* slots, int T, int logT, int key) {
    int h = hash_slot(key, logT);
    for (int probe = 0; probe < T; ++probe) {
        int* kp = &slots[h].x;
        int cur = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == key) return h;
        if (cur == -1) {
            int old = atomicCAS(kp, -1, key);
            if (old == -1 || old == key) return h;
        }
        h = (h + 1) & (T - 1);
    }
    return -1;
}


template <int G, int MODE, typename T>
// (one row per wavefront: 72 VGPRs give 7 waves per SIMD without spilling)
__global__ __launch_bounds__(G * rows_per_wg<G>()) __attribute__((amdgpu_waves_per_eu(G == 64 ? 7 : 4)))
void k_num(NumArgs a) {
    constexpr int RPW = rows_per_wg<G>();
    constexpr int KB = sizeof(T) == 8 ? FLAT_KB_F64 : FLAT_KB_F32;
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[48];
    const int bytes = tier_bytes(a.tier);
    const int per_row = bytes + stage_bytes(G);
    // a group of 64 or more lanes owns whole wavefronts: its row is wave-uniform
    const int sub = G >= 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / G) : threadIdx.x / G;
    const int lane = threadIdx.x % G, wv = lane >> 6;
    const unsigned long long le = (2ull << (lane & 63)) - 1;
    const int slot = xcd_block<G>(blockIdx.x, gridDim.x) * RPW + sub;
    if (slot >= a.count) return;
    const int4 d = a.desc[slot];
    const int i = d.x, a0 = d.y, a1 = d.z, off = d.w;
    const T* av = reinterpret_cast<const T*>(a.av);
    const T* bv = reinterpret_cast<const T*>(a.bv);
    // Loads are issued in the order their data is needed (vector memory
    // returns in order): the first chunk's A entries and values, the row's
    // list, then the B headers of the chunk; all of them before the table is
    // cleared, so their latencies overlap each other and the clear.
    int aj = -1;
    T v0 = T(0);
    if (lane < a1 - a0) {
        aj = a.aci[a0 + lane];
        v0 = av[a0 + lane];
    }
    const int n = a.crp[i + 1] - off;
    const RowInfo ri = a.rinfo[i];
    const int nb = a.row_blocks[i];
    const int2* lst = a.lists + a.lofs[i];  // rows of these classes always have a list
    int2 e_first = make_int2(0, 0);         // the lane's entry of the list's first round
    if (lane < nb) e_first = lst[lane];
    int4 h0 = make_int4(0, 0, 0, 0);        // B headers of the first chunk
    if (aj >= 0) h0 = a.bhdr[aj];
    const int base = ri.x >> 5;
    const int words = (ri.y >> 5) - base + 1;
    const int w1 = (words + 31) >> 5;
    uint8_t* row_lds = reinterpret_cast<uint8_t*>(smem) + (size_t)sub * per_row;
    uint8_t* tab = row_lds;
    int2* bq = reinterpret_cast<int2*>(row_lds + bytes);              // staged B {offset, end}
    T* ava = reinterpret_cast<T*>(row_lds + bytes + G * 8);           // their A values
    Win* winb = reinterpret_cast<Win*>(row_lds + bytes + G * 16);     // B group windows
    // direct: {mask, prefix} per word.  two-level: l1 {bits, first list index}
    // per 32 blocks, then {mask, prefix} per occupied block.  hashed: slots.
    // Indices and prefixes are kept as LDS byte offsets from the start of the
    // dynamic LDS (the l1 index as the offset of its first {mask, prefix}
    // entry, a prefix as the offset of its value), so that a lookup is one
    // shift-and-add per level with the base folded into the LDS access.
    uint8_t* const lds0 = reinterpret_cast<uint8_t*>(smem);
    uint2* dw = reinterpret_cast<uint2*>(tab);
    uint2* l1 = reinterpret_cast<uint2*>(tab);
    uint2* cm = l1 + w1;
    int4* slots = reinterpret_cast<int4*>(tab);
    T* vals;
    int TT = 0, logT = 0;
    if constexpr (MODE == MODE_DIRECT) {
        vals = reinterpret_cast<T*>(tab + align8((int64_t)words * 8));
    } else if constexpr (MODE == MODE_TWOLEVEL) {
        vals = reinterpret_cast<T*>(tab + align8((int64_t)w1 * 8 + (int64_t)nb * 8));
    } else {
        TT = (int)num_hash_slots(nb);
        logT = 31 - __clz(TT);
        vals = reinterpret_cast<T*>(tab + (int64_t)TT * 16);
    }
    const uint32_t vals_off = (uint32_t)(reinterpret_cast<uint8_t*>(vals) - lds0);
    const uint32_t cm_off = (uint32_t)(reinterpret_cast<uint8_t*>(cm) - lds0);
    if constexpr (MODE == MODE_DIRECT) {
        // pairs of words per 16-byte store; an odd last word spills 8 bytes into vals, cleared below
        for (int c = 2 * lane; c < words; c += 2 * G) *reinterpret_cast<uint4*>(&dw[c]) = make_uint4(0, 0, 0, 0);
    } else if constexpr (MODE == MODE_TWOLEVEL) {
        for (int c = lane; c < w1; c += G) l1[c] = make_uint2(0u, ~0u);
    } else {
        for (int c = lane; c < TT; c += G) slots[c] = make_int4(-1, 0, 0, 0);
    }
    for (int r = lane; r < n; r += G) vals[r] = T(0);
    win_clear<G, KB>(winb, lane);
    group_sync<G>();

    // ---- staging (chunks of G entries of A's row; a window table of one batch)
    bool ne = false;
    int pb = 0, P = 0;
    int staged = -1, wb0 = 0;
    // h, v: the lane's B header and A value in chunk e0 (window table
    // cleared and synchronised by the caller)
    auto stage = [&](int e0, int4 h, T v) {
        ne = h.y > 0;
        int2 tot;
        const int2 ex = group_excl_scan2<G>(make_int2(ne, (h.y + FLAT_VB - 1) / FLAT_VB), tot, red);
        pb = ex.y, P = tot.y;
        if (ne) {
            bq[ex.x] = make_int2(h.x - FLAT_VB * ex.y, h.x + h.y);
            ava[ex.x] = v;
        }
        win_mark<G, KB>(winb, ne, pb, 0);
        group_sync<G>();
        win_scan<G, KB, 0>(winb, nullptr, 0, 0, lane, red);
        group_sync<G>();
        staged = e0, wb0 = 0;
    };
    auto restage = [&](int e0) {
        if (staged == e0) return;
        int4 h = make_int4(0, 0, 0, 0);
        T v = T(0);
        if (lane < a1 - e0) {
            h = a.bhdr[a.aci[e0 + lane]];
            v = av[e0 + lane];
        }
        group_sync<G>();
        win_clear<G, KB>(winb, lane);
        group_sync<G>();
        stage(e0, h, v);
    };
    // window table rebuilt for the batch starting at P0
    auto rewin = [&](int P0) {
        if (wb0 == P0) return;
        group_sync<G>();
        win_clear<G, KB>(winb, lane);
        group_sync<G>();
        win_mark<G, KB>(winb, ne, pb, P0);
        const int before = group_sum<G>(ne && pb < P0, red);
        group_sync<G>();
        win_scan<G, KB, 0>(winb, nullptr, before, 0, lane, red);
        group_sync<G>();
        wb0 = P0;
    };
    auto load_cv = [&](int q, int end) { return load_b<T>(a.bci, bv, a.bnnz, q, end); };

    // ---- the table from the row's list: prefix of popcounts in list order
    // (ascending blocks), every block placed with its prefix, and its columns
    // written straight to C
    int32_t* cc = a.ccol + off;
    auto build = [&]() {
        int carry = 0;
        for (int t0 = 0; t0 < nb; t0 += G) {
            const int t = t0 + lane;
            int2 e = e_first;
            if (t0 > 0) {
                e = make_int2(0, 0);
                if (t < nb) e = lst[t];
            }
            int tot;
            const int ex = carry + group_excl_scan<G>(__popc((uint32_t)e.y), tot, red);
            carry += tot;
            if (t < nb) {
                const int b = e.x;
                uint32_t mk = (uint32_t)e.y;
                const uint32_t vo = vals_off + (uint32_t)(ex * (int)sizeof(T));
                if constexpr (MODE == MODE_DIRECT) {
                    dw[b - base] = make_uint2(mk, vo);
                } else if constexpr (MODE == MODE_TWOLEVEL) {
                    cm[t] = make_uint2(mk, vo);
                    const int w = b - base;
                    atomicOr(&l1[w >> 5].x, 1u << (w & 31));
                    atomicMin(&l1[w >> 5].y, cm_off + 8u * (uint32_t)t);
                } else {
                    const int h = slot_insert(slots, TT, logT, b);
                    slots[h].y = (int)mk;
                    slots[h].z = (int)vo;
                }
                int r = ex;
                while (mk) {
                    cc[r++] = (b << 5) + (__ffs(mk) - 1);
                    mk &= mk - 1;
                }
            }
        }
        group_sync<G>();
    };
    // the value slot of column c of the row (in its table)
    auto val_at = [&](int c) {
        uint32_t vo;
        if constexpr (MODE == MODE_DIRECT) {
            const uint2 mp = dw[(c >> 5) - base];
            vo = mp.y + (uint32_t)sizeof(T) * __popc(mp.x & below(c & 31));
        } else if constexpr (MODE == MODE_TWOLEVEL) {
            const int w = (c >> 5) - base;
            const uint2 L = l1[w >> 5];
            const uint2 mp = *reinterpret_cast<const uint2*>(lds0 + L.y + 8u * __popc(L.x & below(w & 31)));
            vo = mp.y + (uint32_t)sizeof(T) * __popc(mp.x & below(c & 31));
        } else {
            const int key = c >> 5;
            int h = hash_slot(key, logT);
            int4 sl = slots[h];
            for (int probe = 1; sl.x != key && probe < TT; ++probe) {
                h = (h + 1) & (TT - 1);
                sl = slots[h];
            }
            vo = (uint32_t)sl.z + (uint32_t)sizeof(T) * __popc((uint32_t)sl.y & below(c & 31));
        }
        return reinterpret_cast<T*>(lds0 + vo);
    };
    // a group's slots are looked up together (elements past the group's end
    // repeat its first column), then its valid products are added
    auto add = [&](const BGroup<T>& g, int e) {
        const T x = ava[e];
        T* pv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pv[j] = val_at(j < g.n ? g.c[j] : g.c[0]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < g.n) atomicAdd(pv[j], x * g.y[j]);
    };

    stage(a0, h0, v0);
    if (a1 - a0 <= G && P <= KB * G) {
        // the whole row in one batch: its B loads are in flight while the table is built
        Batch<G, KB, FLAT_VB, decltype(load_cv)> bb;
        bb.issue(bq, winb, 0, P, lane, wv, le, load_cv);
        build();
        bb.consume(0, P, lane, wv, le, add);
    } else {
        build();
        for (int e0 = a0; e0 < a1; e0 += G) {
            restage(e0);
            for (int P0 = 0; P0 < P; P0 += KB * G) {
                rewin(P0);
                Batch<G, KB, FLAT_VB, decltype(load_cv)> bt;
                bt.issue(bq, winb, P0, P, lane, wv, le, load_cv);
                bt.consume(P0, P, lane, wv, le, add);
            }
        }
    }
    if (a.dinv) {
        // Jacobi-fused product: C(i,:) = B(i,:) - omega D^-1(i) E(i,:); the
        // row's table holds E(i,:), B(i,:) lies inside its pattern
        group_sync<G>();
        const T sc = -(T)a.omega * reinterpret_cast<const T*>(a.dinv)[i];
        for (int r = lane; r < n; r += G) vals[r] *= sc;
        group_sync<G>();
        for (int q = a.brp[i] + lane; q < a.brp[i + 1]; q += G) atomicAdd(val_at(a.bci[q]), bv[q]);
    }
    group_sync<G>();
    T* cv = reinterpret_cast<T*>(a.cval) + off;
    for (int r = lane; r < n; r += G) cv[r] = vals[r];
}

// Global path of the numeric phase.  Values are summed in LDS, one segment
// of `wide_vals` ranks at a time (every segment walks the row's products and
// keeps those whose rank falls in it), then copied out coalesced; a row with
// more than eight segments instead adds straight into C with global atomics.
template <typename T, bool IN_LDS>
__device__ void wide_num_row(const NumArgs& a, int i, uint32_t* masks, int2* off, T* ava, Win* win, T* lv,
                             int* red) {
    constexpr int G = WIDE_THREADS;
    constexpr int KB = 2;  // B groups per lane and batch (1024 lanes: 8192 products per batch)
    const int tid = threadIdx.x;
    const int coff = a.crp[i];
    const int n = a.crp[i + 1] - coff;
    const RowInfo ri = a.rinfo[i];
    const int base = ri.x >> 5;
    const int words = (ri.y >> 5) - base + 1;
    const int seg = a.wide_vals;
    const bool in_lds = seg > 0 && n <= 8 * seg;
    int32_t* pref = reinterpret_cast<int32_t*>(masks + words);
    T* cv = reinterpret_cast<T*>(a.cval) + coff;
    int32_t* cc = a.ccol + coff;
    for (int c = tid; c < words; c += G) masks[c] = 0;
    if (!in_lds)
        for (int r = tid; r < n; r += G) cv[r] = T(0);
    wg_fence();
    __syncthreads();
    const int a0 = a.arp[i], a1 = a.arp[i + 1];
    const T* av = reinterpret_cast<const T*>(a.av);
    const T* bv = reinterpret_cast<const T*>(a.bv);
    auto load_run = [&](int q, int end) { return load_runs<FLAT_VC>(a.bc, a.bc_total, q, end); };
    auto load_cv = [&](int q, int end) { return load_b<T>(a.bci, bv, a.bnnz, q, end); };
    auto orb = [&](int2 run, int) { atomicOr(&masks[run.x - base], (uint32_t)run.y); };
    const int lo = a.lofs[i];
    if (lo >= 0) {  // masks from the row's list, else from compressed B
        if (!IN_LDS) wg_fence();
        __syncthreads();
        const int nbk = a.row_blocks[i];
        for (int t = tid; t < nbk; t += G) {
            const int2 e = a.lists[lo + t];
            masks[e.x - base] = (uint32_t)e.y;
        }
    } else {
        flat_walk<G, FLAT_KC_NUM, FLAT_VC, true, T>(a.aci, a.bhdr, av, a0, a1, off, ava, win, red, load_run,
                                                    each(orb));
    }
    if (!IN_LDS) wg_fence();
    __syncthreads();
    {
        const int chunk = (words + G - 1) / G;
        const int beg = tid * chunk;
        const int end = min(beg + chunk, words);
        int local = 0;
        for (int t = beg; t < end; ++t) local += __popc(ld_tab<IN_LDS>(&masks[t]));
        int total;
        int ex = group_excl_scan<G>(local, total, red);
        for (int t = beg; t < end; ++t) {
            pref[t] = ex;
            ex += __popc(ld_tab<IN_LDS>(&masks[t]));
        }
    }
    if (!IN_LDS) wg_fence();
    __syncthreads();
    auto rank_of = [&](int c) {
        const int w = (c >> 5) - base;
        const uint32_t mk = ld_tab<IN_LDS>(&masks[w]);
        return (int)ld_tab<IN_LDS>(reinterpret_cast<uint32_t*>(&pref[w])) + __popc(mk & below(c & 31));
    };
    // a group's ranks are looked up together (elements past its end repeat its first column)
    auto ranks = [&](const BGroup<T>& g, int* rk) {
#pragma unroll
        for (int j = 0; j < 4; ++j) rk[j] = rank_of(j < g.n ? g.c[j] : g.c[0]);
    };
    if (in_lds) {
        for (int s0 = 0; s0 < n; s0 += seg) {
            const int len = min(seg, n - s0);
            for (int r = tid; r < len; r += G) lv[r] = T(0);
            __syncthreads();
            flat_walk<G, KB, FLAT_VB, false, T>(a.aci, a.bhdr, av, a0, a1, off, ava, win, red, load_cv,
                                                [&](const BGroup<T>& g, int e) {
                                                    const T x = ava[e];
                                                    int rk[4];
                                                    ranks(g, rk);
#pragma unroll
                                                    for (int j = 0; j < 4; ++j) {
                                                        const int r = rk[j] - s0;
                                                        if (j < g.n && (unsigned)r < (unsigned)len)
                                                            atomicAdd(&lv[r], x * g.y[j]);
                                                    }
                                                });
            if (a.dinv) {  // Jacobi-fused: scale the segment, then add B(i,:)'s entries in it
                const T sc = -(T)a.omega * reinterpret_cast<const T*>(a.dinv)[i];
                for (int r = tid; r < len; r += G) lv[r] *= sc;
                __syncthreads();
                for (int q = a.brp[i] + tid; q < a.brp[i + 1]; q += G) {
                    const int r = rank_of(a.bci[q]) - s0;
                    if ((unsigned)r < (unsigned)len) atomicAdd(&lv[r], bv[q]);
                }
                __syncthreads();
            }
            for (int r = tid; r < len; r += G) cv[s0 + r] = lv[r];
            __syncthreads();
        }
    } else {
        flat_walk<G, KB, FLAT_VB, false, T>(a.aci, a.bhdr, av, a0, a1, off, ava, win, red, load_cv,
                                            [&](const BGroup<T>& g, int e) {
                                                const T x = ava[e];
                                                int rk[4];
                                                ranks(g, rk);
#pragma unroll
                                                for (int j = 0; j < 4; ++j)
                                                    if (j < g.n) atomicAdd(&cv[rk[j]], x * g.y[j]);
                                            });
        if (a.dinv) {  // Jacobi-fused, in C's own storage (summed by atomics in L2: read and written there)
            const T sc = -(T)a.omega * reinterpret_cast<const T*>(a.dinv)[i];
            wg_fence();
            __syncthreads();
            for (int r = tid; r < n; r += G)
                __hip_atomic_store(&cv[r], __hip_atomic_load(&cv[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * sc,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wg_fence();
            __syncthreads();
            for (int q = a.brp[i] + tid; q < a.brp[i + 1]; q += G) atomicAdd(&cv[rank_of(a.bci[q])], bv[q]);
        }
    }
    for (int t = tid; t < words; t += G) {
        uint32_t mk = ld_tab<IN_LDS>(&masks[t]);
        int r = (int)ld_tab<IN_LDS>(reinterpret_cast<uint32_t*>(&pref[t]));
        const int b = base + t;
        while (mk) {
            cc[r++] = (b << 5) + (__ffs(mk) - 1);
            mk &= mk - 1;
        }
    }
    wg_fence();
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(WIDE_THREADS) void k_num_wide(NumArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[48];
    uint32_t* slab = a.slab ? a.slab + (int64_t)blockIdx.x * a.slab_words : nullptr;
    uint8_t* stage = reinterpret_cast<uint8_t*>(smem) + a.wide_lds;
    int2* off = reinterpret_cast<int2*>(stage);
    T* ava = reinterpret_cast<T*>(stage + WIDE_THREADS * 8);
    Win* win = reinterpret_cast<Win*>(stage + WIDE_THREADS * 16);
    T* lv = reinterpret_cast<T*>(stage + WIDE_THREADS * 16 + WIDE_WIN_BYTES);
    const int count = a.count_dev ? *a.count_dev : a.count;
    for (int r = blockIdx.x; r < count; r += gridDim.x) {
        const int i = a.perm[r];
        const RowInfo ri = a.rinfo[i];
        const int64_t words = row_words(ri.x, ri.y);
        if (words * 8 <= a.wide_lds) wide_num_row<T, true>(a, i, smem, off, ava, win, lv, red);
        else wide_num_row<T, false>(a, i, slab, off, ava, win, lv, red);
    }
}

// ---------------------------------------------------- tiled global path
// Long rows of the numeric phase, cut by column tile.  B's columns are split
// into tiles of W = TILE_BYTES / (element size) columns, and every B row
// keeps the offsets where its entries of each tile begin (built once per
// symbolic result; the entries of a row must be grouped by tile, which holds
// for rows stored in ascending column order).  A work item is one (row, tile)
// pair: its products are exactly the products of the B rows' entries in the
// tile, summed into a dense LDS window indexed by column minus the tile's
// first column (the paper's dense accumulator restricted to one tile), so no
// product is walked twice and no rank is looked up per product.  The row's
// list pairs of the tile (its occupied 32-column blocks, ascending, with the
// rank of the first) then place every column, and the values go out
// coalesced.  Items are numbered tile-major, so the workgroups in flight work
// on the same tile of B and share it in L2.

// Tile offsets: per B row, toff[t] = first entry whose column lies in tile t
// or later (t = 0..T-1), toff[T] = the row's end.  Sixteen lanes per row; a
// row whose tiles go down somewhere raises b_tile_unordered (the items then
// all take the segment path).
__global__ __launch_bounds__(256) void k_b_tiles(TileArgs a) {
    const int T = a.ntiles;
    const int64_t total = (int64_t)a.n * 16;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(g >> 4), l = (int)(g & 15);
        const int s0 = a.brp[j], e0 = a.brp[j + 1];
        int32_t* to = a.toff + (int64_t)j * (T + 1);
        if (s0 == e0) {
            for (int t = l; t <= T; t += 16) to[t] = s0;
            continue;
        }
        for (int q = s0 + l; q < e0; q += 16) {
            const int tq = a.bci[q] >> a.log_cols;
            const int tp = q > s0 ? a.bci[q - 1] >> a.log_cols : -1;
            if (tq < tp) {
                a.ctl->b_tile_unordered = 1;
                continue;
            }
            for (int t = tp + 1; t <= tq; ++t) to[t] = q;
            if (q == e0 - 1)
                for (int t = tq + 1; t <= T; ++t) to[t] = e0;
        }
    }
}

// Work items: one wavefront per row of the class walks the row's list once
// and records, per tile, the list pairs that fall in it and the rank of the
// first.  Rows without a list (or all rows, if B's rows are not grouped by
// tile) go to the fallback list for the segment path, with empty items.
__global__ __launch_bounds__(256) void k_tile_items(TileArgs a) {
    __shared__ int3 tl[4][TILE_MAX];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int T = a.ntiles, R = a.rows;
    const int log_blocks = a.log_cols - 5;
    const bool unordered = a.ctl->b_tile_unordered != 0;
    for (int r = blockIdx.x * 4 + w; r < R; r += gridDim.x * 4) {
        const int i = a.perm[r];
        const int lo = a.lofs[i];
        if (lo < 0 || unordered) {
            if (lane == 0) a.fallback[atomicAdd(&a.ctl->tile_fallback, 1)] = i;
            for (int t = lane; t < T; t += 64) a.items[(int64_t)t * R + r] = make_int4(i, 0, 0, 0);
            continue;
        }
        if (lane == 0) {
            if (a.arp[i + 1] - a.arp[i] > TILE_G) a.heavy[atomicAdd(&a.ctl->tile_heavy, 1)] = r;
            else a.light[atomicAdd(&a.ctl->tile_light, 1)] = r;
        }
        for (int t = lane; t < T; t += 64) tl[w][t] = make_int3(0, 0, 0);
        __builtin_amdgcn_wave_barrier();
        const int nbk = a.row_blocks[i];
        const int2* L = a.lists + lo;
        int run = 0;
        for (int p0 = 0; p0 < nbk; p0 += 64) {
            const int p = p0 + lane;
            const bool ok = p < nbk;
            const int2 e = ok ? L[p] : make_int2(0, 0);
            const int tile = e.x >> log_blocks;
            const int prev = ok && p > 0 ? L[p - 1].x >> log_blocks : -1;
            const int next = ok && p + 1 < nbk ? L[p + 1].x >> log_blocks : -1;
            const int pop = ok ? __popc((uint32_t)e.y) : 0;
            const int incl = wave_incl_scan<64>(pop);
            if (ok && tile != prev) tl[w][tile].x = p, tl[w][tile].z = run + incl - pop;
            if (ok && tile != next) tl[w][tile].y = p + 1;
            run += __builtin_amdgcn_readlane(incl, 63);
        }
        __builtin_amdgcn_wave_barrier();
        for (int t = lane; t < T; t += 64) {
            const int3 v = tl[w][t];
            a.items[(int64_t)t * R + r] = make_int4(i, lo + v.x, lo + v.y, v.z);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Work units, strided over the grid: first one per (tile, row) of the rows
// of more than TILE_G entries of A (their chunks are restaged per tile, and
// the units of one row run on many workgroups), then one per other row, whose
// tiles run in order on one workgroup with the row's entries held in
// registers.  There each lane loads its entry's offset of the tile after next
// while the current tile is walked (consecutive tiles share a boundary) and
// the next tile's item is fetched early, so a tile waits only for its B
// loads; the tile's list pairs are loaded before the walk and scanned after
// it.
template <typename T>
__global__ __launch_bounds__(TILE_G) void k_num_tiled(TileArgs a) {
    constexpr int G = TILE_G;
    // The window sums in FP64 whatever T is: LDS atomic adds of FP32 values
    // ran at half the rate of FP64 ones here (R-MAT scale 18, FP32: 21.3 ms
    // with an FP32 window of 8192 columns, 15.0 with this one of 4096), and
    // the FP64 sum is the closer one to the exact result.
    using D = double;
    constexpr int W = TILE_BYTES / (int)sizeof(D);  // columns per tile
    constexpr int NB = W / 32;                       // blocks per tile
    constexpr int K = sizeof(T) == 8 ? FLAT_KB_F64 : FLAT_KB_F32;
    static_assert(NB <= G, "a tile's list pairs must fit one per lane");
    __shared__ D dense[W];
    __shared__ int2 off[G];
    __shared__ T ava[G];
    __shared__ Win win[K * (G / 64)];
    __shared__ int red[48];
    const int tid = threadIdx.x;
    const int T_ = a.ntiles, R = a.rows;
    const int nh = a.ctl->tile_heavy, nl = a.ctl->tile_light;
    const int64_t units = (int64_t)nh * T_ + nl;
    const T* av = reinterpret_cast<const T*>(a.av);
    const T* bv = reinterpret_cast<const T*>(a.bv);
    T* cvals = reinterpret_cast<T*>(a.cval);
    auto load_cv = [&](int q, int end) { return load_b<T>(a.bci, bv, a.bnnz, q, end); };
    // The dense window is zero between tiles: cleared once here, and every
    // entry a tile writes (its products and, fused, B(i,:) all fall on C's
    // columns) is read once and set back to zero as the tile goes out.
    for (int c = tid; c < W; c += G) dense[c] = D(0);
    __syncthreads();
    // a tile's table before the walk: window table cleared, its list pairs
    // loaded (pr, scanned after the walk)
    auto begin_tile = [&](int p0, int np, int2& pr) {
        win_clear<G, K>(win, tid);
        pr = make_int2(0, 0);
        if (tid < np) pr = a.lists[p0 + tid];
    };
    // Jacobi-fused product: the tile's window holds E(i, tile); scale it by
    // -omega D^-1(i) and add B(i,:)'s entries of the tile (toff of row i)
    auto jacobi_tile = [&](int i, int t, int col0) {
        if (!a.dinv) return;
        const T sc = -(T)a.omega * reinterpret_cast<const T*>(a.dinv)[i];
        for (int c = tid; c < W; c += G) dense[c] *= (D)sc;
        __syncthreads();
        const int* tr = a.toff + (int64_t)i * (T_ + 1);
        for (int q = tr[t] + tid; q < tr[t + 1]; q += G) atomicAdd(&dense[a.bci[q] - col0], (D)bv[q]);
        __syncthreads();
    };
    // after the walk: the tile's columns in rank order, then columns and
    // values out (coalesced).  Each lane holds one list pair (np <= W / 32 =
    // G) and places its columns at their ranks (its exclusive prefix of
    // popcounts on): chunk by chunk of 2G ranks into the staging area, which
    // the walk no longer needs, and each chunk is then written out.
    // pos: the lane's pair's first rank (the exclusive prefix of the pairs'
    // popcounts), n_t: the tile's columns
    auto place_tile = [&](int i, int col0, int4 d, int np, int2 pr, int pos, int n_t) {
        constexpr int CH = 2 * G;
        int* cbuf = reinterpret_cast<int*>(off);
        uint32_t rest = tid < np ? (uint32_t)pr.y : 0u;  // the pair's columns not yet placed
        const int first = tid < np ? (pr.x << 5) - col0 : 0;
        const int64_t coff = (int64_t)a.crp[i] + d.w;
        for (int q0 = 0; q0 < n_t; q0 += CH) {
            while (rest && pos < q0 + CH) {
                cbuf[pos - q0] = first + __builtin_ctz(rest);
                rest &= rest - 1u;
                ++pos;
            }
            __syncthreads();
            const int q1 = min(q0 + CH, n_t);
            for (int q = q0 + tid; q < q1; q += G) {
                const int cl = cbuf[q - q0];
                a.ccol[coff + q] = col0 + cl;
                cvals[coff + q] = (T)dense[cl];
                dense[cl] = D(0);
            }
            __syncthreads();
        }
    };
    auto end_tile = [&](int i, int col0, int4 d, int np, int2 pr) {
        int n_t;
        const int pos = group_excl_scan<G>(tid < np ? __popc((uint32_t)pr.y) : 0, n_t, red);
        place_tile(i, col0, d, np, pr, pos, n_t);
    };
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        if (u < (int64_t)nh * T_) {
            // one tile of a long row; units are numbered tile-major, so the
            // workgroups in flight share a tile of B
            const int r = a.heavy[u % nh];
            const int t = (int)(u / nh);
            const int4 d = a.items[(int64_t)t * R + r];
            const int i = __builtin_amdgcn_readfirstlane(d.x);
            const int p0 = __builtin_amdgcn_readfirstlane(d.y);
            const int np = __builtin_amdgcn_readfirstlane(d.z) - p0;
            if (np <= 0) continue;
            const int col0 = t * W;
            int2 pr;
            begin_tile(p0, np, pr);
            auto add = [&](const BGroup<T>& g, int e) {
                const T x = ava[e];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < g.n) atomicAdd(&dense[g.c[j] - col0], (D)x * (D)g.y[j]);
            };
            const int* to = a.toff + t;
            auto hdr = [&](int j) {
                const int64_t o = (int64_t)j * (T_ + 1);
                const int s0 = to[o], s1 = to[o + 1];
                return make_int2(s0, s1 - s0);
            };
            flat_walk_hdr<G, K, FLAT_VB, false, T>(a.aci, hdr, av, a.arp[i], a.arp[i + 1], off, ava, win, red, load_cv,
                                                   add);
            jacobi_tile(i, t, col0);
            end_tile(i, col0, d, np, pr);
            continue;
        }
        // a row of at most G entries, all its tiles
        const int r = a.light[u - (int64_t)nh * T_];
        int4 d = a.items[r];
        const int i = __builtin_amdgcn_readfirstlane(d.x);
        const int a0 = a.arp[i], a1 = a.arp[i + 1];
        const int* tj = nullptr;
        T v = T(0);
        int s_cur = 0, s_nxt = 0, s_nn = 0;
        if (tid < a1 - a0) {
            const int j = a.aci[a0 + tid];
            v = av[a0 + tid];
            tj = a.toff + (int64_t)j * (T_ + 1);
            s_cur = tj[0];
            s_nxt = tj[1];
            if (T_ > 1) s_nn = tj[2];
        }
        // items are fetched two tiles ahead and list pairs one tile ahead
        // (every lane loads: a lane past the tile's pairs reloads its last);
        // the pairs' rank prefix is scanned with the walk's staging
        auto pairs_of = [&](int4 it) {
            const int q0 = __builtin_amdgcn_readfirstlane(it.y);
            const int nq = __builtin_amdgcn_readfirstlane(it.z) - q0;
            return nq > 0 ? a.lists[q0 + min(tid, nq - 1)] : make_int2(0, 0);
        };
        int4 dn = T_ > 1 ? a.items[(int64_t)R + r] : make_int4(0, 0, 0, 0);
        int2 pr = pairs_of(d);
        for (int t = 0; t < T_; ++t) {
            const int4 dnn = t + 2 < T_ ? a.items[(int64_t)(t + 2) * R + r] : make_int4(0, 0, 0, 0);
            const int2 pr_next = t + 1 < T_ ? pairs_of(dn) : make_int2(0, 0);
            const int p0 = __builtin_amdgcn_readfirstlane(d.y);
            const int np = __builtin_amdgcn_readfirstlane(d.z) - p0;
            const int2 h = make_int2(s_cur, s_nxt - s_cur);
            if (tj) {  // shift the offsets one tile on, fetching the next one early
                s_cur = s_nxt;
                s_nxt = s_nn;
                if (t + 3 <= T_) s_nn = tj[t + 3];
            }
            if (np > 0) {
                const int col0 = t * W;
                win_clear<G, K>(win, tid);
                auto add = [&](const BGroup<T>& g, int e) {
                    const T x = ava[e];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j < g.n) atomicAdd(&dense[g.c[j] - col0], (D)x * (D)g.y[j]);
                };
                group_sync<G>();
                int2 sc;
                walk_chunk<G, K, FLAT_VB, false, T>(h, v, off, ava, win, red, load_cv, add,
                                                    tid < np ? __popc((uint32_t)pr.y) : 0, &sc);
                group_sync<G>();
                jacobi_tile(i, t, col0);
                place_tile(i, col0, d, np, pr, sc.x, sc.y);
            }
            d = dn;
            dn = dnn;
            pr = pr_next;
        }
    }
}

template <int G, int MODE>
void sym_launch(hipStream_t s, const SymArgs& a) {
    constexpr int RPW = rows_per_wg<G>();
    const unsigned grid = (unsigned)((a.count + RPW - 1) / RPW);
    const size_t smem = (size_t)RPW * (tier_bytes(a.tier) + sym_stage_bytes(G));
    hipLaunchKernelGGL((k_sym<G, MODE>), dim3(grid), dim3(G * RPW), smem, s, a);
}

template <int MODE>
void sym_dispatch(hipStream_t s, const SymArgs& a) {
    switch (tier_threads(a.tier)) {
        case 8: sym_launch<8, MODE>(s, a); break;
        case 16: sym_launch<16, MODE>(s, a); break;
        case 32: sym_launch<32, MODE>(s, a); break;
        case 64: sym_launch<64, MODE>(s, a); break;
        case 128: sym_launch<128, MODE>(s, a); break;
        case 256: sym_launch<256, MODE>(s, a); break;
        case 512: sym_launch<512, MODE>(s, a); break;
        default: sym_launch<1024, MODE>(s, a); break;
    }
}

template <int G>
int sym_tier_launch(hipStream_t s, const SymArgs& a, int64_t max_rows, int n_cu) {
    constexpr int RPW = rows_per_wg<G>();
    const size_t smem = (size_t)RPW * (tier_bytes(a.tier) + sym_stage_bytes(G));
    // workgroups per compute unit at this LDS size, looked up once per tier
    static int occupancy[NTIER] = {};
    int occ = occupancy[a.tier];
    if (occ <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sym_tier<G>, G * RPW, smem) != hipSuccess || occ < 1)
            occ = 1;
        occupancy[a.tier] = occ;
    }
    const int64_t groups = (max_rows + RPW - 1) / RPW;
    int64_t grid = std::min<int64_t>((int64_t)occ * n_cu, std::max<int64_t>(groups, 1));
    grid = (grid + 7) / 8 * 8;
    hipLaunchKernelGGL(k_sym_tier<G>, dim3((unsigned)grid), dim3(G * RPW), smem, s, a);
    return (int)grid;
}

template <int G, int MODE, typename T>
void num_launch(hipStream_t s, const NumArgs& a) {
    constexpr int RPW = rows_per_wg<G>();
    const unsigned grid = (unsigned)((a.count + RPW - 1) / RPW);
    const size_t smem = (size_t)RPW * (tier_bytes(a.tier) + stage_bytes(G));
    hipLaunchKernelGGL((k_num<G, MODE, T>), dim3(grid), dim3(G * RPW), smem, s, a);
}


template <int MODE, typename T>
void num_dispatch(hipStream_t s, const NumArgs& a) {
    switch (tier_threads(a.tier)) {
        case 8: num_launch<8, MODE, T>(s, a); break;
        case 16: num_launch<16, MODE, T>(s, a); break;
        case 32: num_launch<32, MODE, T>(s, a); break;
        case 64: num_launch<64, MODE, T>(s, a); break;
        case 128: num_launch<128, MODE, T>(s, a); break;
        case 256: num_launch<256, MODE, T>(s, a); break;
        case 512: num_launch<512, MODE, T>(s, a); break;
        default: num_launch<1024, MODE, T>(s, a); break;
    }
}

}  // namespace

size_t wide_smem_bytes(int wide_lds, int phase, int vals_bytes) {
    return (size_t)wide_lds + WIDE_THREADS * 16 + WIDE_WIN_BYTES + (phase ? vals_bytes : 0);
}

int launch_sym_class(hipStream_t s, const SymArgs& a, int grid_cap) {
    if (a.tier == TIER_GLOBAL) {
        int grid = a.count_dev ? grid_cap : (a.count < grid_cap ? a.count : grid_cap);
        if (grid < 1) return 0;
        hipLaunchKernelGGL(k_sym_wide, dim3(grid), dim3(WIDE_THREADS), wide_smem_bytes(a.wide_lds, 0, 0), s, a);
        return grid;
    }
    if (a.count <= 0) return 0;
    if (a.mode == MODE_DIRECT) sym_dispatch<MODE_DIRECT>(s, a);
    else if (a.mode == MODE_HASHED) sym_dispatch<MODE_HASHED>(s, a);
    else sym_dispatch<MODE_TWOLEVEL>(s, a);
    return 1;
}

int launch_sym_tier(hipStream_t s, const SymArgs& a, int64_t max_rows, int n_cu) {
    if (max_rows <= 0 || a.tier < 0 || a.tier >= TIER_GLOBAL) return 0;
    switch (tier_threads(a.tier)) {
        case 8: return sym_tier_launch<8>(s, a, max_rows, n_cu);
        case 16: return sym_tier_launch<16>(s, a, max_rows, n_cu);
        case 32: return sym_tier_launch<32>(s, a, max_rows, n_cu);
        case 64: return sym_tier_launch<64>(s, a, max_rows, n_cu);
        case 128: return sym_tier_launch<128>(s, a, max_rows, n_cu);
        case 256: return sym_tier_launch<256>(s, a, max_rows, n_cu);
        case 512: return sym_tier_launch<512>(s, a, max_rows, n_cu);
        default: return sym_tier_launch<1024>(s, a, max_rows, n_cu);
    }
}

int launch_num_class(hipStream_t s, const NumArgs& a, int elem_bytes, int grid_cap) {
    if (a.count <= 0 && !a.count_dev) return 0;
    if (a.tier == TIER_GLOBAL) {
        int grid = a.count_dev ? grid_cap : (a.count < grid_cap ? a.count : grid_cap);
        if (grid < 1) return 0;
        const size_t smem = wide_smem_bytes(a.wide_lds, 1, a.wide_vals * elem_bytes);
        if (elem_bytes == 8) hipLaunchKernelGGL(k_num_wide<double>, dim3(grid), dim3(WIDE_THREADS), smem, s, a);
        else hipLaunchKernelGGL(k_num_wide<float>, dim3(grid), dim3(WIDE_THREADS), smem, s, a);
        return grid;
    }
    if (a.count <= 0) return 0;
    if (elem_bytes == 8) {
        if (a.mode == MODE_DIRECT) num_dispatch<MODE_DIRECT, double>(s, a);
        else if (a.mode == MODE_HASHED) num_dispatch<MODE_HASHED, double>(s, a);
        else num_dispatch<MODE_TWOLEVEL, double>(s, a);
    } else {
        if (a.mode == MODE_DIRECT) num_dispatch<MODE_DIRECT, float>(s, a);
        else if (a.mode == MODE_HASHED) num_dispatch<MODE_HASHED, float>(s, a);
        else num_dispatch<MODE_TWOLEVEL, float>(s, a);
    }
    return 1;
}

void launch_tile_build(hipStream_t s, const TileArgs& a) {
    const int64_t lanes = (int64_t)a.n * 16;
    const unsigned gb = (unsigned)std::min<int64_t>((lanes + 255) / 256, 8192);
    if (gb > 0) hipLaunchKernelGGL(k_b_tiles, dim3(gb), dim3(256), 0, s, a);
    const unsigned gi = (unsigned)std::min<int64_t>(((int64_t)a.rows + 3) / 4, 4096);
    if (gi > 0) hipLaunchKernelGGL(k_tile_items, dim3(gi), dim3(256), 0, s, a);
}

int launch_num_tiled(hipStream_t s, const TileArgs& a, int elem_bytes, int n_cu) {
    if (a.ntiles <= 0 || a.rows <= 0) return 0;
    // four 256-lane workgroups fit a compute unit's LDS (the unit counts are
    // read on the device; workgroups beyond them exit at once)
    const int grid = (int)std::min<int64_t>((int64_t)a.rows * a.ntiles, (int64_t)n_cu * 4);
    if (elem_bytes == 8) hipLaunchKernelGGL(k_num_tiled<double>, dim3(grid), dim3(TILE_G), 0, s, a);
    else hipLaunchKernelGGL(k_num_tiled<float>, dim3(grid), dim3(TILE_G), 0, s, a);
    return grid;
}

}  // namespace spg
