// The paper's own SpGEMM design (section 2.2.1), kept beside this library's
// per-row classes so that the two can be compared on the same inputs.
//
//  * One parallelisation method for the whole matrix, picked from the
//    products (multiply-adds) per row: with few, a group of 16 lanes per
//    row (many rows per workgroup), the referenced B rows taken one after the
//    other and each B row's entries spread over the group's lanes; with many,
//    a workgroup of 256 lanes per row, every lane taking an equal share of
//    the flattened (A entry, B entry) iteration space.
//  * A two-level hash-map accumulator: level 1 in LDS, level 2 in global
//    memory.  Keys go to level 1 until it holds three quarters of its slots;
//    after that a key found in level 1 is still accumulated there, but a new
//    key goes to level 2, which a row uses only from its first such key on.
//    Keys are 32-column blocks with OR-ed masks in the symbolic phase
//    (compressed B), columns with summed values in the numeric phase.  Each
//    map keeps the list of its occupied slots in insertion order, so reading
//    a row out and clearing the map for the next row cost in proportion to
//    the row's keys, not to the map's size.
//  * The numeric phase leaves each row in hash order (the accumulator's
//    order), as the paper's accumulator does; the product's main path emits
//    rows in ascending column order instead.
// Level-2 maps live in a slab with one region per concurrently processed
// row, sized for the longest row's bound on its keys.  The slab is all zeros
// when allocated and every row leaves the slots it used at zero, so a key is
// stored as key + 1 (zero marks an empty slot) in both levels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spg_internal.h"

namespace spg {

namespace {

constexpr int L1_SYM_VEC = 256;     // level-1 slots per row, symbolic, group method
constexpr int L1_NUM_VEC = 128;     // numeric, group method
constexpr int L1_SYM_TEAM = 4096;   // symbolic, team method
constexpr int L1_NUM_TEAM = 2048;   // numeric, team method

__device__ inline uint32_t hslot(int key, uint32_t mask) { return ((uint32_t)key * 2654435761u) & mask; }

// Group-wide helpers.  Groups of up to 64 lanes are aligned inside one
// wavefront; a team is the whole workgroup.
template <int G>
__device__ inline void gsync() {
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

// Lanes of the group with p set (counted) / whether any has it.  A team
// synchronises the workgroup doing it.
template <int G>
__device__ inline int gcount(bool p) {
    if constexpr (G <= 64) {
        const uint64_t b = __ballot(p);
        const int g0 = (threadIdx.x & 63) / G * G;
        const uint64_t gm = G == 64 ? ~0ull : (((1ull << G) - 1) << g0);
        return __popcll(b & gm);
    } else {
        return __syncthreads_count(p);
    }
}

// Exclusive prefix sum over the group; total receives the sum.
template <int G>
__device__ inline int gscan(int v, int& total, int* red) {
    const int lane = threadIdx.x & 63;
    const int w = G < 64 ? G : 64;
    int x = v;
    for (int d = 1; d < w; d <<= 1) {
        const int y = __shfl_up(x, d, w);
        if ((lane % w) >= d) x += y;
    }
    if constexpr (G <= 64) {
        total = __shfl(x, w - 1, w);
        return x - v;
    } else {
        const int wv = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 63) red[wv] = x;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int u = 0; u < G / 64; ++u) {
            if (u < wv) pre += red[u];
            tot += red[u];
        }
        total = tot;
        return pre + x - v;
    }
}

// A hash map of one level: open addressing with linear probing over S slots
// (key + 1 stored, 0 when empty), plus the list of its occupied slots in insertion
// order, so that reading the row out and clearing the map cost in proportion
// to the keys present, not to the map's size.
struct Level {
    int* keys;
    int* used;    // occupied slots in insertion order
    int* nused;   // their number (LDS)
    int S;
};

// Insert-or-find: returns the slot, or -1 if the key is absent and `open` is
// false; *fresh tells whether this call inserted the key.  Both levels are
// private to one workgroup (level 2 is the row's region of the slab), so
// workgroup scope orders every access; the group barriers publish them.
__device__ inline int level_put(const Level& L, int key, bool open, bool& fresh) {
    fresh = false;
    const int k1 = key + 1;
    uint32_t h = hslot(key, L.S - 1);
    for (int probe = 0; probe < L.S; ++probe) {
        const int cur = __hip_atomic_load(&L.keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == k1) return (int)h;
        if (cur == 0) {
            if (!open) return -1;
            const int old = atomicCAS(&L.keys[h], 0, k1);
            if (old == 0) {
                fresh = true;
                L.used[atomicAdd(L.nused, 1)] = (int)h;
                return (int)h;
            }
            if (old == k1) return (int)h;
        }
        h = (h + 1) & (L.S - 1);
    }
    return -1;
}

// A load of level-2 data at device scope: it was written by atomics, which
// act in L2, so the load must not be served from a stale L1 line.
template <typename T>
__device__ inline T ld_l2(T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-row counters of one group (LDS).
struct RowState {
    int n1;  // occupied level-1 slots
    int n2;  // occupied level-2 slots
};

// Visits items p in [0, n_items) in rounds of G, one per lane; item(p) gives
// {key, payload}, acc1 / acc2 accumulate a payload into a level-1 / level-2
// slot.  Level 1 takes new keys while it holds fewer than close_at (its count
// is kept by every lane from the group's per-round tally, so all lanes of a
// round agree); after that a key it holds is still accumulated there and a
// new key goes to level 2, which is the row's from the first such key on.
template <int G, typename Item, typename Acc1, typename Acc2>
__device__ inline void accumulate_rounds(int n_items, int& count1, bool& l2_on, int close_at, const Level& L1,
                                         const Level& L2, Item item, Acc1 acc1, Acc2 acc2) {
    const int lane = threadIdx.x % G;
    for (int base = 0; base < n_items; base += G) {
        if constexpr (G <= 64) gsync<G>();  // the previous round's level-1 keys are in (a team's tallies synchronised)
        const int p = base + lane;
        const bool open = count1 < close_at;
        bool fresh = false, need2 = false;
        int key = 0;
        decltype(item(0).y) pay{};
        if (p < n_items) {
            const auto it = item(p);
            key = it.x;
            pay = it.y;
            const int h = level_put(L1, key, open, fresh);
            if (h >= 0) acc1(h, pay);
            else need2 = true;
        }
        count1 += gcount<G>(fresh);
        if (gcount<G>(need2)) {
            l2_on = true;
            if (need2) {
                bool f2;
                const int h = level_put(L2, key, true, f2);
                acc2(h, pay);
            }
        }
    }
}

template <typename T>
struct KV {
    int x;
    T y;
};

struct PaperArgs {
    int32_t m;
    int32_t team;            // 1: team method, 0: group method
    const int32_t* arp;
    const int32_t* aci;
    const void* av;
    const int32_t* brp;
    const int32_t* bci;
    const void* bv;
    const int2* bc;          // compressed B runs {block, mask}
    const int4* bhdr;        // per B row {start, length, run start, run count}
    const RowInfo* rinfo;
    int32_t* row_nnz;
    int32_t* row_blocks;
    const int32_t* crp;
    int32_t* ccol;
    void* cval;
    int32_t* slab;           // level-2 maps: one region per concurrent row, all zeros between rows
    int64_t slab_slots;
};

// Level-2 slots of row i: twice a bound on its keys (blocks or columns), a power of two.
__device__ inline int l2_slots(const RowInfo& ri, bool blocks, int64_t cap) {
    const int64_t words = row_words(ri.x, ri.y);
    int64_t bound = blocks ? words : (int64_t)(ri.y - ri.x + 1);
    if ((int64_t)ri.z < bound) bound = ri.z;
    int64_t s = 16;
    while (s < 2 * bound) s <<= 1;
    return (int)(s < cap ? s : cap);
}

// Entry of flattened item p for the team method: the chunk's staged A
// entries carry the exclusive prefix of their lengths; binary search.
__device__ inline int team_entry(const int* pre, int cnt, int p) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Symbolic: keys are 32-column blocks of compressed B, masks OR-ed.  Slab
// region of one row: keys[slots], masks[slots], used[slots].
template <int G>
__global__ __launch_bounds__(256) void k_paper_sym(PaperArgs a) {
    constexpr int RPW = 256 / G;
    constexpr int S1 = G <= 64 ? L1_SYM_VEC : L1_SYM_TEAM;
    __shared__ int keys1[RPW][S1];
    __shared__ uint32_t masks1[RPW][S1];
    __shared__ int used1[RPW][S1];
    __shared__ RowState st_[RPW];
    __shared__ int pre_[G <= 64 ? 1 : G], first_[G <= 64 ? 1 : G];
    __shared__ int red[8];
    const int sub = threadIdx.x / G, lane = threadIdx.x % G;
    uint32_t* masks = masks1[sub];
    RowState* st = &st_[sub];
    const int slot = blockIdx.x * RPW + sub;
    int* k2 = a.slab + (int64_t)slot * a.slab_slots * 3;
    uint32_t* m2 = reinterpret_cast<uint32_t*>(k2 + a.slab_slots);
    int* u2 = k2 + 2 * a.slab_slots;
    for (int t = lane; t < S1; t += G) keys1[sub][t] = 0, masks[t] = 0;
    gsync<G>();
    for (int i = slot; i < a.m; i += gridDim.x * RPW) {
        const RowInfo ri = a.rinfo[i];
        if (ri.z == 0) continue;  // empty row: sized by the analysis
        if (lane == 0) st->n1 = 0, st->n2 = 0;
        gsync<G>();
        const Level L1{keys1[sub], used1[sub], &st->n1, S1};
        const Level L2{k2, u2, &st->n2, l2_slots(ri, true, a.slab_slots)};
        int count1 = 0;
        bool l2_on = false;
        auto acc1 = [&](int h, uint32_t bits) { atomicOr(&masks[h], bits); };
        auto acc2 = [&](int h, uint32_t bits) { atomicOr(&m2[h], bits); };
        const int a0 = a.arp[i], a1 = a.arp[i + 1];
        if constexpr (G <= 64) {
            // group method: referenced B rows one after the other
            for (int e = a0; e < a1; ++e) {
                const int4 h = a.bhdr[a.aci[e]];
                accumulate_rounds<G>(h.w, count1, l2_on, S1 * 3 / 4, L1, L2, [&](int p) {
                    const int2 r = a.bc[h.z + p];
                    return KV<uint32_t>{r.x, (uint32_t)r.y};
                }, acc1, acc2);
            }
        } else {
            // team method: the flattened (A entry, compressed-B run) space, chunk by chunk
            for (int e0 = a0; e0 < a1; e0 += G) {
                const int cnt = min(G, a1 - e0);
                int len = 0, first = 0;
                if (lane < cnt) {
                    const int4 h = a.bhdr[a.aci[e0 + lane]];
                    len = h.w, first = h.z;
                }
                int tot;
                const int ex = gscan<G>(len, tot, red);
                if (lane < cnt) pre_[lane] = ex, first_[lane] = first;
                gsync<G>();
                accumulate_rounds<G>(tot, count1, l2_on, S1 * 3 / 4, L1, L2, [&](int p) {
                    const int q = team_entry(pre_, cnt, p);
                    const int2 r = a.bc[first_[q] + (p - pre_[q])];
                    return KV<uint32_t>{r.x, (uint32_t)r.y};
                }, acc1, acc2);
                gsync<G>();
            }
        }
        gsync<G>();
        // the row's size from the occupied slots of both levels, which are cleared on the way
        const int n1 = st->n1, n2 = l2_on ? st->n2 : 0;
        int cnt = 0;
        for (int t = lane; t < n1; t += G) {
            const int h = used1[sub][t];
            cnt += __popc(masks[h]);
            keys1[sub][h] = 0, masks[h] = 0;
        }
        for (int t = lane; t < n2; t += G) {
            // level 2 was written by atomics in L2: read it there
            const int h = ld_l2(&u2[t]);
            cnt += __popc(ld_l2(&m2[h]));
            k2[h] = 0, m2[h] = 0, u2[t] = 0;
        }
        int tot_c;
        gscan<G>(cnt, tot_c, red);
        if (lane == 0) a.row_nnz[i] = tot_c, a.row_blocks[i] = n1 + n2;
        gsync<G>();
    }
}

// Numeric: keys are columns, values summed.  Slab region of one row:
// keys[slots], used[slots], values[slots] (8-byte aligned).
template <int G, typename T>
__global__ __launch_bounds__(256) void k_paper_num(PaperArgs a) {
    constexpr int RPW = 256 / G;
    constexpr int S1 = G <= 64 ? L1_NUM_VEC : L1_NUM_TEAM;
    __shared__ int keys1[RPW][S1];
    __shared__ T vals1[RPW][S1];
    __shared__ int used1[RPW][S1];
    __shared__ RowState st_[RPW];
    __shared__ int pre_[G <= 64 ? 1 : G], first_[G <= 64 ? 1 : G];
    __shared__ T aval_[G <= 64 ? 1 : G];
    __shared__ int red[8];
    const int sub = threadIdx.x / G, lane = threadIdx.x % G;
    T* vals = vals1[sub];
    RowState* st = &st_[sub];
    const T* av = reinterpret_cast<const T*>(a.av);
    const T* bv = reinterpret_cast<const T*>(a.bv);
    T* cv = reinterpret_cast<T*>(a.cval);
    const int slot = blockIdx.x * RPW + sub;
    int* k2 = a.slab + (int64_t)slot * a.slab_slots * 4;
    int* u2 = k2 + a.slab_slots;
    T* v2 = reinterpret_cast<T*>(k2 + 2 * a.slab_slots);
    for (int t = lane; t < S1; t += G) keys1[sub][t] = 0, vals[t] = T(0);
    gsync<G>();
    for (int i = slot; i < a.m; i += gridDim.x * RPW) {
        const RowInfo ri = a.rinfo[i];
        if (ri.z == 0) continue;
        if (lane == 0) st->n1 = 0, st->n2 = 0;
        gsync<G>();
        const Level L1{keys1[sub], used1[sub], &st->n1, S1};
        const Level L2{k2, u2, &st->n2, l2_slots(ri, false, a.slab_slots)};
        int count1 = 0;
        bool l2_on = false;
        auto acc1 = [&](int h, T x) { atomicAdd(&vals[h], x); };
        auto acc2 = [&](int h, T x) { atomicAdd(&v2[h], x); };
        const int a0 = a.arp[i], a1 = a.arp[i + 1];
        if constexpr (G <= 64) {
            for (int e = a0; e < a1; ++e) {
                const int j = a.aci[e];
                const T x = av[e];
                const int b0 = a.brp[j], nb = a.brp[j + 1] - b0;
                accumulate_rounds<G>(nb, count1, l2_on, S1 * 3 / 4, L1, L2,
                                     [&](int p) { return KV<T>{a.bci[b0 + p], x * bv[b0 + p]}; }, acc1, acc2);
            }
        } else {
            for (int e0 = a0; e0 < a1; e0 += G) {
                const int cnt = min(G, a1 - e0);
                int len = 0, first = 0;
                T x = T(0);
                if (lane < cnt) {
                    const int j = a.aci[e0 + lane];
                    first = a.brp[j];
                    len = a.brp[j + 1] - first;
                    x = av[e0 + lane];
                }
                int tot;
                const int ex = gscan<G>(len, tot, red);
                if (lane < cnt) pre_[lane] = ex, first_[lane] = first, aval_[lane] = x;
                gsync<G>();
                accumulate_rounds<G>(tot, count1, l2_on, S1 * 3 / 4, L1, L2, [&](int p) {
                    const int q = team_entry(pre_, cnt, p);
                    const int b = first_[q] + (p - pre_[q]);
                    return KV<T>{a.bci[b], aval_[q] * bv[b]};
                }, acc1, acc2);
                gsync<G>();
            }
        }
        gsync<G>();
        // the row out in hash order (level 1's keys in insertion order, then
        // level 2's), both levels cleared on the way
        int* cc = a.ccol + a.crp[i];
        T* cvr = cv + a.crp[i];
        const int nrow = a.crp[i + 1] - a.crp[i];  // the symbolic count: a bound on every position below
        const int n1 = st->n1, n2 = l2_on ? st->n2 : 0;
        for (int t = lane; t < n1; t += G) {
            const int h = used1[sub][t];
            if (t < nrow) cc[t] = keys1[sub][h] - 1, cvr[t] = vals[h];
            keys1[sub][h] = 0, vals[h] = T(0);
        }
        for (int t = lane; t < n2; t += G) {
            const int h = ld_l2(&u2[t]);
            if (n1 + t < nrow) cc[n1 + t] = ld_l2(&k2[h]) - 1, cvr[n1 + t] = ld_l2(&v2[h]);
            k2[h] = 0, v2[h] = T(0), u2[t] = 0;
        }
        gsync<G>();
    }
}

}  // namespace

int launch_paper(hipStream_t s, const PaperLaunch& p, bool numeric, int elem_bytes, int n_cu) {
    PaperArgs a{};
    a.m = p.m, a.team = p.team;
    a.arp = p.arp, a.aci = p.aci, a.av = p.av, a.brp = p.brp, a.bci = p.bci, a.bv = p.bv;
    a.bc = p.bc, a.bhdr = p.bhdr, a.rinfo = p.rinfo, a.row_nnz = p.row_nnz, a.row_blocks = p.row_blocks;
    a.crp = p.crp, a.ccol = p.ccol, a.cval = p.cval, a.slab = p.slab, a.slab_slots = p.slab_slots;
    const int grid = p.grid;
    if (p.m <= 0 || grid <= 0) return 0;
    if (!numeric) {
        if (p.team) hipLaunchKernelGGL(k_paper_sym<256>, dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_paper_sym<16>, dim3(grid), dim3(256), 0, s, a);
    } else if (elem_bytes == 8) {
        if (p.team) hipLaunchKernelGGL((k_paper_num<256, double>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_paper_num<16, double>), dim3(grid), dim3(256), 0, s, a);
    } else {
        if (p.team) hipLaunchKernelGGL((k_paper_num<256, float>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_paper_num<16, float>), dim3(grid), dim3(256), 0, s, a);
    }
    return grid;
}

}  // namespace spg
