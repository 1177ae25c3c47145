// Row analysis, binning, row-pointer scan and small utility kernels.
//
// The symbolic phase of section 2.2.1 needs each row's size before C can be
// allocated.  These kernels produce what the accumulator kernels consume:
//   - per B row: length and column range (one pass over B's structure);
//   - per A row: products (the row's FLOP count, which the paper uses to pick
//     a parallelisation method), column range of C's row, largest referenced
//     B row, and the row's accumulator class;
//   - the permutation that groups rows of one class together;
//   - C's row pointer as the exclusive prefix sum of the row counts (section
//     2.2.1), single pass with decoupled look-back, plus the numeric-phase
//     class of every row.
// Index validity is checked in the same passes that read the indices.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <climits>

#include "spg_internal.h"

namespace spg {

namespace {

constexpr int ROW_LANES = 8;        // lanes per B row when compressing B
constexpr int AN_LANES = 4;         // lanes per row in the row analysis passes
constexpr int AN_LOADS = 8;         // independent entry loads per lane and round trip there
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Reductions over aligned groups of AN_LANES = 4 lanes with DPP: swaps of
// neighbours and of pairs inside each quad, after which every lane of the
// group holds the result.  No LDS.
static_assert(AN_LANES == 4, "the row reductions below cover one quad");
template <typename Op>
__device__ inline int rowq_reduce(int v, Op op) {
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    return v;
}
__device__ inline int rowq_sum(int v) { return rowq_reduce(v, [](int x, int y) { return x + y; }); }
__device__ inline int rowq_min(int v) { return rowq_reduce(v, [](int x, int y) { return min(x, y); }); }
__device__ inline int rowq_max(int v) { return rowq_reduce(v, [](int x, int y) { return max(x, y); }); }
__device__ inline int rowq_or(int v) { return rowq_reduce(v, [](int x, int y) { return x | y; }); }
template <int CTRL>
__device__ inline int64_t dpp64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)((uint64_t)v >> 32), CTRL, 0xf, 0xf, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int64_t rowq_sum64(int64_t v) {
    v += dpp64<0xb1>(v);
    v += dpp64<0x4e>(v);
    return v;
}

__device__ inline float log2p1(int64_t v) { return log2f(1.0f + (float)v); }

// A rows: products, column range, largest B row; symbolic class from an upper
// bound on the row's occupied blocks (binning 0: its products, 2: the
// compressed-B runs it reads, 3: the exact count of a previous run) or
// features only (binning 1, learned: classified by k_mlp_classify).
__global__ __launch_bounds__(256) void k_a_rowinfo(int32_t m, int32_t n, const int32_t* __restrict__ arp,
                                                   const int32_t* __restrict__ aci, int64_t annz,
                                                   const int4* __restrict__ binfo, RowInfo* __restrict__ rinfo,
                                                   float* __restrict__ feats, ClassCfg cfg, int binning,
                                                   uint8_t* __restrict__ sym_cls, int32_t* __restrict__ row_nnz,
                                                   int32_t* __restrict__ row_blocks, int32_t* __restrict__ lofs,
                                                   Control* ctl) {
    __shared__ int32_t hist[NCLS];
    __shared__ int32_t empties, nodiag;
    __shared__ unsigned long long prod_sum, wmax_all, wmax_glob, pmax;
    if (threadIdx.x < NCLS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) empties = 0, nodiag = 0, prod_sum = 0, wmax_all = 0, wmax_glob = 0, pmax = 0;
    __syncthreads();
    const int lane = (int)(threadIdx.x % AN_LANES);
    const int64_t rows_per_block = blockDim.x / AN_LANES;
    // grid-stride: few workgroups, one flush of the counters each
    for (int64_t rb = blockIdx.x * rows_per_block; rb < m; rb += (int64_t)gridDim.x * rows_per_block) {
        const int64_t row = rb + threadIdx.x / AN_LANES;
        int64_t ub = 0, rs = 0;  // products; compressed-B runs (a bound on occupied blocks)
        int mx = 0, cmin = INT_MAX, cmax = -1, bad = 0, len = 0, diag = 0;
        if (row < m) {
            int32_t s = arp[row], e = arp[row + 1];
            if (s < 0 || e < s || (int64_t)e > annz || (row == 0 && s != 0) || (row == m - 1 && (int64_t)e != annz)) {
                bad = ERR_A_ROWPTR;
            } else {
                len = e - s;
                // independent index loads, then their gathers.  Every load is
                // unconditional (indices clamped into the row, and to B's
                // first row for entries that are past the row's end or
                // invalid; n > 0 whenever the row has an entry that can be
                // valid) and its value is discarded afterwards where it does
                // not count: a load under a condition with a default in the
                // other branch makes the compiler wait for it before the
                // next one is issued.
                for (int32_t p0 = s + lane; p0 < e; p0 += AN_LOADS * AN_LANES) {
                    int jj[AN_LOADS];
    #pragma unroll
                    for (int u = 0; u < AN_LOADS; ++u) jj[u] = aci[min(p0 + u * AN_LANES, e - 1)];
    #pragma unroll
                    for (int u = 0; u < AN_LOADS; ++u) {
                        const bool in_row = p0 + u * AN_LANES < e;
                        if (in_row && (jj[u] < 0 || jj[u] >= n)) bad = ERR_A_COL;
                        if (!in_row || jj[u] < 0 || jj[u] >= n) jj[u] = -1;
                        diag |= jj[u] == row;  // a stored diagonal entry (square A)
                    }
                    if (n <= 0) continue;  // every entry is invalid: nothing to gather
                    int4 bb[AN_LOADS];
    #pragma unroll
                    for (int u = 0; u < AN_LOADS; ++u) bb[u] = binfo[max(jj[u], 0)];
    #pragma unroll
                    for (int u = 0; u < AN_LOADS; ++u) {
                        if (jj[u] < 0) continue;
                        ub += bb[u].x;
                        rs += bb[u].w;
                        mx = max(mx, bb[u].x);
                        cmin = min(cmin, bb[u].y);
                        cmax = max(cmax, bb[u].z);
                    }
                }
            }
        }
        ub = rowq_sum64(ub);
        rs = rowq_sum64(rs);
        mx = rowq_max(mx);
        cmin = rowq_min(cmin);
        cmax = rowq_max(cmax);
        int anybad = rowq_or(bad);
        diag = rowq_or(diag);
        if (bad) atomicOr(&ctl->err, bad);
        if (row < m && lane == 0 && m == n && !diag) atomicAdd(&nodiag, 1);
        if (row < m && lane == 0) {
            if (anybad) ub = 0;
            int32_t ubc = ub > INT_MAX ? INT_MAX : (int32_t)ub;
            if (ub == 0) cmin = 0, cmax = 0;
            rinfo[row] = make_int4(cmin, cmax, ubc, mx);
            if (feats) {
                feats[row * 3 + 0] = log2p1(len);
                feats[row * 3 + 1] = log2p1(ub);
                feats[row * 3 + 2] = log2p1(mx);
            }
            int cls = CLS_EMPTY;
            if (ub == 0) {
                row_nnz[row] = 0;
                row_blocks[row] = 0;
                atomicAdd(&empties, 1);
                sym_cls[row] = CLS_EMPTY;
            } else {
                int64_t words = row_words(cmin, cmax);
                lofs[row] = list_capacity(rs, words);
                atomicMax(&wmax_all, (unsigned long long)words);
                atomicAdd(&prod_sum, (unsigned long long)ub);
                atomicMax(&pmax, (unsigned long long)ub);
                if (binning != 1) {
                    // binning 3 (ideal estimate): the row's exact occupied blocks, left in
                    // row_blocks by a previous symbolic run of the same matrices
                    const int64_t est = binning == 2 ? rs : binning == 3 ? (int64_t)row_blocks[row] : ub;
                    cls = sym_class(ub, cmin, cmax, est, cfg, true);
                    sym_cls[row] = (uint8_t)cls;
                    atomicAdd(&hist[cls], 1);
                    if (cls % NTIER == TIER_GLOBAL) atomicMax(&wmax_glob, (unsigned long long)words);
                }
            }
        }
    }
    __syncthreads();
    // one global update per workgroup
    if (threadIdx.x < NCLS && hist[threadIdx.x]) atomicAdd(&ctl->sym_hist[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0) {
        if (empties) atomicAdd(&ctl->empty_rows, empties);
        if (nodiag) atomicAdd(&ctl->a_missing_diag, nodiag);
        if (prod_sum) atomicAdd((unsigned long long*)&ctl->products, prod_sum);
        if (wmax_all) atomicMax((unsigned long long*)&ctl->max_words_all, wmax_all);
        if (pmax) atomicMax((unsigned long long*)&ctl->max_products, pmax);
        if (wmax_glob) atomicMax((unsigned long long*)&ctl->max_words_sym_global, wmax_glob);
    }
}

// Learned binning: the 3-32-32-1 network on each row's features (weights are
// wave-uniform, so they are read as scalars) sizes the symbolic table from
// 2^(y + margin) - 1 occupied blocks.  Consecutive rows with the same
// features (a stencil's interior) share one evaluation: per pass of 256 rows
// the first row of every run of equal features takes a slot (a block scan of
// the run starts, so slots follow row order), the slots are evaluated packed
// into as few wavefronts as possible, and every row reads its run's result.
__device__ inline float mlp_eval(const float* __restrict__ w, float x0, float x1, float x2) {
    const float* W1 = w;
    const float* b1 = w + 96;
    const float* W2 = w + 128;
    const float* b2 = w + 1152;
    const float* w3 = w + 1184;
    const float b3 = w[1216];
    float h1[32];
#pragma unroll
    for (int o = 0; o < 32; ++o) {
        float z = b1[o] + W1[o * 3] * x0 + W1[o * 3 + 1] * x1 + W1[o * 3 + 2] * x2;
        h1[o] = z > 0.f ? z : 0.f;
    }
    float y = b3;
#pragma unroll 4
    for (int o = 0; o < 32; ++o) {
        float z = b2[o];
#pragma unroll
        for (int i = 0; i < 32; ++i) z += W2[o * 32 + i] * h1[i];
        y += w3[o] * (z > 0.f ? z : 0.f);
    }
    return y;
}

__global__ __launch_bounds__(256) void k_mlp_classify(int32_t m, const float* __restrict__ feats,
                                                      const float* __restrict__ w, const RowInfo* __restrict__ rinfo,
                                                      ClassCfg cfg, float margin, uint8_t* __restrict__ sym_cls,
                                                      Control* ctl) {
    __shared__ int32_t hist[NCLS];
    __shared__ unsigned long long wmax_glob;
    __shared__ float xs[3][256];      // each row's features
    __shared__ float ys[256];         // the prediction of each run (by slot)
    __shared__ int32_t wsum[4];
    if (threadIdx.x < NCLS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) wmax_glob = 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int cur = CLS_EMPTY, n_cur = 0;
    unsigned long long my_wglob = 0;
    // every thread runs the same number of passes (the barriers below)
    for (int64_t r0 = blockIdx.x * (int64_t)blockDim.x; r0 < m; r0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = r0 + tid;
        RowInfo ri = make_int4(0, 0, 0, 0);
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if (row < m) {
            ri = rinfo[row];
            x0 = feats[row * 3], x1 = feats[row * 3 + 1], x2 = feats[row * 3 + 2];
        }
        const bool valid = row < m && ri.z > 0;
        __syncthreads();  // the previous pass is done with xs and ys
        // an invalid row holds NaN, which equals nothing: the next valid row starts a run
        xs[0][tid] = valid ? x0 : __builtin_nanf(""), xs[1][tid] = x1, xs[2][tid] = x2;
        __syncthreads();
        const bool start = valid && (tid == 0 || xs[0][tid - 1] != x0 || xs[1][tid - 1] != x1 ||
                                     xs[2][tid - 1] != x2);
        // slots of the run starts in row order: block scan of the start flags
        int inc = start ? 1 : 0;
        for (int d = 1; d < 64; d <<= 1) {
            const int up = __shfl_up(inc, d, 64);
            if (lane >= d) inc += up;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();  // every start test has read xs
        int before = 0, nslots = 0;
        for (int u = 0; u < 4; ++u) {
            if (u < wv) before += wsum[u];
            nslots += wsum[u];
        }
        // the run a valid row belongs to (its own start or the latest one before it)
        const int slot = before + inc - 1;
        if (start) xs[0][slot] = x0, xs[1][slot] = x1, xs[2][slot] = x2;  // slot <= tid
        __syncthreads();
        // the runs' features evaluated packed from thread 0
        if (tid < nslots) ys[tid] = mlp_eval(w, xs[0][tid], xs[1][tid], xs[2][tid]);
        __syncthreads();
        if (valid) {
            // a valid row that starts no run continues the run of a valid row before it
            const float y = ys[slot];
            float e = exp2f(fminf(y + margin, 40.f)) - 1.f;
            int64_t est = e < 1.f ? 1 : (int64_t)ceilf(e);
            int cls = sym_class(ri.z, ri.x, ri.y, est, cfg);
            sym_cls[row] = (uint8_t)cls;
            if (cls != cur) {
                if (n_cur) atomicAdd(&hist[cur], n_cur);
                cur = cls, n_cur = 0;
            }
            n_cur += 1;
            if (cls % NTIER == TIER_GLOBAL) my_wglob = max(my_wglob, (unsigned long long)row_words(ri.x, ri.y));
        }
    }
    if (n_cur) atomicAdd(&hist[cur], n_cur);
    if (my_wglob) atomicMax(&wmax_glob, my_wglob);
    __syncthreads();
    if (threadIdx.x < NCLS && hist[threadIdx.x]) atomicAdd(&ctl->sym_hist[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0 && wmax_glob) atomicMax((unsigned long long*)&ctl->max_words_sym_global, wmax_glob);
}

// Status word of a decoupled look-back: 2 flag bits over a 62-bit value.
constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_PRE = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;

// Groups rows by class, each class in ascending row order up to the order
// inside a chunk: a workgroup takes chunks of 2048 consecutive rows by
// ticket, ranks each row inside its class with LDS atomics, and finds the
// chunk's range in every class from the counts of the chunks before it (a
// decoupled look-back per class over the chunks in ticket order), then
// writes the row ids there, with each row's descriptor {row, A start, A end,
// C start (or list offset)} beside it.  The order matters for speed: the
// row kernels take their rows in this order, so rows that share B rows run
// close together and, where row index and row size go together (R-MAT), the
// longest rows start first.  For the symbolic rows it also places the rows'
// lists: a scan of the chunk's capacities and one global atomic for the
// chunk's range.  state: the ticket, then a status word per chunk and class
// (scatter_state_bytes, all zero on entry).
constexpr int SCATTER_ITEMS = 8;
constexpr int SCATTER_CHUNK = 256 * SCATTER_ITEMS;
__global__ __launch_bounds__(256) void k_scatter(int32_t m, const uint8_t* __restrict__ cls, int merge,
                                                 const int32_t* __restrict__ hist, int32_t* __restrict__ state,
                                                 int32_t* __restrict__ perm, const int32_t* __restrict__ arp,
                                                 const int32_t* __restrict__ crp, int4* __restrict__ desc,
                                                 int32_t* __restrict__ lofs, Control* ctl, int64_t list_limit) {
    __shared__ int32_t cnt[NCLS];
    __shared__ int32_t base[NCLS];
    __shared__ int32_t off[NCLS];
    __shared__ int64_t wsum[4];
    __shared__ int64_t lbase;
    __shared__ uint8_t remap[NCLS];
    __shared__ int32_t chunk_sh;
    int32_t* ticket = state;
    uint64_t* status = reinterpret_cast<uint64_t*>(state + 16);
    if (threadIdx.x == 0) {
        int32_t h[NCLS], merged[NCLS];
        for (int c = 0; c < NCLS; ++c) h[c] = hist[c];
        merge_classes(h, remap, merged, merge != 0);
        if (lofs) {
            // symbolic rows tier-major (a persistent launch per tier takes its
            // three modes as one range); the first workgroup publishes the ranges
            sym_class_offsets(merged, off);
            if (blockIdx.x == 0)
                for (int c = 0; c < NCLS; ++c) ctl->sym_cnt[c] = merged[c], ctl->sym_off[c] = off[c];
        } else {
            int32_t run = 0;
            for (int c = 0; c < NCLS; ++c) off[c] = run, run += merged[c];
        }
    }
    const int64_t nchunks = ((int64_t)m + SCATTER_CHUNK - 1) / SCATTER_CHUNK;
    for (;;) {
        if (threadIdx.x < NCLS) cnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) chunk_sh = atomicAdd(ticket, 1);
        __syncthreads();
        const int64_t chunk = chunk_sh;
        if (chunk >= nchunks) break;  // uniform
        const int64_t r0 = chunk * SCATTER_CHUNK;
        // the chunk's inputs first, as unconditional loads (a row past the end
        // reads the last row's, unused; arp has m + 1 entries): a load under a
        // condition would be waited for before the next one is issued
        uint8_t raw[SCATTER_ITEMS];
        int32_t lraw[SCATTER_ITEMS], a_lo[SCATTER_ITEMS], a_hi[SCATTER_ITEMS], cw[SCATTER_ITEMS];
#pragma unroll
        for (int t = 0; t < SCATTER_ITEMS; ++t) {
            const int64_t row = r0 + t * 256 + threadIdx.x;
            const int64_t rr = row < m ? row : m - 1;
            raw[t] = cls[rr];
            a_lo[t] = arp[rr];
            a_hi[t] = arp[rr + 1];
            lraw[t] = lofs ? lofs[rr] : 0;
            cw[t] = crp ? crp[rr] : 0;
        }
        int c[SCATTER_ITEMS], local[SCATTER_ITEMS];
#pragma unroll
        for (int t = 0; t < SCATTER_ITEMS; ++t) {
            const int64_t row = r0 + t * 256 + threadIdx.x;
            c[t] = row < m ? raw[t] : CLS_EMPTY;
            if (c[t] != CLS_EMPTY) c[t] = remap[c[t]];
            local[t] = c[t] != CLS_EMPTY ? atomicAdd(&cnt[c[t]], 1) : 0;
        }
        // list capacities of the chunk (rows of the global path get none)
        int32_t cap[SCATTER_ITEMS];
        int64_t lsum = 0;
#pragma unroll
        for (int t = 0; t < SCATTER_ITEMS; ++t) {
            cap[t] = 0;
            if (lofs && c[t] != CLS_EMPTY && c[t] % NTIER != TIER_GLOBAL) cap[t] = lraw[t];
            lsum += cap[t];
        }
        int64_t lex = 0;
        if (lofs) {
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            int64_t x = lsum;
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            if (lane == 63) wsum[wv] = x;
            __syncthreads();
            int64_t pre = 0, tot = 0;
            for (int u = 0; u < 4; ++u) {
                if (u < wv) pre += wsum[u];
                tot += wsum[u];
            }
            lex = pre + x - lsum;
            if (threadIdx.x == 0) lbase = tot ? (int64_t)atomicAdd((unsigned long long*)&ctl->list_total,
                                                                   (unsigned long long)tot)
                                              : 0;
        }
        __syncthreads();
        if (threadIdx.x < NCLS) {
            // the chunk's start in class c: the counts of every chunk before it
            // (chunks are taken in ticket order, so each one waited for is
            // resident or finished and the wait ends)
            const int c = threadIdx.x;
            const uint64_t agg = (uint32_t)cnt[c];
            uint64_t* mine = status + chunk * NCLS + c;
            int64_t prefix = 0;
            if (chunk == 0) {
                __hip_atomic_store(mine, ST_PRE | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(mine, ST_AGG | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int64_t t = chunk - 1; t >= 0; --t) {
                    uint64_t w;
                    do {
                        w = __hip_atomic_load(status + t * NCLS + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } while ((w >> 62) == 0);
                    prefix += (int64_t)(w & ST_VAL);
                    if ((w >> 62) == 2) break;
                }
                __hip_atomic_store(mine, ST_PRE | (uint64_t)(prefix + (int64_t)agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            base[c] = (int32_t)prefix;
        }
        __syncthreads();
        int64_t lpos = lofs ? lbase + lex : 0;
#pragma unroll
        for (int t = 0; t < SCATTER_ITEMS; ++t) {
            if (c[t] == CLS_EMPTY) continue;
            const int32_t row = (int32_t)(r0 + t * 256 + threadIdx.x);
            const int32_t pos = off[c[t]] + base[c[t]] + local[t];
            int32_t w = cw[t];
            if (lofs) {
                w = cap[t] > 0 && lpos + cap[t] <= list_limit ? (int32_t)lpos : -1;
                lofs[row] = w;
                lpos += cap[t];
            }
            perm[pos] = row;
            desc[pos] = make_int4(row, a_lo[t], a_hi[t], w);
        }
        __syncthreads();
    }
}

// Row pointer = exclusive prefix sum of row_nnz, in 64-bit, single pass with
// decoupled look-back over tiles taken in launch order.  Also assigns each
// row's numeric class (its exact size is now known; rows without a list take
// the global path) and counts rows whose symbolic class differed from the
// class their true size asks for.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(int32_t m, const int32_t* __restrict__ row_nnz,
                                                       const int32_t* __restrict__ row_blocks,
                                                       const RowInfo* __restrict__ rinfo,
                                                       const int32_t* __restrict__ arp,
                                                       const uint8_t* __restrict__ sym_cls,
                                                       const int32_t* __restrict__ lofs,
                                                       int32_t* __restrict__ c_row_ptr, uint64_t* tile_status,
                                                       ClassCfg cfg, uint8_t* __restrict__ num_cls, Control* ctl) {
    __shared__ int32_t tile_sh;
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    __shared__ int64_t tile_prefix;
    __shared__ int32_t hist[NCLS];
    __shared__ unsigned long long s_annz[NCLS], s_cnnz[NCLS], s_prod[NCLS];
    __shared__ int32_t mispred;
    __shared__ unsigned long long wmax_glob;
    if (threadIdx.x == 0) tile_sh = atomicAdd(&ctl->tile_counter, 1), mispred = 0, wmax_glob = 0;
    if (threadIdx.x < NCLS) hist[threadIdx.x] = 0, s_annz[threadIdx.x] = 0, s_cnnz[threadIdx.x] = 0,
                                    s_prod[threadIdx.x] = 0;
    __syncthreads();
    const int tile = tile_sh;
    const int64_t r0 = (int64_t)tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
    // every row's inputs first, as unconditional loads (a row past the end
    // reads the last row's, unused; arp has m + 1 entries): a load under a
    // condition would be waited for before the next one is issued
    int32_t nz[SCAN_ITEMS], bl[SCAN_ITEMS], lo[SCAN_ITEMS], ap[SCAN_ITEMS + 1];
    RowInfo rf[SCAN_ITEMS];
    uint8_t sc[SCAN_ITEMS];
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        const int64_t rr = r0 + t < m ? r0 + t : m - 1;
        nz[t] = row_nnz[rr];
        rf[t] = rinfo[rr];
        bl[t] = row_blocks[rr];
        lo[t] = lofs[rr];
        sc[t] = sym_cls[rr];
    }
#pragma unroll
    for (int t = 0; t <= SCAN_ITEMS; ++t) ap[t] = arp[r0 + t < m ? r0 + t : m];
    // the thread's consecutive rows of one class are counted in registers and
    // added to the workgroup's counters once per run of equal classes
    int cur = CLS_EMPTY, n_cur = 0, miss = 0;
    unsigned long long a_cur = 0, c_cur = 0, p_cur = 0;
    auto flush = [&]() {
        if (cur == CLS_EMPTY) return;
        atomicAdd(&hist[cur], n_cur);
        atomicAdd(&s_annz[cur], a_cur);
        atomicAdd(&s_cnnz[cur], c_cur);
        atomicAdd(&s_prod[cur], p_cur);
    };
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        int64_t r = r0 + t;
        int64_t c = 0;
        if (r < m) {
            c = nz[t];
            const RowInfo ri = rf[t];
            const int blocks = bl[t];
            int nc = num_class(ri.z, ri.x, ri.y, c, blocks, cfg);
            // a row kernel builds its table from the row's list: without one, the global path
            if (nc != CLS_EMPTY && nc % NTIER != TIER_GLOBAL && lo[t] < 0) nc = MODE_DIRECT * NTIER + TIER_GLOBAL;
            num_cls[r] = (uint8_t)nc;
            if (nc != CLS_EMPTY) {
                if (nc != cur) {
                    flush();
                    cur = nc, n_cur = 0, a_cur = c_cur = p_cur = 0;
                }
                n_cur += 1;
                a_cur += (unsigned long long)(ap[t + 1] - ap[t]);
                c_cur += (unsigned long long)c;
                p_cur += (unsigned long long)ri.z;
                if (nc % NTIER == TIER_GLOBAL) atomicMax(&wmax_glob, (unsigned long long)row_words(ri.x, ri.y));
                // the class the exact size asks for, under the same sizing rule as the estimate's
                miss += sym_class(ri.z, ri.x, ri.y, blocks, cfg, cfg.bound_est != 0) != sc[t];
            }
        }
        run += c;
        v[t] = run;
    }
    flush();
    if (miss) atomicAdd(&mispred, miss);
    // block scan of the per-thread totals
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t x = run;
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int64_t wpre = 0, agg = 0;
    for (int u = 0; u < SCAN_THREADS / 64; ++u) {
        if (u < wv) wpre += wsum[u];
        agg += wsum[u];
    }
    const int64_t thread_excl = wpre + x - run;
    // decoupled look-back: publish the aggregate, then add predecessors
    if (threadIdx.x == 0) {
        int64_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(&tile_status[0], ST_PRE | (uint64_t)agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&tile_status[tile], ST_AGG | (uint64_t)agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            // tiles are numbered in the order they started, so every predecessor
            // is resident or finished and each wait below ends
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
    }
    __syncthreads();
    const int64_t base = tile_prefix + thread_excl;
    bool ovf = false;
#pragma unroll
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        int64_t r = r0 + t;
        if (r < m) {
            int64_t val = base + v[t];
            if (val > INT_MAX) ovf = true;
            c_row_ptr[r + 1] = (int32_t)val;
            if (r == m - 1) ctl->nnz_c = val;
        }
    }
    if (tile == 0 && threadIdx.x == 0) c_row_ptr[0] = 0;
    if (ovf) atomicOr(&ctl->err, ERR_NNZ_OVERFLOW);
    __syncthreads();
    if (threadIdx.x < NCLS && hist[threadIdx.x]) {
        atomicAdd(&ctl->num_hist[threadIdx.x], hist[threadIdx.x]);
        atomicAdd((unsigned long long*)&ctl->num_a_nnz[threadIdx.x], s_annz[threadIdx.x]);
        atomicAdd((unsigned long long*)&ctl->num_c_nnz[threadIdx.x], s_cnnz[threadIdx.x]);
        atomicAdd((unsigned long long*)&ctl->num_products[threadIdx.x], s_prod[threadIdx.x]);
    }
    if (threadIdx.x == 0 && mispred) atomicAdd(&ctl->mispredicted, mispred);
    if (threadIdx.x == 0 && wmax_glob) atomicMax((unsigned long long*)&ctl->max_words_num_global, wmax_glob);
}

__global__ void k_export_rows(int32_t m, const float* __restrict__ feats, const int32_t* __restrict__ row_blocks,
                              const int32_t* __restrict__ row_nnz_in, float* __restrict__ x, float* __restrict__ y,
                              int32_t* __restrict__ row_nnz_out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    x[r * 3] = feats[r * 3];
    x[r * 3 + 1] = feats[r * 3 + 1];
    x[r * 3 + 2] = feats[r * 3 + 2];
    y[r] = log2f(1.0f + (float)row_blocks[r]);
    if (row_nnz_out) row_nnz_out[r] = row_nnz_in[r];
}


// Batched products as one block-diagonal product: product p's rows are
// appended to the packed row pointer (entry offsets made global) and, for A,
// its column indices are shifted by the number of B rows before it so they
// address its own B rows.  B's columns stay local: a row of C only ever
// meets the columns of its own product's B.  Each product's local arrays are
// checked (row pointer from 0 to its nnz, columns below its own width).
__global__ __launch_bounds__(256) void k_pack(int32_t count, const int64_t* __restrict__ desc,
                                              const int32_t* __restrict__ rp_pool,
                                              const int32_t* __restrict__ col_pool, int32_t* __restrict__ rp_out,
                                              int32_t* __restrict__ col_out, int32_t* __restrict__ err) {
    // desc per product: row offset, row-pointer offset, nnz offset, rows, nnz, column shift, column limit
    for (int p = blockIdx.x; p < count; p += gridDim.x) {
        const int64_t* d = desc + 7 * (int64_t)p;
        const int64_t roff = d[0], rpoff = d[1], noff = d[2], rows = d[3], nnz = d[4], shift = d[5], lim = d[6];
        int bad = 0;
        if (threadIdx.x == 0 && (rp_pool[rpoff] != 0 || (int64_t)rp_pool[rpoff + rows] != nnz)) bad = 1;
        for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
            const int32_t v = rp_pool[rpoff + r];
            if (v < 0 || (int64_t)v > nnz || v > rp_pool[rpoff + r + 1]) bad = 1;
            rp_out[roff + r] = (int32_t)(noff + v);
        }
        for (int64_t q = threadIdx.x; q < nnz; q += blockDim.x) {
            const int32_t c = col_pool[noff + q];
            if (c < 0 || (int64_t)c >= lim) bad = 1;
            if (col_out) col_out[noff + q] = (int32_t)(c + shift);
        }
        if (bad) atomicOr(err, 1);
    }
}

// Reduction over an aligned group of 8 lanes: quad swaps, then the half-row
// mirror (lane i with lane 7 - i), after which every lane holds the result.
template <typename Op>
__device__ inline int row8_reduce(int v, Op op) {
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, false));  // row_half_mirror
    return v;
}

// B rows in one pass, ROW_LANES lanes per row reading it in coalesced chunks:
// the row pointer and the columns are checked; the row's length, smallest
// and largest column go to binfo; and the row is compressed (section 2.2.1):
// every run of consecutive entries that share a 32-column block becomes one
// {block, OR of the column bits} entry.  A row has at most as many runs as
// entries, so its runs are stored from the row's own first entry on (no scan
// places them), and the header {first entry, length, first run, run count}
// and binfo's run count follow.  An entry starts a run when its block differs
// from the previous entry's; a segmented OR across the chunk gathers each
// run's bits, and the lane holding a run's last entry writes it at the run's
// index (runs begun before it in the row).  A malformed row gets length and
// runs 0 and raises the error flag, on which every later kernel exits.
__global__ __launch_bounds__(256) void k_b_rows(int32_t n, int32_t k, const int32_t* __restrict__ brp,
                                                const int32_t* __restrict__ bci, int64_t bnnz, int4* __restrict__ binfo,
                                                int2* __restrict__ bc, int4* __restrict__ bhdr, Control* ctl) {
    constexpr int L = ROW_LANES;
    static_assert(L == 8, "the DPP shifts and swizzles below assume 8-lane groups");
    __shared__ unsigned long long runs_sum;
    if (threadIdx.x == 0) runs_sum = 0;
    __syncthreads();
    const int sl = threadIdx.x % L;
    const int shift = (threadIdx.x & 63) & ~(L - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / L;
    for (int64_t j = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / L; j < n; j += stride) {
        const int32_t s = brp[j], e = brp[j + 1];
        int bad = 0;
        if (s < 0 || e < s || (int64_t)e > bnnz || (j == 0 && s != 0) || (j == n - 1 && (int64_t)e != bnnz))
            bad = ERR_B_ROWPTR;
        int done = 0;          // runs begun in earlier chunks
        int mn = INT_MAX, mx = -1;
        uint32_t carry = 0;    // bits of the run still open at the end of the last chunk
        int last_blk = -1;     // block of the last chunk's final entry
        // four chunks' entries (and the entry after each chunk) are loaded at once
        for (int32_t Q0 = s; !bad && Q0 < e; Q0 += 4 * L) {
            // unconditional loads, indices clamped into the row (a load under
            // a condition would be waited for before the next one is issued);
            // entries past the row's end are not used
            int cc[4], nx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t q = Q0 + u * L + sl;
                cc[u] = bci[min(q, e - 1)];
                nx[u] = bci[min(q + 1, e - 1)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
            const int32_t q0 = Q0 + u * L;
            if (q0 >= e) break;  // uniform in the row's lanes
            const int32_t q = q0 + sl;
            const bool v = q < e;
            const int c = cc[u];
            if (v) {
                if (c < 0 || c >= k) bad = ERR_B_COL;
                mn = min(mn, c);
                mx = max(mx, c);
            }
            const int blk = v ? c >> 5 : -1;
            // neighbours inside the 8-lane group: DPP row shifts (a group is an
            // aligned half of a 16-lane row; the lanes whose neighbour lies
            // outside the group take it from elsewhere)
            int prev = __builtin_amdgcn_mov_dpp(blk, 0x111, 0xf, 0xf, false);  // row_shr:1
            if (sl == 0) prev = last_blk;
            int next = __builtin_amdgcn_mov_dpp(blk, 0x101, 0xf, 0xf, false);  // row_shl:1
            if (sl == L - 1) next = q + 1 < e ? nx[u] >> 5 : -1;
            const int start = v && blk != prev;
            const bool last = v && (q + 1 >= e || next != blk);
            // segmented inclusive OR of the column bits, segments begin at run starts
            uint32_t m = v ? 1u << (c & 31) : 0u;
            int f = start;
            const auto seg_step = [&](uint32_t mu, int fu, int d) {
                if (sl >= d && !f) {
                    m |= mu;
                    f = fu;
                }
            };
            seg_step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x111, 0xf, 0xf, false),
                     __builtin_amdgcn_mov_dpp(f, 0x111, 0xf, 0xf, false), 1);  // row_shr:1
            seg_step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x112, 0xf, 0xf, false),
                     __builtin_amdgcn_mov_dpp(f, 0x112, 0xf, 0xf, false), 2);  // row_shr:2
            seg_step((uint32_t)__builtin_amdgcn_mov_dpp((int)m, 0x114, 0xf, 0xf, false),
                     __builtin_amdgcn_mov_dpp(f, 0x114, 0xf, 0xf, false), 4);  // row_shr:4
            if (!f) m |= carry;
            const uint64_t starts = (__ballot(start) >> shift) & ((1ull << L) - 1);
            const int idx = done + __popcll(starts & ((2ull << sl) - 1)) - 1;
            if (last) bc[s + idx] = make_int2(blk, (int)m);
            done += __popcll(starts);
            // lane 7 of each group to the whole group: swizzle lane -> (lane & 0x18) | 7
            carry = (uint32_t)__builtin_amdgcn_ds_swizzle((int)m, 0xF8);
            last_blk = __builtin_amdgcn_ds_swizzle(blk, 0xF8);
            }
            bad = row8_reduce(bad, [](int x, int y) { return x | y; });
        }
        mn = row8_reduce(mn, [](int x, int y) { return min(x, y); });
        mx = row8_reduce(mx, [](int x, int y) { return max(x, y); });
        if (sl == 0) {
            if (bad) {
                atomicOr(&ctl->err, bad);
                binfo[j] = make_int4(0, INT_MAX, -1, 0);
                bhdr[j] = make_int4(0, 0, 0, 0);
            } else {
                binfo[j] = make_int4(e - s, mn, mx, done);
                bhdr[j] = make_int4(s, e - s, s, done);
                if (done) atomicAdd(&runs_sum, (unsigned long long)done);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && runs_sum) atomicAdd((unsigned long long*)&ctl->bc_total, runs_sum);
}

inline unsigned grid_for(int64_t threads, int per_block) {
    int64_t g = (threads + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int64_t scan_tiles(int32_t m) { return ((int64_t)m + SCAN_TILE - 1) / SCAN_TILE; }

void launch_pack(hipStream_t s, int32_t count, const int64_t* desc, const int32_t* rp_pool, const int32_t* col_pool,
                 int32_t* rp_out, int32_t* col_out, int32_t* err) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)std::min(count, 4096)), dim3(256), 0, s, count, desc, rp_pool, col_pool,
                       rp_out, col_out, err);
}

void launch_fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
}

void launch_fill_u8(hipStream_t s, void* p, uint8_t v, int64_t bytes) {
    if (bytes <= 0) return;
    int64_t g = (bytes + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)g), dim3(256), 0, s, (uint8_t*)p, v, bytes);
}

void launch_b_rows(hipStream_t s, int32_t n, int32_t k, const int32_t* brp, const int32_t* bci, int64_t bnnz,
                   int4* binfo, int2* bc, int4* bhdr, Control* ctl) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_b_rows, dim3(std::min(grid_for((int64_t)n * ROW_LANES, 256), 4096u)), dim3(256), 0, s, n, k,
                       brp, bci, bnnz, binfo, bc, bhdr, ctl);
}

void launch_a_rowinfo(hipStream_t s, int32_t m, int32_t n, const int32_t* arp, const int32_t* aci, int64_t annz,
                      const int4* binfo, RowInfo* rinfo, float* feats, ClassCfg cfg, int binning,
                      uint8_t* sym_cls, int32_t* row_nnz, int32_t* row_blocks, int32_t* lofs, Control* ctl) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_a_rowinfo, dim3(std::min(grid_for((int64_t)m * AN_LANES, 256), 4096u)), dim3(256), 0, s, m, n,
                       arp, aci, annz, binfo, rinfo, feats, cfg, binning, sym_cls, row_nnz, row_blocks, lofs, ctl);
}

void launch_mlp_classify(hipStream_t s, int32_t m, const float* feats, const float* w, const RowInfo* rinfo,
                         ClassCfg cfg, float margin, uint8_t* sym_cls, Control* ctl) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_mlp_classify, dim3(std::min(grid_for(m, 256), 1024u)), dim3(256), 0, s, m, feats, w, rinfo,
                       cfg, margin,
                       sym_cls, ctl);
}

size_t scatter_state_bytes(int32_t m) {
    return 64 + (size_t)(((int64_t)std::max(m, 0) + SCATTER_CHUNK - 1) / SCATTER_CHUNK) * NCLS * 8;
}

void launch_scatter(hipStream_t s, int32_t m, const uint8_t* cls, int merge, const int32_t* hist, int32_t* state,
                    int32_t* perm, const int32_t* arp, const int32_t* crp, int4* desc, int32_t* lofs, Control* ctl,
                    int64_t list_limit) {
    if (m <= 0) return;
    launch_fill_u8(s, state, 0, (int64_t)scatter_state_bytes(m));
    hipLaunchKernelGGL(k_scatter, dim3(std::min(grid_for(m, SCATTER_CHUNK), 1024u)), dim3(256), 0, s, m, cls, merge,
                       hist, state, perm, arp, crp, desc, lofs, ctl, list_limit);
}

void launch_scan(hipStream_t s, int32_t m, const int32_t* row_nnz, const int32_t* row_blocks, const RowInfo* rinfo,
                 const int32_t* arp, const uint8_t* sym_cls, const int32_t* lofs, int32_t* c_row_ptr,
                 uint64_t* tile_status, ClassCfg cfg, uint8_t* num_cls, Control* ctl) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)scan_tiles(m)), dim3(SCAN_THREADS), 0, s, m, row_nnz, row_blocks,
                       rinfo, arp, sym_cls, lofs, c_row_ptr, tile_status, cfg, num_cls, ctl);
}

void launch_export_rows(hipStream_t s, int32_t m, const float* feats, const int32_t* row_blocks,
                        const int32_t* row_nnz_in, float* x, float* y, int32_t* row_nnz_out) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_export_rows, dim3(grid_for(m, 256)), dim3(256), 0, s, m, feats, row_blocks, row_nnz_in, x,
                       y, row_nnz_out);
}

}  // namespace spg
