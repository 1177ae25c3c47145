// Learned row-size predictor: a 3-32-32-1 ReLU network in FP32.
//
// The paper sizes work per matrix from FLOPs per row (section 2.2.1); here a
// small regressor predicts, per row, log2(1 + occupied 32-column blocks of
// C's row) from three symbolic-phase features (log2 of one plus: A's row
// length, the sum and the max of the referenced B row lengths), so the
// symbolic table can be sized from the prediction instead of the upper bound.
//
// Parameter layout (1217 floats): W1[32][3], b1[32], W2[32][32], b2[32],
// w3[32], b3.  Forward keeps z1 and z2 per row for backward.  Backward
// accumulates per-workgroup partial gradients over tiles of rows held in LDS,
// then a second kernel sums the partials in a fixed order (deterministic).
// Training is minibatch Adam on the mean squared error or a pinball loss.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "spg_internal.h"

namespace {

constexpr int H = 32;
constexpr int NW = 1217;
constexpr int OFF_B1 = 96, OFF_W2 = 128, OFF_B2 = 1152, OFF_W3 = 1184, OFF_B3 = 1216;
constexpr int TILE = 64;          // rows per backward tile
constexpr int BWD_THREADS = 256;
constexpr int PER_THREAD = (NW + BWD_THREADS - 1) / BWD_THREADS;

__global__ __launch_bounds__(256) void k_fwd(const float* __restrict__ w, const float* __restrict__ x, int32_t rows,
                                             float* __restrict__ y, float* __restrict__ act) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const float x0 = x[r * 3], x1 = x[r * 3 + 1], x2 = x[r * 3 + 2];
    float h1[H];
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float z = w[OFF_B1 + o] + w[o * 3] * x0 + w[o * 3 + 1] * x1 + w[o * 3 + 2] * x2;
        if (act) act[r * 64 + o] = z;
        h1[o] = z > 0.f ? z : 0.f;
    }
    float out = w[OFF_B3];
#pragma unroll 4
    for (int o = 0; o < H; ++o) {
        float z = w[OFF_B2 + o];
#pragma unroll
        for (int i = 0; i < H; ++i) z += w[OFF_W2 + o * H + i] * h1[i];
        if (act) act[r * 64 + 32 + o] = z;
        out += w[OFF_W3 + o] * (z > 0.f ? z : 0.f);
    }
    y[r] = out;
}

// Partial gradient of sum_r dy[r] * y[r] over this workgroup's row tiles.
__global__ __launch_bounds__(BWD_THREADS) void k_bwd_partial(const float* __restrict__ w, const float* __restrict__ x,
                                                             const float* __restrict__ act,
                                                             const float* __restrict__ dy, int32_t rows,
                                                             float* __restrict__ partial) {
    __shared__ float sx[TILE][3];
    __shared__ float sh1[TILE][H + 1];
    __shared__ float sdz1[TILE][H + 1];
    __shared__ float sdz2[TILE][H + 1];
    __shared__ float sh2[TILE][H + 1];
    __shared__ float sdy[TILE];
    float acc[PER_THREAD];
#pragma unroll
    for (int t = 0; t < PER_THREAD; ++t) acc[t] = 0.f;
    const int tid = threadIdx.x;
    const int ntiles = (rows + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int r0 = tile * TILE;
        if (tid < TILE) {
            const int64_t r = r0 + tid;
            if (r < rows) {
                const float g = dy[r];
                float z1[H], z2[H], dz2[H];
                for (int o = 0; o < H; ++o) z1[o] = act[r * 64 + o], z2[o] = act[r * 64 + 32 + o];
                for (int i = 0; i < 3; ++i) sx[tid][i] = x[r * 3 + i];
                for (int o = 0; o < H; ++o) {
                    sh1[tid][o] = z1[o] > 0.f ? z1[o] : 0.f;
                    sh2[tid][o] = z2[o] > 0.f ? z2[o] : 0.f;
                    dz2[o] = z2[o] > 0.f ? g * w[OFF_W3 + o] : 0.f;
                    sdz2[tid][o] = dz2[o];
                }
                for (int i = 0; i < H; ++i) {
                    float s = 0.f;
                    for (int o = 0; o < H; ++o) s += w[OFF_W2 + o * H + i] * dz2[o];
                    sdz1[tid][i] = z1[i] > 0.f ? s : 0.f;
                }
                sdy[tid] = g;
            } else {
                for (int i = 0; i < 3; ++i) sx[tid][i] = 0.f;
                for (int o = 0; o < H; ++o) sh1[tid][o] = sh2[tid][o] = sdz1[tid][o] = sdz2[tid][o] = 0.f;
                sdy[tid] = 0.f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER_THREAD; ++t) {
            const int p = tid + t * BWD_THREADS;
            if (p >= NW) break;
            float s = 0.f;
            if (p < OFF_B1) {
                const int o = p / 3, i = p % 3;
                for (int r = 0; r < TILE; ++r) s += sdz1[r][o] * sx[r][i];
            } else if (p < OFF_W2) {
                const int o = p - OFF_B1;
                for (int r = 0; r < TILE; ++r) s += sdz1[r][o];
            } else if (p < OFF_B2) {
                const int o = (p - OFF_W2) / H, i = (p - OFF_W2) % H;
                for (int r = 0; r < TILE; ++r) s += sdz2[r][o] * sh1[r][i];
            } else if (p < OFF_W3) {
                const int o = p - OFF_B2;
                for (int r = 0; r < TILE; ++r) s += sdz2[r][o];
            } else if (p < OFF_B3) {
                const int o = p - OFF_W3;
                for (int r = 0; r < TILE; ++r) s += sdy[r] * sh2[r][o];
            } else {
                for (int r = 0; r < TILE; ++r) s += sdy[r];
            }
            acc[t] += s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < PER_THREAD; ++t) {
        const int p = tid + t * BWD_THREADS;
        if (p < NW) partial[(int64_t)blockIdx.x * NW + p] = acc[t];
    }
}

__global__ void k_reduce_partials(const float* __restrict__ partial, int nblocks, float* __restrict__ dw) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NW) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * NW + p];
    dw[p] = s;
}

// Loss gradient with respect to the predictions, for the batch mean:
//   squared error (q == 0): dy = 2 (y - t) / rows, loss (y - t)^2
//   pinball of level q:     d = t - y, loss q d (d >= 0) or (q - 1) d,
//                           dy = -q / rows (d > 0) or (1 - q) / rows (d <= 0)
// loss[0] += sum of row losses * loss_scale
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int32_t rows,
                                              float q, float* __restrict__ dy, float* __restrict__ loss,
                                              float loss_scale) {
    __shared__ float red[256];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (r < rows) {
        if (q == 0.f) {
            const float d = y[r] - t[r];
            dy[r] = 2.f * d / (float)rows;
            e = d * d;
        } else {
            const float d = t[r] - y[r];
            dy[r] = (d > 0.f ? -q : 1.f - q) / (float)rows;
            e = d >= 0.f ? q * d : (q - 1.f) * d;
        }
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] * loss_scale);
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NW) return;
    const float gp = g[p];
    const float mp = 0.9f * m[p] + 0.1f * gp;
    const float vp = 0.999f * v[p] + 0.001f * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + 1e-8f);
}

__global__ void k_zero(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

constexpr int MAX_BWD_BLOCKS = 256;  // backward grid cap (row tiles are strided over it)

int bwd_blocks(int32_t rows) {
    int t = (rows + TILE - 1) / TILE;
    return t < 1 ? 1 : (t > MAX_BWD_BLOCKS ? MAX_BWD_BLOCKS : t);
}

// Partial gradients of spg_mlp_backward_noalloc: one slice of NW floats per
// backward workgroup (1.19 MiB), held by every device the library runs on
// until the process ends.  Host code never passes this name to a kernel: it
// is a host-side stand-in; the device address comes from scratch_address().
constexpr size_t SCRATCH_FLOATS = (size_t)MAX_BWD_BLOCKS * NW;
static __device__ __align__(256) float scratch[SCRATCH_FLOATS];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
spg_status scratch_address(float** out) {
    static std::mutex mu;
    static float* addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return SPG_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SPG_ERR_HIP;
        }
        addr[dev] = static_cast<float*>(p);
    }
    *out = addr[dev];
    return SPG_OK;
}

spg_status launch_backward(hipStream_t s, const float* w, const float* x, const float* act, const float* dy,
                           int32_t rows, float* dw, float* partial) {
    const int nb = bwd_blocks(rows);
    hipLaunchKernelGGL(k_bwd_partial, dim3(nb), dim3(BWD_THREADS), 0, s, w, x, act, dy, rows, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3((NW + 255) / 256), dim3(256), 0, s, partial, nb, dw);
    return hipGetLastError() == hipSuccess ? SPG_OK : SPG_ERR_HIP;
}

}  // namespace

extern "C" {

spg_status spg_mlp_forward(void* stream, const float* w, const float* x, int32_t rows, float* y, float* act) {
    if (rows < 0 || (rows > 0 && (!w || !x || !y))) return SPG_ERR_ARG;
    if (rows == 0) return SPG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fwd, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, w, x, rows, y, act);
    return hipGetLastError() == hipSuccess ? SPG_OK : SPG_ERR_HIP;
}

spg_status spg_mlp_backward(void* stream, const float* w, const float* x, const float* act, const float* dy,
                            int32_t rows, float* dw) {
    if (rows < 0 || !w || !dw || (rows > 0 && (!x || !act || !dy))) return SPG_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* partial = nullptr;
    const int nb = bwd_blocks(rows);
    if (hipMallocAsync((void**)&partial, (size_t)nb * NW * sizeof(float), s) != hipSuccess) {
        (void)hipGetLastError();
        return SPG_ERR_ALLOC;
    }
    spg_status st = launch_backward(s, w, x, act, dy, rows, dw, partial);
    if (hipFreeAsync(partial, s) != hipSuccess) st = SPG_ERR_HIP;
    return st;
}

spg_status spg_mlp_backward_noalloc(void* stream, const float* w, const float* x, const float* act,
                                    const float* dy, int32_t rows, float* dw) {
    if (rows < 0 || !w || !dw || (rows > 0 && (!x || !act || !dy))) return SPG_ERR_ARG;
    const int nb = bwd_blocks(rows);
    if ((size_t)nb * NW > SCRATCH_FLOATS) return SPG_ERR_ARG;  // cannot happen: the grid is capped
    float* partial = nullptr;
    spg_status st = scratch_address(&partial);
    if (st != SPG_OK) return st;
    // every workgroup of the backward grid writes its whole slice and the
    // reduction reads only those slices: nothing needs clearing first
    return launch_backward(static_cast<hipStream_t>(stream), w, x, act, dy, rows, dw, partial);
}

spg_status spg_mlp_train(void* stream, const float* x, const float* y, int32_t rows, int32_t epochs, int32_t batch,
                         float lr, float quantile, float* w_inout, float* loss_out) {
    if (rows <= 0 || epochs < 0 || batch <= 0 || !x || !y || !w_inout || !(lr > 0.f)) return SPG_ERR_ARG;
    if (!(quantile >= 0.f && quantile < 1.f)) return SPG_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t bmax = batch < rows ? batch : rows;
    const int nb = bwd_blocks(bmax);
    // scratch: activations, predictions, dy, partials, gradient, Adam moments
    const size_t floats = (size_t)bmax * 64 + 2 * (size_t)bmax + (size_t)nb * NW + 3 * (size_t)NW;
    float* buf = nullptr;
    if (hipMallocAsync((void**)&buf, floats * sizeof(float), s) != hipSuccess) {
        (void)hipGetLastError();
        return SPG_ERR_ALLOC;
    }
    float* act = buf;
    float* yp = act + (size_t)bmax * 64;
    float* dy = yp + bmax;
    float* partial = dy + bmax;
    float* g = partial + (size_t)nb * NW;
    float* m = g + NW;
    float* v = m + NW;
    hipLaunchKernelGGL(k_zero, dim3(8), dim3(256), 0, s, m, (int64_t)2 * NW);
    if (loss_out && epochs > 0) hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, loss_out, (int64_t)epochs);
    spg_status st = SPG_OK;
    double b1t = 1.0, b2t = 1.0;
    for (int ep = 0; ep < epochs && st == SPG_OK; ++ep) {
        for (int32_t r0 = 0; r0 < rows; r0 += batch) {
            const int32_t nr = rows - r0 < batch ? rows - r0 : batch;
            const float* xb = x + (int64_t)r0 * 3;
            const float* tb = y + r0;
            hipLaunchKernelGGL(k_fwd, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, w_inout, xb, nr, yp, act);
            hipLaunchKernelGGL(k_loss, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, yp, tb, nr, quantile, dy,
                               loss_out ? loss_out + ep : nullptr, 1.0f / (float)rows);
            st = launch_backward(s, w_inout, xb, act, dy, nr, g, partial);
            if (st != SPG_OK) break;
            b1t *= 0.9;
            b2t *= 0.999;
            hipLaunchKernelGGL(k_adam, dim3((NW + 255) / 256), dim3(256), 0, s, w_inout, g, m, v, lr,
                               (float)(1.0 - b1t), (float)(1.0 - b2t));
        }
    }
    if (hipGetLastError() != hipSuccess) st = SPG_ERR_HIP;
    if (hipFreeAsync(buf, s) != hipSuccess) st = SPG_ERR_HIP;
    return st;
}

}  // extern "C"
