// Warm-start network kernels for gfx950: 3x3 convolutions as implicit GEMMs on the
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), their gradients,
// loss, Adam, and the raster <-> region transfers. C ABI in include/cnn.h.
//
// MFMA 16x16x32 operand layout (per lane l of a wavefront): A supplies row l % 16,
// k = 8 (l / 16) .. + 7; B supplies column l % 16, the same k; the 16x16 FP32 result
// holds rows 4 (l / 16) .. + 3 of column l % 16.
#include <cmath>
#include <cstdint>
#include <mutex>

#include <hip/hip_runtime.h>

#include "cnn.h"
#include "moc.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                     // round to nearest even
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// ---------------------------------------------------------------- forward
// Block = 4 wavefronts = 64 MT consecutive pixels of one image row; wave w owns pixels
// [16 MT w, 16 MT (w + 1)) as MT tiles of 16 and all Co = 16 NCT output channels, so each
// weight operand it loads feeds MT matrix-core products. Taps sit dil pixels apart.
template <int NCT, int MT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *__restrict__ x, const uint16_t *__restrict__ w,
                                                  const float *__restrict__ bias, int N, int H, int W, int Ci, int relu,
                                                  int dil, uint16_t *__restrict__ yb, float *__restrict__ yf) {
    const int Co = NCT * 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (W + 64 * MT - 1) / (64 * MT);
    int t = blockIdx.x;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int y = t % H, n = t / H;
    const int xbase = tx * 64 * MT + wv * 16 * MT;
    const int m = lane & 15, kb = lane >> 4;
    f32x4 acc[MT][NCT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[u][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + (tap / 3 - 1) * dil;
        int64_t xoff[MT];
        bool inb[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int xx = xbase + u * 16 + m + (tap % 3 - 1) * dil;
            inb[u] = yy >= 0 && yy < H && xx >= 0 && xx < W;
            xoff[u] = inb[u] ? (((int64_t)n * H + yy) * W + xx) * Ci : 0;
        }
        for (int c0 = 0; c0 < Ci; c0 += 32) {
            bf16x8 a[MT];
#pragma unroll
            for (int u = 0; u < MT; ++u)
                a[u] = as_bf16x8(inb[u] ? *reinterpret_cast<const uint4 *>(x + xoff[u] + c0 + kb * 8)
                                        : make_uint4(0, 0, 0, 0));
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const int co = c * 16 + m;
                const bf16x8 b = as_bf16x8(*reinterpret_cast<const uint4 *>(w + ((int64_t)co * 9 + tap) * Ci + c0 + kb * 8));
#pragma unroll
                for (int u = 0; u < MT; ++u) acc[u][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b, acc[u][c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            const int co = c * 16 + (lane & 15);
            const float b = bias ? bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = xbase + u * 16 + 4 * (lane >> 4) + i;
                if (px >= W) continue;
                float v = acc[u][c][i] + b;
                if (relu) v = fmaxf(v, 0.f);
                const int64_t o = (((int64_t)n * H + y) * W + px) * Co + co;
                if (yb) yb[o] = f2bf(v);
                if (yf) yf[o] = v;
            }
        }
}

// ---------------------------------------------------------------- weight gradient
// Block (row chunk, tap): rows [r0, r0 + rows) of the N*H image rows. The 16x16
// output tiles (co, ci) are spread over the 4 wavefronts; K = pixels in steps of 32.
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz, int N,
                                                    int H, int W, int Ci, int Co, int dil, float *__restrict__ dw,
                                                    int rows) {
    const int tap = blockIdx.y, ky = tap / 3, kx = tap % 3;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kb = lane >> 4;
    const int nct = Co / 16, ncit = Ci / 16;
    const int r0 = blockIdx.x * rows, r1 = min(N * H, r0 + rows);
    for (int tile = wv; tile < nct * ncit; tile += 4) {
        const int ct = tile / ncit, it = tile % ncit;
        const int co = ct * 16 + m, ci = it * 16 + m;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int row = r0; row < r1; ++row) {
            const int n = row / H, y = row % H;
            const int yy = y + (ky - 1) * dil;
            if (yy < 0 || yy >= H) continue;     // uniform over the block
            const uint16_t *dzr = dz + ((int64_t)n * H + y) * W * Co;
            const uint16_t *xr = x + ((int64_t)n * H + yy) * W * Ci;
            for (int p0 = 0; p0 < W; p0 += 32) {
                uint16_t av[8], bv[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int px = p0 + kb * 8 + i;
                    const int xx = px + (kx - 1) * dil;
                    av[i] = px < W ? dzr[(int64_t)px * Co + co] : uint16_t(0);
                    bv[i] = (px < W && xx >= 0 && xx < W) ? xr[(int64_t)xx * Ci + ci] : uint16_t(0);
                }
                const uint4 a4 = make_uint4(av[0] | (uint32_t(av[1]) << 16), av[2] | (uint32_t(av[3]) << 16),
                                            av[4] | (uint32_t(av[5]) << 16), av[6] | (uint32_t(av[7]) << 16));
                const uint4 b4 = make_uint4(bv[0] | (uint32_t(bv[1]) << 16), bv[2] | (uint32_t(bv[3]) << 16),
                                            bv[4] | (uint32_t(bv[5]) << 16), bv[6] | (uint32_t(bv[7]) << 16));
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a4), as_bf16x8(b4), acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cor = ct * 16 + 4 * (lane >> 4) + i, cic = it * 16 + (lane & 15);
            atomicAdd(&dw[((int64_t)cor * 9 + tap) * Ci + cic], acc[i]);
        }
    }
}

// ---------------------------------------------------------------- small kernels
__global__ void k_weights_for_dgrad(const float *__restrict__ w, int Co, int Ci, uint16_t *__restrict__ wt) {
    const int64_t n = (int64_t)Co * 9 * Ci;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int co = int(i % Co);
        const int tap = int((i / Co) % 9);
        const int ci = int(i / ((int64_t)Co * 9));
        wt[i] = f2bf(w[((int64_t)co * 9 + (8 - tap)) * Ci + ci]);   // wt[ci][tap][co]
    }
}

__global__ void k_bias_grad(const float *__restrict__ dz, int64_t npix, int Co, float *__restrict__ db) {
    // one block per channel group of 64 threads; grid-stride over pixels
    const int co = blockIdx.y;
    float s = 0.f;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
        s += dz[p * Co + co];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        atomicAdd(&db[co], t);
    }
}

__global__ void k_relu_backward(const float *__restrict__ dy, const uint16_t *__restrict__ y, int64_t n, float *__restrict__ dzf,
                                uint16_t *__restrict__ dzb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = bf2f(y[i]) > 0.f ? dy[i] : 0.f;
        if (dzf) dzf[i] = v;
        if (dzb) dzb[i] = f2bf(v);
    }
}

__global__ void k_mse_grad(const float *__restrict__ y, const float *__restrict__ t, int64_t npix, int cs, int cv,
                           float *__restrict__ dy, double *__restrict__ partials) {
    const int64_t n = npix * cs;
    const double count = (double)npix * cv;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = int(i % cs);
        float g = 0.f;
        if (c < cv) {
            const float d = y[i] - t[i];
            g = float(2.0 * d / count);
            acc += (double)d * d;
        }
        dy[i] = g;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
        partials[blockIdx.x] = s;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *__restrict__ pb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

__global__ void k_to_bf16(const float *__restrict__ s, int64_t n, uint16_t *__restrict__ d) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = f2bf(s[i]);
}

__global__ void k_gather_rows(const float *__restrict__ table, const int32_t *__restrict__ idx, int64_t npix, int C, int Cp,
                              uint16_t *__restrict__ out) {
    const int64_t n = npix * Cp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / Cp;
        const int c = int(i - p * Cp);
        out[i] = c < C ? f2bf(table[(int64_t)idx[p] * C + c]) : uint16_t(0);
    }
}

__global__ void k_gather_log(const double *__restrict__ table, const int32_t *__restrict__ idx, int64_t npix, int C, int Cp,
                             float *__restrict__ out) {
    const int64_t n = npix * Cp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / Cp;
        const int c = int(i - p * Cp);
        out[i] = c < C ? (float)log(table[(int64_t)idx[p] * C + c]) : 0.f;
    }
}

// subtract, per image, the mean over its pixels and channels [0, C) from those entries
// (one 1024-thread block per image, fixed summation order)
__global__ __launch_bounds__(1024) void k_center(float *__restrict__ img, int64_t npix, int C, int Cp) {
    __shared__ double sh[16];
    float *x = img + (int64_t)blockIdx.x * npix * Cp;
    const int64_t n = npix * C;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t p = i / C;
        acc += (double)x[p * Cp + (i - p * C)];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += sh[w];
    const float mean = (float)(tot / (double)n);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t p = i / C;
        x[p * Cp + (i - p * C)] -= mean;
    }
}

__global__ void k_bilinear(const float *__restrict__ img, int H, int W, int Cs, int C, const float *__restrict__ uv, int64_t n,
                           int apply_exp, double *__restrict__ out) {
    const int64_t tot = n * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / C;
        const int c = int(i - r * C);
        const float u = fminf(fmaxf(uv[2 * r], 0.f), float(W - 1));
        const float v = fminf(fmaxf(uv[2 * r + 1], 0.f), float(H - 1));
        const int x0 = min(int(u), W - 2 < 0 ? 0 : W - 2), y0 = min(int(v), H - 2 < 0 ? 0 : H - 2);
        const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
        const float fx = u - float(x0), fy = v - float(y0);
        auto at = [&](int yy, int xx) { return img[((int64_t)yy * W + xx) * Cs + c]; };
        const float val = (1.f - fy) * ((1.f - fx) * at(y0, x0) + fx * at(y0, x1)) + fy * ((1.f - fx) * at(y1, x0) + fx * at(y1, x1));
        out[i] = apply_exp ? exp((double)val) : (double)val;
    }
}

// The 8 symmetries of a square image of side S, as the source pixel of output pixel
// (r, c): identity, the three rotations, the transpose, the two mirrors and the
// anti-transpose. Op 1 and op 3 are each other's inverse; the others are their own.
__device__ __forceinline__ void d4_source(int op, int S, int r, int c, int &sr, int &sc) {
    switch (op) {
        case 0: sr = r; sc = c; break;
        case 1: sr = c; sc = S - 1 - r; break;
        case 2: sr = S - 1 - r; sc = S - 1 - c; break;
        case 3: sr = S - 1 - c; sc = r; break;
        case 4: sr = c; sc = r; break;
        case 5: sr = r; sc = S - 1 - c; break;
        case 6: sr = S - 1 - c; sc = S - 1 - r; break;
        default: sr = S - 1 - r; sc = c; break;
    }
}

// y[n][r][c][:] = x[n][source(r, c)][:] (BF16 images)
__global__ void k_d4_transform(const uint16_t *__restrict__ x, int N, int S, int C, int op, uint16_t *__restrict__ y) {
    const int64_t tot = (int64_t)N * S * S * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = i / C;
        const int ch = int(i - px * C);
        const int n = int(px / ((int64_t)S * S));
        const int rc = int(px - (int64_t)n * S * S);
        int sr, sc;
        d4_source(op, S, rc / S, rc % S, sr, sc);
        y[i] = x[(((int64_t)n * S + sr) * S + sc) * C + ch];
    }
}

// acc[r][c][ch] += w * y[source_inv(r, c)][ch] for ch < C (FP32 images, row stride Cs):
// maps the output of the network on a transformed image back to the original frame
__global__ void k_d4_accumulate(const float *__restrict__ y, int S, int Cs, int C, int op_inv, float w,
                                float *__restrict__ acc) {
    const int64_t tot = (int64_t)S * S * C;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t px = i / C;
        const int ch = int(i - px * C);
        int sr, sc;
        d4_source(op_inv, S, int(px / S), int(px % S), sr, sc);
        acc[px * Cs + ch] += w * y[((int64_t)sr * S + sc) * Cs + ch];
    }
}

inline int grid_for(int64_t n, int block, int cap = 4096) {
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

inline int launched() { return hipGetLastError() == hipSuccess ? MOC_OK : MOC_EHIP; }

// ---------------------------------------------------------------- allocation-free loss
// Blocks of the loss kernel: the partial sums of squares have exactly this many entries.
constexpr int kMseBlocks = 256;

// Sum of the per-block partials in block order, divided by the element count.
__global__ void k_mse_finish(const double *__restrict__ partials, int nblk, double inv_count, double *__restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nblk; ++i) s += partials[i];
        loss[0] = s * inv_count;
    }
}

}  // namespace

// Partial sums of cnn_mse_grad_noalloc: a file-scope device array instead of a caller's
// workspace, held by every device the library runs on until the process ends. In host
// code this name denotes a host-side stand-in; the device address of each device's copy
// comes from hipGetSymbolAddress and is the only form host code passes to kernels.
static __device__ __align__(256) double scratch[kMseBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_on_current_device(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MOC_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return MOC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MOC_EHIP;
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return MOC_OK;
}

}  // namespace

extern "C" {

int cnn_conv3x3_forward(const uint16_t *x, const uint16_t *w, const float *bias, int32_t N, int32_t H, int32_t W, int32_t Ci,
                        int32_t Co, int32_t dilation, int32_t relu, uint16_t *y_bf16, float *y_f32, void *stream) {
    if (!x || !w || (!y_bf16 && !y_f32) || N <= 0 || H <= 0 || W <= 0 || Ci <= 0 || Ci % 32 || Co <= 0 || Co % 16 ||
        dilation < 1)
        return MOC_EINVAL;
    // two pixel tiles per wavefront once a row fills 128 pixels (each weight load then feeds
    // two products); one for narrower images
    const int mt = W >= 128 ? 2 : 1;
    const dim3 grid((unsigned)((int64_t)N * H * ((W + 64 * mt - 1) / (64 * mt))));
    hipStream_t s = (hipStream_t)stream;
    switch ((Co / 16) * 4 + mt) {
        case 5: hipLaunchKernelGGL((k_conv_fwd<1, 1>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        case 6: hipLaunchKernelGGL((k_conv_fwd<1, 2>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        case 9: hipLaunchKernelGGL((k_conv_fwd<2, 1>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        case 10: hipLaunchKernelGGL((k_conv_fwd<2, 2>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        case 17: hipLaunchKernelGGL((k_conv_fwd<4, 1>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        case 18: hipLaunchKernelGGL((k_conv_fwd<4, 2>), grid, dim3(256), 0, s, x, w, bias, N, H, W, Ci, relu, dilation, y_bf16, y_f32); break;
        default: return MOC_EINVAL;
    }
    return launched();
}

int cnn_weights_for_dgrad(const float *w, int32_t Co, int32_t Ci, uint16_t *wt, void *stream) {
    if (!w || !wt || Co <= 0 || Ci <= 0) return MOC_EINVAL;
    const int64_t n = (int64_t)Co * 9 * Ci;
    hipLaunchKernelGGL(k_weights_for_dgrad, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, w, Co, Ci, wt);
    return launched();
}

int cnn_conv3x3_wgrad(const uint16_t *x, const uint16_t *dz, int32_t N, int32_t H, int32_t W, int32_t Ci, int32_t Co,
                      int32_t dilation, float *dw, void *stream) {
    if (!x || !dz || !dw || N <= 0 || H <= 0 || W <= 0 || Ci <= 0 || Ci % 16 || Co <= 0 || Co % 16 || dilation < 1)
        return MOC_EINVAL;
    const int rows = 4;
    const dim3 grid((unsigned)(((int64_t)N * H + rows - 1) / rows), 9);
    hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, (hipStream_t)stream, x, dz, N, H, W, Ci, Co, dilation, dw, rows);
    return launched();
}

int cnn_bias_grad(const float *dz, int64_t npix, int32_t Co, float *db, void *stream) {
    if (!dz || !db || npix <= 0 || Co <= 0) return MOC_EINVAL;
    hipLaunchKernelGGL(k_bias_grad, dim3(grid_for(npix, 256, 64), Co), dim3(256), 0, (hipStream_t)stream, dz, npix, Co, db);
    return launched();
}

int cnn_relu_backward(const float *dy, const uint16_t *y, int64_t n, float *dz_f32, uint16_t *dz_bf16, void *stream) {
    if (!dy || !y || n <= 0 || (!dz_f32 && !dz_bf16)) return MOC_EINVAL;
    hipLaunchKernelGGL(k_relu_backward, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, dy, y, n, dz_f32, dz_bf16);
    return launched();
}

int cnn_mse_grad(const float *y, const float *t, int64_t npix, int32_t cs, int32_t cv, float *dy, double *loss_partials,
                 void *stream) {
    if (!y || !t || !dy || !loss_partials || npix <= 0 || cs <= 0 || cv <= 0 || cv > cs) return MOC_EINVAL;
    hipLaunchKernelGGL(k_mse_grad, dim3(kMseBlocks), dim3(256), 0, (hipStream_t)stream, y, t, npix, cs, cv, dy,
                       loss_partials);
    return launched();
}

int cnn_mse_grad_noalloc(const float *y, const float *t, int64_t npix, int32_t cs, int32_t cv, float *dy, double *loss,
                         void *stream) {
    if (!y || !t || !dy || !loss || npix <= 0 || cs <= 0 || cv <= 0 || cv > cs) return MOC_EINVAL;
    double *part = nullptr;
    const int rc = scratch_on_current_device(&part);
    if (rc != MOC_OK) return rc;
    // every one of the kMseBlocks blocks writes its own partial, so the array needs no
    // clearing between calls
    hipLaunchKernelGGL(k_mse_grad, dim3(kMseBlocks), dim3(256), 0, (hipStream_t)stream, y, t, npix, cs, cv, dy, part);
    hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(64), 0, (hipStream_t)stream, part, kMseBlocks,
                       1.0 / ((double)npix * (double)cv), loss);
    return launched();
}

int cnn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2, float eps, int32_t t,
             uint16_t *p_bf16, void *stream) {
    if (!p || !g || !m || !v || n <= 0 || t < 1) return MOC_EINVAL;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, beta1, beta2, eps, c1,
                       c2, p_bf16);
    return launched();
}

int cnn_to_bf16(const float *src, int64_t n, uint16_t *dst, void *stream) {
    if (!src || !dst || n <= 0) return MOC_EINVAL;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, src, n, dst);
    return launched();
}

int cnn_gather_rows(const float *table, const int32_t *idx, int64_t npix, int32_t C, int32_t Cp, uint16_t *out, void *stream) {
    if (!table || !idx || !out || npix <= 0 || C <= 0 || Cp < C) return MOC_EINVAL;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(npix * Cp, 256)), dim3(256), 0, (hipStream_t)stream, table, idx, npix, C, Cp,
                       out);
    return launched();
}

int cnn_gather_log(const double *table, const int32_t *idx, int64_t npix, int32_t C, int32_t Cp, float *out, void *stream) {
    if (!table || !idx || !out || npix <= 0 || C <= 0 || Cp < C) return MOC_EINVAL;
    hipLaunchKernelGGL(k_gather_log, dim3(grid_for(npix * Cp, 256)), dim3(256), 0, (hipStream_t)stream, table, idx, npix, C, Cp,
                       out);
    return launched();
}

int cnn_center(float *img, int64_t n_images, int64_t npix, int32_t C, int32_t Cp, void *stream) {
    if (!img || n_images <= 0 || npix <= 0 || C <= 0 || Cp < C || n_images > 65535) return MOC_EINVAL;
    hipLaunchKernelGGL(k_center, dim3((unsigned)n_images), dim3(1024), 0, (hipStream_t)stream, img, npix, C, Cp);
    return launched();
}

int cnn_d4_transform(const uint16_t *x, int32_t N, int32_t S, int32_t C, int32_t op, uint16_t *y, void *stream) {
    if (!x || !y || x == y || N <= 0 || S <= 0 || C <= 0 || op < 0 || op > 7) return MOC_EINVAL;
    const int64_t n = (int64_t)N * S * S * C;
    hipLaunchKernelGGL(k_d4_transform, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, x, N, S, C, op, y);
    return launched();
}

int cnn_d4_accumulate(const float *y, int32_t S, int32_t Cs, int32_t C, int32_t op, float weight, float *acc,
                      void *stream) {
    if (!y || !acc || y == acc || S <= 0 || C <= 0 || Cs < C || op < 0 || op > 7) return MOC_EINVAL;
    static const int inverse[8] = {0, 3, 2, 1, 4, 5, 6, 7};
    const int64_t n = (int64_t)S * S * C;
    hipLaunchKernelGGL(k_d4_accumulate, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, y, S, Cs, C,
                       inverse[op], weight, acc);
    return launched();
}

int cnn_bilinear_sample(const float *img, int32_t H, int32_t W, int32_t Cs, int32_t C, const float *uv, int64_t n,
                        int32_t apply_exp, double *out, void *stream) {
    if (!img || !uv || !out || H <= 0 || W <= 0 || C <= 0 || Cs < C || n <= 0) return MOC_EINVAL;
    hipLaunchKernelGGL(k_bilinear, dim3(grid_for(n * C, 256)), dim3(256), 0, (hipStream_t)stream, img, H, W, Cs, C, uv, n,
                       apply_exp, out);
    return launched();
}

}  // extern "C"
