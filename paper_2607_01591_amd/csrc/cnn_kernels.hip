// Warm-start network kernels for gfx950: 3x3 convolutions as implicit GEMMs on the
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), their gradients,
// loss, Adam, and the raster <-> region transfers. C ABI in include/cnn.h.
//
// MFMA 16x16x32 operand layout (per lane l of a wavefront): A supplies row l % 16,
// k = 8 (l / 16) .. + 7; B supplies column l % 16, the same k; the 16x16 FP32 result
// holds rows 4 (l / 16) .. + 3 of column l % 16.
#include <algorithm>
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

// Forward with the weights in LDS. Persistent blocks (two per compute unit) each stage W
// (Co x 9 x Ci BF16; the rows of one output channel padded by 8 elements so the 16 lanes
// of an operand read fall on distinct banks) once, then take tiles of 16 MT NW consecutive
// pixels of the flattened N x H x W image: wave w of the NW owns pixels
// [16 MT w, 16 MT (w + 1)) of a tile as MT 16-pixel tiles and all Co = 16 NCT output
// channels, every lane's pixel with its own (n, y, x), so tiles may cross rows and
// images. The input operands come from global memory (16 bytes, 8 channels of one pixel
// per lane) and are loaded two (tap, 32-channel) steps ahead of the matrix-core products
// that use them.
template <int NCT, int MT, int NW>
__global__ __launch_bounds__(64 * NW) void k_conv_fwd_lds(const uint16_t *__restrict__ x, const uint16_t *__restrict__ w,
                                                      const float *__restrict__ bias, int N, int H, int W, int Ci,
                                                      int relu, int dil, uint16_t *__restrict__ yb,
                                                      float *__restrict__ yf) {
    constexpr int Co = NCT * 16;
    extern __shared__ uint4 lds_u4[];
    uint16_t *const wl = reinterpret_cast<uint16_t *>(lds_u4);
    const int WS = 9 * Ci + 8;
    {
        const int per = 9 * Ci / 8;   // 16-byte pieces per output channel
        for (int e = threadIdx.x; e < Co * per; e += 64 * NW) {
            const int co = e / per, k = e - co * per;
            *reinterpret_cast<uint4 *>(wl + co * WS + 8 * k) =
                *reinterpret_cast<const uint4 *>(w + (int64_t)co * 9 * Ci + 8 * k);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kb = lane >> 4;
    const int64_t NP = (int64_t)N * H * W;
    const int64_t ntile = (NP + 16 * MT * NW - 1) / (16 * MT * NW);
    const int nc = Ci / 32, nit = 9 * nc;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t pbase = tile * 16 * MT * NW + wv * 16 * MT;
        int pimg[MT], py[MT], px[MT];
        bool pv[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int64_t p = pbase + 16 * u + m;
            pv[u] = p < NP;
            const int64_t q = pv[u] ? p : 0;
            px[u] = int(q % W);
            const int64_t r = q / W;
            py[u] = int(r % H);
            pimg[u] = int(r / H);
        }
        auto load_a = [&](int it, bf16x8 (&a)[MT]) {
            const int tap = it / nc, c0 = (it - tap * nc) * 32;
            const int dy = (tap / 3 - 1) * dil, dx = (tap % 3 - 1) * dil;
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const int yy = py[u] + dy, xx = px[u] + dx;
                const bool ib = pv[u] && yy >= 0 && yy < H && xx >= 0 && xx < W;
                const int64_t off = ib ? (((int64_t)pimg[u] * H + yy) * W + xx) * Ci + c0 + kb * 8 : 0;
                a[u] = as_bf16x8(ib ? *reinterpret_cast<const uint4 *>(x + off) : make_uint4(0, 0, 0, 0));
            }
        };
        f32x4 acc[MT][NCT];
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[u][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto step = [&](int it, const bf16x8 (&a)[MT]) {
            const int tap = it / nc, c0 = (it - tap * nc) * 32;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const bf16x8 b = as_bf16x8(*reinterpret_cast<const uint4 *>(wl + (16 * c + m) * WS + tap * Ci + c0 + kb * 8));
#pragma unroll
                for (int u = 0; u < MT; ++u) acc[u][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b, acc[u][c], 0, 0, 0);
            }
        };
        // the input operands of step it + 2 are loaded while step it computes (three register
        // sets, unrolled by three so no set is copied; the step count 9 Ci / 32 is a multiple
        // of three)
        bf16x8 a0[MT], a1[MT], a2[MT];
        load_a(0, a0);
        load_a(1, a1);
        for (int it = 0; it < nit; it += 3) {
            load_a(it + 2, a2);
            step(it, a0);
            if (it + 3 < nit) load_a(it + 3, a0);
            step(it + 1, a1);
            if (it + 4 < nit) load_a(it + 4, a1);
            step(it + 2, a2);
        }
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const int co = c * 16 + m;
                const float bv = bias ? bias[co] : 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t pix = pbase + 16 * u + 4 * kb + i;
                    if (pix >= NP) continue;
                    float v = acc[u][c][i] + bv;
                    if (relu) v = fmaxf(v, 0.f);
                    const int64_t o = pix * Co + co;
                    if (yb) yb[o] = f2bf(v);
                    if (yf) yf[o] = v;
                }
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

// ---------------------------------------------------------------- weight gradient, LDS
// dw[co][3 ky + kx][ci] += sum over pixels of dz[p][co] x[p + ((ky-1) d, (kx-1) d)][ci]:
// a GEMM over pixels, so each matrix-core operand needs 8 consecutive pixels of one
// channel, while NHWC keeps a pixel's channels together. Block (ky, chunk of `rows` image
// rows); each row is taken in segments of kSeg pixels, staged transposed in LDS
// (channel-major, pixels contiguous): dzT[co][p] for the segment and xT[ci][p] for the
// matching x row with a halo of d pixels on both sides (zeros outside the image), so every
// operand is one 16-byte LDS read (x shifts by kx d that break 16-byte alignment take
// 4-byte or 2-byte reads). Global loads are 16 bytes (8 channels of one pixel), four
// pixels per thread, turned into 8-byte LDS writes (4 pixels of one channel) by byte
// permutes; the next segment's loads are issued before the current one is computed. The
// four waves split each segment's 128 pixels into four k-steps of 32 and each keeps all
// 3 x NCO x NCI output tiles; at the end the waves' partial sums meet in LDS and each
// output element takes one global atomic per block (16 rows per block: the atomics of
// all blocks on one word serialise, so fewer, longer blocks won: 72 us against 111 us
// with 8 rows and 150 us with 4 on the 8 x 128 x 128, 64 -> 64 layer).
constexpr int kSeg = 128;   // pixels per staged segment
constexpr int kWgXU = 3;    // x staging units per thread (units of 4 pixels x 8 channels)

__host__ __device__ constexpr int wg_dz_stride() { return kSeg + 8; }                            // = 8 mod 128
__host__ __device__ inline int wg_x_stride(int dil) { return ((kSeg + 2 * dil - 8 + 127) / 128) * 128 + 8; }
__host__ __device__ inline int wg_x_units(int Ci, int dil) { return (Ci / 8) * ((kSeg + 2 * dil + 3) / 4); }

__device__ __forceinline__ uint32_t bf_pair(uint32_t hi_src, uint32_t lo_src, int half) {
    // the 16-bit half `half` of lo_src in the low half, that of hi_src in the high half
    return __builtin_amdgcn_perm(hi_src, lo_src, half ? 0x07060302u : 0x05040100u);
}

// 4 pixels x 8 channels (v[i] = channels of pixel i) -> 8 LDS rows of 4 pixels each
__device__ __forceinline__ void wg_store_unit(uint16_t *dst, int stride, const uint4 (&v)[4]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int h = j & 1;
        uint32_t w0, w1, w2, w3;
        switch (j >> 1) {
        case 0: w0 = v[0].x; w1 = v[1].x; w2 = v[2].x; w3 = v[3].x; break;
        case 1: w0 = v[0].y; w1 = v[1].y; w2 = v[2].y; w3 = v[3].y; break;
        case 2: w0 = v[0].z; w1 = v[1].z; w2 = v[2].z; w3 = v[3].z; break;
        default: w0 = v[0].w; w1 = v[1].w; w2 = v[2].w; w3 = v[3].w; break;
        }
        const uint2 pk = make_uint2(bf_pair(w1, w0, h), bf_pair(w3, w2, h));
        *reinterpret_cast<uint2 *>(dst + (int64_t)j * stride) = pk;
    }
}

// 8 consecutive BF16 values from LDS at any 2-byte alignment (mode 0: 16-byte aligned,
// 1: 4-byte aligned, 2: 2-byte aligned)
__device__ __forceinline__ bf16x8 wg_read8(const uint16_t *src, int mode) {
    uint4 r;
    if (mode == 0) {
        r = *reinterpret_cast<const uint4 *>(src);
    } else if (mode == 1) {
        const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);
        r = make_uint4(s32[0], s32[1], s32[2], s32[3]);
    } else {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = uint32_t(src[2 * k]) | (uint32_t(src[2 * k + 1]) << 16);
        r = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return as_bf16x8(r);
}

template <int NCO, int NCI>
__global__ __launch_bounds__(256) void k_conv_wgrad_lds(const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz,
                                                        int N, int H, int W, int dil, float *__restrict__ dw, int rows) {
    constexpr int Co = 16 * NCO, Ci = 16 * NCI;
    constexpr int DS = wg_dz_stride();
    constexpr int ndz = (Co / 8) * (kSeg / 4);   // dz staging units per segment
    extern __shared__ uint4 lds_u4[];
    uint16_t *const dzT = reinterpret_cast<uint16_t *>(lds_u4);
    const int XS = wg_x_stride(dil);
    uint16_t *const xT = dzT + Co * DS;
    const int nqx = (kSeg + 2 * dil + 3) / 4, nx = (Ci / 8) * nqx;
    const int ky = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, m = lane & 15, kb = lane >> 4;
    const int r0 = blockIdx.x * rows, r1 = min(N * H, r0 + rows);
    auto valid = [&](int row) {
        const int yy = row % H + (ky - 1) * dil;
        return yy >= 0 && yy < H;
    };
    // work items: (row, segment start) over the rows whose x row lies inside the image
    int row = r0, s0 = 0;
    while (row < r1 && !valid(row)) ++row;
    auto advance = [&](int &rw, int &sg) {
        sg += kSeg;
        if (sg >= W) {
            sg = 0;
            do {
                ++rw;
            } while (rw < r1 && !valid(rw));
        }
    };
    uint4 vd[4], vx[kWgXU][4];
    auto load = [&](int rw, int sg) {
        const int n = rw / H, y = rw % H, yy = y + (ky - 1) * dil;
        if (tid < ndz) {
            const int c8 = tid / (kSeg / 4), q = tid % (kSeg / 4);
            const uint16_t *base = dz + (((int64_t)n * H + y) * W) * Co + 8 * c8;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = sg + 4 * q + i;
                vd[i] = px < W ? *reinterpret_cast<const uint4 *>(base + (int64_t)px * Co) : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < kWgXU; ++k) {
            const int u = tid + 256 * k;
            if (u < nx) {
                const int c8 = u / nqx, q = u % nqx;
                const uint16_t *base = x + (((int64_t)n * H + yy) * W) * Ci + 8 * c8;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xx = sg - dil + 4 * q + i;
                    vx[k][i] = (xx >= 0 && xx < W) ? *reinterpret_cast<const uint4 *>(base + (int64_t)xx * Ci)
                                                    : make_uint4(0, 0, 0, 0);
                }
            }
        }
    };
    auto store = [&]() {
        if (tid < ndz) {
            const int c8 = tid / (kSeg / 4), q = tid % (kSeg / 4);
            wg_store_unit(dzT + (8 * c8) * DS + 4 * q, DS, vd);
        }
#pragma unroll
        for (int k = 0; k < kWgXU; ++k) {
            const int u = tid + 256 * k;
            if (u < nx) {
                const int c8 = u / nqx, q = u % nqx;
                wg_store_unit(xT + (8 * c8) * XS + 4 * q, XS, vx[k]);
            }
        }
    };
    f32x4 acc[3][NCO][NCI];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
        for (int c = 0; c < NCO; ++c)
#pragma unroll
            for (int t = 0; t < NCI; ++t) acc[kx][c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // read mode of each kx: the x operand starts at pixel pk + kx d of the staged row
    int mode[3];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
        const int o = kx * dil;
        mode[kx] = o % 8 == 0 ? 0 : (o % 2 == 0 ? 1 : 2);
    }
    if (row < r1) load(row, s0);
    while (row < r1) {
        __syncthreads();   // the previous item's operand reads are done
        store();
        int nrow = row, ns = s0;
        advance(nrow, ns);
        if (nrow < r1) load(nrow, ns);   // in flight while this item computes
        __syncthreads();
        const int pk = 32 * wv + 8 * kb;
        bf16x8 a[NCO];
#pragma unroll
        for (int c = 0; c < NCO; ++c) a[c] = as_bf16x8(*reinterpret_cast<const uint4 *>(dzT + (16 * c + m) * DS + pk));
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int off = pk + kx * dil;
#pragma unroll
            for (int t = 0; t < NCI; ++t) {
                const bf16x8 b = wg_read8(xT + (16 * t + m) * XS + off, mode[kx]);
#pragma unroll
                for (int c = 0; c < NCO; ++c)
                    acc[kx][c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b, acc[kx][c][t], 0, 0, 0);
            }
        }
        row = nrow;
        s0 = ns;
    }
    // the four waves' partial sums meet in LDS ([kx][co][ci] floats), then one atomic each
    float *red = reinterpret_cast<float *>(lds_u4);
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
#pragma unroll
                for (int c = 0; c < NCO; ++c)
#pragma unroll
                    for (int t = 0; t < NCI; ++t)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int idx = (kx * Co + 16 * c + 4 * kb + i) * Ci + 16 * t + m;
                            red[idx] = (w == 0 ? 0.f : red[idx]) + acc[kx][c][t][i];
                        }
        }
        __syncthreads();
    }
    for (int e = tid; e < 3 * Co * Ci; e += 256) {
        const int kx = e / (Co * Ci), co = (e / Ci) % Co, ci = e % Ci;
        const float v = red[e];
        if (v != 0.f) unsafeAtomicAdd(&dw[((int64_t)co * 9 + 3 * ky + kx) * Ci + ci], v);
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

// db[co] += sum over pixels of dz[p][co]. Thread t of a block keeps channel t mod Co of
// every (256 / Co)-th pixel (coalesced rows when Co divides 256), the block folds its
// 256 / Co partial sums per channel in LDS and adds them with one atomic per channel. At
// most 256 blocks: the atomics of all blocks on one channel's word serialise (1024 blocks
// took 28 us on the 131072 x 64 gradient, 256 blocks 12 us).
__global__ __launch_bounds__(256) void k_bias_grad(const float *__restrict__ dz, int64_t npix, int Co, float *__restrict__ db) {
    __shared__ float sh[256];
    const int ppb = 256 / Co;                    // pixels per block step
    const int c = threadIdx.x % Co, j = threadIdx.x / Co;
    float s = 0.f;
    if (j < ppb) {
        const int64_t step = (int64_t)gridDim.x * ppb;
        int64_t p = (int64_t)blockIdx.x * ppb + j;
        float s1 = 0.f, s2 = 0.f, s3 = 0.f;   // four chains, so four loads are in flight
        for (; p + 3 * step < npix; p += 4 * step) {
            s += dz[p * Co + c];
            s1 += dz[(p + step) * Co + c];
            s2 += dz[(p + 2 * step) * Co + c];
            s3 += dz[(p + 3 * step) * Co + c];
        }
        for (; p < npix; p += step) s += dz[p * Co + c];
        s += (s1 + s2) + s3;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < Co) {
        float t = 0.f;
        for (int k = 0; k < ppb; ++k) t += sh[k * Co + threadIdx.x];
        atomicAdd(&db[threadIdx.x], t);
    }
}

// the same for Co > 256 or not dividing 256: one block column per channel
__global__ void k_bias_grad_col(const float *__restrict__ dz, int64_t npix, int Co, float *__restrict__ db) {
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

// ---------------------------------------------------------------- input features
// Input features of the warm-start network, one thread per material m (FP64 arithmetic,
// FP32 output row [4 G]): the infinite-medium spectrum phi solving
// (diag(Sigma_t) - Sigma_s^T) phi = chi_m (Gaussian elimination with partial pivoting;
// a material that does not fission takes the mean chi of the fissile ones, or a flat
// 1/G if none does), then log(|phi| / sum |phi|) with |phi| floored at 1e-30, Sigma_t,
// Sigma_a = Sigma_t - sum_g' Sigma_s,g->g' and nuSigma_f.
constexpr int kFeatMaxG = 32;
__global__ void k_material_features(const double *__restrict__ st, const double *__restrict__ ss,
                                    const double *__restrict__ nsf, const double *__restrict__ chi, int M, int G,
                                    float *__restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double A[kFeatMaxG * kFeatMaxG], b[kFeatMaxG];
    auto fissile = [&](int mm) {
        double f = 0.0;
        for (int g = 0; g < G; ++g) f += nsf[(int64_t)mm * G + g];
        return f > 0.0;
    };
    if (fissile(m)) {
        for (int g = 0; g < G; ++g) b[g] = chi[(int64_t)m * G + g];
    } else {
        int nf = 0;
        for (int g = 0; g < G; ++g) b[g] = 0.0;
        for (int mm = 0; mm < M; ++mm)
            if (fissile(mm)) {
                ++nf;
                for (int g = 0; g < G; ++g) b[g] += chi[(int64_t)mm * G + g];
            }
        for (int g = 0; g < G; ++g) b[g] = nf > 0 ? b[g] / nf : 1.0 / G;
    }
    // row g: Sigma_t,g phi_g - sum_g' Sigma_s,g'->g phi_g'
    const double *S = ss + (int64_t)m * G * G;   // S[g][g'] = Sigma_s, g -> g'
    for (int g = 0; g < G; ++g)
        for (int gp = 0; gp < G; ++gp) A[g * G + gp] = (g == gp ? st[(int64_t)m * G + g] : 0.0) - S[gp * G + g];
    for (int c = 0; c < G; ++c) {
        int piv = c;
        for (int r = c + 1; r < G; ++r)
            if (fabs(A[r * G + c]) > fabs(A[piv * G + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < G; ++j) {
                const double t = A[c * G + j];
                A[c * G + j] = A[piv * G + j];
                A[piv * G + j] = t;
            }
            const double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < G; ++r) {
            const double f = A[r * G + c] / A[c * G + c];
            for (int j = c; j < G; ++j) A[r * G + j] -= f * A[c * G + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = G - 1; r >= 0; --r) {
        double v = b[r];
        for (int j = r + 1; j < G; ++j) v -= A[r * G + j] * b[j];
        b[r] = v / A[r * G + r];
    }
    double tot = 0.0;
    for (int g = 0; g < G; ++g) {
        b[g] = fmax(fabs(b[g]), 1e-30);
        tot += b[g];
    }
    float *o = out + (int64_t)m * 4 * G;
    for (int g = 0; g < G; ++g) {
        double sa = 0.0;
        for (int gp = 0; gp < G; ++gp) sa += S[g * G + gp];
        o[g] = (float)log(b[g] / tot);
        o[G + g] = (float)st[(int64_t)m * G + g];
        o[2 * G + g] = (float)(st[(int64_t)m * G + g] - sa);
        o[3 * G + g] = (float)nsf[(int64_t)m * G + g];
    }
}

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
    hipStream_t s = (hipStream_t)stream;
    // weights in LDS when they fit the device's per-block LDS: persistent blocks, two per
    // compute unit
    {
        const size_t lds = sizeof(uint16_t) * (size_t)Co * (9 * (size_t)Ci + 8);
        int dev = 0, lds_max = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && lds <= (size_t)lds_max &&
            (Co == 16 || Co == 32 || Co == 64)) {
            // 16 waves of two 16-pixel tiles each: occupancy hides the input loads' latency
            // (64 x 64 layer, 8 x 128 x 128: 4 waves x 4 tiles 36-42 us, 8 x 2 29-33 us,
            // 16 x 2 28-32 us, 8 x 4 33-38 us, 4 x 8 51-55 us)
            constexpr int MT = 2, NW = 16;
            const int64_t ntile = ((int64_t)N * H * W + 16 * MT * NW - 1) / (16 * MT * NW);
            const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ntile, 2 * (int64_t)ncu));
#define FWD_LAUNCH(A) hipLaunchKernelGGL((k_conv_fwd_lds<A, MT, NW>), dim3(grid), dim3(64 * NW), lds, s, x, w, bias, N, H, W, \
                                         Ci, relu, dilation, y_bf16, y_f32)
            if (Co == 16) FWD_LAUNCH(1);
            else if (Co == 32) FWD_LAUNCH(2);
            else FWD_LAUNCH(4);
#undef FWD_LAUNCH
            return launched();
        }
    }
    // two pixel tiles per wavefront once a row fills 128 pixels (each weight load then feeds
    // two products); one for narrower images
    const int mt = W >= 128 ? 2 : 1;
    const dim3 grid((unsigned)((int64_t)N * H * ((W + 64 * mt - 1) / (64 * mt))));
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
    // LDS-staged kernel for Co in {16, 32, 64}, Ci in {32, 64} when its staging fits;
    // otherwise the gather kernel
    const int nco = Co / 16, nci = Ci / 16;
    const size_t stage = sizeof(uint16_t) * ((size_t)Co * wg_dz_stride() + (size_t)Ci * wg_x_stride(dilation));
    const size_t lds = std::max(stage, sizeof(float) * 3 * (size_t)Co * Ci);
    const bool fits = (nco == 1 || nco == 2 || nco == 4) && (nci == 2 || nci == 4) && lds <= 64 * 1024 &&
                      wg_x_units(Ci, dilation) <= 256 * kWgXU;
    if (fits) {
        const int64_t nrows = (int64_t)N * H;
        const int rows = (int)std::max<int64_t>(1, std::min<int64_t>(16, (nrows * 3 + 191) / 192));
        const dim3 grid((unsigned)((nrows + rows - 1) / rows), 3);
        const hipStream_t s = (hipStream_t)stream;
#define WG_LAUNCH(A, B) hipLaunchKernelGGL((k_conv_wgrad_lds<A, B>), grid, dim3(256), lds, s, x, dz, N, H, W, dilation, dw, rows)
        switch (nco * 8 + nci) {
        case 10: WG_LAUNCH(1, 2); break;
        case 12: WG_LAUNCH(1, 4); break;
        case 18: WG_LAUNCH(2, 2); break;
        case 20: WG_LAUNCH(2, 4); break;
        case 34: WG_LAUNCH(4, 2); break;
        default: WG_LAUNCH(4, 4); break;
        }
#undef WG_LAUNCH
        return launched();
    }
    const int rows = 4;
    const dim3 grid((unsigned)(((int64_t)N * H + rows - 1) / rows), 9);
    hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, (hipStream_t)stream, x, dz, N, H, W, Ci, Co, dilation, dw, rows);
    return launched();
}

int cnn_bias_grad(const float *dz, int64_t npix, int32_t Co, float *db, void *stream) {
    if (!dz || !db || npix <= 0 || Co <= 0) return MOC_EINVAL;
    if (Co <= 256 && 256 % Co == 0)
        hipLaunchKernelGGL(k_bias_grad, dim3(grid_for(npix * Co, 256 * 16, 256)), dim3(256), 0, (hipStream_t)stream, dz, npix, Co, db);
    else
        hipLaunchKernelGGL(k_bias_grad_col, dim3(grid_for(npix, 256, 64), Co), dim3(256), 0, (hipStream_t)stream, dz, npix, Co,
                           db);
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

int cnn_material_features(const double *sigma_t, const double *sigma_s, const double *nu_sigma_f, const double *chi,
                          int32_t M, int32_t G, float *features, void *stream) {
    if (!sigma_t || !sigma_s || !nu_sigma_f || !chi || !features || M <= 0 || G <= 0 || G > kFeatMaxG) return MOC_EINVAL;
    hipLaunchKernelGGL(k_material_features, dim3((M + 63) / 64), dim3(64), 0, (hipStream_t)stream, sigma_t, sigma_s,
                       nu_sigma_f, chi, M, G, features);
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
