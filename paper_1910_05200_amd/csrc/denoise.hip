// fadenoise: U-Net denoiser for low-spp renders on MI355X (gfx950).
//
// Layout: activations NHWC bfloat16 [H*W][C] (bf16 stored as its 16 high
// bits), weights [Cout][9][Cin].  A network made for n images keeps them
// stacked as one image n*H rows tall: the pooling, upsampling and
// elementwise kernels run over the stack unchanged (every level's image
// height is even, so no 2x2 window crosses two images), and the 3x3
// convolutions take the rows per image and read zeros across an image's
// top and bottom edges as they do outside the stack.  Every 3x3 convolution is an implicit GEMM
// (rows = pixels, columns = output channels, reduction = 9 taps x input
// channels) on gfx950's v_mfma_f32_32x32x16_bf16 with fp32 accumulation; a
// block owns an 8 x 16-pixel tile and 32 or 64 output channels, and stages
// the tile's input patch (with its halo) once per group of input channels
// for all nine taps (k_conv3x3).  The gradient with respect to a
// convolution's input is the same kernel on the flipped, transposed
// weights; the weight gradient is a second GEMM (rows = output channels,
// columns = input channels of one tap, reduction = pixels) split over pixel
// chunks and summed with fp32 atomics (k_conv3x3_wgrad).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fadenoise.h"

typedef uint16_t bf16;
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bf16 f2bf(float f) {        // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}

constexpr float kSlope = 0.01f;    // leaky ReLU
// Radiance enters as log(1 + kExposure x): the light stage's pixel values
// are a few hundredths, and this brings them to order one.
constexpr float kExposure = 16.0f;
// pixels of all images of one network: every index of its largest tensor
// (96 channels at full size) stays below 2^31
constexpr long long kMaxBatchPixels = ((1ll << 31) - 1) / 96;

// ------------------------------------------------------------ conv 3x3 --
// Y[p][co] = act(bias[co] + sum_{t, ci} W[co][t][ci] X[nbr(p, t)][ci]), zero
// outside the image; act = leaky ReLU when relu, else identity (bias may be
// NULL).  Y has ldy channels per pixel starting at channel yoff (so a result
// can land inside a concatenation).
//
// Implicit GEMM on v_mfma_f32_32x32x16_bf16 (rows = pixels, columns =
// output channels, reduction = 9 taps x input channels).  A block of four
// waves owns a tile of 8 x 16 pixels and NT output channels; each wave owns
// two of its pixel rows (32 pixels) and all NT channels (NT / 32
// accumulators).  The reduction runs in stages of KC input channels: the
// stage's input patch (the tile plus a one-pixel halo, 10 x 18 pixels) and
// its weights for all nine taps go to LDS once, and every tap reads its
// shifted window of the same patch, so the input is fetched once per stage
// instead of once per tap.  The next stage's global loads are issued into
// registers before the current stage's MFMAs.  LDS rows are padded by 16
// bytes, which spreads a half-wave's 16-byte reads over all 64 banks.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t pack2(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }
// eight consecutive values as bf16 (16 bytes)
__device__ __forceinline__ uint4 load8(const bf16 *p) { return *(const uint4 *)p; }
__device__ __forceinline__ uint4 load8(const float *p) {
    const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
    return make_uint4(pack2(a.x, a.y), pack2(a.z, a.w), pack2(b.x, b.y), pack2(b.z, b.w));
}
__device__ __forceinline__ void store1(bf16 *p, float v) { *p = f2bf(v); }
__device__ __forceinline__ void store1(float *p, float v) { *p = v; }

constexpr int kPR = 8;                            // pixel tile: 8 rows x PC columns (16 or 32)
constexpr int kLPad = 8;                          // bf16 of padding per LDS row

// H is the stack's height and Himg the rows of one image (H for a single
// image); when images are stacked, Himg is a multiple of the tile's rows, so
// a tile never spans two images.  Each wave owns two pixel rows of the tile
// (2 PC pixels, PC / 16 row blocks of 32 pixels for the instruction) and all
// NT channels: with 32 columns every weight fragment read from LDS serves
// two instructions instead of one, which halves the LDS reads per
// instruction of the B operand.
// act (nullable, [P][Cout] like Y): the leaky ReLU outputs whose derivative
// multiplies the result (the input gradient of a layer whose input is an
// activation), so that no separate pass over the gradient is needed.
template <class TX, class TY, int NT, int KC, int PC>
__global__ __launch_bounds__(256) void k_conv3x3(int H, int Himg, int W, int Cin, int Cout, const TX *__restrict__ X,
        const bf16 *__restrict__ Wt, const float *__restrict__ bias, int relu, TY *__restrict__ Y, int ldy,
        int yoff, const bf16 *__restrict__ act) {
    constexpr int kHR = kPR + 2, kHC = PC + 2;    // the patch: the tile with its one-pixel halo
    constexpr int NA = NT / 32;                   // accumulators per wave and row block
    constexpr int MB = PC / 16;                   // row blocks of 32 pixels per wave
    constexpr int XQ = KC / 8;                    // 16-byte parts per pixel per stage
    constexpr int XN = kHR * kHC * XQ, WN = 9 * NT * XQ;
    constexpr int XI = (XN + 255) / 256, WI = (WN + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 Xs[kHR * kHC][KC + kLPad];
    __shared__ __attribute__((aligned(16))) bf16 Ws[9 * NT][KC + kLPad];
    const int tiles_x = (W + PC - 1) / PC;
    const int ty0 = (int)(blockIdx.x / tiles_x) * kPR, tx0 = (int)(blockIdx.x % tiles_x) * PC;
    const int co0 = blockIdx.y * NT;
    const int ylo = ty0 - ty0 % Himg, yhi = min(H, ylo + Himg);   // the tile's image
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 31, kh = (lane >> 5) * 8;   // the lane's pixel (A) / channel (B) row, k half
    f16v acc[MB][NA];
    for (int mb = 0; mb < MB; ++mb)
        for (int a = 0; a < NA; ++a)
            for (int r = 0; r < 16; ++r) acc[mb][a][r] = 0.0f;
    uint4 xr[XI], wr[WI];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int u = 0; u < XI; ++u) {
            const int idx = tid + u * 256;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (idx < XN) {
                const int q = idx / XQ, part = idx % XQ;
                const int py = ty0 - 1 + q / kHC, px = tx0 - 1 + q % kHC;
                if (py >= ylo && py < yhi && px >= 0 && px < W) v = load8(X + ((size_t)py * W + px) * Cin + c0 + part * 8);
            }
            xr[u] = v;
        }
#pragma unroll
        for (int u = 0; u < WI; ++u) {
            const int idx = tid + u * 256;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (idx < WN) {
                const int part = idx % XQ, row = idx / XQ, co = row % NT, t = row / NT;
                if (co0 + co < Cout) v = load8(Wt + ((size_t)(co0 + co) * 9 + t) * Cin + c0 + part * 8);
            }
            wr[u] = v;
        }
    };
    fetch(0);
    for (int c0 = 0; c0 < Cin; c0 += KC) {
        __syncthreads();                           // the previous stage's LDS reads are done
#pragma unroll
        for (int u = 0; u < XI; ++u) {
            const int idx = tid + u * 256;
            if (idx < XN) *(uint4 *)&Xs[idx / XQ][(idx % XQ) * 8] = xr[u];
        }
#pragma unroll
        for (int u = 0; u < WI; ++u) {
            const int idx = tid + u * 256;
            if (idx < WN) *(uint4 *)&Ws[idx / XQ][(idx % XQ) * 8] = wr[u];
        }
        __syncthreads();
        if (c0 + KC < Cin) fetch(c0 + KC);         // in flight during this stage's MFMAs
#pragma unroll
        for (int t = 0; t < 9; ++t) {
#pragma unroll
            for (int ks = 0; ks < KC; ks += 16) {
                bf8v a[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int pi = mb * 32 + m, pr = 2 * wave + pi / PC, pc = pi % PC;
                    a[mb] = *(const bf8v *)&Xs[(pr + t / 3) * kHC + pc + t % 3][ks + kh];
                }
#pragma unroll
                for (int na = 0; na < NA; ++na) {
                    const bf8v b = *(const bf8v *)&Ws[t * NT + na * 32 + m][ks + kh];
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[mb][na] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mb], b, acc[mb][na], 0, 0, 0);
                }
            }
        }
    }
    // acc[mb][na][r] holds pixel 32 mb + 8 (r / 4) + 4 (lane / 32) + r % 4 of
    // the wave's 2 PC (row-major) and channel na * 32 + lane % 32
#pragma unroll
    for (int na = 0; na < NA; ++na) {
        const int co = co0 + na * 32 + m;
        if (co >= Cout) continue;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int pi = mb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int py = ty0 + 2 * wave + pi / PC, px = tx0 + pi % PC;
                if (py >= H || px >= W) continue;
                float v = acc[mb][na][r] + bv;
                if (relu) v = v > 0.0f ? v : kSlope * v;
                if (act && !(bf2f(act[((size_t)py * W + px) * Cout + co]) > 0.0f)) v *= kSlope;
                store1(&Y[((size_t)py * W + px) * ldy + yoff + co], v);
            }
    }
}

template <class TX, class TY, int PC>
static void conv3x3_launch_pc(hipStream_t s, int H, int Himg, int W, int Cin, int Cout, const TX *X, const bf16 *Wt,
                              const float *bias, int relu, TY *Y, int ldy, int yoff, const bf16 *act) {
    const unsigned tiles = (unsigned)(((H + kPR - 1) / kPR) * ((W + PC - 1) / PC));
    if (Cout >= 64) {
        dim3 g(tiles, (unsigned)((Cout + 63) / 64));
        if (Cin % 32 == 0) hipLaunchKernelGGL((k_conv3x3<TX, TY, 64, 32, PC>), g, dim3(256), 0, s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
        else hipLaunchKernelGGL((k_conv3x3<TX, TY, 64, 16, PC>), g, dim3(256), 0, s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
    } else {
        dim3 g(tiles, (unsigned)((Cout + 31) / 32));
        if (Cin % 32 == 0) hipLaunchKernelGGL((k_conv3x3<TX, TY, 32, 32, PC>), g, dim3(256), 0, s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
        else hipLaunchKernelGGL((k_conv3x3<TX, TY, 32, 16, PC>), g, dim3(256), 0, s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
    }
}

// Launch k_conv3x3 for one layer: NT = 64 channels per block when Cout >= 64
// (else 32), stages of 32 input channels when Cin allows (else 16); tiles of
// 32 columns when the layer still has kWideBlocks blocks with them (the chip
// stays full), else 16.
constexpr long long kWideBlocks = 2048;
template <class TX, class TY>
static void conv3x3_launch(hipStream_t s, int H, int Himg, int W, int Cin, int Cout, const TX *X, const bf16 *Wt,
                           const float *bias, int relu, TY *Y, int ldy, int yoff, const bf16 *act = nullptr) {
    const long long wide = (long long)((H + kPR - 1) / kPR) * ((W + 31) / 32) * ((Cout + (Cout >= 64 ? 63 : 31)) / (Cout >= 64 ? 64 : 32));
    if (wide >= kWideBlocks) conv3x3_launch_pc<TX, TY, 32>(s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
    else conv3x3_launch_pc<TX, TY, 16>(s, H, Himg, W, Cin, Cout, X, Wt, bias, relu, Y, ldy, yoff, act);
}

// Weight gradient of one tap, one chunk of pixels:
// dW[co][t][ci] += sum_{p in chunk} G[p][co] X[nbr(p, t)][ci]  (fp32 atomics
// per block).  GEMM rows = output channels, columns = input channels,
// reduction = pixels, 16 per v_mfma_f32_32x32x16_bf16; a block of four waves
// owns a 64 x 64 tile, each wave a 32 x 32 quarter, and stages 32 pixels of
// G and of the tap-shifted X in LDS (pixel-contiguous rows, padded to 16-byte
// multiples) per step.
constexpr int kWTile = 64, kWStep = 32, kWChunk = 2048;
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(int H, int Himg, int W, int Cin, int Cout, const bf16 *__restrict__ X,
        const float *__restrict__ G, float *__restrict__ dW) {
    __shared__ __attribute__((aligned(16))) bf16 As[kWTile][kWStep + kLPad];   // [co][px]
    __shared__ __attribute__((aligned(16))) bf16 Bs[kWTile][kWStep + kLPad];   // [ci][px]
    const int P = H * W;
    const int nco = (Cout + kWTile - 1) / kWTile;      // grid: (channel tiles x pixel chunks, ci tiles, taps)
    const int co0 = (int)(blockIdx.x % nco) * kWTile, chunk = (int)(blockIdx.x / nco), ci0 = blockIdx.y * kWTile;
    const int t = blockIdx.z;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m = lane & 31, kh = (lane >> 5) * 8;
    const int lpx = tid >> 3, lc = (tid & 7) * 8;       // loader: pixel of the step, 8 channels
    f16v acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int pbeg = chunk * kWChunk, pend = min(P, pbeg + kWChunk);
    for (int pb = pbeg; pb < pend; pb += kWStep) {
        const int p = pb + lpx;
        uint4 vg = make_uint4(0u, 0u, 0u, 0u), vx = make_uint4(0u, 0u, 0u, 0u);
        if (p < pend) {
            const int y = p / W, x = p - y * W;
            const int sy = y + dy, sx = x + dx, ylo = y - y % Himg;   // the pixel's image: rows [ylo, ylo + Himg)
            if (co0 + lc < Cout) vg = load8(G + (size_t)p * Cout + co0 + lc);
            if (ci0 + lc < Cin && sy >= ylo && sy < ylo + Himg && sy < H && sx >= 0 && sx < W)
                vx = load8(X + ((size_t)sy * W + sx) * Cin + ci0 + lc);
        }
        __syncthreads();
        const bf16 *g8 = (const bf16 *)&vg, *x8 = (const bf16 *)&vx;
#pragma unroll
        for (int q = 0; q < 8; ++q) { As[lc + q][lpx] = g8[q]; Bs[lc + q][lpx] = x8[q]; }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kWStep; ks += 16) {
            const bf8v a = *(const bf8v *)&As[wm * 32 + m][ks + kh];
            const bf8v b = *(const bf8v *)&Bs[wn * 32 + m][ks + kh];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
    const int ci = ci0 + wn * 32 + m;
    if (ci >= Cin) return;
    for (int r = 0; r < 16; ++r) {
        const int co = co0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (co < Cout && acc[r] != 0.0f) atomicAdd(&dW[((size_t)co * 9 + t) * Cin + ci], acc[r]);
    }
}

// bias gradient: db[c] += sum_p G[p][c], one block per 256 pixels.  With
// C < 256 channels the block's threads form 256 / C rows of C channels
// (consecutive threads read consecutive channels of one pixel), each row
// summing every (256 / C)-th pixel; the rows' partial sums meet in LDS and
// each channel takes one atomic per block.
__global__ __launch_bounds__(256) void k_bias_grad(int P, int C, const float *__restrict__ G, float *__restrict__ db) {
    __shared__ float part[256];
    const int p0 = blockIdx.x * 256, p1 = min(P, p0 + 256);
    if (C >= 256) {
        for (int c = threadIdx.x; c < C; c += 256) {
            float s = 0.0f;
            for (int p = p0; p < p1; ++p) s += G[(size_t)p * C + c];
            if (s != 0.0f) atomicAdd(&db[c], s);
        }
        return;
    }
    const int rows = 256 / C, c = threadIdx.x % C, r = threadIdx.x / C;
    float s = 0.0f;
    if (r < rows)
        for (int p = p0 + r; p < p1; p += rows) s += G[(size_t)p * C + c];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.0f;
        for (int k = 0; k < rows; ++k) t += part[k * C + threadIdx.x];
        if (t != 0.0f) atomicAdd(&db[threadIdx.x], t);
    }
}

// flipped, transposed bf16 weights for the input gradient:
// Wt'[ci][t][co] = W[co][8 - t][ci]
__global__ __launch_bounds__(256) void k_flip_weights(int Cin, int Cout, const float *__restrict__ w, bf16 *__restrict__ wf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Cin * 9 * Cout) return;
    int co = i % Cout, t = (i / Cout) % 9, ci = i / (9 * Cout);
    wf[i] = f2bf(w[((size_t)co * 9 + (8 - t)) * Cin + ci]);
}

// ------------------------------------------------------- elementwise ----
__global__ void k_to_bf16(size_t n, const float *__restrict__ a, bf16 *__restrict__ b) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}
__global__ void k_zero_f(size_t n, float *a) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0f;
}

// network input: log(1 + rgb), albedo, normal, depth, zeros -> 16 channels
__global__ void k_pack_input(int P, const float *__restrict__ rgb, const float *__restrict__ aux, bf16 *__restrict__ x) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    bf16 *o = x + (size_t)p * 16;
    for (int c = 0; c < 3; ++c) o[c] = f2bf(log1pf(kExposure * fmaxf(rgb[3 * p + c], 0.0f)));
    for (int c = 0; c < FD_IN_AUX; ++c) o[3 + c] = f2bf(aux[FD_IN_AUX * p + c]);
    for (int c = 3 + FD_IN_AUX; c < 16; ++c) o[c] = 0;
}

// 2x2 average pool: [H][W][C] (ld channels, offset off) -> [H/2][W/2][C]
__global__ void k_pool2(int H, int W, int C, const bf16 *__restrict__ x, int ldx, bf16 *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int Ho = H / 2, Wo = W / 2;
    if (i >= Ho * Wo * C) return;
    int c = i % C, q = i / C, ox = q % Wo, oy = q / Wo;
    float s = 0.0f;
    for (int k = 0; k < 4; ++k) s += bf2f(x[((size_t)(2 * oy + (k >> 1)) * W + 2 * ox + (k & 1)) * ldx + c]);
    y[i] = f2bf(0.25f * s);
}
// gradient of the pool, added: gx[p][c] += gy[p/2][c] / 4
__global__ void k_pool2_bwd_add(int H, int W, int C, const float *__restrict__ gy, float *__restrict__ gx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H * W * C) return;
    int c = i % C, q = i / C, x = q % W, y = q / W;
    gx[i] += 0.25f * gy[((size_t)(y / 2) * (W / 2) + x / 2) * C + c];
}
// nearest 2x upsample of x [H/2][W/2][C] into y [H][W][ldy], channels from 0
__global__ void k_up2(int H, int W, int C, const bf16 *__restrict__ x, bf16 *__restrict__ y, int ldy) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H * W * C) return;
    int c = i % C, q = i / C, px = q % W, py = q / W;
    y[(size_t)q * ldy + c] = x[((size_t)(py / 2) * (W / 2) + px / 2) * C + c];
}
// gradient of the upsample: gx[q][c] = sum of the four gy[.][c] (gy [H][W][ldy])
__global__ void k_up2_bwd(int H, int W, int C, const float *__restrict__ gy, int ldy, float *__restrict__ gx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int Ho = H / 2, Wo = W / 2;
    if (i >= Ho * Wo * C) return;
    int c = i % C, q = i / C, ox = q % Wo, oy = q / Wo;
    float s = 0.0f;
    for (int k = 0; k < 4; ++k) s += gy[((size_t)(2 * oy + (k >> 1)) * W + 2 * ox + (k & 1)) * ldy + c];
    gx[i] = s;
}
// copy C channels between tensors with different channel strides / offsets
template <class T>
__global__ void k_copy_ch(int P, int C, const T *__restrict__ x, int ldx, int xoff, T *__restrict__ y, int ldy,
                          int yoff) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    int c = i % C, p = i / C;
    y[(size_t)p * ldy + yoff + c] = x[(size_t)p * ldx + xoff + c];
}
// leaky-ReLU backward in place: g *= (y > 0 ? 1 : slope)
__global__ void k_act_bwd(size_t n, const bf16 *__restrict__ y, float *__restrict__ g) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(bf2f(y[i]) > 0.0f)) g[i] *= kSlope;
}

// 1x1 output convolution (fp32) as a correction of the input's
// log-radiance: pred[p][k] = log(1 + kExposure rgb[p][k]) + b[k] + sum_c w[k][c] x[p][c]
__global__ void k_out_fwd(int P, int C, const bf16 *__restrict__ x, const float *__restrict__ w, const float *__restrict__ b,
                          const float *__restrict__ rgb, float *__restrict__ pred) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    for (int k = 0; k < 3; ++k) {
        float s = b[k];
        for (int c = 0; c < C; ++c) s += w[k * C + c] * bf2f(x[(size_t)p * C + c]);
        pred[3 * p + k] = log1pf(kExposure * fmaxf(rgb[3 * p + k], 0.0f)) + s;
    }
}
__global__ void k_expm1(int n, const float *__restrict__ pred, float *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = expm1f(pred[i]) / kExposure;
}
// loss and its gradient: d = pred - log(1 + kExposure target); loss += d^2 / n; dpred = 2 d / n.
// One block per kLossBlock values; the block's sum takes one atomic (one per
// wave serialised on the single loss word once many images run per call).
constexpr int kLossBlock = 4096;
__global__ __launch_bounds__(256) void k_loss(int n, const float *__restrict__ pred, const float *__restrict__ tgt,
                                             float *__restrict__ dpred, float *__restrict__ loss) {
    __shared__ float part[4];
    float e = 0.0f;
    const int i1 = min(n, (int)(blockIdx.x + 1) * kLossBlock);
    for (int i = (int)blockIdx.x * kLossBlock + (int)threadIdx.x; i < i1; i += 256) {
        float d = pred[i] - log1pf(kExposure * fmaxf(tgt[i], 0.0f));
        dpred[i] = 2.0f * d / (float)n;
        e += d * d / (float)n;
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = (part[0] + part[1]) + (part[2] + part[3]);
        if (t != 0.0f) atomicAdd(loss, t);
    }
}
// output layer backward: dw[k][c] += sum_p dpred[p][k] x[p][c]; db[k] += sum_p dpred;
// gx[p][c] = sum_k dpred[p][k] w[k][c].  One block per 256 pixels (C <= 64):
// first one thread per pixel writes gx; then one thread per (k, c) weight
// and per k bias sums its products over the block's pixels (staged in LDS)
// and adds them with one atomic.
__global__ __launch_bounds__(256) void k_out_bwd(int P, int C, const bf16 *__restrict__ x, const float *__restrict__ w,
        const float *__restrict__ dpred, float *__restrict__ dw, float *__restrict__ db, float *__restrict__ gx) {
    __shared__ float sd[256][3];
    const int p0 = blockIdx.x * 256, p = p0 + threadIdx.x, np = min(256, P - p0);
    if (p < P) {
        const float d0 = dpred[3 * p], d1 = dpred[3 * p + 1], d2 = dpred[3 * p + 2];
        sd[threadIdx.x][0] = d0; sd[threadIdx.x][1] = d1; sd[threadIdx.x][2] = d2;
        for (int c = 0; c < C; ++c) gx[(size_t)p * C + c] = d0 * w[c] + d1 * w[C + c] + d2 * w[2 * C + c];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 3 * C) {
        const int k = t / C, c = t % C;
        float s = 0.0f;
        for (int q = 0; q < np; ++q) s += sd[q][k] * bf2f(x[(size_t)(p0 + q) * C + c]);
        if (s != 0.0f) atomicAdd(&dw[t], s);
    } else if (t < 3 * C + 3) {
        const int k = t - 3 * C;
        float s = 0.0f;
        for (int q = 0; q < np; ++q) s += sd[q][k];
        if (s != 0.0f) atomicAdd(&db[k], s);
    }
}

// d loss / d pred from d loss / d out, out = expm1(pred) / kExposure
__global__ void k_dout_dpred(int n, const float *__restrict__ pred, const float *__restrict__ gout, float *__restrict__ dpred) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dpred[i] = gout[i] * expf(pred[i]) / kExposure;
}
// d loss / d rgb: the residual path and the packed input's first three
// channels, through log(1 + kExposure rgb) (zero where rgb < 0)
__global__ void k_drgb(int P, const float *__restrict__ rgb, const float *__restrict__ dpred, const float *__restrict__ gx0,
                       float *__restrict__ drgb) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * P) return;
    int p = i / 3, k = i % 3;
    float x = rgb[i];
    drgb[i] = x < 0.0f ? 0.0f : (dpred[i] + gx0[(size_t)p * 16 + k]) * kExposure / (1.0f + kExposure * x);
}

// Adam (Kingma and Ba 2015) over all parameters
__global__ void k_adam(size_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float c1, float c2) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ====================================================================== //
//                                  host                                   //
// ====================================================================== //
namespace {
struct Layer { int cin, cout, k, level; size_t woff, boff; };
struct Act { bf16 *y = nullptr; float *g = nullptr; int c = 0, level = 0; };   // values bf16, gradients fp32
inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }
}

struct fd_net {
    std::string err;
    hipStream_t stream = nullptr;
    int H = 0, W = 0, N = 1;         // image size, images per call (stacked)
    std::vector<Layer> L;
    size_t nparam = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    bf16 *wbf = nullptr, *wflip = nullptr;      // bf16 copies of all conv weights, flipped scratch
    int step = 0;
    bool have_forward = false;
    // activations (see build()), index by name
    Act x0, e0a, e0, p1, e1a, e1, p2, e2a, e2, p3, e3a, e3, c2, d2a, d2, c1, d1a, d1, c0, d0a, d0;
    float *pred = nullptr, *dpred = nullptr, *loss_s = nullptr;
    std::vector<void *> allocs;
};

static int fail(fd_net *n, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n) n->err = buf;
    return code;
}
#define HIPCK(n, x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return fail(n, -3, "%s: %s", #x, hipGetErrorString(e_)); } while (0)

template <class T> static int dalloc(fd_net *n, T **p, size_t count) {
    if (hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return -2;
    n->allocs.push_back(*p);
    return 0;
}

// pixels of all n images at a level; rows of the stack and of one image
static int pix(const fd_net *n, int level) { return n->N * (n->H >> level) * (n->W >> level); }
static int rows(const fd_net *n, int level) { return n->N * (n->H >> level); }

static int conv(fd_net *n, int li, const Act &x, bf16 *y, int ldy, int yoff, bool relu) {
    const Layer &l = n->L[li];
    int H = rows(n, l.level), Himg = n->H >> l.level, W = n->W >> l.level;
    conv3x3_launch<bf16, bf16>(n->stream, H, Himg, W, l.cin, l.cout, x.y, n->wbf + l.woff, n->params + l.boff,
                               relu ? 1 : 0, y, ldy, yoff);
    return 0;
}

// backward of conv layer li: g_out (bf16 [P][cout], already multiplied by
// the activation's derivative) -> weight and bias gradients, and (when gx)
// the input gradient gx [P][cin], multiplied by the derivative of x's leaky
// ReLU when x_act (x is an activation output).
static void conv_bwd(fd_net *n, int li, const Act &x, const float *gout, float *gx, bool wgrad, bool x_act = false) {
    const Layer &l = n->L[li];
    int H = rows(n, l.level), Himg = n->H >> l.level, W = n->W >> l.level, P = H * W;
    if (wgrad) {
        dim3 gw(nblk(l.cout, kWTile) * nblk(P, kWChunk), nblk(l.cin, kWTile), 9);
        hipLaunchKernelGGL(k_conv3x3_wgrad, gw, dim3(256), 0, n->stream, H, Himg, W, l.cin, l.cout, x.y, gout,
                           n->grads + l.woff);
        hipLaunchKernelGGL(k_bias_grad, dim3(nblk(P, 256)), dim3(256), 0, n->stream, P, l.cout, gout, n->grads + l.boff);
    }
    if (gx) {
        hipLaunchKernelGGL(k_flip_weights, dim3(nblk((size_t)l.cin * 9 * l.cout, 256)), dim3(256), 0, n->stream,
                           l.cin, l.cout, n->params + l.woff, n->wflip);
        conv3x3_launch<float, float>(n->stream, H, Himg, W, l.cout, l.cin, gout, n->wflip, (const float *)nullptr, 0,
                                     gx, l.cin, 0, x_act ? x.y : nullptr);
    }
}

static void act_bwd(fd_net *n, const Act &a) {
    size_t cnt = (size_t)pix(n, a.level) * a.c;
    hipLaunchKernelGGL(k_act_bwd, dim3(nblk(cnt, 256)), dim3(256), 0, n->stream, cnt, a.y, a.g);
}

static void forward(fd_net *n, const float *rgb, const float *aux) {
    const int P0 = pix(n, 0);
    hipStream_t s = n->stream;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n->nparam, 256)), dim3(256), 0, s, n->nparam, n->params, n->wbf);
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(P0, 256)), dim3(256), 0, s, P0, rgb, aux, n->x0.y);
    auto pool = [&](const Act &x, const Act &y) {
        int H = rows(n, x.level), W = n->W >> x.level;
        hipLaunchKernelGGL(k_pool2, dim3(nblk((size_t)(H / 2) * (W / 2) * x.c, 256)), dim3(256), 0, s, H, W, x.c, x.y,
                           x.c, y.y);
    };
    auto upcat = [&](const Act &lo, const Act &skip, const Act &cat) {
        int H = rows(n, cat.level), W = n->W >> cat.level;
        hipLaunchKernelGGL(k_up2, dim3(nblk((size_t)H * W * lo.c, 256)), dim3(256), 0, s, H, W, lo.c, lo.y, cat.y, cat.c);
        hipLaunchKernelGGL(k_copy_ch<bf16>, dim3(nblk((size_t)H * W * skip.c, 256)), dim3(256), 0, s, H * W, skip.c,
                           skip.y, skip.c, 0, cat.y, cat.c, lo.c);
    };
    conv(n, 0, n->x0, n->e0a.y, 32, 0, true);
    conv(n, 1, n->e0a, n->e0.y, 32, 0, true);
    pool(n->e0, n->p1);
    conv(n, 2, n->p1, n->e1a.y, 64, 0, true);
    conv(n, 3, n->e1a, n->e1.y, 64, 0, true);
    pool(n->e1, n->p2);
    conv(n, 4, n->p2, n->e2a.y, 128, 0, true);
    conv(n, 5, n->e2a, n->e2.y, 128, 0, true);
    pool(n->e2, n->p3);
    conv(n, 6, n->p3, n->e3a.y, 256, 0, true);
    conv(n, 7, n->e3a, n->e3.y, 256, 0, true);
    upcat(n->e3, n->e2, n->c2);
    conv(n, 8, n->c2, n->d2a.y, 128, 0, true);
    conv(n, 9, n->d2a, n->d2.y, 128, 0, true);
    upcat(n->d2, n->e1, n->c1);
    conv(n, 10, n->c1, n->d1a.y, 64, 0, true);
    conv(n, 11, n->d1a, n->d1.y, 64, 0, true);
    upcat(n->d1, n->e0, n->c0);
    conv(n, 12, n->c0, n->d0a.y, 32, 0, true);
    conv(n, 13, n->d0a, n->d0.y, 32, 0, true);
    const Layer &lo = n->L[14];
    hipLaunchKernelGGL(k_out_fwd, dim3(nblk(P0, 256)), dim3(256), 0, s, P0, 32, n->d0.y, n->params + lo.woff,
                       n->params + lo.boff, rgb, n->pred);
}

// wgrad: parameter gradients into n->grads; input: the input's gradient
// into x0.g (channels of the packed input)
static void backward(fd_net *n, bool wgrad, bool input) {
    const int P0 = pix(n, 0);
    hipStream_t s = n->stream;
    hipLaunchKernelGGL(k_zero_f, dim3(nblk(n->nparam, 256)), dim3(256), 0, s, n->nparam, n->grads);
    const Layer &lo = n->L[14];
    hipLaunchKernelGGL(k_out_bwd, dim3(nblk(P0, 256)), dim3(256), 0, s, P0, 32, n->d0.y, n->params + lo.woff, n->dpred,
                       n->grads + lo.woff, n->grads + lo.boff, n->d0.g);
    auto split = [&](const Act &cat, const Act &lo_, const Act &skip) {   // cat grad -> lo grad, skip grad (set)
        int H = rows(n, cat.level), W = n->W >> cat.level;
        hipLaunchKernelGGL(k_up2_bwd, dim3(nblk((size_t)(H / 2) * (W / 2) * lo_.c, 256)), dim3(256), 0, s, H, W, lo_.c,
                           cat.g, cat.c, lo_.g);
        hipLaunchKernelGGL(k_copy_ch<float>, dim3(nblk((size_t)H * W * skip.c, 256)), dim3(256), 0, s, H * W, skip.c,
                           cat.g, cat.c, lo_.c, skip.g, skip.c, 0);
    };
    auto pool_bwd = [&](const Act &py, const Act &x) {   // x.g += pool gradient
        int H = rows(n, x.level), W = n->W >> x.level;
        hipLaunchKernelGGL(k_pool2_bwd_add, dim3(nblk((size_t)H * W * x.c, 256)), dim3(256), 0, s, H, W, x.c, py.g, x.g);
    };
    act_bwd(n, n->d0);  conv_bwd(n, 13, n->d0a, n->d0.g, n->d0a.g, wgrad, true);
    conv_bwd(n, 12, n->c0, n->d0a.g, n->c0.g, wgrad);
    split(n->c0, n->d1, n->e0);
    act_bwd(n, n->d1);  conv_bwd(n, 11, n->d1a, n->d1.g, n->d1a.g, wgrad, true);
    conv_bwd(n, 10, n->c1, n->d1a.g, n->c1.g, wgrad);
    split(n->c1, n->d2, n->e1);
    act_bwd(n, n->d2);  conv_bwd(n, 9, n->d2a, n->d2.g, n->d2a.g, wgrad, true);
    conv_bwd(n, 8, n->c2, n->d2a.g, n->c2.g, wgrad);
    split(n->c2, n->e3, n->e2);
    act_bwd(n, n->e3);  conv_bwd(n, 7, n->e3a, n->e3.g, n->e3a.g, wgrad, true);
    conv_bwd(n, 6, n->p3, n->e3a.g, n->p3.g, wgrad);
    pool_bwd(n->p3, n->e2);
    act_bwd(n, n->e2);  conv_bwd(n, 5, n->e2a, n->e2.g, n->e2a.g, wgrad, true);
    conv_bwd(n, 4, n->p2, n->e2a.g, n->p2.g, wgrad);
    pool_bwd(n->p2, n->e1);
    act_bwd(n, n->e1);  conv_bwd(n, 3, n->e1a, n->e1.g, n->e1a.g, wgrad, true);
    conv_bwd(n, 2, n->p1, n->e1a.g, n->p1.g, wgrad);
    pool_bwd(n->p1, n->e0);
    act_bwd(n, n->e0);  conv_bwd(n, 1, n->e0a, n->e0.g, n->e0a.g, wgrad, true);
    conv_bwd(n, 0, n->x0, n->e0a.g, input ? n->x0.g : nullptr, wgrad);
}

extern "C" {

int fd_create(int32_t H, int32_t W, fd_net **out) { return fd_create_batch(H, W, 1, out); }

int fd_create_batch(int32_t H, int32_t W, int32_t N, fd_net **out) {
    if (!out) return -1;
    *out = nullptr;
    if (H <= 0 || W <= 0 || H % 8 || W % 8 || H > 4096 || W > 4096 || N < 1 || (N > 1 && H % 64) ||
        (long long)N * H * W > kMaxBatchPixels)
        return -1;
    fd_net *n = new fd_net();
    n->H = H; n->W = W; n->N = N;
    const int cin[15] = {16, 32, 32, 64, 64, 128, 128, 256, 384, 128, 192, 64, 96, 32, 32};
    const int cout[15] = {32, 32, 64, 64, 128, 128, 256, 256, 128, 128, 64, 64, 32, 32, 3};
    const int lev[15] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    size_t off = 0;
    for (int i = 0; i < 15; ++i) {
        Layer l{cin[i], cout[i], i < 14 ? 3 : 1, lev[i], 0, 0};
        l.woff = off; off += (size_t)l.cout * l.k * l.k * l.cin;
        l.boff = off; off += (size_t)l.cout;
        n->L.push_back(l);
    }
    n->nparam = off;
    int rc = 0;
    auto A = [&](Act &a, int c, int level) {
        a.c = c; a.level = level;
        size_t cnt = (size_t)N * (size_t)((H >> level) * (W >> level)) * c;
        if (!rc) rc = dalloc(n, &a.y, cnt);
        if (!rc) rc = dalloc(n, &a.g, cnt);
    };
    A(n->x0, 16, 0); A(n->e0a, 32, 0); A(n->e0, 32, 0); A(n->p1, 32, 1); A(n->e1a, 64, 1); A(n->e1, 64, 1);
    A(n->p2, 64, 2); A(n->e2a, 128, 2); A(n->e2, 128, 2); A(n->p3, 128, 3); A(n->e3a, 256, 3); A(n->e3, 256, 3);
    A(n->c2, 384, 2); A(n->d2a, 128, 2); A(n->d2, 128, 2); A(n->c1, 192, 1); A(n->d1a, 64, 1); A(n->d1, 64, 1);
    A(n->c0, 96, 0); A(n->d0a, 32, 0); A(n->d0, 32, 0);
    size_t P0 = (size_t)N * H * W;
    if (!rc) rc = dalloc(n, &n->params, n->nparam);
    if (!rc) rc = dalloc(n, &n->grads, n->nparam);
    if (!rc) rc = dalloc(n, &n->m, n->nparam);
    if (!rc) rc = dalloc(n, &n->v, n->nparam);
    if (!rc) rc = dalloc(n, &n->wbf, n->nparam);
    size_t wmax = 0;
    for (const Layer &l : n->L) wmax = std::max(wmax, (size_t)l.cin * l.k * l.k * l.cout);
    if (!rc) rc = dalloc(n, &n->wflip, wmax);
    if (!rc) rc = dalloc(n, &n->loss_s, 1);
    if (!rc) rc = dalloc(n, &n->pred, 3 * P0);
    if (!rc) rc = dalloc(n, &n->dpred, 3 * P0);
    if (rc) { fd_destroy(n); return -2; }
    (void)hipMemset(n->params, 0, n->nparam * sizeof(float));
    (void)hipMemset(n->m, 0, n->nparam * sizeof(float));
    (void)hipMemset(n->v, 0, n->nparam * sizeof(float));
    if (hipDeviceSynchronize() != hipSuccess) { fd_destroy(n); return -3; }
    *out = n;
    return 0;
}

int fd_set_stream(fd_net *n, void *s) {
    if (!n) return -1;
    n->stream = (hipStream_t)s;
    return 0;
}

int64_t fd_num_params(const fd_net *n) { return n ? (int64_t)n->nparam : -1; }

int fd_layer_shape(const fd_net *n, int32_t i, int32_t *cin, int32_t *cout, int32_t *k) {
    if (!n || i < 0 || i >= (int)n->L.size()) return -1;
    if (cin) *cin = n->L[i].cin;
    if (cout) *cout = n->L[i].cout;
    if (k) *k = n->L[i].k;
    return 0;
}

int fd_set_params(fd_net *n, const float *p) {
    if (!n) return -1;
    n->err.clear();
    if (!p) return fail(n, -1, "fd_set_params: null params");
    HIPCK(n, hipMemcpyAsync(n->params, p, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    HIPCK(n, hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->stream));
    HIPCK(n, hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->stream));
    n->step = 0;
    return 0;
}

int fd_get_params(const fd_net *n, float *p) {
    if (!n || !p) return -1;
    if (hipMemcpyAsync(p, n->params, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream) != hipSuccess) return -3;
    return 0;
}

int fd_get_state(const fd_net *n, float *p, float *m, float *v, int32_t *step) {
    if (!n) return -1;
    const size_t bytes = n->nparam * sizeof(float);
    if (p && hipMemcpyAsync(p, n->params, bytes, hipMemcpyDeviceToDevice, n->stream) != hipSuccess) return -3;
    if (m && hipMemcpyAsync(m, n->m, bytes, hipMemcpyDeviceToDevice, n->stream) != hipSuccess) return -3;
    if (v && hipMemcpyAsync(v, n->v, bytes, hipMemcpyDeviceToDevice, n->stream) != hipSuccess) return -3;
    if (step) *step = n->step;
    return 0;
}

int fd_set_state(fd_net *n, const float *p, const float *m, const float *v, int32_t step) {
    if (!n) return -1;
    n->err.clear();
    if (!p || !m || !v || step < 0) return fail(n, -1, "fd_set_state: null array or negative step");
    const size_t bytes = n->nparam * sizeof(float);
    HIPCK(n, hipMemcpyAsync(n->params, p, bytes, hipMemcpyDeviceToDevice, n->stream));
    HIPCK(n, hipMemcpyAsync(n->m, m, bytes, hipMemcpyDeviceToDevice, n->stream));
    HIPCK(n, hipMemcpyAsync(n->v, v, bytes, hipMemcpyDeviceToDevice, n->stream));
    n->step = step;
    return 0;
}

int fd_forward(fd_net *n, const float *rgb, const float *aux, float *out) {
    if (!n) return -1;
    n->err.clear();
    if (!rgb || !aux || !out) return fail(n, -1, "fd_forward: null argument");
    forward(n, rgb, aux);
    n->have_forward = true;
    int cnt = 3 * pix(n, 0);
    hipLaunchKernelGGL(k_expm1, dim3(nblk(cnt, 256)), dim3(256), 0, n->stream, cnt, n->pred, out);
    HIPCK(n, hipGetLastError());
    return 0;
}

int fd_train_step(fd_net *n, const float *rgb, const float *aux, const float *target, float lr, float *loss,
                  float *grads) {
    if (!n) return -1;
    n->err.clear();
    if (!rgb || !aux || !target) return fail(n, -1, "fd_train_step: null argument");
    if (!std::isfinite(lr)) return fail(n, -1, "fd_train_step: non-finite lr");
    forward(n, rgb, aux);
    n->have_forward = false;     // activations now belong to this step, not to an fd_forward
    int cnt = 3 * pix(n, 0);
    float *lp = loss ? loss : n->loss_s;
    hipLaunchKernelGGL(k_zero_f, dim3(1), dim3(64), 0, n->stream, (size_t)1, lp);
    hipLaunchKernelGGL(k_loss, dim3(nblk(cnt, kLossBlock)), dim3(256), 0, n->stream, cnt, n->pred, target, n->dpred, lp);
    backward(n, true, false);
    if (grads) HIPCK(n, hipMemcpyAsync(grads, n->grads, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    ++n->step;
    float c1 = (float)(1.0 - std::pow(0.9, n->step)), c2 = (float)(1.0 - std::pow(0.999, n->step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->nparam, 256)), dim3(256), 0, n->stream, n->nparam, n->params, n->grads, n->m,
                       n->v, lr, c1, c2);
    HIPCK(n, hipGetLastError());
    return 0;
}

int fd_backward_input(fd_net *n, const float *rgb, const float *dL_dout, float *dL_drgb) {
    if (!n) return -1;
    n->err.clear();
    if (!rgb || !dL_dout || !dL_drgb) return fail(n, -1, "fd_backward_input: null argument");
    if (!n->have_forward) return fail(n, -4, "fd_backward_input: no prior fd_forward");
    int P = pix(n, 0), cnt = 3 * P;
    hipLaunchKernelGGL(k_dout_dpred, dim3(nblk(cnt, 256)), dim3(256), 0, n->stream, cnt, n->pred, dL_dout, n->dpred);
    backward(n, false, true);
    hipLaunchKernelGGL(k_drgb, dim3(nblk(cnt, 256)), dim3(256), 0, n->stream, P, rgb, n->dpred, n->x0.g, dL_drgb);
    HIPCK(n, hipGetLastError());
    return 0;
}

// ---------------------------------------------------- single layers ----
int fd_conv3x3(void *stream, int32_t H, int32_t W, int32_t cin, int32_t cout, const void *x, int32_t x_is_f32,
               const uint16_t *w, const float *bias, int32_t relu, float *y) {
    if (H < 1 || W < 1 || H > 4096 || W > 4096 || cin < 16 || cin % 16 || cin > 4096 || cout < 1 || cout > 4096 ||
        !x || !w || !y)
        return -1;
    hipStream_t s = (hipStream_t)stream;
    if (x_is_f32)
        conv3x3_launch<float, float>(s, H, H, W, cin, cout, (const float *)x, (const bf16 *)w, bias, relu ? 1 : 0, y, cout, 0);
    else
        conv3x3_launch<bf16, float>(s, H, H, W, cin, cout, (const bf16 *)x, (const bf16 *)w, bias, relu ? 1 : 0, y, cout, 0);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int fd_conv3x3_wgrad(void *stream, int32_t H, int32_t W, int32_t cin, int32_t cout, const uint16_t *x, const float *g,
                     float *dw, float *db) {
    if (H < 1 || W < 1 || H > 4096 || W > 4096 || cin < 8 || cin % 8 || cin > 4096 || cout < 8 || cout % 8 ||
        cout > 4096 || !x || !g || !dw)
        return -1;
    hipStream_t s = (hipStream_t)stream;
    const size_t nw = (size_t)cout * 9 * cin;
    const int P = H * W;
    hipLaunchKernelGGL(k_zero_f, dim3(nblk(nw, 256)), dim3(256), 0, s, nw, dw);
    dim3 gw(nblk(cout, kWTile) * nblk(P, kWChunk), nblk(cin, kWTile), 9);
    hipLaunchKernelGGL(k_conv3x3_wgrad, gw, dim3(256), 0, s, H, H, W, cin, cout, (const bf16 *)x, g, dw);
    if (db) {
        hipLaunchKernelGGL(k_zero_f, dim3(nblk(cout, 256)), dim3(256), 0, s, (size_t)cout, db);
        hipLaunchKernelGGL(k_bias_grad, dim3(nblk(P, 256)), dim3(256), 0, s, P, cout, g, db);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

const char *fd_last_error(const fd_net *n) { return n ? n->err.c_str() : "null network"; }

void fd_destroy(fd_net *n) {
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream); else (void)hipDeviceSynchronize();
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

}  // extern "C"
