// Learned denoiser of low-count EPID images (Sec. 4.1): a 4-level U-Net in BF16 with FP32
// accumulation on the gfx950 matrix cores, its training (backward passes and Adam), and the
// C ABI of epidmc_denoise.h.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16.  The reduction index runs
// over groups of 8 input channels of one tap ("k-groups", kg = tap * c_in/8 + channel
// group), so every MFMA operand is one 16-byte word of 8 consecutive NHWC channels:
//   forward / backward-data   rows = pixels, columns = output channels.  3x3 layers with
//                             c_in a multiple of 32 (k_conv3_lds) stage a pixel tile with
//                             its halo and the weight slab in LDS per 32-channel step and
//                             read every operand from there, the 8-channel input layer
//                             (k_conv3_lds<2, true>) its whole patch at once; 1x1 layers
//                             (k_conv) load each lane's operands straight from memory;
//   backward-weights          rows = output channels, columns = (tap, input channel), the
//                             reduction runs over pixels, so both operands are staged
//                             through LDS transposed; pixel chunks give FP32 partials that
//                             a second kernel adds in a fixed order (deterministic).
// The backward-data convolution is the forward kernel on the gradient with the weights'
// channels transposed and taps reversed, its ReLU derivative fused as an output gate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "epidmc_denoise.h"

namespace dn {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;

__device__ __forceinline__ uint16_t f2bf(float f)   // round to nearest even (finite inputs)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ uint32_t pack(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }

// 8 BF16 values with every one whose gate element is not > 0 set to +0 (the ReLU derivative
// of a backward-data pass)
__device__ __forceinline__ u32x4 gated(u32x4 v, u32x4 g)
{
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t keep = (lo(g[w]) > 0.0f ? 0x0000FFFFu : 0u) | (hi(g[w]) > 0.0f ? 0xFFFF0000u : 0u);
        v[w] &= keep;
    }
    return v;
}

constexpr int HC = 32;   // head input channels

// the head's correction r = bh + wh . t for one pixel's HC BF16 channels (t, 16-byte aligned)
__device__ __forceinline__ float head_r(const u32x4 *src, const float *wh, const float *bh)
{
    float t[HC];
#pragma unroll
    for (int q = 0; q < HC / 8; ++q) {
        const u32x4 v = src[q];
#pragma unroll
        for (int j = 0; j < 4; ++j) { t[8 * q + 2 * j] = lo(v[j]); t[8 * q + 2 * j + 1] = hi(v[j]); }
    }
    float r = bh[0];
#pragma unroll
    for (int c = 0; c < HC; ++c) r += wh[c] * t[c];
    return r;
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// ---------------------------------------------------------------------------------------
// convolution (forward and backward-data)
// ---------------------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t *x, *w, *gate;
    const float *bias;
    uint16_t *y;
    uint16_t *pool;          // k_conv3_lds only: also the 2 x 2 average of y (h, w even), or null
    long long P;             // pixels n * h * w
    int ldx, ldy, ldg, cin, cout, h, wd, relu, ldp;
    int up;                  // k_conv only: y is the 2x nearest-neighbour upsampling (2h x 2w) of the output
    // k_conv3_lds with c_out = 32 only (inference): instead of storing y, apply the network's
    // head to it and write the denoised image, img = (x0 + bh + wh . y) * s per pixel
    const float *head_w, *head_b, *head_x0;
    const double *head_s;
    double *head_img;
    int cg_shift, kg_total;  // log2(c_in / 8), k * k * c_in / 8
};

// A wave computes MT*16 pixels (MT row tiles) x NT*16 output channels; the 4 waves of a block
// take consecutive pixel tiles and share the weight columns.  MT = 1 gives four times the
// blocks of MT = 4, for layers whose pixel count would otherwise leave CUs idle.
template <int KS, int NT, int MT, bool UP = false>
__global__ __launch_bounds__(WG) void k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const long long p0 = ((long long)blockIdx.x * 4 + wave) * (16 * MT);
    const int co0 = blockIdx.y * NT * 16;
    const int hw = a.h * a.wd;
    int py[MT], px[MT];
    long long pbase[MT];
    bool pv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const long long p = p0 + m * 16 + row;
        pv[m] = p < a.P;
        const long long pc = pv[m] ? p : 0;
        const int n = (int)(pc / hw), r = (int)(pc - (long long)n * hw);
        py[m] = r / a.wd;
        px[m] = r - py[m] * a.wd;
        pbase[m] = (long long)n * hw;
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kstride = a.kg_total * 8;
    const uint16_t *wrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) wrow[t] = a.w + (long long)(co0 + t * 16 + row) * kstride;
    const int steps = (a.kg_total + 3) >> 2;
    const int cmask = (1 << a.cg_shift) - 1;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    // operands of step s: A (4 pixel rows) and B (NT weight columns), zero past the end
    auto load = [&](int s, u32x4 *A, u32x4 *B) {
        const int kg = s * 4 + grp;
        const bool kv = kg < a.kg_total;
        const int tap = kg >> a.cg_shift, cg = kg & cmask;
        const int dy = KS == 3 ? tap / 3 - 1 : 0;
        const int dx = KS == 3 ? tap - (tap / 3) * 3 - 1 : 0;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int yy = py[m] + dy, xx = px[m] + dx;
            const bool ok = kv && pv[m] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
            const long long off = ok ? ((pbase[m] + (long long)yy * a.wd + xx) * a.ldx + cg * 8) : 0;
            const u32x4 v = *(const u32x4 *)(a.x + off);
            A[m] = ok ? v : zero;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const u32x4 v = *(const u32x4 *)(wrow[t] + (kv ? kg * 8 : 0));
            B[t] = kv ? v : zero;
        }
    };
    // two register stages: the loads of step s+1 are in flight during step s's MFMAs.  The
    // step count is rounded up to even; a step past the end loads zeros.
    const int steps2 = (steps + 1) & ~1;
    u32x4 A0[MT], B0[NT], A1[MT], B1[NT];
    load(0, A0, B0);
    for (int s = 0; s < steps2; s += 2) {
        load(s + 1, A1, B1);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A0[m], B0[t], acc[m][t]);
        load(s + 2 < steps2 ? s + 2 : s + 1, A0, B0);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A1[m], B1[t], acc[m][t]);
    }
    // Epilogue through LDS: the wave's MT*16-pixel x NT*16-channel tile of BF16 outputs
    // (bias, ReLU and gate applied; lane (row, grp) holds pixels 4*grp + r of each 16-pixel
    // tile, channel `row` of each channel tile) is written pixel-major and read back as
    // 16-byte runs of 8 channels, so that every global store writes 8 consecutive NHWC
    // channels (four of them, the 2 x 2 block, with UP).
    constexpr int EP = NT * 16 + 8;   // bf16 per staged pixel
    __shared__ __align__(16) uint16_t Es[4 * 16 * MT * EP];
    uint16_t *E = Es + wave * 16 * MT * EP;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = co0 + t * 16 + row;
        const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[m][t][r] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                E[(m * 16 + grp * 4 + r) * EP + t * 16 + row] = f2bf(v);
            }
    }
    __syncthreads();
    constexpr int CG = NT * 2;   // 8-channel groups per pixel
#pragma unroll
    for (int k = 0; k < (16 * MT * CG + 63) / 64; ++k) {
        const int j = k * 64 + lane;
        const int P = j / CG, c8 = j % CG;
        const long long p = p0 + P;
        if (P >= 16 * MT || p >= a.P) continue;
        const u32x4 v = *(const u32x4 *)(E + P * EP + c8 * 8);
        if (UP) {
            const int n = (int)(p / hw), rr = (int)(p - (long long)n * hw);
            const int yi = rr / a.wd, xi = rr - yi * a.wd;
            const long long q = ((long long)n * 2 * a.h + 2 * yi) * (2 * a.wd) + 2 * xi, q2 = q + 2 * a.wd;
            uint16_t *d = a.y + co0 + c8 * 8;
            *(u32x4 *)(d + q * a.ldy) = v;
            *(u32x4 *)(d + (q + 1) * a.ldy) = v;
            *(u32x4 *)(d + q2 * a.ldy) = v;
            *(u32x4 *)(d + (q2 + 1) * a.ldy) = v;
        } else {
            *(u32x4 *)(a.y + p * a.ldy + co0 + c8 * 8) =
                a.gate ? gated(v, *(const u32x4 *)(a.gate + p * a.ldg + co0 + c8 * 8)) : v;
        }
    }
}

// 3x3 convolution with LDS tiles (c_in a multiple of 32): a workgroup owns an 8 x 32 pixel
// tile of one image and NT*16 output channels.  Per step of 32 input channels it stages the
// 10 x 34 input patch (halo included, zeros outside the image) and the weight slab
// [NT*16][9 taps][32], then every wave (2 rows x 32 columns = 4 row tiles) runs the 9 taps
// from LDS.  Row pitches of 80 and 592 bytes make the 16-byte reads of 16 lanes fall on
// distinct banks.
constexpr int TLH = 8, TLW = 32, PH = TLH + 2, PW = TLW + 2;
constexpr int XP = 40;          // bf16 per staged pixel (32 channels + pad)
constexpr int WP = 9 * 32 + 8;  // bf16 per staged output channel (9 taps x 32 + pad)

// C8: the 8-channel input layer (c_in = 8, c_out = 32).  The patch holds 16 bytes per pixel
// and the weights [co][12 taps][8] (taps 9-11 zero); an MFMA's 32-deep K takes 4 taps of 8
// channels, lane group g tap 4s + g at step s, in the order of the generic kernel.
constexpr int W8 = 12 * 8 + 8;  // C8: bf16 per staged output channel (12 taps x 8 + pad)

template <int NT, bool C8 = false>
__global__ __launch_bounds__(WG) void k_conv3_lds(ConvArgs a, int tiles_x)
{
    static_assert(!C8 || NT == 2, "the 8-channel input layer has 32 output channels");
    constexpr int XS = C8 ? 4 * 64 * (NT * 16 + 8) : PH * PW * XP;   // C8: sized for the epilogue
    __shared__ __align__(16) uint16_t Xs[XS];
    __shared__ __align__(16) uint16_t Ws[C8 ? NT * 16 * W8 : NT * 16 * WP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const int ty0 = (blockIdx.x / tiles_x) * TLH, tx0 = (blockIdx.x % tiles_x) * TLW;
    const int img = blockIdx.y;
    const int co0 = blockIdx.z * NT * 16;
    const long long ibase = (long long)img * a.h * a.wd;
    const int kstride = 9 * a.cin;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    if constexpr (C8) {
        for (int it = tid; it < PH * PW; it += WG) {
            const int y = ty0 + it / PW - 1, x = tx0 + it % PW - 1;
            const bool ok = y >= 0 && y < a.h && x >= 0 && x < a.wd;
            const long long off = ok ? (ibase + (long long)y * a.wd + x) * a.ldx : 0;
            const u32x4 v = *(const u32x4 *)(a.x + off);
            *(u32x4 *)(Xs + it * 8) = ok ? v : zero;
        }
        for (int it = tid; it < NT * 16 * 12; it += WG) {
            const int co = it / 12, tap = it % 12;
            const long long off = tap < 9 ? (long long)(co0 + co) * kstride + tap * 8 : 0;
            const u32x4 v = *(const u32x4 *)(a.w + off);
            *(u32x4 *)(Ws + co * W8 + tap * 8) = tap < 9 ? v : zero;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            const int tap = 4 * st + grp;
            const bool tv = tap < 9;
            const int dy = tv ? tap / 3 : 0, dx = tv ? tap - (tap / 3) * 3 : 0;
            u32x4 A[4], B[NT];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int q = (2 * wave + (m >> 1) + dy) * PW + (m & 1) * 16 + row + dx;
                const u32x4 v = *(const u32x4 *)(Xs + q * 8);
                A[m] = tv ? v : zero;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) B[t] = *(const u32x4 *)(Ws + (t * 16 + row) * W8 + tap * 8);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A[m], B[t], acc[m][t]);
        }
        __syncthreads();
    } else {
    // the next step's patch and weights are loaded into registers while the current step's
    // MFMAs run, and stored to LDS after the barrier
    constexpr int XI = PH * PW * 4, XN = (XI + WG - 1) / WG;
    constexpr int WI = NT * 16 * 36, WN = (WI + WG - 1) / WG;
    u32x4 xr[XN], wr[WN];
    auto gload = [&](int c0) {
#pragma unroll
        for (int k = 0; k < XN; ++k) {
            const int it = tid + k * WG;
            const int q = it >> 2, g = it & 3;
            const int y = ty0 + q / PW - 1, x = tx0 + q % PW - 1;
            const bool ok = it < XI && y >= 0 && y < a.h && x >= 0 && x < a.wd;
            const long long off = ok ? (ibase + (long long)y * a.wd + x) * a.ldx + c0 + g * 8 : 0;
            const u32x4 v = *(const u32x4 *)(a.x + off);
            xr[k] = ok ? v : zero;
        }
#pragma unroll
        for (int k = 0; k < WN; ++k) {
            const int it = tid + k * WG;
            const int co = it / 36, r = it % 36, tap = r >> 2, g = r & 3;
            const bool ok = it < WI;
            const long long off = ok ? (long long)(co0 + co) * kstride + tap * a.cin + c0 + g * 8 : 0;
            wr[k] = *(const u32x4 *)(a.w + off);
        }
    };
    gload(0);
    for (int c0 = 0; c0 < a.cin; c0 += 32) {
#pragma unroll
        for (int k = 0; k < XN; ++k) {
            const int it = tid + k * WG;
            if (it < XI) *(u32x4 *)(Xs + (it >> 2) * XP + (it & 3) * 8) = xr[k];
        }
#pragma unroll
        for (int k = 0; k < WN; ++k) {
            const int it = tid + k * WG;
            if (it < WI) {
                const int co = it / 36, r = it % 36;
                *(u32x4 *)(Ws + co * WP + (r >> 2) * 32 + (r & 3) * 8) = wr[k];
            }
        }
        __syncthreads();
        if (c0 + 32 < a.cin) gload(c0 + 32);
#pragma unroll 1
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap - dy * 3;
            u32x4 A[4], B[NT];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int q = (2 * wave + (m >> 1) + dy) * PW + (m & 1) * 16 + row + dx;
                A[m] = *(const u32x4 *)(Xs + q * XP + grp * 8);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) B[t] = *(const u32x4 *)(Ws + (t * 16 + row) * WP + tap * 32 + grp * 8);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[m][t] = mfma(A[m], B[t], acc[m][t]);
        }
        __syncthreads();
    }
    }
    // Epilogue through LDS (the staging buffers are free after the last barrier): each wave
    // writes its 64-pixel x NT*16-channel tile of BF16 outputs (bias, ReLU and gate applied)
    // pixel-major, then reads it back as 16-byte runs of 8 channels, so that every global
    // store writes 8 consecutive NHWC channels instead of one.  Wave-local pixel P = m*16 +
    // grp*4 + r lies at row P / 32 and column P % 32 of the wave's two rows.
    constexpr int EP = NT * 16 + 8;   // bf16 per staged pixel (80 or 144 bytes)
    uint16_t *E = (NT == 4 ? Ws : Xs) + wave * 64 * EP;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = co0 + t * 16 + row;
        const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[m][t][r] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                E[(m * 16 + grp * 4 + r) * EP + t * 16 + row] = f2bf(v);
            }
    }
    __syncthreads();
    if (NT * 16 == HC && a.head_img) {
        // the head (inference): every lane one pixel of the wave's tile, its HC channels read
        // from the staged tile; the convolution's own output is not stored
        const int y = ty0 + 2 * wave + (lane >> 5), x = tx0 + (lane & 31);
        if (y < a.h && x < a.wd) {
            const long long pg = ibase + (long long)y * a.wd + x;
            const float out = a.head_x0[pg] + head_r((const u32x4 *)(E + lane * EP), a.head_w, a.head_b);
            a.head_img[pg] = (double)out * a.head_s[img];
        }
        return;
    }
    constexpr int CG = NT * 2;   // 8-channel groups per pixel
#pragma unroll
    for (int k = 0; k < CG; ++k) {
        const int j = k * 64 + lane, P = j / CG, c8 = j % CG;
        const int y = ty0 + 2 * wave + (P >> 5), x = tx0 + (P & 31);
        if (y >= a.h || x >= a.wd) continue;
        const long long pg = ibase + (long long)y * a.wd + x;
        u32x4 v = *(const u32x4 *)(E + P * EP + c8 * 8);
        if (a.gate) v = gated(v, *(const u32x4 *)(a.gate + pg * a.ldg + co0 + c8 * 8));
        *(u32x4 *)(a.y + pg * a.ldy + co0 + c8 * 8) = v;
    }
    if (a.pool) {
        // the 2 x 2 average of the stored (BF16) outputs, added in the order of a separate
        // pooling pass: the wave's two rows are one pooled row of 16 pixels
        const int y = ty0 + 2 * wave;
#pragma unroll
        for (int k = 0; k < (16 * CG + 63) / 64; ++k) {
            const int j = k * 64 + lane;
            if (j >= 16 * CG) break;
            const int px = j / CG, c8 = j % CG;
            const int x = tx0 + 2 * px;
            if (y >= a.h || x >= a.wd) continue;
            u32x4 w4[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) w4[2 * i + jj] = *(const u32x4 *)(E + (i * 32 + 2 * px + jj) * EP + c8 * 8);
            u32x4 o;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) { s0 += lo(w4[q][w]); s1 += hi(w4[q][w]); }
                o[w] = pack(0.25f * s0, 0.25f * s1);
            }
            const long long q = ((long long)img * (a.h / 2) + y / 2) * (a.wd / 2) + x / 2;
            *(u32x4 *)(a.pool + q * a.ldp + co0 + c8 * 8) = o;
        }
    }
}

// ---------------------------------------------------------------------------------------
// backward-weights convolution
// ---------------------------------------------------------------------------------------
struct WgArgs {
    const uint16_t *x, *g;
    float *part;
    int with_db;
    long long P;
    int ldx, ldg, cin, cout, h, wd, cg_shift, kg_total, cols, cols_pad, chunk_px;
};

// Block tile: TM = 32 * WM output channels x TN = 32 * (4 / WM) columns; each wave a 32 x 32
// sub-tile (2 x 2 MFMA tiles).  Per step of KP = 128 pixels the block stages g (pixels x
// channels) and the shifted input (pixels x columns) into LDS transposed, so that a lane's
// operand is 8 consecutive pixels of one row.  Each staging item is an 8-pixel x 8-channel
// block: eight 16-byte loads, a register transpose (byte permutes) and eight 16-byte LDS
// stores.
constexpr int KP = 128, KPP = KP + 8;   // pixels per step; LDS row pitch (272 bytes)

// out[j] = channel j of pixels 0..7, two pixels per word, from in[p] = pixel p's 8 channels
__device__ __forceinline__ void transpose8(const u32x4 in[8], u32x4 out[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int w = c >> 1;
        const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;   // high or low halves
#pragma unroll
        for (int q = 0; q < 4; ++q) out[c][q] = __builtin_amdgcn_perm(in[2 * q + 1][w], in[2 * q][w], sel);
    }
}

// LDS position of 16-byte chunk `chunk` (8 pixels) of staged row `row`: the chunk index is
// XOR-ed with bits 1-2 of row / 8.  A staging write stores one chunk of 16 rows that are 8
// apart (two pixel groups x eight channel groups), which without the swizzle fall on four bank
// groups of the 272-byte rows; with it, on sixteen.  A read takes one chunk of 16 consecutive
// rows, which share the swizzle and stay on distinct banks.
__device__ __forceinline__ int swz(int chunk, int row) { return chunk ^ ((row >> 3) & 6); }

template <int KS, int WM>
__global__ __launch_bounds__(WG) void k_wgrad(WgArgs a)
{
    constexpr int TM = 32 * WM, TN = 32 * (4 / WM);
    __shared__ __align__(16) uint16_t Gt[TM * KPP];
    __shared__ __align__(16) uint16_t Xt[TN * KPP];
    __shared__ float red[KP / 8][TM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int co0 = blockIdx.x * TM, col0 = blockIdx.y * TN;
    const long long pc0 = (long long)blockIdx.z * a.chunk_px;
    const long long pc1 = min(pc0 + (long long)a.chunk_px, a.P);
    const int hw = a.h * a.wd;
    const int cmask = (1 << a.cg_shift) - 1;
    const bool do_db = a.with_db && blockIdx.y == 0;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbacc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dbacc[j] = 0.0f;
    constexpr int GI = (KP / 8) * (TM / 8), XI = (KP / 8) * (TN / 8);   // 8 x 8 items per tile
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (long long pb = pc0; pb < pc1; pb += KP) {
        if (tid < GI) {   // item: pixel group pg, channel group c8 (fixed per thread)
            const int pg = tid / (TM / 8), c8 = tid % (TM / 8);
            u32x4 in[8], out[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const long long p = pb + pg * 8 + j;
                const bool ok = p < pc1;
                const u32x4 v = *(const u32x4 *)(a.g + (ok ? p * a.ldg + co0 + c8 * 8 : 0));
                in[j] = ok ? v : zero;
#pragma unroll
                for (int q = 0; q < 4; ++q) { dbacc[2 * q] += lo(in[j][q]); dbacc[2 * q + 1] += hi(in[j][q]); }
            }
            transpose8(in, out);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u32x4 *)(Gt + (c8 * 8 + c) * KPP + swz(pg, c8 * 8 + c) * 8) = out[c];
        }
        for (int it = tid; it < XI; it += WG) {
            const int pg = it / (TN / 8), kl = it % (TN / 8);
            const int kg = col0 / 8 + kl;
            const bool kv = kg < a.kg_total;
            const int tap = kg >> a.cg_shift, cg = kg & cmask;
            const int dy = KS == 3 ? tap / 3 - 1 : 0, dx = KS == 3 ? tap % 3 - 1 : 0;
            u32x4 in[8], out[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const long long p = pb + pg * 8 + j;
                bool ok = kv && p < pc1;
                long long off = 0;
                if (ok) {
                    const int n = (int)(p / hw), r = (int)(p - (long long)n * hw);
                    const int y = r / a.wd + dy, x = r % a.wd + dx;
                    ok = y >= 0 && y < a.h && x >= 0 && x < a.wd;
                    off = ((long long)n * hw + (long long)y * a.wd + x) * a.ldx + cg * 8;
                }
                const u32x4 v = *(const u32x4 *)(a.x + (ok ? off : 0));
                in[j] = ok ? v : zero;
            }
            transpose8(in, out);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u32x4 *)(Xt + (kl * 8 + c) * KPP + swz(pg, kl * 8 + c) * 8) = out[c];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks) {
            u32x4 A[2], B[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm * 32 + i * 16 + (lane & 15);
                A[i] = *(const u32x4 *)(Gt + r * KPP + swz(ks * 4 + (lane >> 4), r) * 8);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int r = wn * 32 + j * 16 + (lane & 15);
                B[j] = *(const u32x4 *)(Xt + r * KPP + swz(ks * 4 + (lane >> 4), r) * 8);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma(A[i], B[j], acc[i][j]);
        }
        __syncthreads();
    }
    const size_t R = (size_t)a.cout * a.cols_pad + a.cout;   // one row per pixel chunk: dw, then db
    float *dst = a.part + (size_t)blockIdx.z * R;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = col0 + wn * 32 + j * 16 + (lane & 15);
                dst[(size_t)co * a.cols_pad + col] = acc[i][j][r];
            }
    if (do_db) {
        if (tid < GI) {
            const int pg = tid / (TM / 8), c8 = tid % (TM / 8);
#pragma unroll
            for (int j = 0; j < 8; ++j) red[pg][c8 * 8 + j] = dbacc[j];
        }
        __syncthreads();
        if (tid < TM) {
            float sum = 0.0f;
            for (int pg = 0; pg < KP / 8; ++pg) sum += red[pg][tid];
            dst[(size_t)a.cout * a.cols_pad + co0 + tid] = sum;
        }
    }
}

// Sum of the pixel chunks' partial rows (R floats each) in a fixed order: stage 1 adds
// groups of RG consecutive chunks (threads run along the row, so loads are coalesced),
// stage 2 adds the groups and scatters the row into dw [cout][cols] and db [cout].
constexpr int RG = 32;
__global__ void k_wgrad_sum1(const float *part, long long R, int nchunk, float *stage)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R) return;
    const int c0 = blockIdx.y * RG, c1 = min(c0 + RG, nchunk);
    float s = 0.0f;
    for (int c = c0; c < c1; ++c) s += part[(size_t)c * R + e];
    stage[(size_t)blockIdx.y * R + e] = s;
}

__global__ void k_wgrad_sum2(const float *stage, long long R, int ngroup, int cout, int cols, int cols_pad, float *dw,
                             float *db)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R) return;
    float s = 0.0f;
    for (int g = 0; g < ngroup; ++g) s += stage[(size_t)g * R + e];
    const long long nw = (long long)cout * cols_pad;
    if (e < nw) {
        const int co = (int)(e / cols_pad), col = (int)(e - (long long)co * cols_pad);
        if (col < cols) dw[(long long)co * cols + col] = s;
    } else if (db) {
        db[e - nw] = s;
    }
}

// ---------------------------------------------------------------------------------------
// weights, pooling, upsampling, skip gradient
// ---------------------------------------------------------------------------------------
__global__ void k_weights(const float *w, int cout, int kk, int cin, uint16_t *wf, uint16_t *wb)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)cout * kk * cin) return;
    const int c = (int)(i % cin), tap = (int)((i / cin) % kk), o = (int)(i / ((long long)cin * kk));
    const uint16_t v = f2bf(w[i]);
    if (wf) wf[i] = v;
    if (wb) wb[((long long)c * kk + (kk - 1 - tap)) * cout + o] = v;
}

// all layers' conversions in one launch: layer j takes blocks [first_block[j], first_block[j+1])
constexpr int WT_MAX = 24;
struct WeightTable {
    int n;
    int first_block[WT_MAX + 1];
    long long off[WT_MAX];
    int cout[WT_MAX], kk[WT_MAX], cin[WT_MAX];
};

__global__ void k_weights_all(const float *theta, uint16_t *wf, uint16_t *wb, WeightTable t)
{
    int j = 0;
    while (j + 1 < t.n && (int)blockIdx.x >= t.first_block[j + 1]) ++j;
    const int cout = t.cout[j], kk = t.kk[j], cin = t.cin[j];
    const long long i = (long long)(blockIdx.x - t.first_block[j]) * blockDim.x + threadIdx.x;
    if (i >= (long long)cout * kk * cin) return;
    const int c = (int)(i % cin), tap = (int)((i / cin) % kk), o = (int)(i / ((long long)cin * kk));
    const uint16_t v = f2bf(theta[t.off[j] + i]);
    wf[t.off[j] + i] = v;
    wb[t.off[j] + ((long long)c * kk + (kk - 1 - tap)) * cout + o] = v;
}

// one thread per (output pixel, 8-channel group)
__global__ void k_pool(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int wd)
{
    const int G = c / 8, ho = h / 2, wo = wd / 2;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ho * wo * G) return;
    const int g = (int)(i % G);
    const long long q = i / G;
    const int xo = (int)(q % wo), yo = (int)((q / wo) % ho), im = (int)(q / ((long long)wo * ho));
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const long long p = ((long long)im * h + 2 * yo + a) * wd + 2 * xo + b;
            const u32x4 v = *(const u32x4 *)(x + p * ldx + g * 8);
            for (int j = 0; j < 4; ++j) { s[2 * j] += lo(v[j]); s[2 * j + 1] += hi(v[j]); }
        }
    u32x4 o;
    for (int j = 0; j < 4; ++j) o[j] = pack(0.25f * s[2 * j], 0.25f * s[2 * j + 1]);
    *(u32x4 *)(y + q * ldy + g * 8) = o;
}

// one thread per (input pixel, group), writing its 2 x 2 block
__global__ void k_upsample(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int wd)
{
    const int G = c / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * h * wd * G) return;
    const int g = (int)(i % G);
    const long long q = i / G;
    const int xi = (int)(q % wd), yi = (int)((q / wd) % h), im = (int)(q / ((long long)wd * h));
    const u32x4 v = *(const u32x4 *)(x + q * ldx + g * 8);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const long long p = ((long long)im * 2 * h + 2 * yi + a) * (2 * wd) + 2 * xi + b;
            *(u32x4 *)(y + p * ldy + g * 8) = v;
        }
}

__global__ void k_upsample_bwd(const uint16_t *gi, int ldg, uint16_t *y, int ldy, int c, int n, int h, int wd)
{
    const int G = c / 8, ho = h / 2, wo = wd / 2;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * ho * wo * G) return;
    const int g = (int)(i % G);
    const long long q = i / G;
    const int xo = (int)(q % wo), yo = (int)((q / wo) % ho), im = (int)(q / ((long long)wo * ho));
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const long long p = ((long long)im * h + 2 * yo + a) * wd + 2 * xo + b;
            const u32x4 v = *(const u32x4 *)(gi + p * ldg + g * 8);
            for (int j = 0; j < 4; ++j) { s[2 * j] += lo(v[j]); s[2 * j + 1] += hi(v[j]); }
        }
    u32x4 o;
    for (int j = 0; j < 4; ++j) o[j] = pack(s[2 * j], s[2 * j + 1]);
    *(u32x4 *)(y + q * ldy + g * 8) = o;
}

__global__ void k_skip_bwd(const uint16_t *gs, int lds, const uint16_t *gp, int ldp, const uint16_t *act, int lda,
                           uint16_t *out, int ldo, int c, int n, int h, int wd)
{
    const int G = c / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * h * wd * G) return;
    const int g = (int)(i % G);
    const long long q = i / G;
    const int x = (int)(q % wd), y = (int)((q / wd) % h), im = (int)(q / ((long long)wd * h));
    const long long qp = ((long long)im * (h / 2) + y / 2) * (wd / 2) + x / 2;
    const u32x4 a = *(const u32x4 *)(gs + q * lds + g * 8);
    const u32x4 b = *(const u32x4 *)(gp + qp * ldp + g * 8);
    const u32x4 m = *(const u32x4 *)(act + q * lda + g * 8);
    u32x4 o;
    for (int j = 0; j < 4; ++j) {
        const float v0 = lo(m[j]) > 0.0f ? lo(a[j]) + 0.25f * lo(b[j]) : 0.0f;
        const float v1 = hi(m[j]) > 0.0f ? hi(a[j]) + 0.25f * hi(b[j]) : 0.0f;
        o[j] = pack(v0, v1);
    }
    *(u32x4 *)(out + q * ldo + g * 8) = o;
}

// ---------------------------------------------------------------------------------------
// input normalisation, head and loss, Adam
// ---------------------------------------------------------------------------------------
// partial sums of each image: grid (blocks per image, images)
__global__ void k_img_sum(const double *img, long long hw, int nb, double *part)
{
    __shared__ double sh[WG];
    const int im = blockIdx.y;
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < hw; i += (long long)nb * WG)
        s += img[(long long)im * hw + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = WG / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[im * nb + blockIdx.x] = sh[0];
}

// Scale of image blockIdx.y (its mean; 1 for an image whose mean is not positive) from the
// partial sums, added in a fixed tree order; then the batch's 8-channel BF16 input, FP32
// image channel and target.  Block (0, i) also stores image i's scale for the head.
__global__ __launch_bounds__(WG) void k_prepare(const double *noisy, const double *thick, const double *target,
                                                const double *part, int nb, long long hw, uint16_t *x, float *x0,
                                                float *tgt, double *scale)
{
    __shared__ double sh[WG];
    const int im = blockIdx.y;
    double t = 0.0;
    for (int b = threadIdx.x; b < nb; b += WG) t += part[(long long)im * nb + b];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int k = WG / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    const double m = sh[0] / (double)hw;
    const double sc = m > 0.0 ? m : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) scale[im] = sc;
    const long long q = (long long)blockIdx.x * WG + threadIdx.x;
    if (q >= hw) return;
    const long long p = (long long)im * hw + q;
    const double inv = 1.0 / sc;
    const double v = noisy[p] * inv;
    u32x4 o = {pack((float)v, (float)(thick[p] * (1.0 / 20.0))), 0u, 0u, 0u};
    *(u32x4 *)(x + p * 8) = o;
    x0[p] = (float)v;
    if (target) tgt[p] = (float)(target[p] * inv);
}

// training head, per pixel: r = bh + wh . t0[p]; out = x0 + r; squared error against tgt,
// dL/dr = 2 (out - tgt) / P, gradient at t0 gated by t0 > 0, and per-block partial sums of
// the loss, dL/db and dL/dw (34 floats per block).  (Inference applies the same head in the
// last convolution's epilogue.)
__global__ __launch_bounds__(WG) void k_head(const uint16_t *t0, const float *wh, const float *bh, const float *x0,
                                             const float *tgt, long long P, uint16_t *g0, float *part)
{
    __shared__ float red[WG / 64][HC + 2];
    const long long p = (long long)blockIdx.x * WG + threadIdx.x;
    const bool live = p < P;
    float t[HC];
    const u32x4 *src = (const u32x4 *)(t0 + (live ? p : 0) * HC);
#pragma unroll
    for (int q = 0; q < HC / 8; ++q) {
        const u32x4 v = src[q];
#pragma unroll
        for (int j = 0; j < 4; ++j) { t[8 * q + 2 * j] = lo(v[j]); t[8 * q + 2 * j + 1] = hi(v[j]); }
    }
    const float out = (live ? x0[p] : 0.0f) + head_r(src, wh, bh);
    const float d = live ? out - tgt[p] : 0.0f;
    const float gr = 2.0f * d / (float)P;
    if (live) {
        u32x4 *dst = (u32x4 *)(g0 + p * HC);
#pragma unroll
        for (int q = 0; q < HC / 8; ++q) {
            u32x4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 8 * q + 2 * j;
                o[j] = pack(t[c] > 0.0f ? gr * wh[c] : 0.0f, t[c + 1] > 0.0f ? gr * wh[c + 1] : 0.0f);
            }
            dst[q] = o;
        }
    }
    float v[HC + 2];
#pragma unroll
    for (int c = 0; c < HC; ++c) v[c] = gr * t[c];
    v[HC] = gr;
    v[HC + 1] = d * d;
#pragma unroll
    for (int c = 0; c < HC + 2; ++c)
        for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < HC + 2; ++c) red[wave][c] = v[c];
    __syncthreads();
    if (threadIdx.x < HC + 2) {
        float sum = 0.0f;
        for (int w = 0; w < WG / 64; ++w) sum += red[w][threadIdx.x];
        part[(size_t)blockIdx.x * (HC + 2) + threadIdx.x] = sum;
    }
}

// dw (HC floats), db, and loss = sum of squares / P from the blocks' partials: one block
// per output, strided FP64 sums and a fixed-order tree
__global__ __launch_bounds__(WG) void k_head_reduce(const float *part, int nblk, long long P, float *dw, float *db,
                                                    double *loss)
{
    __shared__ double sh[WG];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += WG) s += part[(size_t)b * (HC + 2) + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = WG / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x) return;
    if (c < HC) dw[c] = (float)sh[0];
    else if (c == HC) db[0] = (float)sh[0];
    else if (loss) loss[0] = sh[0] / (double)P;
}

// Adam on the FP32 master weights; when ema != NULL the exponential moving average of the
// weights follows: ema <- d * ema + (1 - d) * theta (after the step)
__global__ void k_adam(float *th, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, float *ema, float d)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = th[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    th[i] = t;
    if (ema) ema[i] = fmaf(d, ema[i] - t, t);
}

__global__ void k_fill_f32(float *p, long long n, float v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy_f32(const float *a, float *b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
static inline unsigned nblocks(long long n, int per = WG) { return (unsigned)((n + per - 1) / per); }
static int ilog2(int v) { int s = 0; while ((1 << s) < v) ++s; return s; }
static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// compute units of the current device (cached per device)
static int n_cu()
{
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

// the network's head applied in a convolution's epilogue: img = (x0 + b + w . y) * s[image]
struct Head {
    const float *w, *b, *x0;
    const double *s;
    double *img;
};

// y = act(conv(x)); with `pool`, also the 2 x 2 average pooling of y into pool (h and w
// even, no gate), inside the convolution's epilogue where the LDS-tiled kernel runs, else by
// a separate pass; with `up` (1 x 1 convolutions, no gate), y is the output upsampled 2x by
// nearest neighbour, written by the epilogue; with `head` (3 x 3, c_in a multiple of 32,
// c_out = HC, no gate or pool), y is not stored and the head's image is written instead
static hipError_t launch_conv(const uint16_t *x, int ldx, int cin, const uint16_t *w, const float *bias, uint16_t *y,
                              int ldy, int cout, const uint16_t *gate, int ldg, int n, int h, int wd, int k, int relu,
                              hipStream_t s, uint16_t *pool = nullptr, int ldp = 0, int up = 0,
                              const Head *head = nullptr)
{
    ConvArgs a;
    a.x = x; a.w = w; a.gate = gate; a.bias = bias; a.y = y; a.pool = nullptr;
    a.head_w = head ? head->w : nullptr; a.head_b = head ? head->b : nullptr;
    a.head_x0 = head ? head->x0 : nullptr; a.head_s = head ? head->s : nullptr;
    a.head_img = head ? head->img : nullptr;
    a.P = (long long)n * h * wd;
    a.ldx = ldx; a.ldy = ldy; a.ldg = ldg; a.cin = cin; a.cout = cout; a.h = h; a.wd = wd; a.relu = relu; a.ldp = ldp;
    a.up = up;
    a.cg_shift = ilog2(cin / 8);
    a.kg_total = k * k * cin / 8;
    if (a.P == 0) return hipSuccess;
    if (pool && (h % 2 || wd % 2 || gate || cout % 8 || up)) return hipErrorInvalidValue;
    if (up && (k != 1 || gate)) return hipErrorInvalidValue;
    if (k == 3 && cin == 8 && cout == 32 && ldx % 8 == 0 && !head) {
        a.pool = pool;
        const int tx = (wd + TLW - 1) / TLW, ty = (h + TLH - 1) / TLH;
        hipLaunchKernelGGL((k_conv3_lds<2, true>), dim3(tx * ty, n, 1), dim3(WG), 0, s, a, tx);
        return hipGetLastError();
    }
    if (head && (k != 3 || cin % 32 || cout != HC || gate || pool || up || !head->img)) return hipErrorInvalidValue;
    bool wide = cout % 64 == 0;
    if (k == 3 && cin % 32 == 0) {
        a.pool = pool;
        const int tx = (wd + TLW - 1) / TLW, ty = (h + TLH - 1) / TLH;
        // 64 output channels per block unless that leaves fewer than two blocks per CU
        if (wide && (long long)tx * ty * n * (cout / 64) < 2LL * n_cu()) wide = false;
        dim3 grid(tx * ty, n, cout / (wide ? 64 : 32));
        if (wide) hipLaunchKernelGGL((k_conv3_lds<4>), grid, dim3(WG), 0, s, a, tx);
        else hipLaunchKernelGGL((k_conv3_lds<2>), grid, dim3(WG), 0, s, a, tx);
        return hipGetLastError();
    }
    // four row tiles per wave unless that leaves fewer than two blocks per CU
    const bool thin = (long long)nblocks(a.P, 256) * (cout / (wide ? 64 : 32)) < 2LL * n_cu();
    dim3 grid(nblocks(a.P, thin ? 64 : 256), cout / (wide ? 64 : 32));
    if (k == 3) {
        if (wide) {
            if (thin) hipLaunchKernelGGL((k_conv<3, 4, 1>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<3, 4, 4>), grid, dim3(WG), 0, s, a);
        } else {
            if (thin) hipLaunchKernelGGL((k_conv<3, 2, 1>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<3, 2, 4>), grid, dim3(WG), 0, s, a);
        }
    } else if (up) {
        if (wide) {
            if (thin) hipLaunchKernelGGL((k_conv<1, 4, 1, true>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<1, 4, 4, true>), grid, dim3(WG), 0, s, a);
        } else {
            if (thin) hipLaunchKernelGGL((k_conv<1, 2, 1, true>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<1, 2, 4, true>), grid, dim3(WG), 0, s, a);
        }
    } else {
        if (wide) {
            if (thin) hipLaunchKernelGGL((k_conv<1, 4, 1>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<1, 4, 4>), grid, dim3(WG), 0, s, a);
        } else {
            if (thin) hipLaunchKernelGGL((k_conv<1, 2, 1>), grid, dim3(WG), 0, s, a);
            else hipLaunchKernelGGL((k_conv<1, 2, 4>), grid, dim3(WG), 0, s, a);
        }
    }
    if (pool) {
        const long long items = (long long)n * (h / 2) * (wd / 2) * (cout / 8);
        hipLaunchKernelGGL(k_pool, dim3(nblocks(items)), dim3(WG), 0, s, (const uint16_t *)y, ldy, pool, ldp, cout, n, h,
                           wd);
    }
    return hipGetLastError();
}

struct WgPlan {
    int wm, tm, tn, cols, cols_pad, chunk_px, nchunk;
    int ngroup;      // groups of RG chunks in the first reduction stage
    size_t row;      // floats per chunk row (dw then db)
    size_t floats;   // chunk rows and group rows
};

static WgPlan wgrad_plan(long long P, int k, int cin, int cout)
{
    WgPlan q;
    q.wm = cout % 64 == 0 ? 2 : 1;
    q.tm = 32 * q.wm;
    q.tn = 32 * (4 / q.wm);
    q.cols = k * k * cin;
    q.cols_pad = (q.cols + q.tn - 1) / q.tn * q.tn;
    const long long tiles = (long long)(cout / q.tm) * (q.cols_pad / q.tn);
    long long c = (P * tiles + 2047) / 2048;           // about 2048 blocks in all
    c = std::max<long long>(256, (c + KP - 1) / KP * KP);
    q.chunk_px = (int)std::min<long long>(c, 1 << 20);
    q.nchunk = (int)std::max<long long>(1, (P + q.chunk_px - 1) / q.chunk_px);
    q.row = (size_t)cout * q.cols_pad + cout;
    q.ngroup = (q.nchunk + RG - 1) / RG;
    q.floats = q.row * (size_t)(q.nchunk + q.ngroup);
    return q;
}

static hipError_t launch_wgrad(const uint16_t *x, int ldx, int cin, const uint16_t *g, int ldg, int cout, int n, int h,
                               int wd, int k, float *dw, float *db, float *scratch, hipStream_t s)
{
    const long long P = (long long)n * h * wd;
    const WgPlan q = wgrad_plan(P, k, cin, cout);
    WgArgs a;
    a.x = x; a.g = g; a.part = scratch; a.with_db = db != nullptr;
    a.P = P; a.ldx = ldx; a.ldg = ldg; a.cin = cin; a.cout = cout; a.h = h; a.wd = wd;
    a.cg_shift = ilog2(cin / 8); a.kg_total = k * k * cin / 8;
    a.cols = q.cols; a.cols_pad = q.cols_pad; a.chunk_px = q.chunk_px;
    dim3 grid(cout / q.tm, q.cols_pad / q.tn, q.nchunk);
    if (k == 3) {
        if (q.wm == 2) hipLaunchKernelGGL((k_wgrad<3, 2>), grid, dim3(WG), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad<3, 1>), grid, dim3(WG), 0, s, a);
    } else {
        if (q.wm == 2) hipLaunchKernelGGL((k_wgrad<1, 2>), grid, dim3(WG), 0, s, a);
        else hipLaunchKernelGGL((k_wgrad<1, 1>), grid, dim3(WG), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    float *stage = scratch + q.row * (size_t)q.nchunk;
    const long long R = (long long)q.row;
    hipLaunchKernelGGL(k_wgrad_sum1, dim3(nblocks(R), q.ngroup), dim3(WG), 0, s, (const float *)scratch, R, q.nchunk,
                       stage);
    hipLaunchKernelGGL(k_wgrad_sum2, dim3(nblocks(R)), dim3(WG), 0, s, (const float *)stage, R, q.ngroup, cout, q.cols,
                       q.cols_pad, dw, db);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// the network runner
// ---------------------------------------------------------------------------------------
constexpr int LEVELS = 4, BASE = 32, NL = 18;

struct Layer {
    char name[8];
    int k, cin, cout;
    size_t ow, ob;   // offsets in the flat parameter vector (floats)
};

struct Buf {
    size_t off = 0, bytes = 0;
};

}  // namespace dn

using namespace dn;

struct epidmc_unet {
    int device = 0;
    std::string err;
    Layer L[NL];
    size_t nparam = 0;
    // bound shape and workspace
    bool bound = false;
    int n = 0, h = 0, w = 0;
    char *ws = nullptr;
    bool have_params = false;
    int t = 0;   // Adam steps taken
    float ema_decay = 0.0f;   // 0: no moving average of the weights
    struct {
        Buf X, x0, tgt, scale, sumpart, headpart, wgs;
        Buf theta, m, v, grad, wf, wb, ema;
        Buf ea[LEVELS], cat[LEVELS - 1], eb3, pl[LEVELS - 1], da[LEVELS - 1], db[LEVELS - 1];
        Buf gdb[LEVELS - 1], gda[LEVELS - 1], gcat[LEVELS - 1], gul[LEVELS - 1], geb[LEVELS], gea[LEVELS],
            gp[LEVELS - 1];
        size_t total = 0;
    } lay;
    int sum_nb = 0;
    long long head_blocks = 0;
};

namespace dn {

static epidmc_status fail(const epidmc_unet *u, epidmc_status code, const std::string &msg)
{
    if (u) const_cast<epidmc_unet *>(u)->err = msg;
    return code;
}

#define UREQ(cond, code, msg) \
    do { if (!(cond)) return fail(u, code, msg); } while (0)
#define UCHK(x)                                                                                         \
    do {                                                                                                \
        hipError_t e_ = (x);                                                                            \
        if (e_ != hipSuccess) return fail(u, EPIDMC_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static int chan(int l) { return BASE << l; }

static void make_layers(epidmc_unet *u)
{
    int i = 0;
    auto add = [&](const char *nm, int k, int ci, int co) {
        Layer &x = u->L[i++];
        std::snprintf(x.name, sizeof x.name, "%s", nm);
        x.k = k; x.cin = ci; x.cout = co;
    };
    char nm[8];
    int prev = 8;
    for (int l = 0; l < LEVELS; ++l) {
        std::snprintf(nm, 8, "e%da", l); add(nm, 3, prev, chan(l));
        std::snprintf(nm, 8, "e%db", l); add(nm, 3, chan(l), chan(l));
        prev = chan(l);
    }
    for (int l = LEVELS - 2; l >= 0; --l) {
        std::snprintf(nm, 8, "u%d", l); add(nm, 1, chan(l + 1), chan(l));
        std::snprintf(nm, 8, "d%da", l); add(nm, 3, 2 * chan(l), chan(l));
        std::snprintf(nm, 8, "d%db", l); add(nm, 3, chan(l), chan(l));
    }
    add("head", 1, chan(0), 1);
    size_t off = 0;
    for (int j = 0; j < NL; ++j) {   // 64-float alignment keeps every BF16 row 16-byte aligned
        Layer &x = u->L[j];
        x.ow = off;
        off += ((size_t)x.cout * x.k * x.k * x.cin + 63) / 64 * 64;
        x.ob = off;
        off += ((size_t)x.cout + 63) / 64 * 64;
    }
    u->nparam = off;
}

static int find(const epidmc_unet *u, const char *nm)
{
    for (int j = 0; j < NL; ++j)
        if (!std::strcmp(u->L[j].name, nm)) return j;
    return -1;
}

static size_t plan(epidmc_unet *u, int n, int h, int w)
{
    auto &y = u->lay;
    size_t off = 0;
    auto take = [&](Buf &b, size_t bytes) { b.off = off; b.bytes = bytes; off += (bytes + 255) / 256 * 256; };
    auto P = [&](int l) { return (size_t)n * (size_t)(h >> l) * (size_t)(w >> l); };
    take(y.X, P(0) * 8 * 2);
    take(y.x0, P(0) * 4);
    take(y.tgt, P(0) * 4);
    take(y.scale, (size_t)n * 8);
    u->sum_nb = 512;
    take(y.sumpart, (size_t)n * u->sum_nb * 8);
    u->head_blocks = (long long)((P(0) + WG - 1) / WG);
    take(y.headpart, (size_t)u->head_blocks * (HC + 2) * 4);
    size_t wg = 0;
    for (int j = 0; j < NL - 1; ++j) {
        const Layer &x = u->L[j];
        int lev = 0;
        if (x.name[0] == 'e' || x.name[0] == 'd') lev = x.name[1] - '0';
        else lev = x.name[1] - '0' + 1;   // u{l} runs at level l+1
        wg = std::max(wg, wgrad_plan((long long)P(lev), x.k, x.cin, x.cout).floats);
    }
    take(y.wgs, wg * 4);
    const size_t np = u->nparam;
    take(y.theta, np * 4); take(y.m, np * 4); take(y.v, np * 4); take(y.grad, np * 4); take(y.ema, np * 4);
    take(y.wf, np * 2); take(y.wb, np * 2);
    for (int l = 0; l < LEVELS; ++l) {
        take(y.ea[l], P(l) * chan(l) * 2);
        take(y.gea[l], P(l) * chan(l) * 2);
        take(y.geb[l], P(l) * chan(l) * 2);
    }
    take(y.eb3, P(LEVELS - 1) * chan(LEVELS - 1) * 2);
    for (int l = 0; l < LEVELS - 1; ++l) {
        take(y.cat[l], P(l) * 2 * chan(l) * 2);
        take(y.gcat[l], P(l) * 2 * chan(l) * 2);
        take(y.pl[l], P(l + 1) * chan(l) * 2);
        take(y.gp[l], P(l + 1) * chan(l) * 2);
        take(y.gul[l], P(l + 1) * chan(l) * 2);
        take(y.da[l], P(l) * chan(l) * 2);
        take(y.gda[l], P(l) * chan(l) * 2);
        take(y.db[l], P(l) * chan(l) * 2);
        take(y.gdb[l], P(l) * chan(l) * 2);
    }
    y.total = off;
    return off;
}

template <class T> static T *at(epidmc_unet *u, const Buf &b) { return (T *)(u->ws + b.off); }

// the BF16 forward and transposed weights of every convolution (all but the head), one launch
static hipError_t weights_all(epidmc_unet *u, hipStream_t s)
{
    static_assert(NL - 1 <= WT_MAX, "weight table too small");
    WeightTable t;
    t.n = NL - 1;
    long long blocks = 0;
    for (int j = 0; j < NL - 1; ++j) {
        const Layer &x = u->L[j];
        t.first_block[j] = (int)blocks;
        t.off[j] = x.ow;
        t.cout[j] = x.cout; t.kk[j] = x.k * x.k; t.cin[j] = x.cin;
        blocks += nblocks((long long)x.cout * x.k * x.k * x.cin);
    }
    t.first_block[NL - 1] = (int)blocks;
    hipLaunchKernelGGL(k_weights_all, dim3((unsigned)blocks), dim3(WG), 0, s, (const float *)at<float>(u, u->lay.theta),
                       at<uint16_t>(u, u->lay.wf), at<uint16_t>(u, u->lay.wb), t);
    return hipGetLastError();
}

// normalise the batch: scale, 8-channel BF16 input, FP32 image channel and target
static hipError_t prepare(epidmc_unet *u, const double *noisy, const double *thick, const double *target, int n,
                          hipStream_t s)
{
    auto &y = u->lay;
    const long long hw = (long long)u->h * u->w, P = hw * n;
    (void)P;
    hipLaunchKernelGGL(k_img_sum, dim3(u->sum_nb, n), dim3(WG), 0, s, noisy, hw, u->sum_nb, at<double>(u, y.sumpart));
    hipLaunchKernelGGL(k_prepare, dim3(nblocks(hw), n), dim3(WG), 0, s, noisy, thick, target,
                       (const double *)at<double>(u, y.sumpart), u->sum_nb, hw, at<uint16_t>(u, y.X),
                       at<float>(u, y.x0), at<float>(u, y.tgt), at<double>(u, y.scale));
    return hipGetLastError();
}

// the network's activations for the prepared batch; with `img` (inference), the last
// convolution applies the head in its epilogue and writes the denoised image there instead
// of storing its own output
static hipError_t forward(epidmc_unet *u, int n, hipStream_t s, double *img = nullptr)
{
    auto &y = u->lay;
    const uint16_t *wf = at<uint16_t>(u, y.wf);
    const float *th = at<float>(u, y.theta);
    hipError_t e;
    for (int l = 0; l < LEVELS; ++l) {
        const int c = chan(l), hl = u->h >> l, wl = u->w >> l;
        const Layer &A = u->L[2 * l], &B = u->L[2 * l + 1];
        const uint16_t *in = l == 0 ? at<uint16_t>(u, y.X) : at<uint16_t>(u, y.pl[l - 1]);
        const int ldin = l == 0 ? 8 : chan(l - 1);
        if ((e = launch_conv(in, ldin, A.cin, wf + A.ow, th + A.ob, at<uint16_t>(u, y.ea[l]), c, c, nullptr, 0, n, hl,
                             wl, 3, 1, s)) != hipSuccess) return e;
        uint16_t *out = l < LEVELS - 1 ? at<uint16_t>(u, y.cat[l]) : at<uint16_t>(u, y.eb3);
        const int ldo = l < LEVELS - 1 ? 2 * c : c;
        if ((e = launch_conv(at<uint16_t>(u, y.ea[l]), c, c, wf + B.ow, th + B.ob, out, ldo, c, nullptr, 0, n, hl, wl,
                             3, 1, s, l < LEVELS - 1 ? at<uint16_t>(u, y.pl[l]) : nullptr, c)) != hipSuccess)
            return e;
    }
    for (int l = LEVELS - 2; l >= 0; --l) {
        const int c = chan(l), hl = u->h >> l, wl = u->w >> l;
        const Layer &U = u->L[find(u, (std::string("u") + char('0' + l)).c_str())];
        const Layer &A = u->L[find(u, (std::string("d") + char('0' + l) + "a").c_str())];
        const Layer &B = u->L[find(u, (std::string("d") + char('0' + l) + "b").c_str())];
        const uint16_t *in = l == LEVELS - 2 ? at<uint16_t>(u, y.eb3) : at<uint16_t>(u, y.db[l + 1]);
        // the 1 x 1 up-convolution writes its 2x upsampled output straight into the second half
        // of the concatenation
        if ((e = launch_conv(in, chan(l + 1), chan(l + 1), wf + U.ow, th + U.ob, at<uint16_t>(u, y.cat[l]) + c, 2 * c,
                             c, nullptr, 0, n, hl / 2, wl / 2, 1, 0, s, nullptr, 0, 1)) != hipSuccess) return e;
        if ((e = launch_conv(at<uint16_t>(u, y.cat[l]), 2 * c, 2 * c, wf + A.ow, th + A.ob, at<uint16_t>(u, y.da[l]),
                             c, c, nullptr, 0, n, hl, wl, 3, 1, s)) != hipSuccess) return e;
        const Layer &H = u->L[NL - 1];
        const Head head{th + H.ow, th + H.ob, at<float>(u, y.x0), at<double>(u, y.scale), img};
        if ((e = launch_conv(at<uint16_t>(u, y.da[l]), c, c, wf + B.ow, th + B.ob, at<uint16_t>(u, y.db[l]), c, c,
                             nullptr, 0, n, hl, wl, 3, 1, s, nullptr, 0, 0, l == 0 && img ? &head : nullptr)) !=
            hipSuccess) return e;
    }
    return hipGetLastError();
}

// the gradient of the loss (after forward) into y.grad, and the loss into `loss`
static hipError_t backward(epidmc_unet *u, int n, double *loss, hipStream_t s)
{
    auto &y = u->lay;
    const uint16_t *wb = at<uint16_t>(u, y.wb);
    float *gr = at<float>(u, y.grad), *wgs = at<float>(u, y.wgs);
    const long long hw = (long long)u->h * u->w, P = hw * n;
    const Layer &H = u->L[NL - 1];
    const long long hb = nblocks(P);
    hipLaunchKernelGGL(k_head, dim3(hb), dim3(WG), 0, s, (const uint16_t *)at<uint16_t>(u, y.db[0]),
                       (const float *)(at<float>(u, y.theta) + H.ow), (const float *)(at<float>(u, y.theta) + H.ob),
                       (const float *)at<float>(u, y.x0), (const float *)at<float>(u, y.tgt), P,
                       at<uint16_t>(u, y.gdb[0]), at<float>(u, y.headpart));
    hipLaunchKernelGGL(k_head_reduce, dim3(HC + 2), dim3(WG), 0, s, (const float *)at<float>(u, y.headpart), (int)hb, P,
                       gr + H.ow, gr + H.ob, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = 0; l < LEVELS - 1; ++l) {
        const int c = chan(l), hl = u->h >> l, wl = u->w >> l;
        const Layer &U = u->L[find(u, (std::string("u") + char('0' + l)).c_str())];
        const Layer &A = u->L[find(u, (std::string("d") + char('0' + l) + "a").c_str())];
        const Layer &B = u->L[find(u, (std::string("d") + char('0' + l) + "b").c_str())];
        // d{l}b
        if ((e = launch_wgrad(at<uint16_t>(u, y.da[l]), c, c, at<uint16_t>(u, y.gdb[l]), c, c, n, hl, wl, 3,
                              gr + B.ow, gr + B.ob, wgs, s)) != hipSuccess) return e;
        if ((e = launch_conv(at<uint16_t>(u, y.gdb[l]), c, c, wb + B.ow, nullptr, at<uint16_t>(u, y.gda[l]), c, c,
                             at<uint16_t>(u, y.da[l]), c, n, hl, wl, 3, 0, s)) != hipSuccess) return e;
        // d{l}a: input is the concatenation [skip, upsampled]
        if ((e = launch_wgrad(at<uint16_t>(u, y.cat[l]), 2 * c, 2 * c, at<uint16_t>(u, y.gda[l]), c, c, n, hl, wl, 3,
                              gr + A.ow, gr + A.ob, wgs, s)) != hipSuccess) return e;
        if ((e = launch_conv(at<uint16_t>(u, y.gda[l]), c, c, wb + A.ow, nullptr, at<uint16_t>(u, y.gcat[l]), 2 * c,
                             2 * c, nullptr, 0, n, hl, wl, 3, 0, s)) != hipSuccess) return e;
        // the upsampled half back to the 1x1 up-convolution's output
        const long long items = (long long)n * (hl / 2) * (wl / 2) * (c / 8);
        hipLaunchKernelGGL(k_upsample_bwd, dim3(nblocks(items)), dim3(WG), 0, s,
                           (const uint16_t *)(at<uint16_t>(u, y.gcat[l]) + c), 2 * c, at<uint16_t>(u, y.gul[l]), c, c,
                           n, hl, wl);
        const uint16_t *in = l == LEVELS - 2 ? at<uint16_t>(u, y.eb3) : at<uint16_t>(u, y.db[l + 1]);
        uint16_t *gin = l == LEVELS - 2 ? at<uint16_t>(u, y.geb[LEVELS - 1]) : at<uint16_t>(u, y.gdb[l + 1]);
        const int c1 = chan(l + 1);
        if ((e = launch_wgrad(in, c1, c1, at<uint16_t>(u, y.gul[l]), c, c, n, hl / 2, wl / 2, 1, gr + U.ow, gr + U.ob,
                              wgs, s)) != hipSuccess) return e;
        if ((e = launch_conv(at<uint16_t>(u, y.gul[l]), c, c, wb + U.ow, nullptr, gin, c1, c1, in, c1, n, hl / 2,
                             wl / 2, 1, 0, s)) != hipSuccess) return e;
    }
    for (int l = LEVELS - 1; l >= 0; --l) {
        const int c = chan(l), hl = u->h >> l, wl = u->w >> l;
        const Layer &A = u->L[2 * l], &B = u->L[2 * l + 1];
        const uint16_t *act_b = l < LEVELS - 1 ? at<uint16_t>(u, y.cat[l]) : at<uint16_t>(u, y.eb3);
        const int ldb = l < LEVELS - 1 ? 2 * c : c;
        if (l < LEVELS - 1) {
            const long long items = (long long)n * hl * wl * (c / 8);
            hipLaunchKernelGGL(k_skip_bwd, dim3(nblocks(items)), dim3(WG), 0, s,
                               (const uint16_t *)at<uint16_t>(u, y.gcat[l]), 2 * c,
                               (const uint16_t *)at<uint16_t>(u, y.gp[l]), c, act_b, ldb, at<uint16_t>(u, y.geb[l]), c,
                               c, n, hl, wl);
        }
        if ((e = launch_wgrad(at<uint16_t>(u, y.ea[l]), c, c, at<uint16_t>(u, y.geb[l]), c, c, n, hl, wl, 3,
                              gr + B.ow, gr + B.ob, wgs, s)) != hipSuccess) return e;
        if ((e = launch_conv(at<uint16_t>(u, y.geb[l]), c, c, wb + B.ow, nullptr, at<uint16_t>(u, y.gea[l]), c, c,
                             at<uint16_t>(u, y.ea[l]), c, n, hl, wl, 3, 0, s)) != hipSuccess) return e;
        const uint16_t *in = l == 0 ? at<uint16_t>(u, y.X) : at<uint16_t>(u, y.pl[l - 1]);
        const int ldin = l == 0 ? 8 : chan(l - 1);
        if ((e = launch_wgrad(in, ldin, A.cin, at<uint16_t>(u, y.gea[l]), c, c, n, hl, wl, 3, gr + A.ow, gr + A.ob, wgs,
                              s)) != hipSuccess) return e;
        if (l > 0 && (e = launch_conv(at<uint16_t>(u, y.gea[l]), c, c, wb + A.ow, nullptr, at<uint16_t>(u, y.gp[l - 1]),
                                      chan(l - 1), chan(l - 1), nullptr, 0, n, hl, wl, 3, 0, s)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

static epidmc_status check_batch(epidmc_unet *u, int n)
{
    UREQ(u->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    UREQ(u->have_params, EPIDMC_E_NOT_READY, "parameters not set");
    UREQ(n >= 1 && n <= u->n, EPIDMC_E_SHAPE, "batch larger than the bound batch");
    return EPIDMC_OK;
}

static epidmc_status conv_shape_ok(int ldx, int cin, int ldy, int cout, int n, int h, int w, int k)
{
    if (!(k == 1 || k == 3) || n < 0 || h < 0 || w < 0) return EPIDMC_E_ARG;
    if (cin < 8 || cin % 8 || !pow2(cin / 8) || cout < 32 || cout % 32 || ldx < cin || ldx % 8 || ldy < cout ||
        ldy % 8)
        return EPIDMC_E_SHAPE;
    return EPIDMC_OK;
}

}  // namespace dn

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
extern "C" {

epidmc_status epidmc_dn_conv(const uint16_t *x, int ldx, int c_in, const uint16_t *w, const float *bias, uint16_t *y,
                             int ldy, int c_out, const uint16_t *gate, int ldg, int n, int h, int w_px, int k, int relu,
                             void *stream)
{
    epidmc_status st = conv_shape_ok(ldx, c_in, ldy, c_out, n, h, w_px, k);
    if (st != EPIDMC_OK) return st;
    if (!x || !w || !y || (gate && (ldg < c_out || ldg % 8))) return EPIDMC_E_ARG;
    return launch_conv(x, ldx, c_in, w, bias, y, ldy, c_out, gate, ldg, n, h, w_px, k, relu, (hipStream_t)stream) ==
                   hipSuccess
               ? EPIDMC_OK
               : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_dn_wgrad_scratch(int n, int h, int w_px, int k, int c_in, int c_out, size_t *floats)
{
    epidmc_status st = conv_shape_ok(c_in, c_in, c_out, c_out, n, h, w_px, k);
    if (st != EPIDMC_OK || !floats) return st != EPIDMC_OK ? st : EPIDMC_E_ARG;
    *floats = wgrad_plan((long long)n * h * w_px, k, c_in, c_out).floats;
    return EPIDMC_OK;
}

epidmc_status epidmc_dn_wgrad(const uint16_t *x, int ldx, int c_in, const uint16_t *g, int ldg, int c_out, int n,
                              int h, int w_px, int k, float *dw, float *db, float *scratch, size_t scratch_floats,
                              void *stream)
{
    epidmc_status st = conv_shape_ok(ldx, c_in, ldg, c_out, n, h, w_px, k);
    if (st != EPIDMC_OK) return st;
    if (!x || !g || !dw || !scratch || (long long)n * h * w_px == 0) return EPIDMC_E_ARG;
    if (scratch_floats < wgrad_plan((long long)n * h * w_px, k, c_in, c_out).floats) return EPIDMC_E_WORKSPACE;
    return launch_wgrad(x, ldx, c_in, g, ldg, c_out, n, h, w_px, k, dw, db, scratch, (hipStream_t)stream) == hipSuccess
               ? EPIDMC_OK
               : EPIDMC_E_DEVICE;
}

// Scratch of the allocation-free weight gradient: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, once per device, with
// that device current.
static __device__ __align__(256) float scratch[EPIDMC_DN_WGRAD_NOALLOC_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static epidmc_status noalloc_scratch(float **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return EPIDMC_E_DEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EPIDMC_E_DEVICE;
        scratch_ptr[dev] = (float *)p;
    }
    *out = scratch_ptr[dev];
    return EPIDMC_OK;
}

epidmc_status epidmc_dn_wgrad_noalloc(const uint16_t *x, int ldx, int c_in, const uint16_t *g, int ldg, int c_out,
                                      int n, int h, int w_px, int k, float *dw, float *db, void *stream)
{
    epidmc_status st = conv_shape_ok(ldx, c_in, ldg, c_out, n, h, w_px, k);
    if (st != EPIDMC_OK) return st;
    if (!x || !g || !dw || (long long)n * h * w_px == 0) return EPIDMC_E_ARG;
    if (wgrad_plan((long long)n * h * w_px, k, c_in, c_out).floats > (size_t)EPIDMC_DN_WGRAD_NOALLOC_FLOATS)
        return EPIDMC_E_WORKSPACE;
    float *ws = nullptr;
    st = noalloc_scratch(&ws);
    if (st != EPIDMC_OK) return st;
    return launch_wgrad(x, ldx, c_in, g, ldg, c_out, n, h, w_px, k, dw, db, ws, (hipStream_t)stream) == hipSuccess
               ? EPIDMC_OK
               : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_dn_weights(const float *w, int c_out, int k, int c_in, uint16_t *w_fwd, uint16_t *w_bwd,
                                void *stream)
{
    if (!w || c_out < 1 || c_in < 1 || !(k == 1 || k == 3)) return EPIDMC_E_ARG;
    const long long cnt = (long long)c_out * k * k * c_in;
    hipLaunchKernelGGL(k_weights, dim3(nblocks(cnt)), dim3(WG), 0, (hipStream_t)stream, w, c_out, k * k, c_in, w_fwd,
                       w_bwd);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}

static epidmc_status ew_ok(const void *a, const void *b, int lda, int ldb, int c, int n, int h, int w, bool even)
{
    if (!a || !b || c < 8 || c % 8 || lda < c || ldb < c || lda % 8 || ldb % 8 || n < 0 || h < 0 || w < 0)
        return EPIDMC_E_ARG;
    if (even && (h % 2 || w % 2)) return EPIDMC_E_SHAPE;
    return EPIDMC_OK;
}

epidmc_status epidmc_dn_pool(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int w_px,
                             void *stream)
{
    epidmc_status st = ew_ok(x, y, ldx, ldy, c, n, h, w_px, true);
    if (st != EPIDMC_OK) return st;
    const long long items = (long long)n * (h / 2) * (w_px / 2) * (c / 8);
    if (items == 0) return EPIDMC_OK;
    hipLaunchKernelGGL(k_pool, dim3(nblocks(items)), dim3(WG), 0, (hipStream_t)stream, x, ldx, y, ldy, c, n, h, w_px);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_dn_upsample(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int w_px,
                                 void *stream)
{
    epidmc_status st = ew_ok(x, y, ldx, ldy, c, n, h, w_px, false);
    if (st != EPIDMC_OK) return st;
    const long long items = (long long)n * h * w_px * (c / 8);
    if (items == 0) return EPIDMC_OK;
    hipLaunchKernelGGL(k_upsample, dim3(nblocks(items)), dim3(WG), 0, (hipStream_t)stream, x, ldx, y, ldy, c, n, h,
                       w_px);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_dn_upsample_backward(const uint16_t *g, int ldg, uint16_t *y, int ldy, int c, int n, int h,
                                          int w_px, void *stream)
{
    epidmc_status st = ew_ok(g, y, ldg, ldy, c, n, h, w_px, true);
    if (st != EPIDMC_OK) return st;
    const long long items = (long long)n * (h / 2) * (w_px / 2) * (c / 8);
    if (items == 0) return EPIDMC_OK;
    hipLaunchKernelGGL(k_upsample_bwd, dim3(nblocks(items)), dim3(WG), 0, (hipStream_t)stream, g, ldg, y, ldy, c, n,
                       h, w_px);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_dn_skip_backward(const uint16_t *g_skip, int lds, const uint16_t *g_pool, int ldp,
                                      const uint16_t *act, int lda, uint16_t *out, int ldo, int c, int n, int h,
                                      int w_px, void *stream)
{
    epidmc_status st = ew_ok(g_skip, out, lds, ldo, c, n, h, w_px, true);
    if (st != EPIDMC_OK) return st;
    st = ew_ok(g_pool, act, ldp, lda, c, n, h, w_px, true);
    if (st != EPIDMC_OK) return st;
    const long long items = (long long)n * h * w_px * (c / 8);
    if (items == 0) return EPIDMC_OK;
    hipLaunchKernelGGL(k_skip_bwd, dim3(nblocks(items)), dim3(WG), 0, (hipStream_t)stream, g_skip, lds, g_pool, ldp,
                       act, lda, out, ldo, c, n, h, w_px);
    return hipGetLastError() == hipSuccess ? EPIDMC_OK : EPIDMC_E_DEVICE;
}

epidmc_status epidmc_unet_create(epidmc_unet **out, int device)
{
    if (!out) return EPIDMC_E_ARG;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return EPIDMC_E_DEVICE;
    epidmc_unet *u = new epidmc_unet();
    u->device = device;
    make_layers(u);
    *out = u;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_destroy(epidmc_unet *u)
{
    delete u;
    return EPIDMC_OK;
}

const char *epidmc_unet_last_error(const epidmc_unet *u) { return u ? u->err.c_str() : "null context"; }

int epidmc_unet_layers(const epidmc_unet *u) { return u ? NL : 0; }

epidmc_status epidmc_unet_param_count(const epidmc_unet *u, size_t *floats)
{
    if (!u || !floats) return EPIDMC_E_ARG;
    *floats = u->nparam;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_layer(const epidmc_unet *u, int layer, char name[8], int *k, int *c_in, int *c_out,
                                size_t *off_w, size_t *off_b)
{
    if (!u || layer < 0 || layer >= NL) return EPIDMC_E_ARG;
    const Layer &x = u->L[layer];
    if (name) std::memcpy(name, x.name, 8);
    if (k) *k = x.k;
    if (c_in) *c_in = x.cin;
    if (c_out) *c_out = x.cout;
    if (off_w) *off_w = x.ow;
    if (off_b) *off_b = x.ob;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_workspace_size(const epidmc_unet *u, int n, int h, int w_px, size_t *bytes)
{
    if (!u || !bytes) return EPIDMC_E_ARG;
    if (n < 1 || h < 8 || w_px < 8 || h % 8 || w_px % 8) return fail(u, EPIDMC_E_SHAPE, "n >= 1, h and w multiples of 8");
    epidmc_unet tmp = *u;
    *bytes = plan(&tmp, n, h, w_px);
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_bind(epidmc_unet *u, void *dev_ptr, size_t bytes, int n, int h, int w_px, void *stream)
{
    if (!u) return EPIDMC_E_ARG;
    UREQ(dev_ptr && ((uintptr_t)dev_ptr % 256) == 0, EPIDMC_E_ARG, "workspace must be 256-byte aligned");
    UREQ(n >= 1 && h >= 8 && w_px >= 8 && h % 8 == 0 && w_px % 8 == 0, EPIDMC_E_SHAPE,
         "n >= 1, h and w multiples of 8");
    const size_t need = plan(u, n, h, w_px);
    UREQ(bytes >= need, EPIDMC_E_WORKSPACE, "workspace too small");
    UCHK(hipSetDevice(u->device));
    u->ws = (char *)dev_ptr;
    u->n = n; u->h = h; u->w = w_px;
    hipStream_t s = (hipStream_t)stream;
    const long long np = (long long)u->nparam;
    for (const Buf *b : {&u->lay.theta, &u->lay.m, &u->lay.v, &u->lay.grad})
        hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(np)), dim3(WG), 0, s, (float *)(u->ws + b->off), np, 0.0f);
    UCHK(hipGetLastError());
    UCHK(weights_all(u, s));
    u->bound = true;
    u->have_params = false;
    u->t = 0;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_set_params(epidmc_unet *u, const float *dev_params, void *stream)
{
    if (!u) return EPIDMC_E_ARG;
    UREQ(u->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    UREQ(dev_params, EPIDMC_E_ARG, "null parameters");
    hipStream_t s = (hipStream_t)stream;
    const long long np = (long long)u->nparam;
    hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(np)), dim3(WG), 0, s, dev_params, at<float>(u, u->lay.theta), np);
    hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(np)), dim3(WG), 0, s, dev_params, at<float>(u, u->lay.ema), np);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(np)), dim3(WG), 0, s, at<float>(u, u->lay.m), np, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(np)), dim3(WG), 0, s, at<float>(u, u->lay.v), np, 0.0f);
    UCHK(hipGetLastError());
    UCHK(weights_all(u, s));
    u->have_params = true;
    u->t = 0;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_get_params(const epidmc_unet *u, float *dev_params, void *stream)
{
    if (!u || !dev_params) return EPIDMC_E_ARG;
    UREQ(u->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    const long long np = (long long)u->nparam;
    hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(np)), dim3(WG), 0, (hipStream_t)stream,
                       (const float *)(u->ws + u->lay.theta.off), dev_params, np);
    UCHK(hipGetLastError());
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_set_ema(epidmc_unet *u, float decay)
{
    if (!u) return EPIDMC_E_ARG;
    UREQ(std::isfinite(decay) && decay >= 0.0f && decay < 1.0f, EPIDMC_E_ARG, "decay must be in [0, 1)");
    u->ema_decay = decay;
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_get_ema_params(const epidmc_unet *u, float *dev_params, void *stream)
{
    if (!u || !dev_params) return EPIDMC_E_ARG;
    UREQ(u->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    const long long np = (long long)u->nparam;
    hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(np)), dim3(WG), 0, (hipStream_t)stream,
                       (const float *)(u->ws + u->lay.ema.off), dev_params, np);
    UCHK(hipGetLastError());
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_forward(epidmc_unet *u, const double *noisy, const double *thickness, double *out, int n,
                                  void *stream)
{
    if (!u) return EPIDMC_E_ARG;
    epidmc_status st = check_batch(u, n);
    if (st != EPIDMC_OK) return st;
    UREQ(noisy && thickness && out, EPIDMC_E_ARG, "null image");
    UCHK(hipSetDevice(u->device));
    hipStream_t s = (hipStream_t)stream;
    UCHK(prepare(u, noisy, thickness, nullptr, n, s));
    UCHK(forward(u, n, s, out));
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_gradient(epidmc_unet *u, const double *noisy, const double *thickness, const double *target,
                                   int n, float *dev_grad, double *loss, void *stream)
{
    if (!u) return EPIDMC_E_ARG;
    epidmc_status st = check_batch(u, n);
    if (st != EPIDMC_OK) return st;
    UREQ(noisy && thickness && target, EPIDMC_E_ARG, "null image");
    UCHK(hipSetDevice(u->device));
    hipStream_t s = (hipStream_t)stream;
    UCHK(prepare(u, noisy, thickness, target, n, s));
    UCHK(forward(u, n, s));
    UCHK(backward(u, n, loss, s));
    if (dev_grad) {
        const long long np = (long long)u->nparam;
        hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(np)), dim3(WG), 0, s, (const float *)at<float>(u, u->lay.grad),
                           dev_grad, np);
        UCHK(hipGetLastError());
    }
    return EPIDMC_OK;
}

epidmc_status epidmc_unet_train_step(epidmc_unet *u, const double *noisy, const double *thickness,
                                     const double *target, int n, float lr, double *loss, void *stream)
{
    if (!u) return EPIDMC_E_ARG;
    UREQ(std::isfinite(lr) && lr >= 0.0f, EPIDMC_E_ARG, "learning rate must be finite and >= 0");
    epidmc_status st = epidmc_unet_gradient(u, noisy, thickness, target, n, nullptr, loss, stream);
    if (st != EPIDMC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    u->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, u->t)), bc2 = (float)(1.0 - std::pow(b2, u->t));
    const long long np = (long long)u->nparam;
    hipLaunchKernelGGL(k_adam, dim3(nblocks(np)), dim3(WG), 0, s, at<float>(u, u->lay.theta),
                       (const float *)at<float>(u, u->lay.grad), at<float>(u, u->lay.m), at<float>(u, u->lay.v), np, lr,
                       (float)b1, (float)b2, 1e-8f, bc1, bc2,
                       u->ema_decay > 0.0f ? at<float>(u, u->lay.ema) : (float *)nullptr, u->ema_decay);
    UCHK(hipGetLastError());
    UCHK(weights_all(u, s));
    return EPIDMC_OK;
}

}  // extern "C"
