// Learned surrogate of the IMPM sensor: U-shaped 3x3 convolutional network,
// BF16 activations and weights on the gfx950 matrix cores (v_mfma_f32_16x16x32
// _bf16, FP32 accumulation), FP32 master weights and Adam.  The network, its
// inputs and the parameter layout are documented in include/sur.h.
//
// Convolutions run as implicit GEMMs: rows are pixels (NHWC, so a pixel's
// channels are contiguous), columns are output channels, and the reduction
// runs over the 9 taps times the input channels in chunks of 32.  Each lane
// feeds the MFMA with 16-byte loads taken straight from the tensors (8
// consecutive channels of one gathered pixel, or 8 consecutive weights), so no
// im2col buffer exists.  The same kernel computes the data gradient with the
// transposed weights and the inverse gather.  The weight gradient reduces over
// pixels, which are strided in NHWC, so that kernel stages tiles through LDS
// transposed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sur.h"

namespace sur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// ------------------------------------------------------------------ implicit-GEMM convolution

enum { EPI_FWD = 0, EPI_DX_MASK = 1, EPI_DX_RAW = 2 };

struct ConvArgs {
    const uint16_t* src;    // gathered operand, NHWC [N][Hs][Ws][Ka]
    const uint16_t* wt;     // [Nn][9][Ka]
    int N, Hm, Wm;          // GEMM rows: N * Hm * Wm pixels
    int Hs, Ws, Ka, Nn;
    int stride, up, transpose;
    int epi;
    const float* bias;      // [Nn] (EPI_FWD)
    const uint16_t* add;    // [rows][Nn] skip (EPI_FWD) or skip gradient (EPI_DX_MASK), may be null
    const uint16_t* mask;   // [rows][Nn] activation whose > 0 passes the gradient (EPI_DX_MASK)
    uint16_t* out;          // [rows][Nn] BF16 (EPI_FWD, EPI_DX_MASK)
    float* outf;            // [rows][Nn] FP32 (EPI_DX_RAW)
};

// Source pixel of row pixel (n, y, x) for tap (ty, tx), or -1 (zero padding).
//  forward:   input position s*y + t - 1 (of the 2x upsampled source if up)
//  transpose: output position p with s*p + t - 1 = y (data gradient)
// Indices are 32-bit: sur_create keeps every tensor below 2^31 elements.
__device__ __forceinline__ int gather(const ConvArgs& a, int n, int y, int x, int ty, int tx) {
    int sy, sx;
    if (!a.transpose) {
        const int yy = y * a.stride + ty - 1, xx = x * a.stride + tx - 1;
        const int he = a.up ? 2 * a.Hs : a.Hs, we = a.up ? 2 * a.Ws : a.Ws;
        if (yy < 0 || yy >= he || xx < 0 || xx >= we) return -1;
        sy = a.up ? yy >> 1 : yy;
        sx = a.up ? xx >> 1 : xx;
    } else {
        int yy = y + 1 - ty, xx = x + 1 - tx;
        if (yy < 0 || xx < 0) return -1;
        if (a.stride == 2) {
            if ((yy | xx) & 1) return -1;
            yy >>= 1;
            xx >>= 1;
        }
        if (yy >= a.Hs || xx >= a.Ws) return -1;
        sy = yy;
        sx = xx;
    }
    return (n * a.Hs + sy) * a.Ws + sx;
}

// Block = 4 waves laid out WVM x WVN; a wave owns WMT x WNT MFMA tiles of 16 x 16.
template <int WMT, int WNT, int WVM, int WVN>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    constexpr int BM = WVM * WMT * 16, BN = WVN * WNT * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WVM, wn = wave / WVM;
    const int r = lane & 15, kq = lane >> 4;
    const int M = a.N * a.Hm * a.Wm;
    const int m0 = blockIdx.x * BM + wm * WMT * 16;
    const int n0 = blockIdx.y * BN + wn * WNT * 16;
    int pn[WMT], py[WMT], px[WMT];
    bool pv[WMT];
#pragma unroll
    for (int i = 0; i < WMT; ++i) {
        const int m = m0 + i * 16 + r;
        pv[i] = m < M;
        const unsigned mm = pv[i] ? (unsigned)m : 0u;
        const unsigned row = mm / (unsigned)a.Wm;
        px[i] = (int)(mm - row * (unsigned)a.Wm);
        pn[i] = (int)(row / (unsigned)a.Hm);
        py[i] = (int)(row - (unsigned)pn[i] * (unsigned)a.Hm);
    }
    f32x4 acc[WMT][WNT];
#pragma unroll
    for (int i = 0; i < WMT; ++i)
#pragma unroll
        for (int j = 0; j < WNT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int t = 0; t < 9; ++t) {
        const int ty = t / 3, tx = t % 3;
        const uint16_t* sp[WMT];
#pragma unroll
        for (int i = 0; i < WMT; ++i) {
            const int q = pv[i] ? gather(a, pn[i], py[i], px[i], ty, tx) : -1;
            sp[i] = q >= 0 ? a.src + q * a.Ka + kq * 8 : nullptr;
        }
        const uint16_t* wp[WNT];
#pragma unroll
        for (int j = 0; j < WNT; ++j) wp[j] = a.wt + ((size_t)(n0 + j * 16 + r) * 9 + t) * a.Ka + kq * 8;
        for (int c0 = 0; c0 < a.Ka; c0 += 32) {
            bf16x8 av[WMT], bv[WNT];
#pragma unroll
            for (int i = 0; i < WMT; ++i) av[i] = sp[i] ? load8(sp[i] + c0) : zero8();
#pragma unroll
            for (int j = 0; j < WNT; ++j) bv[j] = load8(wp[j] + c0);
#pragma unroll
            for (int i = 0; i < WMT; ++i)
#pragma unroll
                for (int j = 0; j < WNT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // D layout: lane holds rows 4*kq + e (e = 0..3) of column r of each tile
#pragma unroll
    for (int i = 0; i < WMT; ++i)
#pragma unroll
        for (int j = 0; j < WNT; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + i * 16 + kq * 4 + e;
                if (m >= M) continue;
                const int n = n0 + j * 16 + r;
                const int o = m * a.Nn + n;
                float v = acc[i][j][e];
                if (a.epi == EPI_FWD) {
                    v += a.bias[n];
                    if (a.add) v += bf2f(a.add[o]);
                    a.out[o] = f2bf(fmaxf(v, 0.f));
                } else if (a.epi == EPI_DX_MASK) {
                    if (a.add) v += bf2f(a.add[o]);
                    a.out[o] = f2bf(bf2f(a.mask[o]) > 0.f ? v : 0.f);
                } else {
                    a.outf[o] = v;
                }
            }
}

// Stride-1 convolutions without upsampling (forward, or the data gradient with
// the transposed weights), staged through LDS.  A block owns a 16 x 16 pixel
// tile of one image and 32 output columns; per 32-channel chunk it stages the
// tile's 18 x 18 input patch (zero padded) and the 9 taps x 32 channels of its
// 32 weight columns with all loads in flight at once, then runs the 9 taps
// from LDS.  Wave w owns image rows 4w..4w+3 of the tile; an MFMA row block is
// 16 consecutive pixels of one row.
//   HALF = 0: stride 1, same resolution (18 x 18 patch);
//   HALF = 1: forward convolution of the 2x upsampled source: tap positions
//             y + t - 1 read source pixel (y + t - 1) >> 1 (10 x 10 patch);
//   HALF = 2: data gradient of a stride-2 convolution: position y + 1 - t is
//             a source pixel (y + 1 - t) / 2 only when even (10 x 10 patch).
// Positions outside the source read the patch's zero border.
constexpr int LDS_TILE = 16;                       // tile side (pixels)
constexpr int LDS_PATCH = LDS_TILE + 2;            // patch side
constexpr int LDS_BPITCH = 9 * 32 + 8;             // weight column pitch (elements)

template <int HALF>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t sP[LDS_PATCH * LDS_PATCH * 32];
    __shared__ __attribute__((aligned(16))) uint16_t sW[32 * LDS_BPITCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int tiles_x = (a.Wm + LDS_TILE - 1) / LDS_TILE, tiles_y = (a.Hm + LDS_TILE - 1) / LDS_TILE;
    const int bx = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
    const int by = rest % tiles_y, n = rest / tiles_y;
    const int x0 = bx * LDS_TILE, y0 = by * LDS_TILE;
    const int n0 = blockIdx.y * 32;
    // patch origin and side in source pixels
    const int py0 = HALF ? (y0 - 1) >> 1 : y0 - 1, px0 = HALF ? (x0 - 1) >> 1 : x0 - 1;
    constexpr int SIDE = HALF ? LDS_TILE / 2 + 2 : LDS_PATCH;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    constexpr int PV = SIDE * SIDE * 4;            // 16-byte vectors of a patch chunk
    constexpr int WV = 32 * 9 * 4;                 // 16-byte vectors of a weight chunk
    constexpr int PPT = (PV + 255) / 256, WPT = (WV + 255) / 256;
    for (int c0 = 0; c0 < a.Ka; c0 += 32) {
        uint4 pv[PPT], wv[WPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int v = threadIdx.x + k * 256;
            pv[k] = make_uint4(0, 0, 0, 0);
            if (v < PV) {
                const int pix = v >> 2, ch = (v & 3) * 8;
                const int y = py0 + pix / SIDE, x = px0 + pix % SIDE;
                if (y >= 0 && y < a.Hs && x >= 0 && x < a.Ws)
                    pv[k] = *reinterpret_cast<const uint4*>(a.src + ((n * a.Hs + y) * a.Ws + x) * a.Ka + c0 + ch);
            }
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int v = threadIdx.x + k * 256;
            wv[k] = make_uint4(0, 0, 0, 0);
            if (v < WV) {
                const int col = v / 36, t = (v / 4) % 9, ch = (v & 3) * 8;
                wv[k] = *reinterpret_cast<const uint4*>(a.wt + ((size_t)(n0 + col) * 9 + t) * a.Ka + c0 + ch);
            }
        }
        __syncthreads();                               // the previous chunk's reads are done
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int v = threadIdx.x + k * 256;
            if (v < PV) reinterpret_cast<uint4*>(sP)[v] = pv[k];
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int v = threadIdx.x + k * 256;
            if (v < WV) {
                const int col = v / 36, t = (v / 4) % 9, ch = (v & 3) * 8;
                *reinterpret_cast<uint4*>(sW + col * LDS_BPITCH + t * 32 + ch) = wv[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ty = t / 3, tx = t % 3;
            bf16x8 av[4], bv[2];
            if (HALF == 0) {
                const int oy = a.transpose ? 2 - ty : ty, ox = a.transpose ? 2 - tx : tx;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    av[i] = load8(sP + (((wave * 4 + i + oy) * LDS_PATCH) + r + ox) * 32 + kq * 8);
            } else {
                const int xx = HALF == 1 ? x0 + r + tx - 1 : x0 + r + 1 - tx;
                const int lx = (xx >> 1) - px0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int yy = HALF == 1 ? y0 + wave * 4 + i + ty - 1 : y0 + wave * 4 + i + 1 - ty;
                    const bool ok = HALF == 1 || ((yy | xx) & 1) == 0;
                    av[i] = ok ? load8(sP + (((yy >> 1) - py0) * SIDE + lx) * 32 + kq * 8) : zero8();
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = load8(sW + (j * 16 + r) * LDS_BPITCH + t * 32 + kq * 8);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // D: lane holds rows 4*kq + e (pixels x0 + 4 kq + e) of column r of each tile
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = y0 + wave * 4 + i;
        if (y >= a.Hm) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = x0 + kq * 4 + e;
                if (x >= a.Wm) continue;
                const int nn = n0 + j * 16 + r;
                const int o = ((n * a.Hm + y) * a.Wm + x) * a.Nn + nn;
                float v = acc[i][j][e];
                if (a.epi == EPI_FWD) {
                    v += a.bias[nn];
                    if (a.add) v += bf2f(a.add[o]);
                    a.out[o] = f2bf(fmaxf(v, 0.f));
                } else if (a.epi == EPI_DX_MASK) {
                    if (a.add) v += bf2f(a.add[o]);
                    a.out[o] = f2bf(bf2f(a.mask[o]) > 0.f ? v : 0.f);
                } else {
                    a.outf[o] = v;
                }
            }
    }
}

// ------------------------------------------------------------------ weight gradient

struct DwArgs {
    const uint16_t* dz;     // [N*Ho*Wo][Cout]
    const uint16_t* src;    // layer input, NHWC [N][Hs][Ws][Cin] (low resolution if up)
    int N, Ho, Wo, Hs, Ws, Cout, Cin, stride, up;
    int ppb;                // pixels per block
    float* dw;              // [Cout][9][Cin], accumulated
    float* db;              // [Cout] bias gradient (column sums of dZ), accumulated; may be null
};

// dW[co][t][ci] = sum_p dZ[p][co] X(p, t)[ci].  Block: one tap, a TCO x TCI
// tile, a range of pixels; KP pixels per stage, transposed into LDS so each
// lane reads 8 consecutive pixels of one channel with one 16-byte load.
template <int TCO, int TCI>
__global__ __launch_bounds__(256) void k_conv_dw(DwArgs d) {
    constexpr int KP = 64, PITCH = KP + 8;
    constexpr int MI = TCO / 32, NJ = TCI / 32;
    __shared__ __attribute__((aligned(16))) uint16_t sA[TCO * PITCH];
    __shared__ __attribute__((aligned(16))) uint16_t sB[TCI * PITCH];
    const int t = blockIdx.z, ty = t / 3, tx = t % 3;
    const int nco = d.Cout / TCO;
    const int co0 = (blockIdx.y % nco) * TCO, ci0 = (blockIdx.y / nco) * TCI;
    const int P = d.N * d.Ho * d.Wo;
    const int pbeg = blockIdx.x * d.ppb;
    const int pend = min(P, pbeg + d.ppb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wco = wave & 1, wci = wave >> 1;
    const int r = lane & 15, kq = lane >> 4;
    f32x4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int he = d.up ? 2 * d.Hs : d.Hs, we = d.up ? 2 * d.Ws : d.Ws;
    // the tap-0 blocks of the first input-channel tile also sum dZ per column
    const bool bias = d.db && t == 0 && ci0 == 0;
    float bsum = 0.f;

    for (int pb = pbeg; pb < pend; pb += KP) {
        for (int c = threadIdx.x; c < KP * (TCO / 8); c += 256) {
            const int pix = c / (TCO / 8), ch = (c % (TCO / 8)) * 8;
            const int p = pb + pix;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < pend) v = *reinterpret_cast<const uint4*>(d.dz + p * d.Cout + co0 + ch);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int e = 0; e < 8; ++e) sA[(ch + e) * PITCH + pix] = h[e];
        }
        for (int c = threadIdx.x; c < KP * (TCI / 8); c += 256) {
            const int pix = c / (TCI / 8), ch = (c % (TCI / 8)) * 8;
            const int p = pb + pix;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (p < pend) {
                const unsigned row = (unsigned)p / (unsigned)d.Wo;
                const int x = p - (int)row * d.Wo;
                const int n = (int)(row / (unsigned)d.Ho);
                const int y = (int)row - n * d.Ho;
                const int yy = y * d.stride + ty - 1, xx = x * d.stride + tx - 1;
                if (yy >= 0 && yy < he && xx >= 0 && xx < we) {
                    const int sy = d.up ? yy >> 1 : yy, sx = d.up ? xx >> 1 : xx;
                    const int q = (n * d.Hs + sy) * d.Ws + sx;
                    v = *reinterpret_cast<const uint4*>(d.src + q * d.Cin + ci0 + ch);
                }
            }
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int e = 0; e < 8; ++e) sB[(ch + e) * PITCH + pix] = h[e];
        }
        __syncthreads();
        if (bias && threadIdx.x < TCO)
            for (int k = 0; k < KP; ++k) bsum += bf2f(sA[threadIdx.x * PITCH + k]);   // rows past the range are 0
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks) {
            bf16x8 av[MI], bv[NJ];
#pragma unroll
            for (int i = 0; i < MI; ++i)
                av[i] = load8(&sA[(wco * (TCO / 2) + i * 16 + r) * PITCH + ks * 32 + kq * 8]);
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                bv[j] = load8(&sB[(wci * (TCI / 2) + j * 16 + r) * PITCH + ks * 32 + kq * 8]);
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = co0 + wco * (TCO / 2) + i * 16 + kq * 4 + e;
                const int ci = ci0 + wci * (TCI / 2) + j * 16 + r;
                atomicAdd(&d.dw[((size_t)co * 9 + t) * d.Cin + ci], acc[i][j][e]);
            }
    if (bias && threadIdx.x < TCO) atomicAdd(&d.db[co0 + threadIdx.x], bsum);
}

// ------------------------------------------------------------------ small kernels

// Data gradient through the 2x upsampling: sum the four fine pixels, add the
// skip gradient, pass where the activation is positive, round to BF16.
__global__ __launch_bounds__(256) void k_pool_mask(const float* dxu, int N, int H, int W, int C,
                                                   const uint16_t* add, const uint16_t* mask, uint16_t* out) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int total = N * H * W * C;
    if (idx >= total) return;
    const unsigned pix = (unsigned)idx / (unsigned)C;
    const int c = idx - (int)pix * C;
    const unsigned row = pix / (unsigned)W;
    const int x = (int)(pix - row * (unsigned)W);
    const int n = (int)(row / (unsigned)H);
    const int y = (int)row - n * H;
    const int W2 = 2 * W;
    const int b = ((n * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
    float v = (dxu[b] + dxu[b + C]) + (dxu[b + W2 * C] + dxu[b + W2 * C + C]);
    if (add) v += bf2f(add[idx]);
    out[idx] = f2bf(bf2f(mask[idx]) > 0.f ? v : 0.f);
}

// Network input: depth (mm, clipped to [-3, 3]), six pose-change values,
// previous displacement (mm), zero padding to 32 channels; BF16.
__global__ __launch_bounds__(256) void k_assemble(const float* depth, const float* pose, const float* prev,
                                                  int P, int HW, uint16_t* X) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int n = (int)((unsigned)p / (unsigned)HW);
    uint16_t v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = 0;
    v[0] = f2bf(fminf(fmaxf(depth[p], -3.f), 3.f));
#pragma unroll
    for (int k = 0; k < 6; ++k) v[1 + k] = f2bf(pose[n * 6 + k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[7 + k] = f2bf(prev[p * 3 + k]);
    uint4* o = reinterpret_cast<uint4*>(X + p * 32);
    const uint4* s = reinterpret_cast<const uint4*>(v);
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = s[k];
}

// 1x1 head: next = prev + a13 Wh^T + bh.  Training also forms the loss
// gradient 2 (next - target) / count, the BF16 pre-activation gradient of a13
// (masked by a13 > 0), the head's bias gradient and loss (wave sums), and its
// weight gradient: per 256-pixel chunk the pixels' loss gradients go to LDS
// and thread (k, group) accumulates dout[p][c] a13[p][k] over a share of them.
template <int C0, bool TRAIN>
__global__ __launch_bounds__(256) void k_head(const uint16_t* a13, const float* whf, const float* bh,
                                              const float* prev, const float* tgt, long long P, float two_over_count,
                                              float* out, uint16_t* dz13, float* gwh, float* gbh, float* loss) {
    constexpr int G = 256 / C0;              // pixel groups of the weight-gradient phase
    __shared__ float sw[3 * C0 + 3];
    __shared__ float sd[256 * 3];
    __shared__ float red[256];
    const int tid = threadIdx.x;
    for (int k = tid; k < 3 * C0; k += 256) sw[k] = whf[k];
    if (tid < 3) sw[3 * C0 + tid] = bh[tid];
    __syncthreads();
    const int kk = tid % C0, grp = tid / C0;
    float gwa[3] = {0.f, 0.f, 0.f}, gb[3] = {0.f, 0.f, 0.f}, ls = 0.f;
    for (long long base = (long long)blockIdx.x * 256; base < P; base += (long long)gridDim.x * 256) {
        const long long p = base + tid;
        float dout[3] = {0.f, 0.f, 0.f};
        if (p < P) {
            float a[C0];
            const uint4* s = reinterpret_cast<const uint4*>(a13 + p * C0);
#pragma unroll
            for (int q = 0; q < C0 / 8; ++q) {
                const uint4 v = s[q];
                const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
                for (int e = 0; e < 8; ++e) a[q * 8 + e] = bf2f(h[e]);
            }
            float hd[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < C0; ++k) acc += a[k] * sw[c * C0 + k];
                hd[c] = prev[p * 3 + c] + (acc + sw[3 * C0 + c]);
            }
            if (!TRAIN) {
#pragma unroll
                for (int c = 0; c < 3; ++c) out[p * 3 + c] = hd[c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float df = hd[c] - tgt[p * 3 + c];
                    ls += df * df;
                    dout[c] = two_over_count * df;
                    gb[c] += dout[c];
                }
                uint16_t dz[C0];
#pragma unroll
                for (int k = 0; k < C0; ++k) {
                    const float g = dout[0] * sw[k] + dout[1] * sw[C0 + k] + dout[2] * sw[2 * C0 + k];
                    dz[k] = f2bf(a[k] > 0.f ? g : 0.f);
                }
                uint4* o = reinterpret_cast<uint4*>(dz13 + p * C0);
#pragma unroll
                for (int q = 0; q < C0 / 8; ++q) o[q] = reinterpret_cast<const uint4*>(dz)[q];
            }
        }
        if (!TRAIN) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) sd[tid * 3 + c] = dout[c];
        __syncthreads();
        for (int q = grp; q < 256; q += G) {
            const long long pq = base + q;
            if (pq >= P) break;
            const float av = bf2f(a13[pq * C0 + kk]);
#pragma unroll
            for (int c = 0; c < 3; ++c) gwa[c] += sd[q * 3 + c] * av;
        }
        __syncthreads();
    }
    if (!TRAIN) return;
    // weight gradient: sum the groups through LDS
    for (int c = 0; c < 3; ++c) {
        red[tid] = gwa[c];
        __syncthreads();
        if (tid < C0) {
            float v = 0.f;
            for (int g2 = 0; g2 < G; ++g2) v += red[g2 * C0 + tid];
            atomicAdd(&gwh[c * C0 + tid], v);
        }
        __syncthreads();
    }
    // bias gradient and loss: wave shuffles, then the four waves
    const int lane = tid & 63, wave = tid >> 6;
    float vals[4] = {gb[0], gb[1], gb[2], ls};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float v = vals[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave * 4 + q] = v;
    }
    __syncthreads();
    if (tid < 4) {
        const float v = (red[tid] + red[4 + tid]) + (red[8 + tid] + red[12 + tid]);
        if (tid < 3) atomicAdd(&gbh[tid], v);
        else atomicAdd(loss, v);
    }
}

__global__ __launch_bounds__(256) void k_adam(float* th, const float* g, float* m, float* v, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// BF16 copies of a convolution's master weights [Cout][9][Cin]: as stored and
// transposed to [Cin][9][Cout] for the data gradient.
__global__ __launch_bounds__(256) void k_cast_w(const float* th, int Cout, int Cin, uint16_t* w, uint16_t* wt) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)Cout * 9 * Cin) return;
    const int ci = (int)(i % Cin), t = (int)((i / Cin) % 9), co = (int)(i / (9LL * Cin));
    const uint16_t b = f2bf(th[i]);
    w[i] = b;
    wt[((size_t)ci * 9 + t) * Cout + co] = b;
}

__global__ __launch_bounds__(256) void k_cast_head(const float* th, int n, float* whf) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) whf[i] = bf2f(f2bf(th[i]));
}

// Contact area (pixels) of each sample: pixels where the indenter's lower
// surface is within tol of the displaced elastomer surface or below it,
// depth + u_z >= -tol (all mm).  One block per sample.
__global__ __launch_bounds__(256) void k_contact_area(const float* depth, const float* disp, int HW, float tol,
                                                      float* area) {
    __shared__ int red[4];
    const long long base = (long long)blockIdx.x * HW;
    int c = 0;
    for (int q = threadIdx.x; q < HW; q += 256) c += depth[base + q] + disp[(base + q) * 3 + 2] >= -tol ? 1 : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) area[blockIdx.x] = (float)(red[0] + red[1] + red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_zero(float* p, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = 0.f;
}

}  // namespace sur

using namespace sur;

// ------------------------------------------------------------------ host

namespace {

struct Layer {
    int cin, cin_pad, cout, stride, up, skip;  // skip: index of the added activation, or -1
    int hin, win;       // spatial size of the source tensor (low resolution for up layers)
    int hout, wout;
    long long w_off, b_off;         // internal (padded) master layout
    long long lw_off, lb_off;       // logical layout of sur_get_params
    uint16_t* w = nullptr;          // [cout][9][cin_pad] BF16
    uint16_t* wt = nullptr;         // [cin_pad][9][cout] BF16
};

}  // namespace

struct sur_s {
    sur_params P;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<Layer> L;
    int consumer_of[14];            // decoder layer that adds activation i, or -1
    long long n_int = 0, n_log = 0; // master parameters: internal (padded) and logical counts
    long long head_w_off = 0, head_b_off = 0, head_lw_off = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    float* whf = nullptr;           // head weights rounded to BF16, as FP32
    float* loss = nullptr;          // device accumulator
    uint16_t* x0 = nullptr;         // [B][H][W][32]
    uint16_t* act[14] = {};
    uint16_t* dz[14] = {};
    float* dxu = nullptr;           // FP32 data gradient at the upsampled resolution
    long long dxu_elems = 0;
    long long t = 0;                // Adam steps taken
    int n_last = 0;                 // batch of the last forward pass
    std::string err;
};

static int sfail(sur_t* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

#define SHIP(s, call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return sfail((s), SUR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

static void launch_conv(const ConvArgs& a, hipStream_t st) {
    const long long M = (long long)a.N * a.Hm * a.Wm;
    const int tiles = ((a.Wm + LDS_TILE - 1) / LDS_TILE) * ((a.Hm + LDS_TILE - 1) / LDS_TILE) * a.N;
    if (a.stride == 1 && !a.up) {
        hipLaunchKernelGGL(k_conv_lds<0>, dim3((unsigned)tiles, a.Nn / 32), dim3(256), 0, st, a);
        return;
    }
    if (a.up && !a.transpose && a.stride == 1) {
        hipLaunchKernelGGL(k_conv_lds<1>, dim3((unsigned)tiles, a.Nn / 32), dim3(256), 0, st, a);
        return;
    }
    if (a.transpose && a.stride == 2 && !a.up) {
        hipLaunchKernelGGL(k_conv_lds<2>, dim3((unsigned)tiles, a.Nn / 32), dim3(256), 0, st, a);
        return;
    }
    if (a.Nn == 32) {
        hipLaunchKernelGGL((k_conv<4, 2, 4, 1>), dim3((unsigned)((M + 255) / 256), 1), dim3(256), 0, st, a);
    } else if (a.Nn == 64) {
        hipLaunchKernelGGL((k_conv<4, 4, 4, 1>), dim3((unsigned)((M + 255) / 256), 1), dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_conv<4, 4, 2, 2>), dim3((unsigned)((M + 127) / 128), a.Nn / 128), dim3(256), 0, st, a);
    }
}

static void launch_dw(const DwArgs& d, hipStream_t st) {
    const int tco = std::min(64, d.Cout), tci = std::min(64, d.Cin);
    const int tiles = (d.Cout / tco) * (d.Cin / tci);
    const long long P = (long long)d.N * d.Ho * d.Wo;
    long long splits = std::max(1LL, (2048 + 9LL * tiles - 1) / (9LL * tiles));
    long long ppb = (P + splits - 1) / splits;
    ppb = std::max(64LL, (ppb + 63) / 64 * 64);
    splits = (P + ppb - 1) / ppb;
    DwArgs a = d;
    a.ppb = (int)ppb;
    const dim3 grid((unsigned)splits, (unsigned)tiles, 9);
    if (tco == 64 && tci == 64) hipLaunchKernelGGL((k_conv_dw<64, 64>), grid, dim3(256), 0, st, a);
    else if (tco == 64) hipLaunchKernelGGL((k_conv_dw<64, 32>), grid, dim3(256), 0, st, a);
    else if (tci == 64) hipLaunchKernelGGL((k_conv_dw<32, 64>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_conv_dw<32, 32>), grid, dim3(256), 0, st, a);
}

static void launch_head(sur_t* s, bool train, int n, const float* prev, const float* tgt, float* out) {
    const long long P = (long long)n * s->P.H * s->P.W;
    const float toc = 2.0f / (float)(P * 3);
    const unsigned nb = (unsigned)std::min<long long>((P + 255) / 256, 1024);
    float* g = s->grad;
    const float* bh = s->theta + s->head_b_off;
    if (s->P.channels[0] == 32) {
        if (train)
            hipLaunchKernelGGL((k_head<32, true>), dim3(nb), dim3(256), 0, s->stream, s->act[13], s->whf, bh, prev, tgt,
                               P, toc, out, s->dz[13], g + s->head_w_off, g + s->head_b_off, s->loss);
        else
            hipLaunchKernelGGL((k_head<32, false>), dim3(nb), dim3(256), 0, s->stream, s->act[13], s->whf, bh, prev,
                               tgt, P, toc, out, s->dz[13], g + s->head_w_off, g + s->head_b_off, s->loss);
    } else {
        if (train)
            hipLaunchKernelGGL((k_head<64, true>), dim3(nb), dim3(256), 0, s->stream, s->act[13], s->whf, bh, prev, tgt,
                               P, toc, out, s->dz[13], g + s->head_w_off, g + s->head_b_off, s->loss);
        else
            hipLaunchKernelGGL((k_head<64, false>), dim3(nb), dim3(256), 0, s->stream, s->act[13], s->whf, bh, prev,
                               tgt, P, toc, out, s->dz[13], g + s->head_w_off, g + s->head_b_off, s->loss);
    }
}

static void cast_all(sur_t* s) {
    for (Layer& l : s->L) {
        const long long n = (long long)l.cout * 9 * l.cin_pad;
        hipLaunchKernelGGL(k_cast_w, dim3(blocks_for(n)), dim3(256), 0, s->stream, s->theta + l.w_off, l.cout,
                           l.cin_pad, l.w, l.wt);
    }
    const int nh = 3 * s->P.channels[0];
    hipLaunchKernelGGL(k_cast_head, dim3(blocks_for(nh)), dim3(256), 0, s->stream, s->theta + s->head_w_off, nh,
                       s->whf);
}

static int check_io(sur_t* s, const void* a, const void* b, const void* c, int n) {
    if (!s) return SUR_EINVAL;
    if (!a || !b || !c) return sfail(s, SUR_EINVAL, "null input pointer");
    if (n < 1 || n > s->P.max_batch) return sfail(s, SUR_EINVAL, "n must be in [1, max_batch]");
    return SUR_OK;
}

static void forward(sur_t* s, int n, const float* depth, const float* pose, const float* prev) {
    const int H = s->P.H, W = s->P.W;
    s->n_last = n;
    const long long P = (long long)n * H * W;
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(P)), dim3(256), 0, s->stream, depth, pose, prev, (int)P, H * W,
                       s->x0);
    for (int li = 0; li < 14; ++li) {
        const Layer& l = s->L[li];
        ConvArgs a{};
        a.src = li == 0 ? s->x0 : s->act[li - 1];
        a.wt = l.w;
        a.N = n; a.Hm = l.hout; a.Wm = l.wout;
        a.Hs = l.hin; a.Ws = l.win; a.Ka = l.cin_pad; a.Nn = l.cout;
        a.stride = l.stride; a.up = l.up; a.transpose = 0;
        a.epi = EPI_FWD;
        a.bias = s->theta + l.b_off;
        a.add = l.skip >= 0 ? s->act[l.skip] : nullptr;
        a.out = s->act[li];
        launch_conv(a, s->stream);
    }
}

static void backward(sur_t* s, int n, const float* prev, const float* tgt) {
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s->stream, s->grad, s->n_int);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s->stream, s->loss, 1LL);
    launch_head(s, true, n, prev, tgt, nullptr);
    for (int li = 13; li >= 0; --li) {
        const Layer& l = s->L[li];
        DwArgs d{};
        d.dz = s->dz[li];
        d.src = li == 0 ? s->x0 : s->act[li - 1];
        d.N = n; d.Ho = l.hout; d.Wo = l.wout; d.Hs = l.hin; d.Ws = l.win;
        d.Cout = l.cout; d.Cin = l.cin_pad; d.stride = l.stride; d.up = l.up;
        d.dw = s->grad + l.w_off;
        d.db = s->grad + l.b_off;
        launch_dw(d, s->stream);
        if (li == 0) break;
        const int prevl = li - 1;
        const uint16_t* sg = s->consumer_of[prevl] >= 0 ? s->dz[s->consumer_of[prevl]] : nullptr;
        ConvArgs a{};
        a.src = s->dz[li];
        a.wt = l.wt;
        a.N = n;
        a.Hm = l.up ? 2 * l.hin : l.hin;      // rows: the convolution's input pixels
        a.Wm = l.up ? 2 * l.win : l.win;
        a.Hs = l.hout; a.Ws = l.wout; a.Ka = l.cout; a.Nn = l.cin_pad;
        a.stride = l.stride; a.up = 0; a.transpose = 1;
        if (l.up) {
            a.epi = EPI_DX_RAW;
            a.outf = s->dxu;
            launch_conv(a, s->stream);
            const long long tot = (long long)n * l.hin * l.win * l.cin_pad;
            hipLaunchKernelGGL(k_pool_mask, dim3(blocks_for(tot)), dim3(256), 0, s->stream, s->dxu, n, l.hin, l.win,
                               l.cin_pad, sg, s->act[prevl], s->dz[prevl]);
        } else {
            a.epi = EPI_DX_MASK;
            a.add = sg;
            a.mask = s->act[prevl];
            a.out = s->dz[prevl];
            launch_conv(a, s->stream);
        }
    }
}

// SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller normals for the initial weights.
static uint64_t sm64(uint64_t& st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static double normal(uint64_t& st) {
    const double u1 = ((sm64(st) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (sm64(st) >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// logical (API) <-> internal (padded) master layout
static void to_internal(const sur_t* s, const float* lg, std::vector<float>& in) {
    in.assign(s->n_int, 0.f);
    for (const Layer& l : s->L) {
        for (int co = 0; co < l.cout; ++co)
            for (int t = 0; t < 9; ++t)
                for (int ci = 0; ci < l.cin; ++ci)
                    in[l.w_off + ((long long)co * 9 + t) * l.cin_pad + ci] = lg[l.lw_off + ((long long)co * 9 + t) * l.cin + ci];
        for (int co = 0; co < l.cout; ++co) in[l.b_off + co] = lg[l.lb_off + co];
    }
    const int nh = 3 * s->P.channels[0];
    for (int k = 0; k < nh + 3; ++k) in[s->head_w_off + k] = lg[s->head_lw_off + k];
}
static void to_logical(const sur_t* s, const float* in, float* lg) {
    for (const Layer& l : s->L) {
        for (int co = 0; co < l.cout; ++co)
            for (int t = 0; t < 9; ++t)
                for (int ci = 0; ci < l.cin; ++ci)
                    lg[l.lw_off + ((long long)co * 9 + t) * l.cin + ci] = in[l.w_off + ((long long)co * 9 + t) * l.cin_pad + ci];
        for (int co = 0; co < l.cout; ++co) lg[l.lb_off + co] = in[l.b_off + co];
    }
    const int nh = 3 * s->P.channels[0];
    for (int k = 0; k < nh + 3; ++k) lg[s->head_lw_off + k] = in[s->head_w_off + k];
}

static int upload_params(sur_t* s, const std::vector<float>& in) {
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(s->theta, in.data(), s->n_int * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s->stream, s->m, s->n_int);
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s->stream, s->v, s->n_int);
    cast_all(s);
    SHIP(s, hipGetLastError());
    SHIP(s, hipStreamSynchronize(s->stream));
    s->t = 0;
    return SUR_OK;
}

extern "C" {

int sur_params_default(sur_params* p) {
    if (!p) return SUR_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->H = 128; p->W = 128;
    p->channels[0] = 32; p->channels[1] = 64; p->channels[2] = 128; p->channels[3] = 256;
    p->max_batch = 64;
    p->seed = 2405;
    p->lr = 1e-3f; p->beta1 = 0.9f; p->beta2 = 0.999f; p->eps = 1e-8f;
    return SUR_OK;
}

void sur_destroy(sur_t* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (Layer& l : s->L) {
        if (l.w) (void)hipFree(l.w);
        if (l.wt) (void)hipFree(l.wt);
    }
    void* bufs[] = {s->theta, s->grad, s->m, s->v, s->whf, s->loss, s->x0, s->dxu};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int i = 0; i < 14; ++i) {
        if (s->act[i]) (void)hipFree(s->act[i]);
        if (s->dz[i]) (void)hipFree(s->dz[i]);
    }
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int sur_create(const sur_params* p, void* hip_stream, sur_t** out) {
    if (!p || !out) return SUR_EINVAL;
    *out = nullptr;
    if (p->H < 8 || p->W < 8 || p->H % 8 || p->W % 8 || p->H > 4096 || p->W > 4096 || p->max_batch < 1) {
        std::fprintf(stderr, "sur_create: H, W must be multiples of 8 in [8, 4096], max_batch >= 1\n");
        return SUR_EINVAL;
    }
    // the kernels index every tensor with 32-bit integers
    if ((long long)p->max_batch * p->H * p->W * 256 >= (1LL << 31)) {
        std::fprintf(stderr, "sur_create: max_batch * H * W * 256 must stay below 2^31\n");
        return SUR_EINVAL;
    }
    // the tile shapes of the convolution kernels cover 32, 64, 128 and 256 channels
    for (int k = 0; k < 4; ++k) {
        const int c = p->channels[k];
        if ((c != 32 && c != 64 && c != 128 && c != 256) || (k == 0 && c > 64)) {
            std::fprintf(stderr, "sur_create: channels must be 32, 64, 128 or 256 (c0 <= 64)\n");
            return SUR_EINVAL;
        }
    }
    if (!(p->lr >= 0.f) || !(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f) ||
        !(p->eps > 0.f)) {
        std::fprintf(stderr, "sur_create: bad Adam hyper-parameters\n");
        return SUR_EINVAL;
    }
    sur_t* s = new sur_t();
    s->P = *p;
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) { delete s; return SUR_EHIP; }
        s->own_stream = true;
    }
    auto bail = [&](int rc) { sur_destroy(s); return rc; };
    const int* c = p->channels;
    // (cin, cout, stride, up, skip) of the 14 convolutions
    const int spec[14][5] = {{10, c[0], 1, 0, -1}, {c[0], c[0], 1, 0, -1}, {c[0], c[1], 2, 0, -1},
                             {c[1], c[1], 1, 0, -1}, {c[1], c[2], 2, 0, -1}, {c[2], c[2], 1, 0, -1},
                             {c[2], c[3], 2, 0, -1}, {c[3], c[3], 1, 0, -1}, {c[3], c[2], 1, 1, 5},
                             {c[2], c[2], 1, 0, -1}, {c[2], c[1], 1, 1, 3}, {c[1], c[1], 1, 0, -1},
                             {c[1], c[0], 1, 1, 1}, {c[0], c[0], 1, 0, -1}};
    for (int i = 0; i < 14; ++i) s->consumer_of[i] = -1;
    int h = p->H, w = p->W;
    long long off = 0, loff = 0;
    for (int i = 0; i < 14; ++i) {
        Layer l;
        l.cin = spec[i][0]; l.cin_pad = i == 0 ? 32 : spec[i][0]; l.cout = spec[i][1];
        l.stride = spec[i][2]; l.up = spec[i][3]; l.skip = spec[i][4];
        l.hin = h; l.win = w;
        if (l.stride == 2) { h /= 2; w /= 2; }
        if (l.up) { h *= 2; w *= 2; }
        l.hout = h; l.wout = w;
        l.w_off = off; off += (long long)l.cout * 9 * l.cin_pad;
        l.b_off = off; off += l.cout;
        l.lw_off = loff; loff += (long long)l.cout * 9 * l.cin;
        l.lb_off = loff; loff += l.cout;
        if (l.skip >= 0) s->consumer_of[l.skip] = i;
        s->L.push_back(l);
    }
    s->head_w_off = off; s->head_b_off = off + 3 * c[0]; off += 3 * c[0] + 3;
    s->head_lw_off = loff; loff += 3 * c[0] + 3;
    s->n_int = off;
    s->n_log = loff;
    const size_t B = (size_t)p->max_batch;
    if (hipMalloc(&s->theta, off * 4) != hipSuccess || hipMalloc(&s->grad, off * 4) != hipSuccess ||
        hipMalloc(&s->m, off * 4) != hipSuccess || hipMalloc(&s->v, off * 4) != hipSuccess ||
        hipMalloc(&s->whf, 3 * c[0] * 4) != hipSuccess || hipMalloc(&s->loss, 4) != hipSuccess ||
        hipMalloc(&s->x0, B * p->H * p->W * 32 * 2) != hipSuccess)
        return bail(SUR_ENOMEM);
    for (int i = 0; i < 14; ++i) {
        Layer& l = s->L[i];
        const size_t na = B * l.hout * l.wout * l.cout * 2;
        if (hipMalloc(&s->act[i], na) != hipSuccess || hipMalloc(&s->dz[i], na) != hipSuccess ||
            hipMalloc(&l.w, (size_t)l.cout * 9 * l.cin_pad * 2) != hipSuccess ||
            hipMalloc(&l.wt, (size_t)l.cout * 9 * l.cin_pad * 2) != hipSuccess)
            return bail(SUR_ENOMEM);
        if (l.up) s->dxu_elems = std::max(s->dxu_elems, (long long)B * 4 * l.hin * l.win * l.cin_pad);
    }
    if (hipMalloc(&s->dxu, s->dxu_elems * 4) != hipSuccess) return bail(SUR_ENOMEM);
    // He-normal initial weights, zero biases, a small head
    std::vector<float> lg(s->n_log, 0.f);
    uint64_t st = p->seed;
    for (const Layer& l : s->L) {
        const double sd = std::sqrt(2.0 / (9.0 * l.cin));
        for (long long k = 0; k < (long long)l.cout * 9 * l.cin; ++k) lg[l.lw_off + k] = (float)(sd * normal(st));
    }
    for (int k = 0; k < 3 * c[0]; ++k) lg[s->head_lw_off + k] = (float)(1e-3 * normal(st));
    std::vector<float> in;
    to_internal(s, lg.data(), in);
    const int rc = upload_params(s, in);
    if (rc) { const int r2 = rc; sur_destroy(s); return r2; }
    *out = s;
    return SUR_OK;
}

int sur_num_params(const sur_t* s, int64_t* n) {
    if (!s || !n) return SUR_EINVAL;
    *n = s->n_log;
    return SUR_OK;
}

int sur_infer(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm, float* next_mm, int32_t n) {
    int rc = check_io(s, depth_mm, pose6, prev_mm, n);
    if (rc) return rc;
    if (!next_mm) return sfail(s, SUR_EINVAL, "null output pointer");
    forward(s, n, depth_mm, pose6, prev_mm);
    launch_head(s, false, n, prev_mm, nullptr, next_mm);
    SHIP(s, hipGetLastError());
    return SUR_OK;
}

static int grads_and_loss(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm,
                          const float* target_mm, int32_t n, float* loss_out) {
    int rc = check_io(s, depth_mm, pose6, prev_mm, n);
    if (rc) return rc;
    if (!target_mm) return sfail(s, SUR_EINVAL, "null target pointer");
    forward(s, n, depth_mm, pose6, prev_mm);
    backward(s, n, prev_mm, target_mm);
    SHIP(s, hipGetLastError());
    if (loss_out) {
        float l = 0.f;
        SHIP(s, hipMemcpyAsync(&l, s->loss, 4, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipStreamSynchronize(s->stream));
        *loss_out = l / (float)((long long)n * s->P.H * s->P.W * 3);
    }
    return SUR_OK;
}

int sur_compute_grads(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm,
                      const float* target_mm, int32_t n, float* loss_out) {
    return grads_and_loss(s, depth_mm, pose6, prev_mm, target_mm, n, loss_out);
}

int sur_train_step(sur_t* s, const float* depth_mm, const float* pose6, const float* prev_mm,
                   const float* target_mm, int32_t n, float* loss_out) {
    int rc = grads_and_loss(s, depth_mm, pose6, prev_mm, target_mm, n, loss_out);
    if (rc) return rc;
    s->t += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)s->P.beta1, (double)s->t));
    const double c2 = 1.0 / (1.0 - std::pow((double)s->P.beta2, (double)s->t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(s->n_int)), dim3(256), 0, s->stream, s->theta, s->grad, s->m, s->v,
                       s->n_int, s->P.lr, s->P.beta1, s->P.beta2, s->P.eps, (float)c1, (float)c2);
    cast_all(s);
    SHIP(s, hipGetLastError());
    return SUR_OK;
}

int sur_contact_area(sur_t* s, const float* depth_mm, const float* disp_mm, int32_t n, float tol_mm, float* area) {
    if (!s) return SUR_EINVAL;
    if (!depth_mm || !disp_mm || !area || n < 1 || !(tol_mm >= 0.f))
        return sfail(s, SUR_EINVAL, "bad contact-area arguments");
    hipLaunchKernelGGL(k_contact_area, dim3(n), dim3(256), 0, s->stream, depth_mm, disp_mm, s->P.H * s->P.W, tol_mm,
                       area);
    SHIP(s, hipGetLastError());
    return SUR_OK;
}

int sur_set_lr(sur_t* s, float lr) {
    if (!s) return SUR_EINVAL;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return sfail(s, SUR_EINVAL, "bad learning rate");
    s->P.lr = lr;
    return SUR_OK;
}

int sur_get_grads(sur_t* s, float* out_host) {
    if (!s || !out_host) return SUR_EINVAL;
    std::vector<float> in(s->n_int);
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(in.data(), s->grad, s->n_int * 4, hipMemcpyDeviceToHost));
    to_logical(s, in.data(), out_host);
    return SUR_OK;
}

int sur_get_params(sur_t* s, float* out_host) {
    if (!s || !out_host) return SUR_EINVAL;
    std::vector<float> in(s->n_int);
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(in.data(), s->theta, s->n_int * 4, hipMemcpyDeviceToHost));
    to_logical(s, in.data(), out_host);
    return SUR_OK;
}

int sur_set_params(sur_t* s, const float* in_host) {
    if (!s || !in_host) return SUR_EINVAL;
    for (long long k = 0; k < s->n_log; ++k)
        if (!std::isfinite(in_host[k])) return sfail(s, SUR_EINVAL, "non-finite parameter");
    std::vector<float> in;
    to_internal(s, in_host, in);
    return upload_params(s, in);
}

static const char kMagic[8] = {'I', 'M', 'P', 'M', 'S', 'U', 'R', '1'};

int sur_save(sur_t* s, const char* path) {
    if (!s || !path) return SUR_EINVAL;
    std::vector<float> th(s->n_int), m(s->n_int), v(s->n_int);
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(th.data(), s->theta, s->n_int * 4, hipMemcpyDeviceToHost));
    SHIP(s, hipMemcpy(m.data(), s->m, s->n_int * 4, hipMemcpyDeviceToHost));
    SHIP(s, hipMemcpy(v.data(), s->v, s->n_int * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return sfail(s, SUR_EIO, std::string("cannot open ") + path);
    const int32_t hdr[6] = {s->P.H, s->P.W, s->P.channels[0], s->P.channels[1], s->P.channels[2], s->P.channels[3]};
    const int64_t nt[2] = {s->n_int, s->t};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 6, f) == 6 && std::fwrite(nt, 8, 2, f) == 2 &&
              std::fwrite(th.data(), 4, th.size(), f) == th.size() &&
              std::fwrite(m.data(), 4, m.size(), f) == m.size() && std::fwrite(v.data(), 4, v.size(), f) == v.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SUR_OK : sfail(s, SUR_EIO, std::string("write failed: ") + path);
}

int sur_load(sur_t* s, const char* path) {
    if (!s || !path) return SUR_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return sfail(s, SUR_EIO, std::string("cannot open ") + path);
    char mg[8];
    int32_t hdr[6];
    int64_t nt[2];
    bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0 && std::fread(hdr, 4, 6, f) == 6 &&
              std::fread(nt, 8, 2, f) == 2;
    ok = ok && hdr[0] == s->P.H && hdr[1] == s->P.W && hdr[2] == s->P.channels[0] && hdr[3] == s->P.channels[1] &&
         hdr[4] == s->P.channels[2] && hdr[5] == s->P.channels[3] && nt[0] == s->n_int && nt[1] >= 0;
    std::vector<float> th(s->n_int), m(s->n_int), v(s->n_int);
    ok = ok && std::fread(th.data(), 4, th.size(), f) == th.size() && std::fread(m.data(), 4, m.size(), f) == m.size() &&
         std::fread(v.data(), 4, v.size(), f) == v.size();
    std::fclose(f);
    if (!ok) return sfail(s, SUR_EIO, std::string("not a surrogate file of this shape: ") + path);
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(s->theta, th.data(), s->n_int * 4, hipMemcpyHostToDevice));
    SHIP(s, hipMemcpy(s->m, m.data(), s->n_int * 4, hipMemcpyHostToDevice));
    SHIP(s, hipMemcpy(s->v, v.data(), s->n_int * 4, hipMemcpyHostToDevice));
    cast_all(s);
    SHIP(s, hipGetLastError());
    SHIP(s, hipStreamSynchronize(s->stream));
    s->t = nt[1];
    return SUR_OK;
}

int sur_debug_read(sur_t* s, int32_t which, int32_t layer, uint16_t* out_host) {
    if (!s || !out_host) return SUR_EINVAL;
    if (s->n_last < 1) return sfail(s, SUR_EINVAL, "no forward pass yet");
    const uint16_t* src = nullptr;
    size_t count = 0;
    if (which == 2) {
        src = s->x0;
        count = (size_t)s->n_last * s->P.H * s->P.W * 32;
    } else if ((which == 0 || which == 1) && layer >= 0 && layer < 14) {
        const Layer& l = s->L[layer];
        src = which == 0 ? s->act[layer] : s->dz[layer];
        count = (size_t)s->n_last * l.hout * l.wout * l.cout;
    } else {
        return sfail(s, SUR_EINVAL, "bad which or layer");
    }
    SHIP(s, hipStreamSynchronize(s->stream));
    SHIP(s, hipMemcpy(out_host, src, count * 2, hipMemcpyDeviceToHost));
    return SUR_OK;
}

const char* sur_last_error(const sur_t* s) { return s ? s->err.c_str() : "null handle"; }

}  // extern "C"
