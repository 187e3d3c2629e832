// Warm-start network of libglbm: BF16 MFMA convolutions for gfx950 and the
// small kernels around them (pooling, upsampling, ReLU masks, loss, Adam).
//
// Convolutions are 3x3, stride 1, periodic, channels-last.  The forward pass
// is an implicit GEMM: M = pixels, N = output channels, K = 9 * input channels
// (k = tap * cin + ci).  Each 256-thread workgroup owns 64 consecutive pixels
// of one image row and up to 64 output channels; each wavefront owns 16 of
// those pixels and issues v_mfma_f32_16x16x32_bf16 per 32-wide slice of K:
// the A operand (16 pixels x 8 channels per lane) is read straight from the
// activations, the B operand (weights) from an LDS copy of a 128-wide K chunk.
// The data gradient is the same kernel with flipped, transposed weights; the
// weight gradient is a second MFMA kernel that reduces over pixels (split-K,
// partials summed in a fixed order).
#include "glbm_cnn.h"
#include "glbm_internal.h"

#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace glbm {
void set_error(const char* msg);  // glbm_api.cpp
}

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kConvBlock = 256;
constexpr int kPixTile = 64;   // pixels per workgroup
constexpr int kChTile = 64;    // output channels per workgroup (grid.y)
constexpr int kKChunk = 128;   // K columns staged in LDS at a time
constexpr int kLdsRow = kKChunk + 8;  // padded LDS row (bf16), breaks bank alignment

int rup(int v, int m) { return (v + m - 1) / m * m; }

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (finite inputs); NaN stays NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return uint16_t((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

struct ConvArgs {
    const uint16_t* x;
    const uint16_t* w;
    const float* bias;
    void* y;
    int x_pitch, x_off, cin;
    int y_pitch, y_off, cout;
    int k_real, k_pad, cout_pad;
    int H, W;
    long long npix;
    int y_vec;  // 1: four consecutive output channels may be written with one 8-byte (bf16) / 16-byte (FP32) store
};

// ------------------------------------------------------------------ forward --
template <bool OUT_F32, bool RELU, bool ACC>
__global__ __launch_bounds__(kConvBlock) void k_conv_fwd(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t wt[kChTile * kLdsRow];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, kq = lane >> 4;
    const long long p0 = (long long)blockIdx.x * kPixTile;
    const int n0 = blockIdx.y * kChTile;
    const int nt = min(kChTile, a.cout_pad - n0) >> 4;  // 16-channel blocks (1..4)

    // this lane's A row: pixel p (b, y, x)
    const long long p = p0 + wave * 16 + m;
    const int HW = a.H * a.W;
    const int b = int(p / HW);
    const int rem = int(p - (long long)b * HW);
    const int py = rem / a.W, px = rem - py * a.W;
    const uint16_t* xb = a.x + (size_t)b * HW * a.x_pitch + a.x_off;

    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int kk0 = 0; kk0 < a.k_pad; kk0 += kKChunk) {
        const int kc = min(kKChunk, a.k_pad - kk0);
        __syncthreads();
        // stage w[n0 .. n0 + 64][kk0 .. kk0 + kc] (16-byte pieces)
        for (int e = threadIdx.x; e < kChTile * (kKChunk / 8); e += kConvBlock) {
            const int r = e / (kKChunk / 8), c8 = (e % (kKChunk / 8)) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (n0 + r < a.cout_pad && c8 < kc)
                v = *reinterpret_cast<const uint4*>(a.w + (size_t)(n0 + r) * a.k_pad + kk0 + c8);
            *reinterpret_cast<uint4*>(&wt[r * kLdsRow + c8]) = v;
        }
        __syncthreads();
        for (int ks = 0; ks < kc; ks += 32) {
            const int k = kk0 + ks + 8 * kq;
            uint4 av = make_uint4(0, 0, 0, 0);
            if (k < a.k_real) {
                const int tap = k / a.cin, ci = k - tap * a.cin;
                int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
                yy += yy < 0 ? a.H : (yy >= a.H ? -a.H : 0);
                xx += xx < 0 ? a.W : (xx >= a.W ? -a.W : 0);
                av = *reinterpret_cast<const uint4*>(xb + (size_t)(yy * a.W + xx) * a.x_pitch + ci);
            }
            const bf16x8 af = __builtin_bit_cast(bf16x8, av);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j < nt) {
                    const uint4 bv = *reinterpret_cast<const uint4*>(&wt[(16 * j + m) * kLdsRow + ks + 8 * kq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, __builtin_bit_cast(bf16x8, bv), acc[j], 0, 0,
                                                                      0);
                }
            }
        }
    }
    // epilogue: lane holds D[4 kq + i][m] of each 16 x 16 block
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (j >= nt) continue;
        const int n = n0 + 16 * j + m;
        if (n >= a.cout) continue;
        const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long long q = p0 + wave * 16 + 4 * kq + i;
            float v = acc[j][i] + bias;
            if (RELU) v = fmaxf(v, 0.f);
            if (OUT_F32) {
                static_cast<float*>(a.y)[(size_t)q * a.y_pitch + a.y_off + n] = v;
            } else {
                uint16_t* yp = static_cast<uint16_t*>(a.y) + (size_t)q * a.y_pitch + a.y_off + n;
                if (ACC) v += bf2f(*yp);
                *yp = f2bf(v);
            }
        }
    }
}

// ------------------------------------------------ forward, row-reuse path --
// For cin = 32 CI.  A wavefront owns 16 pixels in each of R consecutive rows;
// the workgroup's four wavefronts sit side by side (64 x R pixels).  K runs
// over 32-channel slices of the input and, within a slice, over the column
// shifts dx = -1, 0, 1: the slice's 16-byte fragments of the R + 2 input rows
// at that shift are loaded once and serve every (dy, output row) pair that
// reads them, so R + 2 loads feed 3 R NT MFMAs (a tap-by-tap loop spends
// one load per NT MFMAs).  The slice's weights for all nine taps (16 NT
// channels x 32) sit in LDS.  The weights are the MFMA's row operand, so a
// lane ends with four consecutive output channels of its own pixel and
// writes them with one 8-byte (bf16) or 16-byte (FP32) store.
constexpr int kRwRow = 40;  // 32 channels + 8 pad (bf16): 80-byte rows, 16 lanes hit 64 distinct banks

template <int CI, int NT, int R, bool OUT_F32, bool RELU, bool ACC>
__global__ __launch_bounds__(kConvBlock) void k_conv_fwd_rows(ConvArgs a)
{
    constexpr int kCin = 32 * CI;
    constexpr int kN = 16 * NT;
    __shared__ __attribute__((aligned(16))) uint16_t wt[9 * kN * kRwRow];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, kq = lane >> 4;
    const int xtiles = a.W >> 6, ytiles = (a.H + R - 1) / R;
    const int xt = (int)blockIdx.x % xtiles, rest = (int)blockIdx.x / xtiles;
    const int yt = rest % ytiles, b = rest / ytiles;
    const int x = (xt << 6) + 16 * wave + m;  // this lane's pixel column
    const int y0 = yt * R;
    const int n0 = blockIdx.y * kN;
    const size_t img = (size_t)b * a.H * a.W;
    const uint16_t* xb = a.x + img * a.x_pitch + a.x_off + 8 * kq;
    int rowoff[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) rowoff[r] = (((y0 - 1 + r) % a.H + a.H) % a.H) * a.W;
    int xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int xx = x + d - 1;
        xs[d] = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
    }
    f32x4 acc[R][NT];
#pragma unroll
    for (int o = 0; o < R; ++o)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[o][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c = 0; c < CI; ++c) {
        __syncthreads();  // the previous slice's weights are no longer read
        // wt[tap][n][0..31] = w[n0 + n][tap * cin + 32 c + 0..31]
        for (int e = threadIdx.x; e < 9 * kN * 4; e += kConvBlock) {
            const int tap = e / (kN * 4), rem = e - tap * (kN * 4), n = rem >> 2, c8 = (rem & 3) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (n0 + n < a.cout_pad)
                v = *reinterpret_cast<const uint4*>(a.w + (size_t)(n0 + n) * a.k_pad + tap * kCin + 32 * c + c8);
            *reinterpret_cast<uint4*>(&wt[(tap * kN + n) * kRwRow + c8]) = v;
        }
        __syncthreads();
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            uint4 av[R + 2];
#pragma unroll
            for (int r = 0; r < R + 2; ++r)
                av[r] = *reinterpret_cast<const uint4*>(xb + (size_t)(rowoff[r] + xs[d]) * a.x_pitch + 32 * c);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const int tap = 3 * e + d;  // dy = e - 1
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const bf16x8 bw = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const uint4*>(&wt[(tap * kN + 16 * j + m) * kRwRow + 8 * kq]));
#pragma unroll
                    for (int o = 0; o < R; ++o)
                        acc[o][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw, __builtin_bit_cast(bf16x8, av[o + e]),
                                                                            acc[o][j], 0, 0, 0);
                }
            }
        }
    }
    // epilogue: lane holds D[4 kq + i][m]: output channels n0 + 16 j + 4 kq + i of pixel (y0 + o, x)
    float bias[NT][4];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = n0 + 16 * j + 4 * kq + i;
            bias[j][i] = (a.bias && n < a.cout) ? a.bias[n] : 0.f;
        }
#pragma unroll
    for (int o = 0; o < R; ++o) {
        if (y0 + o >= a.H) continue;
        const size_t q = img + (size_t)(y0 + o) * a.W + x;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int nb = n0 + 16 * j + 4 * kq;
            if (nb >= a.cout) continue;
            const bool full = a.y_vec && nb + 3 < a.cout;
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = acc[o][j][i] + bias[j][i];
                if (RELU) v[i] = fmaxf(v[i], 0.f);
            }
            if (OUT_F32) {
                float* yp = static_cast<float*>(a.y) + q * a.y_pitch + a.y_off + nb;
                if (full) {
                    *reinterpret_cast<float4*>(yp) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    for (int i = 0; i < 4; ++i)
                        if (nb + i < a.cout) yp[i] = v[i];
                }
            } else {
                uint16_t* yp = static_cast<uint16_t*>(a.y) + q * a.y_pitch + a.y_off + nb;
                if (full) {
                    if (ACC) {
                        const uint2 old = *reinterpret_cast<const uint2*>(yp);
                        v[0] += bf2f(uint16_t(old.x & 0xffffu));
                        v[1] += bf2f(uint16_t(old.x >> 16));
                        v[2] += bf2f(uint16_t(old.y & 0xffffu));
                        v[3] += bf2f(uint16_t(old.y >> 16));
                    }
                    *reinterpret_cast<uint2*>(yp) = make_uint2(uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16),
                                                               uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16));
                } else {
                    for (int i = 0; i < 4; ++i) {
                        if (nb + i >= a.cout) continue;
                        float t = v[i];
                        if (ACC) t += bf2f(yp[i]);
                        yp[i] = f2bf(t);
                    }
                }
            }
        }
    }
}

// -------------------------------------------------------------- flip weights --
__global__ void k_flip(const uint16_t* w, int cin, int cout, int k_pad_w, int cout_pad, uint16_t* wt, int k_pad_t,
                       int rows_t)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows_t * k_pad_t) return;
    const int ci = idx / k_pad_t, kt = idx - ci * k_pad_t;
    uint16_t v = 0;
    if (ci < cin && kt < 9 * cout_pad) {
        const int tapp = kt / cout_pad, co = kt - tapp * cout_pad;
        if (co < cout) v = w[(size_t)co * k_pad_w + (8 - tapp) * cin + ci];
    }
    wt[idx] = v;
}

// ---------------------------------------------------------- weight gradient --
// Workgroup: CT output channels x KT columns of K (CT KT = 4096; 64 x 64, or
// 32 x 128 and 16 x 128 for the layers with few output channels, so that the
// MFMAs do not multiply padding channels), reducing over a range of pixels
// 128 at a time.  dy and the shifted x are staged transposed in LDS
// ([channel][pixel]) so that each lane reads 8 consecutive pixels: a thread
// loads 8 channels (or K columns) of 4 pixels and writes each one's 4 values
// with one 8-byte store.  The four wavefronts sit WC x WK over the tile, each
// owning 16 MI channels x 32 K columns, and issue 8 MI MFMAs per staged chunk.
constexpr int kWgPix = 128;
constexpr int kBgradCh = 128;        // channel slots per split of the bias partials
constexpr int kWgMinSplit = 512;     // fewest pixels per split
constexpr int kWgTargetBlocks = 2048;  // workgroups the split count aims for
constexpr int kWtRow = kWgPix + 8;

// channel tile of the weight gradient for cout_pad output channels (K tile: 4096 / it, at most 128)
__host__ __device__ constexpr int wg_ct(int cout_pad) { return cout_pad <= 16 ? 16 : (cout_pad <= 32 ? 32 : 64); }
__host__ __device__ constexpr int wg_kt(int ct) { return ct == 64 ? 64 : 128; }

struct WgradArgs {
    const uint16_t* x;
    const uint16_t* dy;
    float* part;   // [nsplit][cout_pad16][kreal]
    float* bpart;  // [nsplit][kBgradCh] bias partials, or null
    int x_pitch, x_off, cin;
    int dy_pitch, dy_off, cout;
    int cout_pad, k_real;
    int H, W;
    long long npix;
    int nsplit;
    long long split_pix;  // pixels per split (a multiple of kWgPix)
    int kblocks, cblocks;  // K and channel blocks of the tile
};

// Workgroup order of the weight gradient: the hardware deals consecutive
// workgroups round-robin to the eight XCDs, each with its own L2.  Workgroup b
// takes logical index xcd_order(b): XCD x gets one contiguous run of logical
// indices, and the K blocks of one (split, channel block) are consecutive in
// it, so the workgroups that read the same dy rows and the same input rows run
// side by side on one XCD and share its L2.
__device__ __forceinline__ int xcd_order(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

template <int CT>
__global__ __launch_bounds__(kConvBlock) void k_conv_wgrad(WgradArgs a)
{
    constexpr int KT = wg_kt(CT);
    constexpr int WC = CT >= 32 ? CT / 32 : 1;  // wavefronts along channels
    constexpr int WK = 4 / WC;                   // and along K (32 columns each)
    constexpr int MI = CT / (16 * WC);           // 16-channel MFMA rows per wavefront
    constexpr int NX = KT / 64;                  // K-column groups each loader thread stages
    static_assert(WK * 32 == KT && MI >= 1 && MI <= 2, "weight-gradient tile");
    __shared__ __attribute__((aligned(16))) uint16_t dyt[CT * kWtRow];
    __shared__ __attribute__((aligned(16))) uint16_t xt[KT * kWtRow];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, kq = lane >> 4;
    const int L = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int kb = L % a.kblocks, rest = L / a.kblocks;
    const int k0 = kb * KT;                    // K columns
    const int c0 = (rest % a.cblocks) * CT;    // output channels
    const int split = rest / a.cblocks;
    const long long pbeg = (long long)split * a.split_pix;
    const long long pend = min(pbeg + a.split_pix, a.npix);
    // the blocks of the first K range also sum dy per channel: the bias gradient
    const bool bias = a.bpart && kb == 0;
    // bias partials: each loader thread sums its own pixels of its 8 channels over the
    // chunks (in chunk order); the 32 threads of a channel group are summed at the end
    double bsum[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int HW = a.H * a.W;
    // wave tile: channels c0 + wc .. + 16 MI, K columns k0 + wk .. + 32
    const int wc = 16 * MI * (wave / WK), wk = 32 * (wave % WK);
    f32x4 acc[MI][2];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // loader role: pixels 4 lp .. 4 lp + 3 of the chunk; 8-wide channel group lc
    // (threads with lc < CT / 8) and K-column groups lc + 8 h, h < NX.  lp runs
    // fastest, so that the 8-byte transposed LDS writes of a wavefront fill
    // consecutive slots of two rows (no bank conflicts beyond the minimum).
    const int lp = threadIdx.x & 31, lc = threadIdx.x >> 5;
    const bool dy_loader = lc < CT / 8;
    const int co = c0 + 8 * lc;
    int kk[NX], ci[NX], ty[NX], tx[NX];
#pragma unroll
    for (int h = 0; h < NX; ++h) {
        kk[h] = k0 + 8 * (lc + 8 * h);
        int tap = 0;
        ci[h] = 0;
        if (kk[h] < a.k_real) {
            tap = kk[h] / a.cin;
            ci[h] = kk[h] - tap * a.cin;
        }
        ty[h] = tap / 3 - 1;
        tx[h] = tap % 3 - 1;
    }
    // this loader's first pixel of the chunk and its image coordinates, advanced by
    // one chunk per iteration (W is a multiple of 64, so the four pixels 4 lp ..
    // 4 lp + 3 never straddle a row)
    int b, py, px;
    {
        const long long p0 = pbeg + 4 * lp;
        const long long pc = p0 < a.npix ? p0 : 0;
        b = int(pc / HW);
        const int rem = int(pc - (long long)b * HW);
        py = rem / a.W;
        px = rem - py * a.W;
    }
    for (long long pb = pbeg; pb < pend; pb += kWgPix) {
        uint4 dv[4], xv[NX][4];
        const long long p = pb + 4 * lp;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            dv[u] = make_uint4(0, 0, 0, 0);
            if (dy_loader && p + u < pend && co < a.cout) {
                const uint16_t* src = a.dy + (size_t)(p + u) * a.dy_pitch + a.dy_off + co;
                if (co + 8 <= a.cout) {
                    dv[u] = *reinterpret_cast<const uint4*>(src);
                } else {
                    // the last group of a channel count that is not a multiple of 8
                    const int nv = a.cout - co;
                    uint32_t w[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t lo = 2 * q < nv ? src[2 * q] : 0u, hi = 2 * q + 1 < nv ? src[2 * q + 1] : 0u;
                        w[q] = lo | (hi << 16);
                    }
                    dv[u] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NX; ++h) {
            int yy = py + ty[h];
            yy += yy < 0 ? a.H : (yy >= a.H ? -a.H : 0);
            const size_t row = (size_t)b * HW + (size_t)yy * a.W;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[h][u] = make_uint4(0, 0, 0, 0);
                if (p + u < pend && kk[h] < a.k_real) {
                    int xx = px + u + tx[h];
                    xx += xx < 0 ? a.W : (xx >= a.W ? -a.W : 0);
                    xv[h][u] = *reinterpret_cast<const uint4*>(a.x + (row + xx) * a.x_pitch + a.x_off + ci[h]);
                }
            }
        }
        px += kWgPix;
        while (px >= a.W) {
            px -= a.W;
            if (++py == a.H) {
                py = 0;
                ++b;
            }
        }
        __syncthreads();
        // transposed: row = channel (or K column), 4 consecutive pixels per 8-byte write
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (dy_loader) {
                const uint16_t* d0 = reinterpret_cast<const uint16_t*>(dv);
                const uint2 dq = make_uint2(uint32_t(d0[i]) | (uint32_t(d0[8 + i]) << 16),
                                            uint32_t(d0[16 + i]) | (uint32_t(d0[24 + i]) << 16));
                *reinterpret_cast<uint2*>(&dyt[(8 * lc + i) * kWtRow + 4 * lp]) = dq;
            }
#pragma unroll
            for (int h = 0; h < NX; ++h) {
                const uint16_t* x0 = reinterpret_cast<const uint16_t*>(xv[h]);
                const uint2 xq = make_uint2(uint32_t(x0[i]) | (uint32_t(x0[8 + i]) << 16),
                                            uint32_t(x0[16 + i]) | (uint32_t(x0[24 + i]) << 16));
                *reinterpret_cast<uint2*>(&xt[(8 * (lc + 8 * h) + i) * kWtRow + 4 * lp]) = xq;
            }
        }
        __syncthreads();
        if (bias && dy_loader) {
            const uint16_t* d0 = reinterpret_cast<const uint16_t*>(dv);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                bsum[i] += (double(bf2f(d0[i])) + double(bf2f(d0[8 + i]))) +
                           (double(bf2f(d0[16 + i])) + double(bf2f(d0[24 + i])));
        }
#pragma unroll
        for (int ks = 0; ks < kWgPix / 32; ++ks) {
#pragma unroll
            for (int i = 0; i < MI; ++i) {
                const uint4 av = *reinterpret_cast<const uint4*>(&dyt[(wc + 16 * i + m) * kWtRow + 32 * ks + 8 * kq]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint4 bv =
                        *reinterpret_cast<const uint4*>(&xt[(wk + 16 * j + m) * kWtRow + 32 * ks + 8 * kq]);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                         __builtin_bit_cast(bf16x8, bv), acc[i][j], 0,
                                                                         0, 0);
                }
            }
        }
    }
    if (bias) {
        // red[channel][lp] reuses the dy tile (CT x 32 doubles fit in CT x kWtRow bf16)
        double* red = reinterpret_cast<double*>(dyt);
        __syncthreads();  // every wavefront is done with the dy tile
        if (dy_loader) {
#pragma unroll
            for (int i = 0; i < 8; ++i) red[(8 * lc + i) * 32 + lp] = bsum[i];
        }
        __syncthreads();
        if (threadIdx.x < CT && c0 + threadIdx.x < a.cout) {
            double t = 0.0;
            for (int q = 0; q < 32; ++q) t += red[threadIdx.x * 32 + q];
            a.bpart[(size_t)split * kBgradCh + c0 + threadIdx.x] = float(t);
        }
    }
    // D[4 kq + r][m]: row = output channel, column = K column
    float* out = a.part + (size_t)split * a.cout_pad * a.k_real;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co2 = c0 + wc + 16 * i + 4 * kq + r;
                const int k2 = k0 + wk + 16 * j + m;
                if (co2 < a.cout_pad && k2 < a.k_real) out[(size_t)co2 * a.k_real + k2] = acc[i][j][r];
            }
}

// sum the split partials; dw[co][k] for co < cout.  A workgroup covers 32
// consecutive elements; its eight rows of 32 threads take every eighth split
// (row r: splits r, r + 8, ...), and the eight row sums are then added in row
// order: a fixed order for a given split count.
constexpr int kRedCols = 32, kRedRows = 8;
__global__ __launch_bounds__(kRedCols * kRedRows) void k_wgrad_reduce(const float* part, int nsplit, int cout,
                                                                      int cout_pad, int k_real, float* dw)
{
    __shared__ double red[kRedRows][kRedCols];
    const int j = threadIdx.x % kRedCols, r = threadIdx.x / kRedCols;
    const long long idx = (long long)blockIdx.x * kRedCols + j;
    const long long total = (long long)cout * k_real;
    const size_t stride = (size_t)cout_pad * k_real;
    double sd = 0.0;
    if (idx < total)
        for (int t = r; t < nsplit; t += kRedRows) sd += part[(size_t)t * stride + idx];
    red[r][j] = sd;
    __syncthreads();
    if (r == 0 && idx < total) {
        double t = red[0][j];
        for (int q = 1; q < kRedRows; ++q) t += red[q][j];
        dw[idx] = float(t);
    }
}

// bias gradient: the per-split channel sums written by k_conv_wgrad, reduced
// per channel by one workgroup in a fixed order (strided partial sums, then a
// tree)
__global__ __launch_bounds__(256) void k_bgrad_reduce(const float* part, int nsplit, float* db)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int t = threadIdx.x; t < nsplit; t += 256) s += part[(size_t)t * kBgradCh + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = float(red[0]);
}

// ----------------------------------------------------------- pooling / upsampling --
struct View {
    uint16_t* p;
    int pitch, off;
};

// y (H/2 x W/2) = mean of 2x2 blocks of x (H x W); channels c < C
// The pooling, upsampling and ReLU-mask kernels move 8 channels (16 bytes) per
// thread; channel counts, pitches and offsets are multiples of 8 throughout the
// network.
__device__ __forceinline__ void unpack8(const uint4& v, float (&f)[8])
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8])
{
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = uint32_t(f2bf(f[2 * i])) | (uint32_t(f2bf(f[2 * i + 1])) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ __forceinline__ uint4 ld8(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st8(uint16_t* p, const uint4& v) { *reinterpret_cast<uint4*>(p) = v; }

// y (H/2 x W/2) = mean of 2x2 blocks of x (H x W); channels c < C
__global__ void k_pool_fwd(const uint16_t* x, int xp, int xo, uint16_t* y, int yp, int yo, int C, int B, int H, int W)
{
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int H2 = H / 2, W2 = W / 2, C8 = C >> 3;
    const long long total = (long long)B * H2 * W2 * C8;
    if (idx >= total) return;
    const int c = int(idx % C8) * 8;
    const long long q = idx / C8;
    const int x2 = int(q % W2), y2 = int((q / W2) % H2), b = int(q / ((long long)W2 * H2));
    const size_t base = ((size_t)b * H + 2 * y2) * W + 2 * x2;
    float a[8], t[8];
    unpack8(ld8(x + base * xp + xo + c), a);
    unpack8(ld8(x + (base + 1) * xp + xo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += t[i];
    unpack8(ld8(x + (base + W) * xp + xo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += t[i];
    unpack8(ld8(x + (base + W + 1) * xp + xo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = 0.25f * (a[i] + t[i]);
    st8(y + (size_t)q * yp + yo + c, pack8(a));
}

// dx (H x W) (+)= dy (H/2 x W/2) / 4 broadcast
__global__ void k_pool_bwd(const uint16_t* dy, int yp, int yo, uint16_t* dx, int xp, int xo, int C, int B, int H, int W,
                           int acc)
{
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int C8 = C >> 3;
    const long long total = (long long)B * H * W * C8;
    if (idx >= total) return;
    const int c = int(idx % C8) * 8;
    const long long q = idx / C8;
    const int x = int(q % W), y = int((q / W) % H), b = int(q / ((long long)W * H));
    const size_t qs = ((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2;
    float v[8];
    unpack8(ld8(dy + qs * yp + yo + c), v);
    uint16_t* o = dx + (size_t)q * xp + xo + c;
    float t[8];
    if (acc) unpack8(ld8(o), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.25f * v[i] + (acc ? t[i] : 0.f);
    st8(o, pack8(v));
}

// y (2H x 2W) = nearest upsample of x (H x W)
__global__ void k_up_fwd(const uint16_t* x, int xp, int xo, uint16_t* y, int yp, int yo, int C, int B, int H, int W)
{
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int C8 = C >> 3;
    const long long total = (long long)B * 4 * H * W * C8;
    if (idx >= total) return;
    const int c = int(idx % C8) * 8;
    const long long q = idx / C8;
    const int X = int(q % (2 * W)), Y = int((q / (2 * W)) % (2 * H)), b = int(q / (4LL * W * H));
    const size_t qs = ((size_t)b * H + Y / 2) * W + X / 2;
    st8(y + (size_t)q * yp + yo + c, ld8(x + qs * xp + xo + c));
}

// dx (H x W) = sum of the 2x2 block of dy (2H x 2W)
__global__ void k_up_bwd(const uint16_t* dy, int yp, int yo, uint16_t* dx, int xp, int xo, int C, int B, int H, int W)
{
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int C8 = C >> 3;
    const long long total = (long long)B * H * W * C8;
    if (idx >= total) return;
    const int c = int(idx % C8) * 8;
    const long long q = idx / C8;
    const int x = int(q % W), y = int((q / W) % H), b = int(q / ((long long)W * H));
    const size_t base = ((size_t)b * 2 * H + 2 * y) * 2 * W + 2 * x;
    const size_t W2 = 2 * (size_t)W;
    float a[8], t[8];
    unpack8(ld8(dy + base * yp + yo + c), a);
    unpack8(ld8(dy + (base + 1) * yp + yo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += t[i];
    unpack8(ld8(dy + (base + W2) * yp + yo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += t[i];
    unpack8(ld8(dy + (base + W2 + 1) * yp + yo + c), t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] += t[i];
    st8(dx + (size_t)q * xp + xo + c, pack8(a));
}

// dy *= (y > 0), channel slice of each
__global__ void k_relu_mask(uint16_t* dy, int dp, int dof, const uint16_t* y, int yp, int yo, int C, long long npix)
{
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int C8 = C >> 3;
    if (idx >= npix * C8) return;
    const int c = int(idx % C8) * 8;
    const long long q = idx / C8;
    float yv[8], g[8];
    unpack8(ld8(y + (size_t)q * yp + yo + c), yv);
    uint16_t* o = dy + (size_t)q * dp + dof + c;
    const uint4 gv = ld8(o);
    unpack8(gv, g);
    uint32_t w[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!(yv[2 * i] > 0.f)) w[i] &= 0xffff0000u;
        if (!(yv[2 * i + 1] > 0.f)) w[i] &= 0x0000ffffu;
    }
    (void)g;
    st8(o, make_uint4(w[0], w[1], w[2], w[3]));
}

// masked MSE over channels 0..2: loss partials per block and dL/dout as bf16 [npix][16]
__global__ void k_mse(const float* out, const float* target, const uint8_t* mask, long long npix, double inv_count,
                      uint16_t* dout, double* part)
{
    __shared__ double red[256];
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double l = 0.0;
    if (q < npix) {
        const bool on = mask[q] != 0;
        for (int c = 0; c < 16; ++c) {
            float g = 0.f;
            if (c < 3 && on) {
                const float d = out[(size_t)q * 4 + c] - target[(size_t)q * 4 + c];
                l += double(d) * double(d);
                g = float(2.0 * d * inv_count);
            }
            dout[(size_t)q * 16 + c] = f2bf(g);
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam on a flat FP32 parameter array.  The decay rates and their complements
// are rounded to float separately: 1 - 0.999f would carry a relative error of
// 1.3e-5 into the second moment.
__global__ void k_adam(float* p, const float* g, float* m1, float* m2, long long n, float lr, float b1, float omb1,
                       float b2, float omb2, float c1, float c2, float eps)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + omb1 * gi;
    const float v = b2 * m2[i] + omb2 * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// FP32 master weights [cout][9 cin] (k = tap * cin + ci) -> bf16 [cout_pad][k_pad]
__global__ void k_pack_w(const float* wm, int cout, int kreal, int cout_pad, int k_pad, uint16_t* w)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cout_pad * k_pad) return;
    const int co = idx / k_pad, k = idx - co * k_pad;
    w[idx] = (co < cout && k < kreal) ? f2bf(wm[(size_t)co * kreal + k]) : uint16_t(0);
}

// He-normal initialisation from a counter-based generator (SplitMix64 + Box-Muller)
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
__global__ void k_init_w(float* w, long long n, float stdv, uint64_t seed, uint64_t stream)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t h1 = mix64(seed ^ mix64(stream * 2 + 0) ^ (uint64_t)i);
    const uint64_t h2 = mix64(seed ^ mix64(stream * 2 + 1) ^ (uint64_t)i);
    const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    w[i] = float(stdv * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

unsigned nblocks(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// per-class feature rows (8 floats) -> bf16 [n][8]
__global__ void k_features(const uint8_t* cls, long long n, const float* table, uint16_t* x)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* t = table + 8 * cls[i];
    uint16_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = f2bf(t[k]);
    uint4 o;
    memcpy(&o, v, 16);
    reinterpret_cast<uint4*>(x)[i] = o;
}

__global__ void k_targets(const double* rho, const double* u, const uint8_t* cls, long long n, double rs, double us,
                          float* target, uint8_t* mask)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fluid = cls[i] != 255;
    target[4 * i + 0] = fluid ? float((rho[i] - 1.0) / rs) : 0.f;
    target[4 * i + 1] = fluid ? float(u[i] / us) : 0.f;
    target[4 * i + 2] = fluid ? float(u[n + i] / us) : 0.f;
    target[4 * i + 3] = 0.f;
    mask[i] = fluid ? 1 : 0;
}

// Prediction -> fields for the equilibrium start: rho - 1 (not rho, which
// would round a deviation of 1e-6 to a few digits) and the velocity planes.
__global__ void k_apply(const float* y, long long n, double rs, double us, float* drho, float* u)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    drho[i] = float(rs * y[4 * i + 0]);
    u[i] = float(us * y[4 * i + 1]);
    u[n + i] = float(us * y[4 * i + 2]);
    u[2 * n + i] = 0.f;
}

// ------------------------------------------------------------ host helpers --
thread_local std::string g_cnn_err;
int cfail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    glbm::set_error(buf);
    return code;
}
#define CHK(expr)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return cfail(GLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

int conv_fwd(const uint16_t* x, int xp, int xo, int cin, const uint16_t* w, const float* bias, void* y, int yp, int yo,
             int cout, bool relu, bool yf32, bool acc, int B, int H, int W, hipStream_t s)
{
    if (cin <= 0 || cin % 8 || cout <= 0 || W % kPixTile || H <= 0 || B <= 0 || !x || !w || !y)
        return cfail(GLBM_EINVAL, "conv3x3: need cin % 8 == 0, W % 64 == 0, positive sizes");
    if (xo + cin > xp || yo + cout > yp) return cfail(GLBM_EINVAL, "conv3x3: channel slice exceeds pitch");
    if (yf32 && acc) return cfail(GLBM_EINVAL, "conv3x3: accumulate needs bf16 output");
    if (xp % 8 || xo % 8 || reinterpret_cast<uintptr_t>(x) % 16 || reinterpret_cast<uintptr_t>(w) % 16)
        return cfail(GLBM_EINVAL, "conv3x3: x and w must be 16-byte aligned, x_pitch and x_off multiples of 8");
    ConvArgs a{};
    a.x = x;
    a.w = w;
    a.bias = bias;
    a.y = y;
    a.x_pitch = xp;
    a.x_off = xo;
    a.cin = cin;
    a.y_pitch = yp;
    a.y_off = yo;
    a.cout = cout;
    a.k_real = 9 * cin;
    a.k_pad = rup(9 * cin, 32);
    a.cout_pad = rup(cout, 16);
    a.H = H;
    a.W = W;
    a.npix = (long long)B * H * W;
    a.y_vec = yp % 4 == 0 && yo % 4 == 0 && reinterpret_cast<uintptr_t>(y) % (yf32 ? 16 : 8) == 0;
    const unsigned gy = (unsigned)((a.cout_pad + kChTile - 1) / kChTile);
    const int ci32 = cin % 32 == 0 ? cin / 32 : 0;
    const bool row_path = ci32 == 1 || ci32 == 2 || ci32 == 3 || ci32 == 4 || ci32 == 6;
    if (row_path) {
        constexpr int R = 4;
        const int nt = a.cout_pad % 64 == 0 ? 4 : (a.cout_pad % 32 == 0 ? 2 : 1);
        dim3 grid((unsigned)((long long)B * ((H + R - 1) / R) * (W / 64)), (unsigned)(a.cout_pad / (16 * nt)));
#define LAUNCH_R(C, N, F, Re, A) hipLaunchKernelGGL((k_conv_fwd_rows<C, N, R, F, Re, A>), grid, dim3(kConvBlock), 0, s, a)
#define EPI_R(C, N)                                                                                    \
    do {                                                                                               \
        if (yf32) {                                                                                    \
            if (relu) LAUNCH_R(C, N, true, true, false);                                               \
            else LAUNCH_R(C, N, true, false, false);                                                   \
        } else if (acc) {                                                                              \
            if (relu) LAUNCH_R(C, N, false, true, true);                                               \
            else LAUNCH_R(C, N, false, false, true);                                                   \
        } else {                                                                                       \
            if (relu) LAUNCH_R(C, N, false, true, false);                                              \
            else LAUNCH_R(C, N, false, false, false);                                                  \
        }                                                                                              \
    } while (0)
#define NT_R(C)                                                                                        \
    do {                                                                                               \
        if (nt == 4) EPI_R(C, 4);                                                                      \
        else if (nt == 2) EPI_R(C, 2);                                                                 \
        else EPI_R(C, 1);                                                                              \
    } while (0)
        if (ci32 == 1) NT_R(1);
        else if (ci32 == 2) NT_R(2);
        else if (ci32 == 3) NT_R(3);
        else if (ci32 == 4) NT_R(4);
        else NT_R(6);
#undef NT_R
#undef EPI_R
#undef LAUNCH_R
    } else {
        dim3 grid((unsigned)(a.npix / kPixTile), gy);
#define LAUNCH(F, R, A) hipLaunchKernelGGL((k_conv_fwd<F, R, A>), grid, dim3(kConvBlock), 0, s, a)
        if (yf32) {
            if (relu) LAUNCH(true, true, false);
            else LAUNCH(true, false, false);
        } else if (acc) {
            if (relu) LAUNCH(false, true, true);
            else LAUNCH(false, false, true);
        } else {
            if (relu) LAUNCH(false, true, false);
            else LAUNCH(false, false, false);
        }
#undef LAUNCH
    }
    CHK(hipGetLastError());
    return GLBM_OK;
}

int flip_weights(const uint16_t* w, int cin, int cout, uint16_t* wt, hipStream_t s)
{
    const int cout_pad = rup(cout, 16);
    const int rows_t = rup(cin, 16);
    const int k_pad_t = rup(9 * cout_pad, 32);
    hipLaunchKernelGGL(k_flip, dim3(nblocks((long long)rows_t * k_pad_t)), dim3(256), 0, s, w, cin, cout,
                       rup(9 * cin, 32), cout_pad, wt, k_pad_t, rows_t);
    CHK(hipGetLastError());
    return GLBM_OK;
}

// Split of the pixel range of a weight gradient: enough splits for about
// kWgTargetBlocks workgroups, none shorter than kWgMinSplit pixels.  Depends
// only on the shapes, so the reduction order (and the result) is fixed.
void wgrad_split(int cin, int cout, long long npix, int* nsplit, long long* split_pix)
{
    const int ct = wg_ct(rup(cout, 16)), kt = wg_kt(ct);
    const long long blocks = (long long)((9 * cin + kt - 1) / kt) * ((rup(cout, 16) + ct - 1) / ct);
    long long ns = std::max(1LL, std::min((npix + kWgMinSplit - 1) / kWgMinSplit,
                                          (kWgTargetBlocks + blocks - 1) / blocks));
    long long sp = (npix + ns - 1) / ns;
    sp = (sp + kWgPix - 1) / kWgPix * kWgPix;
    *split_pix = sp;
    *nsplit = (int)((npix + sp - 1) / sp);
}

size_t wgrad_workspace(int cin, int cout, long long npix)
{
    int ns;
    long long sp;
    wgrad_split(cin, cout, npix, &ns, &sp);
    return (size_t)ns * rup(cout, 16) * 9 * cin * sizeof(float) + (size_t)ns * kBgradCh * sizeof(float) + 256;
}

int conv_wgrad(const uint16_t* x, int xp, int xo, int cin, const uint16_t* dy, int dp, int dof, int cout, float* dw,
               float* db, void* ws, int B, int H, int W, hipStream_t s)
{
    if (cin <= 0 || cin % 8 || cout <= 0 || cout > 128 || !x || !dy || !dw || !ws)
        return cfail(GLBM_EINVAL, "conv3x3 weight gradient: need cin % 8 == 0, 0 < cout <= 128");
    WgradArgs a{};
    a.x = x;
    a.dy = dy;
    a.x_pitch = xp;
    a.x_off = xo;
    a.cin = cin;
    a.dy_pitch = dp;
    a.dy_off = dof;
    a.cout = cout;
    a.cout_pad = rup(cout, 16);
    a.k_real = 9 * cin;
    a.H = H;
    a.W = W;
    a.npix = (long long)B * H * W;
    wgrad_split(cin, cout, a.npix, &a.nsplit, &a.split_pix);
    a.part = static_cast<float*>(ws);
    a.bpart = db ? a.part + (size_t)a.nsplit * a.cout_pad * a.k_real : nullptr;
    const int ct = wg_ct(a.cout_pad), kt = wg_kt(ct);
    a.kblocks = (a.k_real + kt - 1) / kt;
    a.cblocks = (a.cout_pad + ct - 1) / ct;
    dim3 grid((unsigned)(a.kblocks * a.cblocks * a.nsplit));
    if (ct == 16)
        hipLaunchKernelGGL(k_conv_wgrad<16>, grid, dim3(kConvBlock), 0, s, a);
    else if (ct == 32)
        hipLaunchKernelGGL(k_conv_wgrad<32>, grid, dim3(kConvBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_conv_wgrad<64>, grid, dim3(kConvBlock), 0, s, a);
    CHK(hipGetLastError());
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)(((long long)cout * a.k_real + kRedCols - 1) / kRedCols)),
                       dim3(kRedCols * kRedRows), 0, s, a.part, a.nsplit, cout, a.cout_pad, a.k_real, dw);
    CHK(hipGetLastError());
    if (db) {
        hipLaunchKernelGGL(k_bgrad_reduce, dim3(cout), dim3(256), 0, s, a.bpart, a.nsplit, db);
        CHK(hipGetLastError());
    }
    return GLBM_OK;
}

}  // namespace

namespace glbm {
hipError_t launch_cnn_features(const uint8_t* cls, long long n, const float* table, uint16_t* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3(nblocks(n)), dim3(256), 0, s, cls, n, table, x);
    return hipGetLastError();
}
hipError_t launch_cnn_targets(const double* rho, const double* u, const uint8_t* cls, long long n, double rs, double us,
                              float* target, uint8_t* mask, hipStream_t s)
{
    hipLaunchKernelGGL(k_targets, dim3(nblocks(n)), dim3(256), 0, s, rho, u, cls, n, rs, us, target, mask);
    return hipGetLastError();
}
hipError_t launch_cnn_apply(const float* y, long long n, double rs, double us, float* drho, float* u, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply, dim3(nblocks(n)), dim3(256), 0, s, y, n, rs, us, drho, u);
    return hipGetLastError();
}
}  // namespace glbm

// ===================================================================== network
namespace {

struct Layer {
    int cin, cout;
    bool relu;
    int level;          // 0: H x W, 1: H/2, 2: H/4
    size_t wofs, bofs;  // offsets in the flat FP32 parameter array (device order)
    uint16_t* w = nullptr;   // bf16 [cout_pad][k_pad]
    uint16_t* wt = nullptr;  // flipped for the data gradient
};

}  // namespace

struct glbm_cnn_s {
    int maxb = 0, H = 0, W = 0;
    hipStream_t s = nullptr;
    std::vector<Layer> L;
    long long nparam = 0;
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    long long step = 0;
    // activations (bf16) and their gradients
    uint16_t *a0 = nullptr, *c1 = nullptr, *p1 = nullptr, *a2 = nullptr, *c2 = nullptr, *p2 = nullptr;
    uint16_t *a4 = nullptr, *e3 = nullptr, *a6 = nullptr, *d2 = nullptr, *a8 = nullptr;
    uint16_t *g_a0 = nullptr, *g_c1 = nullptr, *g_p1 = nullptr, *g_a2 = nullptr, *g_c2 = nullptr, *g_p2 = nullptr;
    uint16_t *g_a4 = nullptr, *g_e3 = nullptr, *g_a6 = nullptr, *g_d2 = nullptr, *g_a8 = nullptr, *g_out = nullptr;
    float* out = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    double* lpart = nullptr;
    std::vector<void*> owned;
};

namespace {

// layer table: (cin, cout, relu, level)
const int kSpec[10][4] = {{8, 32, 1, 0},   {32, 32, 1, 0},  {32, 64, 1, 1}, {64, 64, 1, 1}, {64, 128, 1, 2},
                          {128, 128, 1, 2}, {192, 64, 1, 1}, {64, 64, 1, 1}, {96, 32, 1, 0}, {32, 3, 0, 0}};

int alloc(glbm_cnn c, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return cfail(e == hipErrorOutOfMemory ? GLBM_ENOMEM : GLBM_EDEVICE, "hipMalloc(%zu): %s",
                                      bytes, hipGetErrorString(e));
    c->owned.push_back(*p);
    return GLBM_OK;
}

int pack_all(glbm_cnn c)
{
    for (auto& l : c->L) {
        const int kreal = 9 * l.cin, cpad = rup(l.cout, 16), kpad = rup(kreal, 32);
        hipLaunchKernelGGL(k_pack_w, dim3(nblocks((long long)cpad * kpad)), dim3(256), 0, c->s, c->p + l.wofs, l.cout,
                           kreal, cpad, kpad, l.w);
        CHK(hipGetLastError());
        int rc = flip_weights(l.w, l.cin, l.cout, l.wt, c->s);
        if (rc) return rc;
    }
    return GLBM_OK;
}

int forward(glbm_cnn c, const uint16_t* x, int B)
{
    const int H = c->H, W = c->W, H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4;
    auto& L = c->L;
    hipStream_t s = c->s;
    int rc;
#define CV(li, X, XP, XO, Y, YP, YO, h, w_)                                                                     \
    rc = conv_fwd(X, XP, XO, L[li].cin, L[li].w, c->p + L[li].bofs, Y, YP, YO, L[li].cout, L[li].relu, false, false, \
                  B, h, w_, s);                                                                                 \
    if (rc) return rc;
    CV(0, x, 8, 0, c->a0, 32, 0, H, W);
    CV(1, c->a0, 32, 0, c->c1, 96, 0, H, W);  // e1 -> c1[0:32]
    hipLaunchKernelGGL(k_pool_fwd, dim3(nblocks((long long)B * H1 * W1 * 32 / 8)), dim3(256), 0, s, c->c1, 96, 0, c->p1, 32,
                       0, 32, B, H, W);
    CV(2, c->p1, 32, 0, c->a2, 64, 0, H1, W1);
    CV(3, c->a2, 64, 0, c->c2, 192, 0, H1, W1);  // e2 -> c2[0:64]
    hipLaunchKernelGGL(k_pool_fwd, dim3(nblocks((long long)B * H2 * W2 * 64 / 8)), dim3(256), 0, s, c->c2, 192, 0, c->p2, 64,
                       0, 64, B, H1, W1);
    CV(4, c->p2, 64, 0, c->a4, 128, 0, H2, W2);
    CV(5, c->a4, 128, 0, c->e3, 128, 0, H2, W2);
    hipLaunchKernelGGL(k_up_fwd, dim3(nblocks((long long)B * 4 * H2 * W2 * 128 / 8)), dim3(256), 0, s, c->e3, 128, 0, c->c2,
                       192, 64, 128, B, H2, W2);
    CV(6, c->c2, 192, 0, c->a6, 64, 0, H1, W1);
    CV(7, c->a6, 64, 0, c->d2, 64, 0, H1, W1);
    hipLaunchKernelGGL(k_up_fwd, dim3(nblocks((long long)B * 4 * H1 * W1 * 64 / 8)), dim3(256), 0, s, c->d2, 64, 0, c->c1, 96,
                       32, 64, B, H1, W1);
    CV(8, c->c1, 96, 0, c->a8, 32, 0, H, W);
#undef CV
    rc = conv_fwd(c->a8, 32, 0, 32, L[9].w, c->p + L[9].bofs, c->out, 4, 0, 3, false, true, false, B, H, W, s);
    if (rc) return rc;
    CHK(hipGetLastError());
    return GLBM_OK;
}

// data gradient of layer li: dx (slice) = conv(dy, wt); dy has cout_pad channels
int bwd_data(glbm_cnn c, int li, const uint16_t* dy, int dyp, uint16_t* dx, int dxp, int dxo, bool acc, int B, int h,
             int w)
{
    const Layer& l = c->L[li];
    return conv_fwd(dy, dyp, 0, rup(l.cout, 16), l.wt, nullptr, dx, dxp, dxo, l.cin, false, false, acc, B, h, w, c->s);
}

int bwd_weight(glbm_cnn c, int li, const uint16_t* x, int xp, int xo, const uint16_t* dy, int dyp, int B, int h, int w)
{
    const Layer& l = c->L[li];
    return conv_wgrad(x, xp, xo, l.cin, dy, dyp, 0, l.cout, c->g + l.wofs, c->g + l.bofs, c->ws, B, h, w, c->s);
}

int relu_mask(glbm_cnn c, uint16_t* dy, int dp, int dof, const uint16_t* y, int yp, int yo, int C, long long npix)
{
    if ((C | dp | dof | yp | yo) & 7) return cfail(GLBM_EINVAL, "relu mask: channels, pitches and offsets must be multiples of 8");
    hipLaunchKernelGGL(k_relu_mask, dim3(nblocks(npix * C / 8)), dim3(256), 0, c->s, dy, dp, dof, y, yp, yo, C, npix);
    CHK(hipGetLastError());
    return GLBM_OK;
}

int backward(glbm_cnn c, const uint16_t* x, const float* target, const uint8_t* mask, int B, double* loss)
{
    const int H = c->H, W = c->W, H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4;
    const long long n0 = (long long)B * H * W, n1 = (long long)B * H1 * W1, n2 = (long long)B * H2 * W2;
    hipStream_t s = c->s;
    int rc = forward(c, x, B);
    if (rc) return rc;
    // count of masked nodes (host): the loss is a mean over fluid nodes and 3 channels
    std::vector<uint8_t> hm((size_t)n0);
    CHK(hipMemcpyAsync(hm.data(), mask, (size_t)n0, hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    long long cnt = 0;
    for (uint8_t v : hm) cnt += v != 0;
    if (cnt == 0) return cfail(GLBM_EINVAL, "mask selects no node");
    const double inv = 1.0 / (3.0 * (double)cnt);
    const unsigned nb = nblocks(n0);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, c->out, target, mask, n0, inv, c->g_out, c->lpart);
    CHK(hipGetLastError());
    std::vector<double> lp(nb);
    CHK(hipMemcpyAsync(lp.data(), c->lpart, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    // layer 9 (no ReLU)
    if ((rc = bwd_weight(c, 9, c->a8, 32, 0, c->g_out, 16, B, H, W))) return rc;
    if ((rc = bwd_data(c, 9, c->g_out, 16, c->g_a8, 32, 0, false, B, H, W))) return rc;
    // layer 8: input c1 (96), output a8
    if ((rc = relu_mask(c, c->g_a8, 32, 0, c->a8, 32, 0, 32, n0))) return rc;
    if ((rc = bwd_weight(c, 8, c->c1, 96, 0, c->g_a8, 32, B, H, W))) return rc;
    if ((rc = bwd_data(c, 8, c->g_a8, 32, c->g_c1, 96, 0, false, B, H, W))) return rc;
    // up(d2) -> c1[32:96]
    hipLaunchKernelGGL(k_up_bwd, dim3(nblocks(n1 * 64 / 8)), dim3(256), 0, s, c->g_c1, 96, 32, c->g_d2, 64, 0, 64, B, H1, W1);
    CHK(hipGetLastError());
    // layer 7: a6 -> d2
    if ((rc = relu_mask(c, c->g_d2, 64, 0, c->d2, 64, 0, 64, n1))) return rc;
    if ((rc = bwd_weight(c, 7, c->a6, 64, 0, c->g_d2, 64, B, H1, W1))) return rc;
    if ((rc = bwd_data(c, 7, c->g_d2, 64, c->g_a6, 64, 0, false, B, H1, W1))) return rc;
    // layer 6: c2 (192) -> a6
    if ((rc = relu_mask(c, c->g_a6, 64, 0, c->a6, 64, 0, 64, n1))) return rc;
    if ((rc = bwd_weight(c, 6, c->c2, 192, 0, c->g_a6, 64, B, H1, W1))) return rc;
    if ((rc = bwd_data(c, 6, c->g_a6, 64, c->g_c2, 192, 0, false, B, H1, W1))) return rc;
    // up(e3) -> c2[64:192]
    hipLaunchKernelGGL(k_up_bwd, dim3(nblocks(n2 * 128 / 8)), dim3(256), 0, s, c->g_c2, 192, 64, c->g_e3, 128, 0, 128, B, H2,
                       W2);
    CHK(hipGetLastError());
    // layer 5: a4 -> e3
    if ((rc = relu_mask(c, c->g_e3, 128, 0, c->e3, 128, 0, 128, n2))) return rc;
    if ((rc = bwd_weight(c, 5, c->a4, 128, 0, c->g_e3, 128, B, H2, W2))) return rc;
    if ((rc = bwd_data(c, 5, c->g_e3, 128, c->g_a4, 128, 0, false, B, H2, W2))) return rc;
    // layer 4: p2 -> a4
    if ((rc = relu_mask(c, c->g_a4, 128, 0, c->a4, 128, 0, 128, n2))) return rc;
    if ((rc = bwd_weight(c, 4, c->p2, 64, 0, c->g_a4, 128, B, H2, W2))) return rc;
    if ((rc = bwd_data(c, 4, c->g_a4, 128, c->g_p2, 64, 0, false, B, H2, W2))) return rc;
    // pool(e2): add into c2[0:64] gradient
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblocks(n1 * 64 / 8)), dim3(256), 0, s, c->g_p2, 64, 0, c->g_c2, 192, 0, 64, B, H1, W1,
                       1);
    CHK(hipGetLastError());
    // layer 3: a2 -> e2 (c2[0:64])
    if ((rc = relu_mask(c, c->g_c2, 192, 0, c->c2, 192, 0, 64, n1))) return rc;
    if ((rc = bwd_weight(c, 3, c->a2, 64, 0, c->g_c2, 192, B, H1, W1))) return rc;
    if ((rc = bwd_data(c, 3, c->g_c2, 192, c->g_a2, 64, 0, false, B, H1, W1))) return rc;
    // layer 2: p1 -> a2
    if ((rc = relu_mask(c, c->g_a2, 64, 0, c->a2, 64, 0, 64, n1))) return rc;
    if ((rc = bwd_weight(c, 2, c->p1, 32, 0, c->g_a2, 64, B, H1, W1))) return rc;
    if ((rc = bwd_data(c, 2, c->g_a2, 64, c->g_p1, 32, 0, false, B, H1, W1))) return rc;
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblocks(n0 * 32 / 8)), dim3(256), 0, s, c->g_p1, 32, 0, c->g_c1, 96, 0, 32, B, H, W, 1);
    CHK(hipGetLastError());
    // layer 1: a0 -> e1 (c1[0:32])
    if ((rc = relu_mask(c, c->g_c1, 96, 0, c->c1, 96, 0, 32, n0))) return rc;
    if ((rc = bwd_weight(c, 1, c->a0, 32, 0, c->g_c1, 96, B, H, W))) return rc;
    if ((rc = bwd_data(c, 1, c->g_c1, 96, c->g_a0, 32, 0, false, B, H, W))) return rc;
    // layer 0: x -> a0
    if ((rc = relu_mask(c, c->g_a0, 32, 0, c->a0, 32, 0, 32, n0))) return rc;
    if ((rc = bwd_weight(c, 0, x, 8, 0, c->g_a0, 32, B, H, W))) return rc;
    CHK(hipStreamSynchronize(s));
    double l = 0.0;
    for (double v : lp) l += v;
    if (loss) *loss = l * inv;
    return GLBM_OK;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

int glbm_conv3x3_forward(const uint16_t* x, int32_t x_pitch, int32_t x_off, int32_t cin, const uint16_t* w,
                         const float* bias, void* y, int32_t y_pitch, int32_t y_off, int32_t cout, int32_t relu,
                         int32_t y_is_f32, int32_t accumulate, int32_t batch, int32_t height, int32_t width,
                         void* hip_stream)
{
    return conv_fwd(x, x_pitch, x_off, cin, w, bias, y, y_pitch, y_off, cout, relu != 0, y_is_f32 != 0,
                    accumulate != 0, batch, height, width, static_cast<hipStream_t>(hip_stream));
}

int glbm_conv3x3_flip_weights(const uint16_t* w, int32_t cin, int32_t cout, uint16_t* wt, void* hip_stream)
{
    if (!w || !wt || cin <= 0 || cout <= 0) return cfail(GLBM_EINVAL, "flip: bad arguments");
    return flip_weights(w, cin, cout, wt, static_cast<hipStream_t>(hip_stream));
}

size_t glbm_conv3x3_wgrad_workspace(int32_t cin, int32_t cout, int32_t batch, int32_t height, int32_t width)
{
    return wgrad_workspace(cin, cout, (long long)batch * height * width);
}

int glbm_conv3x3_backward_weight(const uint16_t* x, int32_t x_pitch, int32_t x_off, int32_t cin, const uint16_t* dy,
                                 int32_t dy_pitch, int32_t dy_off, int32_t cout, float* dw, float* db,
                                 void* workspace, int32_t batch, int32_t height, int32_t width, void* hip_stream)
{
    return conv_wgrad(x, x_pitch, x_off, cin, dy, dy_pitch, dy_off, cout, dw, db, workspace, batch, height, width,
                      static_cast<hipStream_t>(hip_stream));
}

int glbm_cnn_create(glbm_cnn* out, int32_t max_batch, int32_t height, int32_t width, uint64_t seed, void* hip_stream)
{
    if (!out) return cfail(GLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || height < 256 || width < 256 || height % 256 || width % 256)
        return cfail(GLBM_EINVAL, "cnn: need max_batch >= 1 and H, W multiples of 256");
    glbm_cnn c = new (std::nothrow) glbm_cnn_s();
    if (!c) return cfail(GLBM_ENOMEM, "host allocation");
    c->maxb = max_batch;
    c->H = height;
    c->W = width;
    c->s = static_cast<hipStream_t>(hip_stream);
    long long off = 0;
    for (int i = 0; i < 10; ++i) {
        Layer l;
        l.cin = kSpec[i][0];
        l.cout = kSpec[i][1];
        l.relu = kSpec[i][2] != 0;
        l.level = kSpec[i][3];
        l.wofs = (size_t)off;
        off += (long long)l.cout * 9 * l.cin;
        l.bofs = (size_t)off;
        off += l.cout;
        c->L.push_back(l);
    }
    c->nparam = off;
    auto fail_out = [&](int rc) {
        glbm_cnn_destroy(c);
        return rc;
    };
    int rc;
    for (float** p : {&c->p, &c->g, &c->m1, &c->m2})
        if ((rc = alloc(c, reinterpret_cast<void**>(p), (size_t)off * sizeof(float)))) return fail_out(rc);
    for (auto& l : c->L) {
        const size_t wb = (size_t)rup(l.cout, 16) * rup(9 * l.cin, 32) * 2;
        const size_t tb = (size_t)rup(l.cin, 16) * rup(9 * rup(l.cout, 16), 32) * 2;
        if ((rc = alloc(c, reinterpret_cast<void**>(&l.w), wb))) return fail_out(rc);
        if ((rc = alloc(c, reinterpret_cast<void**>(&l.wt), tb))) return fail_out(rc);
    }
    const size_t B = (size_t)max_batch, n0 = B * height * width, n1 = n0 / 4, n2 = n0 / 16;
    struct A {
        uint16_t** p;
        size_t n;
    } acts[] = {{&c->a0, n0 * 32}, {&c->c1, n0 * 96},  {&c->p1, n1 * 32},   {&c->a2, n1 * 64},   {&c->c2, n1 * 192},
                {&c->p2, n2 * 64}, {&c->a4, n2 * 128}, {&c->e3, n2 * 128},  {&c->a6, n1 * 64},   {&c->d2, n1 * 64},
                {&c->a8, n0 * 32}, {&c->g_a0, n0 * 32}, {&c->g_c1, n0 * 96}, {&c->g_p1, n1 * 32}, {&c->g_a2, n1 * 64},
                {&c->g_c2, n1 * 192}, {&c->g_p2, n2 * 64}, {&c->g_a4, n2 * 128}, {&c->g_e3, n2 * 128},
                {&c->g_a6, n1 * 64}, {&c->g_d2, n1 * 64}, {&c->g_a8, n0 * 32}, {&c->g_out, n0 * 16}};
    for (auto& a : acts)
        if ((rc = alloc(c, reinterpret_cast<void**>(a.p), a.n * 2))) return fail_out(rc);
    if ((rc = alloc(c, reinterpret_cast<void**>(&c->out), n0 * 4 * sizeof(float)))) return fail_out(rc);
    if ((rc = alloc(c, reinterpret_cast<void**>(&c->lpart), (size_t)nblocks((long long)n0) * sizeof(double))))
        return fail_out(rc);
    size_t ws = 0;
    for (auto& l : c->L) {
        const int lvl = l.level;
        ws = std::max(ws, wgrad_workspace(l.cin, l.cout, (long long)(n0 >> (2 * lvl))));
    }
    c->ws_bytes = ws;
    if ((rc = alloc(c, &c->ws, ws))) return fail_out(rc);
    // He-normal weights, zero biases and moments
    if (hipMemsetAsync(c->out, 0, n0 * 4 * sizeof(float), c->s) != hipSuccess ||
        hipMemsetAsync(c->p, 0, (size_t)off * 4, c->s) != hipSuccess ||
        hipMemsetAsync(c->m1, 0, (size_t)off * 4, c->s) != hipSuccess ||
        hipMemsetAsync(c->m2, 0, (size_t)off * 4, c->s) != hipSuccess ||
        hipMemsetAsync(c->g, 0, (size_t)off * 4, c->s) != hipSuccess)
        return fail_out(cfail(GLBM_EDEVICE, "memset"));
    for (int i = 0; i < 10; ++i) {
        const Layer& l = c->L[i];
        const long long n = (long long)l.cout * 9 * l.cin;
        hipLaunchKernelGGL(k_init_w, dim3(nblocks(n)), dim3(256), 0, c->s, c->p + l.wofs, n,
                           (float)std::sqrt(2.0 / (9.0 * l.cin)), seed, (uint64_t)i);
    }
    if ((rc = pack_all(c))) return fail_out(rc);
    if (hipStreamSynchronize(c->s) != hipSuccess) return fail_out(cfail(GLBM_EDEVICE, "synchronize"));
    *out = c;
    return GLBM_OK;
}

int glbm_cnn_destroy(glbm_cnn c)
{
    if (!c) return GLBM_OK;
    if (c->s) (void)hipStreamSynchronize(c->s);
    else (void)hipDeviceSynchronize();
    for (void* p : c->owned) (void)hipFree(p);
    delete c;
    return GLBM_OK;
}

int64_t glbm_cnn_num_params(glbm_cnn c) { return c ? c->nparam : 0; }

// device order per layer: w[co][tap][ci], b[co]; host order: w[co][ci][tap], b[co]
static void to_host_order(const glbm_cnn c, const std::vector<float>& dev, float* host)
{
    for (const auto& l : c->L) {
        for (int co = 0; co < l.cout; ++co)
            for (int ci = 0; ci < l.cin; ++ci)
                for (int t = 0; t < 9; ++t)
                    host[l.wofs + ((size_t)co * l.cin + ci) * 9 + t] = dev[l.wofs + ((size_t)co * 9 + t) * l.cin + ci];
        for (int co = 0; co < l.cout; ++co) host[l.bofs + co] = dev[l.bofs + co];
    }
}

int glbm_cnn_get_params(glbm_cnn c, float* host)
{
    if (!c || !host) return cfail(GLBM_EINVAL, "null argument");
    std::vector<float> d((size_t)c->nparam);
    CHK(hipMemcpyAsync(d.data(), c->p, d.size() * 4, hipMemcpyDeviceToHost, c->s));
    CHK(hipStreamSynchronize(c->s));
    to_host_order(c, d, host);
    return GLBM_OK;
}

int glbm_cnn_get_grads(glbm_cnn c, float* host)
{
    if (!c || !host) return cfail(GLBM_EINVAL, "null argument");
    std::vector<float> d((size_t)c->nparam);
    CHK(hipMemcpyAsync(d.data(), c->g, d.size() * 4, hipMemcpyDeviceToHost, c->s));
    CHK(hipStreamSynchronize(c->s));
    to_host_order(c, d, host);
    return GLBM_OK;
}

static void to_device_order(const glbm_cnn c, const float* host, std::vector<float>& dev)
{
    dev.assign((size_t)c->nparam, 0.f);
    for (const auto& l : c->L) {
        for (int co = 0; co < l.cout; ++co)
            for (int ci = 0; ci < l.cin; ++ci)
                for (int t = 0; t < 9; ++t)
                    dev[l.wofs + ((size_t)co * 9 + t) * l.cin + ci] = host[l.wofs + ((size_t)co * l.cin + ci) * 9 + t];
        for (int co = 0; co < l.cout; ++co) dev[l.bofs + co] = host[l.bofs + co];
    }
}

int glbm_cnn_set_params(glbm_cnn c, const float* host)
{
    if (!c || !host) return cfail(GLBM_EINVAL, "null argument");
    std::vector<float> d;
    to_device_order(c, host, d);
    CHK(hipMemcpyAsync(c->p, d.data(), d.size() * 4, hipMemcpyHostToDevice, c->s));
    int rc = pack_all(c);
    if (rc) return rc;
    CHK(hipStreamSynchronize(c->s));
    return GLBM_OK;
}

int glbm_cnn_set_grads(glbm_cnn c, const float* host)
{
    if (!c || !host) return cfail(GLBM_EINVAL, "null argument");
    std::vector<float> d;
    to_device_order(c, host, d);
    CHK(hipMemcpyAsync(c->g, d.data(), d.size() * 4, hipMemcpyHostToDevice, c->s));
    CHK(hipStreamSynchronize(c->s));
    return GLBM_OK;
}

int glbm_cnn_adam_step(glbm_cnn c, float lr)
{
    if (!c) return cfail(GLBM_EINVAL, "null argument");
    if (!(lr > 0.f) || !std::isfinite(lr)) return cfail(GLBM_EINVAL, "learning rate must be finite and > 0");
    c->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    // bias corrections 1 - beta^t evaluated in double, then rounded once
    const float c1 = (float)(1.0 - std::pow(b1, (double)c->step));
    const float c2 = (float)(1.0 - std::pow(b2, (double)c->step));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(c->nparam)), dim3(256), 0, c->s, c->p, c->g, c->m1, c->m2, c->nparam, lr,
                       (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), c1, c2, 1e-8f);
    CHK(hipGetLastError());
    return pack_all(c);
}

int glbm_cnn_forward(glbm_cnn c, const uint16_t* x, float* y, int32_t batch)
{
    if (!c || !x || !y) return cfail(GLBM_EINVAL, "null argument");
    if (batch < 1 || batch > c->maxb) return cfail(GLBM_EINVAL, "batch %d outside [1, %d]", batch, c->maxb);
    int rc = forward(c, x, batch);
    if (rc) return rc;
    CHK(hipMemcpyAsync(y, c->out, (size_t)batch * c->H * c->W * 4 * sizeof(float), hipMemcpyDeviceToDevice, c->s));
    return GLBM_OK;
}

int glbm_cnn_backward(glbm_cnn c, const uint16_t* x, const float* target, const uint8_t* mask, int32_t batch,
                      double* loss)
{
    if (!c || !x || !target || !mask) return cfail(GLBM_EINVAL, "null argument");
    if (batch < 1 || batch > c->maxb) return cfail(GLBM_EINVAL, "batch %d outside [1, %d]", batch, c->maxb);
    return backward(c, x, target, mask, batch, loss);
}

int glbm_cnn_train_step(glbm_cnn c, const uint16_t* x, const float* target, const uint8_t* mask, int32_t batch,
                        float lr, double* loss)
{
    int rc = glbm_cnn_backward(c, x, target, mask, batch, loss);
    if (rc) return rc;
    return glbm_cnn_adam_step(c, lr);
}

}  // extern "C"
