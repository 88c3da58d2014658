// Warm-start network for the SR solver on gfx950: BF16 activations and
// weights, FP32 accumulation on the matrix cores, FP32 gradients / master
// weights / Adam moments, and the host runtime behind include/cnn.h.
//
// Every 3x3 convolution (forward and data gradient) is one implicit GEMM:
// rows = pixels (16 per MFMA tile), columns = output channels, reduction
// k = tap*cin + ci over the 9 taps of the zero-padded stencil.  Activations
// are channels-last, so the four k values a lane feeds to
// v_mfma_f32_16x16x16_bf16 are four consecutive channels of one pixel: one
// 8-byte load.  The data gradient of a 3x3 convolution is the same kernel
// run on the masked output gradient with the weights turned by 180 degrees
// and input/output channels swapped.  The weight gradient reduces over
// pixels, so both operands are staged through LDS transposed (pixels
// contiguous) in 64-pixel chunks; each block owns a pixel slab and writes
// its partial tile, and a second pass sums the slabs in a fixed order
// (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/cnn.h"
#include "../../include/sr.h"

namespace cnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16 bits, round to nearest even.
__device__ __forceinline__ uint32_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) {
    return make_uint2(f2bf(a) | (f2bf(b) << 16), f2bf(c) | (f2bf(d) << 16));
}

// 4 pixels x 4 channels of bf16 (v[r] = channels of pixel r) -> rows per channel.
__device__ __forceinline__ void transpose4(const uint2 v[4], uint2 o[4]) {
    o[0] = make_uint2((v[0].x & 0xffffu) | (v[1].x << 16), (v[2].x & 0xffffu) | (v[3].x << 16));
    o[1] = make_uint2((v[0].x >> 16) | (v[1].x & 0xffff0000u), (v[2].x >> 16) | (v[3].x & 0xffff0000u));
    o[2] = make_uint2((v[0].y & 0xffffu) | (v[1].y << 16), (v[2].y & 0xffffu) | (v[3].y << 16));
    o[3] = make_uint2((v[0].y >> 16) | (v[1].y & 0xffff0000u), (v[2].y >> 16) | (v[3].y & 0xffff0000u));
}

__device__ __forceinline__ bf16x4 as_bf16x4(uint2 v) {
    bf16x4 r;
    __builtin_memcpy(&r, &v, 8);
    return r;
}
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

// ---------------------------------------------------------------------------
// 3x3 convolution (forward: bias + ReLU + BF16 out; data gradient: FP32 out)
// ---------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t* x;  // input, channels-last; pixel stride xstride, channel offset xoff
    int xstride, xoff;
    int Hin, Win;       // input grid (half the conv grid when the input is upsampled)
    int H, W, P;        // conv grid and pixel count (n*H*W, a multiple of 16)
    int lcin;           // log2 of the input channel count the weights are laid out for
    int nkb;            // reduction length / 16
    const uint16_t* w;  // [cout][kpad] bf16, k = tap*cin + ci
    int kpad;
    const float* bias;  // forward only
    void* y;            // output: bf16 (forward) or fp32 (gradient); pixel stride, offset
    int ystride, yoff;
};

// One wave computes MT pixel tiles x NT channel tiles; 4 waves per block.
template <int MT, int NT, bool UP, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = (blockIdx.x * 4 + wave) * (16 * MT);
    if (base >= a.P) return;
    const int cbase = blockIdx.y * (16 * NT);
    const int g = lane >> 4, r = lane & 15;
    const int HW = a.H * a.W;

    int pi[MT], pj[MT];
    size_t pb[MT];
    bool pv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int p = base + m * 16 + r;
        pv[m] = p < a.P;
        const int pp = pv[m] ? p : 0;
        const int n = pp / HW, rem = pp - n * HW;
        pi[m] = rem / a.W;
        pj[m] = rem - pi[m] * a.W;
        pb[m] = (size_t)n * a.Hin * a.Win;
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    const uint16_t* wrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) wrow[t] = a.w + (size_t)(cbase + t * 16 + r) * a.kpad + 4 * g;
    const int cmask = (1 << a.lcin) - 1;

    for (int kb = 0; kb < a.nkb; ++kb) {
        const int k0 = kb * 16 + 4 * g;
        const int tap = k0 >> a.lcin, ci = k0 & cmask;
        const int ty = tap / 3;
        const int dy = ty - 1, dx = tap - 3 * ty - 1;
        bf16x4 av[MT], bv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bv[t] = as_bf16x4(*(const uint2*)(wrow[t] + kb * 16));
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            int ii = pi[m] + dy, jj = pj[m] + dx;
            const bool ok = pv[m] && tap < 9 && ii >= 0 && ii < a.H && jj >= 0 && jj < a.W;
            if (UP) {
                ii >>= 1;
                jj >>= 1;
            }
            uint2 v = make_uint2(0u, 0u);
            if (ok) v = *(const uint2*)(a.x + (pb[m] + (size_t)ii * a.Win + jj) * a.xstride + a.xoff + ci);
            av[m] = as_bf16x4(v);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[m], bv[t], acc[m][t], 0, 0, 0);
    }

    // D tile: row (pixel) 4g+i, column (channel) r.
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int o = cbase + t * 16 + r;
        const float bo = F32OUT ? 0.f : a.bias[o];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (!pv[m]) continue;  // whole tile (P is a multiple of 16)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const size_t p = (size_t)(base + m * 16 + 4 * g + i);
                const size_t off = p * a.ystride + a.yoff + o;
                if (F32OUT) {
                    ((float*)a.y)[off] = acc[m][t][i];
                } else {
                    const float v = fmaxf(acc[m][t][i] + bo, 0.f);
                    ((uint16_t*)a.y)[off] = (uint16_t)f2bf(v);
                }
            }
        }
    }
}

// Spatially tiled form (level widths that are multiples of 16, >= 16 input
// channels): a block owns a 16 x 16 output tile of one image and NT x 16
// output channels.  For each chunk of KC input channels it stages the tile
// plus a one-pixel halo (18 x 18 pixels, zeros outside the image, nearest
// upsampling folded into the staging) in LDS; the nine taps then read their
// MFMA A fragments from LDS (8 consecutive channels of one pixel per lane,
// one ds_read_b128) without bounds checks.  v_mfma_f32_16x16x32_bf16: lane l
// holds A[l%16][8(l/16)+i], B[8(l/16)+i][l%16]; D row 4(l/16)+i, column l%16.
// Wave w computes tile rows 4w..4w+3 (four 16-pixel row tiles).
constexpr int kTileR = 16, kTileC = 16;

template <int NT, int KC, bool UP, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a, int tiles_per_block) {
    constexpr int SR = kTileR + 2, SC = kTileC + 2, PITCH = KC + 8, G8 = KC / 8;
    constexpr int NKS = (9 * KC + 31) / 32;
    constexpr int ITEMS = (SR * SC * G8 + 255) / 256;   // staged 16-byte items per thread
    __shared__ __attribute__((aligned(16))) uint16_t tile[SR * SC * PITCH];
    // the block's weight panel for one channel chunk: row = output channel
    // (16 NT of them), column = reduction index tap * KC + ci; a 16-byte pad
    // per row spreads neighbouring rows over the LDS banks
    constexpr int WP = 9 * KC + 8, WG8 = 9 * KC / 8, WN = 16 * NT * WG8;
    constexpr int WITEMS = (WN + 255) / 256;   // staged 16-byte items per thread
    __shared__ __attribute__((aligned(16))) uint16_t wpan[16 * NT * WP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int tiles_w = a.W / kTileC, tiles_h = (a.H + kTileR - 1) / kTileR;
    const int n_tiles = (a.P / (a.H * a.W)) * tiles_h * tiles_w;
    const int tl0 = blockIdx.x * tiles_per_block;
    const int tl1 = min(tl0 + tiles_per_block, n_tiles);
    const int cbase = blockIdx.y * (16 * NT);
    const int cin = 1 << a.lcin;
    const int nch = cin / KC;
    const int nsteps = (tl1 - tl0) * nch;
    const int row0 = 4 * wave;

    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[m][u] = f32x4{0.f, 0.f, 0.f, 0.f};
    // global -> LDS: the weight panel of channel chunk c0
    auto wstage = [&](int c0) {
#pragma unroll
        for (int it = 0; it < WITEMS; ++it) {
            const int e = t + 256 * it;
            if (e < WN) {
                const int row = e / WG8, kk = 8 * (e - row * WG8);
                const int tap = kk / KC, ci = kk - tap * KC;
                *(uint4*)&wpan[row * WP + kk] =
                    *(const uint4*)(a.w + (size_t)(cbase + row) * a.kpad + tap * cin + c0 + ci);
            }
        }
    };

    // global -> registers for step `step` (tile tl0 + step / nch, channel chunk step % nch)
    uint4 pre[ITEMS];
    auto fetch = [&](int step) {
        int b = tl0 + step / nch;
        const int c0 = (step % nch) * KC;
        const int tx = b % tiles_w;
        b /= tiles_w;
        const int ty = b % tiles_h;
        const int n = b / tiles_h;
        const int i0 = ty * kTileR, j0 = tx * kTileC;
        const size_t img = (size_t)n * a.Hin * a.Win;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int e = t + 256 * it;
            pre[it] = make_uint4(0u, 0u, 0u, 0u);
            if (e < SR * SC * G8) {
                const int px = e / G8, cg = e - px * G8;
                const int si = px / SC, sj = px - si * SC;
                int ii = i0 + si - 1, jj = j0 + sj - 1;
                if (ii >= 0 && ii < a.H && jj >= 0 && jj < a.W) {
                    if (UP) {
                        ii >>= 1;
                        jj >>= 1;
                    }
                    pre[it] = *(const uint4*)(a.x + (img + (size_t)ii * a.Win + jj) * a.xstride + a.xoff + c0 + 8 * cg);
                }
            }
        }
    };

    if (nsteps > 0) fetch(0);
    for (int step = 0; step < nsteps; ++step) {
        int b = tl0 + step / nch;
        const int c0 = (step % nch) * KC;
        const int tx = b % tiles_w;
        b /= tiles_w;
        const int ty = b % tiles_h;
        const int n = b / tiles_h;
        const int i0 = ty * kTileR, j0 = tx * kTileC;
        __syncthreads();   // the previous step is done with the LDS tile
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int e = t + 256 * it;
            if (e < SR * SC * G8) {
                const int px = e / G8, cg = e - px * G8;
                *(uint4*)&tile[px * PITCH + 8 * cg] = pre[it];
            }
        }
        if (nch > 1 || step == 0) wstage(c0);   // one chunk: the panel stays for every tile
        __syncthreads();
        if (step + 1 < nsteps) fetch(step + 1);   // in flight during the MFMAs below
        if (i0 + row0 < a.H) {
#pragma unroll 3
            for (int ks = 0; ks < NKS; ++ks) {
                const int kk = ks * 32 + 8 * g;
                const int tap = kk / KC, cc = kk - tap * KC;
                const bool tv = tap < 9;
                const int ty3 = tap / 3, tx3 = tap - 3 * ty3;
                bf16x8 bv[NT], av[4];
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    uint4 w = make_uint4(0u, 0u, 0u, 0u);
                    if (tv) w = *(const uint4*)&wpan[(u * 16 + r) * WP + kk];
                    bv[u] = as_bf16x8(w);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    uint4 v = make_uint4(0u, 0u, 0u, 0u);
                    if (tv) v = *(const uint4*)&tile[((row0 + m + ty3) * SC + r + tx3) * PITCH + cc];
                    av[m] = as_bf16x8(v);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        acc[m][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[u], acc[m][u], 0, 0, 0);
            }
        }
        if (c0 + KC < cin) continue;
        // last chunk of this tile: D tile row (pixel) 4g+i, column (channel) r
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int o = cbase + u * 16 + r;
            const float bo = F32OUT ? 0.f : a.bias[o];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int row = i0 + row0 + m;
                if (row < a.H) {
                    const size_t pbase = ((size_t)n * a.H + row) * a.W + j0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const size_t off = (pbase + 4 * g + i) * a.ystride + a.yoff + o;
                        if (F32OUT) {
                            ((float*)a.y)[off] = acc[m][u][i];
                        } else {
                            const float v = fmaxf(acc[m][u][i] + bo, 0.f);
                            ((uint16_t*)a.y)[off] = (uint16_t)f2bf(v);
                        }
                    }
                }
                acc[m][u] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[z][o][k] = sum over the pixels of slab z of
// dz[p][o] * im2col(x)[p][k]; bpart[z][o] = sum of dz[p][o] over the slab.
// ---------------------------------------------------------------------------
struct WgArgs {
    const uint16_t* x;
    int xstride, xoff, Hin, Win, H, W, P, lcin, K, kpad;
    const uint16_t* dz;  // [P][cout] bf16
    int cout;
    float* part;   // [S][cout][kpad]
    float* bpart;  // [S][cout]
    int slab;      // pixels per block, a multiple of 64
};

constexpr int kLdsPitch = 64 + 4;  // bf16 per transposed row (pads LDS banks)

template <int OT, bool UP>
__global__ __launch_bounds__(256) void k_wgrad(WgArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t dzT[OT][kLdsPitch];
    __shared__ __attribute__((aligned(16))) uint16_t imT[64][kLdsPitch];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int kbase = blockIdx.x * 64, obase = blockIdx.y * OT;
    const int p_begin = blockIdx.z * a.slab;
    const int p_end = min(p_begin + a.slab, a.P);
    const int HW = a.H * a.W;
    const bool kt_ok = kbase + 16 * wave < a.kpad;
    const int pg = t & 15, grp = t >> 4;
    const int cmask = (1 << a.lcin) - 1;

    f32x4 acc[OT / 16];
#pragma unroll
    for (int o = 0; o < OT / 16; ++o) acc[o] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;

    for (int p0 = p_begin; p0 < p_end; p0 += 64) {
        const int pq = p0 + 4 * pg;  // first of this thread's 4 pixels (same image row)
        const bool pok = pq < p_end;
        if (grp < OT / 4) {
            uint2 v[4], o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = pok ? *(const uint2*)(a.dz + (size_t)(pq + q) * a.cout + obase + 4 * grp) : make_uint2(0u, 0u);
            transpose4(v, o);
#pragma unroll
            for (int c = 0; c < 4; ++c) *(uint2*)&dzT[4 * grp + c][4 * pg] = o[c];
        }
        {
            const int k0 = kbase + 4 * grp;
            uint2 v[4], o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = make_uint2(0u, 0u);
            if (pok && k0 < a.K) {
                const int tap = k0 >> a.lcin, ci = k0 & cmask;
                const int ty = tap / 3;
                const int dy = ty - 1, dx = tap - 3 * ty - 1;
                const int n = pq / HW, rem = pq - n * HW;
                const int i = rem / a.W, j = rem - i * a.W;
                const int ii = i + dy;
                if (ii >= 0 && ii < a.H) {
                    const int is = UP ? (ii >> 1) : ii;
                    const size_t rowb = (size_t)n * a.Hin * a.Win + (size_t)is * a.Win;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int jj = j + q + dx;
                        if (jj >= 0 && jj < a.W) {
                            const int js = UP ? (jj >> 1) : jj;
                            v[q] = *(const uint2*)(a.x + (rowb + js) * a.xstride + a.xoff + ci);
                        }
                    }
                }
            }
            transpose4(v, o);
#pragma unroll
            for (int c = 0; c < 4; ++c) *(uint2*)&imT[4 * grp + c][4 * pg] = o[c];
        }
        __syncthreads();
        if (kt_ok) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bf16x4 bv = as_bf16x4(*(const uint2*)&imT[16 * wave + r][16 * s + 4 * g]);
#pragma unroll
                for (int o = 0; o < OT / 16; ++o) {
                    const bf16x4 av = as_bf16x4(*(const uint2*)&dzT[16 * o + r][16 * s + 4 * g]);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[o], 0, 0, 0);
                }
            }
        }
        if (blockIdx.x == 0 && t < OT) {
#pragma unroll
            for (int q = 0; q < 64; q += 4) {
                const uint2 v = *(const uint2*)&dzT[t][q];
                bsum += bf2f(v.x & 0xffffu) + bf2f(v.x >> 16) + bf2f(v.y & 0xffffu) + bf2f(v.y >> 16);
            }
        }
        __syncthreads();
    }
    if (kt_ok) {
        const int k = kbase + 16 * wave + r;
#pragma unroll
        for (int o = 0; o < OT / 16; ++o)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a.part[((size_t)blockIdx.z * a.cout + obase + 16 * o + 4 * g + i) * a.kpad + k] = acc[o][i];
    }
    if (blockIdx.x == 0 && t < OT) a.bpart[(size_t)blockIdx.z * a.cout + obase + t] = bsum;
}

// Spatially tiled weight gradient (level widths that are multiples of 16,
// >= 16 input channels).  A block owns OT output channels and 16 input
// channels and walks a slab of 16 x 16 output tiles.  Per tile it stages the
// masked gradient transposed (dzT[o][pixel]) and the input tile plus halo
// transposed in three column-shifted copies (xT[dx][ci][row][col] = input at
// (row - 1, col + dx - 1) of the tile), so that both MFMA operands of every
// tap are aligned 8-pixel runs: dW[o][tap, ci] += sum over 32-pixel steps of
// dzT[o][px] * xT[dx][ci][row + dy][col].  v_mfma_f32_16x16x32_bf16 with the
// pixels as the reduction.  Wave w owns taps w and w + 4 for every channel
// tile, and tap 8 for channel tile w (w < OT/16), so each 32-pixel step reads
// every masked-gradient fragment once and reuses it across the wave's taps.

template <int OT, bool UP>
__global__ __launch_bounds__(256) void k_wgrad_sp(WgArgs a, int tiles_per_slab) {
    constexpr int DZP = 256 + 8;              // dzT row pitch (pixels)
    constexpr int XR = kTileR + 2;            // staged rows
    constexpr int XP = XR * kTileC + 8;       // xT pitch per (dx, ci)
    constexpr int NO = OT / 16;
    __shared__ __attribute__((aligned(16))) uint16_t dzT[OT * DZP];
    __shared__ __attribute__((aligned(16))) uint16_t xT[3 * 16 * XP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int obase = blockIdx.y * OT, c0 = blockIdx.z * 16;
    const int cin = 1 << a.lcin;
    const int tiles_w = a.W / kTileC, tiles_h = (a.H + kTileR - 1) / kTileR;
    const int n_tiles = (a.P / (a.H * a.W)) * tiles_h * tiles_w;
    const int tile0 = blockIdx.x * tiles_per_slab;
    const int tile1 = min(tile0 + tiles_per_slab, n_tiles);

    f32x4 acc[2][NO], acc8 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < NO; ++u) acc[j][u] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool has8 = wave < NO;
    float bsum = 0.f;

    for (int tl = tile0; tl < tile1; ++tl) {
        int b = tl;
        const int tx = b % tiles_w;
        b /= tiles_w;
        const int ty = b % tiles_h;
        const int n = b / tiles_h;
        const int i0 = ty * kTileR, j0 = tx * kTileC;
        // masked gradient, 4 pixels x 4 channels per step, transposed
        for (int e = t; e < (256 / 4) * (OT / 4); e += 256) {
            const int pg = e % 64, cg = e / 64;
            const int row = pg >> 2, col = (pg & 3) * 4;
            uint2 v[4], o[4];
            const bool ok = i0 + row < a.H;
            const size_t p = ((size_t)n * a.H + i0 + row) * a.W + j0 + col;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = ok ? *(const uint2*)(a.dz + (p + q) * a.cout + obase + 4 * cg) : make_uint2(0u, 0u);
            transpose4(v, o);
#pragma unroll
            for (int c = 0; c < 4; ++c) *(uint2*)&dzT[(4 * cg + c) * DZP + row * kTileC + col] = o[c];
        }
        // input tile + halo, 16 channels, into the three shifted copies
        for (int e = t; e < XR * (kTileC + 2) * 2; e += 256) {
            const int px = e >> 1, h8 = (e & 1) * 8;
            const int sr = px / (kTileC + 2), sc = px - sr * (kTileC + 2);
            int ii = i0 + sr - 1, jj = j0 + sc - 1;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (ii >= 0 && ii < a.H && jj >= 0 && jj < a.W) {
                if (UP) {
                    ii >>= 1;
                    jj >>= 1;
                }
                v = *(const uint4*)(a.x + ((size_t)n * a.Hin * a.Win + (size_t)ii * a.Win + jj) * a.xstride + a.xoff +
                                    c0 + h8);
            }
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int col = sc - dx;
                if (col < 0 || col >= kTileC) continue;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    xT[(dx * 16 + h8 + q) * XP + sr * kTileC + col] =
                        (uint16_t)((q & 1) ? (w[q >> 1] >> 16) : (w[q >> 1] & 0xffffu));
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < 8; ++ks) {
            const int px = 32 * ks + 8 * g;                   // 8 pixels of one tile row
            const int row = px >> 4, col = px & 15;
            bf16x8 av[NO];
#pragma unroll
            for (int u = 0; u < NO; ++u) av[u] = as_bf16x8(*(const uint4*)&dzT[(u * 16 + r) * DZP + px]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int tap = wave + 4 * j;
                const int ty3 = tap / 3, tx3 = tap - 3 * ty3;
                const bf16x8 bv = as_bf16x8(*(const uint4*)&xT[(tx3 * 16 + r) * XP + (row + ty3) * kTileC + col]);
#pragma unroll
                for (int u = 0; u < NO; ++u)
                    acc[j][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[u], bv, acc[j][u], 0, 0, 0);
            }
            if (has8) {   // tap 8 = (2, 2)
                const bf16x8 bv = as_bf16x8(*(const uint4*)&xT[(2 * 16 + r) * XP + (row + 2) * kTileC + col]);
                bf16x8 a8 = av[0];
#pragma unroll
                for (int u = 1; u < NO; ++u)
                    if (u == wave) a8 = av[u];
                acc8 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, bv, acc8, 0, 0, 0);
            }
        }
        if (blockIdx.z == 0 && t < OT) {
            for (int q = 0; q < 256; q += 8) {
                const uint4 v = *(const uint4*)&dzT[t * DZP + q];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int h = 0; h < 4; ++h) bsum += bf2f(w[h] & 0xffffu) + bf2f(w[h] >> 16);
            }
        }
        __syncthreads();
    }
    // D tile: row (output channel) 4g+i, column (input channel) r
    float* prow = a.part + (size_t)blockIdx.x * a.cout * a.kpad;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < NO; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                prow[(size_t)(obase + u * 16 + 4 * g + i) * a.kpad + (wave + 4 * j) * cin + c0 + r] = acc[j][u][i];
    if (has8)
#pragma unroll
        for (int i = 0; i < 4; ++i) prow[(size_t)(obase + wave * 16 + 4 * g + i) * a.kpad + 8 * cin + c0 + r] = acc8[i];
    if (blockIdx.z == 0 && t < OT) a.bpart[(size_t)blockIdx.x * a.cout + obase + t] = bsum;
}

// First level of the slab sum: out[y][e] = sum of in[z][e] over the 32 slabs
// z of group y (fixed order).
__global__ void k_sum_slabs(const float* in, int S, int n, float* out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int z0 = blockIdx.y * 32, z1 = min(z0 + 32, S);
    float s = 0.f;
    for (int z = z0; z < z1; ++z) s += in[(size_t)z * n + e];
    out[(size_t)blockIdx.y * n + e] = s;
}

// Sum the slabs and scatter into the flat gradient ([cout][cin][3][3], then bias).
__global__ void k_reduce_wgrad(const float* part, const float* bpart, int S, int cout, int kpad, int lcin_s,
                               int cin, float* gw, float* gb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * kpad;
    if (idx < nw) {
        const int o = idx / kpad, k = idx - o * kpad;
        const int tap = k >> lcin_s, ci = k & ((1 << lcin_s) - 1);
        if (tap < 9 && ci < cin) {
            float s = 0.f;
            for (int z = 0; z < S; ++z) s += part[(size_t)z * nw + idx];
            gw[(o * cin + ci) * 9 + tap] = s;
        }
    } else if (idx < nw + cout) {
        const int o = idx - nw;
        float s = 0.f;
        for (int z = 0; z < S; ++z) s += bpart[(size_t)z * cout + o];
        gb[o] = s;
    }
}

// ---------------------------------------------------------------------------
// elementwise / small kernels
// ---------------------------------------------------------------------------
// Network input: (f, g, clip(phi0, +-c)/c, 0) per pixel.
__global__ void k_input(const float* f, const float* g, const float* phi0, int P, float clip, uint16_t* x0) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float ph = fminf(fmaxf(phi0[p], -clip), clip) / clip;
    *(uint2*)(x0 + 4 * (size_t)p) = pack4(f[p], g[p], ph, 0.f);
}

// 2x2 average pooling of C channels (bf16 in with stride/offset -> bf16 contiguous).
__global__ void k_pool(const uint16_t* x, int xstride, int xoff, int C, int Ho, int Wo, int Po, uint16_t* y) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int cq = C >> 2;
    if (idx >= Po * cq) return;
    const int p = idx / cq, c = 4 * (idx - p * cq);
    const int HWo = Ho * Wo;
    const int n = p / HWo, rem = p - n * HWo;
    const int io = rem / Wo, jo = rem - io * Wo;
    const int Wi = 2 * Wo;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const size_t pin = (size_t)n * 4 * HWo + (size_t)(2 * io + (d >> 1)) * Wi + 2 * jo + (d & 1);
        const uint2 v = *(const uint2*)(x + pin * xstride + xoff + c);
        s[0] += bf2f(v.x & 0xffffu);
        s[1] += bf2f(v.x >> 16);
        s[2] += bf2f(v.y & 0xffffu);
        s[3] += bf2f(v.y >> 16);
    }
    *(uint2*)(y + (size_t)p * C + c) = pack4(0.25f * s[0], 0.25f * s[1], 0.25f * s[2], 0.25f * s[3]);
}

// Output gradient -> masked BF16 dz of a layer:
// dz = (A + 0.25*poolback(B)) * [act > 0], A either same-grid (stride/offset)
// or the 2x2 sum of a twice-finer tensor (gradient through nearest upsampling).
struct MaskArgs {
    const float* A;
    int astride, aoff, aup;
    const float* B;  // nullable: half-grid tensor [.][C] (gradient through 2x2 average pooling)
    const uint16_t* act;
    int actstride, actoff;
    int H, W, P, C;
    uint16_t* dz;
};

__global__ void k_mask(MaskArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int cq = a.C >> 2;
    if (idx >= a.P * cq) return;
    const int p = idx / cq, c = 4 * (idx - p * cq);
    const int HW = a.H * a.W;
    const int n = p / HW, rem = p - n * HW;
    const int i = rem / a.W, j = rem - i * a.W;
    float4 s;
    if (a.aup) {
        s = make_float4(0.f, 0.f, 0.f, 0.f);
        const int W2 = 2 * a.W;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const size_t q = (size_t)n * 4 * HW + (size_t)(2 * i + (d >> 1)) * W2 + 2 * j + (d & 1);
            const float4 v = *(const float4*)(a.A + q * a.C + c);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
    } else {
        s = *(const float4*)(a.A + (size_t)p * a.astride + a.aoff + c);
    }
    if (a.B) {
        const int Wh = a.W >> 1;
        const size_t q = (size_t)n * (HW >> 2) + (size_t)(i >> 1) * Wh + (j >> 1);
        const float4 v = *(const float4*)(a.B + q * a.C + c);
        s.x += 0.25f * v.x;
        s.y += 0.25f * v.y;
        s.z += 0.25f * v.z;
        s.w += 0.25f * v.w;
    }
    const uint2 m = *(const uint2*)(a.act + (size_t)p * a.actstride + a.actoff + c);
    const float o0 = bf2f(m.x & 0xffffu) > 0.f ? s.x : 0.f;
    const float o1 = bf2f(m.x >> 16) > 0.f ? s.y : 0.f;
    const float o2 = bf2f(m.y & 0xffffu) > 0.f ? s.z : 0.f;
    const float o3 = bf2f(m.y >> 16) > 0.f ? s.w : 0.f;
    *(uint2*)(a.dz + (size_t)p * a.C + c) = pack4(o0, o1, o2, o3);
}

// 1x1 head: y = b + sum_c d0[c] w[c]; phi = clip*y (optional).
__global__ void k_head(const uint16_t* d0, const float* wh, int P, float clip, float* y, float* phi) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint4* src = (const uint4*)(d0 + 16 * (size_t)p);
    float s = wh[16];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint4 v = src[h];
        const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            s += bf2f(u[q] & 0xffffu) * wh[8 * h + 2 * q] + bf2f(u[q] >> 16) * wh[8 * h + 2 * q + 1];
    }
    y[p] = s;
    if (phi) phi[p] = clip * s;
}

constexpr int kHeadPart = 18;  // 16 head weights, head bias, loss

// Loss and head backward, fused with the mask of the last 3x3 layer:
// dy = (2/P)(y - clip(t)/c), dz_D0[c] = dy*w[c]*[d0[c] > 0]; per-block partial
// sums of d0[c]*dy, dy and (y - t)^2.
__global__ __launch_bounds__(256) void k_head_back(const uint16_t* d0, const float* y, const float* target,
                                                   const float* wh, int P, float clip, uint16_t* dz,
                                                   float* part) {
    __shared__ float red[kHeadPart][8];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    float acc[kHeadPart];
#pragma unroll
    for (int q = 0; q < kHeadPart; ++q) acc[q] = 0.f;
    if (p < P) {
        const float tt = fminf(fmaxf(target[p], -clip), clip) / clip;
        const float diff = y[p] - tt;
        const float dy = (2.f / (float)P) * diff;
        const uint4* src = (const uint4*)(d0 + 16 * (size_t)p);
        uint4* dst = (uint4*)(dz + 16 * (size_t)p);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint4 v = src[h];
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
            uint32_t o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 8 * h + 2 * q;
                const float a0 = bf2f(u[q] & 0xffffu), a1 = bf2f(u[q] >> 16);
                acc[c] += a0 * dy;
                acc[c + 1] += a1 * dy;
                const float g0 = a0 > 0.f ? dy * wh[c] : 0.f;
                const float g1 = a1 > 0.f ? dy * wh[c + 1] : 0.f;
                o[q] = f2bf(g0) | (f2bf(g1) << 16);
            }
            dst[h] = make_uint4(o[0], o[1], o[2], o[3]);
        }
        acc[16] = dy;
        acc[17] = diff * diff;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kHeadPart; ++q) {
        float v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < kHeadPart) {
        const int q = threadIdx.x;
        part[(size_t)blockIdx.x * kHeadPart + q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
    }
}

// out[q] = sum over blocks of part[b][q] (one block per q, fixed order).
__global__ __launch_bounds__(256) void k_reduce_head(const float* part, int nb, float* gw, float* gb,
                                                     float* loss, float inv_p) {
    __shared__ float red[4];
    const int q = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(size_t)b * kHeadPart + q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float v = red[0] + red[1] + red[2] + red[3];
        if (q < 16) gw[q] = v;
        else if (q == 16) gb[0] = v;
        else loss[0] = v * inv_p;
    }
}

// bf16 view (stride/offset) -> contiguous fp32 [P][C].
__global__ void k_unpack(const uint16_t* x, int stride, int off, int C, int P, float* out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * C) return;
    const int p = idx / C, c = idx - p * C;
    out[idx] = bf2f(x[(size_t)p * stride + off + c]);
}

// Adam with bias-corrected moments; c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void k_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Flat [cout][cin][3][3] weights -> forward layout [cout][kpad], k = tap*cin_s + ci.
__global__ void k_pack_fwd(const float* w, int cin, int lcin_s, int cout, int kpad, uint16_t* wf) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cout * kpad) return;
    const int o = idx / kpad, k = idx - o * kpad;
    const int tap = k >> lcin_s, ci = k & ((1 << lcin_s) - 1);
    const float v = (tap < 9 && ci < cin) ? w[(o * cin + ci) * 9 + tap] : 0.f;
    wf[idx] = (uint16_t)f2bf(v);
}

// Flat weights -> data-gradient layout [cin][kdpad], k = tap*cout + o (zero
// beyond 9*cout), the stencil turned by 180 degrees (tap (ky,kx) reads
// weight (2-ky, 2-kx)).
__global__ void k_pack_dgrad(const float* w, int cin, int cout, int kdpad, uint16_t* wd) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= cin * kdpad) return;
    const int c = idx / kdpad, k = idx - c * kdpad;
    const int tap = k / cout, o = k - tap * cout;
    wd[idx] = tap < 9 ? (uint16_t)f2bf(w[(o * cin + c) * 9 + (8 - tap)]) : (uint16_t)0;
}

}  // namespace cnn

// ===========================================================================
// host runtime
// ===========================================================================
using namespace cnn;

static thread_local std::string g_cnn_err;

static int cfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_cnn_err = buf;
    return code;
}

#define CHIP(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return cfail(SR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

enum { L0a, L0b, L1a, L1b, L2a, L2b, L3a, L3b, U2, D2, U1, D1, U0, D0, kConv };

struct LayerDesc {
    const char* name;
    int cin, cout, cin_s, level;
    int kpad;         // forward reduction length (multiple of 32)
    int kdpad;        // data-gradient reduction length (multiple of 32)
    size_t pw, pb;    // offsets of weights / bias in the flat parameter vector
    size_t wf, wd;    // offsets (elements) in the packed bf16 weight buffers
};

struct Net {
    LayerDesc L[kConv];
    size_t head_w, head_b, np, nwf, nwd, max_part;
};

static int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

static const Net& net() {
    static Net n = [] {
        Net t{};
        const struct {
            const char* name;
            int cin, cout, level;
        } spec[kConv] = {{"L0a", 3, 16, 0},   {"L0b", 16, 16, 0},  {"L1a", 16, 32, 1},  {"L1b", 32, 32, 1},
                         {"L2a", 32, 64, 2},  {"L2b", 64, 64, 2},  {"L3a", 64, 128, 3}, {"L3b", 128, 128, 3},
                         {"U2", 128, 64, 2},  {"D2", 128, 64, 2},  {"U1", 64, 32, 1},   {"D1", 64, 32, 1},
                         {"U0", 32, 16, 0},   {"D0", 32, 16, 0}};
        size_t off = 0, wf = 0, wd = 0, mp = 0;
        for (int i = 0; i < kConv; ++i) {
            LayerDesc& d = t.L[i];
            d.name = spec[i].name;
            d.cin = spec[i].cin;
            d.cout = spec[i].cout;
            d.level = spec[i].level;
            d.cin_s = d.cin < 4 ? 4 : d.cin;
            d.kpad = (9 * d.cin_s + 31) / 32 * 32;
            d.kdpad = (9 * d.cout + 31) / 32 * 32;
            d.pw = off;
            off += (size_t)d.cout * d.cin * 9;
            d.pb = off;
            off += d.cout;
            d.wf = wf;
            wf += (size_t)d.cout * d.kpad;
            d.wd = wd;
            wd += (size_t)d.cin * d.kdpad;
            mp = std::max(mp, (size_t)d.cout * d.kpad);
        }
        t.head_w = off;
        off += 16;
        t.head_b = off;
        off += 1;
        t.np = off;
        t.nwf = wf;
        t.nwd = wd;
        t.max_part = mp;
        return t;
    }();
    return n;
}

// Weight-gradient grids aim at kWgBlocks blocks (k blocks x channel blocks x
// pixel slabs); the partial tiles of one layer then take at most
// kWgBlocks * 64 * 64 floats.
constexpr int kWgBlocks = 2048;
constexpr size_t kPartFloats = (size_t)kWgBlocks * 64 * 64;

struct Carve {
    char* base;
    size_t off;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct cnn_ctx {
    int B, H, W;
    hipStream_t st;
    // parameters
    float *params, *m, *v, *grad;
    uint16_t *wf, *wd;
    int t_adam;
    // forward activations (bf16, channels-last)
    uint16_t *x0, *aL0a, *C0, *p0, *aL1a, *C1, *p1, *aL2a, *C2, *p2, *aL3a, *bott, *d2, *d1, *d0;
    float* y;
    // backward: masked output gradient of every 3x3 layer (bf16 [P_l][cout])
    uint16_t* dz[kConv];
    float *dcat0, *dcat1, *dcat2, *T0, *T1;
    float *part, *bpart, *part2, *bpart2, *hpart, *loss;
    // state of the last forward / backward
    int n_last, n_grad;
    float clip_last;
};

static size_t carve_all(cnn_ctx* c, char* base, int B, int H, int W) {
    const Net& N = net();
    Carve k{base, 0};
    const size_t P0 = (size_t)B * H * W, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
    c->params = k.take<float>(N.np);
    c->m = k.take<float>(N.np);
    c->v = k.take<float>(N.np);
    c->grad = k.take<float>(N.np);
    c->wf = k.take<uint16_t>(N.nwf);
    c->wd = k.take<uint16_t>(N.nwd);
    c->x0 = k.take<uint16_t>(P0 * 4);
    c->aL0a = k.take<uint16_t>(P0 * 16);
    c->C0 = k.take<uint16_t>(P0 * 32);
    c->p0 = k.take<uint16_t>(P1 * 16);
    c->aL1a = k.take<uint16_t>(P1 * 32);
    c->C1 = k.take<uint16_t>(P1 * 64);
    c->p1 = k.take<uint16_t>(P2 * 32);
    c->aL2a = k.take<uint16_t>(P2 * 64);
    c->C2 = k.take<uint16_t>(P2 * 128);
    c->p2 = k.take<uint16_t>(P3 * 64);
    c->aL3a = k.take<uint16_t>(P3 * 128);
    c->bott = k.take<uint16_t>(P3 * 128);
    c->d2 = k.take<uint16_t>(P2 * 64);
    c->d1 = k.take<uint16_t>(P1 * 32);
    c->d0 = k.take<uint16_t>(P0 * 16);
    c->y = k.take<float>(P0);
    for (int i = 0; i < kConv; ++i) c->dz[i] = k.take<uint16_t>((P0 >> (2 * N.L[i].level)) * N.L[i].cout);
    c->dcat0 = k.take<float>(P0 * 32);
    c->dcat1 = k.take<float>(P1 * 64);
    c->dcat2 = k.take<float>(P2 * 128);
    c->T0 = k.take<float>(P0 * 32);
    c->T1 = k.take<float>(P0 * 16);
    c->part = k.take<float>(kPartFloats);
    c->bpart = k.take<float>((size_t)kWgBlocks * 128);
    c->part2 = k.take<float>((size_t)(kWgBlocks / 32) * N.max_part);
    c->bpart2 = k.take<float>((size_t)(kWgBlocks / 32) * 128);
    c->hpart = k.take<float>((P0 + 255) / 256 * kHeadPart);
    c->loss = k.take<float>(1);
    return k.off;
}

static int check_dims(int32_t B, int32_t H, int32_t W) {
    if (B < 1 || H < 32 || W < 32 || H > 2048 || W > 2048 || H % 32 || W % 32)
        return cfail(SR_EUNSUPPORTED, "batch >= 1 and H, W multiples of 32 in [32, 2048] required (got %d, %d x %d)",
                     B, H, W);
    if ((int64_t)B * H * W > (int64_t(1) << 26))
        return cfail(SR_EUNSUPPORTED, "batch*H*W = %lld exceeds 2^26", (long long)B * H * W);
    return SR_OK;
}

static unsigned blocks(size_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---- launch helpers --------------------------------------------------------
struct Act {  // a channels-last bf16 tensor view
    const uint16_t* p;
    int stride, off;
};

// Grids aim at ~6 resident blocks per CU; each block walks consecutive
// tiles (spatial neighbours) so the staging of the next one overlaps the
// MFMAs of the current one.
constexpr int kConvBlocks = 256 * 6;

template <int KC, bool UP, bool F32>
static void conv_lds_t(const ConvArgs& a, int cout, int nt, hipStream_t st) {
    const int n = a.P / (a.H * a.W);
    const int n_tiles = n * ((a.H + kTileR - 1) / kTileR) * (a.W / kTileC);
    const int ob = cout / (16 * nt);
    const int per = std::max(1, n_tiles / std::max(1, kConvBlocks / ob));
    dim3 grid((n_tiles + per - 1) / per, ob);
    switch (nt) {
        case 1: k_conv_lds<1, KC, UP, F32><<<grid, 256, 0, st>>>(a, per); break;
        case 2: k_conv_lds<2, KC, UP, F32><<<grid, 256, 0, st>>>(a, per); break;
        default: k_conv_lds<4, KC, UP, F32><<<grid, 256, 0, st>>>(a, per); break;
    }
}

// Spatially tiled kernel where the level's width is a multiple of 16 and the
// input has >= 16 channels; the per-pixel-tile kernel otherwise.
template <bool UP, bool F32>
static void conv_t(const ConvArgs& a, int cout, hipStream_t st) {
    const int nt = std::min(cout / 16, 4);
    if (a.W % kTileC == 0 && a.lcin >= 4) {
        if (a.lcin >= 5) conv_lds_t<32, UP, F32>(a, cout, nt, st);
        else conv_lds_t<16, UP, F32>(a, cout, nt, st);
        return;
    }
    dim3 grid(blocks(a.P, 256), cout / (16 * nt));
    switch (nt) {
        case 1: k_conv<4, 1, UP, F32><<<grid, 256, 0, st>>>(a); break;
        case 2: k_conv<4, 2, UP, F32><<<grid, 256, 0, st>>>(a); break;
        default: k_conv<4, 4, UP, F32><<<grid, 256, 0, st>>>(a); break;
    }
}

// forward conv of layer `li` (input view at the conv grid's level or, with up, one level coarser)
static void conv_fwd(cnn_ctx* c, int li, Act in, bool up, uint16_t* out, int ostride, int ooff, int n) {
    const LayerDesc& d = net().L[li];
    const int H = c->H >> d.level, W = c->W >> d.level;
    ConvArgs a{};
    a.x = in.p;
    a.xstride = in.stride;
    a.xoff = in.off;
    a.Hin = up ? H / 2 : H;
    a.Win = up ? W / 2 : W;
    a.H = H;
    a.W = W;
    a.P = n * H * W;
    a.lcin = ilog2(d.cin_s);
    a.nkb = d.kpad / 16;
    a.w = c->wf + d.wf;
    a.kpad = d.kpad;
    a.bias = c->params + d.pb;
    a.y = out;
    a.ystride = ostride;
    a.yoff = ooff;
    if (up) conv_t<true, false>(a, d.cout, c->st);
    else conv_t<false, false>(a, d.cout, c->st);
}

// data gradient of layer li: dz [P][cout] -> out fp32 [P][cin]
static void conv_dgrad(cnn_ctx* c, int li, float* out, int n) {
    const LayerDesc& d = net().L[li];
    const int H = c->H >> d.level, W = c->W >> d.level;
    ConvArgs a{};
    a.x = c->dz[li];
    a.xstride = d.cout;
    a.xoff = 0;
    a.Hin = H;
    a.Win = W;
    a.H = H;
    a.W = W;
    a.P = n * H * W;
    a.lcin = ilog2(d.cout);
    a.nkb = d.kdpad / 16;
    a.w = c->wd + d.wd;
    a.kpad = d.kdpad;
    a.bias = nullptr;
    a.y = out;
    a.ystride = d.cin;
    a.yoff = 0;
    conv_t<false, true>(a, d.cin, c->st);
}

// Slab partials -> flat gradient: a first fixed-order pass over groups of 32
// slabs when there are more than 32, then the scatter.
static void reduce_wgrad(cnn_ctx* c, const LayerDesc& d, int S) {
    const int nw = d.cout * d.kpad;
    const float *part = c->part, *bpart = c->bpart;
    if (S > 32) {
        const int S2 = (S + 31) / 32;
        k_sum_slabs<<<dim3(blocks(nw), S2), 256, 0, c->st>>>(c->part, S, nw, c->part2);
        k_sum_slabs<<<dim3(blocks(d.cout), S2), 256, 0, c->st>>>(c->bpart, S, d.cout, c->bpart2);
        part = c->part2;
        bpart = c->bpart2;
        S = S2;
    }
    k_reduce_wgrad<<<blocks(nw + d.cout), 256, 0, c->st>>>(part, bpart, S, d.cout, d.kpad, ilog2(d.cin_s), d.cin,
                                                            c->grad + d.pw, c->grad + d.pb);
}

static void conv_wgrad(cnn_ctx* c, int li, Act in, bool up, int n) {
    const Net& N = net();
    const LayerDesc& d = N.L[li];
    const int H = c->H >> d.level, W = c->W >> d.level;
    WgArgs a{};
    a.x = in.p;
    a.xstride = in.stride;
    a.xoff = in.off;
    a.Hin = up ? H / 2 : H;
    a.Win = up ? W / 2 : W;
    a.H = H;
    a.W = W;
    a.P = n * H * W;
    a.lcin = ilog2(d.cin_s);
    a.K = 9 * d.cin_s;
    a.kpad = d.kpad;
    a.dz = c->dz[li];
    a.cout = d.cout;
    a.part = c->part;
    a.bpart = c->bpart;
    const size_t nw = (size_t)d.cout * d.kpad;
    const int cap = (int)std::min<size_t>(kWgBlocks, kPartFloats / nw);
    if (W % kTileC == 0 && d.cin_s >= 16) {
        const int OT = std::min(d.cout, 32);
        const int ob = d.cout / OT, nch = d.cin_s / 16;
        const int n_tiles = n * ((H + kTileR - 1) / kTileR) * (W / kTileC);
        int S = std::max(1, std::min(std::min(n_tiles, cap), kWgBlocks / (ob * nch)));
        const int per = (n_tiles + S - 1) / S;
        S = (n_tiles + per - 1) / per;
        dim3 grid(S, ob, nch);
        if (OT == 16) {
            if (up) k_wgrad_sp<16, true><<<grid, 256, 0, c->st>>>(a, per);
            else k_wgrad_sp<16, false><<<grid, 256, 0, c->st>>>(a, per);
        } else {
            if (up) k_wgrad_sp<32, true><<<grid, 256, 0, c->st>>>(a, per);
            else k_wgrad_sp<32, false><<<grid, 256, 0, c->st>>>(a, per);
        }
        reduce_wgrad(c, d, S);
        return;
    }
    const int OT = std::min(d.cout, 64);
    const int kb = (d.kpad + 63) / 64, ob = d.cout / OT;
    const int chunks = (a.P + 63) / 64;
    int S = std::max(1, std::min(std::min(chunks, cap), kWgBlocks / (kb * ob)));
    const int per = (chunks + S - 1) / S;
    a.slab = per * 64;
    S = (a.P + a.slab - 1) / a.slab;
    dim3 grid(kb, ob, S);
    if (OT == 16) {
        if (up) k_wgrad<16, true><<<grid, 256, 0, c->st>>>(a);
        else k_wgrad<16, false><<<grid, 256, 0, c->st>>>(a);
    } else if (OT == 32) {
        if (up) k_wgrad<32, true><<<grid, 256, 0, c->st>>>(a);
        else k_wgrad<32, false><<<grid, 256, 0, c->st>>>(a);
    } else {
        if (up) k_wgrad<64, true><<<grid, 256, 0, c->st>>>(a);
        else k_wgrad<64, false><<<grid, 256, 0, c->st>>>(a);
    }
    reduce_wgrad(c, d, S);
}

static void mask(cnn_ctx* c, int li, const float* A, int astride, int aoff, bool aup, const float* B, Act act,
                 int n) {
    const LayerDesc& d = net().L[li];
    MaskArgs a{};
    a.A = A;
    a.astride = astride;
    a.aoff = aoff;
    a.aup = aup ? 1 : 0;
    a.B = B;
    a.act = act.p;
    a.actstride = act.stride;
    a.actoff = act.off;
    a.H = c->H >> d.level;
    a.W = c->W >> d.level;
    a.P = n * a.H * a.W;
    a.C = d.cout;
    a.dz = c->dz[li];
    k_mask<<<blocks((size_t)a.P * (a.C / 4)), 256, 0, c->st>>>(a);
}

static void pool(cnn_ctx* c, Act in, int C, int level_out, uint16_t* out, int n) {
    const int Ho = c->H >> level_out, Wo = c->W >> level_out;
    const int Po = n * Ho * Wo;
    k_pool<<<blocks((size_t)Po * (C / 4)), 256, 0, c->st>>>(in.p, in.stride, in.off, C, Ho, Wo, Po, out);
}

static void pack_weights(cnn_ctx* c) {
    const Net& N = net();
    for (int i = 0; i < kConv; ++i) {
        const LayerDesc& d = N.L[i];
        k_pack_fwd<<<blocks((size_t)d.cout * d.kpad), 256, 0, c->st>>>(c->params + d.pw, d.cin, ilog2(d.cin_s), d.cout,
                                                                        d.kpad, c->wf + d.wf);
        if (i != L0a)
            k_pack_dgrad<<<blocks((size_t)d.cin * d.kdpad), 256, 0, c->st>>>(c->params + d.pw, d.cin, d.cout,
                                                                              d.kdpad, c->wd + d.wd);
    }
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cnn_last_error(void) { return g_cnn_err.c_str(); }

int cnn_num_params(int64_t* n) {
    if (!n) return cfail(SR_EINVAL, "n is NULL");
    *n = (int64_t)net().np;
    return SR_OK;
}

int cnn_workspace_size(int32_t batch, int32_t H, int32_t W, size_t* bytes) {
    if (!bytes) return cfail(SR_EINVAL, "bytes is NULL");
    int rc = check_dims(batch, H, W);
    if (rc) return rc;
    cnn_ctx tmp{};
    *bytes = carve_all(&tmp, nullptr, batch, H, W);
    return SR_OK;
}

int cnn_create(cnn_ctx** out, int32_t batch, int32_t H, int32_t W, void* workspace, size_t bytes,
               void* hip_stream) {
    if (!out) return cfail(SR_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_dims(batch, H, W);
    if (rc) return rc;
    if (!workspace) return cfail(SR_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256) return cfail(SR_EWORKSPACE, "workspace must be 256-byte aligned");
    cnn_ctx tmp{};
    const size_t need = carve_all(&tmp, nullptr, batch, H, W);
    if (bytes < need) return cfail(SR_EWORKSPACE, "workspace too small: %zu < %zu bytes", bytes, need);
    cnn_ctx* c = new cnn_ctx{};
    c->B = batch;
    c->H = H;
    c->W = W;
    c->st = (hipStream_t)hip_stream;
    carve_all(c, (char*)workspace, batch, H, W);
    const Net& N = net();
    for (float* buf : {c->params, c->m, c->v, c->grad}) {
        hipError_t e = hipMemsetAsync(buf, 0, N.np * sizeof(float), c->st);
        if (e != hipSuccess) {
            delete c;
            return cfail(SR_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
        }
    }
    pack_weights(c);
    *out = c;
    return SR_OK;
}

int cnn_set_params(cnn_ctx* c, const float* params) {
    if (!c || !params) return cfail(SR_EINVAL, "NULL argument");
    const size_t np = net().np;
    CHIP(hipMemcpyAsync(c->params, params, np * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    CHIP(hipMemsetAsync(c->m, 0, np * sizeof(float), c->st));
    CHIP(hipMemsetAsync(c->v, 0, np * sizeof(float), c->st));
    c->t_adam = 0;
    pack_weights(c);
    CHIP(hipGetLastError());
    return SR_OK;
}

int cnn_get_params(cnn_ctx* c, float* params) {
    if (!c || !params) return cfail(SR_EINVAL, "NULL argument");
    CHIP(hipMemcpyAsync(params, c->params, net().np * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    return SR_OK;
}

int cnn_forward(cnn_ctx* c, const float* f, const float* g, const float* phi0, int32_t n, float clip,
                float* phi_pred) {
    if (!c || !f || !g || !phi0) return cfail(SR_EINVAL, "NULL argument");
    if (n < 1 || n > c->B) return cfail(SR_EINVAL, "n = %d outside [1, %d]", n, c->B);
    if (!(clip > 0.f) || !std::isfinite(clip)) return cfail(SR_EINVAL, "clip must be positive and finite");
    const size_t P0 = (size_t)n * c->H * c->W;
    hipStream_t st = c->st;
    k_input<<<blocks(P0), 256, 0, st>>>(f, g, phi0, (int)P0, clip, c->x0);
    conv_fwd(c, L0a, {c->x0, 4, 0}, false, c->aL0a, 16, 0, n);
    conv_fwd(c, L0b, {c->aL0a, 16, 0}, false, c->C0, 32, 16, n);
    pool(c, {c->C0, 32, 16}, 16, 1, c->p0, n);
    conv_fwd(c, L1a, {c->p0, 16, 0}, false, c->aL1a, 32, 0, n);
    conv_fwd(c, L1b, {c->aL1a, 32, 0}, false, c->C1, 64, 32, n);
    pool(c, {c->C1, 64, 32}, 32, 2, c->p1, n);
    conv_fwd(c, L2a, {c->p1, 32, 0}, false, c->aL2a, 64, 0, n);
    conv_fwd(c, L2b, {c->aL2a, 64, 0}, false, c->C2, 128, 64, n);
    pool(c, {c->C2, 128, 64}, 64, 3, c->p2, n);
    conv_fwd(c, L3a, {c->p2, 64, 0}, false, c->aL3a, 128, 0, n);
    conv_fwd(c, L3b, {c->aL3a, 128, 0}, false, c->bott, 128, 0, n);
    conv_fwd(c, U2, {c->bott, 128, 0}, true, c->C2, 128, 0, n);
    conv_fwd(c, D2, {c->C2, 128, 0}, false, c->d2, 64, 0, n);
    conv_fwd(c, U1, {c->d2, 64, 0}, true, c->C1, 64, 0, n);
    conv_fwd(c, D1, {c->C1, 64, 0}, false, c->d1, 32, 0, n);
    conv_fwd(c, U0, {c->d1, 32, 0}, true, c->C0, 32, 0, n);
    conv_fwd(c, D0, {c->C0, 32, 0}, false, c->d0, 16, 0, n);
    k_head<<<blocks(P0), 256, 0, st>>>(c->d0, c->params + net().head_w, (int)P0, clip, c->y, phi_pred);
    CHIP(hipGetLastError());
    c->n_last = n;
    c->n_grad = 0;
    c->clip_last = clip;
    return SR_OK;
}

int cnn_get_activation(cnn_ctx* c, int32_t which, float* out) {
    if (!c || !out) return cfail(SR_EINVAL, "NULL argument");
    if (c->n_last < 1) return cfail(SR_ESTATE, "cnn_get_activation before cnn_forward");
    if (which < 0 || which > 18 + kConv) return cfail(SR_EINVAL, "which = %d outside [0, %d]", which, 18 + kConv);
    const int n = c->n_last;
    const size_t P0 = (size_t)n * c->H * c->W;
    if (which > 18) {
        if (c->n_grad != n) return cfail(SR_ESTATE, "no cnn_backward since the last cnn_forward");
        const LayerDesc& d = net().L[which - 19];
        const int P = (int)(P0 >> (2 * d.level));
        k_unpack<<<blocks((size_t)P * d.cout), 256, 0, c->st>>>(c->dz[which - 19], d.cout, 0, d.cout, P, out);
        CHIP(hipGetLastError());
    } else if (which == 15)
        CHIP(hipMemcpyAsync(out, c->y, P0 * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    else {
        struct View {
            const uint16_t* p;
            int stride, off, C, level;
        };
        const View v[19] = {{c->aL0a, 16, 0, 16, 0}, {c->C0, 32, 16, 16, 0},  {c->aL1a, 32, 0, 32, 1},
                            {c->C1, 64, 32, 32, 1},  {c->aL2a, 64, 0, 64, 2}, {c->C2, 128, 64, 64, 2},
                            {c->aL3a, 128, 0, 128, 3}, {c->bott, 128, 0, 128, 3}, {c->C2, 128, 0, 64, 2},
                            {c->d2, 64, 0, 64, 2},   {c->C1, 64, 0, 32, 1},   {c->d1, 32, 0, 32, 1},
                            {c->C0, 32, 0, 16, 0},   {c->d0, 16, 0, 16, 0},   {c->x0, 4, 0, 4, 0},
                            {nullptr, 0, 0, 0, 0},   {c->p0, 16, 0, 16, 1},   {c->p1, 32, 0, 32, 2},
                            {c->p2, 64, 0, 64, 3}};
        const View& w = v[which];
        const int P = (int)(P0 >> (2 * w.level));
        k_unpack<<<blocks((size_t)P * w.C), 256, 0, c->st>>>(w.p, w.stride, w.off, w.C, P, out);
        CHIP(hipGetLastError());
    }
    return SR_OK;
}

int cnn_backward(cnn_ctx* c, const float* target, float clip, double* loss, float* grad_out) {
    if (!c || !target) return cfail(SR_EINVAL, "NULL argument");
    if (c->n_last < 1) return cfail(SR_ESTATE, "cnn_backward before cnn_forward");
    if (!(clip > 0.f) || !std::isfinite(clip)) return cfail(SR_EINVAL, "clip must be positive and finite");
    const Net& N = net();
    const int n = c->n_last;
    const size_t P0 = (size_t)n * c->H * c->W;
    hipStream_t st = c->st;
    const unsigned hb = blocks(P0);
    k_head_back<<<hb, 256, 0, st>>>(c->d0, c->y, target, c->params + N.head_w, (int)P0, clip, c->dz[D0],
                                    c->hpart);
    k_reduce_head<<<kHeadPart, 256, 0, st>>>(c->hpart, (int)hb, c->grad + N.head_w, c->grad + N.head_b, c->loss,
                                             1.f / (float)P0);
    // decoder
    conv_dgrad(c, D0, c->dcat0, n);
    conv_wgrad(c, D0, {c->C0, 32, 0}, false, n);
    mask(c, U0, c->dcat0, 32, 0, false, nullptr, {c->C0, 32, 0}, n);
    conv_dgrad(c, U0, c->T0, n);
    conv_wgrad(c, U0, {c->d1, 32, 0}, true, n);
    mask(c, D1, c->T0, 32, 0, true, nullptr, {c->d1, 32, 0}, n);
    conv_dgrad(c, D1, c->dcat1, n);
    conv_wgrad(c, D1, {c->C1, 64, 0}, false, n);
    mask(c, U1, c->dcat1, 64, 0, false, nullptr, {c->C1, 64, 0}, n);
    conv_dgrad(c, U1, c->T0, n);
    conv_wgrad(c, U1, {c->d2, 64, 0}, true, n);
    mask(c, D2, c->T0, 64, 0, true, nullptr, {c->d2, 64, 0}, n);
    conv_dgrad(c, D2, c->dcat2, n);
    conv_wgrad(c, D2, {c->C2, 128, 0}, false, n);
    mask(c, U2, c->dcat2, 128, 0, false, nullptr, {c->C2, 128, 0}, n);
    conv_dgrad(c, U2, c->T0, n);
    conv_wgrad(c, U2, {c->bott, 128, 0}, true, n);
    // encoder
    mask(c, L3b, c->T0, 128, 0, true, nullptr, {c->bott, 128, 0}, n);
    conv_dgrad(c, L3b, c->T1, n);
    conv_wgrad(c, L3b, {c->aL3a, 128, 0}, false, n);
    mask(c, L3a, c->T1, 128, 0, false, nullptr, {c->aL3a, 128, 0}, n);
    conv_dgrad(c, L3a, c->T0, n);
    conv_wgrad(c, L3a, {c->p2, 64, 0}, false, n);
    mask(c, L2b, c->dcat2, 128, 64, false, c->T0, {c->C2, 128, 64}, n);
    conv_dgrad(c, L2b, c->T1, n);
    conv_wgrad(c, L2b, {c->aL2a, 64, 0}, false, n);
    mask(c, L2a, c->T1, 64, 0, false, nullptr, {c->aL2a, 64, 0}, n);
    conv_dgrad(c, L2a, c->T0, n);
    conv_wgrad(c, L2a, {c->p1, 32, 0}, false, n);
    mask(c, L1b, c->dcat1, 64, 32, false, c->T0, {c->C1, 64, 32}, n);
    conv_dgrad(c, L1b, c->T1, n);
    conv_wgrad(c, L1b, {c->aL1a, 32, 0}, false, n);
    mask(c, L1a, c->T1, 32, 0, false, nullptr, {c->aL1a, 32, 0}, n);
    conv_dgrad(c, L1a, c->T0, n);
    conv_wgrad(c, L1a, {c->p0, 16, 0}, false, n);
    mask(c, L0b, c->dcat0, 32, 16, false, c->T0, {c->C0, 32, 16}, n);
    conv_dgrad(c, L0b, c->T1, n);
    conv_wgrad(c, L0b, {c->aL0a, 16, 0}, false, n);
    mask(c, L0a, c->T1, 16, 0, false, nullptr, {c->aL0a, 16, 0}, n);
    conv_wgrad(c, L0a, {c->x0, 4, 0}, false, n);
    CHIP(hipGetLastError());
    c->n_grad = n;
    if (grad_out) CHIP(hipMemcpyAsync(grad_out, c->grad, N.np * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (loss) {
        float lf = 0.f;
        CHIP(hipMemcpyAsync(&lf, c->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        CHIP(hipStreamSynchronize(st));
        *loss = lf;
    }
    return SR_OK;
}

int cnn_adam_step(cnn_ctx* c, float lr, float beta1, float beta2, float eps) {
    if (!c) return cfail(SR_EINVAL, "NULL context");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return cfail(SR_EINVAL, "bad Adam hyper-parameters");
    const size_t np = net().np;
    c->t_adam += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, c->t_adam)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, c->t_adam)));
    k_adam<<<blocks(np), 256, 0, c->st>>>(c->params, c->m, c->v, c->grad, (int)np, lr, beta1, beta2, eps, c1, c2);
    pack_weights(c);
    CHIP(hipGetLastError());
    return SR_OK;
}

void cnn_destroy(cnn_ctx* c) { delete c; }

}  // extern "C"
