// AOS solve of the phi sub-problem with constant A_l (the paper's alternative
// to the FFT solve, end of Sec. 4, in the form of eqs 18 and 20):
//   (1 - 2 tau mu D_l) v_l = F,  l = 1 (along rows index i), 2 (along j),
//   phi^{k+1,s+1} = (v_1 + v_2) / 2,
// with D_l the periodic second difference and F = phi_s + tau (N + D) the
// right-hand side of eq (37).  Each 1-D operator is circulant, symmetric and
// strictly diagonally dominant; its inverse is the circulant whose entries
// c_k decay like r^|k| (r < 1).  The host computes them in FP64 and keeps
// |k| <= K with c_K below 1e-9 c_0, so v_l is a (2K+1)-tap convolution along
// direction l, exact to that truncation (far below FP32 rounding).  The
// right-hand-side kernel delivers r = tau (N + D + mu Lap phi_s); this kernel
// forms F = phi_s + r - tau mu Lap phi_s on a tile and its halo in LDS and
// applies both convolutions.  With Neumann boundaries (mirror ghosts) the
// 1-D operator's inverse is the restriction of the 2n-periodic circulant's
// inverse to the mirror extension of F, so the same convolution with the
// taps of period 2n, read through mirrored indices, is the exact solve.  Two kernels: a gather kernel (one thread per
// output, taps read per output from LDS) for grids below 2048^2, where it
// keeps enough waves in flight, and a sliding (scatter) kernel for larger
// grids, which reads each source once per line.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <vector>

#include "sr_aos.hpp"
#include "sr_device.hpp"

namespace sr {

namespace {
constexpr int kTapOff = 104;                   // mirrored table: T[m] at index m + kTapOff
constexpr int kTapLen = 2 * kTapOff;           // covers |m| <= kAosMaxK + 32 + 4
// device tap buffer: c_x[0..kAosMaxK], c_y[0..kAosMaxK], (pad to 4), T_x[kTapLen], T_y[kTapLen]
constexpr int kOffTx = (2 * (kAosMaxK + 1) + 3) & ~3, kOffTy = kOffTx + kTapLen;
static_assert(kOffTx % 4 == 0 && kTapOff % 4 == 0 && kTapLen % 4 == 0, "float4-aligned tables");
static_assert(kAosTapFloats == kOffTy + kTapLen, "tap buffer size");

// ---- gather kernel: tile 16 x 64, one thread per output -------------------
constexpr int kGW = 64, kGH = 16, kGThreads = 256;

// F = phi + r - tau mu Lap phi on the cross-shaped extended tile (rows
// i0-Kx .. i0+TH+Kx, columns j0-Ky .. j0+64+Ky, periodic), then
// out = (sum_k cx[|k|] F(i+k, j) + sum_k cy[|k|] F(i, j+k)) / 2.
template <int BC>
__global__ __launch_bounds__(kGThreads) void k_aos_gather(const float* __restrict__ rhs,
                                                           const float* __restrict__ phi, float* __restrict__ out,
                                                           const float* __restrict__ taps, int Kx, int Ky,
                                                           float taumu, int M, int N, DevScal* sc) {
    const int z = blockIdx.z;
    if (!sc[z].active) return;
    const size_t MN = (size_t)M * N;
    rhs += z * MN;
    phi += z * MN;
    out += z * MN;
    const float* cx = taps;
    const float* cy = taps + kAosMaxK + 1;
    extern __shared__ float sF[];
    const int EH = kGH + 2 * Kx, EW = kGW + 2 * Ky;
    const int i0 = blockIdx.y * kGH, j0 = blockIdx.x * kGW;
    for (int e = threadIdx.x; e < EH * EW; e += blockDim.x) {
        const int ei = e / EW, ej = e - ei * EW;
        const int ei_ = ei - Kx, ej_ = ej - Ky;
        // only the cross-shaped part is read by the convolutions
        if ((ei_ < 0 || ei_ >= kGH) && (ej_ < 0 || ej_ >= kGW)) continue;
        const int gi = bidx<BC>(i0 + ei_, M), gj = bidx<BC>(j0 + ej_, N);
        const size_t o = (size_t)gi * N + gj;
        const float p = phi[o];
        const float lap = (phi[(size_t)bidx<BC>(gi - 1, M) * N + gj] + phi[(size_t)bidx<BC>(gi + 1, M) * N + gj]) +
                          (phi[(size_t)gi * N + bidx<BC>(gj - 1, N)] + phi[(size_t)gi * N + bidx<BC>(gj + 1, N)]) -
                          4.0f * p;
        sF[e] = p + (rhs[o] - taumu * lap);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kGH * kGW; e += blockDim.x) {
        const int i = e / kGW, j = e - i * kGW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= M || gj >= N) continue;
        const float* col = sF + (i + Kx) * EW + (j + Ky);
        float v1 = cx[0] * col[0], v2 = cy[0] * col[0];
        for (int k = 1; k <= Kx; ++k) v1 += cx[k] * (col[-k * EW] + col[k * EW]);
        for (int k = 1; k <= Ky; ++k) v2 += cy[k] * (col[-k] + col[k]);
        out[(size_t)gi * N + gj] = 0.5f * (v1 + v2);
    }
}

size_t gather_lds_bytes(int Kx, int Ky) { return sizeof(float) * (size_t)(kGH + 2 * Kx) * (kGW + 2 * Ky); }

// ---- sliding kernel: tile TH x TW, TW threads -----------------------------
// Each direction is a scatter convolution: a thread streams the sources of
// its line once and adds each, times the tap of its offset, into TH
// accumulators.  The offset of a source to an output is the same on every
// lane at every step, so the taps are wave-uniform loads from the mirrored
// tables (scalar loads).
//   vertical (along i):   thread j streams rows -K4x .. TH+K4x-1 of its
//                         column, forming F from phi and r on the fly;
//   horizontal (along j): thread (i, s) streams the columns of row i around
//                         its segment of TH columns, reading F from LDS.
// Taps beyond K are zero, so K rounded up to 4 (K4) reads a few sources at
// zero weight; groups of 4 outputs whose offsets all lie beyond K for a
// block of 4 sources are skipped.
template <int TH>
__device__ __forceinline__ void slide4(float (&acc)[TH], const float* __restrict__ T, int r, const float (&f)[4],
                                       int K) {
    // acc[i] += T[r + q - i] f[q], q = 0..3, from the window T[r - TH .. r + 3]
    const float4* T4 = reinterpret_cast<const float4*>(T + kTapOff + r - TH);
    float t[TH + 4];
#pragma unroll
    for (int u = 0; u < (TH + 4) / 4; ++u) {
        const float4 v = T4[u];
        t[4 * u] = v.x;
        t[4 * u + 1] = v.y;
        t[4 * u + 2] = v.z;
        t[4 * u + 3] = v.w;
    }
#pragma unroll
    for (int g = 0; g < TH / 4; ++g) {
        // offsets r + q - i for i in [4g, 4g + 3], q in [0, 3]: skip if all beyond K
        if (r + 3 - 4 * g < -K || r - 4 * g - 3 > K) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 4 * g; i < 4 * g + 4; ++i) acc[i] = __builtin_fmaf(t[TH + q - i], f[q], acc[i]);
    }
}

template <int TH, int TW, int BC>
__global__ __launch_bounds__(TW) void k_aos_slide(const float* __restrict__ rhs, const float* __restrict__ phi,
                                                  float* __restrict__ out, const float* __restrict__ taps, int Kx,
                                                  int Ky, float taumu, int M, int N, DevScal* sc) {
    static_assert(TH % 4 == 0 && TW % TH == 0 && TW % 64 == 0, "tile shape");
    const int z = blockIdx.z;
    if (!sc[z].active) return;
    const uint32_t MN = (uint32_t)M * (uint32_t)N;   // M, N <= 4096
    rhs += (size_t)z * MN;
    phi += (size_t)z * MN;
    out += (size_t)z * MN;
    const float* Tx = taps + kOffTx;
    const float* Ty = taps + kOffTy;
    const int K4x = (Kx + 3) & ~3, K4y = (Ky + 3) & ~3;
    const int pitch = ((TW + 2 * K4y + 63) & ~63) + 4;   // 4 mod 64 words: conflict-free float4 rows
    extern __shared__ float4 lds4[];
    float* sH = reinterpret_cast<float*>(lds4);           // F on rows 0..TH-1, columns -K4y .. TW+K4y-1
    const int tid = threadIdx.x;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;

    // horizontal halo of F: rows 0..TH-1, columns -K4y..-1 and TW..TW+K4y-1
#pragma unroll 2
    for (int e = tid; e < 2 * K4y * TH; e += TW) {
        const int i = e / (2 * K4y), c0 = e - i * 2 * K4y;
        const int c = c0 < K4y ? c0 - K4y : TW + (c0 - K4y);
        const int gi = bidx<BC>(i0 + i, M), gj = bidx<BC>(j0 + c, N);
        const uint32_t o = (uint32_t)gi * N + gj;
        const float p = phi[o];
        const float lap = (phi[(uint32_t)bidx<BC>(gi - 1, M) * N + gj] + phi[(uint32_t)bidx<BC>(gi + 1, M) * N + gj]) +
                          (phi[(uint32_t)gi * N + bidx<BC>(gj - 1, N)] + phi[(uint32_t)gi * N + bidx<BC>(gj + 1, N)]) -
                          4.0f * p;
        sH[i * pitch + K4y + c] = p + (rhs[o] - taumu * lap);
    }

    // vertical pass: thread = column
    float accV[TH];
#pragma unroll
    for (int i = 0; i < TH; ++i) accV[i] = 0.0f;
    {
        // the loads of the next block of 4 rows are issued before the
        // arithmetic of the current one
        const int gjs = bidx<BC>(j0 + tid, N);
        const uint32_t gj = gjs, gl = bidx<BC>(gjs - 1, N), gr = bidx<BC>(gjs + 1, N);
        float pu = phi[(uint32_t)bidx<BC>(i0 - K4x - 1, M) * N + gj];
        float pc = phi[(uint32_t)bidx<BC>(i0 - K4x, M) * N + gj];
        float nd[4], nl[4], nr[4], nh[4];
        auto load_block = [&](int r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t row = (uint32_t)bidx<BC>(i0 + r + q, M) * N;
                nd[q] = phi[(uint32_t)bidx<BC>(i0 + r + q + 1, M) * N + gj];
                nl[q] = phi[row + gl];
                nr[q] = phi[row + gr];
                nh[q] = rhs[row + gj];
            }
        };
        load_block(-K4x);
        for (int r = -K4x; r < TH + K4x; r += 4) {
            float cd[4], cl[4], cr[4], ch[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                cd[q] = nd[q];
                cl[q] = nl[q];
                cr[q] = nr[q];
                ch[q] = nh[q];
            }
            if (r + 4 < TH + K4x) load_block(r + 4);
            float f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float lap = (pu + cd[q]) + (cl[q] + cr[q]) - 4.0f * pc;
                f[q] = pc + (ch[q] - taumu * lap);
                pu = pc;
                pc = cd[q];
                if (r + q >= 0 && r + q < TH) sH[(r + q) * pitch + K4y + tid] = f[q];
            }
            slide4<TH>(accV, Tx, r, f, Kx);
        }
    }
    __syncthreads();

    // horizontal pass: thread = (row i, segment s of TH columns)
    const int hi = tid % TH, hs = tid / TH;
    float accH[TH];
#pragma unroll
    for (int o = 0; o < TH; ++o) accH[o] = 0.0f;
    {
        const float4* row4 = reinterpret_cast<const float4*>(sH + hi * pitch + K4y + hs * TH);
        for (int c = -K4y; c < TH + K4y; c += 4) {
            const float4 v = row4[c / 4];
            const float f[4] = {v.x, v.y, v.z, v.w};
            slide4<TH>(accH, Ty, c, f, Ky);
        }
    }
    __syncthreads();
    {
        float4* dst = reinterpret_cast<float4*>(sH + hi * pitch + K4y + hs * TH);
#pragma unroll
        for (int u = 0; u < TH / 4; ++u)
            dst[u] = make_float4(accH[4 * u], accH[4 * u + 1], accH[4 * u + 2], accH[4 * u + 3]);
    }
    __syncthreads();
    const int gj = j0 + tid;
    if (gj < N) {
#pragma unroll
        for (int i = 0; i < TH; ++i)
            if (i0 + i < M) out[(uint32_t)(i0 + i) * N + gj] = 0.5f * (accV[i] + sH[i * pitch + K4y + tid]);
    }
}

constexpr int kSH = 16, kSW = 256;

size_t slide_lds_bytes(int Ky) {
    const int K4y = (Ky + 3) & ~3;
    const int pitch = ((kSW + 2 * K4y + 63) & ~63) + 4;
    return sizeof(float) * (size_t)kSH * pitch;
}

// The sliding kernel from 2048^2 points on; SR_AOS_KERNEL=gather|slide
// forces one (read at each launch; a graph keeps the kernel it captured).
bool use_slide(int M, int N) {
    const char* e = std::getenv("SR_AOS_KERNEL");
    if (e && !std::strcmp(e, "gather")) return false;
    if (e && !std::strcmp(e, "slide")) return true;
    return (size_t)M * N >= ((size_t)1 << 22);
}
}  // namespace

int aos_taps(int n, double tau, double mu, float* taps) {
    // c_k = (1/n) sum_m cos(2 pi m k / n) / (1 + 2 tau mu (2 - 2 cos(2 pi m / n)))
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<double> c(n / 2 + 1);
    for (int k = 0; k <= n / 2; ++k) {
        double s = 0.0;
        for (int m = 0; m < n; ++m)
            s += std::cos(two_pi * (double)m * k / n) / (1.0 + 2.0 * tau * mu * (2.0 - 2.0 * std::cos(two_pi * m / n)));
        c[k] = s / n;
    }
    int K = 0;
    while (K < n / 2 && K < kAosMaxK && std::fabs(c[K + 1]) > 1e-9 * c[0]) ++K;
    // the offsets -K..K must cover every entry above the cut exactly once
    if (2 * K + 1 > n || (K < n / 2 && std::fabs(c[K + 1]) > 1e-9 * c[0])) return -1;
    for (int k = 0; k <= kAosMaxK; ++k) taps[k] = k <= K ? (float)c[k] : 0.0f;
    return K;
}

int aos_tap_buffer(int M, int N, double tau, double mu, int bc, float* buf, int* Kx, int* Ky) {
    for (int i = 0; i < kAosTapFloats; ++i) buf[i] = 0.0f;
    const int per = bc == 1 ? 2 : 1;   // Neumann: the circulant of the 2n-point mirror extension
    *Kx = aos_taps(per * M, tau, mu, buf);
    *Ky = aos_taps(per * N, tau, mu, buf + kAosMaxK + 1);
    if (*Kx < 0 || *Ky < 0) return -1;
    for (int m = -kTapOff; m < kTapOff; ++m) {
        const int am = m < 0 ? -m : m;
        buf[kOffTx + kTapOff + m] = am <= *Kx ? buf[am] : 0.0f;
        buf[kOffTy + kTapOff + m] = am <= *Ky ? buf[kAosMaxK + 1 + am] : 0.0f;
    }
    return 0;
}

size_t aos_lds_bytes(int Kx, int Ky) {
    const size_t a = gather_lds_bytes(Kx, Ky), b = slide_lds_bytes(Ky);
    return a > b ? a : b;
}

void configure_aos() {
    static bool done = false;
    if (done) return;
    done = true;
    for (const void* f : {(const void*)k_aos_gather<0>, (const void*)k_aos_gather<1>})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
    for (const void* f : {(const void*)k_aos_slide<kSH, kSW, 0>, (const void*)k_aos_slide<kSH, kSW, 1>})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
}

void launch_aos(int M, int N, int bc, const float* rhs, const float* phi_in, float* phi_out, const float* taps,
                int Kx, int Ky, float taumu, int nz, DevScal* sc, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const bool slide = use_slide(M, N);
    auto kern = slide ? (bc ? k_aos_slide<kSH, kSW, 1> : k_aos_slide<kSH, kSW, 0>)
                      : (bc ? k_aos_gather<1> : k_aos_gather<0>);
    const int TH = slide ? kSH : kGH, TW = slide ? kSW : kGW, threads = slide ? kSW : kGThreads;
    const dim3 grid((N + TW - 1) / TW, (M + TH - 1) / TH, nz);
    const uint32_t lds = (uint32_t)(slide ? slide_lds_bytes(Ky) : gather_lds_bytes(Kx, Ky));
    if (ev0)
        hipExtLaunchKernelGGL(kern, grid, dim3(threads), lds, st, ev0, ev1, 0u, rhs, phi_in, phi_out, taps, Kx, Ky,
                              taumu, M, N, sc);
    else
        hipLaunchKernelGGL(kern, grid, dim3(threads), lds, st, rhs, phi_in, phi_out, taps, Kx, Ky, taumu, M, N, sc);
}

}  // namespace sr
