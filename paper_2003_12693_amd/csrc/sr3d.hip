// 3-D Split Bregman solver of the Self-repelling Snake model: the 2-D method
// with a third axis (the paper's volume application, Sec. 5, Fig. 6).  One
// outer iteration (Algorithm 1) on an M x N x P volume, periodic:
//   S x [ the cube window of u = w h(phi_s) (3 components) as three
//         separable passes (k, forming u in LDS; j; i),
//         r = tau (N(phi_s) + mu div(b - w) + mu Lap phi_s) (eq 37 in
//         increment form) formed inside the first pass of the 3-D FFT solve
//         (eqs 30-33): forward along k (real input, half spectrum), along j,
//         along i with the division by the symbol and the inverse along i,
//         inverse along j, inverse along k with phi_{s+1} = phi_s + Re / (M N P) ]
//   then u = w^k h(phi^{k+1}) and the window again, and the w step: B of
//   eq (41), the eq (42) gate and the projection of eq (40) (B / |B|), b of
//   eq (23), per voxel.
// The Gaussian, edge and w-step kernels are per voxel; the window passes and
// the FFTs (the first with the rhs) stage lines or tiles in LDS.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sr3d.h"
#include "sr_device.hpp"

namespace sr {
int api_fail(int code, const char* msg);
}

using sr::KParams;

namespace {

constexpr int kT = 256;   // threads of the per-voxel kernels
constexpr int kLines = 8;          // lines per workgroup of the FFT along k (contiguous)
constexpr int kStridedLines = 16;  // lines per workgroup of the FFTs along i and j (strided)

struct Gauss3 {
    float k[2 * sr::kMaxGaussR + 1];
    int r;
};

__device__ __forceinline__ int wrp(int i, int n) { return i & (n - 1); }

__device__ __forceinline__ size_t vox(int i, int j, int k, int N, int P) { return ((size_t)i * N + j) * P + k; }

// One axis of the cube Gaussian (eq 1), periodic.
__global__ __launch_bounds__(kT) void k3_gauss(const float* __restrict__ src, float* __restrict__ dst, int M, int N,
                                               int P, int axis, Gauss3 t) {
    const size_t v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= (size_t)M * N * P) return;
    const int k = (int)(v % P), j = (int)((v / P) % N), i = (int)(v / ((size_t)N * P));
    float acc = 0.0f;
    for (int q = -t.r; q <= t.r; ++q) {
        const size_t o = axis == 0 ? vox(wrp(i + q, M), j, k, N, P)
                                   : axis == 1 ? vox(i, wrp(j + q, N), k, N, P) : vox(i, j, wrp(k + q, P), N, P);
        acc += t.k[q + t.r] * src[o];
    }
    dst[v] = acc;
}

// g = 1 / (1 + rho |grad fs|^s), central differences.
__global__ __launch_bounds__(kT) void k3_edge(const float* __restrict__ fs, float* __restrict__ g, int M, int N, int P,
                                              float rho, int s_exp) {
    const size_t v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= (size_t)M * N * P) return;
    const int k = (int)(v % P), j = (int)((v / P) % N), i = (int)(v / ((size_t)N * P));
    const float gx = 0.5f * (fs[vox(wrp(i + 1, M), j, k, N, P)] - fs[vox(wrp(i - 1, M), j, k, N, P)]);
    const float gy = 0.5f * (fs[vox(i, wrp(j + 1, N), k, N, P)] - fs[vox(i, wrp(j - 1, N), k, N, P)]);
    const float gz = 0.5f * (fs[vox(i, j, wrp(k + 1, P), N, P)] - fs[vox(i, j, wrp(k - 1, P), N, P)]);
    const float m2 = gx * gx + gy * gy + gz * gz;
    g[v] = 1.0f / (1.0f + rho * (s_exp == 2 ? m2 : sqrtf(m2)));
}

// phi^0, w^0 = grad phi^0 (forward differences), b^0 = 0.
__global__ __launch_bounds__(kT) void k3_init(const float* __restrict__ phi0, float* __restrict__ phi,
                                              float* __restrict__ W, float* __restrict__ B, int M, int N, int P) {
    const size_t n = (size_t)M * N * P, v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    const int k = (int)(v % P), j = (int)((v / P) % N), i = (int)(v / ((size_t)N * P));
    const float p = phi0[v];
    phi[v] = p;
    W[v] = phi0[vox(wrp(i + 1, M), j, k, N, P)] - p;
    W[n + v] = phi0[vox(i, wrp(j + 1, N), k, N, P)] - p;
    W[2 * n + v] = phi0[vox(i, j, wrp(k + 1, P), N, P)] - p;
    B[v] = 0.0f;
    B[n + v] = 0.0f;
    B[2 * n + v] = 0.0f;
}

// The first (k) axis of the cube window with u = w h(phi) formed on the fly:
// dst = sum_q a_q u(x + q e_k), three components.  A workgroup of kT
// voxels holds whole k-lines (P <= kT, both powers of two), so u is formed
// once per voxel in LDS and every tap, wrapped within its line, reads it
// there.
__global__ __launch_bounds__(kT) void k3_win_u(const float* __restrict__ W, const float* __restrict__ phi,
                                               float* __restrict__ dst, int M, int N, int P, KParams kp) {
    __shared__ float su[3][kT];
    const size_t n = (size_t)M * N * P, v = (size_t)blockIdx.x * kT + threadIdx.x;   // n is a multiple of kT
    const int tid = threadIdx.x;
    const float h = sr::band_h(phi[v], kp);
    su[0][tid] = W[v] * h;
    su[1][tid] = W[n + v] * h;
    su[2][tid] = W[2 * n + v] * h;
    __syncthreads();
    const int k = (int)(v % P);
    const int line = tid - k;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int q = -kp.R; q <= kp.R; ++q) {
        const int o = line + wrp(k + q, P);
        const float a = kp.taps[q + kp.R];
        a0 += a * su[0][o];
        a1 += a * su[1][o];
        a2 += a * su[2][o];
    }
    dst[v] = a0;
    dst[n + v] = a1;
    dst[2 * n + v] = a2;
}

// The i or j axis of the cube window on a tile: TA positions along the axis
// times KT consecutive k (KT = min(64, P)), staged with the R-halo along the
// axis in LDS (loads run along k), three components: dst = sum_q a_q
// src(x + q e_axis), q ascending.
constexpr int kWinTA = 16;
constexpr int kWinKT = 64;

static_assert((kWinTA + 2 * sr::kMaxR) * kWinKT % kT == 0, "whole load rounds");
__global__ __launch_bounds__(kT) void k3_win_tile(const float* __restrict__ src, float* __restrict__ dst, int M,
                                                  int N, int P, int axis, KParams kp) {
    __shared__ float sv[3][(kWinTA + 2 * sr::kMaxR) * kWinKT];
    const size_t n = (size_t)M * N * P;
    const int KT = P < kWinKT ? P : kWinKT;
    const int La = axis == 0 ? M : N;
    const int TA = La < kWinTA ? La : kWinTA;
    const int R = kp.R;
    const int k0 = blockIdx.x * KT, a0 = blockIdx.y * TA, other = blockIdx.z;   // other: j (axis 0) or i (axis 1)
    auto at = [&](int a, int k) -> size_t {   // a: index along the axis (wrapped), k: absolute
        return axis == 0 ? vox(a, other, k, N, P) : vox(other, a, k, N, P);
    };
    const int EH = TA + 2 * R;
    // every load of the tile is issued before the first is used (a runtime
    // loop would wait for each round's loads before issuing the next)
    constexpr int kRounds = (kWinTA + 2 * sr::kMaxR) * kWinKT / kT;
    float t0[kRounds], t1[kRounds], t2[kRounds];
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int e = threadIdx.x + it * kT;
        if (e < EH * KT) {
            const int ea = e / KT, ek = e - ea * KT;
            const size_t o = at(wrp(a0 - R + ea, La), k0 + ek);
            t0[it] = src[o];
            t1[it] = src[n + o];
            t2[it] = src[2 * n + o];
        }
    }
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int e = threadIdx.x + it * kT;
        if (e < EH * KT) {
            sv[0][e] = t0[it];
            sv[1][e] = t1[it];
            sv[2][e] = t2[it];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TA * KT; e += kT) {
        const int ta = e / KT, tk = e - ta * KT;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        for (int q = -R; q <= R; ++q) {
            const int l = (ta + R + q) * KT + tk;
            const float a = kp.taps[q + R];
            c0 += a * sv[0][l];
            c1 += a * sv[1][l];
            c2 += a * sv[2][l];
        }
        const size_t o = at(a0 + ta, k0 + tk);
        dst[o] = c0;
        dst[n + o] = c1;
        dst[2 * n + o] = c2;
    }
}

// r = tau (-gamma g |w| delta' + alpha g delta + 2 beta h' w.v + mu div(b - w) + mu Lap phi).
// w and b are fixed over the inner steps of an outer iteration: the first
// inner step (first = 1) forms D = div(b - w) and stores it, the others
// read it.  The force vanishes outside the band |phi| <= l + eps (delta,
// delta' and h' are 0 there), where w, g and v are not read.
// Evaluated at voxel (i, j, k) by the forward k transform, which takes r
// as its input.
__device__ __forceinline__ float rhs_voxel(const float* __restrict__ phi, const float* __restrict__ W,
                                           const float* __restrict__ B, float* __restrict__ D,
                                           const float* __restrict__ g, const float* __restrict__ V, int M, int N,
                                           int P, int i, int j, int k, int first, const KParams& kp) {
    const size_t n = (size_t)M * N * P, v = vox(i, j, k, N, P);
    const size_t oi = vox(wrp(i - 1, M), j, k, N, P), oj = vox(i, wrp(j - 1, N), k, N, P),
                 ok = vox(i, j, wrp(k - 1, P), N, P);
    const float p = phi[v];
    const float lap = (phi[vox(wrp(i + 1, M), j, k, N, P)] + phi[oi]) + (phi[vox(i, wrp(j + 1, N), k, N, P)] + phi[oj]) +
                      (phi[vox(i, j, wrp(k + 1, P), N, P)] + phi[ok]) - 6.0f * p;
    float dv;
    if (first) {
        dv = ((B[v] - W[v]) - (B[oi] - W[oi])) + ((B[n + v] - W[n + v]) - (B[n + oj] - W[n + oj])) +
             ((B[2 * n + v] - W[2 * n + v]) - (B[2 * n + ok] - W[2 * n + ok]));
        D[v] = dv;
    } else {
        dv = D[v];
    }
    const float lim = kp.band_l + kp.eps;
    float force = 0.0f;
    if (p <= lim && p >= -lim) {
        const float w0 = W[v], w1 = W[n + v], w2 = W[2 * n + v];
        float dl, ddl, h, dh;
        sr::dirac_d(p, kp, dl, ddl);
        sr::band_h_dh(p, kp, h, dh);
        const float gv = g[v];
        const float wn = sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
        const float wv = w0 * V[v] + w1 * V[n + v] + w2 * V[2 * n + v];
        force = -kp.gamma * gv * wn * ddl + kp.alpha * gv * dl + 2.0f * kp.beta * dh * wv;
    }
    return kp.tau * (force + kp.mu * dv + kp.mu * lap);
}

// w step: B = grad phi + b + (2 beta / mu) h v, gate (eq 42) and projection
// (eq 40) as B / |B|, b += grad phi - w; in place.
__global__ __launch_bounds__(kT) void k3_wstep(const float* __restrict__ phi, float* __restrict__ W,
                                               float* __restrict__ B, const float* __restrict__ g,
                                               const float* __restrict__ V, int M, int N, int P, KParams kp) {
    const size_t n = (size_t)M * N * P, v = (size_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    const int k = (int)(v % P), j = (int)((v / P) % N), i = (int)(v / ((size_t)N * P));
    const float p = phi[v];
    const float G0 = phi[vox(wrp(i + 1, M), j, k, N, P)] - p;
    const float G1 = phi[vox(i, wrp(j + 1, N), k, N, P)] - p;
    const float G2 = phi[vox(i, j, wrp(k + 1, P), N, P)] - p;
    const float b0 = B[v], b1 = B[n + v], b2 = B[2 * n + v];
    // outside the band |phi| <= l + eps h and delta vanish: B = grad phi + b
    // and the threshold is 0, so v and g are read only inside it
    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, h = 0.0f, thr = 0.0f;
    const float lim = kp.band_l + kp.eps;
    if (p <= lim && p >= -lim) {
        h = sr::band_h(p, kp);
        float H_, dl;
        sr::heav_dirac(p, kp.eps, kp.inv_eps, H_, dl);
        v0 = V[v];
        v1 = V[n + v];
        v2 = V[2 * n + v];
        thr = kp.c_thr * g[v] * dl;
    }
    const float B0 = G0 + b0 + kp.c_rep * h * v0;
    const float B1 = G1 + b1 + kp.c_rep * h * v1;
    const float B2 = G2 + b2 + kp.c_rep * h * v2;
    const float nb = sqrtf(B0 * B0 + B1 * B1 + B2 * B2);
    float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
    if (nb > thr && nb > kp.zero_tol) { w0 = B0 / nb; w1 = B1 / nb; w2 = B2 / nb; }
    W[v] = w0;
    W[n + v] = w1;
    W[2 * n + v] = w2;
    B[v] = b0 + G0 - w0;
    B[n + v] = b1 + G1 - w1;
    B[2 * n + v] = b2 + G2 - w2;
}

// ---- FFT along one axis: G lines of length L per workgroup ---------------
// Stockham (self-sorting) with radix-4 stages, after one radix-2 stage when
// log2 L is odd.  A radix-R stage at sub-transform length Ns takes, for
// butterfly j < L/R, the inputs x[j + r L/R] (r < R), multiplies input r by
// W_L^{r (j mod Ns) L / (R Ns)}, applies the R-point DFT and writes output r
// to y[(j div Ns) R Ns + j mod Ns + r Ns].  A thread runs several
// butterflies of the block per stage.
// mode 1: forward; 2: forward, divide by the symbol of (1 - tau mu Lap),
// inverse; 3: inverse; 4: inverse, real output out = add + scale Re (the
// forward k transform, with real input, is k3_rhs_kfwd).  The volume is real, so the spectrum is kept for k
// frequencies 0..P/2 only: the k pass stores those, the i and j passes
// transform only those lines, and the inverse k pass restores the others as
// complex conjugates.  Along k a line of P real samples runs as a P/2-point
// complex transform of its even (real part) and odd (imaginary part)
// samples, split into the P-point spectrum after it (and joined before the
// inverse).
// Lines of axis 2 are contiguous (kLines per
// workgroup); lines of axes 0 and 1 are strided, and kStridedLines
// neighbours along k share a workgroup so that each load and store touches
// 128-byte runs.
constexpr int fft3_threads(int L, int G) { return G * L / 4 < 1024 ? G * L / 4 : 1024; }

template <int L, int G>
struct FftShape3 {
    static constexpr int T = fft3_threads(L, G);   // threads
    static constexpr int NB2 = G * L / 2 / T;      // radix-2 butterflies per thread
    static constexpr int NB4 = G * L / 4 / T;      // radix-4 butterflies per thread
    static constexpr int NE = G * L / T;           // elements loaded / stored per thread
    static constexpr bool ODD = (__builtin_ctz(L) & 1) != 0;
};

template <int L, int G>
__device__ float2* stockham(float2* a, float2* b, const float2* __restrict__ tw, bool inv) {
    using S = FftShape3<L, G>;
    constexpr int LP = L + 1;
    float2* x = a;
    float2* y = b;
    int Ns = 1;
    if constexpr (S::ODD) {
#pragma unroll
        for (int q = 0; q < S::NB2; ++q) {
            const int u = threadIdx.x + q * S::T;
            const int g = u / (L / 2), bt = u - g * (L / 2);
            const float2 v0 = x[g * LP + bt], v1 = x[g * LP + bt + L / 2];
            y[g * LP + 2 * bt] = sr::cadd(v0, v1);
            y[g * LP + 2 * bt + 1] = sr::csub(v0, v1);
        }
        __syncthreads();
        float2* t = x;
        x = y;
        y = t;
        Ns = 2;
    }
    for (; Ns < L; Ns <<= 2) {
#pragma unroll
        for (int q = 0; q < S::NB4; ++q) {
            const int u = threadIdx.x + q * S::T;
            const int g = u / (L / 4), j = u - g * (L / 4);
            const int kk = j & (Ns - 1);
            const int step = kk * (L / (4 * Ns));
            float2 v0 = x[g * LP + j], v1 = x[g * LP + j + L / 4], v2 = x[g * LP + j + L / 2],
                   v3 = x[g * LP + j + 3 * L / 4];
            if (kk) {
                float2 w1 = tw[step], w2 = tw[2 * step], w3 = tw[3 * step];
                if (inv) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
                v1 = sr::cmul(v1, w1);
                v2 = sr::cmul(v2, w2);
                v3 = sr::cmul(v3, w3);
            }
            const float2 a0 = sr::cadd(v0, v2), a1 = sr::csub(v0, v2), a2 = sr::cadd(v1, v3);
            const float2 d = sr::csub(v1, v3);
            const float2 a3 = inv ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);   // (+-i) d
            const int o = g * LP + ((j - kk) << 2) + kk;
            y[o] = sr::cadd(a0, a2);
            y[o + Ns] = sr::cadd(a1, a3);
            y[o + 2 * Ns] = sr::csub(a0, a2);
            y[o + 3 * Ns] = sr::csub(a1, a3);
        }
        __syncthreads();
        float2* t = x;
        x = y;
        y = t;
    }
    return x;
}

// Forward k transform of a real line of P = 2L samples run as the L-point
// transform Z of z_n = x_2n + i x_2n+1 (line in LDS after the transform):
// X_m = E_m + W_P^m O_m (m = 0..L) from the spectra of the even and odd
// samples, E_m = (Z_m + conj Z_L-m) / 2 and O_m = (Z_m - conj Z_L-m) / 2i
// (indices mod L); X_L = E_0 - O_0.  Cline: the line's half spectrum.
template <int L>
__device__ __forceinline__ void store_k_half(const float2* zline, int pos, float2* __restrict__ Cline,
                                             const float2* __restrict__ twP) {
    const float2 z = zline[pos], zq = zline[(L - pos) & (L - 1)];
    const float2 e = make_float2(0.5f * (z.x + zq.x), 0.5f * (z.y - zq.y));
    const float2 o = make_float2(0.5f * (z.y + zq.y), -0.5f * (z.x - zq.x));
    const float2 wo = sr::cmul(twP[pos], o);
    Cline[pos] = sr::cadd(e, wo);
    if (pos == 0) Cline[L] = sr::csub(e, o);
}

template <int L, int G>
__global__ __launch_bounds__(fft3_threads(L, G)) void k3_fft(float2* __restrict__ C,
                                                             float* __restrict__ rout, const float* __restrict__ radd,
                                                             const float2* __restrict__ twM,
                                                             const float2* __restrict__ twN,
                                                             const float2* __restrict__ twP, int M, int N, int P,
                                                             int Hp, int axis, int mode, float taumu, float scale) {
    using S = FftShape3<L, G>;
    static_assert(S::T % G == 0, "a thread's elements share one line of the block");
    extern __shared__ float2 lds3[];
    constexpr int LP = L + 1;   // line pitch in LDS: strided loads of G lines hit distinct banks
    float2* s0 = lds3;
    float2* s1 = lds3 + G * LP;
    float2* stw = lds3 + 2 * G * LP;   // this axis's twiddle table, L entries
    const int tid = threadIdx.x;
    const int line0 = blockIdx.x * G;
    const float2* tw = axis == 0 ? twM : axis == 1 ? twN : twP;
    // The stages read their twiddles from LDS: from memory, each stage would
    // wait for an L2 round trip before its butterflies.  (The k pass runs
    // L = P/2-point transforms: every second entry of the P-point table.)
    for (int i = tid; i < L; i += S::T) stw[i] = tw[axis == 2 ? 2 * i : i];
    // The spectrum C holds k frequencies 0..P/2 only (the rest follow from
    // those by conjugate symmetry, the volume being real), Hp >= P/2 + 1
    // slots per k-line.  Lines of the strided passes run over every slot;
    // those past P/2 carry zeros and are not stored.
    const int H = P / 2 + 1;
    // mode 2 (axis 0): this thread's elements all lie on line line0 + tid % G
    // (the thread count is a multiple of G); the j and k cosines of that line
    // are loaded with the data
    float cj = 0.0f, ck = 0.0f;
    if (mode == 2) {
        const int l = line0 + tid % G, kk = l % Hp;
        cj = twN[l / Hp].x;
        ck = kk < H ? twP[kk].x : 0.0f;
    }
    // element e of the block -> (line g, position pos), and for the strided
    // passes the line's k slot and the element's address in C
    auto addr = [&](int e, int& g, int& pos, int& kk) -> size_t {
        if (axis == 2) {
            g = e / L;
            pos = e - g * L;
            kk = 0;
            return 0;
        }
        pos = e / G;
        g = e - pos * G;
        const int l = line0 + g;
        kk = l % Hp;
        if (axis == 1) return (size_t)(l / Hp) * N * Hp + (size_t)pos * Hp + kk;
        return (size_t)pos * N * Hp + l;
    };
#pragma unroll
    for (int m = 0; m < S::NE; ++m) {
        const int e = tid + m * S::T;
        int g, pos, kk;
        const size_t o = addr(e, g, pos, kk);
        float2 v;
        if (axis == 2) {
            // mode 4: the inverse of k-line g (P = 2L real samples) as the
            // L-point transform of Z_m = E_m + i O_m, E_m = X_m + conj X_L-m
            // (2x the even samples' spectrum), O_m = (X_m - conj X_L-m) W_P^-m
            const size_t line = (size_t)(line0 + g);
            const float2 xm = C[line * Hp + pos], xq = C[line * Hp + (L - pos)];
            const float2 e = make_float2(xm.x + xq.x, xm.y - xq.y);
            const float2 d = make_float2(xm.x - xq.x, xm.y + xq.y);
            const float2 t = twP[pos];
            const float2 o = make_float2(d.x * t.x + d.y * t.y, d.y * t.x - d.x * t.y);
            v = make_float2(e.x - o.y, e.y + o.x);
        } else {
            v = kk < H ? C[o] : make_float2(0.0f, 0.0f);
        }
        s0[g * LP + pos] = v;
    }
    __syncthreads();
    float2* res = stockham<L, G>(s0, s1, stw, mode >= 3);
    if (mode == 2) {
        // line l = j Hp + k holds frequencies (n, j, k): symbol
        // 1 + tau mu (6 - 2 cos(2 pi n / M) - 2 cos(2 pi j / N) - 2 cos(2 pi k / P))
        float2* other = res == s0 ? s1 : s0;
#pragma unroll
        for (int m = 0; m < S::NE; ++m) {
            const int e = tid + m * S::T;
            const int pos = e / G, gg = e - pos * G;
            const float cs = stw[pos].x + cj + ck;
            const float sym = 1.0f + taumu * (6.0f - 2.0f * cs);
            const float2 z = res[gg * LP + pos];
            res[gg * LP + pos] = make_float2(z.x / sym, z.y / sym);
        }
        __syncthreads();
        res = stockham<L, G>(res, other, stw, true);
    }
#pragma unroll
    for (int m = 0; m < S::NE; ++m) {
        const int e = tid + m * S::T;
        int gg, pos, kk;
        const size_t o = addr(e, gg, pos, kk);
        const float2 z = res[gg * LP + pos];
        if (axis == 2) {   // mode 4: z_n = P (x_2n + i x_2n+1) up to the other axes' factors
            const size_t r = (size_t)(line0 + gg) * P + 2 * pos;
            const float2 ad = *reinterpret_cast<const float2*>(radd + r);
            *reinterpret_cast<float2*>(rout + r) = make_float2(ad.x + scale * z.x, ad.y + scale * z.y);
        } else if (kk < H) {
            C[o] = z;
        }
    }
}

// The right-hand side (rhs_voxel) fused with the forward k transform: each
// k-line's r goes straight into LDS as the transform's input, never to
// memory; the half spectrum is stored as the inverse k pass expects it.
// first: the outer iteration's first inner step (forms D).
template <int L, int G>
__global__ __launch_bounds__(fft3_threads(L, G)) void k3_rhs_kfwd(const float* __restrict__ phi,
                                                                  const float* __restrict__ W,
                                                                  const float* __restrict__ B, float* __restrict__ D,
                                                                  const float* __restrict__ g,
                                                                  const float* __restrict__ V, float2* __restrict__ C,
                                                                  const float2* __restrict__ twP, int M, int N, int P,
                                                                  int Hp, int first, KParams kp) {
    using S = FftShape3<L, G>;
    extern __shared__ float2 lds3[];
    constexpr int LP = L + 1;
    float2* s0 = lds3;
    float2* s1 = lds3 + G * LP;
    float2* stw = lds3 + 2 * G * LP;
    const int tid = threadIdx.x;
    const int line0 = blockIdx.x * G;
    for (int i = tid; i < L; i += S::T) stw[i] = twP[2 * i];
    // consecutive threads on consecutive voxels of a line; voxel k of line
    // gl is component k & 1 of element k / 2 of the line's complex input
#pragma unroll
    for (int m = 0; m < 2 * S::NE; ++m) {
        const int e = tid + m * S::T;
        const int gl = e / (2 * L), k = e - gl * (2 * L);
        const int line = line0 + gl, i = line / N, j = line - i * N;
        reinterpret_cast<float*>(s0 + gl * LP)[k] = rhs_voxel(phi, W, B, D, g, V, M, N, P, i, j, k, first, kp);
    }
    __syncthreads();
    const float2* res = stockham<L, G>(s0, s1, stw, false);
#pragma unroll
    for (int m = 0; m < S::NE; ++m) {
        const int e = tid + m * S::T;
        const int gl = e / L, pos = e - gl * L;
        store_k_half<L>(res + gl * LP, pos, C + (size_t)(line0 + gl) * Hp, twP);
    }
}

std::vector<float2> host_twiddles(int L) {
    std::vector<float2> t(L);
    const double two_pi = 6.283185307179586476925286766559;
    for (int n = 0; n < L; ++n) {
        const double a = two_pi * (double)n / (double)L;
        t[n] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    return t;
}

bool pow2_in(int x) { return x >= 8 && x <= 256 && (x & (x - 1)) == 0; }

// k slots per line of the half spectrum: P/2 + 1 frequencies, rounded up to
// whole groups of strided lines (so that a strided workgroup's lines start
// a 128-byte run)
int half_pitch(int P) { return (P / 2 + 1 + kStridedLines - 1) / kStridedLines * kStridedLines; }

struct Layout3 {
    size_t g, pa, pb, W, B, U, T, D, C, twM, twN, twP, total;
};

Layout3 layout3(int M, int N, int P) {
    Layout3 L{};
    const size_t n = (size_t)M * N * P, pl = sizeof(float) * n;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = (o + bytes + 255) & ~size_t(255); return at; };
    L.g = take(pl);
    L.pa = take(pl);
    L.pb = take(pl);
    L.W = take(3 * pl);
    L.B = take(3 * pl);
    L.U = take(3 * pl);
    L.T = take(3 * pl);
    L.D = take(pl);
    L.C = take(sizeof(float2) * (size_t)M * N * half_pitch(P));
    L.twM = take(sizeof(float2) * M);
    L.twN = take(sizeof(float2) * N);
    L.twP = take(sizeof(float2) * P);
    L.total = o;
    return L;
}

// Events of the launch being timed by sr3_profile (null: plain launch).
thread_local hipEvent_t t_ev[2] = {nullptr, nullptr};

template <typename... KArgs, typename... Args>
void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t st, Args... args) {
    if (t_ev[0])
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, t_ev[0], t_ev[1], 0u,
                              static_cast<KArgs>(args)...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, static_cast<KArgs>(args)...);
}

}  // namespace

struct sr3_ctx {
    int M, N, P;
    size_t n;
    sr_params p;
    KParams kp;
    Gauss3 gauss;
    hipStream_t st;
    float *g, *phi, *alt, *W, *B, *U, *T, *D;   // D = div(b - w) of the current outer iteration
    float2 *C, *twM, *twN, *twP;
    float taumu;
    long long k = 0;
    bool image = false;
    // sr3_profile: per-kind hooks (kind -> events armed before the launch)
    std::vector<hipEvent_t>* prof_ev = nullptr;
    std::vector<int>* prof_kind = nullptr;
};

namespace {

void arm(sr3_ctx* c, int kind) {
    if (!c->prof_ev) return;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    c->prof_ev->push_back(a);
    c->prof_ev->push_back(b);
    c->prof_kind->push_back(kind);
    t_ev[0] = a;
    t_ev[1] = b;
}

void disarm() { t_ev[0] = t_ev[1] = nullptr; }

unsigned vblocks(size_t n) { return (unsigned)((n + kT - 1) / kT); }

template <int L, int G>
void fft_pass_g(sr3_ctx* c, int axis, int mode, float* rout, const float* radd) {
    // the k pass: one line per (i, j); the strided passes: one line per k
    // slot of the half spectrum and (j, or i)
    const int Hp = half_pitch(c->P);
    const int lines = axis == 2 ? c->M * c->N : (axis == 1 ? c->M : c->N) * Hp;
    const float scale = 1.0f / (float)c->n;
    const size_t lds = sizeof(float2) * (2 * G * (L + 1) + L);
    launch(k3_fft<L, G>, dim3(lines / G), dim3(FftShape3<L, G>::T), lds, c->st, c->C, rout, radd, c->twM,
           c->twN, c->twP, c->M, c->N, c->P, Hp, axis, mode, c->taumu, scale);
}

// L is the axis length; the k pass runs L/2-point transforms
template <int L>
void fft_pass_t(sr3_ctx* c, int axis, int mode, float* rout, const float* radd) {
    if (axis == 2)
        fft_pass_g<L / 2, kLines>(c, axis, mode, rout, radd);
    else
        fft_pass_g<L, kStridedLines>(c, axis, mode, rout, radd);
}

// The rhs fused with the forward k transform (P = L real samples per line).
template <int L>
void rhs_kfwd_t(sr3_ctx* c, int first) {
    constexpr int Q = L / 2, G = kLines;
    const size_t lds = sizeof(float2) * (2 * G * (Q + 1) + Q);
    launch(k3_rhs_kfwd<Q, G>, dim3(c->M * c->N / G), dim3(FftShape3<Q, G>::T), lds, c->st, c->phi, c->W, c->B,
           c->D, c->g, c->T, c->C, c->twP, c->M, c->N, c->P, half_pitch(c->P), first, c->kp);
}

template <int L>
void fft_attrs() {
    (void)hipFuncSetAttribute((const void*)k3_fft<L / 2, kLines>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(float2) * (2 * kLines * (L / 2 + 1) + L / 2)));
    (void)hipFuncSetAttribute((const void*)k3_rhs_kfwd<L / 2, kLines>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(float2) * (2 * kLines * (L / 2 + 1) + L / 2)));
    (void)hipFuncSetAttribute((const void*)k3_fft<L, kStridedLines>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(float2) * (2 * kStridedLines * (L + 1) + L)));
}

}  // namespace

namespace {

void fft_pass(sr3_ctx* c, int axis, int mode, float* rout, const float* radd) {
    arm(c, 2);
    const int L = axis == 0 ? c->M : axis == 1 ? c->N : c->P;
    switch (L) {
        case 8: fft_pass_t<8>(c, axis, mode, rout, radd); break;
        case 16: fft_pass_t<16>(c, axis, mode, rout, radd); break;
        case 32: fft_pass_t<32>(c, axis, mode, rout, radd); break;
        case 64: fft_pass_t<64>(c, axis, mode, rout, radd); break;
        case 128: fft_pass_t<128>(c, axis, mode, rout, radd); break;
        default: fft_pass_t<256>(c, axis, mode, rout, radd); break;
    }
    disarm();
}

// r (eq 37) and its forward k transform, one launch.
void rhs_kfwd(sr3_ctx* c, int first) {
    arm(c, 1);
    switch (c->P) {
        case 8: rhs_kfwd_t<8>(c, first); break;
        case 16: rhs_kfwd_t<16>(c, first); break;
        case 32: rhs_kfwd_t<32>(c, first); break;
        case 64: rhs_kfwd_t<64>(c, first); break;
        case 128: rhs_kfwd_t<128>(c, first); break;
        default: rhs_kfwd_t<256>(c, first); break;
    }
    disarm();
}

// phi_out = phi_in + u with (1 - tau mu Lap) u = r, from r's k transform.
void solve(sr3_ctx* c, const float* phi_in, float* phi_out) {
    fft_pass(c, 1, 1, nullptr, nullptr);
    fft_pass(c, 0, 2, nullptr, nullptr);
    fft_pass(c, 1, 3, nullptr, nullptr);
    fft_pass(c, 2, 4, phi_out, phi_in);
}

// V (in T) = cube window of u = W h(phi): the k pass forms u, then j, i.
void window(sr3_ctx* c, const float* phi) {
    const unsigned nb = vblocks(c->n);
    static_assert(kT == 256, "the k window pass holds whole k-lines of up to 256 voxels");
    arm(c, 0);
    launch(k3_win_u, dim3(nb), dim3(kT), 0, c->st, c->W, phi, c->T, c->M, c->N, c->P, c->kp);
    disarm();
    const unsigned kb = (unsigned)(c->P < kWinKT ? 1 : c->P / kWinKT);
    const unsigned jb = (unsigned)(c->N < kWinTA ? 1 : c->N / kWinTA);
    const unsigned ib = (unsigned)(c->M < kWinTA ? 1 : c->M / kWinTA);
    arm(c, 0);
    launch(k3_win_tile, dim3(kb, jb, c->M), dim3(kT), 0, c->st, c->T, c->U, c->M, c->N, c->P, 1, c->kp);
    disarm();
    arm(c, 0);
    launch(k3_win_tile, dim3(kb, ib, c->N), dim3(kT), 0, c->st, c->U, c->T, c->M, c->N, c->P, 0, c->kp);
    disarm();
}

void iteration(sr3_ctx* c) {
    const unsigned nb = vblocks(c->n);
    for (int s = 0; s < c->p.S; ++s) {
        window(c, c->phi);
        rhs_kfwd(c, s == 0 ? 1 : 0);
        solve(c, c->phi, c->alt);
        float* t = c->phi;
        c->phi = c->alt;
        c->alt = t;
    }
    window(c, c->phi);
    arm(c, 3);
    launch(k3_wstep, dim3(nb), dim3(kT), 0, c->st, c->phi, c->W, c->B, c->g, c->T, c->M, c->N, c->P, c->kp);
    disarm();
    ++c->k;
}

int check_params(int M, int N, int P, const sr_params* p) {
    if (!p) return sr::api_fail(SR_EINVAL, "NULL params");
    if (!pow2_in(M) || !pow2_in(N) || !pow2_in(P))
        return sr::api_fail(SR_EUNSUPPORTED, "3-D volumes need M, N, P powers of two in [8, 256]");
    if (p->R < 0 || p->R > sr::kMaxR) return sr::api_fail(SR_EUNSUPPORTED, "R must be in [0, 8]");
    if ((int)std::ceil(3.0 * p->sigma) > sr::kMaxGaussR || p->sigma < 0)
        return sr::api_fail(SR_EUNSUPPORTED, "sigma must be in [0, 16/3]");
    if (p->tau <= 0 || p->mu <= 0 || p->eps <= 0 || p->d <= 0 || p->S < 1)
        return sr::api_fail(SR_EINVAL, "tau, mu, eps, d must be > 0 and S >= 1");
    if (p->s_exp != 1 && p->s_exp != 2) return sr::api_fail(SR_EINVAL, "s_exp must be 1 or 2");
    if (p->tol_inner > 0 || p->w_solver != 0 || p->phi_solver != 0 || p->bc != 0 || p->w0_mode != 0)
        return sr::api_fail(SR_EUNSUPPORTED, "the 3-D solver runs a fixed S with the shrink w solver, the FFT "
                                             "solve, periodic boundaries and w^0 = grad phi^0");
    return SR_OK;
}

}  // namespace

extern "C" {

int sr3_workspace_size(int32_t M, int32_t N, int32_t P, const sr_params* p, size_t* bytes) {
    if (!bytes) return sr::api_fail(SR_EINVAL, "NULL bytes");
    const int rc = check_params(M, N, P, p);
    if (rc) return rc;
    *bytes = layout3(M, N, P).total;
    return SR_OK;
}

int sr3_create(sr3_ctx** out, int32_t M, int32_t N, int32_t P, const sr_params* p, void* workspace, size_t bytes,
               void* hip_stream) {
    if (!out || !workspace) return sr::api_fail(SR_EINVAL, "NULL argument");
    const int rc = check_params(M, N, P, p);
    if (rc) return rc;
    const Layout3 L = layout3(M, N, P);
    if (bytes < L.total) return sr::api_fail(SR_EINVAL, "workspace too small");
    if ((uintptr_t)workspace & 255) return sr::api_fail(SR_EINVAL, "workspace must be 256-byte aligned");
    static bool attrs = false;
    if (!attrs) {
        fft_attrs<8>(); fft_attrs<16>(); fft_attrs<32>(); fft_attrs<64>(); fft_attrs<128>(); fft_attrs<256>();
        attrs = true;
    }
    sr3_ctx* c = new sr3_ctx();
    c->M = M;
    c->N = N;
    c->P = P;
    c->n = (size_t)M * N * P;
    c->p = *p;
    c->st = (hipStream_t)hip_stream;
    KParams& kp = c->kp;
    std::memset(&kp, 0, sizeof kp);
    kp.gamma = (float)p->gamma;
    kp.alpha = (float)p->alpha;
    kp.beta = (float)p->beta;
    kp.mu = (float)p->mu;
    kp.tau = (float)p->tau;
    kp.eps = (float)p->eps;
    kp.inv_eps = (float)(1.0 / p->eps);
    kp.band_l = (float)p->band_l;
    kp.c_rep = (float)(2.0 * p->beta / p->mu);
    kp.c_thr = (float)(p->gamma / p->mu);
    kp.zero_tol = (float)p->zero_tol;
    kp.R = p->R;
    for (int q = -p->R; q <= p->R; ++q) kp.taps[q + p->R] = (float)std::exp(-(double)q * q / (p->d * p->d));
    c->taumu = (float)(p->tau * p->mu);
    // Gaussian taps of eq (1): sampled, truncated at ceil(3 sigma), unit sum
    const int r = (int)std::ceil(3.0 * p->sigma);
    c->gauss.r = r;
    {
        std::vector<double> kd(2 * r + 1);
        double sum = 0.0;
        for (int t = -r; t <= r; ++t) {
            kd[t + r] = r == 0 ? 1.0 : std::exp(-(double)t * t / (2.0 * p->sigma * p->sigma));
            sum += kd[t + r];
        }
        for (int t = 0; t <= 2 * r; ++t) c->gauss.k[t] = (float)(kd[t] / sum);
    }
    char* base = (char*)workspace;
    c->g = (float*)(base + L.g);
    c->phi = (float*)(base + L.pa);
    c->alt = (float*)(base + L.pb);
    c->W = (float*)(base + L.W);
    c->B = (float*)(base + L.B);
    c->U = (float*)(base + L.U);
    c->T = (float*)(base + L.T);
    c->D = (float*)(base + L.D);
    c->C = (float2*)(base + L.C);
    c->twM = (float2*)(base + L.twM);
    c->twN = (float2*)(base + L.twN);
    c->twP = (float2*)(base + L.twP);
    const std::vector<float2> a = host_twiddles(M), b = host_twiddles(N), d = host_twiddles(P);
    hipError_t e = hipMemcpyAsync(c->twM, a.data(), sizeof(float2) * M, hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->twN, b.data(), sizeof(float2) * N, hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->twP, d.data(), sizeof(float2) * P, hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        delete c;
        return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    }
    *out = c;
    return SR_OK;
}

int sr3_set_image(sr3_ctx* c, const float* f, const float* phi0) {
    if (!c || !f || !phi0) return sr::api_fail(SR_EINVAL, "NULL argument");
    const unsigned nb = vblocks(c->n);
    // cube Gaussian: along k (f -> U), j (U -> T), i (T -> U), then g
    hipLaunchKernelGGL(k3_gauss, dim3(nb), dim3(kT), 0, c->st, f, c->U, c->M, c->N, c->P, 2, c->gauss);
    hipLaunchKernelGGL(k3_gauss, dim3(nb), dim3(kT), 0, c->st, c->U, c->T, c->M, c->N, c->P, 1, c->gauss);
    hipLaunchKernelGGL(k3_gauss, dim3(nb), dim3(kT), 0, c->st, c->T, c->U, c->M, c->N, c->P, 0, c->gauss);
    hipLaunchKernelGGL(k3_edge, dim3(nb), dim3(kT), 0, c->st, c->U, c->g, c->M, c->N, c->P, (float)c->p.rho,
                       c->p.s_exp);
    hipLaunchKernelGGL(k3_init, dim3(nb), dim3(kT), 0, c->st, phi0, c->phi, c->W, c->B, c->M, c->N, c->P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    c->k = 0;
    c->image = true;
    return SR_OK;
}

int sr3_set_state(sr3_ctx* c, const float* phi, const float* w, const float* b, int64_t k) {
    if (!c || !phi || !w || !b) return sr::api_fail(SR_EINVAL, "NULL argument");
    if (!c->image) return sr::api_fail(SR_ESTATE, "sr3_set_image first (it computes g)");
    const size_t pl = sizeof(float) * c->n;
    hipError_t e = hipMemcpyAsync(c->phi, phi, pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->W, w, 3 * pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->B, b, 3 * pl, hipMemcpyDeviceToDevice, c->st);
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    c->k = k;
    return SR_OK;
}

int sr3_step(sr3_ctx* c, int32_t n_iter, int64_t* k_out) {
    if (!c) return sr::api_fail(SR_EINVAL, "NULL context");
    if (n_iter < 1) return sr::api_fail(SR_EINVAL, "n_iter must be >= 1");
    if (!c->image) return sr::api_fail(SR_ESTATE, "sr3_set_image first");
    for (int it = 0; it < n_iter; ++it) iteration(c);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    if (k_out) *k_out = c->k;
    return SR_OK;
}

int sr3_get_state(sr3_ctx* c, float* phi, float* w, float* b, float* g) {
    if (!c) return sr::api_fail(SR_EINVAL, "NULL context");
    const size_t pl = sizeof(float) * c->n;
    hipError_t e = hipSuccess;
    if (phi) e = hipMemcpyAsync(phi, c->phi, pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess && w) e = hipMemcpyAsync(w, c->W, 3 * pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess && b) e = hipMemcpyAsync(b, c->B, 3 * pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess && g) e = hipMemcpyAsync(g, c->g, pl, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    return SR_OK;
}

int sr3_profile(sr3_ctx* c, int32_t n_iter, double ms[4], int64_t count[4]) {
    if (!c || !ms || !count) return sr::api_fail(SR_EINVAL, "NULL argument");
    if (n_iter < 1) return sr::api_fail(SR_EINVAL, "n_iter must be >= 1");
    if (!c->image) return sr::api_fail(SR_ESTATE, "sr3_set_image first");
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    c->prof_ev = &ev;
    c->prof_kind = &kind;
    for (int it = 0; it < n_iter; ++it) iteration(c);
    c->prof_ev = nullptr;
    c->prof_kind = nullptr;
    hipError_t e = hipStreamSynchronize(c->st);
    for (int q = 0; q < 4; ++q) { ms[q] = 0.0; count[q] = 0; }
    for (size_t q = 0; q < kind.size() && e == hipSuccess; ++q) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, ev[2 * q], ev[2 * q + 1]);
        ms[kind[q]] += t;
        count[kind[q]] += 1;
    }
    for (hipEvent_t h : ev) (void)hipEventDestroy(h);
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    for (int q = 0; q < 4; ++q)
        if (count[q]) ms[q] /= (double)count[q];
    return SR_OK;
}

void sr3_destroy(sr3_ctx* c) { delete c; }

}  // extern "C"
