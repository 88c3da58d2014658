// Device-side building blocks of the SR Split Bregman solver (gfx950).
//
//  - the compactly supported H_eps, delta_eps, delta'_eps (eqs 5, 6, 29)
//    and the narrow band h_eps, h'_eps (eqs 11, 28), in FP32 from a
//    half-angle Taylor evaluation of sin / cos on the support;
//  - an in-LDS complex FFT (Stockham auto-sort, radix-4 stages plus one
//    radix-2 stage for odd log2 lengths) used by the row and column passes
//    of the semi-implicit solve (eqs 31-33);
//  - deterministic block / grid reductions in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

constexpr int kMaxR = 8;        // largest repulsion window half-width
constexpr int kMaxTaps = 2 * kMaxR + 1;
constexpr int kMaxGaussR = 16;  // largest Gaussian radius ceil(3 sigma)
constexpr int kTileW = 64;      // tile width of the stencil kernels (one wave per row)
constexpr int kTileThreads = 256;
constexpr int kScalStride = 64; // int64 words of per-instance device scalars
constexpr int kRHist = 1024;    // residual history ring (per instance)

// Per-instance device scalars (one block of kScalStride int64 words,
// followed elsewhere by the residual ring).
struct DevScal {
    unsigned int counter;   // reserved
    int inner_done;         // inner stop rule met in this outer iteration
    int active;             // 0: instance finished (batched solve) -> kernels skip it
    int nonfinite;          // NaN/Inf seen in an input
    long long k;            // outer iterations completed
    long long inner_steps;  // inner steps executed (counted when tol_inner > 0)
    double r_last;          // last outer relative change r_k
    double inner_rel;       // last inner relative change
    double energy[3];       // gamma E_g, alpha E_a, beta E_r
    // per-instance stop rule of the batched solve (0 = host decides)
    int max_iter;           // retire when k reaches this
    int min_iter;           // no tolerance stop before this
    double tol_outer;       // retire when r_k < tol_outer
    int converged;          // set when retired by the tolerance
    int spare;
    long long pad[kScalStride - 12];
};
static_assert(sizeof(DevScal) == kScalStride * 8, "DevScal layout");

// Scalars the kernels need, in FP32, plus the FP64-computed window taps.
struct KParams {
    float gamma, alpha, beta, mu, tau;
    float eps, inv_eps, band_l;
    float c_rep;       // 2 beta / mu      (eq 41)
    float c_thr;       // gamma / mu       (eq 42)
    float tol_inner;
    float zero_tol;    // |B| <= zero_tol counts as the zero vector (eq 42)
    int R;
    float taps[kMaxTaps];   // a_q = exp(-q^2/d^2), q = -R..R at index q+R
};

// ---------------------------------------------------------------------------
// sin and cos of the half angle t = pi u / 2 for |u| <= 1, i.e. |t| <= pi/2,
// by the Taylor series of sin and cos truncated after t^11 and t^12 (the
// first omitted terms are below 6e-8 and 7e-9 on that interval).  The
// smoothed Heaviside / Dirac only ever need |u| = |phi / eps| <= 1, so no
// range reduction is required, and every quantity below is built from
// (sin t, cos t) without cancellation:
//   sin(pi u) = 2 sin t cos t,   1 + cos(pi u) = 2 cos^2 t.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void half_sincos(float u, float& sh, float& ch) {
    const float t = 1.5707963267948966f * u;
    const float t2 = t * t;
    float ps = -2.505210838544172e-08f;
    ps = fmaf(ps, t2, 2.7557319223985893e-06f);
    ps = fmaf(ps, t2, -0.0001984126984126984f);
    ps = fmaf(ps, t2, 0.008333333333333333f);
    ps = fmaf(ps, t2, -0.16666666666666666f);
    ps = fmaf(ps, t2, 1.0f);
    float pc = 2.08767569878681e-09f;
    pc = fmaf(pc, t2, -2.755731922398589e-07f);
    pc = fmaf(pc, t2, 2.48015873015873e-05f);
    pc = fmaf(pc, t2, -0.001388888888888889f);
    pc = fmaf(pc, t2, 0.041666666666666664f);
    pc = fmaf(pc, t2, -0.5f);
    pc = fmaf(pc, t2, 1.0f);
    sh = t * ps;
    ch = pc;
}

constexpr float kInvPi = 0.31830988618379067f;

// H_eps and delta_eps (eqs 5, 6), evaluated together:
//   H = (1 + u + sin(pi u)/pi) / 2,   delta = (1 + cos(pi u)) / (2 eps),   u = x / eps.
__device__ __forceinline__ void heav_dirac(float x, float eps, float inv_eps, float& H, float& dl) {
    if (x > eps) { H = 1.0f; dl = 0.0f; return; }
    if (x < -eps) { H = 0.0f; dl = 0.0f; return; }
    const float u = x * inv_eps;
    float sh, ch;
    half_sincos(u, sh, ch);
    H = 0.5f * (1.0f + u) + kInvPi * sh * ch;
    dl = inv_eps * ch * ch;
}

// h_eps = H(phi + l)(1 - H(phi - l))  (eq 11)
__device__ __forceinline__ float band_h(float x, const KParams& kp) {
    const float lim = kp.band_l + kp.eps;
    if (x > lim || x < -lim) return 0.0f;
    float Hp, dp, Hm, dm;
    heav_dirac(x + kp.band_l, kp.eps, kp.inv_eps, Hp, dp);
    heav_dirac(x - kp.band_l, kp.eps, kp.inv_eps, Hm, dm);
    return Hp * (1.0f - Hm);
}

// h_eps and h'_eps (eq 28) together.
__device__ __forceinline__ void band_h_dh(float x, const KParams& kp, float& h, float& dh) {
    const float lim = kp.band_l + kp.eps;
    if (x > lim || x < -lim) { h = 0.0f; dh = 0.0f; return; }
    float Hp, dp, Hm, dm;
    heav_dirac(x + kp.band_l, kp.eps, kp.inv_eps, Hp, dp);
    heav_dirac(x - kp.band_l, kp.eps, kp.inv_eps, Hm, dm);
    h = Hp * (1.0f - Hm);
    dh = dp * (1.0f - Hm) - Hp * dm;
}

// delta_eps and delta'_eps (eqs 6, 29) together:
//   delta' = -(pi / (2 eps^2)) sin(pi u) = -(pi / eps^2) sin t cos t.
__device__ __forceinline__ void dirac_d(float x, const KParams& kp, float& dl, float& ddl) {
    if (x > kp.eps || x < -kp.eps) { dl = 0.0f; ddl = 0.0f; return; }
    float sh, ch;
    half_sincos(x * kp.inv_eps, sh, ch);
    dl = kp.inv_eps * ch * ch;
    ddl = -3.141592653589793f * kp.inv_eps * kp.inv_eps * sh * ch;
}

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

template <int L> struct Ilog2 { static constexpr int v = 1 + Ilog2<L / 2>::v; };
template <> struct Ilog2<1> { static constexpr int v = 0; };

// Work split of one length-L transform: NT threads, E elements each.  Four
// elements (one radix-4 butterfly per stage) for lengths up to 1024 gives
// the most waves per CU; 2048 and 4096 points take 8 and 16 so that the
// four transforms of an 8-row tile still fit one 1024-thread workgroup.
template <int L> struct RowE { static constexpr int v = L <= 1024 ? 4 : (L == 2048 ? 8 : 16); };
// The column pass runs two transforms per workgroup, so it can afford more
// threads per transform (fewer registers per thread) at 4096 points.
template <int L> struct ColE { static constexpr int v = L <= 2048 ? 4 : 8; };
template <int L, int EE = RowE<L>::v> struct FftShape {
    static constexpr int E = EE;
    static constexpr int NT = L / E;
    static constexpr int LOG = Ilog2<L>::v;
};

// LDS skew of the FFT buffers: element i of a transform lives at
// i + i / 16.  Without it the Stockham write pattern (stride 4 Ns between
// lanes for small Ns) maps many lanes of a wave onto the same LDS bank.
__device__ __forceinline__ int sk(int i) { return i + (i >> 4); }
// float2 slots of one skewed length-L buffer, +4 so that consecutive
// transforms start on different banks.
template <int L> struct LdsLen { static constexpr int v = L + L / 16 + 4; };

// One radix-4 Stockham stage: sub-transform size Ns -> 4 Ns.
// Butterfly j reads x[j + r L/4], twiddles by W_{4Ns}^{r k} (k = j mod Ns),
// and writes x[(j - k) 4 + k + r Ns].  Twiddle W_{4Ns}^{m} = tw[m L/(4Ns)],
// tw[n] = exp(-2 pi i n / L).
template <int L, int EE, bool INV>
__device__ __forceinline__ void fft_stage4(float2* x, const float2* __restrict__ tw, int t, int Ns) {
    constexpr int E = FftShape<L, EE>::E, NT = FftShape<L, EE>::NT;
    constexpr int Q = L / 4;
    float2 v[E];
#pragma unroll
    for (int b = 0; b < E / 4; ++b) {
        const int j = t + b * NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * b + r] = x[sk(j + r * Q)];
    }
    __syncthreads();
    const int stride = L / (4 * Ns);
#pragma unroll
    for (int b = 0; b < E / 4; ++b) {
        const int j = t + b * NT;
        const int k = j & (Ns - 1);
        float2 a0 = v[4 * b], a1 = v[4 * b + 1], a2 = v[4 * b + 2], a3 = v[4 * b + 3];
        if (Ns > 1) {
            const float2 w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
            if (INV) { a1 = cmulc(a1, w1); a2 = cmulc(a2, w2); a3 = cmulc(a3, w3); }
            else     { a1 = cmul(a1, w1);  a2 = cmul(a2, w2);  a3 = cmul(a3, w3); }
        }
        const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
        const float2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
        // forward: y1 = d02 - i d13, y3 = d02 + i d13; inverse swaps them
        const float2 id13 = make_float2(-d13.y, d13.x);
        const int base = ((j - k) << 2) + k;
        x[sk(base)] = cadd(s02, s13);
        x[sk(base + 2 * Ns)] = csub(s02, s13);
        if (INV) { x[sk(base + Ns)] = cadd(d02, id13); x[sk(base + 3 * Ns)] = csub(d02, id13); }
        else     { x[sk(base + Ns)] = csub(d02, id13); x[sk(base + 3 * Ns)] = cadd(d02, id13); }
    }
    __syncthreads();
}

// In-place length-L complex FFT of x (in LDS, skewed by sk()) by the NT threads t = 0..NT-1
// of one transform.  Every thread of the workgroup must call it (it
// contains workgroup barriers).  INV: unnormalised inverse (conjugate twiddles).
template <int L, int EE, bool INV>
__device__ __forceinline__ void fft_lds(float2* x, const float2* __restrict__ tw, int t) {
    constexpr int E = FftShape<L, EE>::E, NT = FftShape<L, EE>::NT, LOG = FftShape<L, EE>::LOG;
    __syncthreads();
    int Ns = 1;
    if constexpr (LOG & 1) {
        float2 v[E];
#pragma unroll
        for (int b = 0; b < E / 2; ++b) {
            const int j = t + b * NT;
            v[2 * b] = x[sk(j)];
            v[2 * b + 1] = x[sk(j + L / 2)];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / 2; ++b) {
            const int j = t + b * NT;
            x[sk(2 * j)] = cadd(v[2 * b], v[2 * b + 1]);
            x[sk(2 * j + 1)] = csub(v[2 * b], v[2 * b + 1]);
        }
        __syncthreads();
        Ns = 2;
    }
#pragma unroll
    for (int st = 0; st < LOG / 2; ++st) {
        fft_stage4<L, EE, INV>(x, tw, t, Ns);
        Ns <<= 2;
    }
}

// ---------------------------------------------------------------------------
// reductions (fixed order -> bitwise deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum NV values over the workgroup; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* LDS, NV*16 */) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = wave_sum(v[c]);
        if (lane == 0) red[c * 16 + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[c * 16 + w];
            v[c] = s;
        }
    }
    __syncthreads();
}

// Store this workgroup's NV partial sums at part[c * nblocks + bid]; a
// separate finalize kernel adds them in block order (bitwise deterministic).
// (An in-kernel "last workgroup" reduction would need an agent-scope fence
// per workgroup, which on gfx950 writes back the whole non-coherent L2.)
template <int NV>
__device__ __forceinline__ void store_partials(double (&v)[NV], double* part, int nblocks, int bid, double* red) {
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) part[c * nblocks + bid] = v[c];
    }
}

// Sum of the NV x nblocks partials in fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* part, int nblocks, double (&v)[NV], double* red) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[c * nblocks + b];
        v[c] = s;
    }
    block_sum<NV>(v, red);
}

}  // namespace sr
