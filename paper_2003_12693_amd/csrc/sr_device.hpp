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
constexpr int kTileThreads = 256;   // threads per stencil tile (w step, energy, repulsion)
constexpr int kRhsThreads = 512;    // threads per tile of the right-hand-side kernel
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
#ifndef SR_ROW_E
#define SR_ROW_E 4
#endif
#ifndef SR_COL_E
#define SR_COL_E 4
#endif
template <int L> struct RowE {
    static constexpr int v = L <= 1024 ? (SR_ROW_E < L ? SR_ROW_E : L)
                                       : (L == 2048 ? (SR_ROW_E > 8 ? SR_ROW_E : 8) : 16);
};
// The column pass holds one transform per workgroup, so it can afford more
// threads per transform (fewer registers per thread) at 4096 points.
#ifndef SR_COL_E_LONG
#define SR_COL_E_LONG 8
#endif
template <int L> struct ColE {
    static constexpr int v = L <= 2048 ? (SR_COL_E < L ? SR_COL_E : L) : SR_COL_E_LONG;
};
// Waves per SIMD the column pass is compiled for (a VGPR cap): 8 (64 VGPRs)
// unless 16-element transforms need more registers.
// Four-element transforms (up to 2048 points) hold every stage twiddle in
// registers (tw_preload), so they get the 128-VGPR budget too.
template <int L> struct ColWaves { static constexpr int v = (ColE<L>::v >= 16 || ColE<L>::v <= 4) ? 4 : 8; };
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

// Twiddle tables of the Stockham stages, one per (length L, elements per
// thread EE), built on the host in FP64: for every stage with Ns > 1, in
// stage order, Ns blocks of R float2, block k holding W_{R Ns}^{r k} for
// r = 0..R-1 (entry 0 is 1, kept so that blocks are 16-byte aligned).  A
// thread fetches its R - 1 factors with 16-byte global loads (the table is
// at most ~37 KiB and stays in L1/L2), so no index or quadrant arithmetic
// is left on the vector ALUs.
constexpr int fft_radix(int L, int EE, int Ns) { return EE < L / Ns ? EE : L / Ns; }
constexpr int stage_tab_len(int L, int EE, int Ns = 1) {
    return Ns >= L ? 0
                   : (Ns > 1 ? Ns * fft_radix(L, EE, Ns) : 0) + stage_tab_len(L, EE, Ns * fft_radix(L, EE, Ns));
}

// Multiplication by the constant W_16^m = exp(-2 pi i m / 16) (forward) or
// its conjugate (inverse); m = 0 and m = 4 (= -i) are exact.
template <int m, bool INV>
__device__ __forceinline__ float2 w16(float2 a) {
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    else {
        constexpr float cs[10] = {1.0f, 0.9238795325112867f, 0.7071067811865476f, 0.38268343236508984f, 6.123233995736766e-17f, -0.3826834323650897f, -0.7071067811865475f, -0.9238795325112867f, -1.0f, -0.9238795325112868f};
        constexpr float sn[10] = {0.0f, 0.3826834323650898f, 0.7071067811865475f, 0.9238795325112867f, 1.0f, 0.9238795325112867f, 0.7071067811865476f, 0.3826834323650899f, 1.2246467991473532e-16f, -0.38268343236508967f};
        const float2 w = make_float2(cs[m], INV ? sn[m] : -sn[m]);
        return cmul(a, w);
    }
}

// In-register DFTs of 2, 4, 8, 16 points (outputs in natural order).
template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const float2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
    const float2 id13 = make_float2(-d13.y, d13.x);
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    if (INV) { a1 = cadd(d02, id13); a3 = csub(d02, id13); }
    else     { a1 = csub(d02, id13); a3 = cadd(d02, id13); }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&u)[R]) {
    if constexpr (R == 2) {
        const float2 a = u[0], b = u[1];
        u[0] = cadd(a, b);
        u[1] = csub(a, b);
    } else if constexpr (R == 4) {
        dft4<INV>(u[0], u[1], u[2], u[3]);
    } else if constexpr (R == 8) {
        // n = 2 n1 + n2, k = k1 + 4 k2: two DFT4 over n1, twiddle W_8^{n2 k1}, DFT2 over n2
        float2 a0 = u[0], a1 = u[2], a2 = u[4], a3 = u[6];
        float2 b0 = u[1], b1 = u[3], b2 = u[5], b3 = u[7];
        dft4<INV>(a0, a1, a2, a3);
        dft4<INV>(b0, b1, b2, b3);
        b1 = w16<2, INV>(b1);
        b2 = w16<4, INV>(b2);
        b3 = w16<6, INV>(b3);
        u[0] = cadd(a0, b0); u[4] = csub(a0, b0);
        u[1] = cadd(a1, b1); u[5] = csub(a1, b1);
        u[2] = cadd(a2, b2); u[6] = csub(a2, b2);
        u[3] = cadd(a3, b3); u[7] = csub(a3, b3);
    } else {
        static_assert(R == 16, "radix");
        // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle W_16^{n2 k1}, DFT4 over n2
        float2 A[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            A[n2][0] = u[n2]; A[n2][1] = u[4 + n2]; A[n2][2] = u[8 + n2]; A[n2][3] = u[12 + n2];
            dft4<INV>(A[n2][0], A[n2][1], A[n2][2], A[n2][3]);
        }
        A[1][1] = w16<1, INV>(A[1][1]); A[1][2] = w16<2, INV>(A[1][2]); A[1][3] = w16<3, INV>(A[1][3]);
        A[2][1] = w16<2, INV>(A[2][1]); A[2][2] = w16<4, INV>(A[2][2]); A[2][3] = w16<6, INV>(A[2][3]);
        A[3][1] = w16<3, INV>(A[3][1]); A[3][2] = w16<6, INV>(A[3][2]); A[3][3] = w16<9, INV>(A[3][3]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 b0 = A[0][k1], b1 = A[1][k1], b2 = A[2][k1], b3 = A[3][k1];
            dft4<INV>(b0, b1, b2, b3);
            u[k1] = b0; u[k1 + 4] = b1; u[k1 + 8] = b2; u[k1 + 12] = b3;
        }
    }
}

// Stage twiddle factors one thread applies over a whole length-L transform:
// R - 1 per butterfly of every stage with Ns > 1.  A kernel may load them all
// into registers up front (tw_preload) so that no stage waits on a global
// load; the column pass then uses one set for its forward and inverse
// transforms (the inverse conjugates them).
constexpr int tw_count(int L, int EE, int Ns = 1) {
    return Ns >= L ? 0
                   : (Ns > 1 ? (EE / fft_radix(L, EE, Ns)) * (fft_radix(L, EE, Ns) - 1) : 0) +
                         tw_count(L, EE, Ns * fft_radix(L, EE, Ns));
}
template <int L, int EE> struct TwN { static constexpr int v = tw_count(L, EE) > 0 ? tw_count(L, EE) : 1; };

template <int L, int EE, int Ns, int OFF, int IDX>
__device__ __forceinline__ void tw_preload_stages(const float2* __restrict__ tab, int t,
                                                  float2 (&twr)[TwN<L, EE>::v]) {
    if constexpr (Ns < L) {
        constexpr int R = fft_radix(L, EE, Ns), NB = EE / R, NT = L / EE;
        if constexpr (Ns > 1) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int k = (t + b * NT) & (Ns - 1);
                const float4* p = reinterpret_cast<const float4*>(tab + OFF + (size_t)k * R);
#pragma unroll
                for (int h = 0; h < R / 2; ++h) {
                    const float4 q = p[h];
                    if (h > 0) twr[IDX + b * (R - 1) + 2 * h - 1] = make_float2(q.x, q.y);
                    twr[IDX + b * (R - 1) + 2 * h] = make_float2(q.z, q.w);
                }
            }
        }
        tw_preload_stages<L, EE, Ns * R, OFF + (Ns > 1 ? Ns * R : 0), IDX + (Ns > 1 ? NB * (R - 1) : 0)>(tab, t,
                                                                                                       twr);
    }
}
// All stage twiddles of thread t of a length-L transform (EE elements per
// thread) from the stage table of (L, EE).
template <int L, int EE>
__device__ __forceinline__ void tw_preload(const float2* __restrict__ tab, int t, float2 (&twr)[TwN<L, EE>::v]) {
    tw_preload_stages<L, EE, 1, 0, 0>(tab, t, twr);
}

// One radix-R Stockham stage: sub-transform size Ns -> R Ns.  Butterfly j
// reads x[j + r L/R], twiddles by W_{R Ns}^{r k} (k = j mod Ns), applies the
// R-point DFT and writes x[(j - k) R + k + r Ns].  tws: this stage's block of
// the stage twiddle table.  FROM_REGS (first stage, Ns = 1): the inputs come
// from io instead of LDS, io[e] holding element t + e NT; TO_REGS (last
// stage, Ns = L/R): the outputs go to io in that same layout instead of LDS.
// PIDX >= 0: the twiddles are twr[PIDX ...] (tw_preload) instead of tws.
template <int L, int EE, int R, int Ns, bool INV, bool FROM_REGS, bool TO_REGS, int PIDX>
__device__ __forceinline__ void fft_stage(float2* x, const float2* __restrict__ tws, int t, float2 (&io)[EE],
                                          const float2 (&twr)[TwN<L, EE>::v]) {
    constexpr int E = EE, NT = L / E, NB = E / R, Q = L / R;
    static_assert(!FROM_REGS || Ns == 1, "register input is the first stage");
    static_assert(!TO_REGS || Ns * R == L, "register output is the last stage");
    float2 w[NB][R];
    if constexpr (Ns > 1 && PIDX >= 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 1; r < R; ++r) w[b][r] = twr[PIDX + b * (R - 1) + r - 1];
    } else if constexpr (Ns > 1) {   // issued first: their latency overlaps the LDS reads
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int k = (t + b * NT) & (Ns - 1);
            const float4* p = reinterpret_cast<const float4*>(tws + (size_t)k * R);
#pragma unroll
            for (int h = 0; h < R / 2; ++h) {
                const float4 q = p[h];
                w[b][2 * h] = make_float2(q.x, q.y);
                w[b][2 * h + 1] = make_float2(q.z, q.w);
            }
        }
    }
    float2 v[E];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // element j + r Q = t + (b + r NB) NT
            if constexpr (FROM_REGS) v[b * R + r] = io[b + r * NB];
            else v[b * R + r] = x[sk(t + b * NT + r * Q)];
        }
    }
    if constexpr (!FROM_REGS && !TO_REGS) __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * NT;
        const int k = j & (Ns - 1);
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b * R + r];
        if constexpr (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = INV ? cmulc(u[r], w[b][r]) : cmul(u[r], w[b][r]);
        }
        dft<R, INV>(u);
        if constexpr (TO_REGS) {
            // last stage: k = j, so output r of butterfly b is element j + r L/R
#pragma unroll
            for (int r = 0; r < R; ++r) io[b + r * NB] = u[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) x[sk(base + r * Ns)] = u[r];
        }
    }
    if constexpr (!TO_REGS) __syncthreads();
}

// OFF: offset of this stage's block in the stage twiddle table; PIDX: index
// of its factors in twr (-1: not preloaded).
template <int L, int EE, bool INV, bool IN, bool OUT, int Ns, int OFF, int PIDX>
__device__ __forceinline__ void fft_stages(float2* x, const float2* __restrict__ tab, int t, float2 (&io)[EE],
                                           const float2 (&twr)[TwN<L, EE>::v]) {
    if constexpr (Ns < L) {
        constexpr int R = fft_radix(L, EE, Ns), NB = EE / R;
        fft_stage<L, EE, R, Ns, INV, IN && Ns == 1, OUT && Ns * R == L, PIDX>(x, tab + OFF, t, io, twr);
        constexpr int NEXT = PIDX < 0 ? -1 : PIDX + (Ns > 1 ? NB * (R - 1) : 0);
        fft_stages<L, EE, INV, IN, OUT, Ns * R, OFF + (Ns > 1 ? Ns * R : 0), NEXT>(x, tab, t, io, twr);
    }
}

// In-place length-L complex FFT of x (in LDS, skewed by sk()) by the NT = L/EE
// threads t = 0..NT-1 of one transform: mixed-radix Stockham stages of radix
// min(EE, remaining length); tab: the stage twiddle table of (L, EE).  IN: the
// input is in io (io[e] = element t + e NT) rather than in x; OUT: the output
// is left in io (same layout) rather than in x.  Every thread of the
// workgroup must call it (it contains workgroup barriers); with IN, nothing
// else may be reading x when it starts.  INV: unnormalised inverse.
template <int L, int EE, bool INV, bool IN = false, bool OUT = false>
__device__ __forceinline__ void fft_lds(float2* x, const float2* __restrict__ tab, int t, float2 (&io)[EE]) {
    if constexpr (!IN) __syncthreads();
    float2 none[TwN<L, EE>::v];
    fft_stages<L, EE, INV, IN, OUT, 1, 0, -1>(x, tab, t, io, none);
}
template <int L, int EE, bool INV>
__device__ __forceinline__ void fft_lds(float2* x, const float2* __restrict__ tab, int t) {
    float2 unused[EE];
    fft_lds<L, EE, INV, false, false>(x, tab, t, unused);
}
// The same with every stage twiddle taken from twr (tw_preload of the same
// (L, EE) table for this t).
template <int L, int EE, bool INV, bool IN = false, bool OUT = false>
__device__ __forceinline__ void fft_lds_pre(float2* x, const float2 (&twr)[TwN<L, EE>::v], int t,
                                            float2 (&io)[EE]) {
    if constexpr (!IN) __syncthreads();
    fft_stages<L, EE, INV, IN, OUT, 1, 0, 0>(x, nullptr, t, io, twr);
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

// Sum of the NV x nblocks partials in fixed order; valid in thread 0.  Each
// thread keeps four independent running sums so that its loads overlap.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* part, int nblocks, double (&v)[NV], double* red) {
    const int bd = blockDim.x;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        const double* p = part + (size_t)c * nblocks;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int b = threadIdx.x;
        for (; b + 3 * bd < nblocks; b += 4 * bd) {
            s0 += p[b];
            s1 += p[b + bd];
            s2 += p[b + 2 * bd];
            s3 += p[b + 3 * bd];
        }
        for (; b < nblocks; b += bd) s0 += p[b];
        v[c] = (s0 + s1) + (s2 + s3);
    }
    block_sum<NV>(v, red);
}

// Row / column index i (any integer, e.g. a halo position) on an n-point
// axis, n a power of two: periodic (BC = 0), or mirrored about the half-
// sample points -1/2 and n - 1/2 (BC = 1, the Neumann ghost values; the
// mirror extension has period 2n).
template <int BC>
__device__ __forceinline__ int bidx(int i, int n) {
    if constexpr (BC == 0) {
        return i & (n - 1);
    } else {
        const int m = i & (2 * n - 1);
        return m < n ? m : 2 * n - 1 - m;
    }
}

}  // namespace sr
