// HIP kernels of the SR Split Bregman solver for gfx950 (MI355X).
//
// One outer iteration k of Algorithm 1 is, per inner step s = 0..S-1,
//   k_rhs       : r = tau (N(phi_s) + mu div(b - w) + mu Lap phi_s)      (eq 37,
//                 increment form) with the repulsion window sum v fused in,
//   k_row_fwd   : real-to-complex row FFTs of r (two rows per complex FFT),
//                 (k_rhs_fwd does both in one launch for rows of 64..1024
//                 points with periodic boundaries: r never goes to memory),
//   k_col_solve : column FFT -> divide by the symbol of eq (32) -> inverse,
//   k_row_inv   : complex-to-real row FFTs, phi_{s+1} = phi_s + dphi,
// then
//   k_wstep     : shrink (eq 42), project (eq 40), Bregman (eq 23), the next
//                 mu div(b - w), the outer residual r_k and phi^k <- phi^{k+1}.
//
// Every per-iteration kernel is batch-aware: blockIdx.z selects an instance
// whose planes sit at z * M * N (vector fields at z * 2 M N) from the given
// base pointers and whose device scalars are sc[z]; an instance with
// sc[z].active == 0 is skipped.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include <hip/hip_ext.h>

#include "sr_device.hpp"
#include "sr_kernels.hpp"
#include "sr_pass.hpp"

namespace sr {

// ---------------------------------------------------------------------------
// setup: Gaussian smoothing and the edge map (eq 1)
// ---------------------------------------------------------------------------
struct GaussTaps { float k[2 * kMaxGaussR + 1]; int r; };

template <int BC>
__global__ __launch_bounds__(256) void k_blur_rows(const float* __restrict__ src, float* __restrict__ dst,
                                                   int M, int N, GaussTaps gt, DevScal* sc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t zo = (size_t)blockIdx.z * M * N;
    const float* row = src + zo + (size_t)i * N;
    float acc = 0.0f;
    for (int t = -gt.r; t <= gt.r; ++t) acc += gt.k[t + gt.r] * row[bidx<BC>(j + t, N)];
    const float c = row[j];
    if (!isfinite(c)) sc[blockIdx.z].nonfinite = 1;
    dst[zo + (size_t)i * N + j] = acc;
}

template <int BC>
__global__ __launch_bounds__(256) void k_blur_cols(const float* __restrict__ src, float* __restrict__ dst,
                                                   int M, int N, GaussTaps gt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t zo = (size_t)blockIdx.z * M * N;
    src += zo;
    float acc = 0.0f;
    for (int t = -gt.r; t <= gt.r; ++t) acc += gt.k[t + gt.r] * src[(size_t)bidx<BC>(i + t, M) * N + j];
    dst[zo + (size_t)i * N + j] = acc;
}

// g = 1 / (1 + rho |grad fs|^s), central differences.
template <int BC>
__global__ __launch_bounds__(256) void k_edge(const float* __restrict__ fs, float* __restrict__ g,
                                              int M, int N, float rho, int s_exp) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t zo = (size_t)blockIdx.z * M * N;
    fs += zo;
    g += zo;
    const float gx = 0.5f * (fs[(size_t)bidx<BC>(i + 1, M) * N + j] - fs[(size_t)bidx<BC>(i - 1, M) * N + j]);
    const float gy = 0.5f * (fs[(size_t)i * N + bidx<BC>(j + 1, N)] - fs[(size_t)i * N + bidx<BC>(j - 1, N)]);
    const float m2 = gx * gx + gy * gy;
    const float m = (s_exp == 2) ? m2 : sqrtf(m2);
    g[(size_t)i * N + j] = 1.0f / (1.0f + rho * m);
}

// State initialisation of Algorithm 1: phi = phi0, w = grad+ phi0 (or 0),
// b = 0, D = mu div-(b - w) = -mu Lap phi0 (or 0).
template <int BC>
__global__ __launch_bounds__(256) void k_init(const float* __restrict__ phi0, float* __restrict__ P0,
                                              float* __restrict__ W, float* __restrict__ B,
                                              float* __restrict__ D, int M, int N, float mu, int w0_mode,
                                              DevScal* sc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t MN = (size_t)M * N, o = (size_t)i * N + j;
    const size_t z = blockIdx.z;
    phi0 += z * MN; P0 += z * MN; W += 2 * z * MN; B += 2 * z * MN; D += z * MN;
    const float p = phi0[o];
    if (!isfinite(p)) sc[z].nonfinite = 1;
    const float pd = phi0[(size_t)bidx<BC>(i + 1, M) * N + j];
    const float pr = phi0[(size_t)i * N + bidx<BC>(j + 1, N)];
    const float pu = phi0[(size_t)bidx<BC>(i - 1, M) * N + j];
    const float pl = phi0[(size_t)i * N + bidx<BC>(j - 1, N)];
    P0[o] = p;
    B[o] = 0.0f;
    B[MN + o] = 0.0f;
    if (w0_mode == 0) {
        W[o] = pd - p;
        W[MN + o] = pr - p;
        D[o] = -mu * ((pd + pu + pr + pl) - 4.0f * p);
    } else {
        W[o] = 0.0f;
        W[MN + o] = 0.0f;
        D[o] = 0.0f;
    }
}

// D = mu div-(b - w) (eq 36) from a given state (checkpoint restore); with
// Neumann boundaries the divergence is the negative adjoint of the forward
// difference (terms at index -1 and at the last index dropped).
template <int BC>
__global__ __launch_bounds__(256) void k_set_D(const float* __restrict__ W, const float* __restrict__ B,
                                               float* __restrict__ D, int M, int N, float mu) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t MN = (size_t)M * N, o = (size_t)i * N + j;
    const size_t ou = (size_t)bidx<BC>(i - 1, M) * N + j;
    const size_t ol = (size_t)i * N + bidx<BC>(j - 1, N);
    float e1 = B[o] - W[o], e1u = B[ou] - W[ou];
    float e2 = B[MN + o] - W[MN + o], e2l = B[MN + ol] - W[MN + ol];
    if constexpr (BC == 1) {
        if (i == M - 1) e1 = 0.0f;
        if (i == 0) e1u = 0.0f;
        if (j == N - 1) e2 = 0.0f;
        if (j == 0) e2l = 0.0f;
    }
    D[o] = mu * ((e1 - e1u) + (e2 - e2l));
}

__global__ void k_reset_scal(DevScal* sc, int n, int active) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= n) return;
    DevScal& s = sc[z];
    s.counter = 0u; s.inner_done = 0; s.active = active; s.nonfinite = 0;
    s.k = 0; s.inner_steps = 0; s.r_last = -1.0; s.inner_rel = -1.0;
    s.energy[0] = s.energy[1] = s.energy[2] = 0.0;
    s.max_iter = 0; s.min_iter = 0; s.tol_outer = 0.0; s.converged = 0; s.spare = 0;
}

__global__ void k_set_k(DevScal* sc, long long k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { sc->k = k; sc->inner_done = 0; sc->counter = 0u; }
}

// ---------------------------------------------------------------------------
// shared tile machinery: u = w h(phi) on the tile plus a halo, then the
// separable window sum.  K_pq = a_p a_q exactly, so the (2R+1)^2-tap sum is
// done as a row pass then a column pass over LDS.
// ---------------------------------------------------------------------------
// Horizontal pass: sh[e][j] = sum_q a_q su[e][j+q] for e < eh, j < cw.
__device__ __forceinline__ void window_rows(const float* su1, const float* su2, float* sh1, float* sh2,
                                            int eh, int ew, int cw, const KParams& kp) {
    const int R2 = 2 * kp.R;
    for (int e = threadIdx.x; e < eh * cw; e += blockDim.x) {
        const int ei = e / cw, j = e - ei * cw;
        const float* r1 = su1 + ei * ew + j;
        const float* r2 = su2 + ei * ew + j;
        float a1 = 0.0f, a2 = 0.0f;
        for (int q = 0; q <= R2; ++q) { a1 += kp.taps[q] * r1[q]; a2 += kp.taps[q] * r2[q]; }
        sh1[e] = a1;
        sh2[e] = a2;
    }
}

__device__ __forceinline__ void window_col(const float* sh1, const float* sh2, int ci, int cj, int cw,
                                           const KParams& kp, float& v1, float& v2) {
    const int R2 = 2 * kp.R;
    float a1 = 0.0f, a2 = 0.0f;
    for (int p = 0; p <= R2; ++p) {
        a1 += kp.taps[p] * sh1[(ci + p) * cw + cj];
        a2 += kp.taps[p] * sh2[(ci + p) * cw + cj];
    }
    v1 = a1;
    v2 = a2;
}

// ---------------------------------------------------------------------------
// inner rhs (eq 37) in increment form:
//   r = tau ( -gamma g |w| delta'(phi) + alpha g delta(phi)
//             + 2 beta h'(phi) w . v + D + mu Lap phi ),   D = mu div(b - w)
// ---------------------------------------------------------------------------
// Tile placement: workgroups are dealt to the 8 XCDs round-robin by linear
// id, so linear id b is remapped to tile (b % 8) * (nb / 8) + b / 8.  Each
// XCD then owns a horizontal band of tiles and the halo rows two vertically
// adjacent tiles share are fetched into the same L2.
__device__ __forceinline__ void xcd_tile(int& tx, int& ty) {
    const int gx = gridDim.x, nb = gridDim.x * gridDim.y;
    int b = blockIdx.y * gx + blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    ty = b / gx;
    tx = b - ty * gx;
}

template <int TH, int R>
struct RhsTile {
    static constexpr int TW = kTileW, T = kRhsThreads;
    static constexpr int EH = TH + 2 * R, EW = TW + 2 * R, NEXT = EH * EW;
    static constexpr int PH = TH + 2, PW = TW + 2;
    static constexpr int NE = (NEXT + T - 1) / T, NHZ = (EH * TW + T - 1) / T, NO = TH * TW / T;
    static constexpr size_t lds_floats = 2 * NEXT + 2 * EH * TW + PH * PW;
};

template <int TH, int R, int BC>
__global__ __launch_bounds__(kRhsThreads) void k_rhs(KParams kp, int M, int N,
                                                      const float* __restrict__ phi_s,
                                                      const float* __restrict__ W,
                                                      const float* __restrict__ g,
                                                      const float* __restrict__ D,
                                                      float* __restrict__ out,
                                                      const double* __restrict__ fin_part, int fin_nb,
                                                      double* __restrict__ fin_rhist, DevScal* sc) {
    using C = RhsTile<TH, R>;
    constexpr int TW = C::TW, T = C::T, EH = C::EH, EW = C::EW, NEXT = C::NEXT, PW = C::PW, PH = C::PH;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    if (fin_part != nullptr && blockIdx.x == 0 && blockIdx.y == 0) {   // folded finalize (FinFold)
        __shared__ double fred[2 * 16];
        fin_outer_body(fin_part, fin_nb, fin_rhist, sc[z], z, fred);
    }
    const size_t MN = (size_t)M * N;
    phi_s += z * MN; W += 2 * z * MN; g += z * MN; D += z * MN; out += z * MN;

    extern __shared__ float lds[];
    float* su1 = lds;
    float* su2 = su1 + NEXT;
    float* sh1 = su2 + NEXT;
    float* sh2 = sh1 + EH * TW;
    float* sphi = sh2 + EH * TW;
    int tx, ty;
    xcd_tile(tx, ty);
    const int i0 = ty * TH, j0 = tx * TW;
    const int tid = threadIdx.x;

    // phase 1: phi on the extended tile and D on the tile; is any pixel of
    // the extended tile inside the band |phi| <= l + eps?
    const float lim = kp.band_l + kp.eps;
    float lp[C::NE];
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const int ei = e / EW, ej = e - ei * EW;
            lp[u] = phi_s[(size_t)bidx<BC>(i0 - R + ei, M) * N + bidx<BC>(j0 - R + ej, N)];
        }
    }
    float dv[C::NO];
#pragma unroll
    for (int u = 0; u < C::NO; ++u) {
        const int e = tid + u * T;
        dv[u] = D[(size_t)bidx<BC>(i0 + e / TW, M) * N + bidx<BC>(j0 + (e % TW), N)];
    }
    int inband = 0;
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const int ei = e / EW, ej = e - ei * EW;
            inband |= (lp[u] <= lim && lp[u] >= -lim);
            const int si = ei - R + 1, sj = ej - R + 1;
            if ((unsigned)si < (unsigned)PH && (unsigned)sj < (unsigned)PW) sphi[si * PW + sj] = lp[u];
        }
    }
    if constexpr (R == 0) {
        for (int e = tid; e < PH * PW; e += T) {
            const int si = e / PW, sj = e - si * PW;
            sphi[e] = phi_s[(size_t)bidx<BC>(i0 - 1 + si, M) * N + bidx<BC>(j0 - 1 + sj, N)];
        }
    }
    const bool band = __syncthreads_or(inband) != 0;
    if (!band) {
        // h, h', delta, delta' vanish on the whole extended tile: v = 0 and
        // the force is zero, so r = tau (D + mu Lap phi) exactly.
#pragma unroll
        for (int u = 0; u < C::NO; ++u) {
            const int e = tid + u * T;
            const int i = e / TW, j = e - i * TW;
            const int gi = i0 + i, gj = j0 + j;
            const float* sp = sphi + (i + 1) * PW + (j + 1);
            const float p = sp[0];
            const float lap = (sp[-PW] + sp[PW]) + (sp[-1] + sp[1]) - 4.0f * p;
            const float force = 0.0f;
            if (gi < M && gj < N) out[(size_t)gi * N + gj] = kp.tau * (force + dv[u] + kp.mu * lap);
        }
        return;
    }
    // band tile: u = w h(phi) on the extended tile
    float l1[C::NE], l2[C::NE];
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const int ei = e / EW, ej = e - ei * EW;
            const size_t o = (size_t)bidx<BC>(i0 - R + ei, M) * N + bidx<BC>(j0 - R + ej, N);
            l1[u] = W[o];
            l2[u] = W[MN + o];
        }
    }
    float w1v[C::NO], w2v[C::NO], gv[C::NO];
#pragma unroll
    for (int u = 0; u < C::NO; ++u) {
        const int e = tid + u * T;
        const size_t o = (size_t)bidx<BC>(i0 + e / TW, M) * N + bidx<BC>(j0 + (e % TW), N);
        w1v[u] = W[o]; w2v[u] = W[MN + o]; gv[u] = g[o];
    }
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const float h = band_h(lp[u], kp);
            su1[e] = l1[u] * h;
            su2[e] = l2[u] * h;
        }
    }
    __syncthreads();
    // phase 2: row pass of the separable window
#pragma unroll
    for (int u = 0; u < C::NHZ; ++u) {
        const int e = tid + u * T;
        if (e < EH * TW) {
            const int ei = e / TW, j = e - ei * TW;
            const float* r1 = su1 + ei * EW + j;
            const float* r2 = su2 + ei * EW + j;
            float a1 = 0.0f, a2 = 0.0f;
#pragma unroll
            for (int q = 0; q <= 2 * R; ++q) { a1 += kp.taps[q] * r1[q]; a2 += kp.taps[q] * r2[q]; }
            sh1[e] = a1;
            sh2[e] = a2;
        }
    }
    __syncthreads();
    // phase 3: column pass and the pointwise rhs
#pragma unroll
    for (int u = 0; u < C::NO; ++u) {
        const int e = tid + u * T;
        const int i = e / TW, j = e - i * TW;
        const int gi = i0 + i, gj = j0 + j;
        const float* sp = sphi + (i + 1) * PW + (j + 1);
        const float p = sp[0];
        const float lap = (sp[-PW] + sp[PW]) + (sp[-1] + sp[1]) - 4.0f * p;
        // the force vanishes outside the band (delta, delta' and h' are 0)
        float force = 0.0f;
        if (p <= lim && p >= -lim) {
            float v1 = 0.0f, v2 = 0.0f;
#pragma unroll
            for (int pp = 0; pp <= 2 * R; ++pp) {
                v1 += kp.taps[pp] * sh1[(i + pp) * TW + j];
                v2 += kp.taps[pp] * sh2[(i + pp) * TW + j];
            }
            float dl, ddl, h, dh;
            dirac_d(p, kp, dl, ddl);
            band_h_dh(p, kp, h, dh);
            const float w1 = w1v[u], w2 = w2v[u], gg = gv[u];
            const float wn = sqrtf(w1 * w1 + w2 * w2);
            force = -kp.gamma * gg * wn * ddl + kp.alpha * gg * dl + 2.0f * kp.beta * dh * (w1 * v1 + w2 * v2);
        }
        if (gi < M && gj < N) out[(size_t)gi * N + gj] = kp.tau * (force + dv[u] + kp.mu * lap);
    }
}

// ---------------------------------------------------------------------------
// repulsion field alone (component operator): v = K (*) (w h(phi))
// ---------------------------------------------------------------------------
template <int TH, int BC>
__global__ __launch_bounds__(kTileThreads) void k_repulsion(KParams kp, int M, int N,
                                                            const float* __restrict__ phi,
                                                            const float* __restrict__ W,
                                                            float* __restrict__ V) {
    constexpr int TW = kTileW;
    const size_t MN = (size_t)M * N;
    extern __shared__ float lds[];
    const int R = kp.R;
    const int eh = TH + 2 * R, ew = TW + 2 * R;
    float* su1 = lds;
    float* su2 = su1 + eh * ew;
    float* sh1 = su2 + eh * ew;
    float* sh2 = sh1 + eh * TW;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;
    for (int e = threadIdx.x; e < eh * ew; e += blockDim.x) {
        const int ei = e / ew, ej = e - ei * ew;
        const int gi = bidx<BC>(i0 - R + ei, M), gj = bidx<BC>(j0 - R + ej, N);
        const size_t o = (size_t)gi * N + gj;
        const float h = band_h(phi[o], kp);
        su1[e] = W[o] * h;
        su2[e] = W[MN + o] * h;
    }
    __syncthreads();
    window_rows(su1, su2, sh1, sh2, eh, ew, TW, kp);
    __syncthreads();
    for (int e = threadIdx.x; e < TH * TW; e += blockDim.x) {
        const int i = e / TW, j = e - i * TW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= M || gj >= N) continue;
        float v1, v2;
        window_col(sh1, sh2, i, j, TW, kp, v1, v2);
        const size_t o = (size_t)gi * N + gj;
        V[o] = v1;
        V[MN + o] = v2;
    }
}

// ---------------------------------------------------------------------------
// FFT passes of the semi-implicit solve (eqs 31-33)
// ---------------------------------------------------------------------------
// RT tiles (8 RT rows, 4 RT complex transforms) per workgroup.  LR > 0 fixes
// log2(rows per workgroup) at compile time (the common launch shapes, so the
// index arithmetic folds); LR = 0 takes it from lrpw.
template <int N, int LR>
__global__ __launch_bounds__(1024) void k_row_fwd(const float* __restrict__ src, float2* __restrict__ spec,
                                                  const float2* __restrict__ stN, int M, int lrpw_rt, DevScal* sc) {
    const int lrpw = LR ? LR : lrpw_rt;
    constexpr int NT = FftShape<N>::NT, E = FftShape<N>::E, H = N / 2;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    src += (size_t)z * M * N;
    spec += (size_t)z * M * H;
    extern __shared__ float2 xs[];
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int row0 = row_piece0(blockIdx.x, gridDim.x, lrpw);   // 2^lrpw rows (2^(lrpw-1) transforms)
    const size_t ra = (size_t)(row0 + 2 * g) * N, rb = ra + N;
    constexpr int LX = LdsLen<N>::v;
    float2* x = xs + g * LX;
    float2 io[E];   // element t + e NT of the complex row: the first stage's inputs
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = t + e * NT;
        io[e] = make_float2(src[ra + n], src[rb + n]);
    }
    constexpr bool PRE = E <= 4;   // all stage twiddles in registers
    float2 twr[TwN<N, E>::v];
    if constexpr (PRE) {
        tw_preload<N, E>(stN, t, twr);
        fft_lds_pre<N, E, false, true, false>(x, twr, t, io);
    } else {
        fft_lds<N, E, false, true, false>(x, stN, t, io);
    }
    // Whole 8-row tiles are one contiguous run of 4N float2 each; with fewer
    // rows per workgroup it writes its rows of every 8-row run.
    const int nthr = LR ? ((1 << LR) / 2) * NT : (int)blockDim.x;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = threadIdx.x + e * nthr;
        int r, kk;
        size_t di;
        if (lrpw >= 3) {
            r = o & 7;
            kk = (o >> 3) & (H - 1);
            r += ((o >> 3) / H) * 8;
            di = (size_t)row0 * H + o;
        } else {
            r = o & ((1 << lrpw) - 1);
            kk = o >> lrpw;
            di = ((size_t)(row0 >> 3) * H + kk) * 8 + (row0 & 7) + r;
        }
        const float2* xz = xs + (r >> 1) * LX;
        const float2 Zk = xz[sk(kk)];
        float2 out;
        if (kk == 0) {
            const float2 ZH = xz[sk(H)];
            out = (r & 1) ? make_float2(Zk.y, ZH.y) : make_float2(Zk.x, ZH.x);
        } else {
            const float2 Zm = xz[sk(N - kk)];
            out = (r & 1) ? make_float2(0.5f * (Zk.y + Zm.y), -0.5f * (Zk.x - Zm.x))
                          : make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
        }
        spec[di] = out;
    }
}

// G adjacent spectrum columns per workgroup: forward column FFT, division
// by M N (1 + tau mu (4 - 2cos(2 pi l1/M) - 2cos(2 pi l2/N))), inverse FFT.
// Column 0 holds two real-signal spectra (l2 = 0 and l2 = N/2) packed as
// a + i b; they are separated, scaled by their own symbols and re-packed.
// GT > 0 fixes G at compile time (the common shape); GT = 0 takes G, lrun.
template <int M, int GT>
// VGPR cap from ColWaves: at most 64 VGPRs (8 waves per SIMD) for 8-element
// transforms, so four 512-thread workgroups of the 4096-point pass share a
// CU (their LDS fits four times), which the pass needs to overlap loads with
// transforms.
__global__ __attribute__((amdgpu_flat_work_group_size(1, 1024), amdgpu_waves_per_eu(ColWaves<M>::v))) void k_col_solve(float2* __restrict__ spec, const float2* __restrict__ twM,
                                                    const float2* __restrict__ twN, const float2* __restrict__ stM,
                                                    int N, int G_rt, int lrun_rt, float taumu, float inv_mn,
                                                    DevScal* sc) {
    const int G = GT ? GT : G_rt;
    const int lrun = GT ? Ilog2<kSpecTile * (GT ? GT : 1)>::v : lrun_rt;
    const int nthr = GT ? FftShape<M, ColE<M>::v>::NT * GT : (int)blockDim.x;
    constexpr int NT = FftShape<M, ColE<M>::v>::NT, E = FftShape<M, ColE<M>::v>::E;
    constexpr int LD = LdsLen<M>::v;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    const int H = N / 2;
    spec += (size_t)z * M * H;
    extern __shared__ float2 xs[];
    // Single columns: columns 2c and 2c + 1 (one 128-byte run per 8-row tile)
    // go to workgroups b and b + 8, which share an XCD, so the run is read
    // from HBM once.
    int k0 = blockIdx.x * G;
    if (G == 1 && (gridDim.x & 15) == 0) {
        const int b = blockIdx.x, s = b >> 3;
        k0 = (((s >> 1) << 3) + (b & 7)) * 2 + (s & 1);
    }
    const int run = kSpecTile * G;                 // contiguous float2 per row tile (2^lrun)
    float2* base = spec + (size_t)k0 * kSpecTile;
    // M * G elements over NT * G threads: exactly E per thread, all loads first.
    // With one column per workgroup, element idx of the column is thread
    // idx % NT's input e = idx / NT of the first stage: no staging in LDS.
    constexpr bool ONE = GT == 1;
    float2 io[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = threadIdx.x + e * nthr;
        io[e] = base[(size_t)(idx >> lrun) * H * kSpecTile + (idx & (run - 1))];
    }
    if constexpr (!ONE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * nthr;
            const int rem = idx & (run - 1);
            xs[(rem >> 3) * LD + sk((idx >> lrun) * kSpecTile + (rem & 7))] = io[e];
        }
    }
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int col = k0 + g;
    float2* x = xs + g * LD;
    // The cosines of the symbol, loaded with the data: the transform's
    // barriers would keep the compiler from issuing them any earlier than
    // their use, after the forward transform.
    const float cn = 2.0f * twN[col].x;
    float cmv[E / 2 + 1];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) cmv[e] = 2.0f * twM[t + e * NT].x;
    cmv[E / 2] = 2.0f * twM[M / 2].x;
    // up to 2048 points every stage twiddle is loaded once into registers
    // and serves the forward and the inverse transform
    constexpr bool PRE = E <= 4;
    float2 twr[TwN<M, E>::v];
    if constexpr (PRE) {
        tw_preload<M, E>(stM, t, twr);
        fft_lds_pre<M, E, false, ONE, false>(x, twr, t, io);
    } else {
        fft_lds<M, E, false, ONE, false>(x, stM, t, io);
    }
    // Divide by the symbol.  The symbol is even in l1, so each thread owns the
    // mirror pair (l, M - l): column 0's two packed real spectra mix Z[l]
    // with conj(Z[M - l]), every other column scales pointwise.
    auto scale_pair = [&](int l, float cm) {
        const int m = (M - l) & (M - 1);
        float hp, hm;
        // v_rcp_f32 (1 ulp) in place of an IEEE division: the symbol is >= 1
        if (col != 0) {
            hp = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (4.0f - cm - cn));
            hm = 0.0f;
        } else {
            const float p = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (2.0f - cm));   // l2 = 0
            const float q = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (6.0f - cm));   // l2 = N/2
            hp = 0.5f * (p + q);
            hm = 0.5f * (p - q);
        }
        const float2 zl = x[sk(l)], zm = x[sk(m)];
        x[sk(l)] = make_float2(hp * zl.x + hm * zm.x, hp * zl.y - hm * zm.y);
        if (m != l) x[sk(m)] = make_float2(hp * zm.x + hm * zl.x, hp * zm.y - hm * zl.y);
    };
#pragma unroll
    for (int e = 0; e < E / 2; ++e) scale_pair(t + e * NT, cmv[e]);   // l in [0, M/2)
    if (t == 0) scale_pair(M / 2, cmv[E / 2]);
    // A fresh copy of t (through an empty asm) keeps the compiler from holding
    // the forward transform's LDS addresses live across the division.
    int t_inv = t;
    asm volatile("" : "+v"(t_inv));
    if constexpr (PRE) fft_lds_pre<M, E, true, false, ONE>(x, twr, t_inv, io);
    else fft_lds<M, E, true, false, ONE>(x, stM, t_inv, io);
    if constexpr (!ONE) __syncthreads();
    // An empty asm on the thread index keeps the compiler from computing the
    // store addresses at the top and holding them (or spilling them) through
    // both transforms.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if constexpr (ONE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * nthr;
            base[(size_t)(idx >> lrun) * H * kSpecTile + (idx & (run - 1))] = io[e];
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = tid + e * nthr;
        const int q = idx >> lrun, rem = idx & (run - 1);
        base[(size_t)q * H * kSpecTile + rem] = xs[(rem >> 3) * LD + sk(q * kSpecTile + (rem & 7))];
    }
}

// Inverse row FFTs (two rows per complex FFT) and phi_{s+1} = phi_s + dphi.
// With tol_inner > 0, also the inner stop rule ||dphi|| / (||phi_s|| + 1e-6)
// <= tol (grid-wide sum, last workgroup decides).  Once the rule has fired,
// the remaining inner steps of the outer iteration copy phi_s through.
template <int N, int LR>
__global__ __launch_bounds__(1024) void k_row_inv(const float2* __restrict__ spec, const float* __restrict__ phi_in,
                                                  float* __restrict__ phi_out, const float2* __restrict__ stN,
                                                  int M, int lrpw_rt, float tol_inner, double* __restrict__ part,
                                                  DevScal* sc) {
    const int lrpw = LR ? LR : lrpw_rt;
    constexpr int NT = FftShape<N>::NT, E = FftShape<N>::E, H = N / 2;
    const int z = blockIdx.z;
    DevScal& S = sc[z];
    if (!S.active) return;
    const size_t MN = (size_t)M * N;
    spec += (size_t)z * M * H;
    if (phi_in) phi_in += z * MN;
    phi_out += z * MN;
    const int row0 = row_piece0(blockIdx.x, gridDim.x, lrpw);
    if (S.inner_done) {
        const size_t base = (size_t)row0 * N;
        for (int idx = threadIdx.x; idx < (N << lrpw); idx += blockDim.x)
            phi_out[base + idx] = phi_in ? phi_in[base + idx] : 0.0f;
        return;
    }
    extern __shared__ float2 xs[];
    __shared__ double red[2 * 16];
    constexpr int LX = LdsLen<N>::v;
    const int nthr = LR ? ((1 << LR) / 2) * NT : (int)blockDim.x;
    // stage the half spectra: row a of transform gg at x[k], row b at x[H + k]
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = threadIdx.x + e * nthr;
        int r, kk;
        size_t si;
        if (lrpw >= 3) {
            r = o & 7;
            kk = (o >> 3) & (H - 1);
            r += ((o >> 3) / H) * 8;
            si = (size_t)row0 * H + o;
        } else {
            r = o & ((1 << lrpw) - 1);
            kk = o >> lrpw;
            si = ((size_t)(row0 >> 3) * H + kk) * 8 + (row0 & 7) + r;
        }
        xs[(r >> 1) * LX + sk((r & 1) * H + kk)] = spec[si];
    }
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    // stage twiddles in registers (up to 1024 points), loaded with phi_s
    constexpr bool PRE = E <= 4;
    float2 twr[TwN<N, E>::v];
    if constexpr (PRE) tw_preload<N, E>(stN, t, twr);
    // phi_s of this thread's outputs, loaded now so that the loads overlap the transform
    const size_t ra = (size_t)(row0 + 2 * g) * N, rb = ra + N;
    float pav[E], pbv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = t + e * NT;
        pav[e] = phi_in ? phi_in[ra + n] : 0.0f;
        pbv[e] = phi_in ? phi_in[rb + n] : 0.0f;
    }
    __syncthreads();
    float2* x = xs + g * LX;
    float2 va[E / 2], vb[E / 2];
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int k = t + e * NT;
        va[e] = x[sk(k)];
        vb[e] = x[sk(H + k)];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int k = t + e * NT;
        const float2 Xa = va[e], Xb = vb[e];
        if (k == 0) {
            x[sk(0)] = make_float2(Xa.x, Xb.x);
            x[sk(H)] = make_float2(Xa.y, Xb.y);
        } else {
            x[sk(k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            x[sk(N - k)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
        }
    }
    float2 io[E];   // the last stage's outputs: element t + e NT
    if constexpr (PRE) fft_lds_pre<N, E, true, false, true>(x, twr, t, io);
    else fft_lds<N, E, true, false, true>(x, stN, t, io);
    double sd = 0.0, sp = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = t + e * NT;
        const float2 Zv = io[e];
        const float pa = pav[e], pb = pbv[e];
        phi_out[ra + n] = pa + Zv.x;
        phi_out[rb + n] = pb + Zv.y;
        sd += (double)Zv.x * Zv.x + (double)Zv.y * Zv.y;
        sp += (double)pa * pa + (double)pb * pb;
    }
    if (tol_inner > 0.0f) {
        double v[2] = {sd, sp};
        const int nb = gridDim.x;
        store_partials<2>(v, part + (size_t)z * 2 * nb, nb, blockIdx.x, red);
    }
}

// Inner stop rule after an executed inner step: ||dphi|| / (||phi_s|| + 1e-6) <= tol.
__global__ __launch_bounds__(1024) void k_fin_inner(const double* __restrict__ part, int nb, float tol_inner,
                                                   DevScal* sc) {
    __shared__ double red[2 * 16];
    const int z = blockIdx.x;
    DevScal& S = sc[z];
    if (!S.active || S.inner_done) return;
    double v[2];
    sum_partials<2>(part + (size_t)z * 2 * nb, nb, v, red);
    if (threadIdx.x == 0) {
        const double rel = sqrt(v[0]) / (sqrt(v[1]) + 1e-6);
        S.inner_rel = rel;
        S.inner_steps += 1;
        if (rel <= (double)tol_inner) S.inner_done = 1;
    }
}

// ---------------------------------------------------------------------------
// w step: B (eq 41), shrink (eq 42) + projection (eq 40) in gate form,
// Bregman (eq 23), next D = mu div(b - w), outer residual r_k.  phi^{k+1}
// stays where the last inner step wrote it (the caller alternates the phi^k
// and phi^{k+1} planes with the iteration's parity, as it does w and b).
// The tile computes w, b on one extra row above and column left so that the
// backward divergence of its own pixels is local.
// ---------------------------------------------------------------------------
template <int TH, int R, int TT>
struct WTile {
    static constexpr int TW = kTileW, T = TT;
    static constexpr int CH = TH + 1, CW = TW + 1;           // computed region (one extra row / column)
    static constexpr int EH = CH + 2 * R, EW = CW + 2 * R, NEXT = EH * EW;
    static constexpr int PH = TH + 2, PW = TW + 2;
    static constexpr int NE = (NEXT + T - 1) / T, NHZ = (EH * CW + T - 1) / T;
    static constexpr int NC = (CH * CW + T - 1) / T, NO = TH * TW / T;
    static constexpr size_t su_floats = (2 * NEXT > 2 * CH * CW) ? 2 * NEXT : 2 * CH * CW;
    static constexpr size_t lds_floats = su_floats + 2 * EH * CW + PH * PW;
};

template <int TH, int R, int TT, int BC>
__global__ __launch_bounds__(TT) void k_wstep(KParams kp, int M, int N,
                                                        const float* __restrict__ phin,
                                                        const float* __restrict__ Pk,
                                                        const float* __restrict__ Wold,
                                                        const float* __restrict__ Bold,
                                                        const float* __restrict__ g,
                                                        float* __restrict__ Wnew, float* __restrict__ Bnew,
                                                        float* __restrict__ D, double* __restrict__ part,
                                                        double* __restrict__ rhist, int sweep, DevScal* sc) {
    using C = WTile<TH, R, TT>;
    constexpr int TW = C::TW, T = C::T, CH = C::CH, CW = C::CW, EH = C::EH, EW = C::EW, NEXT = C::NEXT;
    constexpr int PH = C::PH, PW = C::PW;
    const int z = blockIdx.z;
    DevScal& S = sc[z];
    if (!S.active) return;
    const size_t MN = (size_t)M * N;
    phin += z * MN; Pk += z * MN; Wold += 2 * z * MN; Bold += 2 * z * MN; g += z * MN;
    Wnew += 2 * z * MN; Bnew += 2 * z * MN; D += z * MN;

    extern __shared__ float lds[];
    __shared__ double red[2 * 16];
    float* su1 = lds;
    float* su2 = su1 + NEXT;
    float* sh1 = lds + C::su_floats;
    float* sh2 = sh1 + EH * CW;
    float* sphi = sh2 + EH * CW;          // PH x PW, origin (i0-1, j0-1)
    float* sd1 = lds;                     // (b - w) after the row pass, aliases su
    float* sd2 = lds + CH * CW;
    int tx, ty;
    xcd_tile(tx, ty);
    const int i0 = ty * TH, j0 = tx * TW;
    const int tid = threadIdx.x;

    const float lim = kp.band_l + kp.eps;
    float lp[C::NE];
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const int ei = e / EW, ej = e - ei * EW;
            lp[u] = phin[(size_t)bidx<BC>(i0 - 1 - R + ei, M) * N + bidx<BC>(j0 - 1 - R + ej, N)];
        }
    }
    // b on the computed region and phi^k on the tile (both paths need them)
    float b1v[C::NC], b2v[C::NC];
#pragma unroll
    for (int u = 0; u < C::NC; ++u) {
        const int e = tid + u * T;
        if (e < CH * CW) {
            const int ci = e / CW, cj = e - ci * CW;
            const size_t o = (size_t)bidx<BC>(i0 - 1 + ci, M) * N + bidx<BC>(j0 - 1 + cj, N);
            b1v[u] = Bold[o]; b2v[u] = Bold[MN + o];
        }
    }
    float pold[C::NO];
#pragma unroll
    for (int u = 0; u < C::NO; ++u) {
        const int e = tid + u * T;
        pold[u] = Pk[(size_t)bidx<BC>(i0 + e / TW, M) * N + bidx<BC>(j0 + (e % TW), N)];
    }
    int inband = 0;
#pragma unroll
    for (int u = 0; u < C::NE; ++u) {
        const int e = tid + u * T;
        if (e < NEXT) {
            const int ei = e / EW, ej = e - ei * EW;
            inband |= (lp[u] <= lim && lp[u] >= -lim);
            const int si = ei - R, sj = ej - R;
            if ((unsigned)si < (unsigned)PH && (unsigned)sj < (unsigned)PW) sphi[si * PW + sj] = lp[u];
        }
    }
    if constexpr (R == 0) {
        for (int e = tid; e < PH * PW; e += T) {
            const int si = e / PW, sj = e - si * PW;
            sphi[e] = phin[(size_t)bidx<BC>(i0 - 1 + si, M) * N + bidx<BC>(j0 - 1 + sj, N)];
        }
    }
    const bool band = __syncthreads_or(inband) != 0;
    if (band) {
        float l1[C::NE], l2[C::NE];
#pragma unroll
        for (int u = 0; u < C::NE; ++u) {
            const int e = tid + u * T;
            if (e < NEXT) {
                const int ei = e / EW, ej = e - ei * EW;
                const size_t o = (size_t)bidx<BC>(i0 - 1 - R + ei, M) * N + bidx<BC>(j0 - 1 - R + ej, N);
                l1[u] = Wold[o];
                l2[u] = Wold[MN + o];
            }
        }
        float gv[C::NC];
#pragma unroll
        for (int u = 0; u < C::NC; ++u) {
            const int e = tid + u * T;
            if (e < CH * CW) {
                const int ci = e / CW, cj = e - ci * CW;
                gv[u] = g[(size_t)bidx<BC>(i0 - 1 + ci, M) * N + bidx<BC>(j0 - 1 + cj, N)];
            }
        }
#pragma unroll
        for (int u = 0; u < C::NE; ++u) {
            const int e = tid + u * T;
            if (e < NEXT) {
                const float h = band_h(lp[u], kp);
                su1[e] = l1[u] * h;
                su2[e] = l2[u] * h;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < C::NHZ; ++u) {
            const int e = tid + u * T;
            if (e < EH * CW) {
                const int ei = e / CW, j = e - ei * CW;
                const float* r1 = su1 + ei * EW + j;
                const float* r2 = su2 + ei * EW + j;
                float a1 = 0.0f, a2 = 0.0f;
#pragma unroll
                for (int q = 0; q <= 2 * R; ++q) { a1 += kp.taps[q] * r1[q]; a2 += kp.taps[q] * r2[q]; }
                sh1[e] = a1;
                sh2[e] = a2;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < C::NC; ++u) {
            const int e = tid + u * T;
            if (e < CH * CW) {
                const int ci = e / CW, cj = e - ci * CW;
                float v1 = 0.0f, v2 = 0.0f;
#pragma unroll
                for (int pp = 0; pp <= 2 * R; ++pp) {
                    v1 += kp.taps[pp] * sh1[(ci + pp) * CW + cj];
                    v2 += kp.taps[pp] * sh2[(ci + pp) * CW + cj];
                }
                const float* sp = sphi + ci * PW + cj;
                const float p = sp[0];
                const float G1 = sp[PW] - p, G2 = sp[1] - p;
                const float b1 = b1v[u], b2 = b2v[u];
                const float h = band_h(p, kp);
                float H_, dl;
                heav_dirac(p, kp.eps, kp.inv_eps, H_, dl);
                const float B1 = G1 + b1 + kp.c_rep * h * v1;
                const float B2 = G2 + b2 + kp.c_rep * h * v2;
                const float thr = kp.c_thr * gv[u] * dl;
                const float nb = sqrtf(B1 * B1 + B2 * B2);
                float w1 = 0.0f, w2 = 0.0f;
                if (nb > thr && nb > kp.zero_tol) { w1 = B1 / nb; w2 = B2 / nb; }
                const float bn1 = b1 + G1 - w1, bn2 = b2 + G2 - w2;
                sd1[e] = bn1 - w1;
                sd2[e] = bn2 - w2;
                if (ci >= 1 && cj >= 1 && i0 - 1 + ci < M && j0 - 1 + cj < N) {
                    const size_t o = (size_t)(i0 - 1 + ci) * N + (j0 - 1 + cj);
                    Wnew[o] = w1; Wnew[MN + o] = w2;
                    if (!sweep) { Bnew[o] = bn1; Bnew[MN + o] = bn2; }
                }
            }
        }
    } else {
        // no band pixel on the extended tile: v = 0, h = 0 and the threshold
        // is 0, so B = grad phi + b exactly and the gate is |B| > zero_tol.
#pragma unroll
        for (int u = 0; u < C::NC; ++u) {
            const int e = tid + u * T;
            if (e < CH * CW) {
                const int ci = e / CW, cj = e - ci * CW;
                const float* sp = sphi + ci * PW + cj;
                const float p = sp[0];
                const float G1 = sp[PW] - p, G2 = sp[1] - p;
                const float b1 = b1v[u], b2 = b2v[u];
                const float B1 = G1 + b1, B2 = G2 + b2;
                const float nb = sqrtf(B1 * B1 + B2 * B2);
                float w1 = 0.0f, w2 = 0.0f;
                if (nb > 0.0f && nb > kp.zero_tol) { w1 = B1 / nb; w2 = B2 / nb; }
                const float bn1 = b1 + G1 - w1, bn2 = b2 + G2 - w2;
                sd1[e] = bn1 - w1;
                sd2[e] = bn2 - w2;
                if (ci >= 1 && cj >= 1 && i0 - 1 + ci < M && j0 - 1 + cj < N) {
                    const size_t o = (size_t)(i0 - 1 + ci) * N + (j0 - 1 + cj);
                    Wnew[o] = w1; Wnew[MN + o] = w2;
                    if (!sweep) { Bnew[o] = bn1; Bnew[MN + o] = bn2; }
                }
            }
        }
    }
    if (sweep) return;   // a fixed-point sweep writes w only
    __syncthreads();
    double sdiff = 0.0, sold = 0.0;
#pragma unroll
    for (int u = 0; u < C::NO; ++u) {
        const int e = tid + u * T;
        const int i = e / TW, j = e - i * TW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi < M && gj < N) {
            const int c = (i + 1) * CW + (j + 1);
            float dvv;
            if constexpr (BC == 0) {
                dvv = (sd1[c] - sd1[c - CW]) + (sd2[c] - sd2[c - 1]);
            } else {   // negative adjoint of the Neumann forward difference
                const float e1 = gi < M - 1 ? sd1[c] : 0.0f, e1u = gi > 0 ? sd1[c - CW] : 0.0f;
                const float e2 = gj < N - 1 ? sd2[c] : 0.0f, e2l = gj > 0 ? sd2[c - 1] : 0.0f;
                dvv = (e1 - e1u) + (e2 - e2l);
            }
            const size_t o = (size_t)gi * N + gj;
            D[o] = kp.mu * dvv;
            const float pn = sphi[(i + 1) * PW + (j + 1)];
            const float po = pold[u];
            const double df = (double)pn - (double)po;
            sdiff += df * df;
            sold += (double)po * po;
        }
    }
    double v[2] = {sdiff, sold};
    const int nb = gridDim.x * gridDim.y;
    store_partials<2>(v, part + (size_t)z * 2 * nb, nb, blockIdx.y * gridDim.x + blockIdx.x, red);
}

// End of an outer iteration: r_k = ||phi^{k+1} - phi^k||_F / (||phi^k||_F + 1e-6).
__global__ __launch_bounds__(1024) void k_fin_outer(const double* __restrict__ part, int nb,
                                                   double* __restrict__ rhist, DevScal* sc) {
    __shared__ double red[2 * 16];
    const int z = blockIdx.x;
    DevScal& S = sc[z];
    if (!S.active) return;
    fin_outer_body(part, nb, rhist, S, z, red);
}

// ---------------------------------------------------------------------------
// SR energy (eqs 7-10) of phi, partial sums in double, last workgroup totals.
// ---------------------------------------------------------------------------
template <int TH, int BC>
__global__ __launch_bounds__(kTileThreads) void k_energy(KParams kp, int M, int N,
                                                         const float* __restrict__ phi,
                                                         const float* __restrict__ g,
                                                         double* __restrict__ part, DevScal* sc) {
    constexpr int TW = kTileW;
    const int z = blockIdx.z;
    DevScal& S = sc[z];
    const size_t MN = (size_t)M * N;
    phi += z * MN; g += z * MN;
    extern __shared__ float lds[];
    __shared__ double red[3 * 16];
    const int R = kp.R;
    const int eh = TH + 2 * R, ew = TW + 2 * R;
    float* su1 = lds;
    float* su2 = su1 + eh * ew;
    float* sh1 = su2 + eh * ew;
    float* sh2 = sh1 + eh * TW;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;
    for (int e = threadIdx.x; e < eh * ew; e += blockDim.x) {
        const int ei = e / ew, ej = e - ei * ew;
        const int gi = bidx<BC>(i0 - R + ei, M), gj = bidx<BC>(j0 - R + ej, N);
        const float p = phi[(size_t)gi * N + gj];
        const float G1 = phi[(size_t)bidx<BC>(gi + 1, M) * N + gj] - p;
        const float G2 = phi[(size_t)gi * N + bidx<BC>(gj + 1, N)] - p;
        const float h = band_h(p, kp);
        su1[e] = G1 * h;
        su2[e] = G2 * h;
    }
    __syncthreads();
    window_rows(su1, su2, sh1, sh2, eh, ew, TW, kp);
    __syncthreads();
    double eg = 0.0, ea = 0.0, er = 0.0;
    for (int e = threadIdx.x; e < TH * TW; e += blockDim.x) {
        const int i = e / TW, j = e - i * TW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= M || gj >= N) continue;
        float v1, v2;
        window_col(sh1, sh2, i, j, TW, kp, v1, v2);
        const int c = (i + R) * ew + (j + R);
        const float u1 = su1[c], u2 = su2[c];
        const size_t o = (size_t)gi * N + gj;
        const float p = phi[o];
        const float G1 = phi[(size_t)bidx<BC>(gi + 1, M) * N + gj] - p;
        const float G2 = phi[(size_t)gi * N + bidx<BC>(gj + 1, N)] - p;
        float H_, dl;
        heav_dirac(p, kp.eps, kp.inv_eps, H_, dl);
        const float gg = g[o];
        eg += (double)(gg * sqrtf(G1 * G1 + G2 * G2) * dl);
        ea += (double)(gg * (1.0f - H_));
        er += (double)(u1 * v1 + u2 * v2);
    }
    double v[3] = {eg, ea, er};
    const int nb = gridDim.x * gridDim.y;
    store_partials<3>(v, part + (size_t)z * 3 * nb, nb, blockIdx.y * gridDim.x + blockIdx.x, red);
}

__global__ __launch_bounds__(1024) void k_fin_energy(const double* __restrict__ part, int nb, KParams kp,
                                                    DevScal* sc) {
    __shared__ double red[3 * 16];
    const int z = blockIdx.x;
    DevScal& S = sc[z];
    double v[3];
    sum_partials<3>(part + (size_t)z * 3 * nb, nb, v, red);
    if (threadIdx.x == 0) {
        S.energy[0] = (double)kp.gamma * v[0];
        S.energy[1] = (double)kp.alpha * v[1];
        S.energy[2] = -(double)kp.beta * v[2];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
constexpr int kTH = 32;   // tile height of the stencil kernels

inline dim3 tile_grid(int M, int N, int TH, int nz) {
    return dim3((N + kTileW - 1) / kTileW, (M + TH - 1) / TH, nz);
}
inline size_t lds_energy(int TH, int R) {
    const int eh = TH + 2 * R, ew = kTileW + 2 * R;
    return sizeof(float) * (2 * eh * ew + 2 * eh * kTileW);
}
}  // namespace

int tile_blocks(int M, int N) { return ((N + kTileW - 1) / kTileW) * ((M + 7) / 8); }

// Row-tile count per workgroup of the row passes: enough rows for at least
// one full wave (each 8-row tile is 4 transforms of NT threads).
static int fft_nt_rt(int L, bool col) {
    switch (L) {
        case 8: return col ? FftShape<8, ColE<8>::v>::NT : FftShape<8>::NT;
        case 16: return col ? FftShape<16, ColE<16>::v>::NT : FftShape<16>::NT;
        case 32: return col ? FftShape<32, ColE<32>::v>::NT : FftShape<32>::NT;
        case 64: return col ? FftShape<64, ColE<64>::v>::NT : FftShape<64>::NT;
        case 128: return col ? FftShape<128, ColE<128>::v>::NT : FftShape<128>::NT;
        case 256: return col ? FftShape<256, ColE<256>::v>::NT : FftShape<256>::NT;
        case 512: return col ? FftShape<512, ColE<512>::v>::NT : FftShape<512>::NT;
        case 1024: return col ? FftShape<1024, ColE<1024>::v>::NT : FftShape<1024>::NT;
        case 2048: return col ? FftShape<2048, ColE<2048>::v>::NT : FftShape<2048>::NT;
        default: return col ? FftShape<4096, ColE<4096>::v>::NT : FftShape<4096>::NT;
    }
}
// log2 of the rows per workgroup of the row passes: whole 8-row tiles
// (several for short rows, so a workgroup holds at least one wave), split
// into 4- or 2-row pieces (down to 2^min_lr rows) while the grid would have
// fewer than min_wg workgroups and a piece still holds a full wave; the
// pieces of a tile share an XCD (row_piece0).  Measured (per launch, 1024^2 /
// 4096^2): forward pass 8 rows 6.5 / 43.5 us, split to 1024 workgroups
// 6.2 / 39.5; inverse pass (phi_s prefetched) 4 rows 5.3 / 44.0 us, 2 rows
// at 1024^2 5.8, 8 rows at 4096^2 52.1.
#ifndef SR_ROW_FWD_MIN_WG
#define SR_ROW_FWD_MIN_WG 1024
#endif
#ifndef SR_ROW_INV_MIN_WG
#define SR_ROW_INV_MIN_WG 1024
#endif
int fft_row_split(int M, int N, int nz, int min_wg, int min_lr) {
    const int NT = fft_nt_rt(N, false);
    int lr = 3;
    while ((1 << lr) * 2 * NT < 64 * 4 && (2 << lr) <= M) ++lr;   // 4 * RT transforms of NT threads >= 64
    while (lr > min_lr && lr > 1 && (M >> lr) * nz < min_wg && (1 << (lr - 2)) * NT >= 64) --lr;
    return lr;
}
// Columns per workgroup of the column pass: one column when its transform
// fills at least a wave (the two columns of a 128-byte run then go to
// workgroups on one XCD), else as many as make a wave.  Measured per launch
// (1024^2 / 4096^2): one column 7.6 / 46.4 us, two 8.0 / 50.5 us (more
// workgroups per CU overlap one another's loads with their transforms).
int fft_col_group(int M, int N, int nz) {
    (void)nz;
    const int NT = fft_nt_rt(M, true);
    if (NT >= 64) return 1;
    int G = 2;
    while (G * NT < 64 && G * 2 <= N / 2) G <<= 1;
    if (G > N / 2) G = N / 2;
    return G;
}


// Per-launch timing of the iteration kernels: while events are set on the
// calling host thread, their launches go through hipExtLaunchKernel with
// those events, which the runtime records at the kernel's own start and end
// (never used under stream capture).
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}
void launch_kernel_ev(const void* fn, dim3 grid, dim3 block, void** args, size_t lds, hipStream_t st) {
    if (t_ev_start)
        (void)hipExtLaunchKernel(fn, grid, block, args, lds, st, t_ev_start, t_ev_stop, 0);
    else
        (void)hipLaunchKernel(fn, grid, block, args, lds, st);
}

// Elements per thread of the row (col = false) or column transforms of length L.
static int fft_e(int L, bool col) {
    switch (L) {
        case 8: return col ? ColE<8>::v : RowE<8>::v;
        case 16: return col ? ColE<16>::v : RowE<16>::v;
        case 32: return col ? ColE<32>::v : RowE<32>::v;
        case 64: return col ? ColE<64>::v : RowE<64>::v;
        case 128: return col ? ColE<128>::v : RowE<128>::v;
        case 256: return col ? ColE<256>::v : RowE<256>::v;
        case 512: return col ? ColE<512>::v : RowE<512>::v;
        case 1024: return col ? ColE<1024>::v : RowE<1024>::v;
        case 2048: return col ? ColE<2048>::v : RowE<2048>::v;
        default: return col ? ColE<4096>::v : RowE<4096>::v;
    }
}
int fft_stage_table_len(int L, bool col) { return stage_tab_len(L, fft_e(L, col)); }
int fft_elems(int L, bool col) { return fft_e(L, col); }
void fft_stage_table(int L, bool col, float2* out) {
    const int E = fft_e(L, col);
    const double two_pi = 6.283185307179586476925286766559;
    size_t o = 0;
    for (int Ns = 1; Ns < L;) {
        const int R = fft_radix(L, E, Ns);
        if (Ns > 1)
            for (int k = 0; k < Ns; ++k)
                for (int r = 0; r < R; ++r) {
                    const double a = two_pi * (double)(r * k) / (double)(R * Ns);
                    out[o++] = make_float2((float)std::cos(a), (float)-std::sin(a));
                }
        Ns *= R;
    }
}

#define SR_FFT_DISPATCH(FN, LEN, ...)                                   \
    switch (LEN) {                                                      \
        case 8: FN<8>(__VA_ARGS__); break;                              \
        case 16: FN<16>(__VA_ARGS__); break;                            \
        case 32: FN<32>(__VA_ARGS__); break;                            \
        case 64: FN<64>(__VA_ARGS__); break;                            \
        case 128: FN<128>(__VA_ARGS__); break;                          \
        case 256: FN<256>(__VA_ARGS__); break;                          \
        case 512: FN<512>(__VA_ARGS__); break;                          \
        case 1024: FN<1024>(__VA_ARGS__); break;                        \
        case 2048: FN<2048>(__VA_ARGS__); break;                        \
        case 4096: FN<4096>(__VA_ARGS__); break;                        \
        default: break;                                                 \
    }

template <int N>
static void launch_row_fwd_t(const float* src, float2* spec, const float2* stN, int M, int nz, DevScal* sc,
                             hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int lr = fft_row_split(M, N, nz, SR_ROW_FWD_MIN_WG, 1);
    const size_t lds = sizeof(float2) * ((1 << lr) / 2) * LdsLen<N>::v;
    auto k = lr == 3 ? k_row_fwd<N, 3> : lr == 2 ? k_row_fwd<N, 2> : lr == 1 ? k_row_fwd<N, 1> : k_row_fwd<N, 0>;
    launch_iter(k, dim3(M >> lr, 1, nz), dim3(((1 << lr) / 2) * NT), lds, st, src, spec, stN, M, lr, sc);
}
template <int M>
static void launch_col_t(float2* spec, const float2* twM, const float2* twN, const float2* stM, int N, float taumu,
                         float inv_mn, int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<M, ColE<M>::v>::NT;
    const int G = fft_col_group(M, N, nz);
    const size_t lds = sizeof(float2) * G * LdsLen<M>::v;
    int lrun = 0;
    while ((1 << lrun) < kSpecTile * G) ++lrun;
    auto k = G == 2 ? k_col_solve<M, 2> : G == 1 ? k_col_solve<M, 1> : k_col_solve<M, 0>;
    launch_iter(k, dim3(N / 2 / G, 1, nz), dim3(NT * G), lds, st, spec, twM, twN, stM, N, G, lrun, taumu, inv_mn, sc);
}
template <int N>
static void launch_row_inv_t(const float2* spec, const float* phi_in, float* phi_out, const float2* stN, int M,
                             float tol, double* part, int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int lr = fft_row_split(M, N, nz, SR_ROW_INV_MIN_WG, 2);
    const size_t lds = sizeof(float2) * ((1 << lr) / 2) * LdsLen<N>::v;
    const int nb = M >> lr;
    auto k = lr == 3 ? k_row_inv<N, 3> : lr == 2 ? k_row_inv<N, 2> : k_row_inv<N, 0>;
    launch_iter(k, dim3(nb, 1, nz), dim3(((1 << lr) / 2) * NT), lds, st, spec, phi_in, phi_out, stN, M, lr, tol, part,
                sc);
    if (tol > 0.0f) launch_fin_inner(part, nb, tol, nz, sc, st);
}

template <int L>
static void set_fft_attrs() {
    const int bytes = 160 * 1024 - 1024;
    const void* fns[] = {(const void*)k_row_fwd<L, 0>, (const void*)k_row_fwd<L, 1>, (const void*)k_row_fwd<L, 2>,
                         (const void*)k_row_fwd<L, 3>,
                         (const void*)k_col_solve<L, 0>, (const void*)k_col_solve<L, 1>, (const void*)k_col_solve<L, 2>,
                         (const void*)k_row_inv<L, 0>, (const void*)k_row_inv<L, 2>, (const void*)k_row_inv<L, 3>};
    for (const void* f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_fin_inner(const double* part, int nb, float tol, int nz, DevScal* sc, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_inner, dim3(nz), dim3(1024), 0, st, part, nb, tol, sc);
}

void launch_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                       float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st) {
    if (geo.bc == 1) {   // the DCT-II solve of the mirrored Laplacian (sr_dct.hip)
        launch_dct_solve_pass(pass, geo, rhs, phi_in, phi_out, spec, tol_inner, part, nz, sc, st);
        return;
    }
    const int M = geo.M, N = geo.N;
    if (pass == 0) {
        SR_FFT_DISPATCH(launch_row_fwd_t, N, rhs, spec, geo.stN, M, nz, sc, st);
    } else if (pass == 1) {
        const float inv_mn = 1.0f / ((float)M * (float)N);
        SR_FFT_DISPATCH(launch_col_t, M, spec, geo.twM, geo.twN, geo.stM, N, geo.taumu, inv_mn, nz, sc, st);
    } else {
        SR_FFT_DISPATCH(launch_row_inv_t, N, spec, phi_in, phi_out, geo.stN, M, tol_inner, part, nz, sc, st);
    }
}

void launch_solve(const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out, float2* spec,
                  float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st) {
    for (int pass = 0; pass < 3; ++pass)
        launch_solve_pass(pass, geo, rhs, phi_in, phi_out, spec, tol_inner, part, nz, sc, st);
}

// Tile height of the right-hand-side kernel: the context's (from the
// autotuner or SR_TILE_TH), else 16 rows.
static int tile_height(const Geometry& geo, int nz) {
    if (geo.tile_th == 8 || geo.tile_th == 16 || geo.tile_th == 32) return geo.tile_th;
    (void)nz;
    return 16;
}

template <int TH, int R>
static void launch_rhs_t(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                         const float* D, float* out, int nz, DevScal* sc, hipStream_t st, const FinFold* fold) {
    launch_iter(geo.bc ? k_rhs<TH, R, 1> : k_rhs<TH, R, 0>, tile_grid(geo.M, geo.N, TH, nz), dim3(kRhsThreads),
                sizeof(float) * RhsTile<TH, R>::lds_floats, st, kp, geo.M, geo.N, phi_s, W, g, D, out,
                fold ? fold->part : nullptr, fold ? fold->nb : 0, fold ? fold->rhist : nullptr, sc);
}
template <int TH, int R, int TT>
static void launch_wstep_t(const Geometry& geo, const KParams& kp, const float* phin, const float* Pk, const float* Wold,
                           const float* Bold, const float* g, float* Wnew, float* Bnew, float* D, double* part,
                           double* rhist, int sweep, int nz, DevScal* sc, hipStream_t st) {
    launch_iter(geo.bc ? k_wstep<TH, R, TT, 1> : k_wstep<TH, R, TT, 0>, tile_grid(geo.M, geo.N, TH, nz), dim3(TT),
                sizeof(float) * WTile<TH, R, TT>::lds_floats, st, kp, geo.M, geo.N, phin, Pk, Wold, Bold, g, Wnew,
                Bnew, D, part, rhist, sweep, sc);
}
// The two w-step tile shapes in use: 64 x 32 on 512 threads up to 4 Mpx per
// launch, 64 x 16 on 256 threads above (measured 16.0 / 171 us against
// 17.8 / 160 us at 1024^2 / 4096^2).
template <int TH, int R>
static void launch_wstep_small(const Geometry& geo, const KParams& kp, const float* phin, const float* Pk,
                               const float* Wold, const float* Bold, const float* g, float* Wnew, float* Bnew,
                               float* D, double* part, double* rhist, int sweep, int nz, DevScal* sc,
                               hipStream_t st) {
    launch_wstep_t<TH, R, 512>(geo, kp, phin, Pk, Wold, Bold, g, Wnew, Bnew, D, part, rhist, sweep, nz, sc, st);
}
template <int TH, int R>
static void launch_wstep_large(const Geometry& geo, const KParams& kp, const float* phin, const float* Pk,
                               const float* Wold, const float* Bold, const float* g, float* Wnew, float* Bnew,
                               float* D, double* part, double* rhist, int sweep, int nz, DevScal* sc,
                               hipStream_t st) {
    launch_wstep_t<TH, R, 256>(geo, kp, phin, Pk, Wold, Bold, g, Wnew, Bnew, D, part, rhist, sweep, nz, sc, st);
}

#define SR_R_DISPATCH(FN, TH, R, ...)                                                          \
    switch (R) {                                                                               \
        case 0: FN<TH, 0>(__VA_ARGS__); break;                                                 \
        case 1: FN<TH, 1>(__VA_ARGS__); break;                                                 \
        case 2: FN<TH, 2>(__VA_ARGS__); break;                                                 \
        case 3: FN<TH, 3>(__VA_ARGS__); break;                                                 \
        case 4: FN<TH, 4>(__VA_ARGS__); break;                                                 \
        case 5: FN<TH, 5>(__VA_ARGS__); break;                                                 \
        case 6: FN<TH, 6>(__VA_ARGS__); break;                                                 \
        case 7: FN<TH, 7>(__VA_ARGS__); break;                                                 \
        case 8: FN<TH, 8>(__VA_ARGS__); break;                                                 \
        default: break;                                                                        \
    }

void launch_rhs(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                const float* D, float* out, int nz, DevScal* sc, hipStream_t st, const FinFold* fold) {
    const int TH = tile_height(geo, nz);
    if (TH == 32) {
        SR_R_DISPATCH(launch_rhs_t, 32, kp.R, geo, kp, phi_s, W, g, D, out, nz, sc, st, fold);
    } else if (TH == 16) {
        SR_R_DISPATCH(launch_rhs_t, 16, kp.R, geo, kp, phi_s, W, g, D, out, nz, sc, st, fold);
    } else {
        SR_R_DISPATCH(launch_rhs_t, 8, kp.R, geo, kp, phi_s, W, g, D, out, nz, sc, st, fold);
    }
}

static bool wstep_small(const Geometry& geo, int nz) { return (size_t)geo.M * geo.N * nz <= ((size_t)1 << 22); }
int wstep_blocks(const Geometry& geo, int nz) {
    const int TH = wstep_small(geo, nz) ? 32 : 16;
    return ((geo.N + kTileW - 1) / kTileW) * ((geo.M + TH - 1) / TH);
}

void launch_wstep(const Geometry& geo, const KParams& kp, const float* phin, const float* Pk, const float* Wold,
                  const float* Bold, const float* g, float* Wnew, float* Bnew, float* D, double* part,
                  double* rhist, int nz, DevScal* sc, hipStream_t st, bool finalize, bool sweep) {
    // Fixed shapes, whatever tile height the autotuner picks for the right-hand
    // side (on 256 threads, 8 and 32 rows measured 18.8 / 180 and 19.5 / 194 us).
    const bool small = wstep_small(geo, nz);
    if (small) {
        SR_R_DISPATCH(launch_wstep_small, 32, kp.R, geo, kp, phin, Pk, Wold, Bold, g, Wnew, Bnew, D, part, rhist,
                      (int)sweep, nz, sc, st);
    } else {
        SR_R_DISPATCH(launch_wstep_large, 16, kp.R, geo, kp, phin, Pk, Wold, Bold, g, Wnew, Bnew, D, part, rhist,
                      (int)sweep, nz, sc, st);
    }
    if (!finalize || sweep) return;
    hipLaunchKernelGGL(k_fin_outer, dim3(nz), dim3(1024), 0, st, part, wstep_blocks(geo, nz), rhist, sc);
}

template <int TH, int R>
static void set_tile_attrs_one() {
    const int bytes = 160 * 1024 - 1024;
    (void)hipFuncSetAttribute((const void*)k_rhs<TH, R, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_rhs<TH, R, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if constexpr (TH == 32) {
        (void)hipFuncSetAttribute((const void*)k_wstep<32, R, 512, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  bytes);
        (void)hipFuncSetAttribute((const void*)k_wstep<32, R, 512, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  bytes);
    }
    if constexpr (TH == 16) {
        (void)hipFuncSetAttribute((const void*)k_wstep<16, R, 256, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  bytes);
        (void)hipFuncSetAttribute((const void*)k_wstep<16, R, 256, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  bytes);
    }
}
template <int TH>
static void set_tile_attrs() {
    set_tile_attrs_one<TH, 0>(); set_tile_attrs_one<TH, 1>(); set_tile_attrs_one<TH, 2>();
    set_tile_attrs_one<TH, 3>(); set_tile_attrs_one<TH, 4>(); set_tile_attrs_one<TH, 5>();
    set_tile_attrs_one<TH, 6>(); set_tile_attrs_one<TH, 7>(); set_tile_attrs_one<TH, 8>();
}

void launch_energy(const Geometry& geo, const KParams& kp, const float* phi, const float* g, double* part,
                   int nz, DevScal* sc, hipStream_t st) {
    auto kern = geo.bc ? k_energy<kTH, 1> : k_energy<kTH, 0>;
    hipLaunchKernelGGL(kern, tile_grid(geo.M, geo.N, kTH, nz), dim3(kTileThreads), lds_energy(kTH, kp.R), st, kp,
                       geo.M, geo.N, phi, g, part, sc);
    const int nb = ((geo.N + kTileW - 1) / kTileW) * ((geo.M + kTH - 1) / kTH);
    hipLaunchKernelGGL(k_fin_energy, dim3(nz), dim3(1024), 0, st, part, nb, kp, sc);
}

void launch_repulsion(const Geometry& geo, const KParams& kp, const float* phi, const float* W, float* V,
                      hipStream_t st) {
    auto kern = geo.bc ? k_repulsion<kTH, 1> : k_repulsion<kTH, 0>;
    hipLaunchKernelGGL(kern, tile_grid(geo.M, geo.N, kTH, 1), dim3(kTileThreads), lds_energy(kTH, kp.R), st, kp,
                       geo.M, geo.N, phi, W, V);
}

void launch_edge(const Geometry& geo, const float* f, float* tmp, float* fs, float* g, const float* taps, int r,
                 float rho, int s_exp, DevScal* sc, hipStream_t st, int nz) {
    GaussTaps gt;
    gt.r = r;
    for (int t = 0; t <= 2 * r; ++t) gt.k[t] = taps[t];
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M, nz);
    auto rows = geo.bc ? k_blur_rows<1> : k_blur_rows<0>;
    auto cols = geo.bc ? k_blur_cols<1> : k_blur_cols<0>;
    auto edge = geo.bc ? k_edge<1> : k_edge<0>;
    hipLaunchKernelGGL(rows, grd, blk, 0, st, f, tmp, geo.M, geo.N, gt, sc);
    hipLaunchKernelGGL(cols, grd, blk, 0, st, tmp, fs, geo.M, geo.N, gt);
    hipLaunchKernelGGL(edge, grd, blk, 0, st, fs, g, geo.M, geo.N, rho, s_exp);
}

void launch_init(const Geometry& geo, const float* phi0, float* P0, float* W, float* B, float* D, float mu,
                 int w0_mode, DevScal* sc, hipStream_t st, int nz) {
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M, nz);
    auto kern = geo.bc ? k_init<1> : k_init<0>;
    hipLaunchKernelGGL(kern, grd, blk, 0, st, phi0, P0, W, B, D, geo.M, geo.N, mu, w0_mode, sc);
}

void launch_set_D(const Geometry& geo, const float* W, const float* B, float* D, float mu, hipStream_t st) {
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M);
    auto kern = geo.bc ? k_set_D<1> : k_set_D<0>;
    hipLaunchKernelGGL(kern, grd, blk, 0, st, W, B, D, geo.M, geo.N, mu);
}

void launch_reset_scal(DevScal* sc, int n, int active, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_scal, dim3((n + 63) / 64), dim3(64), 0, st, sc, n, active);
}

void launch_set_k(DevScal* sc, long long k, hipStream_t st) {
    hipLaunchKernelGGL(k_set_k, dim3(1), dim3(64), 0, st, sc, k);
}


}  // namespace sr

namespace sr {
// Allow the stencil kernels more than the default 64 KiB of dynamic LDS
// (gfx950 has 160 KiB per CU); done once per process.
void configure_kernels() {
    static bool done = false;
    if (done) return;
    const int bytes = 160 * 1024 - 1024;
    set_tile_attrs<8>();
    set_tile_attrs<16>();
    set_tile_attrs<32>();
    (void)hipFuncSetAttribute((const void*)k_energy<kTH, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_energy<kTH, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_repulsion<kTH, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_repulsion<kTH, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    set_fft_attrs<8>(); set_fft_attrs<16>(); set_fft_attrs<32>(); set_fft_attrs<64>(); set_fft_attrs<128>();
    set_fft_attrs<256>(); set_fft_attrs<512>(); set_fft_attrs<1024>(); set_fft_attrs<2048>(); set_fft_attrs<4096>();
    configure_fused();
    configure_dct();
    done = true;
}
}  // namespace sr
