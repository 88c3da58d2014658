// HIP kernels of the SR Split Bregman solver for gfx950 (MI355X).
//
// One outer iteration k of Algorithm 1 is, per inner step s = 0..S-1,
//   k_rhs       : r = tau (N(phi_s) + mu div(b - w) + mu Lap phi_s)      (eq 37,
//                 increment form) with the repulsion window sum v fused in,
//   k_row_fwd   : real-to-complex row FFTs of r (two rows per complex FFT),
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
#include "sr_device.hpp"
#include "sr_kernels.hpp"

namespace sr {

// ---------------------------------------------------------------------------
// setup: Gaussian smoothing and the edge map (eq 1)
// ---------------------------------------------------------------------------
struct GaussTaps { float k[2 * kMaxGaussR + 1]; int r; };

__global__ __launch_bounds__(256) void k_blur_rows(const float* __restrict__ src, float* __restrict__ dst,
                                                   int M, int N, GaussTaps gt, DevScal* sc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const float* row = src + (size_t)i * N;
    float acc = 0.0f;
    for (int t = -gt.r; t <= gt.r; ++t) acc += gt.k[t + gt.r] * row[(j + t) & (N - 1)];
    const float c = row[j];
    if (!isfinite(c)) sc->nonfinite = 1;
    dst[(size_t)i * N + j] = acc;
}

__global__ __launch_bounds__(256) void k_blur_cols(const float* __restrict__ src, float* __restrict__ dst,
                                                   int M, int N, GaussTaps gt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    float acc = 0.0f;
    for (int t = -gt.r; t <= gt.r; ++t) acc += gt.k[t + gt.r] * src[(size_t)((i + t) & (M - 1)) * N + j];
    dst[(size_t)i * N + j] = acc;
}

// g = 1 / (1 + rho |grad fs|^s), central differences.
__global__ __launch_bounds__(256) void k_edge(const float* __restrict__ fs, float* __restrict__ g,
                                              int M, int N, float rho, int s_exp) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const float gx = 0.5f * (fs[(size_t)((i + 1) & (M - 1)) * N + j] - fs[(size_t)((i - 1) & (M - 1)) * N + j]);
    const float gy = 0.5f * (fs[(size_t)i * N + ((j + 1) & (N - 1))] - fs[(size_t)i * N + ((j - 1) & (N - 1))]);
    const float m2 = gx * gx + gy * gy;
    const float m = (s_exp == 2) ? m2 : sqrtf(m2);
    g[(size_t)i * N + j] = 1.0f / (1.0f + rho * m);
}

// State initialisation of Algorithm 1: phi = phi0, w = grad+ phi0 (or 0),
// b = 0, D = mu div-(b - w) = -mu Lap phi0 (or 0).
__global__ __launch_bounds__(256) void k_init(const float* __restrict__ phi0, float* __restrict__ P0,
                                              float* __restrict__ W, float* __restrict__ B,
                                              float* __restrict__ D, int M, int N, float mu, int w0_mode,
                                              DevScal* sc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t MN = (size_t)M * N, o = (size_t)i * N + j;
    const float p = phi0[o];
    if (!isfinite(p)) sc->nonfinite = 1;
    const float pd = phi0[(size_t)((i + 1) & (M - 1)) * N + j];
    const float pr = phi0[(size_t)i * N + ((j + 1) & (N - 1))];
    const float pu = phi0[(size_t)((i - 1) & (M - 1)) * N + j];
    const float pl = phi0[(size_t)i * N + ((j - 1) & (N - 1))];
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

// D = mu div-(b - w) (eq 36) from a given state (checkpoint restore).
__global__ __launch_bounds__(256) void k_set_D(const float* __restrict__ W, const float* __restrict__ B,
                                               float* __restrict__ D, int M, int N, float mu) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= N) return;
    const size_t MN = (size_t)M * N, o = (size_t)i * N + j;
    const size_t ou = (size_t)((i - 1) & (M - 1)) * N + j;
    const size_t ol = (size_t)i * N + ((j - 1) & (N - 1));
    const float e1 = B[o] - W[o], e1u = B[ou] - W[ou];
    const float e2 = B[MN + o] - W[MN + o], e2l = B[MN + ol] - W[MN + ol];
    D[o] = mu * ((e1 - e1u) + (e2 - e2l));
}

__global__ void k_reset_scal(DevScal* sc, int n, int active) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= n) return;
    DevScal& s = sc[z];
    s.counter = 0u; s.inner_done = 0; s.active = active; s.nonfinite = 0;
    s.k = 0; s.inner_steps = 0; s.r_last = -1.0; s.inner_rel = -1.0;
    s.energy[0] = s.energy[1] = s.energy[2] = 0.0;
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
template <int TH>
__global__ __launch_bounds__(kTileThreads) void k_rhs(KParams kp, int M, int N,
                                                      const float* __restrict__ phi_s,
                                                      const float* __restrict__ W,
                                                      const float* __restrict__ g,
                                                      const float* __restrict__ D,
                                                      float* __restrict__ out, DevScal* sc) {
    constexpr int TW = kTileW;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    const size_t MN = (size_t)M * N;
    phi_s += z * MN; W += 2 * z * MN; g += z * MN; D += z * MN; out += z * MN;

    extern __shared__ float lds[];
    const int R = kp.R;
    const int eh = TH + 2 * R, ew = TW + 2 * R;
    float* su1 = lds;
    float* su2 = su1 + eh * ew;
    float* sh1 = su2 + eh * ew;
    float* sh2 = sh1 + eh * TW;
    float* sphi = sh2 + eh * TW;               // (TH+2) x (TW+2)
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;

    for (int e = threadIdx.x; e < eh * ew; e += blockDim.x) {
        const int ei = e / ew, ej = e - ei * ew;
        const int gi = (i0 - R + ei) & (M - 1), gj = (j0 - R + ej) & (N - 1);
        const size_t o = (size_t)gi * N + gj;
        const float p = phi_s[o];
        const float h = band_h(p, kp);
        su1[e] = W[o] * h;
        su2[e] = W[MN + o] * h;
        const int si = ei - R + 1, sj = ej - R + 1;
        if ((unsigned)si < (unsigned)(TH + 2) && (unsigned)sj < (unsigned)(TW + 2)) sphi[si * (TW + 2) + sj] = p;
    }
    // R = 0 still needs the one-pixel halo of phi for the Laplacian
    if (R == 0) {
        for (int e = threadIdx.x; e < (TH + 2) * (TW + 2); e += blockDim.x) {
            const int si = e / (TW + 2), sj = e - si * (TW + 2);
            const int gi = (i0 - 1 + si) & (M - 1), gj = (j0 - 1 + sj) & (N - 1);
            sphi[e] = phi_s[(size_t)gi * N + gj];
        }
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
        const float* sp = sphi + (i + 1) * (TW + 2) + (j + 1);
        const float p = sp[0];
        const float lap = (sp[-(TW + 2)] + sp[TW + 2]) + (sp[-1] + sp[1]) - 4.0f * p;
        const size_t o = (size_t)gi * N + gj;
        const float w1 = W[o], w2 = W[MN + o];
        const float gg = g[o];
        float dl, ddl, h, dh;
        dirac_d(p, kp, dl, ddl);
        band_h_dh(p, kp, h, dh);
        const float wn = sqrtf(w1 * w1 + w2 * w2);
        const float force = -kp.gamma * gg * wn * ddl + kp.alpha * gg * dl
                            + 2.0f * kp.beta * dh * (w1 * v1 + w2 * v2);
        out[o] = kp.tau * (force + D[o] + kp.mu * lap);
    }
}

// ---------------------------------------------------------------------------
// repulsion field alone (component operator): v = K (*) (w h(phi))
// ---------------------------------------------------------------------------
template <int TH>
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
        const int gi = (i0 - R + ei) & (M - 1), gj = (j0 - R + ej) & (N - 1);
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
// Rows 2m and 2m+1 of the real field r are transformed together as one
// complex row z = r_a + i r_b.  The half spectrum of each row (N/2 complex,
// the DC slot carrying (X[0], X[N/2]) as its real and imaginary parts) is
// stored row-major: spec[i][k], k < N/2.
template <int N>
__global__ __launch_bounds__(256) void k_row_fwd(const float* __restrict__ src, float2* __restrict__ spec,
                                                 const float2* __restrict__ twN, int M, int G, DevScal* sc) {
    constexpr int NT = FftShape<N>::NT, E = FftShape<N>::E, H = N / 2;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    src += (size_t)z * M * N;
    spec += (size_t)z * M * H;
    extern __shared__ float2 xs[];
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int m = blockIdx.x * G + g;
    const size_t ra = (size_t)(2 * m) * N, rb = ra + N;
    float2* x = xs + g * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = t + e * NT;
        x[n] = make_float2(src[ra + n], src[rb + n]);
    }
    fft_lds<N, false>(x, twN, t);
    float2* sa = spec + (size_t)(2 * m) * H;
    float2* sb = sa + H;
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int k = t + e * NT;
        const float2 Zk = x[k];
        if (k == 0) {
            const float2 ZH = x[H];
            sa[0] = make_float2(Zk.x, ZH.x);
            sb[0] = make_float2(Zk.y, ZH.y);
        } else {
            const float2 Zm = x[N - k];
            sa[k] = make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
            sb[k] = make_float2(0.5f * (Zk.y + Zm.y), -0.5f * (Zk.x - Zm.x));
        }
    }
}

// G adjacent spectrum columns per workgroup: forward column FFT, division
// by M N (1 + tau mu (4 - 2cos(2 pi l1/M) - 2cos(2 pi l2/N))), inverse FFT.
// Column 0 holds two real-signal spectra (l2 = 0 and l2 = N/2) packed as
// a + i b; they are separated, scaled by their own symbols and re-packed.
template <int M>
__global__ __launch_bounds__(256) void k_col_solve(float2* __restrict__ spec, const float2* __restrict__ twM,
                                                   const float2* __restrict__ twN, int N, int G,
                                                   float taumu, float inv_mn, DevScal* sc) {
    constexpr int NT = FftShape<M>::NT, E = FftShape<M>::E;
    constexpr int LD = M + 1;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    const int H = N / 2;
    spec += (size_t)z * M * H;
    extern __shared__ float2 xs[];
    const int k0 = blockIdx.x * G;
    for (int e = threadIdx.x; e < G * M; e += blockDim.x) {
        const int c = e % G, l = e / G;
        xs[c * LD + l] = spec[(size_t)l * H + k0 + c];
    }
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int col = k0 + g;
    float2* x = xs + g * LD;
    fft_lds<M, false>(x, twM, t);
    float2 vz[E], vm[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = t + e * NT;
        vz[e] = x[l];
        vm[e] = x[(M - l) & (M - 1)];
    }
    __syncthreads();
    const float cn = 2.0f * twN[col].x;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = t + e * NT;
        const float cm = 2.0f * twM[l].x;
        if (col != 0) {
            const float s = inv_mn / (1.0f + taumu * (4.0f - cm - cn));
            x[l] = cscale(vz[e], s);
        } else {
            const float p = inv_mn / (1.0f + taumu * (2.0f - cm));   // l2 = 0
            const float q = inv_mn / (1.0f + taumu * (6.0f - cm));   // l2 = N/2
            const float hp = 0.5f * (p + q), hm = 0.5f * (p - q);
            x[l] = make_float2(hp * vz[e].x + hm * vm[e].x, hp * vz[e].y - hm * vm[e].y);
        }
    }
    fft_lds<M, true>(x, twM, t);
    __syncthreads();
    for (int e = threadIdx.x; e < G * M; e += blockDim.x) {
        const int c = e % G, l = e / G;
        spec[(size_t)l * H + k0 + c] = xs[c * LD + l];
    }
}

// Inverse row FFTs of two rows at once and phi_{s+1} = phi_s + dphi.  With
// tol_inner > 0, also the inner stop rule ||dphi|| / (||phi_s|| + 1e-6) <= tol
// (grid-wide sum, last workgroup decides).  Once the rule has fired, the
// remaining inner steps of the outer iteration copy phi_s through.
template <int N>
__global__ __launch_bounds__(256) void k_row_inv(const float2* __restrict__ spec, const float* __restrict__ phi_in,
                                                 float* __restrict__ phi_out, const float2* __restrict__ twN,
                                                 int M, int G, float tol_inner, double* __restrict__ part,
                                                 DevScal* sc) {
    constexpr int NT = FftShape<N>::NT, E = FftShape<N>::E, H = N / 2;
    const int z = blockIdx.z;
    DevScal& S = sc[z];
    if (!S.active) return;
    const size_t MN = (size_t)M * N;
    spec += (size_t)z * M * H;
    if (phi_in) phi_in += z * MN;
    phi_out += z * MN;
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int m = blockIdx.x * G + g;
    const size_t ra = (size_t)(2 * m) * N, rb = ra + N;
    if (S.inner_done) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int n = t + e * NT;
            phi_out[ra + n] = phi_in ? phi_in[ra + n] : 0.0f;
            phi_out[rb + n] = phi_in ? phi_in[rb + n] : 0.0f;
        }
        return;
    }
    extern __shared__ float2 xs[];
    __shared__ double red[2 * 16];
    float2* x = xs + g * N;
    const float2* sa = spec + (size_t)(2 * m) * H;
    const float2* sb = sa + H;
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        const int k = t + e * NT;
        const float2 Xa = sa[k], Xb = sb[k];
        if (k == 0) {
            x[0] = make_float2(Xa.x, Xb.x);
            x[H] = make_float2(Xa.y, Xb.y);
        } else {
            x[k] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            x[N - k] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
        }
    }
    fft_lds<N, true>(x, twN, t);
    double sd = 0.0, sp = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n = t + e * NT;
        const float2 Z = x[n];
        const float pa = phi_in ? phi_in[ra + n] : 0.0f;
        const float pb = phi_in ? phi_in[rb + n] : 0.0f;
        phi_out[ra + n] = pa + Z.x;
        phi_out[rb + n] = pb + Z.y;
        sd += (double)Z.x * Z.x + (double)Z.y * Z.y;
        sp += (double)pa * pa + (double)pb * pb;
    }
    if (tol_inner > 0.0f) {
        double v[2] = {sd, sp};
        const int nb = gridDim.x;
        if (grid_sum<2>(v, part + (size_t)z * 2 * nb, nb, blockIdx.x, &S.counter, red) && threadIdx.x == 0) {
            const double rel = sqrt(v[0]) / (sqrt(v[1]) + 1e-6);
            S.inner_rel = rel;
            S.inner_steps += 1;
            if (rel <= (double)tol_inner) S.inner_done = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// w step: B (eq 41), shrink (eq 42) + projection (eq 40) in gate form,
// Bregman (eq 23), next D = mu div(b - w), outer residual r_k, phi^k <- phi^{k+1}.
// The tile computes w, b on one extra row above and column left so that the
// backward divergence of its own pixels is local.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(kTileThreads) void k_wstep(KParams kp, int M, int N,
                                                        const float* __restrict__ phin,
                                                        float* __restrict__ P0,
                                                        const float* __restrict__ Wold,
                                                        const float* __restrict__ Bold,
                                                        const float* __restrict__ g,
                                                        float* __restrict__ Wnew, float* __restrict__ Bnew,
                                                        float* __restrict__ D, double* __restrict__ part,
                                                        double* __restrict__ rhist, DevScal* sc) {
    constexpr int TW = kTileW;
    constexpr int CH = TH + 1, CW = TW + 1;
    const int z = blockIdx.z;
    DevScal& S = sc[z];
    if (!S.active) return;
    const size_t MN = (size_t)M * N;
    phin += z * MN; P0 += z * MN; Wold += 2 * z * MN; Bold += 2 * z * MN; g += z * MN;
    Wnew += 2 * z * MN; Bnew += 2 * z * MN; D += z * MN;

    extern __shared__ float lds[];
    __shared__ double red[2 * 16];
    const int R = kp.R;
    const int eh = CH + 2 * R, ew = CW + 2 * R;
    float* su1 = lds;
    float* su2 = su1 + eh * ew;
    float* sh1 = su2 + eh * ew;
    float* sh2 = sh1 + eh * CW;
    float* sphi = sh2 + eh * CW;          // (TH+2) x (TW+2), origin (i0-1, j0-1)
    float* sd1 = su1;                     // (b - w) after the row pass, aliases su
    float* sd2 = su1 + CH * CW;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;

    for (int e = threadIdx.x; e < eh * ew; e += blockDim.x) {
        const int ei = e / ew, ej = e - ei * ew;
        const int gi = (i0 - 1 - R + ei) & (M - 1), gj = (j0 - 1 - R + ej) & (N - 1);
        const size_t o = (size_t)gi * N + gj;
        const float p = phin[o];
        const float h = band_h(p, kp);
        su1[e] = Wold[o] * h;
        su2[e] = Wold[MN + o] * h;
        const int si = ei - R, sj = ej - R;
        if ((unsigned)si < (unsigned)(TH + 2) && (unsigned)sj < (unsigned)(TW + 2)) sphi[si * (TW + 2) + sj] = p;
    }
    if (R == 0) {
        for (int e = threadIdx.x; e < (TH + 2) * (TW + 2); e += blockDim.x) {
            const int si = e / (TW + 2), sj = e - si * (TW + 2);
            const int gi = (i0 - 1 + si) & (M - 1), gj = (j0 - 1 + sj) & (N - 1);
            sphi[e] = phin[(size_t)gi * N + gj];
        }
    }
    __syncthreads();
    window_rows(su1, su2, sh1, sh2, eh, ew, CW, kp);
    __syncthreads();
    for (int e = threadIdx.x; e < CH * CW; e += blockDim.x) {
        const int ci = e / CW, cj = e - ci * CW;
        const int gi = (i0 - 1 + ci) & (M - 1), gj = (j0 - 1 + cj) & (N - 1);
        float v1, v2;
        window_col(sh1, sh2, ci, cj, CW, kp, v1, v2);
        const float* sp = sphi + ci * (TW + 2) + cj;
        const float p = sp[0];
        const float G1 = sp[TW + 2] - p, G2 = sp[1] - p;
        const size_t o = (size_t)gi * N + gj;
        const float b1 = Bold[o], b2 = Bold[MN + o];
        const float h = band_h(p, kp);
        float H_, dl;
        heav_dirac(p, kp.eps, kp.inv_eps, H_, dl);
        const float B1 = G1 + b1 + kp.c_rep * h * v1;
        const float B2 = G2 + b2 + kp.c_rep * h * v2;
        const float thr = kp.c_thr * g[o] * dl;
        const float nb = sqrtf(B1 * B1 + B2 * B2);
        float w1 = 0.0f, w2 = 0.0f;
        if (nb > thr && nb > kp.zero_tol) { w1 = B1 / nb; w2 = B2 / nb; }
        const float bn1 = b1 + G1 - w1, bn2 = b2 + G2 - w2;
        sd1[e] = bn1 - w1;
        sd2[e] = bn2 - w2;
        if (ci >= 1 && cj >= 1 && i0 - 1 + ci < M && j0 - 1 + cj < N) {
            Wnew[o] = w1; Wnew[MN + o] = w2;
            Bnew[o] = bn1; Bnew[MN + o] = bn2;
        }
    }
    __syncthreads();
    double sdiff = 0.0, sold = 0.0;
    for (int e = threadIdx.x; e < TH * TW; e += blockDim.x) {
        const int i = e / TW, j = e - i * TW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= M || gj >= N) continue;
        const int c = (i + 1) * CW + (j + 1);
        const float dv = (sd1[c] - sd1[c - CW]) + (sd2[c] - sd2[c - 1]);
        const size_t o = (size_t)gi * N + gj;
        D[o] = kp.mu * dv;
        const float pn = sphi[(i + 1) * (TW + 2) + (j + 1)];
        const float po = P0[o];
        P0[o] = pn;
        const double df = (double)pn - (double)po;
        sdiff += df * df;
        sold += (double)po * po;
    }
    double v[2] = {sdiff, sold};
    const int nb = gridDim.x * gridDim.y;
    if (grid_sum<2>(v, part + (size_t)z * 2 * nb, nb, blockIdx.y * gridDim.x + blockIdx.x, &S.counter, red) &&
        threadIdx.x == 0) {
        const double r = sqrt(v[0]) / (sqrt(v[1]) + 1e-6);
        S.r_last = r;
        rhist[(size_t)z * kRHist + (S.k % kRHist)] = r;
        S.k += 1;
        S.inner_done = 0;
    }
}

// ---------------------------------------------------------------------------
// SR energy (eqs 7-10) of phi, partial sums in double, last workgroup totals.
// ---------------------------------------------------------------------------
template <int TH>
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
        const int gi = (i0 - R + ei) & (M - 1), gj = (j0 - R + ej) & (N - 1);
        const float p = phi[(size_t)gi * N + gj];
        const float G1 = phi[(size_t)((gi + 1) & (M - 1)) * N + gj] - p;
        const float G2 = phi[(size_t)gi * N + ((gj + 1) & (N - 1))] - p;
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
        const float G1 = phi[(size_t)((gi + 1) & (M - 1)) * N + gj] - p;
        const float G2 = phi[(size_t)gi * N + ((gj + 1) & (N - 1))] - p;
        float H_, dl;
        heav_dirac(p, kp.eps, kp.inv_eps, H_, dl);
        const float gg = g[o];
        eg += (double)(gg * sqrtf(G1 * G1 + G2 * G2) * dl);
        ea += (double)(gg * (1.0f - H_));
        er += (double)(u1 * v1 + u2 * v2);
    }
    double v[3] = {eg, ea, er};
    const int nb = gridDim.x * gridDim.y;
    if (grid_sum<3>(v, part + (size_t)z * 3 * nb, nb, blockIdx.y * gridDim.x + blockIdx.x, &S.counter, red) &&
        threadIdx.x == 0) {
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
inline size_t lds_rhs(int TH, int R) {
    const int eh = TH + 2 * R, ew = kTileW + 2 * R;
    return sizeof(float) * (2 * eh * ew + 2 * eh * kTileW + (TH + 2) * (kTileW + 2));
}
inline size_t lds_wstep(int TH, int R) {
    const int CH = TH + 1, CW = kTileW + 1;
    const int eh = CH + 2 * R, ew = CW + 2 * R;
    size_t su = 2 * eh * ew;
    if (su < (size_t)(2 * CH * CW)) su = 2 * CH * CW;
    return sizeof(float) * (su + 2 * eh * CW + (TH + 2) * (kTileW + 2));
}
inline size_t lds_energy(int TH, int R) {
    const int eh = TH + 2 * R, ew = kTileW + 2 * R;
    return sizeof(float) * (2 * eh * ew + 2 * eh * kTileW);
}
}  // namespace

int tile_blocks(int M, int N) { return ((N + kTileW - 1) / kTileW) * ((M + kTH - 1) / kTH); }

// Transforms per workgroup: as many as fit 256 threads, fewer when that
// would leave less than ~2 workgroups per CU.
int fft_group(int count, int L) {
    const int E = L < 16 ? L : 16;
    const int NT = L / E;
    int G = 256 / NT;
    const int Gmin = NT >= 64 ? 1 : 64 / NT;   // keep at least one full wave
    if (G < 1) G = 1;
    while (G > Gmin && count / G < 512) G >>= 1;
    if (G > count) G = count;
    return G;
}

template <int L> struct Dispatch;

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
static void launch_row_fwd_t(const float* src, float2* spec, const float2* twN, int M, int nz, DevScal* sc,
                             hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int G = fft_group(M / 2, N);
    hipLaunchKernelGGL(k_row_fwd<N>, dim3(M / 2 / G, 1, nz), dim3(NT * G), sizeof(float2) * G * N, st,
                       src, spec, twN, M, G, sc);
}
template <int M>
static void launch_col_t(float2* spec, const float2* twM, const float2* twN, int N, float taumu, float inv_mn,
                         int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<M>::NT;
    const int G = fft_group(N / 2, M);
    hipLaunchKernelGGL(k_col_solve<M>, dim3(N / 2 / G, 1, nz), dim3(NT * G), sizeof(float2) * G * (M + 1), st,
                       spec, twM, twN, N, G, taumu, inv_mn, sc);
}
template <int N>
static void launch_row_inv_t(const float2* spec, const float* phi_in, float* phi_out, const float2* twN, int M,
                             float tol, double* part, int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int G = fft_group(M / 2, N);
    hipLaunchKernelGGL(k_row_inv<N>, dim3(M / 2 / G, 1, nz), dim3(NT * G), sizeof(float2) * G * N, st,
                       spec, phi_in, phi_out, twN, M, G, tol, part, sc);
}

void launch_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                       float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st) {
    const int M = geo.M, N = geo.N;
    if (pass == 0) {
        SR_FFT_DISPATCH(launch_row_fwd_t, N, rhs, spec, geo.twN, M, nz, sc, st);
    } else if (pass == 1) {
        const float inv_mn = 1.0f / ((float)M * (float)N);
        SR_FFT_DISPATCH(launch_col_t, M, spec, geo.twM, geo.twN, N, geo.taumu, inv_mn, nz, sc, st);
    } else {
        SR_FFT_DISPATCH(launch_row_inv_t, N, spec, phi_in, phi_out, geo.twN, M, tol_inner, part, nz, sc, st);
    }
}

void launch_solve(const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out, float2* spec,
                  float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st) {
    for (int pass = 0; pass < 3; ++pass)
        launch_solve_pass(pass, geo, rhs, phi_in, phi_out, spec, tol_inner, part, nz, sc, st);
}

void launch_rhs(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                const float* D, float* out, int nz, DevScal* sc, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs<kTH>, tile_grid(geo.M, geo.N, kTH, nz), dim3(kTileThreads), lds_rhs(kTH, kp.R), st,
                       kp, geo.M, geo.N, phi_s, W, g, D, out, sc);
}

void launch_wstep(const Geometry& geo, const KParams& kp, const float* phin, float* P0, const float* Wold,
                  const float* Bold, const float* g, float* Wnew, float* Bnew, float* D, double* part,
                  double* rhist, int nz, DevScal* sc, hipStream_t st) {
    hipLaunchKernelGGL(k_wstep<kTH>, tile_grid(geo.M, geo.N, kTH, nz), dim3(kTileThreads), lds_wstep(kTH, kp.R),
                       st, kp, geo.M, geo.N, phin, P0, Wold, Bold, g, Wnew, Bnew, D, part, rhist, sc);
}

void launch_energy(const Geometry& geo, const KParams& kp, const float* phi, const float* g, double* part,
                   int nz, DevScal* sc, hipStream_t st) {
    hipLaunchKernelGGL(k_energy<kTH>, tile_grid(geo.M, geo.N, kTH, nz), dim3(kTileThreads), lds_energy(kTH, kp.R),
                       st, kp, geo.M, geo.N, phi, g, part, sc);
}

void launch_repulsion(const Geometry& geo, const KParams& kp, const float* phi, const float* W, float* V,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_repulsion<kTH>, tile_grid(geo.M, geo.N, kTH, 1), dim3(kTileThreads),
                       lds_energy(kTH, kp.R), st, kp, geo.M, geo.N, phi, W, V);
}

void launch_edge(const Geometry& geo, const float* f, float* tmp, float* fs, float* g, const float* taps, int r,
                 float rho, int s_exp, DevScal* sc, hipStream_t st) {
    GaussTaps gt;
    gt.r = r;
    for (int t = 0; t <= 2 * r; ++t) gt.k[t] = taps[t];
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M);
    hipLaunchKernelGGL(k_blur_rows, grd, blk, 0, st, f, tmp, geo.M, geo.N, gt, sc);
    hipLaunchKernelGGL(k_blur_cols, grd, blk, 0, st, tmp, fs, geo.M, geo.N, gt);
    hipLaunchKernelGGL(k_edge, grd, blk, 0, st, fs, g, geo.M, geo.N, rho, s_exp);
}

void launch_init(const Geometry& geo, const float* phi0, float* P0, float* W, float* B, float* D, float mu,
                 int w0_mode, DevScal* sc, hipStream_t st) {
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M);
    hipLaunchKernelGGL(k_init, grd, blk, 0, st, phi0, P0, W, B, D, geo.M, geo.N, mu, w0_mode, sc);
}

void launch_set_D(const Geometry& geo, const float* W, const float* B, float* D, float mu, hipStream_t st) {
    const dim3 blk(256), grd((geo.N + 255) / 256, geo.M);
    hipLaunchKernelGGL(k_set_D, grd, blk, 0, st, W, B, D, geo.M, geo.N, mu);
}

void launch_reset_scal(DevScal* sc, int n, int active, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_scal, dim3((n + 63) / 64), dim3(64), 0, st, sc, n, active);
}

void launch_set_k(DevScal* sc, long long k, hipStream_t st) {
    hipLaunchKernelGGL(k_set_k, dim3(1), dim3(64), 0, st, sc, k);
}

size_t lds_max_needed(int R) {
    size_t a = lds_rhs(kTH, R), b = lds_wstep(kTH, R), c = lds_energy(kTH, R);
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

}  // namespace sr

namespace sr {
// Allow the stencil kernels more than the default 64 KiB of dynamic LDS
// (gfx950 has 160 KiB per CU); done once per process.
void configure_kernels() {
    static bool done = false;
    if (done) return;
    const int bytes = 160 * 1024 - 1024;
    (void)hipFuncSetAttribute((const void*)k_rhs<kTH>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_wstep<kTH>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_energy<kTH>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_repulsion<kTH>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    done = true;
}
}  // namespace sr
