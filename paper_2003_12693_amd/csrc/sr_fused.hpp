// The right-hand side of eq (37) fused into the forward row transform of its
// solve: the kernel template k_rhs_fwd and its launch templates.  The
// instances are compiled in three translation units by row length
// (sr_fused_small.hip: 64, 128, 256; sr_fused_512.hip; sr_fused_1024.hip);
// sr_fused.hip chooses the strip height and dispatches.
#pragma once

#include <hip/hip_runtime.h>

#include "sr_device.hpp"
#include "sr_kernels.hpp"
#include "sr_pass.hpp"

namespace sr {

// ---------------------------------------------------------------------------
// Inner right-hand side of eq (37) fused into the forward row FFT of its
// solve (eqs 31-33): a workgroup owns RW = 2^LR whole rows and computes
//   F = tau ( -gamma g |w| delta'(phi) + alpha g delta(phi)
//             + 2 beta h'(phi) w . v + D + mu Lap phi )       (increment form)
// on them, then transforms them (RW / 2 complex FFTs of two rows each) and
// stores the half spectra, so the right-hand side never goes to memory.
// Each thread owns whole columns of the strip: it loads phi on the RW rows
// plus a halo of max(R, 1) rows above and below, forms u = w h(phi) on the
// window's rows and sums them vertically in registers (the column factor of
// the separable window K_pq = a_p a_q); the vertical sums and phi go through
// LDS once for the horizontal factor and the Laplacian's left / right
// neighbours (a whole row is in the workgroup, so the column halo is the
// row itself, periodic or mirrored).  w and g are only read where the pixel
// lies in the band |phi| <= l + eps: outside it h, h', delta and delta'
// vanish, so u and the force are exactly zero there.  With Neumann
// boundaries (BC = 1) the halo indices mirror and the rows are transformed
// by the DCT-II (through the reordered FFT, as in sr_dct.hip).
// ---------------------------------------------------------------------------
template <int N, int LR, int R>
struct RhsFwdShape {
    static constexpr int RW = 1 << LR, NTR = RW / 2;
    static constexpr int E = FftShape<N>::E, NT = FftShape<N>::NT, T = NTR * NT;
    static constexpr int CPT = N / T;                     // columns per thread
    static constexpr int RH = R > 0 ? R : 1;              // halo rows of phi
    static constexpr int NR = RW + 2 * RH;                // rows of phi a column reads
    static constexpr int NU = RW + 2 * R;                 // rows of u a column sums
    static constexpr int LX = LdsLen<N>::v;
    static constexpr size_t lds_win = sizeof(float) * 3 * RW * N;
    static constexpr size_t lds_fft = sizeof(float2) * NTR * LX;
    static constexpr size_t lds_bytes = lds_win > lds_fft ? lds_win : lds_fft;
    static_assert(CPT >= 1 && CPT * T == N, "a thread owns whole columns");
    static_assert(E <= 4, "stage twiddles preloaded into registers");
};

template <int N, int LR, int R, int BC>
__global__ __launch_bounds__((RhsFwdShape<N, LR, R>::T)) void k_rhs_fwd(KParams kp, int M,
                                                                     const float* __restrict__ phi_s,
                                                                     const float* __restrict__ W,
                                                                     const float* __restrict__ g,
                                                                     const float* __restrict__ D,
                                                                     float2* __restrict__ spec,
                                                                     const float2* __restrict__ stN,
                                                                     const float2* __restrict__ dtN,
                                                                     const double* __restrict__ fin_part, int fin_nb,
                                                                     double* __restrict__ fin_rhist, DevScal* sc) {
    using C = RhsFwdShape<N, LR, R>;
    constexpr int RW = C::RW, T = C::T, CPT = C::CPT, RH = C::RH, NR = C::NR, NU = C::NU;
    constexpr int NT = C::NT, E = C::E, LX = C::LX, H = N / 2;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    if (fin_part != nullptr && blockIdx.x == 0) {   // folded finalize (FinFold)
        __shared__ double fred[2 * 16];
        fin_outer_body(fin_part, fin_nb, fin_rhist, sc[z], z, fred);
    }
    const size_t MN = (size_t)M * N;
    phi_s += z * MN; W += 2 * z * MN; g += z * MN; D += z * MN;
    spec += (size_t)z * M * H;
    extern __shared__ float lds[];
    float* sv1 = lds;             // vertical window sums, RW rows x N
    float* sv2 = sv1 + RW * N;
    float* sph = sv2 + RW * N;    // phi on the RW rows
    const int row0 = strip_row0(blockIdx.x, gridDim.x, LR);
    const int tid = threadIdx.x;
    const float lim = kp.band_l + kp.eps;
    // the transform's stage twiddles, loaded now so that they arrive with phi
    const int gq = tid / NT, t = tid - gq * NT;
    float2 twr[TwN<N, E>::v];
    tw_preload<N, E>(stN, t, twr);

    // phase 1 (per owned column): loads, u = w h(phi), vertical sums
    float ph[CPT][RW], lv[CPT][RW], dv[CPT][RW], w1o[CPT][RW], w2o[CPT][RW], go[CPT][RW];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int c = tid + q * T;
        float p[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) p[rr] = phi_s[(size_t)bidx<BC>(row0 - RH + rr, M) * N + c];
#pragma unroll
        for (int r = 0; r < RW; ++r) dv[q][r] = D[(size_t)(row0 + r) * N + c];
        float a1[NU], a2[NU];
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            const float pv = p[RH - R + m];
            a1[m] = 0.0f;
            a2[m] = 0.0f;
            if (pv <= lim && pv >= -lim) {
                const size_t o = (size_t)bidx<BC>(row0 - R + m, M) * N + c;
                a1[m] = W[o];
                a2[m] = W[MN + o];
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const float pv = p[RH + r];
            go[q][r] = 0.0f;
            if (pv <= lim && pv >= -lim) go[q][r] = g[(size_t)(row0 + r) * N + c];
            w1o[q][r] = a1[R + r];
            w2o[q][r] = a2[R + r];
            ph[q][r] = pv;
            lv[q][r] = p[RH + r - 1] + p[RH + r + 1];
        }
        float u1[NU], u2[NU];
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            const float h = band_h(p[RH - R + m], kp);
            u1[m] = a1[m] * h;
            u2[m] = a2[m] * h;
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
            for (int pp = 0; pp <= 2 * R; ++pp) {
                s1 += kp.taps[pp] * u1[r + pp];
                s2 += kp.taps[pp] * u2[r + pp];
            }
            sv1[r * N + c] = s1;
            sv2[r * N + c] = s2;
            sph[r * N + c] = ph[q][r];
        }
    }
    __syncthreads();
    // phase 2: horizontal window factor, Laplacian, force, F
    float F[CPT][RW];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int c = tid + q * T;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const float p = ph[q][r];
            float force = 0.0f;
            if (p <= lim && p >= -lim) {
                float v1 = 0.0f, v2 = 0.0f;
#pragma unroll
                for (int qq = 0; qq <= 2 * R; ++qq) {
                    const int cc = bidx<BC>(c - R + qq, N);
                    v1 += kp.taps[qq] * sv1[r * N + cc];
                    v2 += kp.taps[qq] * sv2[r * N + cc];
                }
                float dl, ddl, h, dh;
                dirac_d(p, kp, dl, ddl);
                band_h_dh(p, kp, h, dh);
                const float w1 = w1o[q][r], w2 = w2o[q][r], gg = go[q][r];
                const float wn = sqrtf(w1 * w1 + w2 * w2);
                force = -kp.gamma * gg * wn * ddl + kp.alpha * gg * dl + 2.0f * kp.beta * dh * (w1 * v1 + w2 * v2);
            }
            const float left = sph[r * N + bidx<BC>(c - 1, N)], right = sph[r * N + bidx<BC>(c + 1, N)];
            const float lap = lv[q][r] + (left + right) - 4.0f * p;
            F[q][r] = kp.tau * (force + dv[q][r] + kp.mu * lap);
        }
    }
    __syncthreads();   // the FFT buffers alias the window buffers
    // phase 3: rows 2m, 2m + 1 as one complex row, forward FFT, R2C split, store
    extern __shared__ float2 xs[];
    float2* x = xs + gq * LX;
    float2 io[E];
    if constexpr (BC == 1) {
        // Neumann: the DCT-II of each row through its even / odd reordering
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int c = tid + q * T, pc = dct_pos(c, N);
#pragma unroll
            for (int r = 0; r < RW; r += 2) xs[(r >> 1) * LX + sk(pc)] = make_float2(F[q][r], F[q][r + 1]);
        }
        fft_lds_pre<N, E, false>(x, twr, t, io);
        dct_row_store<N, LR>(xs, spec, row0, tid, T, dtN);
        return;
    } else if constexpr (C::NTR == 1) {
        // one transform: thread t's columns t + q NT are its first-stage inputs
#pragma unroll
        for (int q = 0; q < CPT; ++q) io[q] = make_float2(F[q][0], F[q][1]);
        fft_lds_pre<N, E, false, true, false>(x, twr, t, io);
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int c = tid + q * T;
#pragma unroll
            for (int r = 0; r < RW; r += 2) xs[(r >> 1) * LX + sk(c)] = make_float2(F[q][r], F[q][r + 1]);
        }
        fft_lds_pre<N, E, false>(x, twr, t, io);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = tid + e * T;
        int r, kk;
        size_t di;
        if constexpr (LR >= 3) {
            r = o & 7;
            kk = (o >> 3) & (H - 1);
            r += ((o >> 3) / H) * 8;
            di = (size_t)row0 * H + o;
        } else {
            r = o & (RW - 1);
            kk = o >> LR;
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

// ---------------------------------------------------------------------------
// launch templates
// ---------------------------------------------------------------------------
struct FusedArgs {
    const Geometry* geo;
    const KParams* kp;
    const float *phi_s, *W, *g, *D;
    float2* spec;
    int nz;
    DevScal* sc;
    hipStream_t st;
    const FinFold* fold;
    int lr;   // log2 rows per workgroup (one of the instantiated strip heights)
};

// Strip heights instantiated per row length: the smallest whose workgroup
// fills a wave, and the next (8-row strips only below 256 points: at 1024
// they measured slowest).
template <int N, int LR, int R>
void launch_rhs_fwd_nlr(const FusedArgs& a) {
    using Cs = RhsFwdShape<N, LR, R>;
    const Geometry& geo = *a.geo;
    launch_iter(geo.bc ? k_rhs_fwd<N, LR, R, 1> : k_rhs_fwd<N, LR, R, 0>, dim3(geo.M >> LR, 1, a.nz), dim3(Cs::T),
                Cs::lds_bytes, a.st, *a.kp, geo.M, a.phi_s, a.W, a.g, a.D, a.spec, geo.stN, geo.dtN,
                a.fold ? a.fold->part : nullptr, a.fold ? a.fold->nb : 0, a.fold ? a.fold->rhist : nullptr, a.sc);
}
template <int N, int R>
void launch_rhs_fwd_n(const FusedArgs& a) {
    if constexpr (N >= 256) {
        if (a.lr == 1) return launch_rhs_fwd_nlr<N, 1, R>(a);
        return launch_rhs_fwd_nlr<N, 2, R>(a);
    } else if constexpr (N == 128) {
        if (a.lr == 2) return launch_rhs_fwd_nlr<N, 2, R>(a);
        return launch_rhs_fwd_nlr<N, 3, R>(a);
    } else {
        return launch_rhs_fwd_nlr<N, 3, R>(a);
    }
}
template <int N>
void fused_launch_len(const FusedArgs& a) {
    switch (a.kp->R) {
        case 0: launch_rhs_fwd_n<N, 0>(a); break;
        case 1: launch_rhs_fwd_n<N, 1>(a); break;
        case 2: launch_rhs_fwd_n<N, 2>(a); break;
        case 3: launch_rhs_fwd_n<N, 3>(a); break;
        case 4: launch_rhs_fwd_n<N, 4>(a); break;
        case 5: launch_rhs_fwd_n<N, 5>(a); break;
        case 6: launch_rhs_fwd_n<N, 6>(a); break;
        case 7: launch_rhs_fwd_n<N, 7>(a); break;
        case 8: launch_rhs_fwd_n<N, 8>(a); break;
        default: break;
    }
}
template <int N, int LR, int R>
void set_fused_attr() {
    const int bytes = 160 * 1024 - 1024;
    (void)hipFuncSetAttribute((const void*)k_rhs_fwd<N, LR, R, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute((const void*)k_rhs_fwd<N, LR, R, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
template <int N, int R>
void set_fused_attrs_nr() {
    if constexpr (N >= 256) {
        set_fused_attr<N, 1, R>();
        set_fused_attr<N, 2, R>();
    } else if constexpr (N == 128) {
        set_fused_attr<N, 2, R>();
        set_fused_attr<N, 3, R>();
    } else {
        set_fused_attr<N, 3, R>();
    }
}
template <int N>
void fused_configure_len() {
    set_fused_attrs_nr<N, 0>(); set_fused_attrs_nr<N, 1>(); set_fused_attrs_nr<N, 2>();
    set_fused_attrs_nr<N, 3>(); set_fused_attrs_nr<N, 4>(); set_fused_attrs_nr<N, 5>();
    set_fused_attrs_nr<N, 6>(); set_fused_attrs_nr<N, 7>(); set_fused_attrs_nr<N, 8>();
}

// per-length entry points (one per translation unit group)
void fused_launch_64(const FusedArgs& a);
void fused_launch_128(const FusedArgs& a);
void fused_launch_256(const FusedArgs& a);
void fused_launch_512(const FusedArgs& a);
void fused_launch_1024(const FusedArgs& a);
void fused_configure_small();
void fused_configure_512();
void fused_configure_1024();

}  // namespace sr
