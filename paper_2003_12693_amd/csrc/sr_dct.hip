// The semi-implicit solve of the phi sub-problem with Neumann boundaries
// (the zero normal derivative of eqs 17 and 27): (1 - tau mu Lap) u = r for
// the mirrored five-point Laplacian, diagonalised by the DCT-II, whose
// eigenvalues are 1 + tau mu (4 - 2 cos(pi l1 / M) - 2 cos(pi l2 / N)) (the
// Neumann counterpart of eq 32).
//
// Each DCT-II of length L is computed through one L-point complex FFT of the
// even / odd reordering v[n] = x[2n], v[L-1-n] = x[2n+1], followed by
//   X[k] = Re(exp(-i pi k / (2L)) V[k])
// (Makhoul's reordering), and inverted by
//   V[k] = exp(i pi k / (2L)) (X[k] - i X[L-k]),  X[L] = 0,  v = IFFT(V),
// with the reordering undone.  As in the periodic solve, two real rows (two
// real columns) share one complex transform, and the passes have the same
// shapes and memory traffic:
//   k_row_dct_fwd   : reordered load of two rows, FFT, split into the two
//                     rows' spectra, post-twiddle; a row's N real DCT
//                     coefficients are stored as N/2 float2 in the 8-row
//                     spectrum tiles of the periodic solve;
//   k_col_dct_solve : a float2 column of that layout is two real columns of
//                     coefficients: reordered load, FFT, per frequency pair
//                     (l, M - l) the forward post-twiddle, the division by
//                     the two columns' eigenvalues (and 1/(MN)), the inverse
//                     pre-twiddle, then the inverse FFT and the reordered
//                     store;
//   k_row_dct_inv   : the inverse pre-twiddle of two rows, inverse FFT,
//                     un-reordering, phi_{s+1} = phi_s + u.
#include <hip/hip_runtime.h>

#include "sr_device.hpp"
#include "sr_kernels.hpp"
#include "sr_pass.hpp"

namespace sr {

// Forward row DCT-II of the right-hand side plane (rows of 2048 and 4096
// points; shorter rows go through the fused right-hand-side kernel).
template <int N, int LR>
__global__ __launch_bounds__(1024) void k_row_dct_fwd(const float* __restrict__ src, float2* __restrict__ spec,
                                                      const float2* __restrict__ stN, const float2* __restrict__ dtN,
                                                      int M, int lrpw_rt, DevScal* sc) {
    const int lrpw = LR ? LR : lrpw_rt;
    constexpr int NT = FftShape<N>::NT, E = FftShape<N>::E, H = N / 2;
    const int z = blockIdx.z;
    if (!sc[z].active || sc[z].inner_done) return;
    src += (size_t)z * M * N;
    spec += (size_t)z * M * H;
    extern __shared__ float2 xs[];
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int row0 = row_piece0(blockIdx.x, gridDim.x, lrpw);
    const size_t ra = (size_t)(row0 + 2 * g) * N, rb = ra + N;
    constexpr int LX = LdsLen<N>::v;
    float2* x = xs + g * LX;
    float2 io[E];   // element n = t + e NT of the reordered complex row
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = dct_src(t + e * NT, N);
        io[e] = make_float2(src[ra + c], src[rb + c]);
    }
    constexpr bool PRE = E <= 4;
    float2 twr[TwN<N, E>::v];
    if constexpr (PRE) {
        tw_preload<N, E>(stN, t, twr);
        fft_lds_pre<N, E, false, true, false>(x, twr, t, io);
    } else {
        fft_lds<N, E, false, true, false>(x, stN, t, io);
    }
    const int nthr = LR ? ((1 << LR) / 2) * NT : (int)blockDim.x;
    if constexpr (LR > 0) {
        dct_row_store<N, LR>(xs, spec, row0, threadIdx.x, nthr, dtN);
    } else {
        // runtime strip height: the same store with the index split at run time
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int o = threadIdx.x + e * nthr;
            int r, m;
            size_t di;
            if (lrpw >= 3) {
                r = o & 7;
                m = (o >> 3) & (H - 1);
                r += ((o >> 3) / H) * 8;
                di = (size_t)row0 * H + o;
            } else {
                r = o & ((1 << lrpw) - 1);
                m = o >> lrpw;
                di = ((size_t)(row0 >> 3) * H + m) * 8 + (row0 & 7) + r;
            }
            const float2* xz = xs + (r >> 1) * LX;
            float X[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 2 * m + h;
                const float2 Zk = xz[sk(k)], Zm = xz[sk((N - k) & (N - 1))];
                const float2 V = (r & 1) ? make_float2(0.5f * (Zk.y + Zm.y), -0.5f * (Zk.x - Zm.x))
                                         : make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
                const float2 d = dtN[k];
                X[h] = d.x * V.x - d.y * V.y;
            }
            spec[di] = make_float2(X[0], X[1]);
        }
    }
}

// Column pass: G float2 columns (2G real columns) per workgroup.
template <int M, int GT>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 1024), amdgpu_waves_per_eu(ColWaves<M>::v))) void
k_col_dct_solve(float2* __restrict__ spec, const float* __restrict__ cM, const float* __restrict__ cN,
                const float2* __restrict__ dtM, const float2* __restrict__ stM, int N, int G_rt, int lrun_rt,
                float taumu, float inv_mn, DevScal* sc) {
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
    int k0 = blockIdx.x * G;
    if (G == 1 && (gridDim.x & 15) == 0) {
        const int b = blockIdx.x, s = b >> 3;
        k0 = (((s >> 1) << 3) + (b & 7)) * 2 + (s & 1);
    }
    const int run = kSpecTile * G;
    float2* base = spec + (size_t)k0 * kSpecTile;
    constexpr bool ONE = GT == 1;
    // Element p of the reordered column is row dct_src(p, M).  With one
    // column per workgroup, thread t loads the rows of its first-stage
    // inputs p = t + e NT directly.
    float2 io[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = threadIdx.x + e * nthr;
        if constexpr (ONE) {
            const int q = dct_src(idx, M);
            io[e] = base[(size_t)(q >> 3) * H * kSpecTile + (q & 7)];
        } else {
            io[e] = base[(size_t)(idx >> lrun) * H * kSpecTile + (idx & (run - 1))];
        }
    }
    if constexpr (!ONE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * nthr;
            const int rem = idx & (run - 1);
            const int row = (idx >> lrun) * kSpecTile + (rem & 7);
            xs[(rem >> 3) * LD + sk(dct_pos(row, M))] = io[e];
        }
    }
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    const int col = k0 + g;   // float2 column m: real columns 2m and 2m + 1
    float2* x = xs + g * LD;
    // the tables the frequency pairs need, loaded with the data (the
    // transform's barriers would hold them back until after it)
    const float ca = 4.0f - cN[2 * col], cb = 4.0f - cN[2 * col + 1];
    float2 dtv[E / 2 + 1];
    float cl[E / 2 + 1], cr[E / 2 + 1];
#pragma unroll
    for (int e = 0; e <= E / 2; ++e) {
        const int l = e < E / 2 ? t + e * NT : M / 2, lm = (M - l) & (M - 1);
        dtv[e] = dtM[l];
        cl[e] = cM[l];
        cr[e] = cM[lm];
    }
    constexpr bool PRE = E <= 4;
    float2 twr[TwN<M, E>::v];
    if constexpr (PRE) {
        tw_preload<M, E>(stM, t, twr);
        fft_lds_pre<M, E, false, ONE, false>(x, twr, t, io);
    } else {
        fft_lds<M, E, false, ONE, false>(x, stM, t, io);
    }
    // frequency pair (l, M - l) of both real columns: forward post-twiddle,
    // division by the eigenvalues (1/(MN) folded in), inverse pre-twiddle
    auto solve_pair = [&](int l, float2 c, float cml, float cmm) {
        const int lm = (M - l) & (M - 1);
        const float2 Zl = x[sk(l)], Zm = x[sk(lm)];
        const float2 Va = make_float2(0.5f * (Zl.x + Zm.x), 0.5f * (Zl.y - Zm.y));
        const float2 Vb = make_float2(0.5f * (Zl.y + Zm.y), -0.5f * (Zl.x - Zm.x));
        const float2 pa = cmul(c, Va), pb = cmul(c, Vb);
        // coefficients Y[l] = Re(c V[l]) and Y[M - l] = -Im(c V[l]) (none for l = 0)
        const float sl_a = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (ca - cml));
        const float sl_b = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (cb - cml));
        const float sm_a = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (ca - cmm));
        const float sm_b = inv_mn * __builtin_amdgcn_rcpf(1.0f + taumu * (cb - cmm));
        const float ua = pa.x * sl_a, ub = pb.x * sl_b;
        const float uam = l ? -pa.y * sm_a : 0.0f, ubm = l ? -pb.y * sm_b : 0.0f;
        // P[l] = conj(c) (U[l] - i U[M - l]) per column, packed a + i b
        const float2 Pa = make_float2(c.x * ua - c.y * uam, -c.x * uam - c.y * ua);
        const float2 Pb = make_float2(c.x * ub - c.y * ubm, -c.x * ubm - c.y * ub);
        x[sk(l)] = make_float2(Pa.x - Pb.y, Pa.y + Pb.x);
        if (l != lm) x[sk(lm)] = make_float2(Pa.x + Pb.y, Pb.x - Pa.y);
    };
#pragma unroll
    for (int e = 0; e < E / 2; ++e) solve_pair(t + e * NT, dtv[e], cl[e], cr[e]);   // l in [0, M/2)
    if (t == 0) solve_pair(M / 2, dtv[E / 2], cl[E / 2], cr[E / 2]);
    int t_inv = t;
    asm volatile("" : "+v"(t_inv));
    if constexpr (PRE) fft_lds_pre<M, E, true, false, ONE>(x, twr, t_inv, io);
    else fft_lds<M, E, true, false, ONE>(x, stM, t_inv, io);
    if constexpr (!ONE) __syncthreads();
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if constexpr (ONE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = dct_src(tid + e * nthr, M);
            base[(size_t)(q >> 3) * H * kSpecTile + (q & 7)] = io[e];
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = tid + e * nthr;
        const int q = idx >> lrun, rem = idx & (run - 1);
        const int row = q * kSpecTile + (rem & 7);
        base[(size_t)q * H * kSpecTile + rem] = xs[(rem >> 3) * LD + sk(dct_pos(row, M))];
    }
}

// Inverse row DCT (two rows per complex FFT) and phi_{s+1} = phi_s + u; the
// inner stop rule's partial sums as in the periodic inverse pass.
template <int N, int LR>
__global__ __launch_bounds__(1024) void k_row_dct_inv(const float2* __restrict__ spec,
                                                      const float* __restrict__ phi_in, float* __restrict__ phi_out,
                                                      const float2* __restrict__ stN, const float2* __restrict__ dtN,
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
    // stage the coefficients as real rows: row a of transform g at floats [0, N), row b at [N, 2N)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = threadIdx.x + e * nthr;
        int r, m;
        size_t si;
        if (lrpw >= 3) {
            r = o & 7;
            m = (o >> 3) & (H - 1);
            r += ((o >> 3) / H) * 8;
            si = (size_t)row0 * H + o;
        } else {
            r = o & ((1 << lrpw) - 1);
            m = o >> lrpw;
            si = ((size_t)(row0 >> 3) * H + m) * 8 + (row0 & 7) + r;
        }
        float* xf = reinterpret_cast<float*>(xs + (r >> 1) * LX) + (r & 1) * N;
        const float2 v = spec[si];
        xf[2 * m] = v.x;
        xf[2 * m + 1] = v.y;
    }
    const int g = threadIdx.x / NT, t = threadIdx.x - g * NT;
    constexpr bool PRE = E <= 4;
    float2 twr[TwN<N, E>::v];
    if constexpr (PRE) tw_preload<N, E>(stN, t, twr);
    const size_t ra = (size_t)(row0 + 2 * g) * N, rb = ra + N;
    float pav[E], pbv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = t + e * NT;
        pav[e] = phi_in ? phi_in[ra + c] : 0.0f;
        pbv[e] = phi_in ? phi_in[rb + c] : 0.0f;
    }
    __syncthreads();
    float2* x = xs + g * LX;
    const float* xa = reinterpret_cast<const float*>(x);
    const float* xb = xa + N;
    float2 P[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * NT;
        const int km = (N - k) & (N - 1);
        const float ua = xa[k], ub = xb[k];
        const float uam = k ? xa[km] : 0.0f, ubm = k ? xb[km] : 0.0f;
        const float2 c = dtN[k];
        const float2 Pa = make_float2(c.x * ua - c.y * uam, -c.x * uam - c.y * ua);
        const float2 Pb = make_float2(c.x * ub - c.y * ubm, -c.x * ubm - c.y * ub);
        P[e] = make_float2(Pa.x - Pb.y, Pa.y + Pb.x);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) x[sk(t + e * NT)] = P[e];
    float2 unused[E];
    if constexpr (PRE) fft_lds_pre<N, E, true, false, false>(x, twr, t, unused);
    else fft_lds<N, E, true, false, false>(x, stN, t, unused);
    double sd = 0.0, sp = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = t + e * NT;
        const float2 Zv = x[sk(dct_pos(c, N))];
        const float pa = pav[e], pb = pbv[e];
        phi_out[ra + c] = pa + Zv.x;
        phi_out[rb + c] = pb + Zv.y;
        sd += (double)Zv.x * Zv.x + (double)Zv.y * Zv.y;
        sp += (double)pa * pa + (double)pb * pb;
    }
    if (tol_inner > 0.0f) {
        double v[2] = {sd, sp};
        const int nb = gridDim.x;
        store_partials<2>(v, part + (size_t)z * 2 * nb, nb, blockIdx.x, red);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
static void launch_row_dct_fwd_t(const float* src, float2* spec, const float2* stN, const float2* dtN, int M,
                                 int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int lr = fft_row_split(M, N, nz, 1024, 1);
    const size_t lds = sizeof(float2) * ((1 << lr) / 2) * LdsLen<N>::v;
    auto k = lr == 3 ? k_row_dct_fwd<N, 3> : lr == 2 ? k_row_dct_fwd<N, 2> : lr == 1 ? k_row_dct_fwd<N, 1>
                                                                                     : k_row_dct_fwd<N, 0>;
    launch_iter(k, dim3(M >> lr, 1, nz), dim3(((1 << lr) / 2) * NT), lds, st, src, spec, stN, dtN, M, lr, sc);
}
template <int M>
static void launch_col_dct_t(float2* spec, const float* cM, const float* cN, const float2* dtM, const float2* stM,
                             int N, float taumu, float inv_mn, int nz, DevScal* sc, hipStream_t st) {
    const int NT = FftShape<M, ColE<M>::v>::NT;
    const int G = fft_col_group(M, N, nz);
    const size_t lds = sizeof(float2) * G * LdsLen<M>::v;
    int lrun = 0;
    while ((1 << lrun) < kSpecTile * G) ++lrun;
    auto k = G == 2 ? k_col_dct_solve<M, 2> : G == 1 ? k_col_dct_solve<M, 1> : k_col_dct_solve<M, 0>;
    launch_iter(k, dim3(N / 2 / G, 1, nz), dim3(NT * G), lds, st, spec, cM, cN, dtM, stM, N, G, lrun, taumu, inv_mn,
                sc);
}
template <int N>
static void launch_row_dct_inv_t(const float2* spec, const float* phi_in, float* phi_out, const float2* stN,
                                 const float2* dtN, int M, float tol, double* part, int nz, DevScal* sc,
                                 hipStream_t st) {
    const int NT = FftShape<N>::NT;
    const int lr = fft_row_split(M, N, nz, 1024, 2);
    const size_t lds = sizeof(float2) * ((1 << lr) / 2) * LdsLen<N>::v;
    const int nb = M >> lr;
    auto k = lr == 3 ? k_row_dct_inv<N, 3> : lr == 2 ? k_row_dct_inv<N, 2> : k_row_dct_inv<N, 0>;
    launch_iter(k, dim3(nb, 1, nz), dim3(((1 << lr) / 2) * NT), lds, st, spec, phi_in, phi_out, stN, dtN, M, lr, tol,
                part, sc);
    if (tol > 0.0f) launch_fin_inner(part, nb, tol, nz, sc, st);
}

#define SR_DCT_DISPATCH(FN, LEN, ...)                                   \
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

void launch_dct_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                           float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st) {
    const int M = geo.M, N = geo.N;
    if (pass == 0) {
        SR_DCT_DISPATCH(launch_row_dct_fwd_t, N, rhs, spec, geo.stN, geo.dtN, M, nz, sc, st);
    } else if (pass == 1) {
        const float inv_mn = 1.0f / ((float)M * (float)N);
        SR_DCT_DISPATCH(launch_col_dct_t, M, spec, geo.cM, geo.cN, geo.dtM, geo.stM, N, geo.taumu, inv_mn, nz, sc,
                        st);
    } else {
        SR_DCT_DISPATCH(launch_row_dct_inv_t, N, spec, phi_in, phi_out, geo.stN, geo.dtN, M, tol_inner, part, nz,
                        sc, st);
    }
}

template <int L>
static void set_dct_attrs() {
    const int bytes = 160 * 1024 - 1024;
    const void* fns[] = {(const void*)k_row_dct_fwd<L, 0>, (const void*)k_row_dct_fwd<L, 1>,
                         (const void*)k_row_dct_fwd<L, 2>, (const void*)k_row_dct_fwd<L, 3>,
                         (const void*)k_col_dct_solve<L, 0>, (const void*)k_col_dct_solve<L, 1>,
                         (const void*)k_col_dct_solve<L, 2>,
                         (const void*)k_row_dct_inv<L, 0>, (const void*)k_row_dct_inv<L, 2>,
                         (const void*)k_row_dct_inv<L, 3>};
    for (const void* f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void configure_dct() {
    set_dct_attrs<8>(); set_dct_attrs<16>(); set_dct_attrs<32>(); set_dct_attrs<64>(); set_dct_attrs<128>();
    set_dct_attrs<256>(); set_dct_attrs<512>(); set_dct_attrs<1024>(); set_dct_attrs<2048>(); set_dct_attrs<4096>();
}

}  // namespace sr
