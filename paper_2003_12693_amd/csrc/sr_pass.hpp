// Device helpers and the launch helper shared by the kernels of the
// semi-implicit solve's passes (sr_kernels.hip, sr_fused.hip, sr_dct.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>

#include "sr_device.hpp"

namespace sr {

// Rows 2m and 2m+1 of the real field r are transformed together as one
// complex row z = r_a + i r_b.  Each row's half spectrum X[k], k < N/2 (the
// DC slot carrying (X[0], X[N/2]) as its real and imaginary parts) is stored
// in 8-row tiles: element (row i, k) at ((i / 8) * (N/2) + k) * 8 + i % 8.
// Row passes then write / read 64-byte runs (8 rows of one frequency) and
// the column pass reads 64-byte runs (8 rows of one column; the two columns
// of a 128-byte run are read by workgroups on one XCD).
constexpr int kSpecTile = 8;

// First row of workgroup b's rows (2^lrpw of them; nb workgroups).  When a
// workgroup holds fewer than the 8 rows of a spectrum tile, the pieces of one
// tile go to workgroups b, b + 8, ... which the dispatcher sends to the same
// XCD (it deals workgroups to the 8 XCDs in turn), so each tile's 64-byte
// runs are completed (written, or re-read) in one L2.
__device__ __forceinline__ int row_piece0(int b, int nb, int lrpw) {
    if (lrpw >= 3) return b << lrpw;
    const int P = 8 >> lrpw;                 // pieces per tile
    if (nb % (8 * P)) return b << lrpw;      // small grids: linear order
    const int x = b & 7, s = b >> 3;
    return ((s / P) * 8 + x) * 8 + ((s % P) << lrpw);
}

// Outer-iteration finalize of instance z, by every thread of one workgroup.
__device__ __forceinline__ void fin_outer_body(const double* __restrict__ part, int nb, double* __restrict__ rhist,
                                               DevScal& S, int z, double* red) {
    double v[2];
    sum_partials<2>(part + (size_t)z * 2 * nb, nb, v, red);
    if (threadIdx.x == 0) {
        const double r = sqrt(v[0]) / (sqrt(v[1]) + 1e-6);
        S.r_last = r;
        rhist[(size_t)z * kRHist + (S.k % kRHist)] = r;
        S.k += 1;
        if (S.inner_done) S.inner_done = 0;   // (a folded finalize never finds it set)
        // batched solves retire an instance on the device: cap, tolerance, NaN
        if (!(r == r) || r > 1e30) { S.nonfinite = 1; S.active = 0; }
        else if (S.tol_outer > 0.0 && S.k >= S.min_iter && r < S.tol_outer) { S.converged = 1; S.active = 0; }
        else if (S.max_iter > 0 && S.k >= S.max_iter) S.active = 0;
    }
}

// First row of workgroup b's strip of 2^lrpw rows.  Workgroups are dealt to
// the 8 XCDs in turn, so XCD x = b % 8 is given a contiguous band of 8-row
// spectrum tiles (the halo rows of neighbouring strips then meet in one L2),
// and the pieces of one tile stay on one XCD.
__device__ __forceinline__ int strip_row0(int b, int nb, int lrpw) {
    const int P = lrpw >= 3 ? 1 : 8 >> lrpw;          // workgroups per 8-row tile
    const int per = lrpw >= 3 ? 1 << (lrpw - 3) : 1;  // tiles per workgroup
    if (nb & 7) return b << lrpw;
    const int x = b & 7, s = b >> 3, nx = nb >> 3;    // s-th workgroup on XCD x
    if (P == 1) return (x * nx + s) * per * 8;
    if (nx % P) return b << lrpw;
    const int tile = x * (nx / P) + s / P;
    return tile * 8 + ((s % P) << lrpw);
}

// DCT-II by Makhoul's reordering (the Neumann solve, sr_dct.hip): element n
// of the reordered sequence v[n] = x[2n], v[L-1-n] = x[2n+1].
// Column (row) index of element n of the reordered sequence of length L.
__device__ __forceinline__ int dct_src(int n, int L) { return n < L / 2 ? 2 * n : 2 * (L - 1 - n) + 1; }
// Position in the reordered sequence of element c.
__device__ __forceinline__ int dct_pos(int c, int L) { return (c & 1) ? L - 1 - (c >> 1) : c >> 1; }

// Stores the DCT-II coefficients of the rows a strip's transforms hold (xs:
// transform g's output at xs + g LX, rows 2g and 2g + 1 packed as a + i b)
// into the spectrum tiles: slot (row r, m) = (X_r[2m], X_r[2m + 1]).
template <int N, int LR>
__device__ __forceinline__ void dct_row_store(const float2* xs, float2* __restrict__ spec, int row0, int tid,
                                              int nthr, const float2* __restrict__ dtN) {
    constexpr int H = N / 2, E = FftShape<N>::E, LX = LdsLen<N>::v;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int o = tid + e * nthr;
        int r, m;
        size_t di;
        if constexpr (LR >= 3) {
            r = o & 7;
            m = (o >> 3) & (H - 1);
            r += ((o >> 3) / H) * 8;
            di = (size_t)row0 * H + o;
        } else {
            r = o & ((1 << LR) - 1);
            m = o >> LR;
            di = ((size_t)(row0 >> 3) * H + m) * 8 + (row0 & 7) + r;
        }
        const float2* xz = xs + (r >> 1) * LX;
        float X[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * m + h;
            const float2 Zk = xz[sk(k)], Zm = xz[sk((N - k) & (N - 1))];
            // this row's spectrum V[k]: (Z[k] + conj Z[N-k]) / 2 for row a, (Z[k] - conj Z[N-k]) / 2i for b
            const float2 V = (r & 1) ? make_float2(0.5f * (Zk.y + Zm.y), -0.5f * (Zk.x - Zm.x))
                                     : make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
            const float2 d = dtN[k];
            X[h] = d.x * V.x - d.y * V.y;
        }
        spec[di] = make_float2(X[0], X[1]);
    }
}

// Launch of an iteration kernel: through hipExtLaunchKernel with the start /
// stop events set by set_launch_events on this host thread (per-kernel
// timing), else a plain launch.  launch_iter converts the arguments to the
// kernel's parameter types.
void launch_kernel_ev(const void* fn, dim3 grid, dim3 block, void** args, size_t lds, hipStream_t st);
template <typename... KArgs, typename... Args>
inline void launch_iter(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        Args... args) {
    std::tuple<KArgs...> vals(static_cast<KArgs>(args)...);
    std::apply(
        [&](auto&... v) {
            void* ptrs[] = {static_cast<void*>(&v)...};
            launch_kernel_ev(reinterpret_cast<const void*>(kernel), grid, block, ptrs, lds, st);
        },
        vals);
}

}  // namespace sr
