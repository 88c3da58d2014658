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
// applies both convolutions.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "sr_aos.hpp"
#include "sr_device.hpp"

namespace sr {

namespace {
constexpr int kAosTW = 64;    // tile columns (one wave per row)
constexpr int kAosTH = 16;    // tile rows
constexpr int kAosThreads = 256;

// F = phi + r - tau mu Lap phi on the extended tile (rows i0-Kx .. i0+TH+Kx,
// columns j0-Ky .. j0+64+Ky, periodic), then
// out = (sum_k cx[|k|] F(i+k, j) + sum_k cy[|k|] F(i, j+k)) / 2.
__global__ __launch_bounds__(kAosThreads) void k_aos(const float* __restrict__ rhs, const float* __restrict__ phi,
                                                      float* __restrict__ out, const float* __restrict__ cx, int Kx,
                                                      const float* __restrict__ cy, int Ky, float taumu, int M, int N,
                                                      DevScal* sc) {
    const int z = blockIdx.z;
    if (!sc[z].active) return;
    const size_t MN = (size_t)M * N;
    rhs += z * MN;
    phi += z * MN;
    out += z * MN;
    extern __shared__ float sF[];
    const int EH = kAosTH + 2 * Kx, EW = kAosTW + 2 * Ky;
    const int i0 = blockIdx.y * kAosTH, j0 = blockIdx.x * kAosTW;
    for (int e = threadIdx.x; e < EH * EW; e += blockDim.x) {
        const int ei = e / EW, ej = e - ei * EW;
        const int ei_ = ei - Kx, ej_ = ej - Ky;
        // only the cross-shaped part is read by the convolutions
        if ((ei_ < 0 || ei_ >= kAosTH) && (ej_ < 0 || ej_ >= kAosTW)) continue;
        const int gi = (i0 + ei_) & (M - 1), gj = (j0 + ej_) & (N - 1);
        const size_t o = (size_t)gi * N + gj;
        const float p = phi[o];
        const float lap = (phi[(size_t)((gi - 1) & (M - 1)) * N + gj] + phi[(size_t)((gi + 1) & (M - 1)) * N + gj]) +
                          (phi[(size_t)gi * N + ((gj - 1) & (N - 1))] + phi[(size_t)gi * N + ((gj + 1) & (N - 1))]) -
                          4.0f * p;
        sF[e] = p + (rhs[o] - taumu * lap);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kAosTH * kAosTW; e += blockDim.x) {
        const int i = e / kAosTW, j = e - i * kAosTW;
        const int gi = i0 + i, gj = j0 + j;
        if (gi >= M || gj >= N) continue;
        const float* col = sF + (i + Kx) * EW + (j + Ky);
        float v1 = cx[0] * col[0], v2 = cy[0] * col[0];
        for (int k = 1; k <= Kx; ++k) v1 += cx[k] * (col[-k * EW] + col[k * EW]);
        for (int k = 1; k <= Ky; ++k) v2 += cy[k] * (col[-k] + col[k]);
        out[(size_t)gi * N + gj] = 0.5f * (v1 + v2);
    }
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
    for (int k = 0; k <= K; ++k) taps[k] = (float)c[k];
    return K;
}

size_t aos_lds_bytes(int Kx, int Ky) { return sizeof(float) * (size_t)(kAosTH + 2 * Kx) * (kAosTW + 2 * Ky); }

void configure_aos() {
    static bool done = false;
    if (done) return;
    done = true;
    (void)hipFuncSetAttribute((const void*)k_aos, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
}

void launch_aos(int M, int N, const float* rhs, const float* phi_in, float* phi_out, const float* cx, int Kx,
                const float* cy, int Ky, float taumu, int nz, DevScal* sc, hipStream_t st, hipEvent_t ev0,
                hipEvent_t ev1) {
    const dim3 grid((N + kAosTW - 1) / kAosTW, (M + kAosTH - 1) / kAosTH, nz);
    const uint32_t lds = (uint32_t)aos_lds_bytes(Kx, Ky);
    if (ev0)
        hipExtLaunchKernelGGL(k_aos, grid, dim3(kAosThreads), lds, st, ev0, ev1, 0u, rhs, phi_in, phi_out, cx, Kx,
                              cy, Ky, taumu, M, N, sc);
    else
        hipLaunchKernelGGL(k_aos, grid, dim3(kAosThreads), lds, st, rhs, phi_in, phi_out, cx, Kx, cy, Ky, taumu, M,
                           N, sc);
}

}  // namespace sr
