// The semi-implicit solve of eqs (31)-(33) without a context, a workspace or
// any allocation: sr_implicit_solve_noalloc (include/sr.h).  Everything the
// solve needs besides its input and output -- the half spectrum, the twiddle
// tables of both transform lengths and the per-instance flags the FFT
// kernels read -- lives in one file-scope device array, `scratch`, of fixed
// size.  Host code never uses the array's name as an address: the device
// address is looked up once per device with hipGetSymbolAddress and kept.
// The tables are built on the device (FP64 sincospi, rounded to FP32) by a
// kernel, so a call enqueues kernels only and can be captured into a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "../../include/sr.h"
#include "sr_device.hpp"
#include "sr_kernels.hpp"

namespace sr {
int api_fail(int code, const char* msg);
void configure_kernels();
}

namespace {

constexpr int kMaxSide = 4096;
constexpr size_t kMaxPixels = (size_t)1 << 22;   // M * N at most 4 Mpx
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
// Layout of the scratch array: spectrum, twM, twN, stM, stN, flags.
constexpr size_t kSpecBytes = kMaxPixels * 4;             // (M x N/2) float2
constexpr size_t kTwBytes = align_up(sizeof(float2) * kMaxSide);
constexpr size_t kStageBytes = align_up(sizeof(float2) * 4 * kMaxSide);   // >= any stage table
constexpr size_t kScalBytes = align_up(sizeof(sr::DevScal));
constexpr size_t kPartBytes = align_up(sizeof(double) * 64);
constexpr size_t kScratchBytes = kSpecBytes + 2 * kTwBytes + 2 * kStageBytes + kScalBytes + kPartBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[64] = {};   // device address of `scratch`, per device

// Table of length L: tw[n] = exp(-2 pi i n / L), n < L, and the stage twiddle
// table of (L, E) in the order the Stockham stages read it: for every stage
// with Ns > 1, Ns blocks of R entries W_{R Ns}^{r k} (r < R).
__global__ void k_noalloc_tables(float2* tw, float2* st, int L, int E) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < L) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)L, &s, &c);
        tw[t] = make_float2((float)c, (float)s);
    }
    // stage table entry t: find its stage
    int off = 0;
    for (int Ns = 1; Ns < L;) {
        const int R = sr::fft_radix(L, E, Ns);
        if (Ns > 1) {
            const int len = Ns * R;
            if (t >= off && t < off + len) {
                const int k = (t - off) / R, r = (t - off) - k * R;
                double s, c;
                sincospi(-2.0 * (double)(r * k) / (double)(R * Ns), &s, &c);
                st[t] = make_float2((float)c, (float)s);
            }
            off += len;
        }
        Ns *= R;
    }
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

}  // namespace

extern "C" int sr_implicit_solve_noalloc(int32_t M, int32_t N, double tau, double mu, const float* rhs,
                                         float* u_out, void* hip_stream) {
    if (!rhs || !u_out) return sr::api_fail(SR_EINVAL, "NULL argument");
    if (!pow2_in(M, 8, kMaxSide) || !pow2_in(N, 8, kMaxSide))
        return sr::api_fail(SR_EUNSUPPORTED, "M and N must be powers of two in [8, 4096]");
    if ((size_t)M * (size_t)N > kMaxPixels)
        return sr::api_fail(SR_EUNSUPPORTED, "sr_implicit_solve_noalloc: M * N must be at most 4194304 "
                                             "(its fixed scratch holds the half spectrum of 4 Mpx)");
    if (!(tau > 0.0) || !(mu > 0.0) || !std::isfinite(tau * mu))
        return sr::api_fail(SR_EINVAL, "tau and mu must be positive and finite");
    const int LM = sr::fft_stage_table_len(M, true), LN = sr::fft_stage_table_len(N, false);
    if ((size_t)LM * sizeof(float2) > kStageBytes || (size_t)LN * sizeof(float2) > kStageBytes)
        return sr::api_fail(SR_EUNSUPPORTED, "stage table exceeds its scratch slot");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return sr::api_fail(SR_EUNSUPPORTED, "device index beyond 63");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                char msg[256];
                std::snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
                return sr::api_fail(SR_EHIP, msg);
            }
            g_scratch_ptr[dev] = p;
        }
        base = g_scratch_ptr[dev];
    }
    unsigned char* b = static_cast<unsigned char*>(base);
    float2* spec = reinterpret_cast<float2*>(b);
    float2* twM = reinterpret_cast<float2*>(b + kSpecBytes);
    float2* twN = reinterpret_cast<float2*>(b + kSpecBytes + kTwBytes);
    float2* stM = reinterpret_cast<float2*>(b + kSpecBytes + 2 * kTwBytes);
    float2* stN = reinterpret_cast<float2*>(b + kSpecBytes + 2 * kTwBytes + kStageBytes);
    sr::DevScal* sc = reinterpret_cast<sr::DevScal*>(b + kSpecBytes + 2 * kTwBytes + 2 * kStageBytes);
    double* part = reinterpret_cast<double*>(b + kSpecBytes + 2 * kTwBytes + 2 * kStageBytes + kScalBytes);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    sr::configure_kernels();
    // tables and flags are rebuilt on every call: the array keeps whatever
    // the previous call (of any size) left in it
    const int nM = std::max(M, LM), nN = std::max(N, LN);
    hipLaunchKernelGGL(k_noalloc_tables, dim3((nM + 255) / 256), dim3(256), 0, st, twM, stM, M,
                       sr::fft_elems(M, true));
    hipLaunchKernelGGL(k_noalloc_tables, dim3((nN + 255) / 256), dim3(256), 0, st, twN, stN, N,
                       sr::fft_elems(N, false));
    sr::launch_reset_scal(sc, 1, 1, st);
    sr::Geometry geo{};
    geo.M = M;
    geo.N = N;
    geo.twM = twM;
    geo.twN = twN;
    geo.stM = stM;
    geo.stN = stN;
    geo.taumu = (float)(tau * mu);
    geo.bc = 0;
    sr::launch_solve(geo, rhs, nullptr, u_out, spec, 0.0f, part, 1, sc, st);
    e = hipGetLastError();
    if (e != hipSuccess) return sr::api_fail(SR_EHIP, hipGetErrorString(e));
    return SR_OK;
}
