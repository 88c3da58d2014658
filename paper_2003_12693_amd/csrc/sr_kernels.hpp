// Host-callable launchers of the SR kernels (see sr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "sr_device.hpp"

namespace sr {

// Per-size constants the FFT passes need: twiddle tables
// tw[n] = exp(-2 pi i n / L) (FP64-computed, rounded to FP32) for the row
// length N and the column length M, and tau * mu of eq (32).
struct Geometry {
    int M, N;
    const float2* twM;
    const float2* twN;
    float taumu;
    int tile_th = 0;   // stencil tile height (16 or 32); 0 = size heuristic
};

int tile_blocks(int M, int N);

void launch_edge(const Geometry& geo, const float* f, float* tmp, float* fs, float* g, const float* taps, int r,
                 float rho, int s_exp, DevScal* sc, hipStream_t st, int nz = 1);
void launch_init(const Geometry& geo, const float* phi0, float* P0, float* W, float* B, float* D, float mu,
                 int w0_mode, DevScal* sc, hipStream_t st, int nz = 1);
void launch_set_D(const Geometry& geo, const float* W, const float* B, float* D, float mu, hipStream_t st);
void launch_reset_scal(DevScal* sc, int n, int active, hipStream_t st);
void launch_set_k(DevScal* sc, long long k, hipStream_t st);

void launch_rhs(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                const float* D, float* out, int nz, DevScal* sc, hipStream_t st);
void launch_solve(const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out, float2* spec,
                  float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st);
// The three passes of launch_solve separately (pass 0: forward rows,
// 1: column solve, 2: inverse rows), for per-kernel timing.
void launch_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                       float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st);
// finalize = false launches the w step alone (no outer-residual finalize):
// used by the per-kernel timing.
void launch_wstep(const Geometry& geo, const KParams& kp, const float* phin, float* P0, const float* Wold,
                  const float* Bold, const float* g, float* Wnew, float* Bnew, float* D, double* part,
                  double* rhist, int nz, DevScal* sc, hipStream_t st, bool finalize = true);
void launch_energy(const Geometry& geo, const KParams& kp, const float* phi, const float* g, double* part,
                   int nz, DevScal* sc, hipStream_t st);
void launch_repulsion(const Geometry& geo, const KParams& kp, const float* phi, const float* W, float* V,
                      hipStream_t st);

}  // namespace sr
