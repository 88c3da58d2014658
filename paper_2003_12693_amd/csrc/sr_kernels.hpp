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
    const float2* twM;      // W_M^n, n < M (FP64-computed, rounded)
    const float2* twN;      // W_N^n, n < N
    const float2* stM;      // stage twiddle table of the column transforms (length M)
    const float2* stN;      // stage twiddle table of the row transforms (length N)
    float taumu;
    int tile_th = 0;   // stencil tile height (16 or 32); 0 = size heuristic
    int bc = 0;        // boundaries: 0 periodic, 1 Neumann (mirror ghosts)
    // Neumann (DCT-II) solve: exp(-i pi k / (2L)) for k < L, and 2 cos(pi k / L)
    const float2* dtM = nullptr;
    const float2* dtN = nullptr;
    const float* cM = nullptr;
    const float* cN = nullptr;
};

int tile_blocks(int M, int N);
// Stage twiddle tables of the FFT passes: float2 entries, and the host-side
// construction (col: the column pass's table for length L, else the row passes').
int fft_stage_table_len(int L, bool col);
// Elements per thread of those transforms (their stage radices follow from it).
int fft_elems(int L, bool col);
// While set (non-null) on the calling host thread, the iteration kernels
// (rhs, the three FFT passes, w step) are launched with these events, which
// record the kernel's own start and end; set both to nullptr to stop.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
void fft_stage_table(int L, bool col, float2* out);

void launch_edge(const Geometry& geo, const float* f, float* tmp, float* fs, float* g, const float* taps, int r,
                 float rho, int s_exp, DevScal* sc, hipStream_t st, int nz = 1);
void launch_init(const Geometry& geo, const float* phi0, float* P0, float* W, float* B, float* D, float mu,
                 int w0_mode, DevScal* sc, hipStream_t st, int nz = 1);
void launch_set_D(const Geometry& geo, const float* W, const float* B, float* D, float mu, hipStream_t st);
void launch_reset_scal(DevScal* sc, int n, int active, hipStream_t st);
void launch_set_k(DevScal* sc, long long k, hipStream_t st);

// The outer-iteration finalize (residual r_k, iteration count, retirement)
// of the preceding w step, folded into a right-hand-side launch: its first
// workgroup of each instance runs it before its own tile.  Only valid while
// the inner stop rule is off (tol_inner = 0), since the other workgroups of
// that launch may read the instance's flags before the finalize updates them.
struct FinFold {
    const double* part;   // the w step's residual partials
    int nb;               // their count per instance (wstep_blocks)
    double* rhist;
};
void launch_rhs(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                const float* D, float* out, int nz, DevScal* sc, hipStream_t st, const FinFold* fold = nullptr);
// The right-hand side of eq (37) fused with the forward row FFT of its
// solve: writes the half spectrum of the rhs into spec (as pass 0 of
// launch_solve_pass would from the rhs plane).  Only where
// fused_rhs_supported (periodic, 64 <= N <= 1024).
bool fused_rhs_supported(const Geometry& geo, const KParams& kp);
void configure_fused();   // dynamic LDS limits of the fused kernels (once per process)
void launch_rhs_fwd(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                    const float* D, float2* spec, int nz, DevScal* sc, hipStream_t st, const FinFold* fold = nullptr);
// Pass `pass` (0..2) of the Neumann solve (phi_out = phi_in + u, phi_in
// nullable, with (1 - tau mu Lap) u = rhs for the mirrored Laplacian): the
// DCT-II passes of sr_dct.hip, same shapes and spectrum layout as the
// periodic passes.  launch_solve_pass calls it when geo.bc = 1.
void launch_dct_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                           float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st);
void configure_dct();
// Shapes of the FFT passes: log2 rows per workgroup of the row passes, and
// columns per workgroup of the column pass.
int fft_row_split(int M, int N, int nz, int min_wg, int min_lr);
int fft_col_group(int M, int N, int nz);
// The inner stop rule's finalize after an inverse row pass's partial sums.
void launch_fin_inner(const double* part, int nb, float tol, int nz, DevScal* sc, hipStream_t st);
void launch_solve(const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out, float2* spec,
                  float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st);
// The three passes of launch_solve separately (pass 0: forward rows,
// 1: column solve, 2: inverse rows), for per-kernel timing.
void launch_solve_pass(int pass, const Geometry& geo, const float* rhs, const float* phi_in, float* phi_out,
                       float2* spec, float tol_inner, double* part, int nz, DevScal* sc, hipStream_t st);
// finalize = false leaves the outer-iteration finalize to a FinFold in the
// next right-hand-side launch.  sweep = true: one sweep of the fixed-point w
// solver only, w from Wold into Wnew (Bnew, D, part, rhist unused; no
// finalize).  phin is phi^{k+1}, Pk phi^k (read for the outer residual only).
void launch_wstep(const Geometry& geo, const KParams& kp, const float* phin, const float* Pk, const float* Wold,
                  const float* Bold, const float* g, float* Wnew, float* Bnew, float* D, double* part,
                  double* rhist, int nz, DevScal* sc, hipStream_t st, bool finalize = true, bool sweep = false);
// Residual partials per instance written by launch_wstep.
int wstep_blocks(const Geometry& geo, int nz);
void launch_energy(const Geometry& geo, const KParams& kp, const float* phi, const float* g, double* part,
                   int nz, DevScal* sc, hipStream_t st);
void launch_repulsion(const Geometry& geo, const KParams& kp, const float* phi, const float* W, float* V,
                      hipStream_t st);

}  // namespace sr
