/* C ABI of the 3-D Split Bregman solver of the Self-repelling Snake model
 * (the paper's volume application, Sec. 5, Fig. 6: the 2-D method with a
 * third axis -- 3-component w and b, seven-point Laplacian, cube Gaussian
 * (eq 1) and cube repulsion window (weights exp(-(p^2+q^2+r^2)/d^2)), the
 * 3-D FFT solve of eqs 30-33 and 37, soft thresholding and projection of
 * 3-vectors (eqs 40-42), the Bregman update (eq 23)).  Periodic boundaries.
 *
 * Volumes are M x N x P float32, C order (index (i*N + j)*P + k), all of
 * M, N, P powers of two in [8, 256].  w and b are 3 such volumes back to
 * back (component along i, then j, then k).  Every pointer argument is a
 * device pointer; the library launches on the caller's stream and never
 * allocates device memory (the caller's workspace holds every buffer).
 * Return codes are those of sr.h (SR_OK, SR_EINVAL, SR_EUNSUPPORTED,
 * SR_ESTATE, SR_EHIP); sr_last_error() describes the last failure. */
#ifndef SR3D_H
#define SR3D_H

#include <stddef.h>
#include <stdint.h>

#include "sr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sr3_ctx sr3_ctx;

/* Workspace bytes for an M x N x P volume.  Uses gamma, alpha, beta, mu, tau,
 * eps, band_l, d, R, sigma, rho, s_exp, S, zero_tol of p; needs tol_inner = 0,
 * w_solver = 0, phi_solver = 0, bc = 0 (SR_EUNSUPPORTED otherwise). */
int sr3_workspace_size(int32_t M, int32_t N, int32_t P, const sr_params* p, size_t* bytes);

/* Context on `workspace` (device memory of sr3_workspace_size bytes, owned
 * by the caller, 256-byte aligned) and `hip_stream` (a hipStream_t, or NULL
 * for the default stream). */
int sr3_create(sr3_ctx** out, int32_t M, int32_t N, int32_t P, const sr_params* p, void* workspace,
               size_t bytes, void* hip_stream);

/* g from f (eq 1, cube Gaussian, central differences); phi^0 = phi0,
 * w^0 = grad phi^0 (forward differences), b^0 = 0, k = 0. */
int sr3_set_image(sr3_ctx* ctx, const float* f, const float* phi0);

/* State (phi, w, b) from the caller; k counts on from k. */
int sr3_set_state(sr3_ctx* ctx, const float* phi, const float* w, const float* b, int64_t k);

/* n_iter >= 1 outer iterations of Algorithm 1 (S inner steps each);
 * synchronises; *k_out (nullable) receives the total iteration count. */
int sr3_step(sr3_ctx* ctx, int32_t n_iter, int64_t* k_out);

/* Copies of phi, w (3 volumes), b (3 volumes) and g; any pointer may be NULL. */
int sr3_get_state(sr3_ctx* ctx, float* phi, float* w, float* b, float* g);

/* Per-kernel-kind average duration (ms) over n_iter further iterations,
 * each kernel launch timed with its own events: [0] the three window
 * passes (the first forms u = w h(phi)), [1] right-hand side with the
 * forward k transform, [2] the other FFT passes (four per solve), [3] w
 * step; count[] the launches per kind.  Synchronises. */
int sr3_profile(sr3_ctx* ctx, int32_t n_iter, double ms[4], int64_t count[4]);

void sr3_destroy(sr3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
