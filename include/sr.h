/*
 * sr.h - C ABI of the MI355X (gfx950) Split Bregman solver for the
 * Self-repelling Snake (SR) model of Pan et al., "Using the Split Bregman
 * Algorithm to Solve the Self-repelling Snake Model" (arXiv:2003.12693).
 *
 * The library minimises the SR energy (eqs 7-10) under |grad phi| = 1 (eq 13)
 * by Algorithm 1 of the paper: an outer loop k over
 *   - S semi-implicit FFT steps of the phi sub-problem (eqs 30-33, 37),
 *   - soft thresholding of the auxiliary gradient variable w (eqs 41-42)
 *     followed by its projection onto |w| = 1 (eq 40),
 *   - the Bregman update of b (eq 23).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids are M x N, M rows by N columns, row-major, pitch N, float32.
 *    Row index i is the first gradient component, column index j the second
 *    (eq 35).  M and N must be powers of two in [8, 4096].
 *  - Vector fields (w, b, the repulsion field v) are two planes [2][M][N]
 *    (component 1 first), i.e. 2*M*N floats.
 *  - Boundaries are periodic for every operator (the symbol of eq 32 is the
 *    periodic five-point Laplacian's) unless sr_params.bc selects the
 *    Neumann condition of eqs (17) and (27).
 *  - Pointers are device pointers unless the call takes `flags` and
 *    SR_HOST is set, in which case they are host pointers and the call
 *    stages through the workspace and synchronises the stream.
 *  - The library never allocates device memory.  The caller asks for a
 *    workspace size, allocates it (any 256-byte aligned device buffer) and
 *    passes it in; the caller owns it and every in/out buffer, and keeps the
 *    workspace alive until sr_destroy.  The context itself is a small host
 *    object owned by the library.
 *  - Every call enqueues its GPU work on the stream given to sr_create (a
 *    hipStream_t passed as void*; NULL means the default stream).  Calls that
 *    return host values (sr_step info, sr_energy, SR_HOST copies) synchronise
 *    that stream before returning.
 *  - Return codes: 0 = SR_OK; > 0 warning; < 0 error.  Arguments are
 *    validated before any HIP call; on error nothing is enqueued and
 *    sr_last_error() returns a thread-local description.
 */
#ifndef SR_H_
#define SR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SR_OK               0
#define SR_NOT_CONVERGED    1   /* warning: iteration cap reached before tol_outer */
#define SR_EINVAL          -1   /* bad argument (null pointer, bad parameter) */
#define SR_EUNSUPPORTED    -2   /* size not a power of two in [8, 4096], R > 8 ... */
#define SR_EWORKSPACE      -3   /* workspace too small or misaligned */
#define SR_EHIP            -4   /* a HIP runtime call failed */
#define SR_ENONFINITE      -5   /* NaN / Inf in an input or in the iterate */
#define SR_ESTATE          -6   /* call out of order (e.g. sr_step before sr_set_image) */

/* ---- flags ----------------------------------------------------------- */
#define SR_HOST            1u   /* pointer arguments are host memory */

/* ---- parameters -------------------------------------------------------
 * Names follow the paper.  sr_params_default fills the parameter set of the
 * paper's two-circles experiment (alpha = gamma = 4, beta = 0.2, mu = 8,
 * tau = 0.1, l = 1, d = 5, S = 3) with eps = 1.5, R = 3, sigma = 1.5,
 * rho = 1000, s = 2, zero_tol = 1e-3.                                     */
typedef struct sr_params {
    uint32_t struct_size;  /* sizeof(sr_params), for ABI versioning         */
    double gamma;          /* weight of the geodesic length E_g (eq 7)       */
    double alpha;          /* weight of the balloon / area term E_a (eq 7)   */
    double beta;           /* weight of the repulsion E_r (eq 7)             */
    double mu;             /* splitting penalty (eq 22) and implicit weight (eq 30) */
    double tau;            /* time step of the semi-implicit scheme (eq 30)  */
    double eps;            /* half-width of H_eps, delta_eps (eqs 5-6)       */
    double band_l;         /* narrow-band half-width l of h_eps (eq 11)      */
    double d;              /* Gaussian scale of the repulsion kernel (eq 10) */
    int32_t R;             /* repulsion window half-width: (2R+1)^2 taps, 0..8 */
    double sigma;          /* pre-smoothing std of G_sigma in g (eq 1), 0..5 */
    double rho;            /* scaling of |grad| in g (eq 1)                  */
    int32_t s_exp;         /* exponent s of g (eq 1): 1 or 2                 */
    int32_t S;             /* inner phi steps per outer iteration (eq 37), 1..64 */
    double tol_inner;      /* inner stop: ||dphi|| / (||phi|| + 1e-6) <= tol; 0 = always S */
    double tol_outer;      /* outer stop on the relative phi change r_k; 0 = never */
    int32_t min_iter;      /* no outer stop before this many iterations      */
    int32_t check_every;   /* outer stop checked every this many iterations (>= 1) */
    int32_t w0_mode;       /* 0: w^0 = grad phi^0 (Algorithm 1), 1: w^0 = 0 (eq 23's text) */
    double zero_tol;       /* |B| <= zero_tol is the zero vector of eq (42) (its
                              0 (0/|0|) = 0 rule at rounding level); 0 = literal */
    int32_t w_solver;      /* 0: w by soft thresholding, eqs (41)-(42), then eq (40);
                              1: by the fixed-point iteration of eqs (38)-(39), each
                              sweep projected by eq (40) (same zero rule)        */
    int32_t w_sweeps;      /* sweeps of that iteration, 1..16 (the paper's r = 0..R,
                              R = w_sweeps - 1); ignored when w_solver = 0       */
    int32_t phi_solver;    /* 0: FFT solve of the phi sub-problem (eqs 30-33);
                              1: AOS with constant A_l (end of Sec. 4; eqs 18, 20):
                              phi = (v_1 + v_2) / 2, (1 - 2 tau mu D_l) v_l = F per
                              direction.  AOS needs tol_inner = 0, and M, N large
                              enough for the inverse's entries to fall below 1e-9
                              of the centre within +-64 (SR_EUNSUPPORTED otherwise) */
    int32_t bc;            /* boundaries.  0: periodic (every stencil, the Gaussian
                              and the window wrap; the FFT symbol of eq 32).
                              1: Neumann, the zero normal derivative of eqs (17)
                              and (27): mirror ghost values (the edge sample
                              repeated) for every stencil, the Gaussian and the
                              repulsion window, the forward difference zero on
                              the last row / column, the divergence its negative
                              adjoint.  The phi solve is then the DCT-II one
                              (phi_solver = 0: eigenvalues 1 + tau mu (4 -
                              2 cos(pi l1/M) - 2 cos(pi l2/N)), every size, the
                              inner stop rule allowed; sr_implicit_solve
                              follows it) or AOS with the Neumann tridiagonal
                              systems (phi_solver = 1)                          */
} sr_params;

/* Per-call report of sr_step. */
typedef struct sr_step_info {
    int64_t iters_done;    /* outer iterations run by this call              */
    int64_t k;             /* total outer iterations since sr_set_image/state */
    double r_last;         /* r_k = ||phi^{k+1}-phi^k||_F / (||phi^k||_F + 1e-6) of the last iteration */
    int64_t inner_steps;   /* inner steps executed by this call (S per iteration unless tol_inner > 0) */
    int32_t converged;     /* 1 if r_k < tol_outer stopped the call          */
    int32_t reserved;
} sr_step_info;

typedef struct sr_ctx sr_ctx;

/* Fill *p with the defaults above (struct_size included).  SR_EINVAL on NULL. */
int sr_params_default(sr_params* p);

/* Bytes of device workspace a context of this size needs (256-byte aligned
 * base required).  Validates M, N and *p exactly as sr_create does. */
int sr_workspace_size(int32_t M, int32_t N, const sr_params* p, size_t* bytes);

/* Create a context.  `workspace` is a device buffer of at least
 * sr_workspace_size bytes, `hip_stream` a hipStream_t (NULL: default stream).
 * Builds the FP64-computed twiddle / cosine / tap tables and uploads them
 * into the workspace.  *out receives the context (free with sr_destroy). */
int sr_create(sr_ctx** out, int32_t M, int32_t N, const sr_params* p,
              void* workspace, size_t bytes, void* hip_stream);

/* Load an image and an initial level set (Algorithm 1, "Initialize"):
 * g = 1 / (1 + rho |grad(G_sigma * f)|^s) (eq 1); phi = phi0 (a signed
 * distance function, negative inside the contour, eqs 2-3);
 * w^0 = grad phi^0 (forward differences, eq 35) or 0 (w0_mode); b^0 = 0;
 * k = 0.  f and phi0 are M*N floats.  Synchronises; SR_ENONFINITE if f or
 * phi0 holds NaN/Inf. */
int sr_set_image(sr_ctx* ctx, const float* f, const float* phi0, uint32_t flags);

/* Run up to n_iter outer iterations of Algorithm 1.  If tol_outer > 0 the
 * relative change r_k is read back every check_every iterations and the
 * call stops once r_k < tol_outer and k >= min_iter (returns SR_OK with
 * info->converged = 1), else returns SR_NOT_CONVERGED after n_iter.  With
 * tol_outer = 0 it runs exactly n_iter iterations and returns SR_OK.
 * `info` may be NULL; if given, the call synchronises to fill it.
 * SR_ENONFINITE if the iterate became non-finite. */
int sr_step(sr_ctx* ctx, int32_t n_iter, sr_step_info* info);

/* Copy the current phi (M*N floats) out. */
int sr_get_phi(sr_ctx* ctx, float* phi_out, uint32_t flags);

/* Copy the edge map g (M*N floats) computed by sr_set_image out. */
int sr_get_g(sr_ctx* ctx, float* g_out, uint32_t flags);

/* SR energy of the current phi, eqs (7)-(10), with the forward-difference
 * gradient, unit cell area and the repulsion integral truncated to the same
 * (2R+1)^2 window as the solver:
 *   terms[0] = gamma * sum g |grad phi| delta_eps(phi)
 *   terms[1] = alpha * sum g (1 - H_eps(phi))
 *   terms[2] = -beta * sum (grad phi h)(x) . sum_y K(x-y) (grad phi h)(y)
 * accumulated in double.  `terms` may be NULL.  Synchronises. */
int sr_energy(sr_ctx* ctx, double* E_total, double terms[3]);

/* Checkpoint / teacher forcing: copy (phi, w, b) and k out, or in.  phi is
 * M*N floats, w and b are 2*M*N floats each.  sr_set_state also rebuilds the
 * per-iteration constant mu div(b - w).  Requires sr_set_image first (for g). */
int sr_get_state(sr_ctx* ctx, float* phi, float* w, float* b, int64_t* k, uint32_t flags);
int sr_set_state(sr_ctx* ctx, const float* phi, const float* w, const float* b, int64_t k,
                 uint32_t flags);

/* ---- component operators (the steps of one iteration, on caller data) ----
 * They use the context's sizes, parameters, tables and scratch buffers and
 * leave the solver state (phi, w, b, g) untouched. */

/* g of eq (1) for image f: periodic Gaussian (taps exp(-t^2/(2 sigma^2)),
 * |t| <= ceil(3 sigma), normalised), central differences, then
 * 1 / (1 + rho |grad|^s). */
int sr_edge_map(sr_ctx* ctx, const float* f, float* g_out, uint32_t flags);

/* Repulsion window sum (the discrete v of Sec. 4, after eq 37):
 * v[i,j] = sum_{|p|,|q|<=R} exp(-(p^2+q^2)/d^2) w[i+p,j+q] h_eps(phi[i+p,j+q]),
 * periodic.  w and v_out are 2*M*N floats, phi M*N floats. */
int sr_repulsion(sr_ctx* ctx, const float* w, const float* phi, float* v_out, uint32_t flags);

/* Semi-implicit solve of eqs (31)-(33): u = Re F^{-1}( F(rhs) / (1 - tau mu
 * (2 cos z1 + 2 cos z2 - 4)) ), i.e. (1 - tau mu Lap) u = rhs on the periodic
 * grid, through the library's LDS-staged Stockham FFTs (radix 16/8/4/2);
 * with bc = 1 the same solve for the mirrored Laplacian through DCT-II
 * passes built on those FFTs. */
int sr_implicit_solve(sr_ctx* ctx, const float* rhs, float* u_out, uint32_t flags);

/* The solve of sr_implicit_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): no context, no workspace.  u_out = the solution of
 * (1 - tau mu Lap) u = rhs on the periodic M x N grid (eqs 31-33), rhs and
 * u_out device pointers to M*N floats (they may not overlap), enqueued on
 * hip_stream (NULL: the default stream); returns without synchronising.
 * The half spectrum, the twiddle tables (built on the device) and the FFT
 * kernels' flags live in one fixed array of the library's (16.5 MiB per
 * device, held until the process ends): M and N powers of two in
 * [8, 4096] with M * N <= 4194304, else SR_EUNSUPPORTED.  Every call on a
 * device uses that device's one array, so calls that overlap in time on
 * one device (different streams or threads) race and must be serialised by
 * the caller.  SR_EINVAL on NULL pointers or tau, mu <= 0; SR_EHIP if a
 * launch fails.  Calls no allocating routine. */
int sr_implicit_solve_noalloc(int32_t M, int32_t N, double tau, double mu, const float* rhs, float* u_out,
                              void* hip_stream);

/* ---- measurement -------------------------------------------------------
 * Per-kernel timing of the iteration: runs n_iter outer iterations from the
 * current state (the iterate advances exactly as under sr_step(ctx, n_iter),
 * bitwise), launched directly on the context's stream instead of through a
 * graph, each iteration kernel with its own start / stop hipEvents recorded
 * at the kernel's own start and end (hipExtLaunchKernel), so every launch is
 * timed in the cache state the iteration gives it.  Reports the average
 * duration of a launch of each kind in milliseconds:
 *   ms[0] rhs + repulsion window (eq 37)   ms[1] forward row FFT
 *   ms[2] column FFT solve (eqs 31-33)     ms[3] inverse row FFT + update
 *   ms[4] w / b step (eqs 40-42, 23)
 * Where the right-hand side is fused with the forward row FFT (FFT phi
 * solve, periodic boundaries, 64 <= N <= 1024) that one launch is timed as
 * kind 0 and kind 1 reports count 0.
 * count[i] receives the number of launches timed (n_iter S for the first
 * four kinds, n_iter for the w step, n_iter w_sweeps with the fixed-point
 * w solver, whose intermediate sweeps count as w-step launches).  With the
 * AOS phi solver its one launch per inner step is timed as ms[2] and the
 * FFT kinds 1 and 3 are not launched (count 0).
 * Synchronises; ignores tol_outer.
 * Returns SR_EINVAL for n_iter < 1, SR_ESTATE before sr_set_image. */
#define SR_NUM_KERNEL_KINDS 5
int sr_profile_kernels(sr_ctx* ctx, int32_t n_iter, double ms[SR_NUM_KERNEL_KINDS],
                       int64_t count[SR_NUM_KERNEL_KINDS]);

/* ---- autotuner ----------------------------------------------------------
 * Chooses the row height of the stencil tiles (8, 16 or 32 rows of 64
 * columns) of the right-hand-side window kernel (eq 37), launched S times
 * per outer iteration (the w step, eqs 40-42, always takes 16-row tiles,
 * its fastest at every measured size).  Each candidate is timed on the
 * context's current state by
 * launching the right-hand-side kernel, which reads the state and writes
 * only its own scratch plane, so the iterate is unchanged and so is every
 * later result (the per-pixel arithmetic does not depend on the tile
 * height).  The fastest is kept (16 rows unless another is at least 3%
 * faster, so that near ties give one choice) for the context and recorded process-wide
 * for its size class (M, N, R); sr_create and every size-class group of
 * sr_solve_batch take a recorded choice, and sr_solve_batch tunes classes
 * it has not seen.  reps >= 1 timed launches per candidate after one warm-
 * up; us_out (nullable, host) receives the mean duration of each candidate
 * in microseconds, *tile_th (nullable) the choice.  Requires sr_set_image;
 * synchronises; SR_EINVAL / SR_ESTATE / SR_EHIP on error. */
int sr_autotune(sr_ctx* ctx, int32_t reps, int32_t* tile_th, double us_out[3]);

/* ---- launch preparation -------------------------------------------------
 * sr_step replays HIP graphs of 1, 2, 4, 8 and 16 outer iterations (one
 * set per parity of the phi / w / b ping-pong; n iterations are split into powers
 * of two, largest first), capturing each the first time it is needed.
 * sr_prepare captures and instantiates all ten now, without
 * running any kernel or changing the state, so that a later sr_step spends
 * no time on capture (e.g. before a timed region).  sr_autotune drops the
 * graphs when it changes the tile height; call sr_prepare after it.
 * SR_EINVAL on NULL, SR_EHIP if capture or instantiation fails. */
int sr_prepare(sr_ctx* ctx);

/* Identity of the compiled sources: a hex digest of the HIP sources and
 * headers the library was built from (set by the build script), or
 * "unknown".  The string is static; never NULL. */
const char* sr_build_id(void);

/* ---- batched solve (many independent images of uneven sizes) ----------
 * Each item is solved by Algorithm 1 from its own f and phi0, with its own
 * params (R may differ per item), until r_k < tol_outer (after min_iter) or
 * max_iter.  Items with equal (M, N, params) are grouped and advanced
 * together in single launches (one grid slice per instance); converged
 * instances drop out of further work.  All pointers are device pointers.
 * The workspace size comes from sr_batch_workspace_size for the same items. */
typedef struct sr_batch_item {
    int32_t M, N;
    const float* f;        /* in:  image, M*N floats (device)              */
    const float* phi0;     /* in:  initial level set, M*N floats (device)  */
    float* phi_out;        /* out: final phi, M*N floats (device)          */
    sr_params params;      /* per-item parameters (tol_outer, min_iter, check_every used) */
    int32_t max_iter;      /* iteration cap                                 */
    /* outputs */
    int32_t iters;         /* iterations run                                */
    int32_t status;        /* SR_OK, SR_NOT_CONVERGED or SR_ENONFINITE      */
    int32_t reserved;
    double r_last;         /* last relative phi change                      */
    double energy;         /* final SR energy (eq 7)                        */
    float* w_out;          /* out, nullable: final w, 2*M*N floats (device)  */
    float* b_out;          /* out, nullable: final b, 2*M*N floats (device)  */
} sr_batch_item;

int sr_batch_workspace_size(const sr_batch_item* items, int32_t n, size_t* bytes);
int sr_solve_batch(sr_batch_item* items, int32_t n, void* workspace, size_t bytes,
                   void* hip_stream);

/* Release the context (not the caller's workspace).  NULL is a no-op. */
void sr_destroy(sr_ctx* ctx);

/* Thread-local message describing the last error ("" if none). */
const char* sr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SR_H_ */
