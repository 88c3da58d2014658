// Host runtime of the SR Split Bregman library: argument validation,
// workspace carving, FP64 table construction, the per-iteration launch
// sequence (captured once into HIP graphs and replayed) and the C ABI of
// include/sr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sr.h"
#include "sr_aos.hpp"
#include "sr_device.hpp"
#include "sr_kernels.hpp"

namespace sr {
void configure_kernels();
}

using sr::DevScal;
using sr::Geometry;
using sr::KParams;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// The error text of the 3-D entry points (sr3d.hip) goes to the same
// thread-local string that sr_last_error() returns.
namespace sr {
int api_fail(int code, const char* msg) {
    g_err = msg;
    return code;
}
}  // namespace sr

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(SR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// autotuner of the stencil tile height, with a process-wide record per size
// class (M, N, R, batch depth)
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, int> g_tuned;
static const int kTileHeights[3] = {8, 16, 32};

static int tuned_tile_height(int M, int N, int R, int nz) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(M, N, R, nz));
    return it == g_tuned.end() ? 0 : it->second;
}

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

static int validate(int32_t M, int32_t N, const sr_params* p) {
    if (!p) return fail(SR_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(sr_params))
        return fail(SR_EINVAL, "params.struct_size %u != %zu (call sr_params_default)", p->struct_size,
                    sizeof(sr_params));
    if (!is_pow2(M) || !is_pow2(N) || M < 8 || N < 8 || M > 4096 || N > 4096)
        return fail(SR_EUNSUPPORTED, "M, N must be powers of two in [8, 4096] (got %d x %d)", M, N);
    const double v[] = {p->gamma, p->alpha, p->beta, p->mu, p->tau, p->eps, p->band_l, p->d,
                        p->sigma, p->rho, p->tol_inner, p->tol_outer, p->zero_tol};
    for (double x : v)
        if (!std::isfinite(x)) return fail(SR_EINVAL, "non-finite parameter");
    if (p->tau <= 0) return fail(SR_EINVAL, "tau must be > 0");
    if (p->mu <= 0) return fail(SR_EINVAL, "mu must be > 0 (it divides beta and gamma in eqs 41-42)");
    if (p->eps <= 0) return fail(SR_EINVAL, "eps must be > 0");
    if (p->band_l < 0) return fail(SR_EINVAL, "band_l must be >= 0");
    if (p->d <= 0) return fail(SR_EINVAL, "d must be > 0");
    if (p->R < 0 || p->R > sr::kMaxR) return fail(SR_EUNSUPPORTED, "R must be in [0, %d]", sr::kMaxR);
    if (p->sigma < 0 || std::ceil(3.0 * p->sigma) > sr::kMaxGaussR)
        return fail(SR_EUNSUPPORTED, "sigma must be in [0, %g]", sr::kMaxGaussR / 3.0);
    if (p->rho < 0) return fail(SR_EINVAL, "rho must be >= 0");
    if (p->s_exp != 1 && p->s_exp != 2) return fail(SR_EINVAL, "s_exp must be 1 or 2");
    if (p->S < 1 || p->S > 64) return fail(SR_EINVAL, "S must be in [1, 64]");
    if (p->tol_inner < 0 || p->tol_outer < 0) return fail(SR_EINVAL, "tolerances must be >= 0");
    if (p->check_every < 1) return fail(SR_EINVAL, "check_every must be >= 1");
    if (p->min_iter < 0) return fail(SR_EINVAL, "min_iter must be >= 0");
    if (p->w0_mode != 0 && p->w0_mode != 1) return fail(SR_EINVAL, "w0_mode must be 0 or 1");
    if (p->zero_tol < 0) return fail(SR_EINVAL, "zero_tol must be >= 0");
    if (p->w_solver != 0 && p->w_solver != 1) return fail(SR_EINVAL, "w_solver must be 0 or 1");
    if (p->w_sweeps < 1 || p->w_sweeps > 16) return fail(SR_EINVAL, "w_sweeps must be in [1, 16]");
    if (p->phi_solver != 0 && p->phi_solver != 1) return fail(SR_EINVAL, "phi_solver must be 0 or 1");
    if (p->bc != 0 && p->bc != 1) return fail(SR_EINVAL, "bc must be 0 (periodic) or 1 (Neumann)");
    if (p->phi_solver == 1) {
        if (p->tol_inner > 0) return fail(SR_EUNSUPPORTED, "the AOS phi solver runs a fixed S (tol_inner = 0)");
        std::vector<float> taps(sr::kAosTapFloats);
        int kx, ky;
        if (sr::aos_tap_buffer(M, N, p->tau, p->mu, p->bc, taps.data(), &kx, &ky) < 0)
            return fail(SR_EUNSUPPORTED, "AOS: the inverse of (1 - 2 tau mu D) on %d or %d points does not decay "
                        "below 1e-9 within +-%d", M, N, sr::kAosMaxK);
    }
    return SR_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t twM, twN, stM, stN, dtM, dtN, cM, cN, aos, g, P0, P1, P2, W0, W1, B0, B1, D, Rb, spec, part, scal, rhist;
    size_t X0, X1;
    size_t total;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// w buffers of the intermediate sweeps of the fixed-point w solver.
static int sweep_buffers(const sr_params& p) {
    return p.w_solver == 1 ? std::min(2, p.w_sweeps - 1) : 0;
}

// nz instances of one size class laid out plane-by-plane ([nz][M][N] each).
static Layout make_layout(int M, int N, int nz, int xbufs = 0) {
    Layout L{};
    const size_t MN = (size_t)M * N, pl = MN * 4 * nz, vec = 2 * pl;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.twM = take(sizeof(float2) * M);
    L.twN = take(sizeof(float2) * N);
    L.stM = take(sizeof(float2) * sr::fft_stage_table_len(M, true));
    L.stN = take(sizeof(float2) * sr::fft_stage_table_len(N, false));
    L.dtM = take(sizeof(float2) * M);
    L.dtN = take(sizeof(float2) * N);
    L.cM = take(sizeof(float) * M);
    L.cN = take(sizeof(float) * N);
    L.aos = take(sizeof(float) * sr::kAosTapFloats);
    L.g = take(pl);
    L.P0 = take(pl);
    L.P1 = take(pl);
    L.P2 = take(pl);
    L.W0 = take(vec);
    L.W1 = take(vec);
    L.B0 = take(vec);
    L.B1 = take(vec);
    L.D = take(pl);
    L.Rb = take(pl);
    L.spec = take(pl);
    const int nb = std::max(sr::tile_blocks(M, N), M);
    L.part = take(sizeof(double) * 3 * (size_t)nb * nz);
    L.scal = take(sizeof(DevScal) * nz);
    L.rhist = take(sizeof(double) * sr::kRHist * nz);
    L.X0 = xbufs > 0 ? take(vec) : 0;
    L.X1 = xbufs > 1 ? take(vec) : 0;
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Bufs {
    float2 *twM, *twN, *stM, *stN, *dtM, *dtN;
    float *cM, *cN;
    float* aos;    // AOS tap buffer (sr::aos_tap_buffer layout)
    float *g, *W[2], *B[2], *D, *Rb;
    // phi^k in Ph[parity]: the last inner step of an outer iteration writes
    // phi^{k+1} into Ph[parity ^ 1] (no copy back); Ph[2] is the spare inner
    // iterate
    float* Ph[3];
    float2* spec;
    double* part;
    DevScal* scal;
    double* rhist;
    float* X[2];   // intermediate w of the fixed-point sweeps (when allocated)
};

constexpr int kGraphLevels = 5;   // graphs of 1, 2, 4, 8 and 16 iterations

struct sr_ctx {
    int M, N, nz;
    sr_params p;
    KParams kp;
    Geometry geo;
    Bufs b;
    hipStream_t stream;
    hipStream_t cap;           // capture stream (graphs are replayed on `stream`)
    // graphs of 2^j outer iterations (j = 0..kGraphLevels-1) from parity p
    hipGraphExec_t gr[kGraphLevels][2] = {};
    DevScal* hscal = nullptr;  // pinned host copy of the scalar block (read back after every sr_step)
    bool use_graphs = true;
    bool fused = false;        // rhs fused with the forward row FFT (sr::fused_rhs_supported)
    int parity = 0;            // state in Ph[parity], W[parity], B[parity]
    long long k = 0;
    bool image_set = false;
    int aosKx = 0, aosKy = 0;  // AOS truncation radii (phi_solver = 1)
    std::vector<float> gauss;  // Gaussian taps
    int gauss_r = 0;
};

// phi^k of the current state, and the phi planes that hold no state (host
// staging for the component operators): i = 0 the other half of the pair,
// i = 1 the spare.
static float* phi_state(sr_ctx* c) { return c->b.Ph[c->parity]; }
static float* phi_free(sr_ctx* c, int i) { return i == 0 ? c->b.Ph[c->parity ^ 1] : c->b.Ph[2]; }

static void carve(Bufs& b, char* base, const Layout& L) {
    b.twM = (float2*)(base + L.twM);
    b.twN = (float2*)(base + L.twN);
    b.stM = (float2*)(base + L.stM);
    b.stN = (float2*)(base + L.stN);
    b.dtM = (float2*)(base + L.dtM);
    b.dtN = (float2*)(base + L.dtN);
    b.cM = (float*)(base + L.cM);
    b.cN = (float*)(base + L.cN);
    b.aos = (float*)(base + L.aos);
    b.g = (float*)(base + L.g);
    b.Ph[0] = (float*)(base + L.P0);
    b.Ph[1] = (float*)(base + L.P1);
    b.Ph[2] = (float*)(base + L.P2);
    b.W[0] = (float*)(base + L.W0);
    b.W[1] = (float*)(base + L.W1);
    b.B[0] = (float*)(base + L.B0);
    b.B[1] = (float*)(base + L.B1);
    b.D = (float*)(base + L.D);
    b.Rb = (float*)(base + L.Rb);
    b.spec = (float2*)(base + L.spec);
    b.part = (double*)(base + L.part);
    b.scal = (DevScal*)(base + L.scal);
    b.rhist = (double*)(base + L.rhist);
    b.X[0] = L.X0 ? (float*)(base + L.X0) : nullptr;
    b.X[1] = L.X1 ? (float*)(base + L.X1) : nullptr;
}

// The fused right-hand-side + row FFT kernel replaces the rhs kernel and the
// forward row pass where it exists (FFT phi solve, periodic, 64 <= N <= 1024);
// SR_NO_FUSE=1 keeps the two separate launches (for A/B measurements).
static bool use_fused(const sr_params& p, const Geometry& geo, const KParams& kp) {
    static const bool off = [] {
        const char* s = std::getenv("SR_NO_FUSE");
        return s && s[0] == '1';
    }();
    return !off && p.phi_solver == 0 && sr::fused_rhs_supported(geo, kp);
}

static void make_kparams(const sr_params& p, KParams& kp) {
    std::memset(&kp, 0, sizeof kp);
    kp.gamma = (float)p.gamma;
    kp.alpha = (float)p.alpha;
    kp.beta = (float)p.beta;
    kp.mu = (float)p.mu;
    kp.tau = (float)p.tau;
    kp.eps = (float)p.eps;
    kp.inv_eps = (float)(1.0 / p.eps);
    kp.band_l = (float)p.band_l;
    kp.c_rep = (float)(2.0 * p.beta / p.mu);
    // the fixed-point w solver (eqs 38-39) has no soft-thresholding gate:
    // after the projection its sweep is B / |B| (the positive denominator of
    // eq 39 cancels), i.e. the eq (42) gate with a zero threshold
    kp.c_thr = p.w_solver == 1 ? 0.0f : (float)(p.gamma / p.mu);
    kp.tol_inner = (float)p.tol_inner;
    kp.zero_tol = (float)p.zero_tol;
    kp.R = p.R;
    for (int q = -p.R; q <= p.R; ++q) kp.taps[q + p.R] = (float)std::exp(-(double)q * q / (p.d * p.d));
}

static void make_gauss(double sigma, std::vector<float>& k, int& r) {
    r = (int)std::ceil(3.0 * sigma);
    k.assign(2 * r + 1, 0.0f);
    if (r == 0) { k[0] = 1.0f; return; }
    std::vector<double> kd(2 * r + 1);
    double s = 0;
    for (int t = -r; t <= r; ++t) { kd[t + r] = std::exp(-(double)t * t / (2.0 * sigma * sigma)); s += kd[t + r]; }
    for (int t = 0; t <= 2 * r; ++t) k[t] = (float)(kd[t] / s);
}

static std::vector<float2> twiddles(int L) {
    std::vector<float2> t(L);
    const double two_pi = 6.283185307179586476925286766559;
    for (int n = 0; n < L; ++n) {
        const double a = two_pi * (double)n / (double)L;
        t[n] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    return t;
}

// Twiddle tables of a context (full tables for lengths M and N, stage tables
// of the column and row transforms), copied from pageable host memory.
static hipError_t upload_tables_to(float2* twM, float2* twN, float2* stM, float2* stN, int M, int N,
                                   hipStream_t st) {
    const std::vector<float2> tm = twiddles(M), tn = twiddles(N);
    std::vector<float2> sm(sr::fft_stage_table_len(M, true)), sn(sr::fft_stage_table_len(N, false));
    sr::fft_stage_table(M, true, sm.data());
    sr::fft_stage_table(N, false, sn.data());
    hipError_t e = hipMemcpyAsync(twM, tm.data(), sizeof(float2) * M, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(twN, tn.data(), sizeof(float2) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !sm.empty())
        e = hipMemcpyAsync(stM, sm.data(), sizeof(float2) * sm.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !sn.empty())
        e = hipMemcpyAsync(stN, sn.data(), sizeof(float2) * sn.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors are released on return
    return e;
}

// Tables of the Neumann (DCT-II) solve: exp(-i pi k / (2L)) and 2 cos(pi k / L), k < L.
static void dct_tables(int L, std::vector<float2>& dt, std::vector<float>& cs) {
    const double pi = 3.14159265358979323846264338327950288;
    dt.resize(L);
    cs.resize(L);
    for (int k = 0; k < L; ++k) {
        const double a = pi * (double)k / (2.0 * L);
        dt[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
        cs[k] = (float)(2.0 * std::cos(pi * (double)k / (double)L));
    }
}

static hipError_t upload_tables(const Bufs& b, int M, int N, hipStream_t st) {
    hipError_t e = upload_tables_to(b.twM, b.twN, b.stM, b.stN, M, N, st);
    std::vector<float2> dm, dn;
    std::vector<float> cm, cn;
    dct_tables(M, dm, cm);
    dct_tables(N, dn, cn);
    if (e == hipSuccess) e = hipMemcpyAsync(b.dtM, dm.data(), sizeof(float2) * M, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.dtN, dn.data(), sizeof(float2) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.cM, cm.data(), sizeof(float) * M, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.cN, cn.data(), sizeof(float) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors are released on return
    return e;
}

// AOS inverse taps of a context (phi_solver = 1), after validate() has
// checked that both directions truncate.
static hipError_t upload_aos(sr_ctx* c, hipStream_t st) {
    if (c->p.phi_solver != 1) return hipSuccess;
    std::vector<float> t(sr::kAosTapFloats);
    (void)sr::aos_tap_buffer(c->M, c->N, c->p.tau, c->p.mu, c->p.bc, t.data(), &c->aosKx, &c->aosKy);
    hipError_t e = hipMemcpyAsync(c->b.aos, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// Events of the AOS launch while sr_profile_kernels times a launch.
static thread_local hipEvent_t t_aos_ev[2] = {nullptr, nullptr};

// The launch sequence of one outer iteration from parity p (Algorithm 1):
// S x [rhs -> row FFT -> column solve -> inverse row FFT], then the w step.
// before(kind) runs ahead of each iteration kernel's launch (kinds as in
// sr_profile_kernels); the per-kernel timing uses it to arm events.
// fold_in: the first rhs launch runs the previous iteration's finalize
// (FinFold); fin_out = false: this iteration's w step leaves its finalize to
// the next iteration's first rhs.  Both only inside captured graphs and only
// with the inner stop rule off (can_fold).
struct NoHook { void operator()(int) const {} };
static bool can_fold(const sr_ctx* c) { return c->p.tol_inner <= 0.0; }
template <typename Hook = NoHook>
static void enqueue_iteration(sr_ctx* c, int p, hipStream_t st, Hook&& before = Hook{}, bool fold_in = false,
                              bool fin_out = true) {
    Bufs& b = c->b;
    const int S = c->p.S;
    // phi^k in Ph[p]; the inner iterates alternate between Ph[p ^ 1] and the
    // spare so that the last one, phi^{k+1}, lands in Ph[p ^ 1]
    const float* in = b.Ph[p];
    float* outs[2];
    outs[(S - 1) & 1] = b.Ph[p ^ 1];
    outs[S & 1] = b.Ph[2];
    const sr::FinFold fold{b.part, sr::wstep_blocks(c->geo, c->nz), b.rhist};
    for (int s = 0; s < S; ++s) {
        float* out = outs[s & 1];
        before(0);
        if (c->fused)   // rhs fused with the forward row FFT: writes the spectrum
            sr::launch_rhs_fwd(c->geo, c->kp, in, b.W[p], b.g, b.D, b.spec, c->nz, b.scal, st,
                               (fold_in && s == 0) ? &fold : nullptr);
        else
            sr::launch_rhs(c->geo, c->kp, in, b.W[p], b.g, b.D, b.Rb, c->nz, b.scal, st,
                           (fold_in && s == 0) ? &fold : nullptr);
        if (c->p.phi_solver == 1) {   // AOS: one launch, timed as the solve kind (2)
            before(2);
            sr::launch_aos(c->M, c->N, c->p.bc, b.Rb, in, out, b.aos, c->aosKx, c->aosKy,
                           c->geo.taumu, c->nz, b.scal, st, t_aos_ev[0], t_aos_ev[1]);
        } else {   // FFT solve (periodic) or DCT-II solve (Neumann), by geo.bc
            for (int pass = c->fused ? 1 : 0; pass < 3; ++pass) {
                before(1 + pass);
                sr::launch_solve_pass(pass, c->geo, b.Rb, in, out, b.spec, c->kp.tol_inner, b.part, c->nz, b.scal,
                                      st);
            }
        }
        in = out;
    }
    // fixed-point w solver: w_sweeps - 1 sweeps that write only w (into the
    // X buffers), then the full w step from the last of them
    const float* w_in = b.W[p];
    if (c->p.w_solver == 1)
        for (int r = 0; r + 1 < c->p.w_sweeps; ++r) {
            float* w_out = b.X[r & 1];
            before(4);
            sr::launch_wstep(c->geo, c->kp, in, b.Ph[p], w_in, b.B[p], b.g, w_out, nullptr, nullptr, nullptr,
                             nullptr, c->nz, b.scal, st, false, true);
            w_in = w_out;
        }
    before(4);
    sr::launch_wstep(c->geo, c->kp, in, b.Ph[p], w_in, b.B[p], b.g, b.W[1 - p], b.B[1 - p], b.D, b.part, b.rhist,
                     c->nz, b.scal, st, fin_out);
}

// iters outer iterations from parity p; inside a graph the finalize of each
// but the last is folded into the next iteration's first rhs.
static void enqueue_chunk(sr_ctx* c, int p, int iters, hipStream_t st) {
    const bool fold = can_fold(c);
    for (int i = 0; i < iters; ++i)
        enqueue_iteration(c, (p + i) & 1, st, NoHook{}, fold && i > 0, !fold || i == iters - 1);
}

static int capture(sr_ctx* c, int p, int iters, hipGraphExec_t* out) {
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    enqueue_chunk(c, p, iters, c->cap);
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (e != hipSuccess) return fail(SR_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(SR_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    // upload now, so that the first replay does not pay for it
    e = hipGraphUpload(*out, c->stream);
    if (e != hipSuccess) return fail(SR_EHIP, "graph upload: %s", hipGetErrorString(e));
    return SR_OK;
}

// Time the right-hand-side kernel for each tile height on the current state
// (it writes only the scratch plane Rb) and keep the fastest.
static int tune_tiles(sr_ctx* c, int reps, double us_out[3]) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int p = c->parity;
    Bufs& b = c->b;
    double t[3] = {0.0, 0.0, 0.0};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        c->geo.tile_th = kTileHeights[i];
        sr::launch_rhs(c->geo, c->kp, b.Ph[p], b.W[p], b.g, b.D, b.Rb, c->nz, b.scal, c->stream);
        e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            sr::launch_rhs(c->geo, c->kp, b.Ph[p], b.W[p], b.g, b.D, b.Rb, c->nz, b.scal, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[i] = 1e3 * ms / reps;
        if (us_out) us_out[i] = t[i];
    }
    // The default 16 rows unless another height is at least 3% faster: near
    // ties (1024^2) then give the same choice in every run.
    int best = 16;
    double best_us = t[1];
    for (int i = 0; i < 3; ++i)
        if (t[i] < 0.97 * t[1] && t[i] < best_us) {
            best_us = t[i];
            best = kTileHeights[i];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(SR_EHIP, "autotune: %s", hipGetErrorString(e));
    HIP_TRY(hipGetLastError());
    c->geo.tile_th = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(c->M, c->N, c->kp.R, c->nz)] = best;
    return SR_OK;
}

static void drop_graphs(sr_ctx* c) {
    for (int j = 0; j < kGraphLevels; ++j)
        for (int p = 0; p < 2; ++p) {
            if (c->gr[j][p]) (void)hipGraphExecDestroy(c->gr[j][p]);
            c->gr[j][p] = nullptr;
        }
}

// Enqueue n outer iterations on the context's stream: n split into powers of
// two, largest first, one graph replay each (20 iterations: 16 + 4).  The
// w / b ping-pong keeps its parity across an even-length graph; only the
// one-iteration graph flips it.
static int enqueue_iters(sr_ctx* c, int n) {
    while (n > 0) {
        const int p = c->parity;
        if (!c->use_graphs) {
            enqueue_iteration(c, p, c->stream);
            HIP_TRY(hipGetLastError());
            c->parity ^= 1;
            c->k += 1;
            n -= 1;
            continue;
        }
        int j = kGraphLevels - 1;
        while ((1 << j) > n) --j;
        if (!c->gr[j][p]) { int rc = capture(c, p, 1 << j, &c->gr[j][p]); if (rc) return rc; }
        HIP_TRY(hipGraphLaunch(c->gr[j][p], c->stream));
        if (j == 0) c->parity ^= 1;
        c->k += 1 << j;
        n -= 1 << j;
    }
    return SR_OK;
}

static int copy_in(sr_ctx* c, void* dst, const void* src, size_t bytes, uint32_t flags) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, (flags & SR_HOST) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->stream));
    return SR_OK;
}

static int copy_out(sr_ctx* c, void* dst, const void* src, size_t bytes, uint32_t flags, bool sync = true) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, (flags & SR_HOST) ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           c->stream));
    if ((flags & SR_HOST) && sync) HIP_TRY(hipStreamSynchronize(c->stream));
    return SR_OK;
}

static int read_scal(sr_ctx* c, DevScal* out) {
    HIP_TRY(hipMemcpyAsync(c->hscal, c->b.scal, sizeof(DevScal), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *out = *c->hscal;
    return SR_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int sr_params_default(sr_params* p) {
    if (!p) return fail(SR_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(sr_params);
    p->gamma = 4.0;
    p->alpha = 4.0;
    p->beta = 0.2;
    p->mu = 8.0;
    p->tau = 0.1;
    p->eps = 1.5;
    p->band_l = 1.0;
    p->d = 5.0;
    p->R = 3;
    p->sigma = 1.5;
    p->rho = 1000.0;
    p->s_exp = 2;
    p->S = 3;
    p->tol_inner = 0.0;
    p->tol_outer = 0.0;
    p->min_iter = 0;
    p->check_every = 10;
    p->w0_mode = 0;
    p->zero_tol = 1e-3;
    p->w_solver = 0;
    p->w_sweeps = 1;
    p->phi_solver = 0;
    p->bc = 0;
    return SR_OK;
}

int sr_workspace_size(int32_t M, int32_t N, const sr_params* p, size_t* bytes) {
    if (!bytes) return fail(SR_EINVAL, "bytes is NULL");
    int rc = validate(M, N, p);
    if (rc) return rc;
    *bytes = make_layout(M, N, 1, sweep_buffers(*p)).total;
    return SR_OK;
}

int sr_create(sr_ctx** out, int32_t M, int32_t N, const sr_params* p, void* workspace, size_t bytes,
              void* hip_stream) {
    if (!out) return fail(SR_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(M, N, p);
    if (rc) return rc;
    if (!workspace) return fail(SR_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255) return fail(SR_EWORKSPACE, "workspace must be 256-byte aligned");
    const Layout L = make_layout(M, N, 1, sweep_buffers(*p));
    if (bytes < L.total) return fail(SR_EWORKSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);

    sr::configure_kernels();
    sr::configure_aos();
    sr_ctx* c = new sr_ctx();
    c->M = M;
    c->N = N;
    c->nz = 1;
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    make_kparams(c->p, c->kp);
    make_gauss(c->p.sigma, c->gauss, c->gauss_r);
    carve(c->b, (char*)workspace, L);
    c->geo.M = M;
    c->geo.N = N;
    c->geo.twM = c->b.twM;
    c->geo.twN = c->b.twN;
    c->geo.stM = c->b.stM;
    c->geo.stN = c->b.stN;
    c->geo.dtM = c->b.dtM;
    c->geo.dtN = c->b.dtN;
    c->geo.cM = c->b.cM;
    c->geo.cN = c->b.cN;
    c->geo.taumu = (float)(c->p.tau * c->p.mu);
    c->geo.bc = c->p.bc;
    c->fused = use_fused(c->p, c->geo, c->kp);
    const char* ng = std::getenv("SR_NO_GRAPH");
    c->use_graphs = !(ng && ng[0] == '1');
    const char* th = std::getenv("SR_TILE_TH");
    c->geo.tile_th = th ? std::atoi(th) : tuned_tile_height(M, N, c->kp.R, 1);

    hipError_t e = hipHostMalloc((void**)&c->hscal, sizeof(DevScal), hipHostMallocDefault);
    if (e != hipSuccess) { delete c; return fail(SR_EHIP, "hipHostMalloc: %s", hipGetErrorString(e)); }
    e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipHostFree(c->hscal);
        delete c;
        return fail(SR_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    e = upload_tables(c->b, M, N, c->stream);
    if (e == hipSuccess) e = upload_aos(c, c->stream);
    if (e == hipSuccess) { sr::launch_reset_scal(c->b.scal, 1, 1, c->stream); e = hipGetLastError(); }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(c->cap);
        (void)hipHostFree(c->hscal);
        delete c;
        return fail(SR_EHIP, "sr_create upload: %s", hipGetErrorString(e));
    }
    *out = c;
    return SR_OK;
}

void sr_destroy(sr_ctx* c) {
    if (!c) return;
    drop_graphs(c);
    (void)hipStreamDestroy(c->cap);
    (void)hipHostFree(c->hscal);
    delete c;
}

const char* sr_last_error(void) { return g_err.c_str(); }

int sr_set_image(sr_ctx* c, const float* f, const float* phi0, uint32_t flags) {
    if (!c || !f || !phi0) return fail(SR_EINVAL, "NULL argument");
    const size_t bytes = sizeof(float) * c->M * c->N;
    const float* fd = f;
    const float* pd = phi0;
    if (flags & SR_HOST) {
        int rc = copy_in(c, c->b.Ph[2], f, bytes, flags);
        if (!rc) rc = copy_in(c, c->b.Ph[1], phi0, bytes, flags);
        if (rc) return rc;
        fd = c->b.Ph[2];
        pd = c->b.Ph[1];
    }
    sr::launch_reset_scal(c->b.scal, 1, 1, c->stream);
    sr::launch_edge(c->geo, fd, c->b.Rb, (float*)c->b.spec, c->b.g, c->gauss.data(), c->gauss_r, (float)c->p.rho,
                    c->p.s_exp, c->b.scal, c->stream);
    sr::launch_init(c->geo, pd, c->b.Ph[0], c->b.W[0], c->b.B[0], c->b.D, (float)c->p.mu, c->p.w0_mode, c->b.scal,
                    c->stream);
    HIP_TRY(hipGetLastError());
    c->parity = 0;
    c->k = 0;
    DevScal s;
    int rc = read_scal(c, &s);
    if (rc) return rc;
    if (s.nonfinite) return fail(SR_ENONFINITE, "f or phi0 contains NaN/Inf");
    c->image_set = true;
    return SR_OK;
}

int sr_step(sr_ctx* c, int32_t n_iter, sr_step_info* info) {
    if (!c) return fail(SR_EINVAL, "ctx is NULL");
    if (n_iter < 0) return fail(SR_EINVAL, "n_iter must be >= 0");
    if (!c->image_set) return fail(SR_ESTATE, "sr_step before sr_set_image / sr_set_state");
    const long long k0 = c->k;
    DevScal s0{};
    const bool tolin = c->p.tol_inner > 0;
    if (tolin) { int rc = read_scal(c, &s0); if (rc) return rc; }
    int done = 0, converged = 0;
    double r_last = -1.0;
    if (c->p.tol_outer > 0) {
        while (done < n_iter) {
            const int chunk = std::min(c->p.check_every, n_iter - done);
            int rc = enqueue_iters(c, chunk);
            if (rc) return rc;
            done += chunk;
            DevScal s;
            rc = read_scal(c, &s);
            if (rc) return rc;
            r_last = s.r_last;
            if (!std::isfinite(r_last)) return fail(SR_ENONFINITE, "iterate became non-finite at k=%lld", c->k);
            if (c->k >= c->p.min_iter && r_last < c->p.tol_outer) { converged = 1; break; }
        }
    } else {
        int rc = enqueue_iters(c, n_iter);
        if (rc) return rc;
        done = n_iter;
    }
    if (info || c->p.tol_outer <= 0) {
        DevScal s;
        int rc = read_scal(c, &s);
        if (rc) return rc;
        r_last = s.r_last;
        if (done > 0 && !std::isfinite(r_last)) return fail(SR_ENONFINITE, "iterate became non-finite at k=%lld", c->k);
        if (info) {
            info->iters_done = c->k - k0;
            info->k = c->k;
            info->r_last = r_last;
            info->inner_steps = tolin ? (s.inner_steps - s0.inner_steps) : (long long)c->p.S * (c->k - k0);
            info->converged = converged;
            info->reserved = 0;
        }
    }
    if (c->p.tol_outer > 0 && !converged) return SR_NOT_CONVERGED;
    return SR_OK;
}

int sr_get_phi(sr_ctx* c, float* phi_out, uint32_t flags) {
    if (!c || !phi_out) return fail(SR_EINVAL, "NULL argument");
    return copy_out(c, phi_out, phi_state(c), sizeof(float) * c->M * c->N, flags);
}

int sr_get_g(sr_ctx* c, float* g_out, uint32_t flags) {
    if (!c || !g_out) return fail(SR_EINVAL, "NULL argument");
    if (!c->image_set) return fail(SR_ESTATE, "sr_get_g before sr_set_image");
    return copy_out(c, g_out, c->b.g, sizeof(float) * c->M * c->N, flags);
}

int sr_energy(sr_ctx* c, double* E_total, double terms[3]) {
    if (!c || !E_total) return fail(SR_EINVAL, "NULL argument");
    if (!c->image_set) return fail(SR_ESTATE, "sr_energy before sr_set_image");
    sr::launch_energy(c->geo, c->kp, phi_state(c), c->b.g, c->b.part, 1, c->b.scal, c->stream);
    HIP_TRY(hipGetLastError());
    DevScal s;
    int rc = read_scal(c, &s);
    if (rc) return rc;
    *E_total = s.energy[0] + s.energy[1] + s.energy[2];
    if (terms) { terms[0] = s.energy[0]; terms[1] = s.energy[1]; terms[2] = s.energy[2]; }
    return SR_OK;
}

int sr_get_state(sr_ctx* c, float* phi, float* w, float* b, int64_t* k, uint32_t flags) {
    if (!c || !phi || !w || !b) return fail(SR_EINVAL, "NULL argument");
    const size_t MN = (size_t)c->M * c->N;
    int rc = copy_out(c, phi, phi_state(c), sizeof(float) * MN, flags, false);
    if (!rc) rc = copy_out(c, w, c->b.W[c->parity], 2 * sizeof(float) * MN, flags, false);
    if (!rc) rc = copy_out(c, b, c->b.B[c->parity], 2 * sizeof(float) * MN, flags);
    if (rc) return rc;
    if (k) *k = c->k;
    return SR_OK;
}

int sr_set_state(sr_ctx* c, const float* phi, const float* w, const float* b, int64_t k, uint32_t flags) {
    if (!c || !phi || !w || !b) return fail(SR_EINVAL, "NULL argument");
    if (!c->image_set) return fail(SR_ESTATE, "sr_set_state needs g: call sr_set_image first");
    if (k < 0) return fail(SR_EINVAL, "k must be >= 0");
    const size_t MN = (size_t)c->M * c->N;
    c->parity = 0;
    int rc = copy_in(c, c->b.Ph[0], phi, sizeof(float) * MN, flags);
    if (!rc) rc = copy_in(c, c->b.W[0], w, 2 * sizeof(float) * MN, flags);
    if (!rc) rc = copy_in(c, c->b.B[0], b, 2 * sizeof(float) * MN, flags);
    if (rc) return rc;
    sr::launch_set_D(c->geo, c->b.W[0], c->b.B[0], c->b.D, (float)c->p.mu, c->stream);
    sr::launch_set_k(c->b.scal, k, c->stream);
    HIP_TRY(hipGetLastError());
    if (flags & SR_HOST) HIP_TRY(hipStreamSynchronize(c->stream));
    c->k = k;
    return SR_OK;
}

int sr_edge_map(sr_ctx* c, const float* f, float* g_out, uint32_t flags) {
    if (!c || !f || !g_out) return fail(SR_EINVAL, "NULL argument");
    const size_t bytes = sizeof(float) * c->M * c->N;
    const float* fd = f;
    float* gd = g_out;
    if (flags & SR_HOST) {
        int rc = copy_in(c, phi_free(c, 1), f, bytes, flags);
        if (rc) return rc;
        fd = phi_free(c, 1);
        gd = phi_free(c, 0);
    }
    sr::launch_edge(c->geo, fd, c->b.Rb, (float*)c->b.spec, gd, c->gauss.data(), c->gauss_r, (float)c->p.rho,
                    c->p.s_exp, c->b.scal, c->stream);
    HIP_TRY(hipGetLastError());
    if (flags & SR_HOST) return copy_out(c, g_out, gd, bytes, flags);
    return SR_OK;
}

int sr_repulsion(sr_ctx* c, const float* w, const float* phi, float* v_out, uint32_t flags) {
    if (!c || !w || !phi || !v_out) return fail(SR_EINVAL, "NULL argument");
    const size_t MN = (size_t)c->M * c->N;
    const int q = c->parity ^ 1;   // the free ping-pong buffers hold no state
    const float* wd = w;
    const float* pd = phi;
    float* vd = v_out;
    if (flags & SR_HOST) {
        int rc = copy_in(c, c->b.W[q], w, 2 * sizeof(float) * MN, flags);
        if (!rc) rc = copy_in(c, phi_free(c, 0), phi, sizeof(float) * MN, flags);
        if (rc) return rc;
        wd = c->b.W[q];
        pd = phi_free(c, 0);
        vd = c->b.B[q];
    }
    sr::launch_repulsion(c->geo, c->kp, pd, wd, vd, c->stream);
    HIP_TRY(hipGetLastError());
    if (flags & SR_HOST) return copy_out(c, v_out, vd, 2 * sizeof(float) * MN, flags);
    return SR_OK;
}

int sr_implicit_solve(sr_ctx* c, const float* rhs, float* u_out, uint32_t flags) {
    if (!c || !rhs || !u_out) return fail(SR_EINVAL, "NULL argument");
    const size_t bytes = sizeof(float) * c->M * c->N;
    const float* rd = rhs;
    float* ud = u_out;
    if (flags & SR_HOST) {
        int rc = copy_in(c, phi_free(c, 0), rhs, bytes, flags);
        if (rc) return rc;
        rd = phi_free(c, 0);
        ud = phi_free(c, 1);
    }
    sr::launch_solve(c->geo, rd, nullptr, ud, c->b.spec, 0.0f, c->b.part, 1, c->b.scal, c->stream);
    HIP_TRY(hipGetLastError());
    if (flags & SR_HOST) return copy_out(c, u_out, ud, bytes, flags);
    return SR_OK;
}

int sr_autotune(sr_ctx* c, int32_t reps, int32_t* tile_th, double us_out[3]) {
    if (!c) return fail(SR_EINVAL, "NULL context");
    if (reps < 1) return fail(SR_EINVAL, "reps must be >= 1");
    if (!c->image_set) return fail(SR_ESTATE, "sr_autotune before sr_set_image");
    const int before = c->geo.tile_th;
    int rc = tune_tiles(c, reps, us_out);
    if (rc) return rc;
    if (c->geo.tile_th != before) drop_graphs(c);   // graphs hold the old launch shapes
    if (tile_th) *tile_th = c->geo.tile_th;
    return SR_OK;
}

int sr_prepare(sr_ctx* c) {
    if (!c) return fail(SR_EINVAL, "NULL context");
    if (!c->use_graphs) return SR_OK;
    for (int p = 0; p < 2; ++p) {
        int rc = SR_OK;
        for (int j = 0; j < kGraphLevels && rc == SR_OK; ++j)
            if (!c->gr[j][p]) rc = capture(c, p, 1 << j, &c->gr[j][p]);
        if (rc) return rc;
    }
    return SR_OK;
}

#ifndef SR_BUILD_ID
#define SR_BUILD_ID "unknown"
#endif
const char* sr_build_id(void) { return SR_BUILD_ID; }

int sr_profile_kernels(sr_ctx* c, int32_t n_iter, double ms[SR_NUM_KERNEL_KINDS],
                       int64_t count[SR_NUM_KERNEL_KINDS]) {
    if (!c || !ms || !count) return fail(SR_EINVAL, "NULL argument");
    if (n_iter < 1) return fail(SR_EINVAL, "n_iter must be >= 1");
    if (!c->image_set) return fail(SR_ESTATE, "sr_profile_kernels before sr_set_image");
    // n_iter outer iterations launched directly on the stream (no graph), the
    // same kernels in the same order as a graph replay, each iteration kernel
    // with its own start / stop events; synchronised after every iteration.
    // iteration kernels per outer iteration: S x 4, then the w step (one
    // launch per fixed-point sweep with that solver)
    const int per = (c->p.phi_solver == 1 ? 2 : 4) * c->p.S + (c->p.w_solver == 1 ? c->p.w_sweeps : 1);
    std::vector<hipEvent_t> ev(2 * (size_t)per, nullptr);
    std::vector<int> kind(per, 0);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    double tot[SR_NUM_KERNEL_KINDS] = {};
    int64_t cnt[SR_NUM_KERNEL_KINDS] = {};
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        int slot = 0;
        enqueue_iteration(c, c->parity, c->stream, [&](int k) {
            if (slot >= per) {   // cannot happen while per matches enqueue_iteration
                sr::set_launch_events(nullptr, nullptr);
                t_aos_ev[0] = t_aos_ev[1] = nullptr;
                return;
            }
            sr::set_launch_events(ev[2 * slot], ev[2 * slot + 1]);
            t_aos_ev[0] = ev[2 * slot];
            t_aos_ev[1] = ev[2 * slot + 1];
            kind[slot++] = k;
        });
        sr::set_launch_events(nullptr, nullptr);
        t_aos_ev[0] = t_aos_ev[1] = nullptr;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (int s = 0; s < slot && e == hipSuccess; ++s) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ev[2 * s], ev[2 * s + 1]);
            tot[kind[s]] += t;
            cnt[kind[s]] += 1;
        }
        c->parity ^= 1;
        c->k += 1;
    }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(SR_EHIP, "sr_profile_kernels: %s", hipGetErrorString(e));
    for (int k = 0; k < SR_NUM_KERNEL_KINDS; ++k) {
        ms[k] = cnt[k] ? tot[k] / (double)cnt[k] : 0.0;
        count[k] = cnt[k];
    }
    return SR_OK;
}

}  // extern "C"

// ---- batched solve --------------------------------------------------------
// Items are grouped by (M, N, model / solver parameters); each group is one
// sr_ctx whose planes hold nz instances ([nz][M][N]).  All groups' launches
// for a chunk of outer iterations are captured into one HIP graph; instances
// retire on the device (cap, tolerance, NaN) and are skipped by every kernel
// afterwards, so the host only polls the per-instance scalars between chunks.
static bool same_class(const sr_batch_item& a, const sr_batch_item& b) {
    const sr_params &x = a.params, &y = b.params;
    return a.M == b.M && a.N == b.N && x.gamma == y.gamma && x.alpha == y.alpha && x.beta == y.beta &&
           x.mu == y.mu && x.tau == y.tau && x.eps == y.eps && x.band_l == y.band_l && x.d == y.d && x.R == y.R &&
           x.sigma == y.sigma && x.rho == y.rho && x.s_exp == y.s_exp && x.S == y.S &&
           x.tol_inner == y.tol_inner && x.w0_mode == y.w0_mode && x.zero_tol == y.zero_tol &&
           x.w_solver == y.w_solver && (x.w_solver == 0 || x.w_sweeps == y.w_sweeps) &&
           x.phi_solver == y.phi_solver && x.bc == y.bc;
}

struct BatchPlan {
    std::vector<std::vector<int>> groups;   // item indices per group
    std::vector<size_t> offset;             // workspace offset per group
    size_t total = 0;
};

static int plan_batch(const sr_batch_item* items, int32_t n, BatchPlan& plan) {
    if (!items || n < 1) return fail(SR_EINVAL, "items is NULL or n < 1");
    for (int i = 0; i < n; ++i) {
        const sr_batch_item& it = items[i];
        int rc = validate(it.M, it.N, &it.params);
        if (rc) return fail(rc, "item %d: %s", i, g_err.c_str());
        if (it.max_iter < 1) return fail(SR_EINVAL, "item %d: max_iter must be >= 1", i);
        bool placed = false;
        for (auto& g : plan.groups)
            if (same_class(items[g[0]], it)) { g.push_back(i); placed = true; break; }
        if (!placed) plan.groups.push_back({i});
    }
    size_t o = 0;
    for (auto& g : plan.groups) {
        plan.offset.push_back(o);
        o += align256(make_layout(items[g[0]].M, items[g[0]].N, (int)g.size(), sweep_buffers(items[g[0]].params))
                          .total);
    }
    plan.total = o;
    return SR_OK;
}

extern "C" {

int sr_batch_workspace_size(const sr_batch_item* items, int32_t n, size_t* bytes) {
    if (!bytes) return fail(SR_EINVAL, "bytes is NULL");
    BatchPlan plan;
    int rc = plan_batch(items, n, plan);
    if (rc) return rc;
    *bytes = plan.total;
    return SR_OK;
}

int sr_solve_batch(sr_batch_item* items, int32_t n, void* workspace, size_t bytes, void* hip_stream) {
    BatchPlan plan;
    int rc = plan_batch(items, n, plan);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
        if (!items[i].f || !items[i].phi0 || !items[i].phi_out) return fail(SR_EINVAL, "item %d: NULL buffer", i);
    if (!workspace) return fail(SR_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255) return fail(SR_EWORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < plan.total) return fail(SR_EWORKSPACE, "workspace has %zu bytes, needs %zu", bytes, plan.total);
    sr::configure_kernels();
    sr::configure_aos();
    hipStream_t st = (hipStream_t)hip_stream;
    const int G = (int)plan.groups.size();
    std::vector<sr_ctx> ctx(G);
    std::vector<std::vector<DevScal>> hs(G);
    int max_cap = 0;
    for (int gi = 0; gi < G; ++gi) {
        const auto& idx = plan.groups[gi];
        const sr_batch_item& it0 = items[idx[0]];
        sr_ctx& c = ctx[gi];
        c.M = it0.M; c.N = it0.N; c.nz = (int)idx.size();
        c.p = it0.params;
        c.stream = st;
        make_kparams(c.p, c.kp);
        make_gauss(c.p.sigma, c.gauss, c.gauss_r);
        carve(c.b, (char*)workspace + plan.offset[gi],
              make_layout(c.M, c.N, c.nz, sweep_buffers(c.p)));
        c.geo.M = c.M; c.geo.N = c.N; c.geo.twM = c.b.twM; c.geo.twN = c.b.twN;
        c.geo.stM = c.b.stM; c.geo.stN = c.b.stN;
        c.geo.dtM = c.b.dtM; c.geo.dtN = c.b.dtN; c.geo.cM = c.b.cM; c.geo.cN = c.b.cN;
        c.geo.taumu = (float)(c.p.tau * c.p.mu);
        c.geo.bc = c.p.bc;
        c.fused = use_fused(c.p, c.geo, c.kp);
        HIP_TRY(upload_tables(c.b, c.M, c.N, st));
        HIP_TRY(upload_aos(&c, st));
        HIP_TRY(hipStreamSynchronize(st));
        hs[gi].assign(c.nz, DevScal{});
        for (int z = 0; z < c.nz; ++z) {
            const sr_batch_item& it = items[idx[z]];
            DevScal& d = hs[gi][z];
            std::memset(&d, 0, sizeof d);
            d.active = 1;
            d.r_last = -1.0;
            d.max_iter = it.max_iter;
            d.min_iter = it.params.min_iter;
            d.tol_outer = it.params.tol_outer;
            max_cap = std::max(max_cap, it.max_iter);
        }
        HIP_TRY(hipMemcpy(c.b.scal, hs[gi].data(), sizeof(DevScal) * c.nz, hipMemcpyHostToDevice));
        const size_t MN = (size_t)c.M * c.N;
        for (int z = 0; z < c.nz; ++z) {
            HIP_TRY(hipMemcpyAsync(c.b.Ph[2] + z * MN, items[idx[z]].f, MN * 4, hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipMemcpyAsync(c.b.Ph[1] + z * MN, items[idx[z]].phi0, MN * 4, hipMemcpyDeviceToDevice, st));
        }
        sr::launch_edge(c.geo, c.b.Ph[2], c.b.Rb, (float*)c.b.spec, c.b.g, c.gauss.data(), c.gauss_r, (float)c.p.rho,
                        c.p.s_exp, c.b.scal, st, c.nz);
        sr::launch_init(c.geo, c.b.Ph[1], c.b.Ph[0], c.b.W[0], c.b.B[0], c.b.D, (float)c.p.mu, c.p.w0_mode, c.b.scal, st,
                        c.nz);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(st));
    // instances with non-finite inputs are retired before the first iteration
    for (int gi = 0; gi < G; ++gi) {
        sr_ctx& c = ctx[gi];
        HIP_TRY(hipMemcpy(hs[gi].data(), c.b.scal, sizeof(DevScal) * c.nz, hipMemcpyDeviceToHost));
        bool any = false;
        for (auto& d : hs[gi]) if (d.nonfinite) { d.active = 0; any = true; }
        if (any) HIP_TRY(hipMemcpy(c.b.scal, hs[gi].data(), sizeof(DevScal) * c.nz, hipMemcpyHostToDevice));
    }
    // stencil tile height per size class: a recorded choice, else tuned on
    // the group's initial state (state unchanged)
    for (int gi = 0; gi < G; ++gi) {
        sr_ctx& c = ctx[gi];
        c.geo.tile_th = tuned_tile_height(c.M, c.N, c.kp.R, c.nz);
        if (!c.geo.tile_th) {
            rc = tune_tiles(&c, 3, nullptr);
            if (rc) return rc;
        }
    }
    // one graph: a chunk of outer iterations of every group, each group an
    // independent branch (its own capture stream, forked from and joined to
    // the origin), so groups of small instances run beside larger ones
    const int chunk = 10;
    const int NB = std::min(G, 16);
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> br(NB, nullptr);
    std::vector<hipEvent_t> evb(NB, nullptr);
    hipEvent_t fork = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (int i = 0; i < NB && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&evb[i], hipEventDisableTiming);
    }
    auto release = [&]() {
        for (int i = 0; i < NB; ++i) {
            if (evb[i]) (void)hipEventDestroy(evb[i]);
            if (br[i]) (void)hipStreamDestroy(br[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (cap) (void)hipStreamDestroy(cap);
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = hipEventRecord(fork, cap);
        for (int i = 0; i < NB && e == hipSuccess; ++i) e = hipStreamWaitEvent(br[i], fork, 0);
        for (int gi = 0; gi < G && e == hipSuccess; ++gi)
            enqueue_chunk(&ctx[gi], 0, chunk, br[gi % NB]);
        for (int i = 0; i < NB && e == hipSuccess; ++i) {
            e = hipEventRecord(evb[i], br[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(cap, evb[i], 0);
        }
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        release();
        return fail(SR_EHIP, "batch graph: %s", hipGetErrorString(e));
    }
    int done = 0;
    while (done < max_cap) {
        e = hipGraphLaunch(exec, st);
        if (e != hipSuccess) break;
        done += chunk;
        bool any_active = false;
        for (int gi = 0; gi < G && e == hipSuccess; ++gi) {
            e = hipMemcpyAsync(hs[gi].data(), ctx[gi].b.scal, sizeof(DevScal) * ctx[gi].nz, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            for (auto& d : hs[gi]) any_active |= d.active != 0;
        }
        if (!any_active) break;
    }
    (void)hipGraphExecDestroy(exec);
    release();
    if (e != hipSuccess) return fail(SR_EHIP, "batch iterations: %s", hipGetErrorString(e));
    // energies and outputs
    int worst = SR_OK;
    for (int gi = 0; gi < G; ++gi) {
        sr_ctx& c = ctx[gi];
        const size_t MN = (size_t)c.M * c.N;
        // an instance's state is in the ping-pong half of its own iteration
        // count (retired instances are not advanced further); the energy
        // kernel reads phi from Ph[0] for every instance
        for (int z = 0; z < c.nz; ++z)
            if (hs[gi][z].k & 1)
                HIP_TRY(hipMemcpyAsync(c.b.Ph[0] + z * MN, c.b.Ph[1] + z * MN, MN * 4, hipMemcpyDeviceToDevice, st));
        sr::launch_energy(c.geo, c.kp, c.b.Ph[0], c.b.g, c.b.part, c.nz, c.b.scal, st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(hs[gi].data(), c.b.scal, sizeof(DevScal) * c.nz, hipMemcpyDeviceToHost, st));
        const auto& idx = plan.groups[gi];
        for (int z = 0; z < c.nz; ++z) {
            const sr_batch_item& it = items[idx[z]];
            HIP_TRY(hipMemcpyAsync(it.phi_out, c.b.Ph[0] + z * MN, MN * 4, hipMemcpyDeviceToDevice, st));
            const int par = (int)(hs[gi][z].k & 1);
            if (it.w_out)
                HIP_TRY(hipMemcpyAsync(it.w_out, c.b.W[par] + 2 * z * MN, 2 * MN * 4, hipMemcpyDeviceToDevice, st));
            if (it.b_out)
                HIP_TRY(hipMemcpyAsync(it.b_out, c.b.B[par] + 2 * z * MN, 2 * MN * 4, hipMemcpyDeviceToDevice, st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        for (int z = 0; z < c.nz; ++z) {
            sr_batch_item& it = items[idx[z]];
            const DevScal& d = hs[gi][z];
            it.iters = (int32_t)d.k;
            it.r_last = d.r_last;
            it.energy = d.energy[0] + d.energy[1] + d.energy[2];
            if (d.nonfinite) it.status = SR_ENONFINITE;
            else if (d.converged || it.params.tol_outer <= 0) it.status = SR_OK;
            else it.status = SR_NOT_CONVERGED;
            it.reserved = 0;
            if (it.status == SR_NOT_CONVERGED && worst == SR_OK) worst = SR_NOT_CONVERGED;
        }
    }
    return worst;
}

}  // extern "C"
