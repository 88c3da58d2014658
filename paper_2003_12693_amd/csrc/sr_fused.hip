// Dispatch of the fused right-hand-side + forward row transform kernel
// (sr_fused.hpp): strip height and row length.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "sr_fused.hpp"

namespace sr {

// log2 of the rows per workgroup: 4-row strips (2 transforms) where their
// workgroup fills a wave (N >= 128), else 8; SR_FUSED_LR overrides with
// another instantiated height.  Measured at 1024^2 (per launch): 2 rows
// 14.7 us, 4 rows 13.3 us, 8 rows 17.0 us (the separate rhs and row-FFT
// kernels: 11.0 + 5.6 us).
static int fused_lr(int N) {
    static const int env = [] {
        const char* s = std::getenv("SR_FUSED_LR");
        return s ? std::atoi(s) : 0;
    }();
    const int base = N >= 128 ? 2 : 3;
    const bool ok = N >= 256 ? (env == 1 || env == 2) : N == 128 ? (env == 2 || env == 3) : env == 3;
    return ok ? env : base;
}

bool fused_rhs_supported(const Geometry& geo, const KParams& kp) {
    return geo.N >= 64 && geo.N <= 1024 && geo.M >= 8 && kp.R >= 0 && kp.R <= kMaxR;
}

void launch_rhs_fwd(const Geometry& geo, const KParams& kp, const float* phi_s, const float* W, const float* g,
                    const float* D, float2* spec, int nz, DevScal* sc, hipStream_t st, const FinFold* fold) {
    const FusedArgs a{&geo, &kp, phi_s, W, g, D, spec, nz, sc, st, fold, fused_lr(geo.N)};
    switch (geo.N) {
        case 64: fused_launch_64(a); break;
        case 128: fused_launch_128(a); break;
        case 256: fused_launch_256(a); break;
        case 512: fused_launch_512(a); break;
        case 1024: fused_launch_1024(a); break;
        default: break;
    }
}

void configure_fused() {
    fused_configure_small();
    fused_configure_512();
    fused_configure_1024();
}

}  // namespace sr
