// Instances of the fused right-hand-side kernel for rows of 64, 128 and 256 points.
#include "sr_fused.hpp"

namespace sr {
void fused_launch_64(const FusedArgs& a) { fused_launch_len<64>(a); }
void fused_launch_128(const FusedArgs& a) { fused_launch_len<128>(a); }
void fused_launch_256(const FusedArgs& a) { fused_launch_len<256>(a); }
void fused_configure_small() {
    fused_configure_len<64>();
    fused_configure_len<128>();
    fused_configure_len<256>();
}
}  // namespace sr
