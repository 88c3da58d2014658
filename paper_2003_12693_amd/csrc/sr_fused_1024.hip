// Instances of the fused right-hand-side kernel for rows of 1024 points.
#include "sr_fused.hpp"

namespace sr {
void fused_launch_1024(const FusedArgs& a) { fused_launch_len<1024>(a); }
void fused_configure_1024() { fused_configure_len<1024>(); }
}  // namespace sr
