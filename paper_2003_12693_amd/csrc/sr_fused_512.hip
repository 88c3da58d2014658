// Instances of the fused right-hand-side kernel for rows of 512 points.
#include "sr_fused.hpp"

namespace sr {
void fused_launch_512(const FusedArgs& a) { fused_launch_len<512>(a); }
void fused_configure_512() { fused_configure_len<512>(); }
}  // namespace sr
