// fwd9.hip -- the 9x9 instantiations of the forward filter (BVDF and DDF; one
// tile shape, 32 x 16: each thread keeps 81 aggregates, 248 VGPRs for BVDF).
#include "fwd_launch.h"

namespace odf {

hipError_t launch_forward9(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream) {
    return launch_w<9>(kind, dist, u8, aggregates, cfg, prm, stream);
}

}  // namespace odf
