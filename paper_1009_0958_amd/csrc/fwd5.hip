// fwd5.hip -- the 5x5 instantiations of the forward filter.
#include "fwd_launch.h"

namespace odf {

hipError_t launch_forward5(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream) {
    return launch_w<5>(kind, dist, u8, aggregates, cfg, prm, stream);
}

}  // namespace odf
