// fwd7.hip -- the 7x7 instantiations of the forward filter.
#include "fwd_launch.h"

namespace odf {

hipError_t launch_forward7(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream) {
    return launch_w<7>(kind, dist, u8, aggregates, cfg, prm, stream);
}

}  // namespace odf
