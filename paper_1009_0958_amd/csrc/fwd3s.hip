// fwd3s.hip -- the 3x3 instantiations of the strip form of the forward filter.
#include "fwd_strip.h"

namespace odf {

hipError_t launch_strip3(int kind, int dist, bool u8, const FwdParams& prm, int nb,
                         hipStream_t s) {
    return launch_strip_w<3>(kind, dist, u8, prm, nb, s);
}

}  // namespace odf
