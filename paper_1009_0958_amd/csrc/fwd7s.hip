// fwd7s.hip -- the 7x7 instantiations of the strip form of the forward filter.
#include "fwd_strip.h"

namespace odf {

hipError_t launch_strip7(int kind, int dist, bool u8, const FwdParams& prm, int nb,
                         hipStream_t s) {
    return launch_strip_w<7>(kind, dist, u8, prm, nb, s);
}

}  // namespace odf
