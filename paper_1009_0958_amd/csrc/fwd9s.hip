// fwd9s.hip -- the 9x9 instantiations of the strip form of the forward filter.
#include "fwd_strip.h"

namespace odf {

hipError_t launch_strip9(int kind, int dist, bool u8, const FwdParams& prm, int nb,
                         hipStream_t s) {
    return launch_strip_w<9>(kind, dist, u8, prm, nb, s);
}

}  // namespace odf
