// fwd.hip -- the tile-shape table of the forward filter, the 3x3
// instantiations and the dispatch over window sizes.
#include "fwd_launch.h"

namespace odf {

// 5x5 ACWDDF keeps four register sets of n values per thread (aggregates
// and centre terms of both passes) and 7x7 keeps a 13 x 7 grid of row sums:
// 512-thread tiles only.  The 5x5 centre-weighted filters share the rule (CWDDF
// parks its weighted angle sums in LDS, which at 32 x 32 would not leave room
// for a float32 tile's pixel arrays).
bool tile_config_valid(int window, int kind, int cfg, bool u8) {
    if (is_strip_config(cfg)) {  // as strip_form (fwd_strip.h)
        if (centre_weighted(kind)) return window == 3 || window == 5 || window == 7;
        return (kind == kBVDF || kind == kDDF) &&
               (window == 3 || window == 5 || window == 7 || (window == 9 && kind == kBVDF && u8));
    }
    if (cfg < 0 || cfg >= kNumTileConfigs) return false;
    if (window == 9) return cfg == 2;  // 32 x 16 (64 x 8 leaves no output row at h = 4)
    if ((window == 5 && centre_weighted(kind)) || window == 7)
        return kTileW[cfg] * kTileH[cfg] <= 512;
    return true;
}

// Default: 32 x 16 for every class.  On 3840 x 2160 it beats 32 x 32 by 10 %
// (3x3 DDF) to 22 % (5x5 BVDF, uint8) and 14 % for 5x5 DDF on float32; at
// 1024 x 1024 it is within 3 % of the fastest shape.  odf_autotune refines it.
int tile_config_default(int, int) { return 2; }

void tile_config_shape(int cfg, int* ext_w, int* ext_h) {
    if (is_strip_config(cfg)) {  // one band of the strip
        *ext_w = 32;
        *ext_h = 16;
        return;
    }
    *ext_w = kTileW[cfg];
    *ext_h = kTileH[cfg];
}

hipError_t launch_forward(int window, int kind, int dist, bool u8, bool aggregates, int cfg,
                          const FwdParams& prm, hipStream_t stream) {
    if (window == 3) return launch_w<3>(kind, dist, u8, aggregates, cfg, prm, stream);
    if (window == 5) return launch_forward5(kind, dist, u8, aggregates, cfg, prm, stream);
    if (window == 7) return launch_forward7(kind, dist, u8, aggregates, cfg, prm, stream);
    if (window == 9 && !centre_weighted(kind))
        return launch_forward9(kind, dist, u8, aggregates, cfg, prm, stream);
    // the direct form: BVDF / DDF past 9x9, the centre-weighted kinds from 9x9
    if (aggregates) return hipErrorInvalidValue;  // no aggregate-inspection form there
    return launch_forward_general(window, kind, dist, u8, prm, stream);
}

}  // namespace odf
