// fd_acoustic_top.hip -- the tiled 3D acoustic kernel of libfd (gfx950) for
// radius 7-8 (space orders 14-16); see fd_acoustic_tiled.h.
#include "fd_acoustic_tiled.h"

namespace fd {

hipError_t launch_acoustic_tiled_r78(const AcousticStep& p, int radius, int cfg,
                                     int shots_per_block, hipStream_t s) {
    switch (radius) {
        case 7: return launch_tiled_cfg<7>(p, cfg, shots_per_block, s);
        case 8: return launch_tiled_cfg<8>(p, cfg, shots_per_block, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fd
