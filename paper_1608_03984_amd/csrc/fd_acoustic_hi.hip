// fd_acoustic_hi.hip -- the tiled 3D acoustic kernel of libfd (gfx950) for
// radius 5-6 (space orders 10-12); see fd_acoustic_tiled.h.
#include "fd_acoustic_tiled.h"

namespace fd {

hipError_t launch_acoustic_tiled_r56(const AcousticStep& p, int radius, int cfg,
                                     int shots_per_block, hipStream_t s) {
    switch (radius) {
        case 5: return launch_tiled_cfg<5>(p, cfg, shots_per_block, s);
        case 6: return launch_tiled_cfg<6>(p, cfg, shots_per_block, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fd
