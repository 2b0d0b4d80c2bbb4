// Tile decoding of the row-marching launches, shared by the kernels and by the plan-time check that
// every launch covers each (half, segment, strip) of every problem exactly once and never leaves a grid.
#pragma once

#if defined(__HIPCC__)
#define FDETD_HD __host__ __device__
#else
#define FDETD_HD
#endif

#include "fdetd_internal.h"

namespace fdetd {

struct TileCoord {
    int half, i0, k0, k1;
};

// Tile r (0-based within problem D of one launch) -> coordinates.  halves = 2 (Maxwell) or 1 (envelope);
// axis = the near-axis launch (segments 0 .. nseg_ax-1) or the main one (segments nseg_ax .. nseg-1);
// cpw = z columns per tile.  Returns false if the tile would leave the grid.
template <typename DESC>
FDETD_HD inline bool decode_tile(DESC &D, int r, int halves, bool axis, int cpw, TileCoord &c)
{
    const int nseg_l = axis ? D.nseg_ax : D.nseg - D.nseg_ax;
    const int per_half = nseg_l * D.nstrip;
    if (per_half <= 0 || r < 0 || r >= halves * per_half) return false;
    c.half = r / per_half;
    r -= c.half * per_half;
    const int sl = r / D.nstrip;  // segment index within this launch
    c.i0 = (r - sl * D.nstrip) * cpw;
    const int seg = sl + (axis ? 0 : D.nseg_ax);
    c.k0 = seg * D.seg_rows;
    c.k1 = c.k0 + D.seg_rows < D.nr ? c.k0 + D.seg_rows : D.nr;
    return c.i0 >= 0 && c.i0 < D.nz && c.k0 >= 0 && c.k0 < D.nr && c.k1 > c.k0;
}

}  // namespace fdetd
