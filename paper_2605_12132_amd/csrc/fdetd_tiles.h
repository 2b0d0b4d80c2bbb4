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
// axis = the near-axis tiles (rows 0 .. ax_rows-1 in segments of seg_ax rows, nstrip_ax strips) or the
// main ones (rows ax_rows .. nr-1 in segments of seg_rows rows, nstrip strips); cpw = z columns per tile
// of that kind.  Strips are numbered fastest, so a contiguous range of tiles -- what one XCD receives --
// holds neighbouring strips; D.tile_order puts halves before segments (0) or segments before halves (1:
// every range holds as many E-half as B-half tiles), whichever the plan measured faster.  Returns false
// if the tile would leave the grid or its kind's rows.
template <typename DESC>
FDETD_HD inline bool decode_tile(DESC &D, int r, int halves, bool axis, int cpw, TileCoord &c)
{
    const int nseg_l = axis ? D.nseg_ax : D.nseg;
    const int nstrip = axis ? D.nstrip_ax : D.nstrip;
    const int per_half = nseg_l * nstrip;
    if (per_half <= 0 || r < 0 || r >= halves * per_half) return false;
    int sl;  // segment index within this launch
    if (D.tile_order) {
        sl = r / (halves * nstrip);
        r -= sl * halves * nstrip;
        c.half = r / nstrip;
        r -= c.half * nstrip;
    } else {
        c.half = r / per_half;
        r -= c.half * per_half;
        sl = r / nstrip;
        r -= sl * nstrip;
    }
    c.i0 = r * cpw;
    const int seg = axis ? D.seg_ax : D.seg_rows;
    const int begin = axis ? 0 : D.ax_rows, end = axis ? D.ax_rows : D.nr;
    c.k0 = begin + sl * seg;
    c.k1 = c.k0 + seg < end ? c.k0 + seg : end;
    return seg > 0 && c.i0 >= 0 && c.i0 < D.nz && c.k0 >= begin && c.k0 < end && end <= D.nr && c.k1 > c.k0;
}

}  // namespace fdetd
