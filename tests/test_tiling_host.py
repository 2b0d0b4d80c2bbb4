"""The tile decoding shared by the row-marching kernels (csrc/fdetd_tiles.h), compiled for the host with
g++ and checked over random tilings: every (half, z column, rho row) of a problem is produced exactly once
by the near-axis tiles (32 columns wide) and the main tiles together, in either tile order, and no tile
leaves the grid or its kind's rows.  This is the same
function the kernels call, so a decoding mistake is caught here before it reaches the GPU."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12132_amd", "csrc")

PROGRAM = r'''
#include "fdetd_tiles.h"
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
using namespace fdetd;
int main() {
    unsigned s = 12345;
    auto rnd = [&](int lo, int hi) { s = s * 1103515245u + 12345u; return lo + (int)((s >> 8) % (unsigned)(hi - lo + 1)); };
    for (int trial = 0; trial < 20000; ++trial) {
        ProbDesc D; std::memset(&D, 0, sizeof D);
        const int cpw = rnd(0, 1) ? 32 : 64, cpw_ax = 32, halves = rnd(1, 2);
        D.tile_order = rnd(0, 1);
        D.nz = rnd(1, 700); D.nr = rnd(1, 300); D.seg_rows = rnd(1, 70);
        D.nstrip = (D.nz + cpw - 1) / cpw;
        if (rnd(0, 1)) {  // FP32C: near-axis tiles over the first rows, 32 columns wide
            D.ax_rows = rnd(1, 32);
            if (D.ax_rows > D.nr) D.ax_rows = D.nr;
            D.seg_ax = rnd(1, 40);
            D.nseg_ax = (D.ax_rows + D.seg_ax - 1) / D.seg_ax;
            D.nstrip_ax = (D.nz + cpw_ax - 1) / cpw_ax;
        }
        D.nseg = (D.nr - D.ax_rows + D.seg_rows - 1) / D.seg_rows;
        // every (half, column, row) must be produced exactly once by the two kinds of tile together
        std::vector<int> seen((size_t)halves * D.nz * D.nr, 0);
        for (int axis = 0; axis < 2; ++axis) {
            const int w = axis ? cpw_ax : cpw;
            const int nl = halves * (axis ? D.nseg_ax * D.nstrip_ax : D.nseg * D.nstrip);
            for (int r = 0; r < nl; ++r) {
                TileCoord c;
                if (!decode_tile(D, r, halves, axis, w, c)) { printf("FAIL decode %d\n", trial); return 1; }
                if (c.i0 < 0 || c.i0 >= D.nz || c.i0 % w || c.k0 < 0 || c.k1 > D.nr || c.k0 >= c.k1) { printf("FAIL bounds %d\n", trial); return 1; }
                if ((axis && c.k1 > D.ax_rows) || (!axis && c.k0 < D.ax_rows)) { printf("FAIL launch %d\n", trial); return 1; }
                if (c.k1 - c.k0 > (axis ? D.seg_ax : D.seg_rows)) { printf("FAIL length %d\n", trial); return 1; }
                for (int i = c.i0; i < c.i0 + w && i < D.nz; ++i)
                    for (int k = c.k0; k < c.k1; ++k) seen[((size_t)c.half * D.nz + i) * D.nr + k]++;
            }
            TileCoord c;
            if (decode_tile(D, nl, halves, axis, w, c) || decode_tile(D, -1, halves, axis, w, c)) { printf("FAIL range %d\n", trial); return 1; }
        }
        for (int v : seen) if (v != 1) { printf("FAIL cover %d\n", trial); return 1; }
    }
    printf("OK\n");
    return 0;
}
'''


def test_tile_decoding_covers_every_tile_once():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as fh:
            fh.write(PROGRAM)
        r = subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", CSRC, "-I", "/opt/rocm/include",
                            "-I", os.path.join(ROOT, "include"), src, "-o", exe], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.fail(r.stderr[-2000:])
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout
