"""Host check of the level order that the sweep kernels use for tiles of the
persistent edge (8^3): the table builder is taken from kernels.hip and
compiled with the host compiler.  For every class, the 512 entries are a
permutation of the tile's cells; for classes 0-5 every level lies in one group
of 64 consecutive slots; with 128 and with 512 threads no thread owns two
cells of one level; every level lies in the 64 slots from its first one
(c_level_start, from which the algorithm-1 pass takes a level's cells); and on
every tile of two octants (16^3 tiles, and a ragged 9 x 13 x 5) the class of
the tile gives every cell a level above the level of each cell of the tile it
reads (the four upstream centres one layer back along its major axis, ties
z > y > x, Sect. 2.1's short characteristics).  A level order that broke one
of these would let a cell read a column before it is formed."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
KERNELS = os.path.join(HERE, "..", "paper_1201_5651_amd", "csrc", "kernels.hip")

HARNESS = r"""
#include <algorithm>
#include <cstdio>
constexpr int PERSIST_TILE = 8;
%(builder)s
static constexpr LevelOrder LO = make_level_order();
static constexpr LevelStart LS = make_level_start();
// major axis of the ray to a cell centre, ties z > y > x
static int major(const int L[3])
{
    const double ad[3] = { L[0] + .5, L[1] + .5, L[2] + .5 };
    return (ad[2] >= ad[0] && ad[2] >= ad[1]) ? 2 : (ad[1] >= ad[0] ? 1 : 0);
}
%(classifier)s
int main()
{
    int bad = 0;
    for (int c = 0; c < LEVEL_CLASSES; ++c) {
        int seen[512] = { 0 }, group[32];
        for (int l = 0; l < 32; ++l) group[l] = -1;
        for (int i = 0; i < 512; ++i) {
            const unsigned e = LO.cell[c][i];
            const int lx = e & 31, ly = (e >> 5) & 31, lz = (e >> 10) & 31, lev = e >> 15;
            if (lx > 7 || ly > 7 || lz > 7 || lev > 21) { ++bad; continue; }
            ++seen[lx + 8 * (ly + 8 * lz)];
            if (c < 6 && group[lev] >= 0 && group[lev] != i / 64) ++bad;
            group[lev] = i / 64;
        }
        for (int q = 0; q < 512; ++q) bad += seen[q] != 1;
        // every level lies in the 64 slots from its first one (a wavefront
        // takes a level's cells from there, lane t the slot that is t mod 64)
        for (int i = 0; i < 512; ++i) {
            const int lev = (int)(LO.cell[c][i] >> 15), f = LS.first[c][lev];
            bad += f < 0 || i < f || i >= f + 64;
        }
        for (int nt : { 128, 512 })
            for (int t = 0; t < nt; ++t) {
                int cnt[32] = { 0 };
                for (int k = 0; k < 512 / nt; ++k) bad += ++cnt[LO.cell[c][t + k * nt] >> 15] > 1;
            }
    }
    const int dims[2][3] = { { 16, 16, 16 }, { 9, 13, 5 } };
    long reads = 0;
    for (int d = 0; d < 2; ++d)
        for (int tx = 0; tx < dims[d][0]; ++tx)
            for (int ty = 0; ty < dims[d][1]; ++ty)
                for (int tz = 0; tz < dims[d][2]; ++tz) {
                    int nlev = 0;
                    const int c = level_class(tx, ty, tz, nlev);
                    int level[512];
                    for (int i = 0; i < 512; ++i) {
                        const unsigned e = LO.cell[c][i];
                        level[(e & 31) + 8 * (((e >> 5) & 31) + 8 * ((e >> 10) & 31))] = e >> 15;
                    }
                    for (int q = 0; q < 512; ++q) {
                        const int l[3] = { q & 7, (q >> 3) & 7, q >> 6 };
                        const int L[3] = { 8 * tx + l[0], 8 * ty + l[1], 8 * tz + l[2] };
                        bad += level[q] >= nlev;
                        const int a = major(L), b = a == 2 ? 0 : a + 1, cc = a == 0 ? 2 : a - 1;
                        if (L[a] == 0) continue;
                        for (int db = 0; db < 2; ++db)
                            for (int dc = 0; dc < 2; ++dc) {
                                int u[3] = { l[0], l[1], l[2] };
                                u[a] -= 1;
                                u[b] -= db;
                                u[cc] -= dc;
                                if (u[0] < 0 || u[1] < 0 || u[2] < 0) continue;   // halo
                                ++reads;
                                bad += level[u[0] + 8 * (u[1] + 8 * u[2])] >= level[q];
                            }
                    }
                }
    std::printf("reads %%ld bad %%d\n", reads, bad);
    return bad != 0;
}
"""


def _section(src, start, end):
    a = src.index(start)
    return src[a:src.index(end, a)]


def test_level_order_is_a_topological_order():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = open(KERNELS).read()
    builder = _section(src, "constexpr int LEVEL_CLASSES", "__constant__ LevelOrder c_level_order")
    cls = _section(src, "__device__ __forceinline__ int level_class", "\n}\n") + "\n}\n"
    cls = cls.replace("__device__ __forceinline__ ", "static ").replace("max(", "std::max(")
    with tempfile.TemporaryDirectory() as d:
        cpp, exe = os.path.join(d, "lev.cpp"), os.path.join(d, "lev")
        with open(cpp, "w") as f:
            f.write(HARNESS % {"builder": builder, "classifier": cls})
        subprocess.run([gxx, "-std=c++17", "-O1", cpp, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout and "reads 0 " not in out.stdout
