"""Host check of the block order the clover-force kernels visit sites in
(order_block in csrc/block_order.h): a permutation of the site blocks for every
lattice, the plain order where the (x, y) planes do not split into chunks.
The header's host/device function is compiled for the host only and run on
the CPU; a wrong permutation would drop or repeat sites of the force."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2212_06635_amd", "csrc")
INC = os.path.join(HERE, "..", "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r"""
#include "block_order.h"
#include <cstdio>
#include <vector>
int main()
{
    const int dims[][4] = {{32, 32, 32, 64}, {64, 64, 64, 128}, {16, 16, 16, 32}, {16, 16, 16, 128},
                           {24, 24, 24, 48}, {8, 8, 8, 8}, {6, 4, 2, 10}, {4, 4, 2, 6}};
    for (auto &d : dims) {
        tmx::Geom g{};
        for (int k = 0; k < 4; ++k) g.L[k] = d[k];
        g.Lxh = d[0] / 2;
        g.Vh = d[0] * d[1] * d[2] * d[3] / 2;
        for (int B : {64, 256}) {
            const long nb = (g.Vh + B - 1) / B;
            std::vector<int> seen(nb, 0);
            bool moved = false;
            for (long i = 0; i < nb; ++i) {
                const long j = tmx::order_block(g, i, B);
                if (j < 0 || j >= nb || seen[j]++) {
                    std::printf("%dx%dx%dx%d B=%d not a permutation\n", d[0], d[1], d[2], d[3], B);
                    return 1;
                }
                moved = moved || j != i;
            }
            std::printf("%dx%dx%dx%d %d %s\n", d[0], d[1], d[2], d[3], B, moved ? "reordered" : "plain");
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def order_table(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("block_order")
    src, exe = os.path.join(d, "check.cpp"), os.path.join(d, "check")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.run([HIPCC, "--offload-host-only", "-std=c++17", "-O1", "-I", CSRC, "-I", INC, src, "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    return {(l.split()[0], int(l.split()[1])): l.split()[2] for l in out if l.strip()}


def test_block_order_is_a_permutation(order_table):
    assert len(order_table) == 16


@pytest.mark.parametrize("lattice,block", [("32x32x32x64", 64), ("32x32x32x64", 256), ("64x64x64x128", 64),
                                           ("64x64x64x128", 256), ("16x16x16x32", 64)])
def test_block_order_active_at_production_sizes(order_table, lattice, block):
    assert order_table[(lattice, block)] == "reordered"


@pytest.mark.parametrize("lattice,block", [("8x8x8x8", 64), ("6x4x2x10", 64), ("4x4x2x6", 256),
                                           ("24x24x24x48", 64), ("16x16x16x32", 256)])
def test_block_order_plain_where_planes_do_not_split(order_table, lattice, block):
    assert order_table[(lattice, block)] == "plain"
