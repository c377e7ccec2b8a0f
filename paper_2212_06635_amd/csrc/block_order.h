// Site-block order of the force kernels (force.hip); host-callable so that
// a CPU test can check that it permutes the blocks.
#pragma once
#include "tmx_device.h"

namespace tmx {

// Order in which a kernel visits blocks of B sites of one parity.  The site
// order runs x, y fastest, then the (z, t) planes, so a site's z and t
// neighbours lie one or more whole planes away; a kernel that reads enough
// bytes per site has evicted them from L2 by the time the neighbouring block
// reads them again.  Within each eighth of the planes (the share of one XCD,
// with the XCD-contiguous workgroup order) the blocks are visited chunk by
// chunk: the first CH sites (whole rows of x) of every plane, then the next
// CH of every plane, so z and t neighbours are read a few blocks apart in
// time (y neighbours across a chunk edge, and t neighbours across an eighth,
// are not).  CH = max(B, 8 Lx/2); lattices whose planes do not split that
// way keep the plain order.  A permutation of the blocks in every case.
__host__ __device__ __forceinline__ long order_block(const Geom &g, long ib, int B)
{
    const int ps = g.Lxh * g.L[1];  // sites of one parity in an (x, y) plane
    const int ch = B > 8 * g.Lxh ? B : 8 * g.Lxh;
    const int np = g.Vh / ps;  // planes
    if (ch % B != 0 || ps % ch != 0 || np % 8 != 0) return ib;
    const long bpc = ch / B, cpp = ps / ch, G = np / 8;
    const long gs = G * cpp * bpc;
    const long grp = ib / gs, j = ib - grp * gs;
    const long b = j % bpc, pl = (j / bpc) % G, c = j / (bpc * G);
    return grp * gs + (pl * cpp + c) * bpc + b;
}

}  // namespace tmx
