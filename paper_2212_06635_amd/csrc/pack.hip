// Canonical complex128 spinors <-> internal site-major fields.
//
// Canonical one-parity field r of nvec: [cb][flavour][spin][colour], at an
// offset of r fields.  Internal multi-vector field: right-hand side r of
// site s sits in slot s * nvec + r of every component array, so a stencil
// thread per (site, rhs) reads a link once for all right-hand sides of a
// wavefront.  Full-lattice internal fields are the even field followed by
// the odd field.
#include "tmx_device.h"
#include "tmx_kernels.h"

namespace tmx {

template <int P>
__global__ void pack_kernel(const double *canon, SpinorPtr dst, int nf, int full, Geom g, int nvec, int unpack,
                            double *canon_out)
{
    using R = typename RealOf<P>::type;
    const long nsite = full ? 2L * g.Vh : (long)g.Vh;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsite * nvec) return;
    const long r = t / nsite;
    const long i = t - r * nsite;
    int parity = 1;
    long s;
    if (!full) {
        // canonical odd site i is the lexicographic site 2i or 2i + 1 that is odd
        int x[4];
        long q = 2 * i;
        x[0] = (int)(q % g.L[0]);
        q /= g.L[0];
        x[1] = (int)(q % g.L[1]);
        q /= g.L[1];
        x[2] = (int)(q % g.L[2]);
        x[3] = (int)(q / g.L[2]);
        if (((x[0] + x[1] + x[2] + x[3]) & 1) == 0) x[0] += 1;
        s = cb_index(g, x);
    } else {
        int x[4];
        long q = i;
        x[0] = (int)(q % g.L[0]);
        q /= g.L[0];
        x[1] = (int)(q % g.L[1]);
        q /= g.L[1];
        x[2] = (int)(q % g.L[2]);
        x[3] = (int)(q / g.L[2]);
        parity = (x[0] + x[1] + x[2] + x[3]) & 1;
        s = cb_index(g, x);
    }
    const SpinorPtr f = full ? parity_half(dst, P, nf, parity) : dst;
    const long slot = s * nvec + r;
    const long coff = (r * nsite + i) * 12 * nf;  // complex offset in the canonical field
    for (int fl = 0; fl < nf; ++fl) {
        cx<R> v[12];
        if (!unpack) {
            const double2 *c = reinterpret_cast<const double2 *>(canon) + coff + 12 * fl;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                double2 d = c[k];
                v[k] = cx<R>{(R)d.x, (R)d.y};
            }
            store_spinor<P>(f, fl, slot, v);
        } else {
            load_spinor<P>(f, fl, slot, v);
            double2 *c = reinterpret_cast<double2 *>(canon_out) + coff + 12 * fl;
#pragma unroll
            for (int k = 0; k < 12; ++k) c[k] = make_double2((double)v[k].re, (double)v[k].im);
        }
    }
}

static hipError_t pack_any(const double *canon, double *canon_out, SpinorPtr f, int prec, int kind, Geom g,
                           int nvec, int unpack, hipStream_t st)
{
    const int nf = (kind == 1 || kind == 3) ? 2 : 1;
    const int full = kind >= 2;
    const long n = (full ? 2L * g.Vh : (long)g.Vh) * nvec;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (prec == F64)
        hipLaunchKernelGGL(pack_kernel<F64>, grid, block, 0, st, canon, f, nf, full, g, nvec, unpack, canon_out);
    else if (prec == F32)
        hipLaunchKernelGGL(pack_kernel<F32>, grid, block, 0, st, canon, f, nf, full, g, nvec, unpack, canon_out);
    else
        hipLaunchKernelGGL(pack_kernel<F16>, grid, block, 0, st, canon, f, nf, full, g, nvec, unpack, canon_out);
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const double *canon, SpinorPtr dst, int prec, int kind, Geom g, int nvec,
                              hipStream_t st)
{
    return pack_any(canon, nullptr, dst, prec, kind, g, nvec, 0, st);
}

hipError_t launch_unpack_spinor(double *canon, SpinorPtr src, int prec, int kind, Geom g, int nvec, hipStream_t st)
{
    return pack_any(nullptr, canon, src, prec, kind, g, nvec, 1, st);
}

}  // namespace tmx
