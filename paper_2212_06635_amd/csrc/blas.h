// Site-parallel vector algebra on spinor fields with FP64 accumulation.
//
// Every operation is a functor applied to each slot (site x right-hand
// side) of the internal layout; values are widened to FP64, combined and
// narrowed back to each field's storage precision (FP16 fields get a fresh
// per-site scale).  Reductions (norms, inner products) are accumulated in
// FP64 per right-hand side: per-thread sums, a fixed-order tree in LDS per
// block, per-block partials in HBM and a fixed-order final pass, so a
// repeated call gives bit-identical results.
//
// Per right-hand-side scalars travel by value in the kernel arguments.
#pragma once

#include "tmx_device.h"

namespace tmx {

constexpr int MAXR = 32;  // right-hand sides / shifts per call

using cd = cx<double>;

template <int P>
__device__ __forceinline__ void ld(const SpinorPtr &f, int fl, long t, cd v[12])
{
    load_spinor<P>(f, fl, t, v);
}
template <int P>
__device__ __forceinline__ void st(const SpinorPtr &f, int fl, long t, const cd v[12])
{
    store_spinor<P>(f, fl, t, v);
}
__device__ __forceinline__ double nrm2(const cd v[12])
{
    double s = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) s += v[k].re * v[k].re + v[k].im * v[k].im;
    return s;
}

// ---------------------------------------------------------------------------
// functors
// ---------------------------------------------------------------------------

// x += a p ; r -= a q ; |r|^2
template <int PX, int PP, int PR, int PQ> struct OpAxpyNorm {
    static constexpr int NRED = 1;
    SpinorPtr x, p, r, q;
    int nf;
    double a[MAXR];
    const double *ad;  // if set: the coefficients in device memory instead of a
    __device__ void operator()(long t, int k, double *acc) const
    {
        const double ak = ad ? ad[k] : a[k];
        for (int f = 0; f < nf; ++f) {
            cd vx[12], vp[12], vr[12], vq[12];
            ld<PX>(x, f, t, vx);
            ld<PP>(p, f, t, vp);
            ld<PR>(r, f, t, vr);
            ld<PQ>(q, f, t, vq);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                vx[c] = vx[c] + ak * vp[c];
                vr[c] = vr[c] - ak * vq[c];
            }
            st<PX>(x, f, t, vx);
            st<PR>(r, f, t, vr);
            acc[0] += nrm2(vr);
        }
    }
};

// sum of a per-slot FP64 array (per right-hand side)
struct OpSlotSum {
    static constexpr int NRED = 1;
    const double *v;
    __device__ void operator()(long t, int, double *acc) const { acc[0] += v[t]; }
};

// r -= a q ; |r|^2
template <int PR, int PQ> struct OpRupdNorm {
    static constexpr int NRED = 1;
    SpinorPtr r, q;
    int nf;
    double a[MAXR];
    __device__ void operator()(long t, int k, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vr[12], vq[12];
            ld<PR>(r, f, t, vr);
            ld<PQ>(q, f, t, vq);
#pragma unroll
            for (int c = 0; c < 12; ++c) vr[c] = vr[c] - a[k] * vq[c];
            st<PR>(r, f, t, vr);
            acc[0] += nrm2(vr);
        }
    }
};

// y = a x + b y (real a, b per rhs).  A zero coefficient means the operand
// is not read (as in BLAS): y = a x overwrites y whatever it held, NaN
// included, so a fresh workspace can be its target.
template <int PY, int PX> struct OpAxpby {
    static constexpr int NRED = 0;
    SpinorPtr y, x;
    int nf;
    double a[MAXR], b[MAXR];
    __device__ void operator()(long t, int k, double *) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vy[12], vx[12];
            if (b[k] != 0.0) {
                ld<PY>(y, f, t, vy);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) vy[c] = cd{0.0, 0.0};
            }
            if (a[k] != 0.0) {
                ld<PX>(x, f, t, vx);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) vx[c] = cd{0.0, 0.0};
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) vy[c] = a[k] * vx[c] + b[k] * vy[c];
            st<PY>(y, f, t, vy);
        }
    }
};

// y += c x (complex c per rhs), optional |y|^2
template <int PY, int PX> struct OpCaxpy {
    static constexpr int NRED = 1;
    SpinorPtr y, x;
    int nf;
    double cre[MAXR], cim[MAXR];
    __device__ void operator()(long t, int k, double *acc) const
    {
        const cd c{cre[k], cim[k]};
        for (int f = 0; f < nf; ++f) {
            cd vy[12], vx[12];
            ld<PY>(y, f, t, vy);
            ld<PX>(x, f, t, vx);
#pragma unroll
            for (int i = 0; i < 12; ++i) cmac(vy[i], c, vx[i]);
            st<PY>(y, f, t, vy);
            acc[0] += nrm2(vy);
        }
    }
};

// d = s (precision conversion), |d|^2 of the source values
template <int PD, int PS> struct OpCopy {
    static constexpr int NRED = 1;
    SpinorPtr d, s;
    int nf;
    __device__ void operator()(long t, int, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd v[12];
            ld<PS>(s, f, t, v);
            st<PD>(d, f, t, v);
            acc[0] += nrm2(v);
        }
    }
};

// d = 0
template <int PD> struct OpZero {
    static constexpr int NRED = 0;
    SpinorPtr d;
    int nf;
    __device__ void operator()(long t, int, double *) const
    {
        cd v[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = cd{0, 0};
        for (int f = 0; f < nf; ++f) st<PD>(d, f, t, v);
    }
};

// x += y ; optionally y = 0
template <int PX, int PY> struct OpAddTo {
    static constexpr int NRED = 0;
    SpinorPtr x, y;
    int nf, zero_y;
    __device__ void operator()(long t, int, double *) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vx[12], vy[12];
            ld<PX>(x, f, t, vx);
            ld<PY>(y, f, t, vy);
#pragma unroll
            for (int c = 0; c < 12; ++c) vx[c] = vx[c] + vy[c];
            st<PX>(x, f, t, vx);
            if (zero_y) {
#pragma unroll
                for (int c = 0; c < 12; ++c) vy[c] = cd{0, 0};
                st<PY>(y, f, t, vy);
            }
        }
    }
};

// r = b - q ; |r|^2 ; optionally also write rlo = r in a second precision
template <int PR, int PB, int PQ, int PL> struct OpXmyNorm {
    static constexpr int NRED = 1;
    SpinorPtr r, b, q, rlo;
    int nf, write_lo;
    __device__ void operator()(long t, int, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vb[12], vq[12];
            ld<PB>(b, f, t, vb);
            ld<PQ>(q, f, t, vq);
#pragma unroll
            for (int c = 0; c < 12; ++c) vb[c] = vb[c] - vq[c];
            st<PR>(r, f, t, vb);
            if (write_lo) st<PL>(rlo, f, t, vb);
            acc[0] += nrm2(vb);
        }
    }
};

// <a, b> (complex): acc[0] = Re, acc[1] = Im
template <int PA, int PB> struct OpCdot {
    static constexpr int NRED = 2;
    SpinorPtr a, b;
    int nf;
    __device__ void operator()(long t, int, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd va[12], vb[12];
            ld<PA>(a, f, t, va);
            ld<PB>(b, f, t, vb);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cd s{0, 0};
                cmac_conj(s, va[c], vb[c]);
                acc[0] += s.re;
                acc[1] += s.im;
            }
        }
    }
};

// <a,b> complex and |b|^2 in one pass
template <int PA, int PB> struct OpCdotNorm {
    static constexpr int NRED = 3;
    SpinorPtr a, b;
    int nf;
    __device__ void operator()(long t, int, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd va[12], vb[12];
            ld<PA>(a, f, t, va);
            ld<PB>(b, f, t, vb);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cd s{0, 0};
                cmac_conj(s, va[c], vb[c]);
                acc[0] += s.re;
                acc[1] += s.im;
            }
            acc[2] += nrm2(vb);
        }
    }
};

// Multishift update after the residual update, for every active shift j:
//   x_j += alpha_j p_j ;  p_j = zeta_j r + beta_j p_j
// reading r once per site.
template <int PX, int PP, int PR> struct OpMsUpdate {
    static constexpr int NRED = 0;
    SpinorPtr r;
    void *xd[MAXR];
    void *pd[MAXR];
    long stride;
    int nf, nshift;
    double alpha[MAXR], zeta[MAXR], beta[MAXR];
    int active[MAXR];
    __device__ SpinorPtr mkf(void *d, int prec) const { return make_spinor(d, prec, nf, stride); }
    __device__ void operator()(long t, int, double *) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vr[12];
            ld<PR>(r, f, t, vr);
            for (int j = 0; j < nshift; ++j) {
                if (!active[j]) continue;
                const SpinorPtr X = mkf(xd[j], PX), Pp = mkf(pd[j], PP);
                cd vx[12], vp[12];
                ld<PX>(X, f, t, vx);
                ld<PP>(Pp, f, t, vp);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    vx[c] = vx[c] + alpha[j] * vp[c];
                    vp[c] = zeta[j] * vr[c] + beta[j] * vp[c];
                }
                st<PX>(X, f, t, vx);
                st<PP>(Pp, f, t, vp);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// generic kernels
// ---------------------------------------------------------------------------
template <class Op>
__global__ void __launch_bounds__(256) blas_kernel(Op op, long nslot, int nrhs, int m, double *partials)
{
    constexpr int NR = Op::NRED;
    double acc[NR > 0 ? NR : 1];
#pragma unroll
    for (int i = 0; i < (NR > 0 ? NR : 1); ++i) acc[i] = 0.0;
    const int k = threadIdx.x % nrhs;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nslot; t += stride) op(t, k, acc);
    if constexpr (NR > 0) {
        __shared__ double sh[NR][256];
#pragma unroll
        for (int i = 0; i < NR; ++i) sh[i][threadIdx.x] = acc[i];
        __syncthreads();
        for (int h = m / 2; h >= 1; h >>= 1) {
            if ((int)threadIdx.x < h * nrhs) {
#pragma unroll
                for (int i = 0; i < NR; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + h * nrhs];
            }
            __syncthreads();
        }
        if ((int)threadIdx.x < nrhs) {
#pragma unroll
            for (int i = 0; i < NR; ++i) partials[((long)blockIdx.x * nrhs + threadIdx.x) * NR + i] = sh[i][threadIdx.x];
        }
    }
}

// result[o] = sum_b partials[b * nout + o], fixed order (one block per output)
static __global__ void __launch_bounds__(256) blas_finish_kernel(const double *partials, int nblocks, int nout, double *result,
                                                                 double *host)
{
    __shared__ double sh[256];
    const int o = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[(long)b * nout + o];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[o] = sh[0];
        if (host) host[o] = sh[0];  // also straight into the host's readback buffer
    }
}

struct RedWork {
    double *partials;  // >= max_blocks * MAXR * 4 doubles
    double *result;    // >= MAXR * 4 doubles (device)
    double *host;      // device view of a coherent pinned host copy of result, or null
    int max_blocks;
};

// Launch op over nslot slots with nrhs right-hand sides interleaved; if the
// op reduces, result[k * NRED + i] (device) receives reduction i of rhs k.
template <class Op>
hipError_t run_blas(const Op &op, long nslot, int nrhs, const RedWork &w, hipStream_t st)
{
    if (nrhs < 1 || nrhs > MAXR) return hipErrorInvalidValue;
    int m = 1;
    while (2 * m * nrhs <= 256) m *= 2;
    const int block = m * nrhs;
    long nb = (nslot + block - 1) / block;
    if (nb > w.max_blocks) nb = w.max_blocks;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((blas_kernel<Op>), dim3((unsigned)nb), dim3(block), 0, st, op, nslot, nrhs, m, w.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (Op::NRED > 0) {
        const int nout = nrhs * Op::NRED;
        hipLaunchKernelGGL(blas_finish_kernel, dim3(nout), dim3(256), 0, st, w.partials, (int)nb, nout, w.result,
                           w.host);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace tmx
