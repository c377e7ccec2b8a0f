// Hopping-term force of the Schur operator (gfx950).
//
// For odd fields X, Y the link derivative of S = Re<Y, Mhat(s) X> through the
// hopping terms H_oe and H_eo (site blocks fixed), for U_mu(x) ->
// exp(i eps T) U_mu(x), is dS/d eps = Re Tr[i T F_mu(x)] with F = TA(Q),
//
//   Q_mu(x) = -kappa^2 bc U_mu(x) [ sum_s ((1 - g_mu) b(x+mu))_s a(x)_s^dagger
//                                  + sum_s ((1 + g_mu) a(x+mu))_s b(x)_s^dagger ],
//
// where on the full lattice b = X (odd) | u = B_ee(s)^{-1} H_eo X (even) and
// a = Y (odd) | w = B_ee(-s)^{-1} g5 H_eo g5 Y (even): every link takes one
// forward outer product from one of the two hopping terms and one backward
// from the other.  w = g5 K1(-s, g5 in)(Y) since the site blocks commute with
// g5.  The outer products are the building block of the fermion force of the
// rational monomials (Section 4.3), which sums them over the shifts.
#include "tmx_device.h"
#include "tmx_kernels.h"

namespace tmx {

using cd = cx<double>;

// (g_mu psi) in the chiral basis: upper = a_mu psi_lower, lower = a_mu^dagger
// psi_upper, a_k = -i sigma_k, a_4 = 1 (the blocks of the stencil's spin
// projection)
template <int MU> __device__ __forceinline__ void gamma_mul(const cd *p, cd *o)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cd p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if constexpr (MU == 0) {  // a = [[0, -i], [-i, 0]], a^dagger = [[0, i], [i, 0]]
            o[c] = -imul(p3);
            o[3 + c] = -imul(p2);
            o[6 + c] = imul(p1);
            o[9 + c] = imul(p0);
        } else if constexpr (MU == 1) {  // a = [[0, -1], [1, 0]], a^dagger = [[0, 1], [-1, 0]]
            o[c] = -p3;
            o[3 + c] = p2;
            o[6 + c] = p1;
            o[9 + c] = -p0;
        } else if constexpr (MU == 2) {  // a = [[-i, 0], [0, i]], a^dagger = [[i, 0], [0, -i]]
            o[c] = -imul(p2);
            o[3 + c] = imul(p3);
            o[6 + c] = imul(p0);
            o[9 + c] = -imul(p1);
        } else {  // a = 1
            o[c] = p2;
            o[3 + c] = p3;
            o[6 + c] = p0;
            o[9 + c] = p1;
        }
    }
}

__device__ __forceinline__ void load_g5(const SpinorPtr &f, long s, bool g5, cd v[12])
{
    load_spinor<F64>(f, 0, s, v);
    if (g5) {
#pragma unroll
        for (int k = 6; k < 12; ++k) v[k] = -v[k];
    }
}

// M += sum_s (p_s) (q_s)^dagger  (colour outer product summed over spin)
__device__ __forceinline__ void outer_acc(const cd *p, const cd *q, cd M[9])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int s = 0; s < 4; ++s) cmac_conj(M[3 * i + j], q[3 * s + j], p[3 * s + i]);
}

template <int MU>
__device__ __forceinline__ void force_link(const ForceArgs &f, const int x[4], int p, const cd ax[12], const cd bx[12],
                                           long lex)
{
    const Geom &g = f.g;
    int y[4] = {x[0], x[1], x[2], x[3]};
    double bc = 1.0;
    if (++y[MU] == g.L[MU]) {
        y[MU] = 0;
        if (MU == 3) bc = f.t_bc;
    }
    const int n = cb_index(g, y);
    const int q = 1 - p;
    cd M[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = cd{0, 0};
    {
        // ((1 - g_mu) b(x+mu)) a(x)^dagger
        cd by[12], gb[12];
        if (q == 1)
            load_g5(f.X, n, false, by);
        else
            load_g5(f.u, n, false, by);
        gamma_mul<MU>(by, gb);
#pragma unroll
        for (int k = 0; k < 12; ++k) by[k] = by[k] - gb[k];
        outer_acc(by, ax, M);
    }
    {
        // ((1 + g_mu) a(x+mu)) b(x)^dagger
        cd ay[12], ga[12];
        if (q == 1)
            load_g5(f.Y, n, false, ay);
        else
            load_g5(f.w, n, true, ay);
        gamma_mul<MU>(ay, ga);
#pragma unroll
        for (int k = 0; k < 12; ++k) ay[k] = ay[k] + ga[k];
        outer_acc(ay, bx, M);
    }
    cd u[9];
    load_link<F64>(f.U, p, MU, cb_index(g, x), u);
    // Q = -kappa^2 bc U M, F = TA(Q)
    const double fac = -f.kfac * bc;
    cd Q[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, u[3 * i + k], M[3 * k + j]);
            Q[3 * i + j] = fac * s;
        }
    double tr = 0.0;  // imaginary part of the trace of the anti-Hermitian part
#pragma unroll
    for (int i = 0; i < 3; ++i) tr += Q[4 * i].im;
    double2 *o = reinterpret_cast<double2 *>(f.out) + (lex * 4 + MU) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // (Q - Q^dagger) / 2 minus its trace / 3 on the diagonal
            cd a{0.5 * (Q[3 * i + j].re - Q[3 * j + i].re), 0.5 * (Q[3 * i + j].im + Q[3 * j + i].im)};
            if (i == j) a.im -= tr / 3.0;
            cd v{f.coeff * a.re, f.coeff * a.im};
            if (f.accumulate) {
                const double2 old = o[3 * i + j];
                v.re += old.x;
                v.im += old.y;
            }
            o[3 * i + j] = make_double2(v.re, v.im);
        }
}

// Workgroups alternate between the parities (workgroup 2i + p: sites
// 256 i ... of parity p), so the contiguous workgroup range of an XCD holds
// both parities of one region and the neighbours of its sites are read
// through its own L2.
__global__ void __launch_bounds__(256) hop_force_kernel(ForceArgs f)
{
    const long blk = xcd_block(f.xcd);
    const int p = (int)(blk & 1);
    const long st = (blk >> 1) * blockDim.x + threadIdx.x;
    if (st >= f.g.Vh) return;
    const int s = (int)st;
    int x[4];
    cb_coords(f.g, s, p, x);
    const long lex = x[0] + (long)f.g.L[0] * (x[1] + (long)f.g.L[1] * (x[2] + (long)f.g.L[2] * x[3]));
    cd ax[12], bx[12];
    if (p == 1) {
        load_g5(f.Y, s, false, ax);
        load_g5(f.X, s, false, bx);
    } else {
        load_g5(f.w, s, true, ax);
        load_g5(f.u, s, false, bx);
    }
    force_link<0>(f, x, p, ax, bx, lex);
    force_link<1>(f, x, p, ax, bx, lex);
    force_link<2>(f, x, p, ax, bx, lex);
    force_link<3>(f, x, p, ax, bx, lex);
}

hipError_t launch_hop_force(const ForceArgs &f, hipStream_t st)
{
    const long vh = f.g.Vh;
    if (vh == 0) return hipSuccess;
    const int block = 256;
    const long nblk = 2 * ((vh + block - 1) / block);  // both parities, interleaved
    hipLaunchKernelGGL(hop_force_kernel, dim3((unsigned)nblk), dim3(block), 0, st, f);
    return hipGetLastError();
}

}  // namespace tmx
