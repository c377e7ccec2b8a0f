// Fermion-force building blocks of the Schur operator (gfx950): the hopping-
// term force, then (further down) the clover-term force.
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
#include "force.h"

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

// ---------------------------------------------------------------------------
// clover-term force
// ---------------------------------------------------------------------------
// The clover term T = i kappa csw sum_{mu<nu} sigma_mu,nu F_mu,nu sits on the
// odd sites (A_oo, weight 1) and inside A_ee^{-1} (weight kappa^2, sign from
// the derivative of the inverse), so with b, a as for the hopping force and
// c = 1 (odd) | kappa^2 (even)
//   dS = Re sum_{z, rho != nu} (i kappa csw / 8) Tr[dQ_rho,nu(z) H_rho,nu(z)],
//   H = G + G^dagger,  G_rho,nu(z) = c sum_s (sigma_rho,nu b(z))_s a(z)_s^dagger,
// Q the four plaquette leaves at z in the (rho, nu) plane.  A link U_rho(y)
// lies in two plaquettes of each plane (rho, nu) oriented rho -> nu, the one
// above it (through U) and the one below (through U^dagger), and enters the
// leaves of all four of their corners: with C_up / E_low the plaquette
// products opened at U / U^dagger with H inserted at each corner in turn,
//   F_rho(y) = TA[(i kappa csw / 8) sum_nu (U C_up - E_low U^dagger)].
// H_nu,rho = -H_rho,nu (sigma is antisymmetric), so six planes are stored.
namespace {

struct Mat3 {
    cd m[9];
};

__device__ __forceinline__ Mat3 mm(const Mat3 &a, const Mat3 &b)  // a b
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a.m[3 * i + k], b.m[3 * k + j]);
            c.m[3 * i + j] = s;
        }
    return c;
}

__device__ __forceinline__ Mat3 mm_nd(const Mat3 &a, const Mat3 &b)  // a b^dagger
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_conj(s, b.m[3 * j + k], a.m[3 * i + k]);
            c.m[3 * i + j] = s;
        }
    return c;
}

__device__ __forceinline__ Mat3 mm_dn(const Mat3 &a, const Mat3 &b)  // a^dagger b
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_conj(s, a.m[3 * k + i], b.m[3 * k + j]);
            c.m[3 * i + j] = s;
        }
    return c;
}

__device__ __forceinline__ void add_to(Mat3 &a, const Mat3 &b)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) a.m[k] = a.m[k] + b.m[k];
}

// stored plane of the pair r < n: xy, xz, xt, yz, yt, zt
__device__ __forceinline__ int plane_of(int r, int n) { return r == 0 ? n - 1 : (r == 1 ? n + 1 : 5); }

__device__ __forceinline__ void shift(const Geom &g, const int x[4], int mu, int d, int y[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] += d;
    if (y[mu] < 0) y[mu] += g.L[mu];
    if (y[mu] >= g.L[mu]) y[mu] -= g.L[mu];
}

__device__ __forceinline__ Mat3 link(const CloverForceArgs &f, const int x[4], int mu)
{
    Mat3 u;
    load_link<F64>(f.U, (x[0] + x[1] + x[2] + x[3]) & 1, mu, cb_index(f.g, x), u.m);
    return u;
}

// H_r,n at site x (r != n): the stored plane, negated for r > n
__device__ __forceinline__ Mat3 insertion(const CloverForceArgs &f, const int x[4], int r, int n)
{
    const long V2 = 2L * f.g.Vh;
    const long site = (long)((x[0] + x[1] + x[2] + x[3]) & 1) * f.g.Vh + cb_index(f.g, x);
    const double2 *h = f.H + (long)plane_of(r < n ? r : n, r < n ? n : r) * 9 * V2 + site;
    const double sg = r < n ? 1.0 : -1.0;
    Mat3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = h[k * V2];
        m.m[k] = cd{sg * v.x, sg * v.y};
    }
    return m;
}

// P_m^chi = sum_{s,t} (s_m)_{st} b_t a_s^dagger over the two spins 2 chi,
// 2 chi + 1 of one chirality (s_m the Pauli matrix, a colour matrix)
template <int M>
__device__ __forceinline__ void pauli_outer(const cd a[12], const cd b[12], int chi, Mat3 &P)
{
    const int s0 = 2 * chi, s1 = 2 * chi + 1;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cd a0 = conj(a[3 * s0 + j]), a1 = conj(a[3 * s1 + j]);
            const cd b0 = b[3 * s0 + i], b1 = b[3 * s1 + i];
            cd v;
            if constexpr (M == 1)
                v = b1 * a0 + b0 * a1;
            else if constexpr (M == 2)
                v = imul(b0 * a1 - b1 * a0);
            else
                v = b0 * a0 - b1 * a1;
            P.m[3 * i + j] = v;
        }
}

__device__ __forceinline__ void store_insertion(const CloverForceArgs &f, int plane, long site, double c,
                                                const Mat3 &G)
{
    const long V2 = 2L * f.g.Vh;
    double2 *h = f.H + (long)plane * 9 * V2 + site;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // c (G + G^dagger), summed over the flavours of a two-flavour field
            const cd v = G.m[3 * i + j] + conj(G.m[3 * j + i]);
            double2 o = make_double2(c * v.re, c * v.im);
            if (f.h_acc) {
                const double2 old = h[(3 * i + j) * V2];
                o.x += old.x;
                o.y += old.y;
            }
            h[(3 * i + j) * V2] = o;
        }
}

// sigma_kl = -eps_klm diag(s_m, s_m), sigma_k4 = diag(s_k, -s_k): the
// spatial plane opposite m takes -eps (P_m^0 + P_m^1), the (m, t) plane
// P_m^0 - P_m^1
template <int M>
__device__ __forceinline__ void planes_of(const CloverForceArgs &f, const cd a[12], const cd b[12], long site,
                                          double c)
{
    Mat3 P0, P1, G;
    pauli_outer<M>(a, b, 0, P0);
    pauli_outer<M>(a, b, 1, P1);
    // G_yz = -(P_1^0 + P_1^1), G_xz = P_2^0 + P_2^1, G_xy = -(P_3^0 + P_3^1)
    const double se = M == 2 ? 1.0 : -1.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) G.m[k] = se * (P0.m[k] + P1.m[k]);
    store_insertion(f, M == 1 ? 3 : (M == 2 ? 1 : 0), site, c, G);
#pragma unroll
    for (int k = 0; k < 9; ++k) G.m[k] = P0.m[k] - P1.m[k];
    store_insertion(f, M == 1 ? 2 : (M == 2 ? 4 : 5), site, c, G);
}

__global__ void __launch_bounds__(256) clover_insertion_kernel(CloverForceArgs f)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2L * f.g.Vh) return;
    const int p = (int)(t / f.g.Vh);
    const int s = (int)(t - (long)p * f.g.Vh);
    cd a[12], b[12];
    if (p == 1) {
        load_g5(f.Y, s, false, a);
        load_g5(f.X, s, false, b);
    } else {
        load_g5(f.w, s, true, a);
        load_g5(f.u, s, false, b);
    }
    const double c = p == 1 ? 1.0 : f.kfac;
    planes_of<1>(f, a, b, t, c);
    planes_of<2>(f, a, b, t, c);
    planes_of<3>(f, a, b, t, c);
}

template <int R>
__device__ __forceinline__ void clover_link(const CloverForceArgs &f, const int y[4], long lex)
{
    Mat3 Z;
#pragma unroll
    for (int k = 0; k < 9; ++k) Z.m[k] = cd{0, 0};
    int yr[4];
    shift(f.g, y, R, +1, yr);
    const Mat3 ur = link(f, y, R);
#pragma unroll 1
    for (int n = 0; n < 4; ++n) {
        if (n == R) continue;
        int yn[4], yrn[4], ymn[4], ymnr[4];
        shift(f.g, y, n, +1, yn);
        shift(f.g, yr, n, +1, yrn);
        shift(f.g, y, n, -1, ymn);
        shift(f.g, ymn, R, +1, ymnr);
        const Mat3 h0 = insertion(f, y, R, n), h1 = insertion(f, yr, R, n);
        {
            // above: y -> y+r -> y+r+n -> y+n -> y, opened at U_r(y):
            // a1 = U_n(y+r), a2 = U_r(y+n)^dagger, a3 = U_n(y)^dagger
            const Mat3 a1 = link(f, yr, n), ur_n = link(f, yn, R), un = link(f, y, n);
            const Mat3 a12 = mm_nd(a1, ur_n);
            const Mat3 B = mm_nd(a12, un);
            Mat3 C = mm(B, h0);
            add_to(C, mm(h1, B));
            add_to(C, mm_nd(mm(a1, insertion(f, yrn, R, n)), mm(un, ur_n)));  // a1 h a2 a3
            add_to(C, mm_nd(mm(a12, insertion(f, yn, R, n)), un));            // a1 a2 h a3
            add_to(Z, mm(ur, C));
        }
        {
            // below: y-n -> y-n+r -> y+r -> y -> y-n, closed by U_r(y)^dagger:
            // d1 = U_n(y-n)^dagger, d2 = U_r(y-n), d3 = U_n(y-n+r)
            const Mat3 d1 = link(f, ymn, n), d2 = link(f, ymn, R), d3 = link(f, ymnr, n);
            const Mat3 d23 = mm(d2, d3);
            const Mat3 D = mm_dn(d1, d23);
            Mat3 E = mm(D, h1);
            add_to(E, mm(h0, D));
            add_to(E, mm_dn(d1, mm(insertion(f, ymn, R, n), d23)));            // d1 h d2 d3
            add_to(E, mm(mm(mm_dn(d1, d2), insertion(f, ymnr, R, n)), d3));    // d1 d2 h d3
            const Mat3 EU = mm_nd(E, ur);
#pragma unroll
            for (int k = 0; k < 9; ++k) Z.m[k] = Z.m[k] - EU.m[k];
        }
    }
    // Q = i (kappa csw / 8) Z, F = TA(Q)
    cd Q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Q[k] = f.kc8 * imul(Z.m[k]);
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) tr += Q[4 * i].im;
    double2 *o = reinterpret_cast<double2 *>(f.out) + (lex * 4 + R) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
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

// One thread per link.  Workgroup 8 i + 4 p + rho takes direction rho of
// sites 256 i ... of parity p: the four directions and both parities of one
// site block are neighbouring workgroups (with the XCD remap, on one XCD),
// so the insertions and links of their common staples are read through one
// L2 instead of once per direction.
__global__ void __launch_bounds__(256) clover_force_kernel(CloverForceArgs f)
{
    const long blk = xcd_block(f.xcd);
    const int r = (int)(blk & 3);
    const int p = (int)((blk >> 2) & 1);
    const long st = (blk >> 3) * blockDim.x + threadIdx.x;
    if (st >= f.g.Vh) return;
    int x[4];
    cb_coords(f.g, (int)st, p, x);
    const long lex = x[0] + (long)f.g.L[0] * (x[1] + (long)f.g.L[1] * (x[2] + (long)f.g.L[2] * x[3]));
    switch (r) {
    case 0: clover_link<0>(f, x, lex); break;
    case 1: clover_link<1>(f, x, lex); break;
    case 2: clover_link<2>(f, x, lex); break;
    default: clover_link<3>(f, x, lex); break;
    }
}

}  // namespace

hipError_t launch_clover_insertions(const CloverForceArgs &f, hipStream_t st)
{
    const long n = 2L * f.g.Vh;
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(clover_insertion_kernel, dim3(nb), dim3(256), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_clover_link_sums(const CloverForceArgs &f, hipStream_t st)
{
    if (f.g.Vh == 0) return hipSuccess;
    const long nlink = 8 * ((f.g.Vh + 255) / 256);  // 4 directions x 2 parities per site block
    hipLaunchKernelGGL(clover_force_kernel, dim3((unsigned)nlink), dim3(256), 0, st, f);
    return hipGetLastError();
}

}  // namespace tmx
