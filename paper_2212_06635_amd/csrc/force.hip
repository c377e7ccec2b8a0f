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
#include "block_order.h"

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
// Three kernels: the insertions per site, the loops per plaquette (each
// plaquette once, not once per link), and the link sums, which take the
// loops of a link's six plaquettes from the stored ones by conjugation.
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
__device__ __forceinline__ constexpr int plane_of(int r, int n) { return r == 0 ? n - 1 : (r == 1 ? n + 1 : 5); }

__device__ __forceinline__ void shift(const Geom &g, const int x[4], int mu, int d, int y[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] += d;
    if (y[mu] < 0) y[mu] += g.L[mu];
    if (y[mu] >= g.L[mu]) y[mu] -= g.L[mu];
}

// Insertions are Hermitian, so a plane stores nine reals per site, each
// component an array of 2 Vh doubles (site index p Vh + s): the diagonal
// H00, H11, H22, then (re, im) of H01, H02, H12.
__device__ __forceinline__ int herm_component(int i, int j)  // first real of entry (i, j), i <= j
{
    return i == j ? i : 3 + 2 * (i + j - 1);
}

// the Pauli combinations of one chirality chi at colour entry (i, j):
// P_m^chi = sum_{s,t} (s_m)_{st} b_t a_s^dagger over spins 2 chi, 2 chi + 1
// (s_m the Pauli matrices; a colour matrix per m), all three m from the four
// spin products of that entry
__device__ __forceinline__ void pauli_entry(const cd a[12], const cd b[12], int chi, int i, int j, cd P[3])
{
    const int s0 = 2 * chi, s1 = 2 * chi + 1;
    const cd a0 = conj(a[3 * s0 + j]), a1 = conj(a[3 * s1 + j]);
    const cd b0 = b[3 * s0 + i], b1 = b[3 * s1 + i];
    const cd b0a0 = b0 * a0, b0a1 = b0 * a1, b1a0 = b1 * a0, b1a1 = b1 * a1;
    P[0] = b1a0 + b0a1;          // s_1
    P[1] = imul(b0a1 - b1a0);    // s_2
    P[2] = b0a0 - b1a1;          // s_3
}

template <bool HACC>
__device__ __forceinline__ void put_real(const CloverForceArgs &f, int plane, long site, int k, double v)
{
    const long V2 = 2L * f.g.Vh;
    double *h = f.H + ((long)plane * 9 + k) * V2 + site;
    if constexpr (HACC) v += *h;  // the next flavour of a two-flavour field adds its part
    *h = v;
}

// entry (i, j), i <= j, of the Hermitian insertion of a plane (the diagonal is real)
template <bool HACC>
__device__ __forceinline__ void put_insertion(const CloverForceArgs &f, int plane, long site, int i, int j, cd v)
{
    const int c = herm_component(i, j);
    put_real<HACC>(f, plane, site, c, v.re);
    if (i != j) put_real<HACC>(f, plane, site, c + 1, v.im);
}

// sigma_kl = -eps_klm diag(s_m, s_m), sigma_k4 = diag(s_k, -s_k): the
// spatial plane opposite m takes G = -eps (P_m^0 + P_m^1), the (m, t) plane
// G = P_m^0 - P_m^1, and H = c (G + G^dagger).  One unordered colour pair
// (i, j) at a time, all six planes from its products (H_ji = conj(H_ij) is
// not stored), so that only the site's two spinors stay live.
template <bool HACC>
__device__ __forceinline__ void all_planes(const CloverForceArgs &f, const cd a[12], const cd b[12], long site,
                                           double c)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            cd p0[3], p1[3], q0[3], q1[3];
            pauli_entry(a, b, 0, i, j, p0);
            pauli_entry(a, b, 1, i, j, p1);
            pauli_entry(a, b, 0, j, i, q0);
            pauli_entry(a, b, 1, j, i, q1);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double se = m == 1 ? 1.0 : -1.0;
                const int ps = m == 0 ? 3 : (m == 1 ? 1 : 0), pt = m == 0 ? 2 : (m == 1 ? 4 : 5);
                const cd hs = c * (se * (p0[m] + p1[m]) + conj(se * (q0[m] + q1[m])));
                const cd ht = c * ((p0[m] - p1[m]) + conj(q0[m] - q1[m]));
                put_insertion<HACC>(f, ps, site, i, j, hs);
                put_insertion<HACC>(f, pt, site, i, j, ht);
            }
        }
}

template <bool HACC>
__global__ void __launch_bounds__(256) clover_insertion_kernel(CloverForceArgs f)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2L * f.g.Vh) return;
    const int p = (int)(t / f.g.Vh);
    const int s = (int)(t - (long)p * f.g.Vh);
    // odd sites: a = Y, b = X; even sites: a = g5 w, b = u (one load of each)
    cd a[12], b[12];
    load_g5(p == 1 ? f.Y : f.w, s, p != 1, a);
    load_g5(p == 1 ? f.X : f.u, s, false, b);
    const double c = p == 1 ? 1.0 : f.kfac;
    all_planes<HACC>(f, a, b, t, c);
}

__device__ __forceinline__ Mat3 dagm(const Mat3 &a)
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.m[3 * i + j] = conj(a.m[3 * j + i]);
    return c;
}

// ---- plaquette loops --------------------------------------------------------
// Per plaquette (x; r < n) with links a = U_r(x), b = U_n(x+r), c = U_r(x+n),
// d = U_n(x) and the (r, n) insertions h0..h3 at its corners x, x+r, x+r+n,
// x+n, the loop opened at x with each corner's insertion in turn,
//     X = a h1 b c+ d+ + a b h2 c+ d+ + a b c+ h3 d+ + a b c+ d+ h0,
// and the plain loop W = a b c+ d+.  The force takes only the Hermitian part
// K = (X + X+)/2 of X and the anti-Hermitian part A = (W - W+)/2 of W (the
// link sums below), and of those only the traceless parts: eight reals each.
//
// The loop opened at the next corner is the conjugate L+ X L (L the link
// between the two corners) plus the commutator [W', h'] of the new corner's
// plain loop and insertion: conjugation moves the insertion of the old open
// corner to the inside of the loop, but leaves the new corner's at the front
// instead of the back.  Every loop a link force needs is such a rotation of
// one stored plaquette (see the link sums).
//
// Hermitian and anti-Hermitian matrices are held as nine reals: the diagonal
// (real part of K, imaginary part of A), then the upper triangle (0,1), (0,2),
// (1,2) as (re, im); K_ji = conj(K_ij), A_ji = -conj(A_ij).  In memory each
// real is its own array of 2 Vh doubles: all nine of an insertion, eight of
// a traceless loop part (the third diagonal entry is minus the other two).
struct Sym3 {
    double d[3];
    cd o[3];
};

__device__ __forceinline__ constexpr int upper(int i, int j) { return i + j - 1; }  // i < j

__device__ __forceinline__ cd herm_get(const Sym3 &k, int i, int j)  // i != j
{
    const cd v = k.o[upper(i < j ? i : j, i < j ? j : i)];
    return i < j ? v : conj(v);
}

__device__ __forceinline__ cd aherm_get(const Sym3 &a, int i, int j)  // i != j
{
    const cd v = a.o[upper(i < j ? i : j, i < j ? j : i)];
    return i < j ? v : cd{-v.re, v.im};
}

__device__ __forceinline__ Sym3 load_sym(const double *p, long V2, long site)
{
    Sym3 k;
#pragma unroll
    for (int i = 0; i < 3; ++i) k.d[i] = p[i * V2 + site];
#pragma unroll
    for (int i = 0; i < 3; ++i) k.o[i] = cd{p[(3 + 2 * i) * V2 + site], p[(4 + 2 * i) * V2 + site]};
    return k;
}

// traceless part as eight reals (d0, d1 of the traceless diagonal, then the
// upper triangle): the trace of K and of A never reaches the force (it only
// adds to tr Z, which the projection removes, or commutes away)
__device__ __forceinline__ Sym3 load_tl(const double *p, long V2, long site)
{
    Sym3 k;
    k.d[0] = p[site];
    k.d[1] = p[V2 + site];
    k.d[2] = -(k.d[0] + k.d[1]);
#pragma unroll
    for (int i = 0; i < 3; ++i) k.o[i] = cd{p[(2 + 2 * i) * V2 + site], p[(3 + 2 * i) * V2 + site]};
    return k;
}

// written once, read by the link sums of the next kernel: streamed past L2
// (non-temporal), which keeps the links and insertions the neighbouring
// plaquettes share in it
__device__ __forceinline__ void store_tl(double *p, long V2, long site, const Sym3 &k)
{
    const double t3 = (k.d[0] + k.d[1] + k.d[2]) / 3.0;
    __builtin_nontemporal_store(k.d[0] - t3, p + site);
    __builtin_nontemporal_store(k.d[1] - t3, p + V2 + site);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        __builtin_nontemporal_store(k.o[i].re, p + (2 + 2 * i) * V2 + site);
        __builtin_nontemporal_store(k.o[i].im, p + (3 + 2 * i) * V2 + site);
    }
}

__device__ __forceinline__ long site_of(const Geom &g, const int x[4])
{
    return (long)((x[0] + x[1] + x[2] + x[3]) & 1) * g.Vh + cb_index(g, x);
}

// link through the caches (neighbouring plaquettes and links share it)
__device__ __forceinline__ Mat3 link_c(const CloverForceArgs &f, const int x[4], int mu)
{
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const double2 *b = static_cast<const double2 *>(f.U.d) + (long)(p * 4 + mu) * 6 * f.U.Vh + cb_index(f.g, x);
    Mat3 u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 v = b[k * f.U.Vh];
        u.m[k] = cd{v.x, v.y};
    }
    // the third row of an SU(3) matrix: conj(row 0 x row 1)
    u.m[6] = conj(u.m[1] * u.m[5] - u.m[2] * u.m[4]);
    u.m[7] = conj(u.m[2] * u.m[3] - u.m[0] * u.m[5]);
    u.m[8] = conj(u.m[0] * u.m[4] - u.m[1] * u.m[3]);
    return u;
}

__device__ __forceinline__ Mat3 hmul(const Sym3 &h, const Mat3 &m)  // h m, h Hermitian
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s = h.d[i] * m.m[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k != i) cmac(s, herm_get(h, i, k), m.m[3 * k + j]);
            c.m[3 * i + j] = s;
        }
    return c;
}

__device__ __forceinline__ Mat3 mulh(const Mat3 &m, const Sym3 &h)  // m h, h Hermitian
{
    Mat3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s = h.d[j] * m.m[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k != j) cmac(s, m.m[3 * i + k], herm_get(h, k, j));
            c.m[3 * i + j] = s;
        }
    return c;
}

// Hermitian part of a t
__device__ __forceinline__ Sym3 herm_of_product(const Mat3 &a, const Mat3 &t)
{
    Sym3 k;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += a.m[3 * i + l].re * t.m[3 * l + i].re - a.m[3 * i + l].im * t.m[3 * l + i].im;
        k.d[i] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            cd xij{0, 0}, xji{0, 0};
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                cmac(xij, a.m[3 * i + l], t.m[3 * l + j]);
                cmac(xji, a.m[3 * j + l], t.m[3 * l + i]);
            }
            k.o[upper(i, j)] = cd{0.5 * (xij.re + xji.re), 0.5 * (xij.im - xji.im)};
        }
    return k;
}

// anti-Hermitian part of a t
__device__ __forceinline__ Sym3 aherm_of_product(const Mat3 &a, const Mat3 &t)
{
    Sym3 k;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += a.m[3 * i + l].re * t.m[3 * l + i].im + a.m[3 * i + l].im * t.m[3 * l + i].re;
        k.d[i] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            cd xij{0, 0}, xji{0, 0};
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                cmac(xij, a.m[3 * i + l], t.m[3 * l + j]);
                cmac(xji, a.m[3 * j + l], t.m[3 * l + i]);
            }
            k.o[upper(i, j)] = cd{0.5 * (xij.re - xji.re), 0.5 * (xij.im + xji.im)};
        }
    return k;
}

template <int R, int N>
__device__ __forceinline__ void plaquette_loop(const CloverForceArgs &f, const int x[4], long site)
{
    constexpr int pl = plane_of(R, N);
    const long V2 = 2L * f.g.Vh;
    const double *h = f.H + (long)pl * 9 * V2;
    int xr[4], xn[4], xrn[4];
    shift(f.g, x, R, +1, xr);
    shift(f.g, x, N, +1, xn);
    shift(f.g, xr, N, +1, xrn);
    // Horner form from the back: t = a (h1 b c+ d+ + b (h2 c+ d+ + c+ (h3 d+ + d+ h0)))
    const Mat3 dd = dagm(link_c(f, x, N));
    Mat3 t = hmul(load_sym(h, V2, site_of(f.g, xn)), dd);
    add_to(t, mulh(dd, load_sym(h, V2, site)));
    const Mat3 c = link_c(f, xn, R);
    Mat3 P = mm_dn(c, dd);  // c+ d+
    t = mm_dn(c, t);
    add_to(t, hmul(load_sym(h, V2, site_of(f.g, xrn)), P));
    const Mat3 b = link_c(f, xr, N);
    t = mm(b, t);
    P = mm(b, P);  // b c+ d+
    add_to(t, hmul(load_sym(h, V2, site_of(f.g, xr)), P));
    const Mat3 a = link_c(f, x, R);
    double *o = f.KA + (long)pl * 16 * V2;
    store_tl(o, V2, site, herm_of_product(a, t));
    store_tl(o + 8 * V2, V2, site, aherm_of_product(a, P));
}

// One thread per (site, plane); workgroup 12 i + 6 p + plane takes the i-th
// 256-site block of parity p in the chunked block order (order_block), so the
// six planes and both parities of a site block are neighbouring workgroups
// (with the XCD remap, on one XCD) and read its links and insertions through
// one L2.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) clover_loop_kernel(CloverForceArgs f)
{
    const long blk = xcd_block(f.xcd);
    const int pl = (int)(blk % 6);
    const int p = (int)((blk / 6) & 1);
    const long s = order_block(f.g, blk / 12, 256) * 256 + threadIdx.x;
    if (s >= f.g.Vh) return;
    const long t = (long)p * f.g.Vh + s;
    int x[4];
    cb_coords(f.g, (int)s, p, x);
    switch (pl) {
    case 0: plaquette_loop<0, 1>(f, x, t); break;
    case 1: plaquette_loop<0, 2>(f, x, t); break;
    case 2: plaquette_loop<0, 3>(f, x, t); break;
    case 3: plaquette_loop<1, 2>(f, x, t); break;
    case 4: plaquette_loop<1, 3>(f, x, t); break;
    default: plaquette_loop<2, 3>(f, x, t); break;
    }
}

// ---- link sums --------------------------------------------------------------
// u+ g u for Hermitian g (Hermitian result), one column of g u at a time
// (the products of a column feed the entries (i, j), i <= j, at once, so only
// three complex values of g u are live)
__device__ __forceinline__ Sym3 conj_herm(const Mat3 &u, const Sym3 &g)
{
    Sym3 r;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        cd m[3];  // column j of g u
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cd s = g.d[i] * u.m[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k != i) cmac(s, herm_get(g, i, k), u.m[3 * k + j]);
            m[i] = s;
        }
        double dj = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) dj += u.m[3 * k + j].re * m[k].re + u.m[3 * k + j].im * m[k].im;
        r.d[j] = dj;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_conj(s, u.m[3 * k + i], m[k]);
            r.o[upper(i, j)] = s;
        }
    }
    return r;
}

// u+ a u for anti-Hermitian a (anti-Hermitian result), column by column
__device__ __forceinline__ Sym3 conj_aherm(const Mat3 &u, const Sym3 &a)
{
    Sym3 r;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        cd m[3];  // column j of a u
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const cd v = u.m[3 * i + j];
            cd s{-a.d[i] * v.im, a.d[i] * v.re};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k != i) cmac(s, aherm_get(a, i, k), u.m[3 * k + j]);
            m[i] = s;
        }
        double dj = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) dj += u.m[3 * k + j].re * m[k].im - u.m[3 * k + j].im * m[k].re;
        r.d[j] = dj;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_conj(s, u.m[3 * k + i], m[k]);
            r.o[upper(i, j)] = s;
        }
    }
    return r;
}

// [a, h] = a h + (a h)+ for anti-Hermitian a and Hermitian h (Hermitian)
__device__ __forceinline__ Sym3 commute(const Sym3 &a, const Sym3 &h)
{
    Sym3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {  // 2 Re (a h)_ii: the term a_ii h_ii is imaginary
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k != i) {
                const cd x = aherm_get(a, i, k), y = herm_get(h, k, i);
                s += x.re * y.re - x.im * y.im;
            }
        r.d[i] = 2.0 * s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            cd e{0, 0}, g{0, 0};  // (a h)_ij, (a h)_ji
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k == i) {
                    const cd v = herm_get(h, i, j);
                    e = e + cd{-a.d[i] * v.im, a.d[i] * v.re};
                    g = g + h.d[i] * aherm_get(a, j, i);
                } else if (k == j) {
                    const cd v = herm_get(h, j, i);
                    e = e + h.d[j] * aherm_get(a, i, j);
                    g = g + cd{-a.d[j] * v.im, a.d[j] * v.re};
                } else {
                    cmac(e, aherm_get(a, i, k), herm_get(h, k, j));
                    cmac(g, aherm_get(a, j, k), herm_get(h, k, i));
                }
            }
            r.o[upper(i, j)] = cd{e.re + g.re, e.im - g.im};
        }
    return r;
}

__device__ __forceinline__ void axpy(Sym3 &z, double s, const Sym3 &k)  // z += s k
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        z.d[i] += s * k.d[i];
        z.o[i] = z.o[i] + s * k.o[i];
    }
}

// The force on U_R(y) from plane (R, N), as Hermitian part of the loops
// (the anti-Hermitian projection below needs no more).  With the stored
// plaquettes P(y) and P(y - N) of the plane (lower direction first),
// u = U_N(y - N), their parts K, A and K', A', and the insertions h(y),
// h' = h(y - N) of the plane:
//   R < N:  K - u+ (K' - [A', h']) u + [u+ A' u, h(y)]
//   R > N: -K + u+ K' u + [A + u+ A' u, h(y)]
// (the first loop opened at y with h(y) at its end, the second the loop
// below taken at its corner y, where the conjugation by u is corrected by the
// commutator terms; for R > N both come from the plaquettes of the opposite
// orientation, reversed).
__device__ __forceinline__ void link_plane(const CloverForceArgs &f, const int y[4], long site, int R, int N, Sym3 &z)
{
    const bool below = R < N;  // the stored plaquettes are oriented R -> N
    const double sg = below ? 1.0 : -1.0;
    const long V2 = 2L * f.g.Vh;
    const int pl = below ? plane_of(R, N) : plane_of(N, R);
    const double *ka = f.KA + (long)pl * 16 * V2;
    const double *h = f.H + (long)pl * 9 * V2;
    int ym[4];
    shift(f.g, y, N, -1, ym);
    const long sm = site_of(f.g, ym);
    const Mat3 u = link_c(f, ym, N);
    const Sym3 a1 = load_tl(ka + 8 * V2, V2, sm);
    Sym3 b = conj_aherm(u, a1);
    Sym3 g = load_tl(ka, V2, sm);
    if (below)
        axpy(g, -1.0, commute(a1, load_sym(h, V2, sm)));
    else
        axpy(b, 1.0, load_tl(ka + 8 * V2, V2, site));
    const Sym3 k0 = load_tl(ka, V2, site);
    const Sym3 hy = load_sym(h, V2, site);
    axpy(z, -sg, conj_herm(u, g));
    axpy(z, sg, k0);
    axpy(z, 1.0, commute(b, hy));
}

__device__ __forceinline__ void link_sum(const CloverForceArgs &f, const int y[4], long site, long lex, int R)
{
    Sym3 z;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        z.d[i] = 0.0;
        z.o[i] = cd{0, 0};
    }
    // one plane at a time (a loop, so that the planes' loads and products
    // do not overlap and the thread holds one plane's operands), plane
    // (R, R ^ k) in step k: the waves of directions R and R ^ k read the
    // plane's loops and insertions at y together
#pragma unroll 1
    for (int k = 1; k < 4; ++k) link_plane(f, y, site, R, R ^ k, z);
    // F = coeff TA(i (kappa csw / 8) Z); only the Hermitian part of Z enters,
    // so F = i coeff (kappa csw / 8) (Z - tr Z / 3)
    const double cc = f.coeff * f.kc8;
    const double tr3 = (z.d[0] + z.d[1] + z.d[2]) / 3.0;
    double2 *o = reinterpret_cast<double2 *>(f.out) + (lex * 4 + R) * 9;
    double2 v[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (i == j) {
                v[3 * i + j] = make_double2(0.0, cc * (z.d[i] - tr3));
            } else {
                const cd w = herm_get(z, i, j);
                v[3 * i + j] = make_double2(-cc * w.im, cc * w.re);
            }
        }
    if (f.accumulate) {  // the nine old entries in one round trip
        double2 old[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) old[k] = o[k];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = make_double2(v[k].x + old[k].x, v[k].y + old[k].y);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) o[k] = v[k];
}

// One thread per link: a workgroup holds 64 sites of one parity (the
// blocks in the chunked block order), one wave per direction, so that the two
// waves of a plane read its data at y through one L1; workgroups alternate
// between the parities.
__global__ void __launch_bounds__(256) clover_link_kernel(CloverForceArgs f)
{
    const long blk = xcd_block(f.xcd);
    const int p = (int)(blk & 1);
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const long s = order_block(f.g, blk >> 1, 64) * 64 + (threadIdx.x & 63);
    if (s >= f.g.Vh) return;
    const long t = (long)p * f.g.Vh + s;
    int y[4];
    cb_coords(f.g, (int)s, p, y);
    const long lex = y[0] + (long)f.g.L[0] * (y[1] + (long)f.g.L[1] * (y[2] + (long)f.g.L[2] * y[3]));
    link_sum(f, y, t, lex, r);
}

}  // namespace

hipError_t launch_clover_insertions(const CloverForceArgs &f, hipStream_t st)
{
    const long n = 2L * f.g.Vh;
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (f.h_acc)
        hipLaunchKernelGGL(clover_insertion_kernel<true>, dim3(nb), dim3(256), 0, st, f);
    else
        hipLaunchKernelGGL(clover_insertion_kernel<false>, dim3(nb), dim3(256), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_clover_link_sums(const CloverForceArgs &f, hipStream_t st)
{
    if (f.g.Vh == 0) return hipSuccess;
    const long nb = 2 * ((f.g.Vh + 63) / 64);  // link sums: blocks of 64 sites, both parities
    hipLaunchKernelGGL(clover_loop_kernel, dim3((unsigned)(12 * ((f.g.Vh + 255) / 256))), dim3(256), 0, st, f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(clover_link_kernel, dim3((unsigned)nb), dim3(256), 0, st, f);
    return hipGetLastError();
}

}  // namespace tmx
