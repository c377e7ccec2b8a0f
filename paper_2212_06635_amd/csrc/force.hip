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

// Insertions are Hermitian, so a plane stores nine reals per site, each
// component an array of 2 Vh doubles (site index p Vh + s): the diagonal
// H00, H11, H22, then (re, im) of H01, H02, H12.
__device__ __forceinline__ int herm_component(int i, int j)  // first real of entry (i, j), i <= j
{
    return i == j ? i : 3 + 2 * (i + j - 1);
}

// H_r,n at site x (r != n): the stored plane, negated for r > n
__device__ __forceinline__ Mat3 insertion(const CloverForceArgs &f, const int x[4], int r, int n)
{
    const long V2 = 2L * f.g.Vh;
    const long site = (long)((x[0] + x[1] + x[2] + x[3]) & 1) * f.g.Vh + cb_index(f.g, x);
    const double *h = f.H + (long)plane_of(r < n ? r : n, r < n ? n : r) * 9 * V2 + site;
    const double sg = r < n ? 1.0 : -1.0;
    double v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = sg * h[k * V2];
    Mat3 m;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        m.m[4 * i] = cd{v[i], 0.0};
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            const int c = herm_component(i, j);
            m.m[3 * i + j] = cd{v[c], v[c + 1]};
            m.m[3 * j + i] = cd{v[c], -v[c + 1]};
        }
    }
    return m;
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

// value of lane l ^ 1 (all lanes active)
__device__ __forceinline__ double pair_swap(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ Mat3 sel(bool c, const Mat3 &a, const Mat3 &b)
{
    Mat3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.m[k] = c ? a.m[k] : b.m[k];
    return m;
}

// Two lanes per link U_R(y): lane half 0 sums the plaquettes above it, lane
// half 1 those below, with one instruction stream.  The one below enters as
// E U^+ = (U E^+)^+, and E^+ has the form of the one above,
//     E^+ = b1 b2 b3 h(y) + b1 b2 h(y-n) b3 + b1 h(y-n+R) b2 b3 + h(y+R) b1 b2 b3,
//     b1 = U_n(y-n+R)^+, b2 = U_R(y-n)^+, b3 = U_n(y-n),
// so both lanes form T = c1 (c2 (c3 h(y) + h3 c3) + h2 c2 c3) + h(y+R) c1 c2 c3
// from their own links c and insertions h3, h2, sum T over the three planes,
// and add X = U sum T (above) or -X^+ (below); the pair then sums its two
// halves.
template <int R>
__device__ __forceinline__ void clover_link_half(const CloverForceArgs &f, const int y[4], long lex, int half,
                                                 bool valid)
{
    Mat3 Z, S;
#pragma unroll
    for (int k = 0; k < 9; ++k) Z.m[k] = S.m[k] = cd{0, 0};
    const bool lo = half == 1;
    if (valid) {
        int yr[4];
        shift(f.g, y, R, +1, yr);
#pragma unroll 1
        for (int n = 0; n < 4; ++n) {
            if (n == R) continue;
            // above: c3 = U_n(y)^+ at y, h3 at y+n, c2 = U_R(y+n)^+, h2 at y+R+n, c1 = U_n(y+R)
            // below: c3 = U_n(y-n) at y-n, h3 at y-n, c2 = U_R(y-n)^+, h2 at y-n+R, c1 = U_n(y-n+R)^+
            int yn[4], y3[4], y2[4];
            shift(f.g, y, n, lo ? -1 : +1, yn);  // y+n above, y-n below
            shift(f.g, yn, R, +1, y2);            // y+n+R / y-n+R
#pragma unroll
            for (int k = 0; k < 4; ++k) y3[k] = lo ? yn[k] : y[k];
            Mat3 l3 = link(f, y3, n);
            Mat3 P = sel(lo, l3, dagm(l3));                                   // c3
            Mat3 T = mm(P, insertion(f, y, R, n));                            // c3 h(y)
            add_to(T, mm(insertion(f, yn, R, n), P));                         // + h3 c3
            const Mat3 l2 = link(f, yn, R);
            const Mat3 c2 = dagm(l2);                                         // U_R(y+-n)^+ in both
            T = mm(c2, T);
            P = mm(c2, P);
            add_to(T, mm(insertion(f, y2, R, n), P));                         // + h2 c2 c3
            const Mat3 l1 = link(f, lo ? y2 : yr, n);
            const Mat3 c1 = sel(lo, dagm(l1), l1);
            T = mm(c1, T);
            P = mm(c1, P);
            add_to(T, mm(insertion(f, yr, R, n), P));                         // + h(y+R) c1 c2 c3
            add_to(S, T);
        }
        const Mat3 X = mm(link(f, y, R), S);
        const Mat3 Xd = dagm(X);
#pragma unroll
        for (int k = 0; k < 9; ++k) Z.m[k] = lo ? cd{-Xd.m[k].re, -Xd.m[k].im} : X.m[k];
    }
    // the pair's two halves
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Z.m[k].re += pair_swap(Z.m[k].re);
        Z.m[k].im += pair_swap(Z.m[k].im);
    }
    if (!valid || lo) return;
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

// Two lanes per link, 128 links per workgroup.  Workgroup 8 i + 4 p + rho
// takes direction rho of sites 128 i ... of parity p: the four directions
// and both parities of one site block are neighbouring workgroups (with the
// XCD remap, on one XCD), so the insertions and links of their common
// staples are read through one L2.
__global__ void __launch_bounds__(256) clover_force_kernel(CloverForceArgs f)
{
    const long blk = xcd_block(f.xcd);
    const int r = (int)(blk & 3);
    const int p = (int)((blk >> 2) & 1);
    const long st = (blk >> 3) * (blockDim.x / 2) + threadIdx.x / 2;
    const int half = threadIdx.x & 1;
    const bool valid = st < f.g.Vh;
    int x[4] = {0, 0, 0, 0};
    if (valid) cb_coords(f.g, (int)st, p, x);
    const long lex = x[0] + (long)f.g.L[0] * (x[1] + (long)f.g.L[1] * (x[2] + (long)f.g.L[2] * x[3]));
    switch (r) {
    case 0: clover_link_half<0>(f, x, lex, half, valid); break;
    case 1: clover_link_half<1>(f, x, lex, half, valid); break;
    case 2: clover_link_half<2>(f, x, lex, half, valid); break;
    default: clover_link_half<3>(f, x, lex, half, valid); break;
    }
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
    const long nlink = 8 * ((f.g.Vh + 127) / 128);  // 4 directions x 2 parities per block of 128 sites
    hipLaunchKernelGGL(clover_force_kernel, dim3((unsigned)nlink), dim3(256), 0, st, f);
    return hipGetLastError();
}

}  // namespace tmx
