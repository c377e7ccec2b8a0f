// Gauge-field and clover set-up kernels (run once per gauge field / mass).
//
//  * link compression: rows 0 and 1 of every SU(3) link are kept (row 2 is
//    conj(row0 x row1), rebuilt in registers by the stencil kernels), split
//    by the parity of the site the link starts at, in the site-major layout.
//  * clover term: F_{mu nu} from the four plaquette leaves, F = (Q - Q^+)/8,
//    T = i kappa csw sum_{mu<nu} sigma_{mu nu} F_{mu nu}.  In the chiral
//    basis sigma_{kl} = -eps_{klm} diag(s_m, s_m) and sigma_{k4} = diag(s_k,
//    -s_k) (s = Pauli matrices), so each chirality block is
//      T_chi = i kappa csw (s_1 (x) G_1 + s_2 (x) G_2 + s_3 (x) G_3),
//      G_1 = -F_yz +- F_xt,  G_2 = F_xz +- F_yt,  G_3 = -F_xy +- F_zt
//    (+ for chirality 0 = spins 0,1, - for chirality 1).  A = 1 + T is stored
//    as two Hermitian 6x6 blocks.
//  * site inverses through (A + i nu)^{-1} = (A - i nu)(A^2 + nu^2)^{-1},
//    with the Hermitian positive A^2 + nu^2 inverted by Cholesky (no
//    pivoting needed), all in FP64.
#include "tmx_device.h"
#include "tmx_kernels.h"

namespace tmx {

using cd = cx<double>;

struct M3 {
    cd m[9];
};

__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b)
{
    M3 c;
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

// a * b^dagger
__device__ __forceinline__ M3 mul_nd(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd s{0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = s + a.m[3 * i + k] * conj(b.m[3 * j + k]);
            c.m[3 * i + j] = s;
        }
    return c;
}

// a^dagger * b
__device__ __forceinline__ M3 mul_dn(const M3 &a, const M3 &b)
{
    M3 c;
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

// ---------------------------------------------------------------------------
// link compression
// ---------------------------------------------------------------------------
__global__ void pack_links_kernel(const double *canon, double *links64, Geom g)
{
    const long V = 2L * g.Vh;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    int x[4];
    long r = i;
    x[0] = (int)(r % g.L[0]);
    r /= g.L[0];
    x[1] = (int)(r % g.L[1]);
    r /= g.L[1];
    x[2] = (int)(r % g.L[2]);
    x[3] = (int)(r / g.L[2]);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int s = cb_index(g, x);
    double2 *out = reinterpret_cast<double2 *>(links64);
    const double2 *in = reinterpret_cast<const double2 *>(canon);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 6; ++k) out[((long)(p * 4 + mu) * 6 + k) * g.Vh + s] = in[(i * 4 + mu) * 9 + k];
}

hipError_t launch_pack_links(const double *canon, double *links64, Geom g, hipStream_t st)
{
    const long V = 2L * g.Vh;
    hipLaunchKernelGGL(pack_links_kernel, dim3((V + 255) / 256), dim3(256), 0, st, canon, links64, g);
    return hipGetLastError();
}

__global__ void convert_links_kernel(const double *links64, void *dst, int prec, long Vh)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 8 * Vh) return;
    const long pm = t / Vh, s = t - pm * Vh;  // (p*4+mu), site
    const double2 *in = reinterpret_cast<const double2 *>(links64) + pm * 6 * Vh;
    float v[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double2 d = in[k * Vh + s];
        v[2 * k] = (float)d.x;
        v[2 * k + 1] = (float)d.y;
    }
    if (prec == F32) {
        float4 *o = static_cast<float4 *>(dst) + pm * 3 * Vh;
#pragma unroll
        for (int k = 0; k < 3; ++k) o[k * Vh + s] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
        uint2 *o = static_cast<uint2 *>(dst) + pm * 3 * Vh;
#pragma unroll
        for (int k = 0; k < 3; ++k) o[k * Vh + s] = f_to_h4(v + 4 * k);
    }
}

hipError_t launch_convert_links(const double *links64, void *dst, int prec, Geom g, hipStream_t st)
{
    const long n = 8L * g.Vh;
    hipLaunchKernelGGL(convert_links_kernel, dim3((n + 255) / 256), dim3(256), 0, st, links64, dst, prec,
                       (long)g.Vh);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// clover term
// ---------------------------------------------------------------------------
__device__ __forceinline__ M3 link_at(const double *links64, const Geom &g, const int x[4], int mu)
{
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    LinkPtr U{links64, g.Vh};
    M3 u;
    load_link<F64>(U, p, mu, cb_index(g, x), u.m);
    return u;
}

__device__ __forceinline__ void step(const Geom &g, const int x[4], int mu, int d, int y[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] += d;
    if (y[mu] < 0) y[mu] += g.L[mu];
    if (y[mu] >= g.L[mu]) y[mu] -= g.L[mu];
}

// F_{mu nu}(x) = (Q - Q^+)/8 with Q the sum of the four leaves
__device__ M3 field_strength(const double *U, const Geom &g, const int x[4], int mu, int nu)
{
    int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xpmmn[4];
    step(g, x, mu, +1, xpm);
    step(g, x, nu, +1, xpn);
    step(g, x, mu, -1, xmm);
    step(g, x, nu, -1, xmn);
    step(g, xmm, nu, +1, xmmpn);
    step(g, xmm, nu, -1, xmmmn);
    step(g, xpm, nu, -1, xpmmn);
    M3 Q;
    {
        // leaf in the (+mu,+nu) quadrant
        M3 a = mul(link_at(U, g, x, mu), link_at(U, g, xpm, nu));
        M3 b = mul_nd(a, link_at(U, g, xpn, mu));
        Q = mul_nd(b, link_at(U, g, x, nu));
    }
    {
        // (-mu,+nu): U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
        M3 a = mul_nd(link_at(U, g, x, nu), link_at(U, g, xmmpn, mu));
        M3 b = mul_nd(a, link_at(U, g, xmm, nu));
        M3 c = mul(b, link_at(U, g, xmm, mu));
#pragma unroll
        for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + c.m[k];
    }
    {
        // (-mu,-nu): U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
        //          = (U_nu(x-mu-nu) U_mu(x-mu))^+ U_mu(x-mu-nu) U_nu(x-nu)
        M3 a = mul(link_at(U, g, xmmmn, nu), link_at(U, g, xmm, mu));
        M3 b = mul_dn(a, link_at(U, g, xmmmn, mu));
        M3 c = mul(b, link_at(U, g, xmn, nu));
#pragma unroll
        for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + c.m[k];
    }
    {
        // (+mu,-nu): U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
        M3 a = mul_dn(link_at(U, g, xmn, nu), link_at(U, g, xmn, mu));
        M3 b = mul(a, link_at(U, g, xpmmn, nu));
        M3 c = mul_nd(b, link_at(U, g, x, mu));
#pragma unroll
        for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + c.m[k];
    }
    M3 F;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F.m[3 * i + j] = 0.125 * (Q.m[3 * i + j] - conj(Q.m[3 * j + i]));
    return F;
}

// packed Hermitian store: 36 reals per chirality (d0..d5, 15 lower (re,im))
__device__ __forceinline__ void store_herm(double *clov64, long stride, long s, int chir, const cd A[6][6])
{
    double a[36];
#pragma unroll
    for (int i = 0; i < 6; ++i) a[i] = A[i][i].re;
    int k = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            a[k] = A[i][j].re;
            a[k + 1] = A[i][j].im;
            k += 2;
        }
    store_seq<F64, 36>(clov64 + (size_t)chir * 18 * stride * 2, stride, s, a);
}

__device__ __forceinline__ void load_herm(const double *clov64, long stride, long s, int chir, cd A[6][6])
{
    double a[36];
    load_seq<F64, 36>(clov64 + (size_t)chir * 18 * stride * 2, stride, s, a);
#pragma unroll
    for (int i = 0; i < 6; ++i) A[i][i] = cd{a[i], 0.0};
    int k = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            A[i][j] = cd{a[k], a[k + 1]};
            A[j][i] = cd{a[k], -a[k + 1]};
            k += 2;
        }
}

// clov64 layout: [parity][72 reals as 36 double2][Vh]
__global__ void clover_build_kernel(const double *links64, double *clov64, Geom g, double kappa, double csw)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    const int p = (int)(t / g.Vh);
    const int s = (int)(t - (long)p * g.Vh);
    int x[4];
    cb_coords(g, s, p, x);
    // plane order: xy, xz, xt, yz, yt, zt
    M3 Fxy = field_strength(links64, g, x, 0, 1);
    M3 Fxz = field_strength(links64, g, x, 0, 2);
    M3 Fxt = field_strength(links64, g, x, 0, 3);
    M3 Fyz = field_strength(links64, g, x, 1, 2);
    M3 Fyt = field_strength(links64, g, x, 1, 3);
    M3 Fzt = field_strength(links64, g, x, 2, 3);
    const double kc = kappa * csw;
    double *base = clov64 + (size_t)p * 36 * g.Vh * 2;
#pragma unroll
    for (int chir = 0; chir < 2; ++chir) {
        const double sg = chir == 0 ? 1.0 : -1.0;
        cd A[6][6];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int k = 3 * a + b;
                const cd G1 = -Fyz.m[k] + sg * Fxt.m[k];
                const cd G2 = Fxz.m[k] + sg * Fyt.m[k];
                const cd G3 = -Fxy.m[k] + sg * Fzt.m[k];
                // T = i kc [[G3, G1 - i G2], [G1 + i G2, -G3]]
                const cd t00 = kc * imul(G3);
                const cd t01 = kc * imul(G1 - imul(G2));
                const cd t10 = kc * imul(G1 + imul(G2));
                A[a][b] = t00;
                A[a][3 + b] = t01;
                A[3 + a][b] = t10;
                A[3 + a][3 + b] = -t00;
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) A[i][i].re += 1.0;
        store_herm(base, g.Vh, s, chir, A);
    }
}

hipError_t launch_clover_build(const double *links64, double *clov64, Geom g, double kappa, double csw,
                               hipStream_t st)
{
    const long n = 2L * g.Vh;
    hipLaunchKernelGGL(clover_build_kernel, dim3((n + 127) / 128), dim3(128), 0, st, links64, clov64, g, kappa,
                       csw);
    return hipGetLastError();
}

// canonical T: [lex][chir][6][6] complex128, A = 1 + T
__global__ void clover_from_canon_kernel(const double *canonT, double *clov64, Geom g, int to_canon)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2L * g.Vh) return;
    int x[4];
    long r = i;
    x[0] = (int)(r % g.L[0]);
    r /= g.L[0];
    x[1] = (int)(r % g.L[1]);
    r /= g.L[1];
    x[2] = (int)(r % g.L[2]);
    x[3] = (int)(r / g.L[2]);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int s = cb_index(g, x);
    double *base = clov64 + (size_t)p * 36 * g.Vh * 2;
    const double2 *cin = reinterpret_cast<const double2 *>(canonT) + i * 72;
    double2 *cout = reinterpret_cast<double2 *>(const_cast<double *>(canonT)) + i * 72;
    for (int chir = 0; chir < 2; ++chir) {
        cd A[6][6];
        if (to_canon) {
            load_herm(base, g.Vh, s, chir, A);
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) {
                    cd v = A[a][b];
                    if (a == b) v.re -= 1.0;
                    cout[chir * 36 + 6 * a + b] = make_double2(v.re, v.im);
                }
        } else {
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) {
                    double2 v = cin[chir * 36 + 6 * a + b];
                    A[a][b] = cd{v.x + (a == b ? 1.0 : 0.0), v.y};
                }
            store_herm(base, g.Vh, s, chir, A);
        }
    }
}

hipError_t launch_clover_from_canonical(const double *canonT, double *clov64, Geom g, hipStream_t st)
{
    const long n = 2L * g.Vh;
    hipLaunchKernelGGL(clover_from_canon_kernel, dim3((n + 127) / 128), dim3(128), 0, st, canonT, clov64, g, 0);
    return hipGetLastError();
}

hipError_t launch_clover_to_canonical(const double *clov64, double *canonT, Geom g, hipStream_t st)
{
    const long n = 2L * g.Vh;
    hipLaunchKernelGGL(clover_from_canon_kernel, dim3((n + 127) / 128), dim3(128), 0, st, canonT,
                       const_cast<double *>(clov64), g, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// site inverses
// ---------------------------------------------------------------------------
// S^{-1} for Hermitian positive definite 6x6 S via Cholesky S = L L^+:
// S^{-1} = L^{-+} L^{-1}.
__device__ void hpd_inverse(const cd S[6][6], cd Sinv[6][6])
{
    cd Lm[6][6];
    double dinv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) Lm[i][j] = cd{0, 0};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = S[j][j].re;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k].re * Lm[j][k].re + Lm[j][k].im * Lm[j][k].im;
        d = sqrt(d);
        Lm[j][j] = cd{d, 0};
        dinv[j] = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            cd v = S[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) {
                // v -= L[i][k] conj(L[j][k])
                const cd a = Lm[i][k], b = Lm[j][k];
                v.re -= a.re * b.re + a.im * b.im;
                v.im -= a.im * b.re - a.re * b.im;
            }
            Lm[i][j] = dinv[j] * v;
        }
    }
    // W = L^{-1} (lower triangular)
    cd W[6][6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) W[i][j] = cd{0, 0};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        W[i][i] = cd{dinv[i], 0};
#pragma unroll
        for (int j = 0; j < i; ++j) {
            cd v{0, 0};
#pragma unroll
            for (int k = j; k < i; ++k) cmac(v, Lm[i][k], W[k][j]);
            W[i][j] = -dinv[i] * v;
        }
    }
    // Sinv = W^+ W
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            cd v{0, 0};
#pragma unroll
            for (int k = (i > j ? i : j); k < 6; ++k) cmac_conj(v, W[k][i], W[k][j]);
            Sinv[i][j] = v;
        }
}

// A^2 + c (Hermitian positive for c > -lambda_min(A^2))
__device__ __forceinline__ void herm_square_shift(const cd A[6][6], double c, cd S[6][6])
{
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            cd v{i == j ? c : 0.0, 0};
#pragma unroll
            for (int k = 0; k < 6; ++k) cmac(v, A[i][k], A[k][j]);
            S[i][j] = v;
        }
}

// thread per (even site, chirality); inv64 layout [72 reals per chirality as
// 36 double2, chirality-major][Vh]
__global__ void clover_inv_kernel(const double *clov_even, double *inv64, long Vh, double nu)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * Vh) return;
    const int chir = (int)(t / Vh);
    const long s = t - chir * Vh;
    cd A[6][6], S[6][6], Si[6][6];
    load_herm(clov_even, Vh, s, chir, A);
    const double tw = chir == 0 ? nu : -nu;  // i nu gamma5 on this chirality
    herm_square_shift(A, tw * tw, S);
    hpd_inverse(S, Si);
    // (A + i tw)^{-1} = (A - i tw) S^{-1}
    double out[72];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            cd v{0, 0};
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                cd a = A[i][k];
                if (i == k) a.im -= tw;
                cmac(v, a, Si[k][j]);
            }
            out[12 * i + 2 * j] = v.re;
            out[12 * i + 2 * j + 1] = v.im;
        }
    store_seq<F64, 72>(inv64 + (size_t)chir * 36 * Vh * 2, Vh, s, out);
}

hipError_t launch_clover_inv(const double *clov64_even, double *inv64, Geom g, double nu, hipStream_t st)
{
    const long n = 2L * g.Vh;
    hipLaunchKernelGGL(clover_inv_kernel, dim3((n + 63) / 64), dim3(64), 0, st, clov64_even, inv64, (long)g.Vh,
                       nu);
    return hipGetLastError();
}

__global__ void clover_inv_nd_kernel(const double *clov_even, double *invnd64, long Vh, double c)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * Vh) return;
    const int chir = (int)(t / Vh);
    const long s = t - chir * Vh;
    cd A[6][6], S[6][6], Si[6][6];
    load_herm(clov_even, Vh, s, chir, A);
    herm_square_shift(A, c, S);
    hpd_inverse(S, Si);
    store_herm(invnd64, Vh, s, chir, Si);
}

hipError_t launch_clover_inv_nd(const double *clov64_even, double *invnd64, Geom g, double nubar, double epst,
                                hipStream_t st)
{
    const long n = 2L * g.Vh;
    hipLaunchKernelGGL(clover_inv_nd_kernel, dim3((n + 63) / 64), dim3(64), 0, st, clov64_even, invnd64,
                       (long)g.Vh, nubar * nubar - epst * epst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// precision conversion of per-site real sequences (8 reals per thread)
// ---------------------------------------------------------------------------
__global__ void convert_seq_kernel(const double *src, void *dst, int prec, int nchunk, long nsite)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nchunk * nsite) return;
    const long c = t / nsite, s = t - c * nsite;
    const double2 *in = reinterpret_cast<const double2 *>(src);
    float v[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double2 d = in[(4 * c + k) * nsite + s];
        v[2 * k] = (float)d.x;
        v[2 * k + 1] = (float)d.y;
    }
    if (prec == F32) {
        float4 *o = static_cast<float4 *>(dst);
        o[(2 * c) * nsite + s] = make_float4(v[0], v[1], v[2], v[3]);
        o[(2 * c + 1) * nsite + s] = make_float4(v[4], v[5], v[6], v[7]);
    } else {
        uint4 *o = static_cast<uint4 *>(dst);
        o[c * nsite + s] = f_to_h8(v);
    }
}

hipError_t launch_convert_seq(const double *src, void *dst, int prec, int nreal, long nsite, hipStream_t st)
{
    const int nchunk = nreal / 8;
    const long n = nchunk * nsite;
    hipLaunchKernelGGL(convert_seq_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, prec, nchunk, nsite);
    return hipGetLastError();
}

}  // namespace tmx
