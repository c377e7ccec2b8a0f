// Wilson twisted-mass clover stencil kernels (gfx950).
//
// One launch computes, for every site s of the output parity p and every
// right-hand side r (slot t = s * nrhs + r; a launch may take a group of the
// right-hand sides, see dslash_kernel):
//
//   MODE_INV  (first half of the Schur operator, "K1"):
//       out = B_p^{-1}(sgn) (H in)(s)
//     degenerate: B^{-1} = (A + i sgn nu g5)^{-1}, a stored full 6x6 per
//     chirality (the -nu inverse is its adjoint);
//     two flavours: (A + X)^{-1} = (A - X) (A^2 + nubar^2 - epst^2)^{-1},
//     X = i sgn nubar g5 tau3 - epst tau1, with A and the Hermitian inverse
//     factor stored.
//   MODE_DIAG (second half, "K2", or one parity of the full operator D):
//       out = (A_p + X(sgn)) x(s) - kfac (H in)(s)
//     with X = i sgn nu g5 (degenerate) or the two-flavour X above; for the
//     mass-preconditioned operator (one flavour) i rho x is added to the
//     final output.
//
// H is the Wilson hopping term with the spin projectors (1 -+ gamma_mu) of
// the chiral basis written out per direction: the projected half spinor
// h = psi_upper + sgn * a_mu psi_lower is transported, and the lower spin
// components are rebuilt as sgn * a_mu^dagger (U h), where gamma_mu =
// [[0, a_mu], [a_mu^dagger, 0]], a_k = -i sigma_k, a_4 = 1.
//
// Optional gamma5 on the hopping input (g5in), on the diagonal input (g5x)
// and on the output (g5out) implement the
// adjoint Mhat^dagger = g5 Mhat(-sgn) g5 and the normal operator without
// extra passes.
#include "tmx_device.h"
#include "tmx_kernels.h"

namespace tmx {

enum { MODE_INV = 0, MODE_DIAG = 1 };

// acc += (1 + sgn gamma_mu) * bc * W psi,  W = U (fwd) or U^dagger (bwd)
template <int MU, int SGN, bool DAG, typename R>
__device__ __forceinline__ void hop_term(const cx<R> u[9], R bc, const cx<R> psi[12], cx<R> acc[12])
{
    // half spinor h[spin 0/1][colour]
    cx<R> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> p0 = psi[c], p1 = psi[3 + c], p2 = psi[6 + c], p3 = psi[9 + c];
        cx<R> a0, a1;  // a_mu psi_lower
        if constexpr (MU == 0) {
            a0 = -imul(p3);
            a1 = -imul(p2);
        } else if constexpr (MU == 1) {
            a0 = -p3;
            a1 = p2;
        } else if constexpr (MU == 2) {
            a0 = -imul(p2);
            a1 = imul(p3);
        } else {
            a0 = p2;
            a1 = p3;
        }
        if constexpr (SGN > 0) {
            h0[c] = p0 + a0;
            h1[c] = p1 + a1;
        } else {
            h0[c] = p0 - a0;
            h1[c] = p1 - a1;
        }
    }
    // k = W h
    cx<R> k0[3], k1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        k0[a] = cx<R>{0, 0};
        k1[a] = cx<R>{0, 0};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (DAG) {
                cmac_conj(k0[a], u[3 * b + a], h0[b]);
                cmac_conj(k1[a], u[3 * b + a], h1[b]);
            } else {
                cmac(k0[a], u[3 * a + b], h0[b]);
                cmac(k1[a], u[3 * a + b], h1[b]);
            }
        }
        k0[a] = bc * k0[a];
        k1[a] = bc * k1[a];
    }
    // reconstruct: upper += k, lower += sgn * a_mu^dagger k
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = acc[c] + k0[c];
        acc[3 + c] = acc[3 + c] + k1[c];
        cx<R> l0, l1;
        if constexpr (MU == 0) {
            l0 = imul(k1[c]);
            l1 = imul(k0[c]);
        } else if constexpr (MU == 1) {
            l0 = k1[c];
            l1 = -k0[c];
        } else if constexpr (MU == 2) {
            l0 = imul(k0[c]);
            l1 = -imul(k1[c]);
        } else {
            l0 = k0[c];
            l1 = k1[c];
        }
        if constexpr (SGN > 0) {
            acc[6 + c] = acc[6 + c] + l0;
            acc[9 + c] = acc[9 + c] + l1;
        } else {
            acc[6 + c] = acc[6 + c] - l0;
            acc[9 + c] = acc[9 + c] - l1;
        }
    }
}

template <int P, typename R>
__device__ __forceinline__ void load_spinor_g5(const SpinorPtr &f, int flav, long slot, bool g5, cx<R> v[12])
{
    load_spinor<P>(f, flav, slot, v);
    if (g5) {
#pragma unroll
        for (int k = 6; k < 12; ++k) v[k] = -v[k];
    }
}

// accumulate (H in)(s) for all flavours
template <int P, int NF, int MU, typename R>
__device__ __forceinline__ void hop_dir(const DslashArgs &a, const int x[4], int s, long rhs, cx<R> acc[NF][12])
{
    const Geom &g = a.g;
    const int p = a.parity;
    // forward: (1 - gamma_mu) U_mu(x) psi(x + mu)
    {
        int y[4] = {x[0], x[1], x[2], x[3]};
        R bc = R(1);
        if (++y[MU] == g.L[MU]) {
            y[MU] = 0;
            if (MU == 3) bc = R(a.t_bc);
        }
        const int n = cb_index(g, y);
        cx<R> u[9];
        load_link<P>(a.U, p, MU, s, u);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cx<R> psi[12];
            load_spinor_g5<P>(a.in, f, (long)n * a.nrhs + rhs, a.g5in, psi);
            hop_term<MU, -1, false>(u, bc, psi, acc[f]);
        }
        // one flavour, and two flavours in FP32: the forward and backward hops
        // of a direction share a fence, so both neighbours' loads are in
        // flight together (FP64: 220 VGPRs, two waves per SIMD; 1-4 % faster
        // than a fence per hop); FP64 and FP16 two-flavour kernels keep a
        // fence per hop (FP16: 5 % slower paired)
        if constexpr (NF != 1 && P != F32) {
#pragma unroll
            for (int f = 0; f < NF; ++f) reg_fence(acc[f], 12);
        }
    }
    // backward: (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu)
    {
        int y[4] = {x[0], x[1], x[2], x[3]};
        R bc = R(1);
        if (--y[MU] < 0) {
            y[MU] = g.L[MU] - 1;
            if (MU == 3) bc = R(a.t_bc);
        }
        const int n = cb_index(g, y);
        cx<R> u[9];
        load_link<P>(a.U, 1 - p, MU, n, u);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cx<R> psi[12];
            load_spinor_g5<P>(a.in, f, (long)n * a.nrhs + rhs, a.g5in, psi);
            hop_term<MU, +1, true>(u, bc, psi, acc[f]);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) reg_fence(acc[f], 12);
    }
}

template <int P, int NF, int MODE>
__device__ __forceinline__ void dslash_slot(const DslashArgs &a, int s, long rhs);

// Thread i takes the work items i, i + G, ..., i + (SPT - 1) G (G the grid's
// thread count); item u is right-hand side r0 + u % rg of site u / rg.  SPT
// is a template parameter: a runtime loop costs registers (and occupancy)
// even when it runs once.
template <int P, int NF, int MODE, int SPT>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a)
{
    const long rg = a.rg;
    const long n = (long)a.g.Vh * rg;
    long u = (long)xcd_block(a.xcd) * blockDim.x + threadIdx.x;
    if constexpr (SPT == 1) {
        if (u >= n) return;
        const int s = (int)(u / rg);
        dslash_slot<P, NF, MODE>(a, s, a.r0 + (u - (long)s * rg));
    } else {
        const long G = (long)gridDim.x * blockDim.x;
        for (int k = 0; k < SPT && u < n; ++k, u += G) {
            const int s = (int)(u / rg);
            dslash_slot<P, NF, MODE>(a, s, a.r0 + (u - (long)s * rg));
        }
    }
}

// one output slot: site s (of the output parity), right-hand side rhs
template <int P, int NF, int MODE>
__device__ __forceinline__ void dslash_slot(const DslashArgs &a, int s, long rhs)
{
    using R = typename RealOf<P>::type;
    const long t = (long)s * a.nrhs + rhs;  // slot of the output, the diagonal input and the norms
    int x[4];
    cb_coords(a.g, s, a.parity, x);

    cx<R> acc[NF][12];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[f][k] = cx<R>{0, 0};

    // one direction at a time (register fences inside hop_dir): holding every
    // neighbour's data at once would need ~4x the registers and drop
    // occupancy to one wave per SIMD.  t first: its neighbours are the
    // farthest in memory (most often past L2), so their loads go out first
    // (FP64 K1 1.4 % faster than x first)
    hop_dir<P, NF, 3>(a, x, s, rhs, acc);
    hop_dir<P, NF, 2>(a, x, s, rhs, acc);
    hop_dir<P, NF, 1>(a, x, s, rhs, acc);
    hop_dir<P, NF, 0>(a, x, s, rhs, acc);

    const long cs = a.g.Vh;  // clover stride
    // site-block epilogue, one chirality block at a time (register fences
    // keep the two blocks' matrices from being live together)
    cx<R> out[NF][12];
    if constexpr (MODE == MODE_INV) {
        if constexpr (NF == 1) {
            const bool dag = a.sgn < 0;
            full_apply<P>(a.inv, cs, s, 0, dag, acc[0], out[0]);
            reg_fence(out[0], 6);
            full_apply<P>(a.inv, cs, s, 1, dag, acc[0] + 6, out[0] + 6);
        } else {
            // (A + X)^{-1} acc = (A - X) t,  t_f = Binv acc_f  (per chirality)
            const R nb = R(a.sgn * a.nu), ep = R(a.epst);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const R tw = c == 0 ? nb : -nb;  // i nubar g5 tau3 on flavour 0
                cx<R> t0[6], t1[6];
                herm_apply_c<P>(a.inv, cs, s, c, R(0), acc[0] + 6 * c, t0);
                herm_apply_c<P>(a.inv, cs, s, c, R(0), acc[1] + 6 * c, t1);
                reg_fence(t0, 6);
                reg_fence(t1, 6);
                herm_apply_c<P>(a.clov, cs, s, c, -tw, t0, out[0] + 6 * c);
                herm_apply_c<P>(a.clov, cs, s, c, tw, t1, out[1] + 6 * c);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    out[0][6 * c + k] = out[0][6 * c + k] + ep * t1[k];
                    out[1][6 * c + k] = out[1][6 * c + k] + ep * t0[k];
                }
                reg_fence(out[0] + 6 * c, 6);
                reg_fence(out[1] + 6 * c, 6);
            }
        }
    } else {
        const R kf = R(a.kfac);
        const R nb = R(a.sgn * a.nu);
        const R g5s = a.g5x ? R(-1) : R(1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const R tw = c == 0 ? nb : -nb;
            const R gx = c == 0 ? R(1) : g5s;  // gamma5 on the diagonal input
            if constexpr (NF == 1) {
                cx<R> xv[6];
                load_chiral<P>(a.x, 0, t, c, xv);
#pragma unroll
                for (int k = 0; k < 6; ++k) xv[k] = gx * xv[k];
                herm_apply_c<P>(a.clov, cs, s, c, tw, xv, out[0] + 6 * c);
                if (a.rho != 0.0) {
                    // + i rho x on the final output: before the output gamma5,
                    // the lower chirality takes the opposite sign
                    const R rs = (c == 1 && a.g5out) ? R(-a.rho) : R(a.rho);
#pragma unroll
                    for (int k = 0; k < 6; ++k) out[0][6 * c + k] = out[0][6 * c + k] + rs * imul(gx * xv[k]);
                }
            } else {
                const R ep = R(a.epst);
                cx<R> x0[6], x1[6];
                load_chiral<P>(a.x, 0, t, c, x0);
                load_chiral<P>(a.x, 1, t, c, x1);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    x0[k] = gx * x0[k];
                    x1[k] = gx * x1[k];
                }
                herm_apply_c<P>(a.clov, cs, s, c, tw, x0, out[0] + 6 * c);
                herm_apply_c<P>(a.clov, cs, s, c, -tw, x1, out[1] + 6 * c);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    out[0][6 * c + k] = out[0][6 * c + k] - ep * x1[k];
                    out[1][6 * c + k] = out[1][6 * c + k] - ep * x0[k];
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int k = 0; k < 6; ++k) out[f][6 * c + k] = out[f][6 * c + k] - kf * acc[f][6 * c + k];
                reg_fence(out[f] + 6 * c, 6);
            }
        }
    }
    if (a.g5out) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 6; k < 12; ++k) out[f][k] = -out[f][k];
    }
    if (MODE == MODE_DIAG && a.nrm) {
        double n2 = 0.0;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < 12; ++k) n2 += (double)out[f][k].re * out[f][k].re + (double)out[f][k].im * out[f][k].im;
        a.nrm[t] = n2;
    }
    // the output is written once per sweep: non-temporal stores keep it from
    // displacing the neighbour spinors in L2 (FP16 outputs, 52 bytes a site,
    // measured no faster that way)
#pragma unroll
    for (int f = 0; f < NF; ++f) store_spinor<P, P != F16>(a.out, f, t, out[f]);
}

template <int P, int NF, int MODE>
static hipError_t launch_one(const DslashArgs &a, hipStream_t st, int block)
{
    const long n = (long)a.g.Vh * (a.rg > 0 ? a.rg : a.nrhs);
    const long per = block * (long)(a.spt > 0 ? a.spt : 1);
    const int grid = (int)((n + per - 1) / per);
    if (n == 0) return hipSuccess;
    if (a.spt == 2)
        hipLaunchKernelGGL((dslash_kernel<P, NF, MODE, 2>), dim3(grid), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((dslash_kernel<P, NF, MODE, 1>), dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dslash(int prec, int nf, int mode, const DslashArgs &a0, hipStream_t st, int block)
{
    if (block <= 0) block = 256;
    DslashArgs a = a0;
    if (a.spt != 2) a.spt = 1;
    if (a.rg <= 0 || a.r0 < 0 || a.r0 + a.rg > a.nrhs) {
        a.r0 = 0;
        a.rg = a.nrhs;
    }
#define TMX_DS(P, NF)                                                                     \
    if (prec == P && nf == NF) {                                                          \
        return mode == MODE_INV ? launch_one<P, NF, MODE_INV>(a, st, block)               \
                                : launch_one<P, NF, MODE_DIAG>(a, st, block);             \
    }
    TMX_DS(F64, 1)
    TMX_DS(F32, 1)
    TMX_DS(F16, 1)
    TMX_DS(F64, 2)
    TMX_DS(F32, 2)
    TMX_DS(F16, 2)
#undef TMX_DS
    return hipErrorInvalidValue;
}

}  // namespace tmx
