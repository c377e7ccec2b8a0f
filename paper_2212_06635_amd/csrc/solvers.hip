// Krylov solvers on the normal operator N = Mhat^dagger Mhat (+ shift).
//
//  * CG: Hestenes-Stiefel, FP64 vectors and operator, nrhs columns advanced
//    together (one N application per iteration serves all columns, links
//    read once per site for all of them), converged columns frozen.
//  * MP-CG: the paper's mixed-precision CG (Section 1, 4.1) with reliable
//    updates in the sense of Clark et al.: inner iterations apply N in FP32
//    or FP16 storage on low-precision vectors; whenever the iterated residual
//    has dropped by a factor delta since the last update (or reached the
//    target), the low-precision solution increment is added to the FP64
//    solution, the FP64 true residual b - N x is recomputed with the FP64
//    operator and the low-precision residual restarted from it.
//  * MS-CG: multishift CG for the rational approximation (Section 4.2):
//    all shifts from the Krylov space of the smallest one (Jegerlehner's
//    collinear-residual recurrences), run in low precision, each shift then
//    refined to the FP64 target by MP-CG started from its multishift
//    solution ("shift-by-shift refinement").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "tmx_ctx.h"

namespace tmx {

namespace {

struct Sys {
    tmx_ctx *c;
    int op, nf, nrhs;
    long stride;
    double bytes_per_N;  // model bytes of one N application (all columns)
    double gbytes = 0;
    bool nomem = false;  // a workspace could not be allocated

    Sys(tmx_ctx *c_, int op_, int nrhs_) : c(c_), op(op_), nf(op_ == TMX_OP_ND ? 2 : 1), nrhs(nrhs_)
    {
        stride = c->Vh * nrhs;
        bytes_per_N = 0;
    }
    SpinorPtr field(const std::string &name, int prec, int cols = -1)
    {
        const long s = cols < 0 ? stride : c->Vh * cols;
        void *d = ws_get(c, "sv_" + name, spinor_field_bytes(prec, nf, s));
        if (!d) nomem = true;
        return make_spinor(d, prec, nf, s);
    }
    // after a group of field() calls: nothing may run on a missing workspace
    int need() const { return nomem ? set_err(c, TMX_ENOMEM, "solver workspace: out of device memory") : TMX_OK; }
    int N(SpinorPtr out, SpinorPtr in, int prec, int cols, double *nrm = nullptr)
    {
        gbytes += 2.0 * mhat_bytes_per_site(prec, nf, cols) * c->Vh * 1e-9;
        return op_mdagm(c, out, in, op, prec, cols, nrm);
    }
};

#define TRY(x)                   \
    do {                         \
        int _r = (x);            \
        if (_r) return _r;       \
    } while (0)
#define HTRY(x, w) TRY(hip_err(c, (x), w))
#define HTRY_S(S, x, w) TRY(hip_err((S).c, (x), w))

}  // namespace

// --------------------------------------------------------------------------
// shifted normal operator: q = N p + sigma p, returns Re<p, q> per column
// --------------------------------------------------------------------------
template <int P> struct OpShiftDot {
    static constexpr int NRED = 1;
    SpinorPtr q, p;
    int nf;
    double sigma[MAXR];
    __device__ void operator()(long t, int k, double *acc) const
    {
        for (int f = 0; f < nf; ++f) {
            cd vq[12], vp[12];
            ld<P>(q, f, t, vq);
            ld<P>(p, f, t, vp);
            double s = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                vq[c] = vq[c] + sigma[k] * vp[c];
                s += vp[c].re * vq[c].re + vp[c].im * vq[c].im;
            }
            if (sigma[k] != 0.0) st<P>(q, f, t, vq);
            acc[0] += s;
        }
    }
};

template <int P>
static int apply_shifted(Sys &S, SpinorPtr q, SpinorPtr p, const double *sigma, int cols, double *pq)
{
    tmx_ctx *c = S.c;
    TRY(S.N(q, p, P, cols));
    OpShiftDot<P> o{};
    o.q = q;
    o.p = p;
    o.nf = S.nf;
    for (int k = 0; k < cols; ++k) o.sigma[k] = sigma ? sigma[k] : 0.0;
    HTRY(run_blas(o, c->Vh * cols, cols, c->red, c->stream), "shifted dot");
    return pq ? fetch(c, cols, pq) : TMX_OK;  // else the dots stay on the device
}

// CG step length alpha_k = rho_k / <p, q>_k from the reduction just taken,
// computed on the device so that the update needs no host round trip;
// inactive columns (and a vanishing <p, q>) get 0, as on the host before
struct AlphaArgs {
    double rho[MAXR];
    int active[MAXR];
    int cols;
};
static __global__ void cg_alpha_kernel(const double *pq, AlphaArgs a, double *alpha)
{
    const int k = threadIdx.x;
    if (k < a.cols) alpha[k] = (a.active[k] && pq[k] != 0.0) ? a.rho[k] / pq[k] : 0.0;
}

// preconditioned CG step length alpha = rho / <p, q> on the device (0 for a
// non-positive <p, q>: breakdown, seen on the host when it reads alpha), also
// stored in the last slot of the pinned reduction buffer so that the host
// reads it with the next readback instead of a round trip of its own
constexpr int PCG_ALPHA_SLOT = MAXR * 4 - 1;
static __global__ void pcg_alpha_kernel(const double *pq, double rho, double *alpha, double *host_red)
{
    if (threadIdx.x == 0) {
        const double a = pq[0] > 0.0 ? rho / pq[0] : 0.0;
        alpha[0] = a;
        if (host_red) host_red[PCG_ALPHA_SLOT] = a;
    }
}

// true residual r = b - (N + sigma) x (FP64); writes rlo if PL given; returns |r|^2 per column
template <int PL>
static int true_residual(Sys &S, SpinorPtr r, SpinorPtr rlo, bool write_lo, SpinorPtr b, SpinorPtr x,
                         const double *sigma, int cols, double *rr)
{
    tmx_ctx *c = S.c;
    SpinorPtr q = S.field("trq", F64, cols);
    TRY(S.need());
    TRY(apply_shifted<F64>(S, q, x, sigma, cols, nullptr));
    OpXmyNorm<F64, F64, F64, PL> o{};
    o.r = r;
    o.b = b;
    o.q = q;
    o.rlo = rlo;
    o.nf = S.nf;
    o.write_lo = write_lo ? 1 : 0;
    HTRY(run_blas(o, c->Vh * cols, cols, c->red, c->stream), "true residual");
    return fetch(c, cols, rr);
}

template <int PD, int PS> static int copy_field(Sys &S, SpinorPtr d, SpinorPtr s, int cols, double *nrm)
{
    tmx_ctx *c = S.c;
    OpCopy<PD, PS> o{};
    o.d = d;
    o.s = s;
    o.nf = S.nf;
    HTRY(run_blas(o, c->Vh * cols, cols, c->red, c->stream), "copy");
    if (nrm) return fetch(c, cols, nrm);
    return TMX_OK;
}

template <int PD> static int zero_field(Sys &S, SpinorPtr d, int cols)
{
    tmx_ctx *c = S.c;
    OpZero<PD> o{};
    o.d = d;
    o.nf = S.nf;
    return hip_err(c, run_blas(o, c->Vh * cols, cols, c->red, c->stream), "zero");
}

// --------------------------------------------------------------------------
// CG / MP-CG on N + sigma_k for `cols` columns (x, b FP64 internal)
// --------------------------------------------------------------------------
// Default reliable-update trigger for iterations in precision P.  Between
// updates the iterated residual is trusted down to a drop of delta; its
// relative error then is about u / delta, u the storage rounding unit (6e-8
// FP32; 5e-4 FP16 with one scale per site), so delta = 0.01 (FP32) and 0.03
// (FP16) keep that error at 2 % or less while needing fewer FP64 residual
// recomputations than delta = 0.1 (one per decade of residual).
template <int P> constexpr double default_delta() { return P == F16 ? 0.03 : 0.01; }

template <int P>
static int cg_core(Sys &S, SpinorPtr x, SpinorPtr b, int cols, const double *sigma, const tmx_solver_cfg &cfg,
                   bool x_is_guess, tmx_info *info)
{
    tmx_ctx *c = S.c;
    const double tol = cfg.tol > 0 ? cfg.tol : 1e-10;
    const int maxiter = cfg.maxiter > 0 ? cfg.maxiter : 10000;
    const double delta = cfg.delta > 0 ? cfg.delta : default_delta<P>();
    constexpr bool mixed = P != F64;

    SpinorPtr r = S.field("r", F64, cols);
    SpinorPtr rl = mixed ? S.field("rl", P, cols) : r;
    SpinorPtr p = S.field("p", P, cols);
    SpinorPtr q = S.field("q", P, cols);
    SpinorPtr xl = mixed ? S.field("xl", F32, cols) : x;
    TRY(S.need());
    double *alpha = static_cast<double *>(ws_get(c, "cg_alpha", sizeof(double) * MAXR));
    // unshifted: <p, N p> = |Mhat p|^2, summed from the per-slot norms the
    // operator's first half writes (no separate pass over p and q)
    bool shifted = false;
    for (int k = 0; k < cols; ++k) shifted = shifted || (sigma && sigma[k] != 0.0);
    double *pnrm = shifted ? nullptr : static_cast<double *>(ws_get(c, "cg_pnrm", sizeof(double) * c->Vh * cols));
    if (!alpha || (!shifted && !pnrm)) return set_err(c, TMX_ENOMEM, "solver workspace: out of device memory");

    double bb[MAXR], rho[MAXR], rho1[MAXR], rmax[MAXR];
    int active[MAXR], iters[MAXR], nrel[MAXR];
    TRY((copy_field<F64, F64>(S, r, b, cols, bb)));
    for (int k = 0; k < cols; ++k)  // a NaN or infinite entry makes |b|^2 non-finite (x untouched)
        if (!std::isfinite(bb[k])) return set_err(c, TMX_EINVAL, "source with a non-finite entry");
    if (!x_is_guess) TRY(zero_field<F64>(S, x, cols));
    // r = b - N x (also for x = 0, to start from an exact residual)
    TRY(true_residual<P>(S, r, rl, mixed, b, x, sigma, cols, rho));
    if (mixed) TRY(zero_field<F32>(S, xl, cols));
    // p = r (low precision)
    if (mixed) {
        TRY((copy_field<P, P>(S, p, rl, cols, nullptr)));
    } else {
        TRY((copy_field<P, F64>(S, p, r, cols, nullptr)));
    }
    int nactive = 0;
    for (int k = 0; k < cols; ++k) {
        rmax[k] = rho[k];
        iters[k] = 0;
        nrel[k] = 0;
        active[k] = (bb[k] > 0 && std::sqrt(rho[k]) > tol * std::sqrt(bb[k])) ? 1 : 0;
        nactive += active[k];
    }
    const double t0 = now_seconds();
    int it = 0;
    while (nactive > 0 && it < maxiter) {
        if (shifted) {
            TRY(apply_shifted<P>(S, q, p, sigma, cols, nullptr));
        } else {
            TRY(S.N(q, p, P, cols, pnrm));
            OpSlotSum sum{};
            sum.v = pnrm;
            HTRY(run_blas(sum, c->Vh * cols, cols, c->red, c->stream), "<p, N p>");
        }
        ++it;
        AlphaArgs aa{};
        aa.cols = cols;
        for (int k = 0; k < cols; ++k) {
            aa.rho[k] = rho[k];
            aa.active[k] = active[k];
        }
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(64), 0, c->stream, c->red.result, aa, alpha);
        HTRY(hipGetLastError(), "cg step length");
        OpAxpyNorm<mixed ? F32 : F64, P, P, P> up{};
        up.x = xl;
        up.p = p;
        up.r = rl;
        up.q = q;
        up.nf = S.nf;
        up.ad = alpha;
        HTRY(run_blas(up, c->Vh * cols, cols, c->red, c->stream), "cg update");
        TRY(fetch(c, cols, rho1));
        bool reliable = false;
        for (int k = 0; k < cols; ++k) {
            if (!active[k]) continue;
            iters[k] = it;
            if (!std::isfinite(rho1[k])) return set_err(c, TMX_ENOCONV, "CG: non-finite residual");
            rmax[k] = std::max(rmax[k], rho1[k]);
            if (mixed) {
                if (std::sqrt(rho1[k]) < delta * std::sqrt(rmax[k]) || std::sqrt(rho1[k]) <= tol * std::sqrt(bb[k]))
                    reliable = true;
            }
        }
        if (mixed && reliable) {
            // x += xl ; xl = 0 ; r = b - N x ; rl = r
            OpAddTo<F64, F32> ad{};
            ad.x = x;
            ad.y = xl;
            ad.nf = S.nf;
            ad.zero_y = 1;
            HTRY(run_blas(ad, c->Vh * cols, cols, c->red, c->stream), "reliable add");
            TRY(true_residual<P>(S, r, rl, true, b, x, sigma, cols, rho1));
            for (int k = 0; k < cols; ++k) {
                if (!active[k]) continue;
                rmax[k] = rho1[k];
                nrel[k]++;
            }
        }
        OpAxpby<P, P> px{};
        px.y = p;
        px.x = rl;
        px.nf = S.nf;
        nactive = 0;
        for (int k = 0; k < cols; ++k) {
            if (active[k] && std::sqrt(rho1[k]) <= tol * std::sqrt(bb[k]) && (!mixed || reliable)) active[k] = 0;
            px.a[k] = 1.0;
            px.b[k] = active[k] ? rho1[k] / rho[k] : 0.0;
            nactive += active[k];
            rho[k] = rho1[k];
        }
        if (nactive == 0) break;
        HTRY(run_blas(px, c->Vh * cols, cols, c->red, c->stream), "cg p update");
    }
    if (mixed && nactive > 0) {
        // iteration cap reached mid-way: fold the low-precision increment in
        OpAddTo<F64, F32> ad{};
        ad.x = x;
        ad.y = xl;
        ad.nf = S.nf;
        ad.zero_y = 1;
        HTRY(run_blas(ad, c->Vh * cols, cols, c->red, c->stream), "final add");
    }
    // FP64 true residual
    double tr[MAXR];
    TRY(true_residual<P>(S, r, rl, false, b, x, sigma, cols, tr));
    const double t1 = now_seconds();
    int rc = TMX_OK;
    for (int k = 0; k < cols; ++k) {
        const double rel = bb[k] > 0 ? std::sqrt(tr[k] / bb[k]) : 0.0;
        if (info) {
            info[k].iters += iters[k];
            info[k].reliable_updates += nrel[k];
            info[k].true_residual = rel;
            info[k].seconds += t1 - t0;
            info[k].gbytes = S.gbytes;
        }
        if (!(rel <= tol)) rc = TMX_ENOCONV;
    }
    return rc;
}

// CG with restarts: the iterated residual of a long FP64 run can drift from
// the true one; a restart from the current x recomputes it exactly.
template <int P>
static int cg_solve(Sys &S, SpinorPtr x, SpinorPtr b, int cols, const double *sigma, const tmx_solver_cfg &cfg,
                    bool guess, tmx_info *info)
{
    int rc = TMX_ENOCONV;
    for (int attempt = 0; attempt < 3 && rc == TMX_ENOCONV; ++attempt) {
        rc = cg_core<P>(S, x, b, cols, sigma, cfg, guess || attempt > 0, info);
        if (rc < 0) return rc;
        if (info && rc == TMX_ENOCONV && info[0].iters >= (cfg.maxiter > 0 ? cfg.maxiter : 10000)) break;
    }
    return rc;
}

// --------------------------------------------------------------------------
// flexible preconditioned CG on N with the learned preconditioner P = K K^dagger
// (Hermitian positive semi-definite by construction), low-precision inner
// iterations and FP64 reliable updates; Polak-Ribiere beta because P is
// applied in BF16 and therefore varies slightly from call to call.
// --------------------------------------------------------------------------
template <int P> struct OpPcgDots {
    static constexpr int NRED = 2;
    SpinorPtr r, z, q;
    int nf;
    __device__ void operator()(long t, int, double *acc) const
    {
        cd vr[12], vz[12], vq[12];
        ld<P>(r, 0, t, vr);
        ld<F32>(z, 0, t, vz);
        ld<P>(q, 0, t, vq);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc[0] += vr[c].re * vz[c].re + vr[c].im * vz[c].im;
            acc[1] += vz[c].re * vq[c].re + vz[c].im * vq[c].im;
        }
    }
};

// z = P r: K K^dagger r (sym = 0), or the network's Hermitian form P (sym =
// 2) or short form P_1 (sym = 3), one application each.  An FP16 residual is
// widened to FP32 (rf) first: the network's first layer reads single spins,
// which FP16's per-site blocks make costly.
template <int P>
static int pcg_apply_pc(Sys &S, SpinorPtr z, SpinorPtr r, SpinorPtr tmp, SpinorPtr rf, int sym)
{
    int pr = P;
    if constexpr (P == F16) {
        OpCopy<F32, F16> cp{};
        cp.d = rf;
        cp.s = r;
        cp.nf = 1;
        HTRY_S(S, run_blas(cp, S.c->Vh, 1, S.c->red, S.c->stream), "widen residual");
        r = rf;
        pr = F32;
    }
    if (sym) return pc_apply_internal(S.c, z, F32, r, pr, sym);
    int rc = pc_apply_internal(S.c, tmp, F32, r, pr, 1);  // K^dagger r
    if (rc) return rc;
    return pc_apply_internal(S.c, z, F32, tmp, F32, 0);  // K K^dagger r
}

template <int P>
static int pcg_nn_core(Sys &S, SpinorPtr x, SpinorPtr b, const double *sigma, const tmx_solver_cfg &cfg,
                       bool x_is_guess, tmx_info *info)
{
    const int sym = cfg.kind == TMX_SOLVER_PCG_NN_SYM ? 2 : (cfg.kind == TMX_SOLVER_PCG_NN_SYM1 ? 3 : 0);
    tmx_ctx *c = S.c;
    const double tol = cfg.tol > 0 ? cfg.tol : 1e-10;
    const int maxiter = cfg.maxiter > 0 ? cfg.maxiter : 10000;
    const double delta = cfg.delta > 0 ? cfg.delta : default_delta<P>();
    SpinorPtr r = S.field("r", F64, 1), rl = S.field("rl", P, 1), p = S.field("p", P, 1), q = S.field("q", P, 1);
    SpinorPtr xl = S.field("xl", F32, 1), z = S.field("z", F32, 1), tz = S.field("tz", F32, 1);
    SpinorPtr rf = P == F16 ? S.field("rf", F32, 1) : SpinorPtr{};
    TRY(S.need());
    // <p, N p> = |Mhat p|^2 from the per-slot norms of the operator's first
    // half when unshifted (as in cg_core); the step length stays on the device
    const bool shifted = sigma && sigma[0] != 0.0;
    double *alpha_d = static_cast<double *>(ws_get(c, "pcg_alpha", sizeof(double)));
    double *pnrm = shifted ? nullptr : static_cast<double *>(ws_get(c, "cg_pnrm", sizeof(double) * c->Vh));
    if (!alpha_d || (!shifted && !pnrm)) return set_err(c, TMX_ENOMEM, "solver workspace: out of device memory");
    double bb, rr, rmax, rho, dots[2];
    TRY((copy_field<F64, F64>(S, r, b, 1, &bb)));
    if (!std::isfinite(bb)) return set_err(c, TMX_EINVAL, "source with a non-finite entry");
    if (!x_is_guess) TRY(zero_field<F64>(S, x, 1));
    if (bb == 0) {
        TRY(zero_field<F64>(S, x, 1));
        if (info) info->true_residual = 0;
        return TMX_OK;
    }
    TRY(true_residual<P>(S, r, rl, true, b, x, sigma, 1, &rr));
    TRY(zero_field<F32>(S, xl, 1));
    TRY(pcg_apply_pc<P>(S, z, rl, tz, rf, sym));
    {
        OpPcgDots<P> d{};
        d.r = rl;
        d.z = z;
        d.q = rl;
        d.nf = 1;
        HTRY(run_blas(d, c->Vh, 1, c->red, c->stream), "pcg dots");
        TRY(fetch(c, 2, dots));
        rho = dots[0];
    }
    TRY((copy_field<P, F32>(S, p, z, 1, nullptr)));
    rmax = rr;
    int it = 0, nrel = 0, npc = 1;
    bool after_reliable = false;
    const double t0 = now_seconds();
    while (std::sqrt(rr) > tol * std::sqrt(bb) && it < maxiter) {
        if (!(rho > 0)) return set_err(c, TMX_ENOCONV, "preconditioned CG breakdown");
        if (shifted) {
            TRY(apply_shifted<P>(S, q, p, sigma, 1, nullptr));
        } else {
            TRY(S.N(q, p, P, 1, pnrm));
            OpSlotSum sum{};
            sum.v = pnrm;
            HTRY(run_blas(sum, c->Vh, 1, c->red, c->stream), "<p, N p>");
        }
        ++it;
        hipLaunchKernelGGL(pcg_alpha_kernel, dim3(1), dim3(64), 0, c->stream, c->red.result, rho, alpha_d,
                           c->red.host);
        HTRY(hipGetLastError(), "pcg step length");
        OpAxpyNorm<F32, P, P, P> up{};
        up.x = xl;
        up.p = p;
        up.r = rl;
        up.q = q;
        up.nf = 1;
        up.ad = alpha_d;
        HTRY(run_blas(up, c->Vh, 1, c->red, c->stream), "pcg update");
        TRY(fetch(c, 1, &rr));
        // the step length, from the pinned slot (written before the readback
        // just taken) or copied when the reduction buffer is not mapped
        double alpha = 0.0;
        if (c->red.host) {
            alpha = c->host_red[PCG_ALPHA_SLOT];
        } else {
            HTRY(hipMemcpy(&alpha, alpha_d, sizeof(double), hipMemcpyDeviceToHost), "pcg step length readback");
        }
        if (!(alpha > 0)) return set_err(c, TMX_ENOCONV, "preconditioned CG breakdown");
        if (!std::isfinite(rr)) return set_err(c, TMX_ENOCONV, "preconditioned CG: non-finite residual");
        rmax = std::max(rmax, rr);
        after_reliable = false;
        if (std::sqrt(rr) < delta * std::sqrt(rmax) || std::sqrt(rr) <= tol * std::sqrt(bb)) {
            OpAddTo<F64, F32> ad{};
            ad.x = x;
            ad.y = xl;
            ad.nf = 1;
            ad.zero_y = 1;
            HTRY(run_blas(ad, c->Vh, 1, c->red, c->stream), "pcg reliable add");
            TRY(true_residual<P>(S, r, rl, true, b, x, sigma, 1, &rr));
            rmax = rr;
            nrel++;
            after_reliable = true;
            if (std::sqrt(rr) <= tol * std::sqrt(bb)) break;
        }
        TRY(pcg_apply_pc<P>(S, z, rl, tz, rf, sym));
        ++npc;
        OpPcgDots<P> d{};
        d.r = rl;
        d.z = z;
        d.q = q;
        d.nf = 1;
        HTRY(run_blas(d, c->Vh, 1, c->red, c->stream), "pcg dots");
        TRY(fetch(c, 2, dots));
        double beta = after_reliable ? dots[0] / rho : -alpha * dots[1] / rho;
        if (!(beta > 0)) beta = 0;  // restart the direction
        OpAxpby<P, F32> px{};
        px.y = p;
        px.x = z;
        px.nf = 1;
        px.a[0] = 1.0;
        px.b[0] = beta;
        HTRY(run_blas(px, c->Vh, 1, c->red, c->stream), "pcg p update");
        rho = dots[0];
    }
    OpAddTo<F64, F32> ad{};
    ad.x = x;
    ad.y = xl;
    ad.nf = 1;
    ad.zero_y = 1;
    HTRY(run_blas(ad, c->Vh, 1, c->red, c->stream), "pcg final add");
    double tr;
    TRY(true_residual<P>(S, r, rl, false, b, x, sigma, 1, &tr));
    const double rel = std::sqrt(tr / bb);
    if (info) {
        info->iters += it;
        info->reliable_updates += nrel;
        info->restarts += npc;  // preconditioner applications (each K^dagger then K)
        info->true_residual = rel;
        info->seconds += now_seconds() - t0;
        info->gbytes += S.gbytes;
    }
    return rel <= tol ? TMX_OK : TMX_ENOCONV;
}

static int dispatch_cg(Sys &S, int prec, SpinorPtr x, SpinorPtr b, int cols, const double *sigma,
                       const tmx_solver_cfg &cfg, bool guess, tmx_info *info)
{
    if (prec == F64) return cg_solve<F64>(S, x, b, cols, sigma, cfg, guess, info);
    if (prec == F32) return cg_solve<F32>(S, x, b, cols, sigma, cfg, guess, info);
    return cg_solve<F16>(S, x, b, cols, sigma, cfg, guess, info);
}

// --------------------------------------------------------------------------
// multishift CG (low precision P), x_k accumulated in F32 (F64 when P = F64)
// --------------------------------------------------------------------------
template <int P>
static int mscg_core(Sys &S, std::vector<SpinorPtr> &xs, SpinorPtr b64, const double *shifts, int ns, double tol,
                     int maxiter, int *iters_out)
{
    tmx_ctx *c = S.c;
    constexpr int PX = P == F64 ? F64 : F32;
    SpinorPtr r = S.field("ms_r", P, 1);
    SpinorPtr q = S.field("ms_q", P, 1);
    std::vector<SpinorPtr> ps(ns);
    for (int k = 0; k < ns; ++k) ps[k] = S.field("ms_p" + std::to_string(k), P, 1);
    TRY(S.need());
    double bb;
    TRY((copy_field<P, F64>(S, r, b64, 1, &bb)));
    if (!std::isfinite(bb)) return set_err(c, TMX_EINVAL, "source with a non-finite entry");
    for (int k = 0; k < ns; ++k) {
        TRY(zero_field<PX>(S, xs[k], 1));
        TRY((copy_field<P, P>(S, ps[k], r, 1, nullptr)));
    }
    std::vector<double> zeta(ns, 1.0), zprev(ns, 1.0);
    std::vector<int> active(ns, bb > 0 ? 1 : 0), it_k(ns, 0);
    double aprev = 1.0, bprev = 0.0, rr = bb, best = bb;
    const double s0 = shifts[0];
    int it = 0, since_best = 0;
    while (it < maxiter) {
        int na = 0;
        for (int k = 0; k < ns; ++k) na += active[k];
        if (na == 0) break;
        double pq;
        TRY(apply_shifted<P>(S, q, ps[0], &s0, 1, &pq));
        ++it;
        if (!(pq > 0)) return set_err(c, TMX_ENOCONV, "multishift CG: breakdown");
        const double a = rr / pq;
        OpMsUpdate<PX, P, P> mu{};
        mu.r = r;
        mu.stride = c->Vh;
        mu.nf = S.nf;
        mu.nshift = ns;
        std::vector<double> zn(ns, 0.0);
        for (int k = 0; k < ns; ++k) {
            mu.xd[k] = xs[k].d;
            mu.pd[k] = ps[k].d;
            mu.active[k] = active[k];
            if (!active[k]) continue;
            const double ds = shifts[k] - s0;
            zn[k] = zeta[k] * zprev[k] * aprev / (a * bprev * (zprev[k] - zeta[k]) + zprev[k] * aprev * (1.0 + ds * a));
            mu.alpha[k] = zeta[k] != 0.0 ? a * zn[k] / zeta[k] : 0.0;
        }
        // r -= a q ; |r|^2
        OpRupdNorm<P, P> ru{};
        ru.r = r;
        ru.q = q;
        ru.nf = S.nf;
        ru.a[0] = a;
        HTRY(run_blas(ru, c->Vh, 1, c->red, c->stream), "ms residual");
        double rr1;
        TRY(fetch(c, 1, &rr1));
        if (!std::isfinite(rr1)) return set_err(c, TMX_ENOCONV, "multishift CG: non-finite residual");
        const double bt = rr1 / rr;
        for (int k = 0; k < ns; ++k) {
            if (!active[k]) continue;
            mu.zeta[k] = zn[k];
            mu.beta[k] = zeta[k] != 0.0 ? bt * (zn[k] / zeta[k]) * (zn[k] / zeta[k]) : 0.0;
        }
        HTRY(run_blas(mu, c->Vh, 1, c->red, c->stream), "ms update");
        for (int k = 0; k < ns; ++k) {
            if (!active[k]) continue;
            zprev[k] = zeta[k];
            zeta[k] = zn[k];
            it_k[k] = it;
            // residual of shift k is |zeta_k| |r|; drop it once converged
            if (std::fabs(zeta[k]) * std::sqrt(rr1) <= tol * std::sqrt(bb)) active[k] = 0;
        }
        aprev = a;
        bprev = bt;
        rr = rr1;
        // low-precision stagnation: the refinement stage takes over
        if (rr1 < best) {
            best = rr1;
            since_best = 0;
        } else if (++since_best > 50 || rr1 > 1e4 * best) {
            break;
        }
    }
    for (int k = 0; k < ns; ++k) iters_out[k] = it_k[k];
    return TMX_OK;
}

// CG from the current x (used to accept or rescue a preconditioned solve):
// sets info->fallback when iterations were needed.
int cg_fallback(tmx_ctx *c, int op, SpinorPtr x, SpinorPtr b, double tol, int maxiter, tmx_info *info)
{
    Sys S(c, op, 1);
    tmx_solver_cfg cfg{};
    cfg.kind = TMX_SOLVER_MPCG_F32;
    cfg.op = op;
    cfg.tol = tol;
    cfg.maxiter = maxiter;
    tmx_info inf{};
    int rc = dispatch_cg(S, F32, x, b, 1, nullptr, cfg, true, &inf);
    if (rc < 0) return rc;
    if (info) {
        if (inf.iters > 0) info->fallback = 1;
        info->iters += inf.iters;
        info->reliable_updates += inf.reliable_updates;
        info->true_residual = inf.true_residual;
        info->gbytes += S.gbytes;
    }
    return rc;
}

}  // namespace tmx

using namespace tmx;

extern "C" {

static int check_cfg(tmx_ctx *c, const tmx_solver_cfg *cfg)
{
    if (!cfg) return set_err(c, TMX_EINVAL, "null solver config");
    if (cfg->op != TMX_OP_PLUS && cfg->op != TMX_OP_MINUS && cfg->op != TMX_OP_ND && cfg->op != TMX_OP_WPLUS &&
        cfg->op != TMX_OP_WMINUS)
        return set_err(c, TMX_EINVAL, "bad op in solver config");
    if (!(cfg->tol > 0) && cfg->tol != 0) return set_err(c, TMX_EINVAL, "bad tolerance");
    return TMX_OK;
}

int tmx_fgcr_solve_internal(tmx_ctx *c, SpinorPtr x, SpinorPtr b, const tmx_solver_cfg *cfg, tmx_info *info);

// The entry points solve for b / |b| (per column) and scale the solution
// back: the FP32 and FP16 fields of the mixed-precision solvers then hold the
// same magnitudes whatever the source's scale (an FP16 solve of a source of
// norm 1e-27 broke down once its residual passed the FP32 range).  Columns of
// norm 0, or of a non-finite norm (rejected by the solver), keep scale 1.
static int normalize_columns(Sys &S, SpinorPtr B, int cols, double *scale)
{
    tmx_ctx *c = S.c;
    double nn[MAXR];
    TRY((copy_field<F64, F64>(S, B, B, cols, nn)));  // |b|^2 per column
    bool any = false;
    for (int k = 0; k < cols; ++k) {
        scale[k] = (nn[k] > 0 && std::isfinite(nn[k])) ? std::sqrt(nn[k]) : 1.0;
        any = any || scale[k] != 1.0;
    }
    if (!any) return TMX_OK;
    OpAxpby<F64, F64> o{};
    o.y = B;
    o.x = B;
    o.nf = S.nf;
    for (int k = 0; k < cols; ++k) {
        o.a[k] = 0.0;
        o.b[k] = 1.0 / scale[k];
    }
    return hip_err(c, run_blas(o, c->Vh * cols, cols, c->red, c->stream), "normalize source");
}

// X *= scale (per column), or X /= scale with inverse
static int scale_columns(Sys &S, SpinorPtr X, int cols, const double *scale, bool inverse)
{
    tmx_ctx *c = S.c;
    bool any = false;
    OpAxpby<F64, F64> o{};
    o.y = X;
    o.x = X;
    o.nf = S.nf;
    for (int k = 0; k < cols; ++k) {
        o.a[k] = 0.0;
        o.b[k] = inverse ? 1.0 / scale[k] : scale[k];
        any = any || scale[k] != 1.0;
    }
    if (!any) return TMX_OK;
    return hip_err(c, run_blas(o, c->Vh * cols, cols, c->red, c->stream), "scale solution");
}

int tmx_solve(tmx_ctx *c, double *x, const double *b, int nrhs, const tmx_solver_cfg *cfg, tmx_info *info)
{
    if (!c || !x || !b || nrhs < 1 || nrhs > MAXR) return c ? set_err(c, TMX_EINVAL, "tmx_solve: bad argument") : TMX_EINVAL;
    TRY(check_cfg(c, cfg));
    const double t0 = now_seconds();
    if (info) std::memset(info, 0, sizeof(tmx_info) * nrhs);
    Sys S(c, cfg->op, nrhs);
    const int kind = cfg->op == TMX_OP_ND ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, cfg->op == TMX_OP_ND));
    SpinorPtr X = S.field("x", F64), B = S.field("b", F64);
    TRY(S.need());
    if (!X.d || !B.d) return set_err(c, TMX_ENOMEM, "solver fields: out of device memory");
    HTRY(launch_pack_spinor(b, B, F64, kind, c->g, nrhs, c->stream), "pack b");
    if (cfg->use_initial_guess) HTRY(launch_pack_spinor(x, X, F64, kind, c->g, nrhs, c->stream), "pack x");
    double bscale[MAXR];
    TRY(normalize_columns(S, B, nrhs, bscale));
    if (cfg->use_initial_guess) TRY(scale_columns(S, X, nrhs, bscale, true));
    int rc;
    switch (cfg->kind) {
    case TMX_SOLVER_CG:
        rc = dispatch_cg(S, F64, X, B, nrhs, nullptr, *cfg, cfg->use_initial_guess != 0, info);
        break;
    case TMX_SOLVER_MPCG_F32:
        rc = dispatch_cg(S, F32, X, B, nrhs, nullptr, *cfg, cfg->use_initial_guess != 0, info);
        break;
    case TMX_SOLVER_MPCG_F16:
        rc = dispatch_cg(S, F16, X, B, nrhs, nullptr, *cfg, cfg->use_initial_guess != 0, info);
        break;
    case TMX_SOLVER_PCG_NN:
    case TMX_SOLVER_PCG_NN_SYM:
    case TMX_SOLVER_PCG_NN_SYM1:
        if (nrhs != 1) return set_err(c, TMX_EINVAL, "the preconditioned CG solves one right-hand side at a time");
        if (cfg->op != TMX_OP_PLUS && cfg->op != TMX_OP_MINUS)
            return set_err(c, TMX_EINVAL, "the learned preconditioner is built for the degenerate Schur operator");
        TRY(ensure_ready(c, F32, false));
        rc = (cfg->inner_prec == TMX_F16)
                 ? pcg_nn_core<F16>(S, X, B, nullptr, *cfg, cfg->use_initial_guess != 0, info)
                 : pcg_nn_core<F32>(S, X, B, nullptr, *cfg, cfg->use_initial_guess != 0, info);
        if (rc == TMX_ENOCONV && info && std::isfinite(info->true_residual)) {
            // fall back to plain mixed-precision CG from the current x
            tmx_info inf{};
            rc = dispatch_cg(S, F32, X, B, 1, nullptr, *cfg, true, &inf);
            info->fallback = 1;
            info->iters += inf.iters;
            info->true_residual = inf.true_residual;
        }
        break;
    case TMX_SOLVER_FGCR_NN:
        if (nrhs != 1) return set_err(c, TMX_EINVAL, "FGCR solves one right-hand side at a time");
        if (!cfg->use_initial_guess) TRY(zero_field<F64>(S, X, 1));
        rc = tmx_fgcr_solve_internal(c, X, B, cfg, info);
        break;
    default:
        return set_err(c, TMX_EINVAL, "unknown solver kind");
    }
    if (rc < 0) return rc;
    TRY(scale_columns(S, X, nrhs, bscale, false));
    HTRY(launch_unpack_spinor(x, X, F64, kind, c->g, nrhs, c->stream), "unpack x");
    HTRY(hipStreamSynchronize(c->stream), "solve sync");
    if (info)
        for (int k = 0; k < nrhs; ++k) info[k].seconds = now_seconds() - t0;
    return rc;
}

static int check_shifts(tmx_ctx *c, const double *shifts, int nshift)
{
    for (int k = 0; k < nshift; ++k)
        if (!(shifts[k] >= 0) || shifts[k] < shifts[0] || !std::isfinite(shifts[k]))
            return set_err(c, TMX_EINVAL, "shifts must be finite, >= 0 and shifts[0] the smallest");
    return TMX_OK;
}

// The batched multishift solve of B (packed FP64) for every shift: one
// low-precision multishift CG, then shift-by-shift refinement with FP64
// reliable updates.  With cfg->kind = TMX_SOLVER_PCG_NN the refinement is
// the CG preconditioned by the learned network (K K^dagger approximates
// N^{-1}, and (N + sigma)^{-1} for the small shifts that dominate the
// cost), falling back to plain MP-CG from its iterate if it stalls.  Each
// refined FP64 solution is handed to consume(k, X_k) in shift order (X_k is
// reused for the next shift).
static int multishift_run(tmx_ctx *c, Sys &S, SpinorPtr B, const double *shifts, int nshift,
                          const tmx_solver_cfg *cfg, tmx_info *info,
                          const std::function<int(int, SpinorPtr)> &consume)
{
    const int prec = (cfg->inner_prec == TMX_F16 || cfg->inner_prec == TMX_F64) ? cfg->inner_prec : TMX_F32;
    const double tol = cfg->tol > 0 ? cfg->tol : 1e-10;
    const double inner = cfg->inner_tol > 0 ? cfg->inner_tol : (prec == TMX_F16 ? 5e-4 : (prec == TMX_F32 ? 1e-6 : tol));
    const int maxiter = cfg->maxiter > 0 ? cfg->maxiter : 10000;
    const bool pcg_nn = cfg->kind == TMX_SOLVER_PCG_NN || cfg->kind == TMX_SOLVER_PCG_NN_SYM ||
                        cfg->kind == TMX_SOLVER_PCG_NN_SYM1;
    if (pcg_nn) {
        if (cfg->op != TMX_OP_PLUS && cfg->op != TMX_OP_MINUS)
            return set_err(c, TMX_EINVAL, "the learned preconditioner is built for the degenerate Schur operator");
        TRY(ensure_ready(c, F32, false));  // the network runs on the FP32 links
    }
    // low-precision multishift stage
    const int PX = prec == F64 ? F64 : F32;
    std::vector<SpinorPtr> xs(nshift);
    for (int k = 0; k < nshift; ++k) xs[k] = S.field("msx" + std::to_string(k), PX, 1);
    TRY(S.need());
    std::vector<int> its(nshift, 0);
    int r;
    if (prec == F64)
        r = mscg_core<F64>(S, xs, B, shifts, nshift, inner, maxiter, its.data());
    else if (prec == F32)
        r = mscg_core<F32>(S, xs, B, shifts, nshift, inner, maxiter, its.data());
    else
        r = mscg_core<F16>(S, xs, B, shifts, nshift, inner, maxiter, its.data());
    if (r < 0) return r;
    const double ms_gb = S.gbytes;
    // shift-by-shift refinement with FP64 reliable updates
    int rc = TMX_OK;
    SpinorPtr X = S.field("msx64", F64, 1);
    TRY(S.need());
    for (int k = 0; k < nshift; ++k) {
        if (prec == F64)
            TRY((copy_field<F64, F64>(S, X, xs[k], 1, nullptr)));
        else
            TRY((copy_field<F64, F32>(S, X, xs[k], 1, nullptr)));
        tmx_solver_cfg rc_cfg = *cfg;
        rc_cfg.tol = tol;
        rc_cfg.maxiter = maxiter;
        tmx_info inf{};
        S.gbytes = 0;
        const double sk = shifts[k];
        int rk;
        if (pcg_nn) {
            rk = prec == F16 ? pcg_nn_core<F16>(S, X, B, &sk, rc_cfg, true, &inf)
                             : pcg_nn_core<F32>(S, X, B, &sk, rc_cfg, true, &inf);
            if (rk == TMX_ENOCONV && std::isfinite(inf.true_residual)) {
                tmx_info fb{};
                rk = dispatch_cg(S, F32, X, B, 1, &sk, rc_cfg, true, &fb);
                inf.fallback = 1;
                inf.iters += fb.iters;
                inf.reliable_updates += fb.reliable_updates;
                inf.true_residual = fb.true_residual;
                inf.gbytes += fb.gbytes;
            }
        } else {
            rk = dispatch_cg(S, prec, X, B, 1, &sk, rc_cfg, true, &inf);
        }
        if (rk < 0) return rk;
        if (rk == TMX_ENOCONV) rc = TMX_ENOCONV;
        TRY(consume(k, X));
        if (info) {
            info[k].iters = its[k] + inf.iters;
            info[k].reliable_updates = inf.reliable_updates;
            info[k].restarts = inf.restarts;
            info[k].fallback = inf.fallback;
            info[k].true_residual = inf.true_residual;
            info[k].gbytes = inf.gbytes + (k == 0 ? ms_gb : 0.0);
        }
    }
    return rc;
}

int tmx_multishift_solve(tmx_ctx *c, double *x, const double *b, const double *shifts, int nshift,
                         const tmx_solver_cfg *cfg, tmx_info *info)
{
    if (!c || !x || !b || !shifts || nshift < 1 || nshift > MAXR)
        return c ? set_err(c, TMX_EINVAL, "tmx_multishift_solve: bad argument") : TMX_EINVAL;
    TRY(check_cfg(c, cfg));
    TRY(check_shifts(c, shifts, nshift));
    const double t0 = now_seconds();
    if (info) std::memset(info, 0, sizeof(tmx_info) * nshift);
    const bool nd = cfg->op == TMX_OP_ND;
    const int kind = nd ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, nd));
    Sys S(c, cfg->op, 1);
    SpinorPtr B = S.field("msb", F64, 1);
    TRY(S.need());
    HTRY(launch_pack_spinor(b, B, F64, kind, c->g, 1, c->stream), "pack b");
    double bscale;
    TRY(normalize_columns(S, B, 1, &bscale));
    const int rc = multishift_run(c, S, B, shifts, nshift, cfg, info, [&](int k, SpinorPtr X) {
        const int r = scale_columns(S, X, 1, &bscale, false);
        if (r) return r;
        return hip_err(c, launch_unpack_spinor(x + (size_t)k * c->Vh * 24 * S.nf, X, F64, kind, c->g, 1, c->stream),
                       "unpack x_k");
    });
    if (rc < 0) return rc;
    HTRY(hipStreamSynchronize(c->stream), "multishift sync");
    if (info)
        for (int k = 0; k < nshift; ++k) info[k].seconds = now_seconds() - t0;
    return rc;
}

static int check_rational(tmx_ctx *c, double a0, const double *coeffs, const double *shifts, int nshift,
                          const tmx_solver_cfg *cfg)
{
    if (!coeffs || !shifts || nshift < 1 || nshift > MAXR || !std::isfinite(a0))
        return set_err(c, TMX_EINVAL, "rational function: bad argument");
    TRY(check_cfg(c, cfg));
    TRY(check_shifts(c, shifts, nshift));
    for (int k = 0; k < nshift; ++k)
        if (!std::isfinite(coeffs[k])) return set_err(c, TMX_EINVAL, "coefficients must be finite");
    return TMX_OK;
}

// out = a0 in + sum_k coeffs[k] (N + shifts[k])^{-1} in on internal FP64
// fields (out != in): out = a0 in, then out += a_k x_k as each shift's
// solution is refined
static int rational_internal(tmx_ctx *c, Sys &S, SpinorPtr out, SpinorPtr in, double a0, const double *coeffs,
                             const double *shifts, int nshift, const tmx_solver_cfg *cfg, tmx_info *info)
{
    TRY(zero_field<F64>(S, out, 1));
    OpAxpby<F64, F64> ax{};
    ax.y = out;
    ax.x = in;
    ax.nf = S.nf;
    ax.a[0] = a0;
    ax.b[0] = 1.0;
    HTRY(run_blas(ax, c->Vh, 1, c->red, c->stream), "rational a0 b");
    return multishift_run(c, S, in, shifts, nshift, cfg, info, [&](int k, SpinorPtr X) {
        OpAxpby<F64, F64> o{};
        o.y = out;
        o.x = X;
        o.nf = S.nf;
        o.a[0] = coeffs[k];
        o.b[0] = 1.0;
        return hip_err(c, run_blas(o, c->Vh, 1, c->red, c->stream), "rational accumulate");
    });
}

int tmx_rational_apply(tmx_ctx *c, double *out, const double *b, double a0, const double *coeffs,
                       const double *shifts, int nshift, const tmx_solver_cfg *cfg, tmx_info *info)
{
    if (!c || !out || !b) return c ? set_err(c, TMX_EINVAL, "tmx_rational_apply: bad argument") : TMX_EINVAL;
    TRY(check_rational(c, a0, coeffs, shifts, nshift, cfg));
    const double t0 = now_seconds();
    if (info) std::memset(info, 0, sizeof(tmx_info) * nshift);
    const bool nd = cfg->op == TMX_OP_ND;
    const int kind = nd ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, nd));
    Sys S(c, cfg->op, 1);
    SpinorPtr B = S.field("msb", F64, 1), A = S.field("ra_acc", F64, 1);
    TRY(S.need());
    HTRY(launch_pack_spinor(b, B, F64, kind, c->g, 1, c->stream), "pack b");
    const int rc = rational_internal(c, S, A, B, a0, coeffs, shifts, nshift, cfg, info);
    if (rc < 0) return rc;
    HTRY(launch_unpack_spinor(out, A, F64, kind, c->g, 1, c->stream), "unpack out");
    HTRY(hipStreamSynchronize(c->stream), "rational sync");
    if (info)
        for (int k = 0; k < nshift; ++k) info[k].seconds = now_seconds() - t0;
    return rc;
}

int tmx_rational_force(tmx_ctx *c, double *force, const double *phi, const double *coeffs, const double *shifts,
                       int nshift, const tmx_solver_cfg *cfg, int accumulate, tmx_info *info)
{
    if (!c || !force || !phi) return c ? set_err(c, TMX_EINVAL, "tmx_rational_force: bad argument") : TMX_EINVAL;
    TRY(check_rational(c, 0.0, coeffs, shifts, nshift, cfg));
    if (cfg->op != TMX_OP_PLUS && cfg->op != TMX_OP_MINUS && cfg->op != TMX_OP_ND)
        return set_err(c, TMX_EINVAL, "the force is built for the degenerate and the two-flavour Schur operators");
    if (c->clover_from_host)
        return set_err(c, TMX_EINVAL, "the clover force needs the clover term built from the links");
    const double t0 = now_seconds();
    if (info) std::memset(info, 0, sizeof(tmx_info) * nshift);
    const bool nd = cfg->op == TMX_OP_ND;
    const int kind = nd ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, nd));
    Sys S(c, cfg->op, 1);
    SpinorPtr B = S.field("msb", F64, 1), Y = S.field("rf_y", F64, 1);
    TRY(S.need());
    HTRY(launch_pack_spinor(phi, B, F64, kind, c->g, 1, c->stream), "pack phi");
    // F = -2 sum_k a_k [hop + clover force](x_k, Mhat x_k), x_k = (N + s_k)^{-1} phi,
    // added shift by shift as each solution is refined
    const int rc = multishift_run(c, S, B, shifts, nshift, cfg, info, [&](int k, SpinorPtr X) {
        int r = op_mhat(c, Y, X, cfg->op, F64, 0, 1);
        if (r) return r;
        return force_internal(c, force, X, Y, cfg->op, -2.0 * coeffs[k], (accumulate || k > 0) ? 1 : 0, 3);
    });
    if (rc < 0) return rc;
    HTRY(hipStreamSynchronize(c->stream), "rational force sync");
    if (info)
        for (int k = 0; k < nshift; ++k) info[k].seconds = now_seconds() - t0;
    return rc;
}

int tmx_rational_correction(tmx_ctx *c, const double *eta, double a0, const double *coeffs, const double *shifts,
                            int nshift, double tol, int maxterms, const tmx_solver_cfg *cfg, double *exponent,
                            int *terms)
{
    if (!c || !eta || !exponent || maxterms < 1 || !(tol > 0))
        return c ? set_err(c, TMX_EINVAL, "tmx_rational_correction: bad argument") : TMX_EINVAL;
    TRY(check_rational(c, a0, coeffs, shifts, nshift, cfg));
    const bool nd = cfg->op == TMX_OP_ND;
    const int kind = nd ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, nd));
    Sys S(c, cfg->op, 1);
    SpinorPtr E = S.field("rc_eta", F64, 1), V = S.field("rc_v", F64, 1), T1 = S.field("rc_t1", F64, 1),
              T2 = S.field("rc_t2", F64, 1), W = S.field("rc_w", F64, 1);
    TRY(S.need());
    HTRY(launch_pack_spinor(eta, E, F64, kind, c->g, 1, c->stream), "pack eta");
    TRY((copy_field<F64, F64>(S, V, E, 1, nullptr)));
    // E = sum_k binom(-1/2, k) <eta, Z^k eta>,  Z = N R(N)^2 - 1
    double sum = 0.0, coef = 1.0, dots[2];
    int k = 0, rc = TMX_OK;
    bool converged = false;
    while (k < maxterms) {
        ++k;
        int r = rational_internal(c, S, T1, V, a0, coeffs, shifts, nshift, cfg, nullptr);
        if (r < 0) return r;
        if (r == TMX_ENOCONV) rc = r;
        r = rational_internal(c, S, T2, T1, a0, coeffs, shifts, nshift, cfg, nullptr);
        if (r < 0) return r;
        if (r == TMX_ENOCONV) rc = r;
        TRY(op_mdagm(c, W, T2, cfg->op, F64, 1));
        OpAxpby<F64, F64> z{};  // V = W - V = Z V
        z.y = V;
        z.x = W;
        z.nf = S.nf;
        z.a[0] = 1.0;
        z.b[0] = -1.0;
        HTRY(run_blas(z, c->Vh, 1, c->red, c->stream), "Z v");
        OpCdot<F64, F64> d{};
        d.a = E;
        d.b = V;
        d.nf = S.nf;
        HTRY(run_blas(d, c->Vh, 1, c->red, c->stream), "<eta, Z^k eta>");
        TRY(fetch(c, 2, dots));
        coef *= (-0.5 - (k - 1)) / k;
        const double term = coef * dots[0];
        sum += term;
        if (!std::isfinite(sum)) return set_err(c, TMX_ENOCONV, "rational correction: non-finite series");
        if (std::fabs(term) <= tol * std::fabs(sum)) {
            converged = true;
            break;
        }
    }
    *exponent = sum;
    if (terms) *terms = k;
    if (!converged && rc == TMX_OK) {
        set_err(c, TMX_ENOCONV, "rational correction: series not converged within maxterms");
        rc = TMX_ENOCONV;
    }
    return rc;
}

int tmx_solve_mhat(tmx_ctx *c, double *x, const double *b, int dagger, const tmx_solver_cfg *cfg, tmx_info *info)
{
    if (!c || !x || !b) return c ? set_err(c, TMX_EINVAL, "tmx_solve_mhat: bad argument") : TMX_EINVAL;
    TRY(check_cfg(c, cfg));
    // Mhat x = b  <=>  N x = Mhat^dagger b ;  Mhat^dagger x = b  <=>  (Mhat Mhat^dagger) x = Mhat b,
    // solved as x = Mhat y with N y = b... use the normal equations of the right operator:
    // for dagger = 1: x = Mhat z where N z = b  (N = Mhat^dagger Mhat).
    const bool nd = cfg->op == TMX_OP_ND;
    const int nf = nd ? 2 : 1;
    const int kind = nd ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    TRY(ensure_ready(c, F64, nd));
    Sys S(c, cfg->op, 1);
    SpinorPtr B = S.field("mh_b", F64, 1), T = S.field("mh_t", F64, 1);
    TRY(S.need());
    const size_t cbytes = (size_t)c->Vh * 24 * nf * sizeof(double);
    void *canon = ws_get(c, "mh_canon", cbytes);
    if (!canon) return set_err(c, TMX_ENOMEM, "solver fields: out of device memory");
    HTRY(launch_pack_spinor(b, B, F64, kind, c->g, 1, c->stream), "pack b");
    if (!dagger) {
        TRY(op_mhat(c, T, B, cfg->op, F64, 1, 1));  // T = Mhat^dagger b
        HTRY(launch_unpack_spinor((double *)canon, T, F64, kind, c->g, 1, c->stream), "unpack");
        tmx_solver_cfg cc = *cfg;
        return tmx_solve(c, x, (const double *)canon, 1, &cc, info);
    }
    // dagger: solve N z = b, then x = Mhat z
    tmx_solver_cfg cc = *cfg;
    int rc = tmx_solve(c, (double *)canon, b, 1, &cc, info);
    if (rc < 0) return rc;
    HTRY(launch_pack_spinor((const double *)canon, T, F64, kind, c->g, 1, c->stream), "pack z");
    TRY(op_mhat(c, B, T, cfg->op, F64, 0, 1));
    HTRY(launch_unpack_spinor(x, B, F64, kind, c->g, 1, c->stream), "unpack x");
    HTRY(hipStreamSynchronize(c->stream), "sync");
    return rc;
}

}  // extern "C"
