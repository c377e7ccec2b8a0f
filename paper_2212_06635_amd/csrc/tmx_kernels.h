// Launch interface of the tmx HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "tmx_device.h"

namespace tmx {

struct DslashArgs {
    Geom g;
    int parity;        // output parity
    int nrhs;          // right-hand sides interleaved per site
    SpinorPtr out;     // output field (output parity)
    SpinorPtr in;      // hopping input (other parity)
    SpinorPtr x;       // diagonal input (output parity), MODE_DIAG only
    LinkPtr U;         // compressed links, both parities
    const void *clov;  // Hermitian A of the output parity
    const void *inv;   // MODE_INV: full inverse (deg) or Hermitian inverse factor (nd)
    double nu;         // nu (deg) or nubar (nd), already times 2 kappa
    double epst;       // 2 kappa epsbar (nd)
    double kfac;       // MODE_DIAG: coefficient of the hopping term
    int sgn;           // sign of the twist
    int t_bc;          // fermion time boundary factor
    int g5in, g5x, g5out;
    int xcd;           // XCD-aware block order
    double *nrm;       // MODE_DIAG, if set: |out|^2 of every slot (FP64), for <p, N p> = |Mhat p|^2
    double rho;        // MODE_DIAG, one flavour: adds i rho x to the final output (after g5out)
    int r0, rg;        // right-hand sides r0 .. r0 + rg - 1 of the nrhs per site (rg = 0: all)
    int spt;           // sites (slots) per thread: 1, or a grid-stride loop over spt of them
};

hipError_t launch_dslash(int prec, int nf, int mode, const DslashArgs &a, hipStream_t st, int block);

// hopping-term force (force.hip): out[lex][mu] (3x3 complex, canonical link
// layout) = coeff TA(Q_mu(x)) (+ out if accumulate); X, Y odd, u = K1(s) X,
// w = K1(-s, g5 in) Y even, all FP64
struct ForceArgs {
    Geom g;
    LinkPtr U;
    SpinorPtr X, Y, u, w;
    int t_bc;
    double kfac;  // kappa^2
    double coeff;
    int accumulate;
    double *out;
    int xcd;
};
hipError_t launch_hop_force(const ForceArgs &f, hipStream_t st);

// ---- gauge / clover set-up (gauge.hip) ----------------------------------
// canonical host-order links (device, complex128) -> compressed FP64 links
hipError_t launch_pack_links(const double *canon, double *links64, Geom g, hipStream_t st);
// compressed FP64 -> compressed FP32 / FP16 links
hipError_t launch_convert_links(const double *links64, void *dst, int prec, Geom g, hipStream_t st);
// clover term A = 1 + T on both parities (Hermitian packed, FP64)
hipError_t launch_clover_build(const double *links64, double *clov64, Geom g, double kappa, double csw,
                               hipStream_t st);
// canonical [lex][2][6][6] complex128 -> packed A = 1 + T (FP64)
hipError_t launch_clover_from_canonical(const double *canonT, double *clov64, Geom g, hipStream_t st);
hipError_t launch_clover_to_canonical(const double *clov64, double *canonT, Geom g, hipStream_t st);
// degenerate inverse (A_ee + i nu g5)^{-1}, full 6x6 per chirality (FP64)
hipError_t launch_clover_inv(const double *clov64_even, double *inv64, Geom g, double nu, hipStream_t st);
// two-flavour inverse factor (A_ee^2 + nubar^2 - epst^2)^{-1}, Hermitian packed (FP64)
hipError_t launch_clover_inv_nd(const double *clov64_even, double *invnd64, Geom g, double nubar, double epst,
                                hipStream_t st);
// FP64 per-site real sequences -> FP32 / FP16 (n reals per site, Vh sites)
hipError_t launch_convert_seq(const double *src, void *dst, int prec, int nreal, long nsite, hipStream_t st);

// ---- layout conversion (pack.hip) ----------------------------------------
// canonical complex128 fields <-> internal spinor fields.
// kind: 0 odd, 1 odd nd, 2 full, 3 full nd
hipError_t launch_pack_spinor(const double *canon, SpinorPtr dst, int prec, int kind, Geom g, int nvec,
                              hipStream_t st);
hipError_t launch_unpack_spinor(double *canon, SpinorPtr src, int prec, int kind, Geom g, int nvec,
                                hipStream_t st);

// ---- vector algebra with FP64 accumulation (blas.hip) -------------------
struct Red;  // reduction workspace
}  // namespace tmx
