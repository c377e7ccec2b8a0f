// Clover-term force (force.hip): declarations shared by the kernels and the
// library entry point.
#pragma once
#include "tmx_device.h"

namespace tmx {

// out[lex][rho] (3x3 complex, canonical link layout) = coeff TA(Z_rho(x))
// (+ out if accumulate), the link derivative of Re<Y, Mhat X> through the
// clover term of both parities (hopping matrices fixed).  X, Y odd,
// u = K1(s) X, w = K1(-s, g5 in) Y even, all FP64.  H is the insertion
// workspace: 6 planes x 9 reals (the Hermitian matrix: diagonal, then the
// upper triangle as (re, im)) x 2 Vh doubles, site index p Vh + s.
struct CloverForceArgs {
    Geom g;
    LinkPtr U;
    SpinorPtr X, Y, u, w;
    double kfac;  // kappa^2, the weight of the even-site term
    double kc8;   // kappa csw / 8
    double coeff;
    int accumulate;
    double *H;
    int h_acc;  // insertions: add to H (the next flavour of a two-flavour field) instead of writing it
    double *KA;  // plaquette loops: 6 planes x 16 reals (traceless Hermitian part K of the loop
                 // with insertions, traceless anti-Hermitian part A of the plain loop) x 2 Vh doubles
    double *out;
    int xcd;  // XCD-contiguous workgroup order of the link sums
};
// the sigma-plane insertions H of one flavour (written, or added with h_acc)
hipError_t launch_clover_insertions(const CloverForceArgs &f, hipStream_t st);
// the plaquette loops with H inserted (into KA), then the link sums from them (into out)
hipError_t launch_clover_link_sums(const CloverForceArgs &f, hipStream_t st);

}  // namespace tmx
