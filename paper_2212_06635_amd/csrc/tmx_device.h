// Device-side building blocks shared by the tmx kernels (gfx950).
//
// Data layout in HBM ("site-major structure of arrays"): every per-site
// record of n reals (a spinor, a compressed link, a clover block) is stored
// as n/w arrays of 16-byte vectors, w = 2 doubles, 4 floats or 8 halves.
// Vector k of site s lives at base[k * stride + s], so one load instruction
// of a 64-lane wavefront reads 64 consecutive 16-byte vectors (1 KiB,
// perfectly coalesced).  FP16 spinors additionally carry one FP32 scale per
// (flavour, site) after the vectors; FP16 links use three 8-byte vectors.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmx {

enum { F64 = 0, F32 = 1, F16 = 2 };

template <int P> struct RealOf { using type = float; };
template <> struct RealOf<F64> { using type = double; };

// -------------------------------------------------------------------------
// complex arithmetic
// -------------------------------------------------------------------------
template <typename R> struct cx {
    R re, im;
};

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// i * a
template <typename R> __device__ __forceinline__ cx<R> imul(cx<R> a) { return {-a.im, a.re}; }
// a += b * c
template <typename R> __device__ __forceinline__ void cmac(cx<R> &a, cx<R> b, cx<R> c)
{
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename R> __device__ __forceinline__ void cmac_conj(cx<R> &a, cx<R> b, cx<R> c)
{
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(-b.im, c.re, a.im);
}

// Register fence: an empty asm that "modifies" the values forces everything
// that produces them to be computed before any later memory operation (the
// asm is volatile, so it is ordered with loads and stores).  Used to keep a
// stencil from holding every neighbour's data in registers at once.
template <typename R> __device__ __forceinline__ void reg_fence(cx<R> *v, int n)
{
#pragma unroll
    for (int i = 0; i < n; ++i) asm volatile("" : "+v"(v[i].re), "+v"(v[i].im));
}

// -------------------------------------------------------------------------
// lattice geometry of one parity
// -------------------------------------------------------------------------
// Internal site order of one parity.  x/2 and y run fastest (a wavefront
// covers whole x rows of consecutive y, so each of its loads is one
// contiguous 1 KiB segment and every neighbour load a uniformly shifted
// one).  The (z, t) planes are then visited in tiles of zb x tb planes,
// z fastest inside a tile, tiles z-major:
//     plane = ((t / tb) * (Lz / zb) + z / zb) * (zb * tb) + (t % tb) * zb + z % zb
//     s     = (plane * Ly + y) * Lx/2 + x/2
// so the z and t neighbours of a site are at most one tile of planes away
// except for the t hops that leave a tile (1 in tb of them).  zb = tb = 1
// is plain checkerboard order.  zb and tb are powers of two.
struct Geom {
    int L[4];    // Lx, Ly, Lz, Lt
    int Lxh;     // Lx / 2
    int Vh;      // sites per parity
    int zbs;     // log2(zb)
    int tbs;     // log2(tb)
};

// coordinates of internal site s of parity p
__device__ __forceinline__ void cb_coords(const Geom &g, int s, int p, int x[4])
{
    const int xh = s % g.Lxh;
    int r = s / g.Lxh;
    x[1] = r % g.L[1];
    r /= g.L[1];  // plane
    const int zl = r & ((1 << g.zbs) - 1);
    r >>= g.zbs;
    const int tl = r & ((1 << g.tbs) - 1);
    r >>= g.tbs;
    const int nzt = g.L[2] >> g.zbs;
    x[2] = ((r % nzt) << g.zbs) + zl;
    x[3] = ((r / nzt) << g.tbs) + tl;
    x[0] = 2 * xh + ((x[1] + x[2] + x[3] + p) & 1);
}

// internal index of the site with coordinates x (any parity)
__device__ __forceinline__ int cb_index(const Geom &g, const int x[4])
{
    const int nzt = g.L[2] >> g.zbs;
    const int plane = ((((x[3] >> g.tbs) * nzt + (x[2] >> g.zbs)) << g.tbs) + (x[3] & ((1 << g.tbs) - 1))) << g.zbs;
    return ((plane + (x[2] & ((1 << g.zbs) - 1))) * g.L[1] + x[1]) * g.Lxh + (x[0] >> 1);
}

// -------------------------------------------------------------------------
// 16-byte vector loads / stores of per-site real sequences
// -------------------------------------------------------------------------
__device__ __forceinline__ void h8_to_f(const uint4 &v, float *o)
{
    const __half2 *h = reinterpret_cast<const __half2 *>(&v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float2 f = __half22float2(h[k]);
        o[2 * k] = f.x;
        o[2 * k + 1] = f.y;
    }
}
__device__ __forceinline__ uint4 f_to_h8(const float *o)
{
    uint4 v;
    __half2 *h = reinterpret_cast<__half2 *>(&v);
#pragma unroll
    for (int k = 0; k < 4; ++k) h[k] = __floats2half2_rn(o[2 * k], o[2 * k + 1]);
    return v;
}
__device__ __forceinline__ void h4_to_f(const uint2 &v, float *o)
{
    const __half2 *h = reinterpret_cast<const __half2 *>(&v);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        float2 f = __half22float2(h[k]);
        o[2 * k] = f.x;
        o[2 * k + 1] = f.y;
    }
}
__device__ __forceinline__ uint2 f_to_h4(const float *o)
{
    uint2 v;
    __half2 *h = reinterpret_cast<__half2 *>(&v);
#pragma unroll
    for (int k = 0; k < 2; ++k) h[k] = __floats2half2_rn(o[2 * k], o[2 * k + 1]);
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  With xcd != 0 the launch index is remapped so that XCD k works on one
// contiguous 1/8 of the sites: neighbours in y, z and t then mostly hit the
// L2 that already holds them.  (The map is a permutation of the blocks for
// any grid, so the result never depends on the dispatch order.)
__device__ __forceinline__ int xcd_block(int xcd)
{
    const int b = blockIdx.x;
    if (!xcd) return b;
    const int nb = gridDim.x, q = nb / 8, r = nb % 8;
    const int k = b % 8, i = b / 8;
    return k * q + (k < r ? k : r) + i;
}

// 16-byte load; NT = non-temporal (streamed operands such as links and
// clover blocks are read once per sweep: keeping them out of the way in L2
// leaves room for the neighbour spinors, which are read eight times)
typedef double ev_d2 __attribute__((ext_vector_type(2)));
typedef float ev_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int ev_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int ev_u2 __attribute__((ext_vector_type(2)));

template <bool NT> __device__ __forceinline__ double2 ldv(const double2 *p)
{
    if constexpr (NT) {
        const ev_d2 v = __builtin_nontemporal_load(reinterpret_cast<const ev_d2 *>(p));
        return make_double2(v.x, v.y);
    } else {
        return *p;
    }
}
template <bool NT> __device__ __forceinline__ float4 ldv(const float4 *p)
{
    if constexpr (NT) {
        const ev_f4 v = __builtin_nontemporal_load(reinterpret_cast<const ev_f4 *>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT> __device__ __forceinline__ uint4 ldv(const uint4 *p)
{
    if constexpr (NT) {
        const ev_u4 v = __builtin_nontemporal_load(reinterpret_cast<const ev_u4 *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT> __device__ __forceinline__ uint2 ldv(const uint2 *p)
{
    if constexpr (NT) {
        const ev_u2 v = __builtin_nontemporal_load(reinterpret_cast<const ev_u2 *>(p));
        return make_uint2(v.x, v.y);
    } else {
        return *p;
    }
}

// Load N reals (N a multiple of the vector width) of site s.
template <int P, int N, typename R, bool NT = false>
__device__ __forceinline__ void load_seq(const void *base, long stride, long s, R *o)
{
    if constexpr (P == F64) {
        const double2 *b = static_cast<const double2 *>(base);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
            double2 v = ldv<NT>(b + k * stride + s);
            o[2 * k] = v.x;
            o[2 * k + 1] = v.y;
        }
    } else if constexpr (P == F32) {
        const float4 *b = static_cast<const float4 *>(base);
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            float4 v = ldv<NT>(b + k * stride + s);
            o[4 * k] = v.x;
            o[4 * k + 1] = v.y;
            o[4 * k + 2] = v.z;
            o[4 * k + 3] = v.w;
        }
    } else {
        const uint4 *b = static_cast<const uint4 *>(base);
#pragma unroll
        for (int k = 0; k < N / 8; ++k) {
            float f8[8];
            h8_to_f(ldv<NT>(b + k * stride + s), f8);
#pragma unroll
            for (int j = 0; j < 8; ++j) o[8 * k + j] = f8[j];
        }
    }
}

// Store N reals of site s; NT marks the stores non-temporal (data written once
// and not read again by the same kernel).
template <int P, int N, typename R, bool NT = false>
__device__ __forceinline__ void store_seq(void *base, long stride, long s, const R *o)
{
    if constexpr (P == F64) {
        ev_d2 *b = static_cast<ev_d2 *>(base);
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
            const ev_d2 v = {(double)o[2 * k], (double)o[2 * k + 1]};
            if constexpr (NT)
                __builtin_nontemporal_store(v, b + k * stride + s);
            else
                b[k * stride + s] = v;
        }
    } else if constexpr (P == F32) {
        ev_f4 *b = static_cast<ev_f4 *>(base);
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const ev_f4 v = {(float)o[4 * k], (float)o[4 * k + 1], (float)o[4 * k + 2], (float)o[4 * k + 3]};
            if constexpr (NT)
                __builtin_nontemporal_store(v, b + k * stride + s);
            else
                b[k * stride + s] = v;
        }
    } else {
        static_assert(!NT, "half-precision stores are not marked non-temporal");
        uint4 *b = static_cast<uint4 *>(base);
#pragma unroll
        for (int k = 0; k < N / 8; ++k) {
            float f8[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) f8[j] = (float)o[8 * k + j];
            b[k * stride + s] = f_to_h8(f8);
        }
    }
}

// bytes of one 16-byte-vector "row" element count: number of 16B vectors for N reals
template <int P> constexpr int reals_per_vec() { return P == F64 ? 2 : (P == F32 ? 4 : 8); }

// -------------------------------------------------------------------------
// spinor fields
// -------------------------------------------------------------------------
// A spinor field of nf flavours over `stride` slots (sites x right-hand
// sides).  Flavour f occupies vectors [f * 24/w, (f+1) * 24/w).  FP16
// fields keep one float scale per (flavour, slot) in `nrm`.
struct SpinorPtr {
    void *d;
    float *nrm;
    long stride;
};

template <int P> __host__ __device__ constexpr long spinor_vecs() { return 24 / reals_per_vec<P>(); }

// bytes of one internal one-parity spinor field of nf flavours over `stride` slots
__host__ __device__ inline long spinor_field_bytes(int prec, int nf, long stride)
{
    const long vecs = prec == F64 ? 12 : (prec == F32 ? 6 : 3);
    return nf * vecs * stride * 16 + (prec == F16 ? nf * stride * 4 : 0);
}

__host__ __device__ inline SpinorPtr make_spinor(void *d, int prec, int nf, long stride)
{
    SpinorPtr f;
    f.d = d;
    f.stride = stride;
    f.nrm = prec == F16 ? reinterpret_cast<float *>(static_cast<char *>(d) + nf * 3 * stride * 16) : nullptr;
    return f;
}

// parity half of a full-lattice internal field (even field, then odd field)
__host__ __device__ inline SpinorPtr parity_half(SpinorPtr f, int prec, int nf, int parity)
{
    if (parity == 0) return f;
    return make_spinor(static_cast<char *>(f.d) + spinor_field_bytes(prec, nf, f.stride), prec, nf, f.stride);
}

template <int P, typename R>
__device__ __forceinline__ void load_spinor(const SpinorPtr &f, int flav, long s, cx<R> *v)
{
    R tmp[24];
    const char *base = static_cast<const char *>(f.d) + (size_t)flav * spinor_vecs<P>() * f.stride * 16;
    load_seq<P, 24>(base, f.stride, s, tmp);
    if constexpr (P == F16) {
        const float sc = f.nrm[flav * f.stride + s];
#pragma unroll
        for (int k = 0; k < 24; ++k) tmp[k] *= sc;
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = cx<R>{tmp[2 * k], tmp[2 * k + 1]};
}

template <int P, bool NT = false, typename R>
__device__ __forceinline__ void store_spinor(const SpinorPtr &f, int flav, long s, const cx<R> *v)
{
    R tmp[24];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        tmp[2 * k] = v[k].re;
        tmp[2 * k + 1] = v[k].im;
    }
    char *base = static_cast<char *>(f.d) + (size_t)flav * spinor_vecs<P>() * f.stride * 16;
    if constexpr (P == F16) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)tmp[k]));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 24; ++k) tmp[k] = (R)((float)tmp[k] * inv);
        f.nrm[flav * f.stride + s] = m;
    }
    store_seq<P, 24, R, NT>(base, f.stride, s, tmp);
}

// -------------------------------------------------------------------------
// compressed links: rows 0 and 1 of U_mu(x) for x of parity p
// -------------------------------------------------------------------------
// FP64: 6 double2 vectors per (p, mu); FP32: 3 float4; FP16: 3 uint2.
// Index of vector k of (p, mu, s): ((p*4 + mu) * nv + k) * Vh + s.
struct LinkPtr {
    const void *d;
    long Vh;
};

template <int P> __host__ __device__ constexpr int link_vecs() { return P == F64 ? 6 : 3; }
template <int P> __host__ __device__ constexpr int link_vec_bytes() { return P == F16 ? 8 : 16; }

template <int P, typename R>
__device__ __forceinline__ void load_link(const LinkPtr &U, int p, int mu, long s, cx<R> u[9])
{
    R t[12];
    const long base = (long)(p * 4 + mu) * link_vecs<P>() * U.Vh;
    if constexpr (P == F64) {
        const double2 *b = static_cast<const double2 *>(U.d) + base;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double2 v = ldv<true>(b + k * U.Vh + s);
            t[2 * k] = v.x;
            t[2 * k + 1] = v.y;
        }
    } else if constexpr (P == F32) {
        const float4 *b = static_cast<const float4 *>(U.d) + base;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float4 v = ldv<true>(b + k * U.Vh + s);
            t[4 * k] = v.x;
            t[4 * k + 1] = v.y;
            t[4 * k + 2] = v.z;
            t[4 * k + 3] = v.w;
        }
    } else {
        const uint2 *b = static_cast<const uint2 *>(U.d) + base;
#pragma unroll
        for (int k = 0; k < 3; ++k) h4_to_f(ldv<true>(b + k * U.Vh + s), t + 4 * k);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = cx<R>{t[2 * k], t[2 * k + 1]};
    // row 2 = conj(row0 x row1)
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

// -------------------------------------------------------------------------
// clover blocks
// -------------------------------------------------------------------------
// Hermitian 6x6 block per chirality, 36 reals: d0..d5, then the 15 strictly
// lower entries (i > j, row-major order: (1,0),(2,0),(2,1),(3,0),...) as
// (re, im).  A site holds chirality 0 then chirality 1: 72 reals.
// Full 6x6 complex block per chirality (row-major), 72 reals; 144 per site.
template <int P, typename R>
__device__ __forceinline__ void herm_apply(const void *base, long stride, long s, int chir, R twist,
                                           const cx<R> *v, cx<R> *o)
{
    // o = (A_chir + i * twist) v, v and o: 6 complex
    R a[36];
    const int off = chir * 36 / reals_per_vec<P>();
    const char *b = static_cast<const char *>(base) + (size_t)off * stride * 16;
    load_seq<P, 36>(b, stride, s, a);
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = cx<R>{a[i] * v[i].re - twist * v[i].im, a[i] * v[i].im + twist * v[i].re};
    int k = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            cx<R> l{a[k], a[k + 1]};
            k += 2;
            cmac(o[i], l, v[j]);
            cmac_conj(o[j], l, v[i]);
        }
}

// Load the 6 components (2 spins x 3 colours) of chirality block chir of a
// spinor: components 6 chir .. 6 chir + 5.  Used for the diagonal input of a
// stencil, read once per launch: the loads are non-temporal.
template <int P, typename R>
__device__ __forceinline__ void load_chiral(const SpinorPtr &f, int flav, long s, int chir, cx<R> *v)
{
    const char *base = static_cast<const char *>(f.d) + (size_t)flav * spinor_vecs<P>() * f.stride * 16;
    R t[12];
    if constexpr (P == F64) {
        load_seq<P, 12, R, true>(base + (size_t)6 * chir * f.stride * 16, f.stride, s, t);
    } else if constexpr (P == F32) {
        load_seq<P, 12, R, true>(base + (size_t)3 * chir * f.stride * 16, f.stride, s, t);
    } else {
        // halves 12 chir .. 12 chir + 11 live in 16-byte vectors chir and chir + 1
        R w[16];
        load_seq<P, 16, R, true>(base + (size_t)chir * f.stride * 16, f.stride, s, w);
        const float sc = f.nrm[flav * f.stride + s];
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = (chir ? w[k + 4] : w[k]) * sc;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = cx<R>{t[2 * k], t[2 * k + 1]};
}

// o = (A_chir + i twist) v for one chirality block of a Hermitian-packed site
// record (FP16: the 36 halves of a block straddle 16-byte vectors, so five
// vectors are read and the block picked out at offset 4 chir).
template <int P, typename R>
__device__ __forceinline__ void herm_apply_c(const void *base, long stride, long s, int chir, R twist,
                                             const cx<R> *v, cx<R> *o)
{
    R a[36];
    if constexpr (P == F16) {
        R w[40];
        load_seq<P, 40, R, true>(static_cast<const char *>(base) + (size_t)4 * chir * stride * 16, stride, s, w);
#pragma unroll
        for (int k = 0; k < 36; ++k) a[k] = chir ? w[k + 4] : w[k];
    } else {
        const int off = chir * 36 / reals_per_vec<P>();
        load_seq<P, 36, R, true>(static_cast<const char *>(base) + (size_t)off * stride * 16, stride, s, a);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = cx<R>{a[i] * v[i].re - twist * v[i].im, a[i] * v[i].im + twist * v[i].re};
    int k = 6;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            cx<R> l{a[k], a[k + 1]};
            k += 2;
            cmac(o[i], l, v[j]);
            cmac_conj(o[j], l, v[i]);
        }
}

// FP16 herm: 36 reals per chirality is 4.5 vectors; the site record of 72
// reals (9 vectors) is therefore loaded whole for F16.
template <typename R>
__device__ __forceinline__ void herm_apply_both_f16(const void *base, long stride, long s, R tw0, R tw1,
                                                    const cx<R> *v, cx<R> *o)
{
    R a[72];
    load_seq<F16, 72>(base, stride, s, a);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const R *ac = a + 36 * c;
        const cx<R> *vc = v + 6 * c;
        cx<R> *oc = o + 6 * c;
        const R tw = c ? tw1 : tw0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            oc[i] = cx<R>{ac[i] * vc[i].re - tw * vc[i].im, ac[i] * vc[i].im + tw * vc[i].re};
        int k = 6;
#pragma unroll
        for (int i = 1; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) {
                cx<R> l{ac[k], ac[k + 1]};
                k += 2;
                cmac(oc[i], l, vc[j]);
                cmac_conj(oc[j], l, vc[i]);
            }
    }
}

// o = (A_0 + i tw0) v_0 ++ (A_1 + i tw1) v_1 for a 12-component (chirality-ordered) vector
template <int P, typename R>
__device__ __forceinline__ void herm_apply_site(const void *base, long stride, long s, R tw0, R tw1,
                                                const cx<R> *v, cx<R> *o)
{
    if constexpr (P == F16) {
        herm_apply_both_f16(base, stride, s, tw0, tw1, v, o);
    } else {
        herm_apply<P>(base, stride, s, 0, tw0, v, o);
        herm_apply<P>(base, stride, s, 1, tw1, v + 6, o + 6);
    }
}

// o = M v (dag = false) or M^dagger v (dag = true); M full 6x6 for chirality chir
template <int P, typename R>
__device__ __forceinline__ void full_apply(const void *base, long stride, long s, int chir, bool dag,
                                           const cx<R> *v, cx<R> *o)
{
    const int off = chir * 72 / reals_per_vec<P>();
    const char *b = static_cast<const char *>(base) + (size_t)off * stride * 16;
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = cx<R>{0, 0};
    // load row by row (12 reals per row) to bound register use
    if constexpr (P == F16) {
        R a[72];
        load_seq<P, 72, R, true>(b, stride, s, a);
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                cx<R> m{a[12 * i + 2 * j], a[12 * i + 2 * j + 1]};
                if (dag)
                    cmac_conj(o[j], m, v[i]);
                else
                    cmac(o[i], m, v[j]);
            }
    } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            R a[12];
            load_seq<P, 12, R, true>(b + (size_t)(12 * i / reals_per_vec<P>()) * stride * 16, stride, s, a);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                cx<R> m{a[2 * j], a[2 * j + 1]};
                if (dag)
                    cmac_conj(o[j], m, v[i]);
                else
                    cmac(o[i], m, v[j]);
            }
        }
    }
}

}  // namespace tmx
