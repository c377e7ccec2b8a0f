// Learned gauge-covariant preconditioner K (a stand-in for the paper's
// multigrid preconditioner of Section 4.1): forward, adjoint, weight
// gradients, Adam training, and the flexible-GCR solver that uses it.
//
// Network: four linear layers 1 -> 8 -> 8 -> 8 -> 1 channels on the full
// lattice, each
//     y_c(x) = sum_{d=0..8} sum_c' C_d[c,c'] (Gamma_d (x) 1) (T_d x_c')(x)
// with the parallel transports T_0 = 1, T_{+mu} psi(x) = U_mu(x) psi(x+mu),
// T_{-mu} psi(x) = U_mu(x-mu)^+ psi(x-mu) (time-boundary factor on hops
// across the edge).  The input is the odd source embedded in the full
// lattice, the output is restricted to the odd sites.
//
// One layer is a GEMM per workgroup tile of 64 sites:
//     Y[m][n] = sum_d W_d[m][k] Z_d[k][n]
// m = (out channel, spin, re/im), k = (in channel, spin, re/im),
// n = (site, colour); W_d = C_d (x) Gamma_d written as a real matrix, Z_d the
// transported input.  Activations and links are BF16; the transports run on
// the matrix cores as 4x4x4 blocks (v_mfma_f32_4x4x4_16b_bf16), the
// contraction on v_mfma_f32_16x16x32_bf16, both with FP32 accumulation.  The
// adjoint layer is the same kernel with W'_d = W_{-d}^H (transport and
// weights commute).  The layers with one input or one output channel run in
// factorised form on the vector ALUs (further below).
//
// The input is supported on odd sites and only the odd sites of the output
// are kept, so the first layer skips zero inputs and the last layer computes
// odd sites only, writing an FP32 odd field.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "tmx_ctx.h"

namespace tmx {

constexpr int NN_L = 4;
constexpr int NN_P = 9;
static const int NN_CIN[NN_L] = {1, 8, 8, 8};
static const int NN_COUT[NN_L] = {8, 8, 8, 1};
constexpr int NN_S = 64;          // sites per workgroup tile
constexpr int NN_N = 3 * NN_S;    // GEMM columns per tile
constexpr int NN_PAD = 8;         // LDS row padding (bf16 elements)

__host__ __device__ constexpr int pad16(int x) { return (x + 15) / 16 * 16; }

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (gfx950 converts pairs in one
// v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float a, float b)
{
    const bf16x2v r = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, r);
}

static size_t layer_param_offset(int l)
{
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)NN_P * (NN_CIN[i] * NN_COUT[i] + 16) * 2;
    return o;
}
static size_t nn_num_params() { return layer_param_offset(NN_L); }

struct PcState {
    size_t nparam = 0;
    float *params = nullptr;  // device FP32 master weights
    float *grad = nullptr;
    float *adam_m = nullptr, *adam_v = nullptr;
    uint16_t *Wf[NN_L] = {};  // forward real weights [9][MD][KD], bf16
    uint16_t *Wa[NN_L] = {};  // adjoint real weights
    bool w_ok = false;
    bool have_weights = false;
    int adam_t = 0;
    uint32_t *lrow = nullptr, *lcol = nullptr;  // BF16 network links (see NnLinks)
    int links_upload = -1;  // gauge upload the links were made from
    struct ThinW *thin = nullptr;  // factorised weights of the one-channel layers (see ThinW)
};

// ---------------------------------------------------------------------------
// weights: complex (C, Gamma) -> real-ified W_d (forward and adjoint)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rev_path(int d) { return d == 0 ? 0 : ((d - 1) % 2 == 0 ? d + 1 : d - 1); }

// thread per (d, m, k) of a [9][MD][KD] matrix
__global__ void nn_build_w_kernel(const float *p, uint16_t *W, int cin, int cout, int adjoint)
{
    // forward: rows over (cout, spin, ri), cols over (cin, spin, ri)
    // adjoint: rows over (cin, ...), cols over (cout, ...), W'_d = W_{rev d}^H
    const int rows = adjoint ? cin : cout, cols = adjoint ? cout : cin;
    const int MD = pad16(8 * rows), KD = pad16(8 * cols);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN_P * MD * KD) return;
    const int d = t / (MD * KD), m = (t / KD) % MD, k = t % KD;
    float v = 0.f;
    if (m < 8 * rows && k < 8 * cols) {
        const int a = m / 8, s = (m % 8) / 2, ri = m % 2;
        const int b = k / 8, sp = (k % 8) / 2, rj = k % 2;
        const int dd = adjoint ? rev_path(d) : d;
        const size_t per = (size_t)cin * cout + 16;
        const float *pd = p + (size_t)dd * per * 2;
        // C[cout][cin], Gamma[4][4]
        float cr, ci, gr, gi;
        if (!adjoint) {
            cr = pd[2 * (a * cin + b)];
            ci = pd[2 * (a * cin + b) + 1];
            gr = pd[2 * (cin * cout + s * 4 + sp)];
            gi = pd[2 * (cin * cout + s * 4 + sp) + 1];
        } else {
            // (C (x) Gamma)^H [(a,s),(b,sp)] = conj(C[b][a]) conj(Gamma[sp][s]), a < cin, b < cout
            cr = pd[2 * (b * cin + a)];
            ci = -pd[2 * (b * cin + a) + 1];
            gr = pd[2 * (cin * cout + sp * 4 + s)];
            gi = -pd[2 * (cin * cout + sp * 4 + s) + 1];
        }
        const float wr = cr * gr - ci * gi, wi = cr * gi + ci * gr;
        v = (ri == 0) ? (rj == 0 ? wr : -wi) : (rj == 0 ? wi : wr);
    }
    W[t] = f2bf(v);
}

// ---------------------------------------------------------------------------
// BF16 operands: activations, links, transports
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Activation field (BF16, full lattice): channel c at site gs (= parity * V/2
// + checkerboard index) is 12 words at d[(c * stride + gs) * 12], spin s
// in words 3 s .. 3 s + 2 (colours 0..2 as (re, im) BF16 pairs).  Lane q of
// a site reads the three words of spin q: the four lanes of a site read 48
// contiguous bytes and consecutive sites follow each other.
struct Act {
    uint32_t *d;
    long stride;
};

struct W3 {
    uint32_t x, y, z;
};
__device__ __forceinline__ W3 ld3(const uint32_t *p)
{
    W3 r;
    r.x = p[0];
    r.y = p[1];
    r.z = p[2];
    return r;
}

// BF16 links of the network: U_mu(x), x of parity p and checkerboard index s,
// as nine (re, im) pairs at row[((p*4 + mu) * Vh + s) * 9 + 3 r + k] = U[r][k]
// and, transposed, col[... + 3 r + k] = U[k][r].
struct NnLinks {
    const uint32_t *row, *col;
    long Vh;
};

// thread per (p, mu, s): from the FP64 two-row master copy (6 complex per link)
__global__ void nn_links_kernel(const double2 *l64, uint32_t *row, uint32_t *col, long Vh)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * Vh) return;
    const long pm = i / Vh, s = i - pm * Vh;
    cx<double> u[9];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 v = l64[(pm * 6 + k) * Vh + s];
        u[k] = cx<double>{v.x, v.y};
    }
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            row[i * 9 + 3 * r + k] = f2bf2((float)u[3 * r + k].re, (float)u[3 * r + k].im);
            col[i * 9 + 3 * r + k] = f2bf2((float)u[3 * k + r].re, (float)u[3 * k + r].im);
        }
}

// neighbour along path d of the site (coordinates x, parity p, index cb)
struct Nbr {
    long idx;   // neighbour site in the activation layout
    int lp;     // link parity
    long lcb;   // link checkerboard index
    float bc;   // boundary factor
    bool dag;   // U^dagger (backward path)
    bool ident; // d = 0
};

__device__ __forceinline__ Nbr path_neighbour_at(const Geom &g, const int x[4], int p, int cb, int d, int t_bc)
{
    Nbr r;
    const long Vh = g.Vh;
    r.bc = 1.f;
    if (d == 0) {
        r.idx = (long)p * Vh + cb;
        r.ident = true;
        r.dag = false;
        r.lp = 0;
        r.lcb = 0;
        return r;
    }
    r.ident = false;
    const int mu = (d - 1) / 2;
    const bool back = ((d - 1) % 2) == 1;
    int y[4] = {x[0], x[1], x[2], x[3]};
    if (!back) {
        if (++y[mu] == g.L[mu]) {
            y[mu] = 0;
            if (mu == 3) r.bc = (float)t_bc;
        }
    } else {
        if (--y[mu] < 0) {
            y[mu] = g.L[mu] - 1;
            if (mu == 3) r.bc = (float)t_bc;
        }
    }
    const int ncb = cb_index(g, y);
    r.idx = (long)(1 - p) * Vh + ncb;
    r.dag = back;
    r.lp = back ? 1 - p : p;
    r.lcb = back ? ncb : cb;
    return r;
}

// site of a staging thread: coordinates decoded once per tile
struct SiteCtx {
    int xs[4], p, cb;
    bool valid;
};

__device__ __forceinline__ void site_ctx(const Geom &g, long gs, long s_end, SiteCtx &sc)
{
    sc.valid = gs < s_end;
    if (!sc.valid) return;
    sc.p = gs >= g.Vh ? 1 : 0;
    sc.cb = (int)(gs - (long)sc.p * g.Vh);
    cb_coords(g, sc.cb, sc.p, sc.xs);
}

// Transport on the matrix cores.  The four lanes of a site (q = lane % 4) are
// one block of v_mfma_f32_4x4x4_16b_bf16 (A[i][k] in lane 4b + i, B[k][j] in
// lane 4b + j, D[i][j] in lane 4b + j, register i).  With the input channel
// as Psi[colour k][spin i] and W = U or U^dagger,
//     D = Psi^T W^T,   D[i][j] = (W Psi)[colour j][spin i],
// so lane q supplies spin q of the input (A row q: colours 0..2, zero) and
// row q of W (B column q), and receives colour q of the result, all four
// spins: exactly one staging row of the contraction.  Complex products take
// four real steps: D_re = A_re B_re - A_im B_im, D_im = A_re B_im + A_im B_re.
struct Wop {
    bf16x4 re, im, nim;  // B column of this lane: re, im and -im of W[q][k]
};

// (re, im) pairs of three complex numbers -> BF16 vectors of the real and
// imaginary parts, fourth entry zero
__device__ __forceinline__ void split3(uint32_t d0, uint32_t d1, uint32_t d2, bf16x4 &re, bf16x4 &im)
{
    re = __builtin_bit_cast(bf16x4, make_uint2(__builtin_amdgcn_perm(d1, d0, 0x05040100u), d2 & 0xffffu));
    im = __builtin_bit_cast(bf16x4, make_uint2(__builtin_amdgcn_perm(d1, d0, 0x07060302u), d2 >> 16));
}

// W operand of lane q for path data: ident -> unit matrix; otherwise row q of
// U (forward) or the conjugate of column q of U (backward), times bc
__device__ __forceinline__ Wop make_wop(bool ident, bool dag, float bc, W3 w, int q)
{
    Wop o;
    if (ident) {
        const uint32_t one = 0x3f80u;  // BF16 1.0
        const uint2 v = make_uint2(q == 0 ? one : (q == 1 ? one << 16 : 0u), q == 2 ? one : 0u);
        o.re = __builtin_bit_cast(bf16x4, v);
        o.im = o.nim = __builtin_bit_cast(bf16x4, make_uint2(0u, 0u));
        return o;
    }
    split3(w.x, w.y, w.z, o.re, o.im);
    const uint32_t neg = 0x80008000u;
    uint2 r = __builtin_bit_cast(uint2, o.re), i = __builtin_bit_cast(uint2, o.im);
    if (dag) i = make_uint2(i.x ^ neg, i.y ^ (neg & 0xffffu));
    if (bc < 0.f) {
        r = make_uint2(r.x ^ neg, r.y ^ (neg & 0xffffu));
        i = make_uint2(i.x ^ neg, i.y ^ (neg & 0xffffu));
    }
    o.re = __builtin_bit_cast(bf16x4, r);
    o.im = __builtin_bit_cast(bf16x4, i);
    o.nim = __builtin_bit_cast(bf16x4, make_uint2(i.x ^ neg, i.y ^ (neg & 0xffffu)));
    return o;
}

// one channel: spin q of the input (colours in x, y, z) -> colour q of the
// transported field, spins 0..3, as BF16 (re, im) pairs
__device__ __forceinline__ void transport4(const Wop &w, W3 psi, uint32_t out[4])
{
    bf16x4 are, aim;
    split3(psi.x, psi.y, psi.z, are, aim);
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 dre = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(are, w.re, z, 0, 0, 0);
    dre = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(aim, w.nim, dre, 0, 0, 0);
    f32x4 dim = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(are, w.im, z, 0, 0, 0);
    dim = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(aim, w.re, dim, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = f2bf2(dre[i], dim[i]);
}

// register staging of one path for lane q of a site: spin q of all CIN
// input channels, and this lane's row / column of the link
template <int CIN> struct Stg {
    W3 psi[CIN];
    W3 w;
    float bc;
    bool ident, dag;
};

// in_odd: the input field is zero on even sites (and never read there)
template <int CIN>
__device__ __forceinline__ void stg_load(const Geom &g, const Act &x, const NnLinks &L, int t_bc, int d, bool in_odd,
                                         const SiteCtx &sc, int q, Stg<CIN> &st)
{
    // zero operands where the input vanishes: the transport still runs on
    // every lane (matrix-core steps are never placed under a divergent branch)
    bool zero = !sc.valid;
    Nbr nb{};
    if (!zero) {
        nb = path_neighbour_at(g, sc.xs, sc.p, sc.cb, d, t_bc);
        const int np = d == 0 ? sc.p : 1 - sc.p;
        zero = in_odd && np == 0;
    }
    const W3 z0 = {0u, 0u, 0u};
    st.ident = !zero && nb.ident;
    st.dag = !zero && nb.dag;
    st.bc = zero ? 1.f : nb.bc;
    st.w = z0;
    if (!zero && !nb.ident && q < 3) {
        const int mu = (d - 1) / 2;
        const long li = ((long)(nb.lp * 4 + mu) * L.Vh + nb.lcb) * 9 + 3 * q;
        st.w = ld3((nb.dag ? L.col : L.row) + li);
    }
#pragma unroll
    for (int c = 0; c < CIN; ++c) st.psi[c] = zero ? z0 : ld3(x.d + ((long)c * x.stride + nb.idx) * 12 + 3 * q);
}

// ---------------------------------------------------------------------------
// layer kernel: Y = sum_d W_d Z_d   (forward or adjoint, by the weights given)
// ---------------------------------------------------------------------------
// Tile of 64 sites (192 GEMM columns), 256 threads.  Staging: four lanes per
// site, lane q loading spin q of every input channel at the neighbour and
// transporting it on the matrix cores (above); lanes q < 3 write the BF16
// rows Z_d[n = (site, colour q)][k = (channel, spin, re/im)] to LDS.
// Contraction: wave w owns the 16-row block m = 16 w .. 16 w + 15 of the
// output (all twelve column blocks) on v_mfma_f32_16x16x32_bf16 (16x16x16
// for a one-channel input).  The paths are unrolled; the weights of path
// i + 2 and the neighbours and links of path i + 2 (i + 1 in the 8 -> 8
// layer) are requested while path i is contracted, so memory latency
// overlaps the steps in between.  One input channel means an input supported on odd
// sites (the embedded source): tiles then hold one parity, and odd tiles
// run the d = 0 path only, even tiles the eight hops only.  One output
// channel means the last layer: only odd sites are computed and the result
// is written in FP32 as an odd spinor field.
constexpr int NL_S = 64;
constexpr int NL_N = 3 * NL_S;

template <int CIN, int COUT>
__global__ void __launch_bounds__(256) nn_layer_kernel(Geom g, Act x, Act y, SpinorPtr yo, NnLinks L,
                                                       const uint16_t *W, int t_bc, long s_begin, long s_end, int xcd)
{
    constexpr int KD = pad16(8 * CIN), MD = pad16(8 * COUT);
    constexpr int KS = KD + NN_PAD;
    constexpr int MT = MD / 16, NT = NL_N / 16;
    constexpr bool K32 = KD % 32 == 0;
    constexpr int KK = K32 ? KD / 32 : KD / 16;
    constexpr int PER = MT >= 4 ? NT : (NT + 3) / 4;
    constexpr bool IN_ODD = CIN == 1;
    constexpr bool ILV = IN_ODD || (CIN == 8 && COUT == 8);  // parity-interleaved tiles
    static_assert(MT == 4 || MT == 1, "output rows: 8 or 1 channels");
    // LDS: the staging rows, then (after the last path) the output tile
    constexpr int ZS_BYTES = NL_N * KS * 2;
    constexpr int YS_BYTES = COUT == 1 ? NL_S * 24 * 4 : NL_S * COUT * 48;
    __shared__ __attribute__((aligned(16))) unsigned char smem[ZS_BYTES > YS_BYTES ? ZS_BYTES : YS_BYTES];
    uint16_t(*Zs)[KS] = reinterpret_cast<uint16_t(*)[KS]>(smem);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int my_mt = MT >= 4 ? wave : 0;
    // tile -> sites.  When both parities are computed, tiles alternate
    // between them (tile 2i + p: sites p V/2 + 64 i ...): every tile has one
    // parity, and the contiguous tile range of an XCD covers both parities of
    // one region, so the hop neighbours of its sites are its own sites (read
    // through its own L2).  With an odd-supported input this also gives every
    // XCD as many 8-path (even) tiles as 1-path (odd) ones.
    const long tile = xcd_block(xcd);
    long site0;
    if (ILV) {
        const long par = tile & 1;
        site0 = par * g.Vh + (tile >> 1) * NL_S;
        s_end = (par + 1) * (long)g.Vh;
    } else {
        site0 = s_begin + tile * NL_S;
    }
    const int sl = threadIdx.x / 4, q = threadIdx.x % 4;

    if (8 * CIN < KD) {
        for (int i = threadIdx.x; i < NL_N; i += blockDim.x)
            for (int k = 8 * CIN; k < KD; ++k) Zs[i][k] = 0;
    }
    SiteCtx sc;
    site_ctx(g, site0 + sl, s_end, sc);
    f32x4 acc[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    using WFrag = typename std::conditional<K32, bf16x8, bf16x4>::type;
    // weight fragments of path d for this wave's output rows
    auto load_w = [&](int d, WFrag (&wa)[KK]) {
        const uint16_t *Wd = W + ((size_t)d * MD + my_mt * 16 + lane % 16) * KD;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
            wa[kk] = K32 ? *reinterpret_cast<const WFrag *>(Wd + kk * 32 + 8 * (lane / 16))
                         : *reinterpret_cast<const WFrag *>(Wd + kk * 16 + 4 * (lane / 16));
    };
    // Neighbour slots: the 8 -> 8 layer keeps one path ahead (two would
    // halve its occupancy), the others two.
    constexpr int NSLOT = (CIN == 8 && COUT == 8) ? 1 : 2;
    // paths D0 .. D0 + NP - 1
    auto run = [&](auto d0c, auto npc) {
        constexpr int D0 = decltype(d0c)::value, NP = decltype(npc)::value;
        Stg<CIN> st[NSLOT];
        WFrag wa[2][KK];
        stg_load<CIN>(g, x, L, t_bc, D0, IN_ODD, sc, q, st[0]);
        load_w(D0, wa[0]);
        if constexpr (NP > 1) {
            if constexpr (NSLOT > 1) stg_load<CIN>(g, x, L, t_bc, D0 + 1, IN_ODD, sc, q, st[1]);
            load_w(D0 + 1, wa[1]);
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int b = i & 1, sb = i % NSLOT;
            {
                const Wop w = make_wop(st[sb].ident, st[sb].dag, st[sb].bc, st[sb].w, q);
#pragma unroll
                for (int c = 0; c < CIN; ++c) {
                    uint32_t z[4];
                    transport4(w, st[sb].psi[c], z);
                    if (q < 3)
                        *reinterpret_cast<uint4 *>(&Zs[sl * 3 + q][c * 8]) = make_uint4(z[0], z[1], z[2], z[3]);
                }
            }
            __syncthreads();
            if (i + NSLOT < NP) stg_load<CIN>(g, x, L, t_bc, D0 + i + NSLOT, IN_ODD, sc, q, st[sb]);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int nt = MT >= 4 ? j : wave + 4 * j;
                if (nt >= NT) break;
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    if constexpr (K32) {
                        const bf16x8 bz =
                            *reinterpret_cast<const bf16x8 *>(&Zs[nt * 16 + lane % 16][kk * 32 + 8 * (lane / 16)]);
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[b][kk], bz, acc[j], 0, 0, 0);
                    } else {
                        const bf16x4 bz =
                            *reinterpret_cast<const bf16x4 *>(&Zs[nt * 16 + lane % 16][kk * 16 + 4 * (lane / 16)]);
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[b][kk], bz, acc[j], 0, 0, 0);
                    }
                }
            }
            if (i + 2 < NP) load_w(D0 + i + 2, wa[b]);
            __syncthreads();
        }
    };
    if constexpr (IN_ODD) {
        // odd tiles: their own (odd) input; even tiles: the odd neighbours
        if (site0 >= g.Vh)
            run(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
        else
            run(std::integral_constant<int, 1>{}, std::integral_constant<int, NN_P - 1>{});
    } else {
        run(std::integral_constant<int, 0>{}, std::integral_constant<int, NN_P>{});
    }

    // D[m][n]: lane holds rows m = 16 mt + 4 (lane/16) + i of column n = 16 nt + lane%16.
    // The tile goes through LDS so that every global store is a whole
    // 16-byte vector and a wave's stores are contiguous.
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int nt = MT >= 4 ? j : wave + 4 * j;
        if (nt >= NT) break;
        const int m0 = my_mt * 16 + 4 * (lane / 16);
        const int n = nt * 16 + lane % 16;
        const int sn = n / 3, col = n % 3;
        if (m0 >= 8 * COUT) continue;
        const int c = m0 / 8, sp = (m0 % 8) / 2;  // channel, first of two spins
        if constexpr (COUT == 1) {
            // [site][k = spin * 3 + colour][re, im] in FP32
            float *Yf = reinterpret_cast<float *>(smem);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = (sp + h) * 3 + col;
                *reinterpret_cast<float2 *>(&Yf[(sn * 12 + k) * 2]) = make_float2(acc[j][2 * h], acc[j][2 * h + 1]);
            }
        } else {
            // [channel][site][12 words], as in the activation layout
            uint32_t *Ys = reinterpret_cast<uint32_t *>(smem);
#pragma unroll
            for (int h = 0; h < 2; ++h)
                Ys[(c * NL_S + sn) * 12 + (sp + h) * 3 + col] = f2bf2(acc[j][2 * h], acc[j][2 * h + 1]);
        }
    }
    __syncthreads();
    if constexpr (COUT == 1) {
        // FP32 odd spinor: vector kv of site cb holds components 2 kv and 2 kv + 1
        const float *Yf = reinterpret_cast<const float *>(smem);
        for (int v = threadIdx.x; v < 6 * NL_S; v += blockDim.x) {
            const int kv = v / NL_S, sn = v % NL_S;
            const long gs = site0 + sn;
            if (gs >= s_end) continue;
            reinterpret_cast<float4 *>(yo.d)[(long)kv * yo.stride + (gs - g.Vh)] =
                *reinterpret_cast<const float4 *>(&Yf[(sn * 12 + 2 * kv) * 2]);
        }
    } else {
        // per channel, the tile's 64 sites are 192 contiguous 16-byte vectors
        const uint4 *Yv = reinterpret_cast<const uint4 *>(smem);
        for (int v = threadIdx.x; v < COUT * NL_S * 3; v += blockDim.x) {
            const int c = v / (NL_S * 3), o = v % (NL_S * 3);
            const long gs = site0 + o / 3;
            if (gs >= s_end) continue;
            reinterpret_cast<uint4 *>(y.d + ((long)c * y.stride + site0) * 12)[o] = Yv[v];
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: P_d[m][k] += sum_n Dl[m][n] Z_d[k][n]   (grid.y = path)
// ---------------------------------------------------------------------------
// Tiles of 64 sites; the transported input (staged as in the layer kernel)
// and the output adjoint are written to LDS with n innermost, the
// contraction over n runs on v_mfma_f32_16x16x32_bf16.  Sites where one of
// the two factors vanishes identically (odd-supported input, odd-only output
// adjoint) are skipped as whole ranges.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) nn_wgrad_kernel(Geom g, Act x, Act dy, NnLinks L, int t_bc, float *partial)
{
    constexpr int KD = pad16(8 * CIN), MD = pad16(8 * COUT);
    constexpr int NSTR = NN_N + NN_PAD;
    constexpr int MT = MD / 16, KT = KD / 16, NTILE = MT * KT;
    constexpr int PER_WAVE = (NTILE + 3) / 4;
    static_assert(NN_S == NL_S, "one tile size");
    __shared__ __attribute__((aligned(16))) uint16_t Dl[MD][NSTR];
    __shared__ __attribute__((aligned(16))) uint16_t Zt[KD][NSTR];
    const long V = 2L * g.Vh;
    const int d = blockIdx.y;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int sl = threadIdx.x / 4, q = threadIdx.x % 4;
    long sb = 0, se = V;
    if (COUT == 1) sb = g.Vh;  // the output adjoint lives on odd sites
    if (CIN == 1) {            // odd-supported input: d = 0 feeds odd sites, hops even ones
        if (d == 0)
            sb = g.Vh;
        else
            se = g.Vh;
    }
    const long ntiles = (se - sb + NN_S - 1) / NN_S;
    for (int i = threadIdx.x; i < MD * NSTR; i += blockDim.x) Dl[i / NSTR][i % NSTR] = 0;
    for (int i = threadIdx.x; i < KD * NSTR; i += blockDim.x) Zt[i / NSTR][i % NSTR] = 0;
    f32x4 acc[PER_WAVE];
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long site0 = sb + tile * NN_S;
        __syncthreads();
        SiteCtx sc;
        site_ctx(g, site0 + sl, se, sc);
        Stg<CIN> st;
        stg_load<CIN>(g, x, L, t_bc, d, CIN == 1, sc, q, st);
        // output adjoint at the site itself: lane q holds spin q of every channel
        {
            const long gs = site0 + sl;
#pragma unroll
            for (int c = 0; c < COUT; ++c) {
                W3 v = {0u, 0u, 0u};
                if (sc.valid) v = ld3(dy.d + ((long)c * dy.stride + gs) * 12 + 3 * q);
                const uint32_t w[3] = {v.x, v.y, v.z};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Dl[c * 8 + 2 * q][sl * 3 + a] = (uint16_t)(w[a] & 0xffffu);
                    Dl[c * 8 + 2 * q + 1][sl * 3 + a] = (uint16_t)(w[a] >> 16);
                }
            }
        }
        {
            const Wop w = make_wop(st.ident, st.dag, st.bc, st.w, q);
#pragma unroll
            for (int c = 0; c < CIN; ++c) {
                uint32_t z[4];
                transport4(w, st.psi[c], z);
                if (q < 3) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        Zt[c * 8 + 2 * s][sl * 3 + q] = (uint16_t)(z[s] & 0xffffu);
                        Zt[c * 8 + 2 * s + 1][sl * 3 + q] = (uint16_t)(z[s] >> 16);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            const int t = wave + 4 * j;
            if (t >= NTILE) break;
            const int mt = t / KT, kt = t % KT;
#pragma unroll
            for (int nk = 0; nk < NN_N / 32; ++nk) {
                const int nb = nk * 32 + 8 * (lane / 16);
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&Dl[mt * 16 + lane % 16][nb]);
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Zt[kt * 16 + lane % 16][nb]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
            }
        }
    }
    float *out = partial + ((size_t)blockIdx.x * NN_P + d) * MD * KD;
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) {
        const int t = wave + 4 * j;
        if (t >= NTILE) break;
        const int mt = t / KT, kt = t % KT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = mt * 16 + 4 * (lane / 16) + i, k = kt * 16 + lane % 16;
            out[m * KD + k] += acc[j][i];
        }
    }
}

// odd source r (precision P) -> one-channel BF16 activation (odd half only)
template <int P> __global__ void nn_embed_kernel(SpinorPtr r, Act a, long Vh)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Vh) return;
    cx<float> v[12];
    load_spinor<P>(r, 0, s, v);
    uint32_t w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = f2bf2(v[k].re, v[k].im);  // spin-major: word 3 s + colour
    uint4 *dst = reinterpret_cast<uint4 *>(a.d + (Vh + s) * 12);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    dst[2] = make_uint4(w[8], w[9], w[10], w[11]);
}

// ---------------------------------------------------------------------------
// the one-channel layers on the vector ALUs
// ---------------------------------------------------------------------------
// A layer with one input or one output channel has, per path, a channel
// vector C_d (8 entries) and the spin matrix Gamma_d, so it is applied in its
// factorised form: 1 -> 8 transports the source, mixes the spins and
// spreads the result over the channels; 8 -> 1 contracts the channels first,
// then mixes the spins and transports (C_d, Gamma_d and T_d commute).  Four
// lanes per site, lane q owning output spin q; a site's four spins are
// exchanged among its lanes (DPP within a quad).  The input of the first
// layer is read straight from the odd source field.
//
// Every complex product runs as two BF16 dot products with FP32 accumulation
// (v_dot2_f32_bf16): for a complex w and z given as the pair (z.re, z.im),
//     Re(w z) = (w.re, -w.im) . z,   Im(w z) = (w.im, w.re) . z,
// so the weights are stored in those two packed forms and an operand is
// rounded to a BF16 pair once, where it is produced (the activations and
// links are BF16 already).  Half the instructions of FP32 multiply-adds and
// no BF16 -> FP32 conversions of links or activations.
struct ThinW {
    uint32_t C[NN_P][8][2];     // channel vector of path d, packed (re, -im), (im, re)
    uint32_t G[NN_P][4][4][2];  // spin matrix of path d, packed likewise
};
// the ThinW sets: forward first layer (1 -> 8), forward last layer (8 -> 1),
// the adjoints of the last (1 -> 8) and of the first (8 -> 1), and the two
// halves of the short Hermitian form P_1 = L_1^dagger L_1 (see nn_p1_down_kernel)
enum { THIN_UP_F = 0, THIN_DOWN_F = 1, THIN_UP_A = 2, THIN_DOWN_A = 3, THIN_P1_UP = 4, THIN_P1_DOWN = 5, THIN_SETS = 6 };

// one thread per path: the channel vector and spin matrix of path d of a
// layer with cin * cout = 8 (forward), or of its adjoint W'_d = W_{rev d}^H
__global__ void nn_build_thin_kernel(const float *p, ThinW *w, int cin, int cout, int adjoint)
{
    const int d = threadIdx.x;
    if (d >= NN_P) return;
    const int dd = adjoint ? rev_path(d) : d;
    const int per = cin * cout + 16;
    const float *pd = p + (size_t)dd * per * 2;
    const float sg = adjoint ? -1.f : 1.f;
    for (int c = 0; c < 8; ++c) {
        const float re = pd[2 * c], im = sg * pd[2 * c + 1];
        w->C[d][c][0] = f2bf2(re, -im);
        w->C[d][c][1] = f2bf2(im, re);
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const int e = adjoint ? b * 4 + a : a * 4 + b;
            const float re = pd[2 * (cin * cout + e)], im = sg * pd[2 * (cin * cout + e) + 1];
            w->G[d][a][b][0] = f2bf2(re, -im);
            w->G[d][a][b][1] = f2bf2(im, re);
        }
}

// The short Hermitian form P_1 = L_1^dagger L_1 without its 8-channel
// intermediate.  With h_d = Gamma_d T_d b (layer 1's path d before the
// channel spread) and L_1^dagger's path d' = (C'_d' (x) Gamma'_d') T_d',
// C'_d' = conj(C_{rev d'}), Gamma'_d' = Gamma_{rev d'}^H, the channel
// contraction of L_1^dagger meets the channel spread of L_1 in
//     M[d'][d] = sum_c C'_d'[c] C_d[c],
//     P_1 b(s) = sum_d' Gamma'_d' T_d' z_d'(s + d'),  z_d'(e) = sum_d M[d'][d] h_d(e).
// b lives on odd sites, so z_0 is needed at odd sites only, where it is
// M[0][0] Gamma_0 b, and z_1 .. z_8 at even sites only, where d = 0
// contributes nothing.  THIN_P1_UP holds C[d][c] = M[c + 1][d] (d, c + 1 >= 1)
// and Gamma_d: the 1 -> 8 kernel on even sites then writes z_1 .. z_8 as its
// eight channels.  THIN_P1_DOWN holds Gamma'_d' for d' >= 1 and, in place of
// Gamma'_0, the site term G00 = M[0][0] Gamma'_0 Gamma_0.  One thread per
// (d', d); p = the first layer's parameters.
__global__ void nn_build_p1_kernel(const float *p, ThinW *w)
{
    const int t = threadIdx.x;
    if (t >= NN_P * NN_P) return;
    const int dp = t / NN_P, d = t % NN_P;
    const int per = 8 + 16;  // one input channel, eight output channels
    auto chan = [&](int path, int c) { return cx<float>{p[(size_t)path * per * 2 + 2 * c], p[(size_t)path * per * 2 + 2 * c + 1]}; };
    auto gam = [&](int path, int a, int b) {
        const float *g = p + (size_t)path * per * 2 + 2 * (8 + 4 * a + b);
        return cx<float>{g[0], g[1]};
    };
    auto pack = [](cx<float> v, uint32_t *o) {
        o[0] = f2bf2(v.re, -v.im);
        o[1] = f2bf2(v.im, v.re);
    };
    const int rdp = rev_path(dp);
    cx<float> m{0.f, 0.f};
    for (int c = 0; c < 8; ++c) {
        const cx<float> a = chan(rdp, c);
        cmac(m, cx<float>{a.re, -a.im}, chan(d, c));
    }
    if (dp >= 1 && d >= 1) pack(m, w[THIN_P1_UP].C[d][dp - 1]);
    if (dp == 0) {
        // Gamma_d for the first half, Gamma'_d = Gamma_{rev d}^H for the second
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                pack(gam(d, a, b), w[THIN_P1_UP].G[d][a][b]);
                if (d >= 1) {
                    const cx<float> g = gam(rev_path(d), b, a);
                    pack(cx<float>{g.re, -g.im}, w[THIN_P1_DOWN].G[d][a][b]);
                }
            }
    }
    if (dp == 0 && d == 0) {
        // G00 = M[0][0] Gamma'_0 Gamma_0, Gamma'_0 = Gamma_0^H
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cx<float> v{0.f, 0.f};
                for (int k = 0; k < 4; ++k) {
                    const cx<float> ga = gam(0, k, a);
                    cmac(v, cx<float>{ga.re, -ga.im}, gam(0, k, b));
                }
                pack(m * v, w[THIN_P1_DOWN].G[0][a][b]);
            }
    }
    if (dp >= 1 && d == 0) {
        // unused channel weights of the first half's d = 0 path (odd tiles are not launched)
        w[THIN_P1_UP].C[0][dp - 1][0] = w[THIN_P1_UP].C[0][dp - 1][1] = 0u;
    }
}

// c + a.lo b.lo + a.hi b.hi over BF16 pairs, FP32 accumulation
__device__ __forceinline__ float dot2bf(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, a), __builtin_bit_cast(bf16x2v, b), c, false);
}

// acc += w z, w a complex weight in its two packed forms, z a BF16 (re, im) pair
__device__ __forceinline__ void cmac_bf(cx<float> &acc, uint32_t w0, uint32_t w1, uint32_t z)
{
    acc.re = dot2bf(w0, z, acc.re);
    acc.im = dot2bf(w1, z, acc.im);
}

// t = bc U v (forward path) or bc U^dagger v (backward path) for the three
// colours of one spin, U the BF16 row-major network link.  With u = U[r][k]
// as the pair (u.re, u.im):
//   (U v)_a = sum_b U[a][b] v_b:           Re = u . (v.re, -v.im), Im = u . (v.im, v.re)
//   (U^dagger v)_a = sum_b conj(U[b][a]) v_b: Re = u . (v.re, v.im),  Im = u . (v.im, -v.re)
__device__ __forceinline__ void transport_bf(const NnLinks &L, const Nbr &nb, int d, const cx<float> v[3],
                                             cx<float> t[3])
{
    const int mu = (d - 1) / 2;
    const bool back = ((d - 1) % 2) == 1;
    const uint32_t *lr = L.row + ((long)(nb.lp * 4 + mu) * L.Vh + nb.lcb) * 9;
    uint32_t u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = lr[e];
    uint32_t vr[3], vi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vr[k] = back ? f2bf2(v[k].re, v[k].im) : f2bf2(v[k].re, -v[k].im);
        vi[k] = back ? f2bf2(v[k].im, -v[k].re) : f2bf2(v[k].im, v[k].re);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t ue = u[back ? 3 * k + a : 3 * a + k];
            re = dot2bf(ue, vr[k], re);
            im = dot2bf(ue, vi[k], im);
        }
        t[a] = cx<float>{nb.bc * re, nb.bc * im};
    }
}

// value of lane q ^ M of this lane's quad (all four lanes active)
template <int M> __device__ __forceinline__ uint32_t quad_xor(uint32_t v)
{
    constexpr int ctrl = M == 1 ? 0xB1 : (M == 2 ? 0x4E : 0x1B);  // quad_perm [1,0,3,2] / [2,3,0,1] / [3,2,1,0]
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}

// h = sum_m Gamma_d[q][q ^ m] z(spin q ^ m): z holds spin q of this lane as
// BF16 pairs, spin q ^ m is held by lane q ^ m of the quad
__device__ __forceinline__ void spin_mix(const ThinW *W, int d, int q, const uint32_t z[3], cx<float> h[3])
{
    uint32_t g0[4], g1[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        g0[m] = W->G[d][q][q ^ m][0];
        g1[m] = W->G[d][q][q ^ m][1];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h[a] = cx<float>{0.f, 0.f};
        cmac_bf(h[a], g0[0], g1[0], z[a]);
        cmac_bf(h[a], g0[1], g1[1], quad_xor<1>(z[a]));
        cmac_bf(h[a], g0[2], g1[2], quad_xor<2>(z[a]));
        cmac_bf(h[a], g0[3], g1[3], quad_xor<3>(z[a]));
    }
}

// spin q (three colours) of the odd source at checkerboard index cb
template <int P>
__device__ __forceinline__ void load_spin(const SpinorPtr &src, long cb, int q, cx<float> v[3])
{
    // spin q holds the reals 6 q .. 6 q + 5 of the site's 24 (three colours)
    float r[6];
    if constexpr (P == F32) {
        const float *b = static_cast<const float *>(src.d);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int e = 6 * q + k;
            r[k] = b[((long)(e / 4) * src.stride + cb) * 4 + e % 4];
        }
    } else if constexpr (P == F64) {
        // component 3 q + a is vector 3 q + a
        const double2 *b = static_cast<const double2 *>(src.d);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double2 w = b[(long)(3 * q + a) * src.stride + cb];
            r[2 * a] = (float)w.x;
            r[2 * a + 1] = (float)w.y;
        }
    } else {
        // the whole site (three 16-byte vectors and the scale), spin q picked
        // by 0/1 weights (a select on q would become register indexing)
        cx<float> all[12];
        load_spinor<P>(src, 0, cb, all);
        const float w0 = q == 0, w1 = q == 1, w2 = q == 2, w3 = q == 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r[2 * a] = w0 * all[a].re + w1 * all[3 + a].re + w2 * all[6 + a].re + w3 * all[9 + a].re;
            r[2 * a + 1] = w0 * all[a].im + w1 * all[3 + a].im + w2 * all[6 + a].im + w3 * all[9 + a].im;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = cx<float>{r[2 * a], r[2 * a + 1]};
}

// paths D0 .. D1 - 1 of the first layer at one site, accumulated into acc:
// lane q transports spin q, the quad exchanges the four transported spins,
// then lane q applies row q of Gamma_d and spreads over the channels
template <int P, int D0, int D1>
__device__ __forceinline__ void up_paths(const Geom &g, const SpinorPtr &src, const NnLinks &L, const ThinW *W, int t_bc,
                                         const int x[4], int p, long s, int q, cx<float> acc[8][3])
{
#pragma unroll
    for (int d = D0; d < D1; ++d) {
        const Nbr nb = path_neighbour_at(g, x, p, (int)s, d, t_bc);
        const long ncb = d == 0 ? s : nb.idx - g.Vh;  // the odd site read
        cx<float> v[3];
        load_spin<P>(src, ncb, q, v);
        uint32_t z[3];
        if (d == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) z[a] = f2bf2(v[a].re, v[a].im);
        } else {
            cx<float> t[3];
            transport_bf(L, nb, d, v, t);
#pragma unroll
            for (int a = 0; a < 3; ++a) z[a] = f2bf2(t[a].re, t[a].im);
        }
        cx<float> h[3];
        spin_mix(W, d, q, z, h);
        uint32_t hb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) hb[a] = f2bf2(h[a].re, h[a].im);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t c0 = W->C[d][c][0], c1 = W->C[d][c][1];
#pragma unroll
            for (int a = 0; a < 3; ++a) cmac_bf(acc[c][a], c0, c1, hb[a]);
        }
    }
}

// 1 -> 8: y_c(x) = sum_d C_d[c] (Gamma_d T_d r)(x) for an odd source r
// (precision P): odd sites take the d = 0 path only, even sites the eight hops.
// Tiles of 64 sites of one parity, alternating (tile 2 i + p); with
// even_only, even tiles only (tile i), the odd half of y left untouched.
template <int P, bool EVEN_ONLY>
__global__ void __launch_bounds__(256) nn_up_kernel(Geom g, SpinorPtr src, Act y, NnLinks L, const ThinW *W,
                                                    int t_bc, int xcd)
{
    constexpr int even_only = EVEN_ONLY ? 1 : 0;
    __shared__ __attribute__((aligned(16))) uint32_t ys[8 * 64 * 12];  // [channel][site][12 words]
    const long tile = xcd_block(xcd);
    const int p = even_only ? 0 : (int)(tile & 1);
    const long s0 = (even_only ? tile : (tile >> 1)) * 64;
    const int sl = threadIdx.x / 4, q = threadIdx.x % 4;
    const long s = s0 + sl;
    // every lane runs the paths (the quad exchange needs all four lanes):
    // lanes past the end compute the last site again, and their rows of the
    // tile are never stored
    const long sc = s < g.Vh ? s : g.Vh - 1;
    int x[4];
    cb_coords(g, (int)sc, p, x);
    cx<float> acc[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[c][a] = cx<float>{0.f, 0.f};
    // odd sites: the d = 0 path; even sites: the eight hops, unrolled so that
    // the loads of later paths are issued before the arithmetic of earlier ones
    if (p == 1)
        up_paths<P, 0, 1>(g, src, L, W, t_bc, x, p, sc, q, acc);
    else
        up_paths<P, 1, NN_P>(g, src, L, W, t_bc, x, p, sc, q, acc);
    // the tile's output through LDS, stored as whole 16-byte vectors
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint32_t *o = ys + (c * 64 + sl) * 12 + 3 * q;
        o[0] = f2bf2(acc[c][0].re, acc[c][0].im);
        o[1] = f2bf2(acc[c][1].re, acc[c][1].im);
        o[2] = f2bf2(acc[c][2].re, acc[c][2].im);
    }
    __syncthreads();
    const long gs0 = (long)p * g.Vh + s0;
    const uint4 *yv = reinterpret_cast<const uint4 *>(ys);
    for (int v = threadIdx.x; v < 8 * 64 * 3; v += blockDim.x) {
        const int c = v / (64 * 3), o = v % (64 * 3);
        if (s0 + o / 3 >= g.Vh) continue;
        reinterpret_cast<uint4 *>(y.d + ((long)c * y.stride + gs0) * 12)[o] = yv[v];
    }
}


// 8 -> 1 on odd sites: y(x) = sum_d T_d Gamma_d (sum_c C_d[c] x_c)(x), written
// as an FP32 odd spinor field.  64 odd sites per block, staged in LDS so that
// the stores are whole 16-byte vectors.
__global__ void __launch_bounds__(256) nn_down_kernel(Geom g, Act xin, SpinorPtr yo, NnLinks L, const ThinW *W,
                                                      int t_bc, int xcd)
{
    __shared__ __attribute__((aligned(16))) float ys[64 * 24];
    const long s0 = (long)xcd_block(xcd) * 64;
    const int sl = threadIdx.x / 4, q = threadIdx.x % 4;
    const long s = s0 + sl;
    const bool valid = s < g.Vh;
    int x[4] = {0, 0, 0, 0};
    if (valid) cb_coords(g, (int)s, 1, x);
    cx<float> acc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = cx<float>{0.f, 0.f};
#pragma unroll
    for (int d = 0; d < NN_P; ++d) {
        // channel contraction of spin q at the neighbour (BF16 activations as they are stored)
        cx<float> w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a] = cx<float>{0.f, 0.f};
        Nbr nb{};
        if (valid) {
            nb = path_neighbour_at(g, x, 1, (int)s, d, t_bc);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint32_t *src = xin.d + ((long)c * xin.stride + nb.idx) * 12 + 3 * q;
                const uint32_t c0 = W->C[d][c][0], c1 = W->C[d][c][1];
                const uint32_t z0 = src[0], z1 = src[1], z2 = src[2];
                cmac_bf(w[0], c0, c1, z0);
                cmac_bf(w[1], c0, c1, z1);
                cmac_bf(w[2], c0, c1, z2);
            }
        }
        uint32_t wb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) wb[a] = f2bf2(w[a].re, w[a].im);
        cx<float> h[3];
        spin_mix(W, d, q, wb, h);
        if (!valid) continue;
        if (d == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] = acc[a] + h[a];
        } else {
            cx<float> t[3];
            transport_bf(L, nb, d, h, t);
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] = acc[a] + t[a];
        }
    }
    // [site][spin q][colour][re, im] in LDS, then 16-byte vectors: vector kv of
    // a site holds its reals 4 kv .. 4 kv + 3
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ys[sl * 24 + 6 * q + 2 * a] = acc[a].re;
        ys[sl * 24 + 6 * q + 2 * a + 1] = acc[a].im;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < 6 * 64; v += blockDim.x) {
        const int kv = v / 64, sn = v % 64;
        if (s0 + sn >= g.Vh) continue;
        reinterpret_cast<float4 *>(yo.d)[(long)kv * yo.stride + s0 + sn] =
            *reinterpret_cast<const float4 *>(&ys[sn * 24 + 4 * kv]);
    }
}

// Second half of P_1 = L_1^dagger L_1 on odd sites (see nn_build_p1_kernel):
//     y(s) = G00 r(s) + sum_{d' >= 1} T_d' Gamma'_d' z_d'(s + d'),
// r the odd source (precision P), z_d' channel d' - 1 of the even half of z
// (written by nn_up_kernel with THIN_P1_UP, even tiles only).  One channel
// per path instead of eight: no channel contraction.  FP32 odd output,
// staged in LDS as in nn_down_kernel.
template <int P>
__global__ void __launch_bounds__(256) nn_p1_down_kernel(Geom g, SpinorPtr src, Act z, SpinorPtr yo, NnLinks L,
                                                         const ThinW *W, int t_bc, int xcd)
{
    __shared__ __attribute__((aligned(16))) float ys[64 * 24];
    const long s0 = (long)xcd_block(xcd) * 64;
    const int sl = threadIdx.x / 4, q = threadIdx.x % 4;
    const long s = s0 + sl;
    // lanes past the end repeat the last site (the quad exchange needs all
    // four lanes of a site); their rows of the tile are never stored
    const long sc = s < g.Vh ? s : g.Vh - 1;
    int x[4];
    cb_coords(g, (int)sc, 1, x);
    cx<float> acc[3];
    {
        cx<float> v[3];
        load_spin<P>(src, sc, q, v);
        uint32_t vb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) vb[a] = f2bf2(v[a].re, v[a].im);
        spin_mix(W, 0, q, vb, acc);
    }
#pragma unroll
    for (int d = 1; d < NN_P; ++d) {
        const Nbr nb = path_neighbour_at(g, x, 1, (int)sc, d, t_bc);
        const uint32_t *zp = z.d + ((long)(d - 1) * z.stride + nb.idx) * 12 + 3 * q;
        const uint32_t w[3] = {zp[0], zp[1], zp[2]};
        cx<float> h[3], t[3];
        spin_mix(W, d, q, w, h);
        transport_bf(L, nb, d, h, t);
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a] = acc[a] + t[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ys[sl * 24 + 6 * q + 2 * a] = acc[a].re;
        ys[sl * 24 + 6 * q + 2 * a + 1] = acc[a].im;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < 6 * 64; v += blockDim.x) {
        const int kv = v / 64, sn = v % 64;
        if (s0 + sn >= g.Vh) continue;
        reinterpret_cast<float4 *>(yo.d)[(long)kv * yo.stride + s0 + sn] =
            *reinterpret_cast<const float4 *>(&ys[sn * 24 + 4 * kv]);
    }
}

// sum of the per-block partials: P[i] = sum_b partial[b][i]
__global__ void nn_reduce_partials_kernel(const float *partial, int nblocks, int n, float *P)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * n + i];
    P[i] = s;
}

// P[l] = sum over blocks of the partials, then the complex weight gradient
//   S[(c,s),(c',s')] = (P00 + P11) + i (P01 - P10)
//   grad C[c,c'] = 2 conj(sum_{s,s'} S Gamma[s,s']), grad Gamma[s,s'] = 2 conj(sum_{c,c'} S C[c,c'])
__global__ void nn_grad_combine_kernel(const float *partial, int nblocks, const float *p, float *grad, int cin,
                                       int cout)
{
    const int MD = pad16(8 * cout), KD = pad16(8 * cin);
    const int per = cin * cout + 16;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN_P * per) return;
    const int d = t / per, e = t % per;
    auto P = [&](int m, int k) {
        float s = 0.f;
        for (int b = 0; b < nblocks; ++b) s += partial[((size_t)b * NN_P + d) * MD * KD + m * KD + k];
        return s;
    };
    auto S = [&](int c, int s, int cp, int sp, float &re, float &im) {
        const int m = c * 8 + s * 2, k = cp * 8 + sp * 2;
        const float p00 = P(m, k), p11 = P(m + 1, k + 1), p01 = P(m, k + 1), p10 = P(m + 1, k);
        re = p00 + p11;
        im = p01 - p10;
    };
    const float *pd = p + (size_t)d * per * 2;
    float gr = 0.f, gi = 0.f;
    if (e < cin * cout) {
        const int c = e / cin, cp = e % cin;
        for (int s = 0; s < 4; ++s)
            for (int sp = 0; sp < 4; ++sp) {
                float sr, si;
                S(c, s, cp, sp, sr, si);
                const float Gr = pd[2 * (cin * cout + s * 4 + sp)], Gi = pd[2 * (cin * cout + s * 4 + sp) + 1];
                gr += sr * Gr - si * Gi;
                gi += sr * Gi + si * Gr;
            }
    } else {
        const int s = (e - cin * cout) / 4, sp = (e - cin * cout) % 4;
        for (int c = 0; c < cout; ++c)
            for (int cp = 0; cp < cin; ++cp) {
                float sr, si;
                S(c, s, cp, sp, sr, si);
                const float Cr = pd[2 * (c * cin + cp)], Ci = pd[2 * (c * cin + cp) + 1];
                gr += sr * Cr - si * Ci;
                gi += sr * Ci + si * Cr;
            }
    }
    grad[(size_t)d * per * 2 + 2 * e] = 2.f * gr;
    grad[(size_t)d * per * 2 + 2 * e + 1] = -2.f * gi;
}

__global__ void nn_adam_kernel(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                               float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.f - b1) * gi;
    v[i] = b2 * v[i] + (1.f - b2) * gi * gi;
    p[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
}

__global__ void nn_zero_kernel(float *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

int nn_ensure(tmx_ctx *c)
{
    if (!c->pc) c->pc = new PcState();
    PcState &s = *c->pc;
    if (s.params) return TMX_OK;
    const size_t bytes = nn_num_params() * sizeof(float);
    float *bufs[4];
    for (int i = 0; i < 4; ++i) bufs[i] = static_cast<float *>(dev_alloc(c, bytes));
    uint16_t *wf[NN_L], *wa[NN_L];
    ThinW *thin = static_cast<ThinW *>(dev_alloc(c, THIN_SETS * sizeof(ThinW)));
    bool ok = bufs[0] && bufs[1] && bufs[2] && bufs[3] && thin;
    for (int l = 0; l < NN_L; ++l) {
        const size_t nf = (size_t)NN_P * pad16(8 * NN_COUT[l]) * pad16(8 * NN_CIN[l]);
        const size_t na = (size_t)NN_P * pad16(8 * NN_CIN[l]) * pad16(8 * NN_COUT[l]);
        wf[l] = static_cast<uint16_t *>(dev_alloc(c, nf * 2));
        wa[l] = static_cast<uint16_t *>(dev_alloc(c, na * 2));
        ok = ok && wf[l] && wa[l];
    }
    if (!ok) {
        dev_free(c, thin);
        for (int i = 0; i < 4; ++i) dev_free(c, bufs[i]);
        for (int l = 0; l < NN_L; ++l) {
            dev_free(c, wf[l]);
            dev_free(c, wa[l]);
        }
        return set_err(c, TMX_ENOMEM, "preconditioner weights: out of device memory");
    }
    s.nparam = nn_num_params();
    s.params = bufs[0];
    s.grad = bufs[1];
    s.adam_m = bufs[2];
    s.adam_v = bufs[3];
    s.thin = thin;
    for (int l = 0; l < NN_L; ++l) {
        s.Wf[l] = wf[l];
        s.Wa[l] = wa[l];
    }
    return TMX_OK;
}

int nn_build_weights(tmx_ctx *c)
{
    PcState &s = *c->pc;
    if (s.w_ok) return TMX_OK;
    for (int l = 0; l < NN_L; ++l) {
        const float *pl = s.params + layer_param_offset(l);
        const int n = NN_P * pad16(8 * NN_COUT[l]) * pad16(8 * NN_CIN[l]);
        hipLaunchKernelGGL(nn_build_w_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, pl, s.Wf[l], NN_CIN[l],
                           NN_COUT[l], 0);
        hipLaunchKernelGGL(nn_build_w_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, pl, s.Wa[l], NN_CIN[l],
                           NN_COUT[l], 1);
    }
    const float *p0 = s.params + layer_param_offset(0), *p3 = s.params + layer_param_offset(NN_L - 1);
    hipLaunchKernelGGL(nn_build_thin_kernel, dim3(1), dim3(64), 0, c->stream, p0, s.thin + THIN_UP_F, 1, 8, 0);
    hipLaunchKernelGGL(nn_build_thin_kernel, dim3(1), dim3(64), 0, c->stream, p3, s.thin + THIN_DOWN_F, 8, 1, 0);
    hipLaunchKernelGGL(nn_build_thin_kernel, dim3(1), dim3(64), 0, c->stream, p3, s.thin + THIN_UP_A, 8, 1, 1);
    hipLaunchKernelGGL(nn_build_thin_kernel, dim3(1), dim3(64), 0, c->stream, p0, s.thin + THIN_DOWN_A, 1, 8, 1);
    hipLaunchKernelGGL(nn_build_p1_kernel, dim3(1), dim3(NN_P * NN_P), 0, c->stream, p0, s.thin);
    int r = hip_err(c, hipGetLastError(), "build weights");
    if (!r) s.w_ok = true;
    return r;
}

// BF16 network links, rebuilt from the FP64 master copy after every gauge upload
int nn_links(tmx_ctx *c, NnLinks &L)
{
    PcState &s = *c->pc;
    const long Vh = c->Vh;
    if (!s.lrow || !s.lcol) {
        if (!s.lrow) s.lrow = static_cast<uint32_t *>(dev_alloc(c, 72 * Vh * sizeof(uint32_t)));
        if (!s.lcol) s.lcol = static_cast<uint32_t *>(dev_alloc(c, 72 * Vh * sizeof(uint32_t)));
        if (!s.lrow || !s.lcol) return set_err(c, TMX_ENOMEM, "network links: out of device memory");
        s.links_upload = -1;
    }
    if (s.links_upload != c->uploads) {
        if (!c->gauge_loaded) return set_err(c, TMX_ENOTLOADED, "no gauge field loaded");
        const long n = 8 * Vh;
        hipLaunchKernelGGL(nn_links_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                           static_cast<const double2 *>(c->links[F64]), s.lrow, s.lcol, Vh);
        int r = hip_err(c, hipGetLastError(), "network links");
        if (r) return r;
        s.links_upload = c->uploads;
    }
    L = NnLinks{s.lrow, s.lcol, Vh};
    return TMX_OK;
}

// one layer: bf16 output y, or (cout == 1) FP32 odd spinor yo
int launch_layer(tmx_ctx *c, int cin, int cout, Act x, Act y, SpinorPtr yo, const uint16_t *W)
{
    NnLinks L;
    int r = nn_links(c, L);
    if (r) return r;
    const long V = 2 * c->Vh;
    const long s_begin = cout == 1 ? c->Vh : 0;
    // one-channel input or 8 -> 8: tiles of the two parities interleaved (see the kernel)
    const bool ilv = cin == 1 || (cin == 8 && cout == 8);
    const long ntiles = ilv ? 2 * ((c->Vh + NL_S - 1) / NL_S) : (V - s_begin + NL_S - 1) / NL_S;
    const dim3 grid((unsigned)ntiles), block(256);
    const int tb = c->par.t_bc, xcd = c->xcd_remap;
    kstat_begin(c, "NN_" + std::to_string(cin) + "x" + std::to_string(cout));
    if (cin == 1 && cout == 8)
        hipLaunchKernelGGL((nn_layer_kernel<1, 8>), grid, block, 0, c->stream, c->g, x, y, yo, L, W, tb, s_begin, V,
                           xcd);
    else if (cin == 8 && cout == 8)
        hipLaunchKernelGGL((nn_layer_kernel<8, 8>), grid, block, 0, c->stream, c->g, x, y, yo, L, W, tb, s_begin, V,
                           xcd);
    else if (cin == 8 && cout == 1)
        hipLaunchKernelGGL((nn_layer_kernel<8, 1>), grid, block, 0, c->stream, c->g, x, y, yo, L, W, tb, s_begin, V,
                           xcd);
    else
        return set_err(c, TMX_EINVAL, "network layer shape");
    kstat_end(c);
    return hip_err(c, hipGetLastError(), "network layer");
}

template <int P>
static void up_launch(tmx_ctx *c, dim3 grid, dim3 block, SpinorPtr r, Act y, const NnLinks &L, const ThinW *W, int tb,
                      int xcd, int even_only)
{
    if (even_only)
        hipLaunchKernelGGL((nn_up_kernel<P, true>), grid, block, 0, c->stream, c->g, r, y, L, W, tb, xcd);
    else
        hipLaunchKernelGGL((nn_up_kernel<P, false>), grid, block, 0, c->stream, c->g, r, y, L, W, tb, xcd);
}

// first layer (1 -> 8) on the odd field r of precision pr, straight from the
// field; with even_only, the even half of y only (the first half of P_1)
int launch_up(tmx_ctx *c, SpinorPtr r, int pr, Act y, const ThinW *W, int even_only = 0)
{
    NnLinks L;
    int rc = nn_links(c, L);
    if (rc) return rc;
    const long tiles = (c->Vh + 63) / 64;
    const dim3 grid((unsigned)(even_only ? tiles : 2 * tiles)), block(256);
    const int tb = c->par.t_bc, xcd = c->xcd_remap;
    kstat_begin(c, even_only ? "NN_P1_UP" : "NN_1x8");
    if (pr == F64)
        up_launch<F64>(c, grid, block, r, y, L, W, tb, xcd, even_only);
    else if (pr == F32)
        up_launch<F32>(c, grid, block, r, y, L, W, tb, xcd, even_only);
    else
        up_launch<F16>(c, grid, block, r, y, L, W, tb, xcd, even_only);
    kstat_end(c);
    return hip_err(c, hipGetLastError(), "network first layer");
}

// second half of P_1 on the odd source r (precision pr) and the path fields z
int launch_p1_down(tmx_ctx *c, SpinorPtr r, int pr, Act z, SpinorPtr yo, const ThinW *W)
{
    NnLinks L;
    int rc = nn_links(c, L);
    if (rc) return rc;
    const dim3 grid((unsigned)((c->Vh + 63) / 64)), block(256);
    const int tb = c->par.t_bc, xcd = c->xcd_remap;
    kstat_begin(c, "NN_P1_DOWN");
    if (pr == F64)
        hipLaunchKernelGGL(nn_p1_down_kernel<F64>, grid, block, 0, c->stream, c->g, r, z, yo, L, W, tb, xcd);
    else if (pr == F32)
        hipLaunchKernelGGL(nn_p1_down_kernel<F32>, grid, block, 0, c->stream, c->g, r, z, yo, L, W, tb, xcd);
    else
        hipLaunchKernelGGL(nn_p1_down_kernel<F16>, grid, block, 0, c->stream, c->g, r, z, yo, L, W, tb, xcd);
    kstat_end(c);
    return hip_err(c, hipGetLastError(), "network P_1");
}

// last layer (8 -> 1) into the FP32 odd field yo
int launch_down(tmx_ctx *c, Act x, SpinorPtr yo, const ThinW *W)
{
    NnLinks L;
    int rc = nn_links(c, L);
    if (rc) return rc;
    const dim3 grid((unsigned)((c->Vh + 63) / 64)), block(256);
    kstat_begin(c, "NN_8x1");
    hipLaunchKernelGGL(nn_down_kernel, grid, block, 0, c->stream, c->g, x, yo, L, W, c->par.t_bc, c->xcd_remap);
    kstat_end(c);
    return hip_err(c, hipGetLastError(), "network last layer");
}

constexpr int WG_BLOCKS = 64;

int launch_wgrad(tmx_ctx *c, int cin, int cout, Act x, Act dy, float *partial)
{
    NnLinks L;
    int r = nn_links(c, L);
    if (r) return r;
    const dim3 grid(WG_BLOCKS, NN_P), block(256);
    const int tb = c->par.t_bc;
    if (cin == 1 && cout == 8)
        hipLaunchKernelGGL((nn_wgrad_kernel<1, 8>), grid, block, 0, c->stream, c->g, x, dy, L, tb, partial);
    else if (cin == 8 && cout == 8)
        hipLaunchKernelGGL((nn_wgrad_kernel<8, 8>), grid, block, 0, c->stream, c->g, x, dy, L, tb, partial);
    else if (cin == 8 && cout == 1)
        hipLaunchKernelGGL((nn_wgrad_kernel<8, 1>), grid, block, 0, c->stream, c->g, x, dy, L, tb, partial);
    else
        return set_err(c, TMX_EINVAL, "network layer shape");
    return hip_err(c, hipGetLastError(), "weight gradient");
}

// activation buffer (channels ch) of the full lattice, BF16
Act act(tmx_ctx *c, const std::string &name, int ch)
{
    const long V = 2 * c->Vh;
    void *d = ws_get(c, "nn_" + name, (size_t)ch * V * 48);
    return Act{static_cast<uint32_t *>(d), V};
}

// odd field r (precision pr) -> one-channel activation supported on odd sites
int embed(tmx_ctx *c, SpinorPtr r, int pr, Act a)
{
    const long Vh = c->Vh;
    const dim3 grid((unsigned)((Vh + 255) / 256)), block(256);
    if (pr == F64)
        hipLaunchKernelGGL(nn_embed_kernel<F64>, grid, block, 0, c->stream, r, a, Vh);
    else if (pr == F32)
        hipLaunchKernelGGL(nn_embed_kernel<F32>, grid, block, 0, c->stream, r, a, Vh);
    else
        hipLaunchKernelGGL(nn_embed_kernel<F16>, grid, block, 0, c->stream, r, a, Vh);
    return hip_err(c, hipGetLastError(), "embed");
}

// The Hermitian form P r = L_1^dagger L_2^dagger L_2 L_1 r (layers 1 and 2 of
// the weights; depth 2) or its short form P_1 r = L_1^dagger L_1 r (depth 1),
// an FP32 odd field; with acts, the inputs of its layer applications are kept
// (for the gradient).
int nn_forward_sym(tmx_ctx *c, SpinorPtr out, SpinorPtr r, int pr, int depth, std::vector<Act> *acts)
{
    const bool keep = acts != nullptr;
    const ThinW *thin = c->pc->thin;
    Act a0{};
    if (keep) {
        a0 = act(c, "a0", 1);
        if (!a0.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        int rc = embed(c, r, pr, a0);
        if (rc) return rc;
        acts->push_back(a0);
    }
    Act a1 = act(c, keep ? "a1" : "p1", 8);
    if (!a1.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
    // P_1 without kept activations: the two path-channel halves (no 8-channel
    // intermediate on odd sites, one channel per path in the second half)
    if (depth == 1 && !keep) {
        int rc = launch_up(c, r, pr, a1, thin + THIN_P1_UP, 1);
        return rc ? rc : launch_p1_down(c, r, pr, a1, out, thin + THIN_P1_DOWN);
    }
    int rc = launch_up(c, r, pr, a1, thin + THIN_UP_F);  // L_1
    if (rc) return rc;
    if (keep) acts->push_back(a1);
    if (depth == 1) return launch_down(c, a1, out, thin + THIN_DOWN_A);  // L_1^dagger
    Act a2 = act(c, keep ? "a2" : "p2", 8), a3 = act(c, keep ? "a3" : "p3", 8);
    if (!a2.d || !a3.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
    rc = launch_layer(c, 8, 8, a1, a2, SpinorPtr{}, c->pc->Wf[1]);  // L_2
    if (!rc) rc = launch_layer(c, 8, 8, a2, a3, SpinorPtr{}, c->pc->Wa[1]);  // L_2^dagger
    if (rc) return rc;
    if (keep) {
        acts->push_back(a2);
        acts->push_back(a3);
    }
    return launch_down(c, a3, out, thin + THIN_DOWN_A);  // L_1^dagger
}

// The network on the odd field r: out = K r (mode 0), K^dagger r (mode 1),
// the Hermitian form P r (mode 2) or its short form P_1 r (mode 3), an FP32
// odd field.  With acts, the layer inputs are kept (for the gradient).
int nn_forward(tmx_ctx *c, SpinorPtr out, SpinorPtr r, int pr, int dagger, std::vector<Act> *acts)
{
    int rc = nn_ensure(c);
    if (rc) return rc;
    if (!c->pc->have_weights) return set_err(c, TMX_ENOTLOADED, "preconditioner weights not set");
    rc = ensure_ready(c, F32, false);
    if (!rc) rc = nn_build_weights(c);
    if (rc) return rc;
    if (dagger == 2 || dagger == 3) return nn_forward_sym(c, out, r, pr, dagger == 2 ? 2 : 1, acts);
    const bool keep = acts != nullptr;
    const ThinW *thin = c->pc->thin;
    Act a{};
    if (keep) {
        // the embedded source is the first layer's input of the weight gradient
        a = act(c, "a0", 1);
        if (!a.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        rc = embed(c, r, pr, a);
        if (rc) return rc;
    }
    for (int i = 0; i < NN_L; ++i) {
        const int l = dagger ? NN_L - 1 - i : i;
        const int cin = dagger ? NN_COUT[l] : NN_CIN[l];
        const int cout = dagger ? NN_CIN[l] : NN_COUT[l];
        const uint16_t *W = dagger ? c->pc->Wa[l] : c->pc->Wf[l];
        if (acts) acts->push_back(a);
        if (cout == 1) return launch_down(c, a, out, thin + (dagger ? THIN_DOWN_A : THIN_DOWN_F));
        Act b = act(c, (keep ? "a" : "p") + std::to_string(i + 1), cout);
        if (!b.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        rc = cin == 1 ? launch_up(c, r, pr, b, thin + (dagger ? THIN_UP_A : THIN_UP_F))
                      : launch_layer(c, cin, cout, a, b, SpinorPtr{}, W);
        if (rc) return rc;
        a = b;
    }
    return set_err(c, TMX_EINVAL, "network without an output layer");
}

}  // namespace

// z = K r (dagger = 0), K^dagger r (dagger = 1) or P r (dagger = 2): odd fields r (precision
// pr, stride Vh) and z (precision pz: F64 or F32)
int pc_apply_internal(tmx_ctx *c, SpinorPtr z, int pz, SpinorPtr r, int pr, int dagger)
{
    if (pz != F32 && pz != F64) return set_err(c, TMX_EINVAL, "preconditioner output precision");
    if (pz == F32) return nn_forward(c, z, r, pr, dagger, nullptr);
    void *po = ws_get(c, "nn_pout", spinor_field_bytes(F32, 1, c->Vh));
    if (!po) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
    SpinorPtr o = make_spinor(po, F32, 1, c->Vh);
    int rc = nn_forward(c, o, r, pr, dagger, nullptr);
    if (rc) return rc;
    OpCopy<F64, F32> cp{};
    cp.d = z;
    cp.s = o;
    cp.nf = 1;
    HIP_CHECK_RET(c, run_blas(cp, c->Vh, 1, c->red, c->stream), "restrict");
    return TMX_OK;
}

// residual of one training pair: r = (K b)_odd - x, loss |r|^2 / |x|^2; writes
// delta = embed(r) * scale into the output-adjoint field
template <int PX> struct OpPairResidual {
    static constexpr int NRED = 2;
    SpinorPtr out;  // odd view of the last activation (F32)
    SpinorPtr x;    // target (PX)
    SpinorPtr delta;  // odd view of the adjoint field (F32)
    double scale;
    __device__ void operator()(long t, int, double *acc) const
    {
        cd vo[12], vx[12];
        ld<F32>(out, 0, t, vo);
        ld<PX>(x, 0, t, vx);
#pragma unroll
        for (int c = 0; c < 12; ++c) vo[c] = vo[c] - vx[c];
        acc[0] += nrm2(vo);
        acc[1] += nrm2(vx);
#pragma unroll
        for (int c = 0; c < 12; ++c) vo[c] = scale * vo[c];
        st<F32>(delta, 0, t, vo);
    }
};

// ---------------------------------------------------------------------------
// flexible GCR with the learned preconditioner
// ---------------------------------------------------------------------------
namespace {

struct Fg {
    tmx_ctx *c;
    long Vh;
    bool nomem = false;  // a workspace could not be allocated
    SpinorPtr f(const std::string &name, int prec)
    {
        void *d = ws_get(c, "fg_" + name, spinor_field_bytes(prec, 1, Vh));
        if (!d) nomem = true;
        return make_spinor(d, prec, 1, Vh);
    }
    // after a group of f() calls: nothing may run on a missing workspace
    int need() const { return nomem ? set_err(c, TMX_ENOMEM, "FGCR workspace: out of device memory") : TMX_OK; }
};

template <class Op> int blas(tmx_ctx *c, const Op &o, long n, double *res, int nres)
{
    HIP_CHECK_RET(c, run_blas(o, n, 1, c->red, c->stream), "fgcr blas");
    if (res) return fetch(c, nres, res);
    return TMX_OK;
}

// r = b - A x in FP64 (A = Mhat or Mhat^dagger); returns |r|^2
int fg_true_residual(tmx_ctx *c, int op, int dagger, SpinorPtr r, SpinorPtr b, SpinorPtr x, SpinorPtr q, double *rr,
                     double *gb)
{
    int rc = op_mhat(c, q, x, op, F64, dagger, 1);
    if (rc) return rc;
    *gb += mhat_bytes_per_site(F64, 1, 1) * c->Vh * 1e-9;
    OpXmyNorm<F64, F64, F64, F64> o{};
    o.r = r;
    o.b = b;
    o.q = q;
    o.rlo = r;
    o.nf = 1;
    return blas(c, o, c->Vh, rr, 1);
}

// one flexible-GCR solve of A x = b to relative tolerance tau (x holds the
// start vector).  Returns TMX_OK, or TMX_ENOCONV on stagnation / maxiter.
int fgcr_stage(tmx_ctx *c, int op, int dagger, SpinorPtr x, SpinorPtr b, double tau, int m, int maxiter,
               int inner_prec, tmx_info *info)
{
    Fg F{c, c->Vh};
    const long Vh = c->Vh;
    SpinorPtr r = F.f("r64", F64), q = F.f("q64", F64), rl = F.f("rl", F32), w = F.f("w", F32);
    std::vector<SpinorPtr> zs(m), ws(m);
    for (int j = 0; j < m; ++j) {
        zs[j] = F.f("z" + std::to_string(j), F32);
        ws[j] = F.f("w" + std::to_string(j), F32);
    }
    {
        const int rn = F.need();
        if (rn) return rn;
    }
    double bb;
    {
        OpCopy<F64, F64> o{};
        o.d = q;
        o.s = b;
        o.nf = 1;
        int rc = blas(c, o, Vh, &bb, 1);
        if (rc) return rc;
    }
    if (!std::isfinite(bb)) return set_err(c, TMX_EINVAL, "source with a non-finite entry");
    if (bb == 0) return TMX_OK;
    double rr;
    int rc = fg_true_residual(c, op, dagger, r, b, x, q, &rr, &info->gbytes);
    if (rc) return rc;
    int it = 0;
    double prev_cycle = rr;
    while (std::sqrt(rr) > tau * std::sqrt(bb) && it < maxiter) {
        // r_lo = r
        {
            OpCopy<F32, F64> o{};
            o.d = rl;
            o.s = r;
            o.nf = 1;
            rc = blas(c, o, Vh, nullptr, 0);
            if (rc) return rc;
        }
        const double cycle_target = std::max(tau * tau * bb, 1e-12 * rr);
        double rlo = rr;
        for (int j = 0; j < m && it < maxiter; ++j) {
            // z_j = K r ; w = A z_j   (low precision)
            rc = pc_apply_internal(c, zs[j], F32, rl, F32, dagger);
            if (rc) return rc;
            rc = op_mhat(c, w, zs[j], op, inner_prec == F64 ? F32 : F32, dagger, 1);
            if (rc) return rc;
            info->gbytes += mhat_bytes_per_site(F32, 1, 1) * Vh * 1e-9;
            ++it;
            // modified Gram-Schmidt against the previous directions
            for (int i = 0; i < j; ++i) {
                OpCdot<F32, F32> d{};
                d.a = ws[i];
                d.b = w;
                d.nf = 1;
                double beta[2];
                rc = blas(c, d, Vh, beta, 2);
                if (rc) return rc;
                OpCaxpy<F32, F32> u{};
                u.y = w;
                u.x = ws[i];
                u.nf = 1;
                u.cre[0] = -beta[0];
                u.cim[0] = -beta[1];
                rc = blas(c, u, Vh, nullptr, 0);
                if (rc) return rc;
                u.y = zs[j];
                u.x = zs[i];
                rc = blas(c, u, Vh, nullptr, 0);
                if (rc) return rc;
            }
            double nw;
            {
                OpCopy<F32, F32> o{};
                o.d = ws[j];
                o.s = w;
                o.nf = 1;
                rc = blas(c, o, Vh, &nw, 1);
                if (rc) return rc;
            }
            if (!(nw > 0) || !std::isfinite(nw)) return set_err(c, TMX_ENOCONV, "FGCR breakdown");
            const double inv = 1.0 / std::sqrt(nw);
            {
                OpAxpby<F32, F32> sc{};
                sc.y = ws[j];
                sc.x = ws[j];
                sc.nf = 1;
                sc.a[0] = 0.0;
                sc.b[0] = inv;
                rc = blas(c, sc, Vh, nullptr, 0);
                if (rc) return rc;
                sc.y = zs[j];
                sc.x = zs[j];
                rc = blas(c, sc, Vh, nullptr, 0);
                if (rc) return rc;
            }
            // alpha = <w_j, r> ; x += alpha z_j ; r -= alpha w_j
            double al[2];
            {
                OpCdot<F32, F32> d{};
                d.a = ws[j];
                d.b = rl;
                d.nf = 1;
                rc = blas(c, d, Vh, al, 2);
                if (rc) return rc;
            }
            {
                OpCaxpy<F64, F32> u{};
                u.y = x;
                u.x = zs[j];
                u.nf = 1;
                u.cre[0] = al[0];
                u.cim[0] = al[1];
                rc = blas(c, u, Vh, nullptr, 0);
                if (rc) return rc;
                OpCaxpy<F32, F32> v{};
                v.y = rl;
                v.x = ws[j];
                v.nf = 1;
                v.cre[0] = -al[0];
                v.cim[0] = -al[1];
                rc = blas(c, v, Vh, &rlo, 1);
                if (rc) return rc;
            }
            if (!std::isfinite(rlo)) return set_err(c, TMX_ENOCONV, "FGCR: non-finite residual");
            if (rlo <= cycle_target) break;
        }
        rc = fg_true_residual(c, op, dagger, r, b, x, q, &rr, &info->gbytes);
        if (rc) return rc;
        info->restarts++;
        if (c->trace)
            std::printf("# TMX: fgcr dagger=%d cycle %d iters %d inner |r|/|b| %.3e true %.3e\n", dagger,
                        info->restarts, it, std::sqrt(rlo / bb), std::sqrt(rr / bb));
        if (!std::isfinite(rr)) return set_err(c, TMX_ENOCONV, "FGCR: non-finite residual");
        // stagnation: less than a factor 2 over a whole cycle
        if (rr > 0.25 * prev_cycle && std::sqrt(rr) > tau * std::sqrt(bb)) {
            info->iters += it;
            return TMX_ENOCONV;
        }
        prev_cycle = rr;
    }
    info->iters += it;
    return std::sqrt(rr) <= tau * std::sqrt(bb) ? TMX_OK : TMX_ENOCONV;
}

}  // namespace

// Solve N x = b (N = Mhat^dagger Mhat, degenerate op) as two preconditioned
// solves, Mhat^dagger y = b with K^dagger and Mhat x = y with K (the "two
// inversions" of a preconditioned solver), each to tol / (1 + cond(Mhat)),
// then check the FP64 true residual of N; plain CG from the current x if the
// network fails to deliver (stagnation, non-finite values or the target missed).
extern "C" int tmx_fgcr_solve_internal(tmx_ctx *c, SpinorPtr x, SpinorPtr b, const tmx_solver_cfg *cfg, tmx_info *info)
{
    if (cfg->op != TMX_OP_PLUS && cfg->op != TMX_OP_MINUS)
        return set_err(c, TMX_EINVAL, "FGCR is built for the degenerate Schur operator");
    tmx_info local{};
    if (!info) info = &local;
    const double tol = cfg->tol > 0 ? cfg->tol : 1e-10;
    const int m = cfg->restart > 0 ? std::min(cfg->restart, 32) : 16;
    const int maxiter = cfg->maxiter > 0 ? cfg->maxiter : 10000;
    const double cond_mhat = 8.0;  // bound on cond(Mhat) for these parameters
    const double tau = tol / (1.0 + cond_mhat);
    int rc = ensure_ready(c, F64, false);
    if (!rc) rc = ensure_ready(c, F32, false);
    if (rc) return rc;
    Fg F{c, c->Vh};
    SpinorPtr y = F.f("y", F64);
    rc = F.need();
    if (rc) return rc;
    // y = 0 ; stage 1: Mhat^dagger y = b
    {
        OpZero<F64> z{};
        z.d = y;
        z.nf = 1;
        rc = blas(c, z, c->Vh, nullptr, 0);
        if (rc) return rc;
    }
    // errors (no memory, a failed launch) end the solve; a stage that does
    // not converge hands over to the CG below
    rc = fgcr_stage(c, cfg->op, 1, y, b, tau, m, maxiter, cfg->inner_prec, info);
    if (rc < 0) return rc;
    bool ok = rc == TMX_OK;
    if (ok) {
        // stage 2: Mhat x = y (x holds the start vector)
        rc = fgcr_stage(c, cfg->op, 0, x, y, tau, m, maxiter, cfg->inner_prec, info);
        if (rc < 0) return rc;
        ok = rc == TMX_OK;
    }
    // acceptance (and fallback) by plain CG on N from the current x: with
    // the network doing its job this only computes the true residual
    int rcg = cg_fallback(c, cfg->op, x, b, tol, maxiter, info);
    if (rcg < 0) return rcg;
    if (!ok || info->fallback) info->fallback = info->fallback || !ok;
    return rcg;
}

}  // namespace tmx

using namespace tmx;

extern "C" {

void tmx_pc_free(tmx_ctx *c)
{
    if (!c || !c->pc) return;
    PcState &s = *c->pc;
    dev_free(c, s.params);
    dev_free(c, s.grad);
    dev_free(c, s.adam_m);
    dev_free(c, s.adam_v);
    for (int l = 0; l < NN_L; ++l) {
        dev_free(c, s.Wf[l]);
        dev_free(c, s.Wa[l]);
    }
    dev_free(c, s.lrow);
    dev_free(c, s.lcol);
    dev_free(c, s.thin);
    delete c->pc;
    c->pc = nullptr;
}

int tmx_pc_num_params(const tmx_ctx *c, size_t *n)
{
    if (!c || !n) return TMX_EINVAL;
    *n = nn_num_params();
    return TMX_OK;
}

int tmx_pc_set_weights(tmx_ctx *c, const float *host_w, size_t n)
{
    if (!c || !host_w) return TMX_EINVAL;
    if (n != nn_num_params()) return set_err(c, TMX_EINVAL, "wrong number of preconditioner weights");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host_w[i])) return set_err(c, TMX_EINVAL, "non-finite preconditioner weight");
    int r = nn_ensure(c);
    if (r) return r;
    PcState &s = *c->pc;
    hipError_t e = hipMemcpyAsync(s.params, host_w, n * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_err(c, e, "set weights");
    s.w_ok = false;
    s.have_weights = true;
    s.adam_t = 0;
    return TMX_OK;
}

int tmx_pc_get_weights(tmx_ctx *c, float *host_w, size_t n)
{
    if (!c || !host_w) return TMX_EINVAL;
    if (n != nn_num_params()) return set_err(c, TMX_EINVAL, "wrong number of preconditioner weights");
    if (!c->pc || !c->pc->have_weights) return set_err(c, TMX_ENOTLOADED, "preconditioner weights not set");
    hipError_t e = hipMemcpyAsync(host_w, c->pc->params, n * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_err(c, e, "get weights");
}

int tmx_pc_apply(tmx_ctx *c, double *out, const double *in, int dagger)
{
    if (!c || !out || !in) return TMX_EINVAL;
    if (dagger < 0 || dagger > 3) return set_err(c, TMX_EINVAL, "tmx_pc_apply: mode is 0 .. 3");
    const long Vh = c->Vh;
    void *pi = ws_get(c, "pca_in", spinor_field_bytes(F32, 1, Vh));
    void *po = ws_get(c, "pca_out", spinor_field_bytes(F32, 1, Vh));
    if (!pi || !po) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
    SpinorPtr I = make_spinor(pi, F32, 1, Vh), O = make_spinor(po, F32, 1, Vh);
    int r = hip_err(c, launch_pack_spinor(in, I, F32, TMX_FIELD_ODD, c->g, 1, c->stream), "pack");
    if (r) return r;
    r = pc_apply_internal(c, O, F32, I, F32, dagger);
    if (r) return r;
    r = hip_err(c, launch_unpack_spinor(out, O, F32, TMX_FIELD_ODD, c->g, 1, c->stream), "unpack");
    if (r) return r;
    return hip_err(c, hipStreamSynchronize(c->stream), "pc apply");
}

// gradient of the loss for a set of pairs (internal helper, also used by the
// gradient check entry point): accumulates into the partial buffers, returns loss
static int pc_loss_grad(tmx_ctx *c, const double *b, const double *x, const int *idx, int n, int loss_kind, int op,
                        double *loss)
{
    PcState &s = *c->pc;
    const long Vh = c->Vh;
    const size_t fb = (size_t)Vh * 24;  // doubles per canonical odd field
    float *partial[NN_L];
    for (int l = 0; l < NN_L; ++l) {
        const size_t np = (size_t)WG_BLOCKS * NN_P * pad16(8 * NN_COUT[l]) * pad16(8 * NN_CIN[l]);
        partial[l] = static_cast<float *>(ws_get(c, "nn_partial" + std::to_string(l), np * sizeof(float)));
        if (!partial[l]) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        hipLaunchKernelGGL(nn_zero_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, c->stream, partial[l], np);
    }
    void *pb = ws_get(c, "tr_b", spinor_field_bytes(F32, 1, Vh));
    void *px = ws_get(c, "tr_x", spinor_field_bytes(F32, 1, Vh));
    if (!pb || !px) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
    SpinorPtr B = make_spinor(pb, F32, 1, Vh), X = make_spinor(px, F32, 1, Vh);
    double L = 0;
    for (int i = 0; i < n; ++i) {
        const int k = idx ? idx[i] : i;
        int r = hip_err(c, launch_pack_spinor(b + (size_t)k * fb, B, F32, TMX_FIELD_ODD, c->g, 1, c->stream), "pack b");
        if (!r) r = hip_err(c, launch_pack_spinor(x + (size_t)k * fb, X, F32, TMX_FIELD_ODD, c->g, 1, c->stream), "pack x");
        if (r) return r;
        // |x|^2 (solution loss) or |b|^2 (residual loss) for the scale
        OpCopy<F32, F32> nx{};
        nx.d = loss_kind == TMX_LOSS_SOLUTION ? X : B;
        nx.s = nx.d;
        nx.nf = 1;
        r = hip_err(c, run_blas(nx, Vh, 1, c->red, c->stream), "norm");
        double xx = 0;
        if (!r) r = fetch(c, 1, &xx);
        if (r) return r;
        if (!(xx > 0)) return set_err(c, TMX_EINVAL, "training pair with zero norm");
        std::vector<Act> acts;
        void *pz = ws_get(c, "tr_z", spinor_field_bytes(F32, 1, Vh));
        void *pd = ws_get(c, "tr_dl", spinor_field_bytes(F32, 1, Vh));
        if (!pz || !pd) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        const SpinorPtr Z = make_spinor(pz, F32, 1, Vh), DL = make_spinor(pd, F32, 1, Vh);
        const bool sym = loss_kind == TMX_LOSS_SYM || loss_kind == TMX_LOSS_SYM1;
        r = nn_forward(c, Z, B, F32, loss_kind == TMX_LOSS_SYM ? 2 : (sym ? 3 : 0), &acts);
        if (r) return r;
        // DL = dLoss / d(K b) (odd field), then as the one-channel output adjoint
        // (the energy loss of P = A^dagger A is the residual loss's formula
        // with P b in place of K b and pairs x = N^{-1} b)
        if (loss_kind == TMX_LOSS_SOLUTION) {
            // (K b - x) / (|x|^2 n)
            OpPairResidual<F32> pr{};
            pr.out = Z;
            pr.x = X;
            pr.delta = DL;
            pr.scale = 1.0 / (xx * n);
            r = hip_err(c, run_blas(pr, Vh, 1, c->red, c->stream), "pair residual");
            double red[2];
            if (!r) r = fetch(c, 2, red);
            if (r) return r;
            L += red[0] / xx / n;
        } else {
            // e = K b - x ; q = Mhat e ; loss |q|^2/|b|^2 ; DL = Mhat^dagger q / (|b|^2 n)
            void *pe = ws_get(c, "tr_e", spinor_field_bytes(F32, 1, Vh));
            void *pq = ws_get(c, "tr_q", spinor_field_bytes(F32, 1, Vh));
            if (!pe || !pq) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
            SpinorPtr E = make_spinor(pe, F32, 1, Vh), Q = make_spinor(pq, F32, 1, Vh);
            OpPairResidual<F32> pr{};
            pr.out = Z;
            pr.x = X;
            pr.delta = E;
            pr.scale = 1.0;
            r = hip_err(c, run_blas(pr, Vh, 1, c->red, c->stream), "pair residual");
            if (!r) r = op_mhat(c, Q, E, op, F32, 0, 1);
            if (r) return r;
            OpCopy<F32, F32> nq{};
            nq.d = Q;
            nq.s = Q;
            nq.nf = 1;
            r = hip_err(c, run_blas(nq, Vh, 1, c->red, c->stream), "residual norm");
            double qq = 0;
            if (!r) r = fetch(c, 1, &qq);
            if (!r) r = op_mhat(c, E, Q, op, F32, 1, 1);
            if (r) return r;
            OpAxpby<F32, F32> sc{};
            sc.y = DL;
            sc.x = E;
            sc.nf = 1;
            sc.a[0] = 1.0 / (xx * n);
            sc.b[0] = 0.0;
            r = hip_err(c, run_blas(sc, Vh, 1, c->red, c->stream), "delta");
            if (r) return r;
            L += qq / xx / n;
        }
        Act delta = act(c, "d4", 1);
        if (!delta.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        r = embed(c, DL, F32, delta);
        if (r) return r;
        if (loss_kind == TMX_LOSS_SYM1) {
            // P_1 = L_1^dagger L_1, inputs a0, a1 (layer gradients as below)
            Act d1 = act(c, "d1", 8);
            if (!d1.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
            r = launch_wgrad(c, 1, 8, delta, acts[1], partial[0]);                     // L_1^dagger
            if (!r) r = launch_layer(c, 1, 8, delta, d1, SpinorPtr{}, s.Wf[0]);
            if (!r) r = launch_wgrad(c, 1, 8, acts[0], d1, partial[0]);                // L_1
            if (r) return r;
            continue;
        }
        if (sym) {
            // P = L_1^dagger L_2^dagger L_2 L_1, inputs a0 .. a3.  A layer used as
            // its adjoint (input x, output adjoint d) takes the gradient of its
            // forward use on d with output adjoint x.
            Act d3 = act(c, "d3", 8), d2 = act(c, "d2", 8), d1 = act(c, "d1", 8);
            if (!d3.d || !d2.d || !d1.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
            r = launch_wgrad(c, 1, 8, delta, acts[3], partial[0]);                     // L_1^dagger
            if (!r) r = launch_layer(c, 1, 8, delta, d3, SpinorPtr{}, s.Wf[0]);
            if (!r) r = launch_wgrad(c, 8, 8, d3, acts[2], partial[1]);                // L_2^dagger
            if (!r) r = launch_layer(c, 8, 8, d3, d2, SpinorPtr{}, s.Wf[1]);
            if (!r) r = launch_wgrad(c, 8, 8, acts[1], d2, partial[1]);                // L_2
            if (!r) r = launch_layer(c, 8, 8, d2, d1, SpinorPtr{}, s.Wa[1]);
            if (!r) r = launch_wgrad(c, 1, 8, acts[0], d1, partial[0]);                // L_1
            if (r) return r;
            continue;
        }
        // backward through the layers
        for (int l = NN_L - 1; l >= 0; --l) {
            r = launch_wgrad(c, NN_CIN[l], NN_COUT[l], acts[l], delta, partial[l]);
            if (r) return r;
            if (l > 0) {
                Act nd = act(c, "d" + std::to_string(l), NN_CIN[l]);
                if (!nd.d) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
                r = launch_layer(c, NN_COUT[l], NN_CIN[l], delta, nd, SpinorPtr{}, s.Wa[l]);
                if (r) return r;
                delta = nd;
            }
        }
    }
    for (int l = 0; l < NN_L; ++l) {
        const int per = NN_CIN[l] * NN_COUT[l] + 16;
        const int nthr = NN_P * per;
        const int np = NN_P * pad16(8 * NN_COUT[l]) * pad16(8 * NN_CIN[l]);
        float *P = static_cast<float *>(ws_get(c, "nn_P" + std::to_string(l), (size_t)np * sizeof(float)));
        if (!P) return set_err(c, TMX_ENOMEM, "network workspace: out of device memory");
        hipLaunchKernelGGL(nn_reduce_partials_kernel, dim3((np + 255) / 256), dim3(256), 0, c->stream, partial[l],
                           WG_BLOCKS, np, P);
        hipLaunchKernelGGL(nn_grad_combine_kernel, dim3((nthr + 127) / 128), dim3(128), 0, c->stream, P, 1,
                           s.params + layer_param_offset(l), s.grad + layer_param_offset(l), NN_CIN[l], NN_COUT[l]);
    }
    int r = hip_err(c, hipGetLastError(), "grad combine");
    if (r) return r;
    *loss = L;
    return TMX_OK;
}

int tmx_pc_loss_grad(tmx_ctx *c, const double *b, const double *x, int npairs, int loss_kind, int op, double *loss,
                     float *host_grad)
{
    if (!c || !b || !x || npairs < 1 || !loss) return TMX_EINVAL;
    if (loss_kind < TMX_LOSS_RESIDUAL || loss_kind > TMX_LOSS_SYM1) return set_err(c, TMX_EINVAL, "unknown loss kind");
    if (op != TMX_OP_PLUS && op != TMX_OP_MINUS)
        return set_err(c, TMX_EINVAL, "the network is trained for Mhat(+mu) or Mhat(-mu)");
    int r = nn_ensure(c);
    if (r) return r;
    if (!c->pc->have_weights) return set_err(c, TMX_ENOTLOADED, "preconditioner weights not set");
    r = ensure_ready(c, F32, false);
    if (!r) r = nn_build_weights(c);
    if (!r) r = pc_loss_grad(c, b, x, nullptr, npairs, loss_kind, op, loss);
    if (r) return r;
    if (host_grad) {
        hipError_t e = hipMemcpyAsync(host_grad, c->pc->grad, c->pc->nparam * sizeof(float), hipMemcpyDeviceToHost,
                                      c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        return hip_err(c, e, "grad download");
    }
    return hip_err(c, hipStreamSynchronize(c->stream), "loss grad");
}

// Adam defaults for unset (zero) fields of a training configuration
static void adam_params(const tmx_train_cfg *cfg, float &lr, float &b1, float &b2, float &eps)
{
    lr = cfg->lr > 0 ? cfg->lr : 1e-3f;
    b1 = cfg->beta1 > 0 ? cfg->beta1 : 0.9f;
    b2 = cfg->beta2 > 0 ? cfg->beta2 : 0.999f;
    eps = cfg->eps > 0 ? cfg->eps : 1e-8f;
}

// one Adam step on the master weights from the gradient in s.grad
static int adam_step(tmx_ctx *c, float lr, float b1, float b2, float eps)
{
    PcState &s = *c->pc;
    if (s.adam_t == 0) {
        hipLaunchKernelGGL(nn_zero_kernel, dim3((unsigned)((s.nparam + 255) / 256)), dim3(256), 0, c->stream, s.adam_m,
                           s.nparam);
        hipLaunchKernelGGL(nn_zero_kernel, dim3((unsigned)((s.nparam + 255) / 256)), dim3(256), 0, c->stream, s.adam_v,
                           s.nparam);
    }
    s.adam_t++;
    // bias corrections 1 - beta^t
    const float c1 = 1.f - std::pow(b1, (float)s.adam_t), c2 = 1.f - std::pow(b2, (float)s.adam_t);
    hipLaunchKernelGGL(nn_adam_kernel, dim3((unsigned)((s.nparam + 255) / 256)), dim3(256), 0, c->stream, s.params,
                       s.grad, s.adam_m, s.adam_v, (int)s.nparam, lr, b1, b2, eps, c1, c2);
    s.w_ok = false;
    return hip_err(c, hipGetLastError(), "adam");
}

int tmx_pc_adam_step(tmx_ctx *c, const float *host_grad, size_t n, const tmx_train_cfg *cfg)
{
    if (!c || !host_grad || !cfg) return c ? set_err(c, TMX_EINVAL, "tmx_pc_adam_step: bad argument") : TMX_EINVAL;
    if (n != nn_num_params()) return set_err(c, TMX_EINVAL, "wrong number of gradient values");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host_grad[i])) return set_err(c, TMX_EINVAL, "non-finite gradient value");
    int r = nn_ensure(c);
    if (r) return r;
    if (!c->pc->have_weights) return set_err(c, TMX_ENOTLOADED, "preconditioner weights not set");
    float lr, b1, b2, eps;
    adam_params(cfg, lr, b1, b2, eps);
    if (!(b1 < 1.f) || !(b2 < 1.f)) return set_err(c, TMX_EINVAL, "Adam decay rates must lie in (0, 1)");
    r = hip_err(c, hipMemcpyAsync(c->pc->grad, host_grad, n * sizeof(float), hipMemcpyHostToDevice, c->stream),
                "gradient upload");
    if (!r) r = adam_step(c, lr, b1, b2, eps);
    if (r) return r;
    return hip_err(c, hipStreamSynchronize(c->stream), "adam step");
}

int tmx_pc_train(tmx_ctx *c, const double *b, const double *x, int npairs, const tmx_train_cfg *cfg, float *loss_out)
{
    if (!c || !b || !x || npairs < 1 || !cfg || cfg->epochs < 1 || cfg->batch < 1) return TMX_EINVAL;
    if (cfg->loss_kind < TMX_LOSS_RESIDUAL || cfg->loss_kind > TMX_LOSS_SYM1)
        return set_err(c, TMX_EINVAL, "unknown loss kind");
    const int op = cfg->op == 0 ? TMX_OP_PLUS : cfg->op;
    if (op != TMX_OP_PLUS && op != TMX_OP_MINUS)
        return set_err(c, TMX_EINVAL, "the network is trained for Mhat(+mu) or Mhat(-mu)");
    int r = nn_ensure(c);
    if (r) return r;
    if (!c->pc->have_weights) return set_err(c, TMX_ENOTLOADED, "preconditioner weights not set");
    r = ensure_ready(c, F32, false);
    if (r) return r;
    float lr, b1, b2, eps;
    adam_params(cfg, lr, b1, b2, eps);
    if (!(b1 < 1.f) || !(b2 < 1.f)) return set_err(c, TMX_EINVAL, "Adam decay rates must lie in (0, 1)");
    // deterministic shuffle (LCG seeded by cfg->seed)
    std::vector<int> order(npairs);
    for (int i = 0; i < npairs; ++i) order[i] = i;
    uint64_t st = 0x9e3779b97f4a7c15ull ^ (uint64_t)(uint32_t)cfg->seed;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        for (int i = npairs - 1; i > 0; --i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            const int j = (int)((st >> 33) % (uint64_t)(i + 1));
            std::swap(order[i], order[j]);
        }
        double eloss = 0;
        int nb = 0;
        for (int i0 = 0; i0 < npairs; i0 += cfg->batch) {
            const int n = std::min(cfg->batch, npairs - i0);
            r = nn_build_weights(c);
            if (r) return r;
            double L;
            r = pc_loss_grad(c, b, x, order.data() + i0, n, cfg->loss_kind, op, &L);
            if (r) return r;
            if (!std::isfinite(L)) return set_err(c, TMX_ENOCONV, "training loss is not finite");
            eloss += L;
            ++nb;
            r = adam_step(c, lr, b1, b2, eps);
            if (r) return r;
        }
        if (loss_out) loss_out[ep] = (float)(eloss / nb);
    }
    return hip_err(c, hipStreamSynchronize(c->stream), "train");
}

}  // extern "C"
