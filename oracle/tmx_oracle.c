/*
 * Plain FP64 CPU oracle for the even-odd preconditioned Wilson twisted-mass
 * clover operator and its solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the GPU library never
 * includes, links or calls it and it shares no code with it.
 *
 * Everything is written as the plain definition: full 4x4 gamma matrices,
 * full 3x3 links, a dense 12x12 (24x24 for two flavours) site block solved
 * by Gaussian elimination, textbook CG.  No blocking, no fusion, no
 * chirality tricks, no compression.  OpenMP only parallelises independent
 * per-site loops.
 *
 * Conventions (readings where the paper is silent):
 *  - sites: lex = x0 + L0*(x1 + L1*(x2 + L2*x3)); parity = sum(x) mod 2;
 *    one-parity vectors are indexed by cb = lex/2 (L0 even).
 *  - links U[lex][mu][3][3], row-major SU(3); spinors [site][flavour][4][3].
 *  - gamma matrices in a chiral basis: gamma_k = [[0,-i s_k],[i s_k,0]] for
 *    mu = k-1 = 0,1,2 and gamma_4 = [[0,1],[1,0]] for mu = 3;
 *    gamma5 = gamma_1 gamma_2 gamma_3 gamma_4 is computed, not assumed.
 *  - fermion boundary: periodic in x,y,z; in t a factor t_bc (-1 =
 *    antiperiodic) on every hop that crosses the time boundary.  The gauge
 *    field itself is periodic.
 *  - hopping normalisation: D = 1 + T + i nu gamma5 - kappa H with
 *    nu = 2 kappa mu (degenerate); two flavours: D_h = (1+T) + i nubar
 *    gamma5 tau3 - epsbar~ tau1 - kappa H with nubar = 2 kappa mubar,
 *    epsbar~ = 2 kappa epsbar (Section 2, equations for Q^{+-}, Q-hat^{+-}
 *    and Q-hat_h).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static long vol4(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(long i, const int *L, int *x)
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(i % L[mu]);
        i /= L[mu];
    }
}

static long lexof(const int *x, const int *L)
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

static int parityof(const int *x) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

/* neighbour of site i in direction mu, forward (dir=+1) or backward (-1);
 * *sign receives the fermion boundary factor of that hop. */
static long neighbour(long i, int mu, int dir, const int *L, int t_bc, double *sign)
{
    int x[4];
    coords(i, L, x);
    double s = 1.0;
    x[mu] += dir;
    if (x[mu] == L[mu]) {
        x[mu] = 0;
        if (mu == 3) s = (double)t_bc;
    } else if (x[mu] < 0) {
        x[mu] = L[mu] - 1;
        if (mu == 3) s = (double)t_bc;
    }
    *sign = s;
    return lexof(x, L);
}

/* ------------------------------------------------------------------ */
/* gamma matrices                                                      */
/* ------------------------------------------------------------------ */

static cplx GAM[5][4][4]; /* 0..3: gamma_mu, 4: gamma5 */
static cplx SIG[4][4][4][4]; /* sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] */
static int gam_ready = 0;

static void init_gammas(void)
{
    if (gam_ready) return;
    const cplx IU = _Complex_I;
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -IU}, {IU, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof(GAM));
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                GAM[k][a][2 + b] = -IU * pauli[k][a][b];
                GAM[k][2 + a][b] = IU * pauli[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        GAM[3][a][2 + a] = 1;
        GAM[3][2 + a][a] = 1;
    }
    /* gamma5 = gamma_1 gamma_2 gamma_3 gamma_4 */
    cplx t1[4][4], t2[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += GAM[0][a][c] * GAM[1][c][b];
            t1[a][b] = s;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += t1[a][c] * GAM[2][c][b];
            t2[a][b] = s;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx s = 0;
            for (int c = 0; c < 4; ++c) s += t2[a][c] * GAM[3][c][b];
            GAM[4][a][b] = s;
        }
    /* sigma_{mu nu} = (i/2)(gamma_mu gamma_nu - gamma_nu gamma_mu) */
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx s = 0;
                    for (int c = 0; c < 4; ++c)
                        s += GAM[mu][a][c] * GAM[nu][c][b] - GAM[nu][a][c] * GAM[mu][c][b];
                    SIG[mu][nu][a][b] = 0.5 * IU * s;
                }
    gam_ready = 1;
}

/* number of OpenMP threads the oracle's parallel loops use */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* export: gamma matrices (5*16 complex) and sigma (16*16 complex) */
void orc_gammas(cplx *g, cplx *sig)
{
    init_gammas();
    if (g) memcpy(g, GAM, sizeof(GAM));
    if (sig) memcpy(sig, SIG, sizeof(SIG));
}

/* ------------------------------------------------------------------ */
/* small dense helpers                                                 */
/* ------------------------------------------------------------------ */

/* c = a * b (3x3) */
static void mm3(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

/* c = a^dagger */
static void dag3(const cplx *a, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[3 * i + j] = conj(a[3 * j + i]);
}

/* Solve A y = b in place (A n x n, row-major, destroyed; b overwritten with
 * y) by Gaussian elimination with partial pivoting.  Returns 0 on success. */
static int gauss_solve(cplx *A, cplx *b, int n)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs(A[k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (cabs(A[r * n + k]) > best) {
                best = cabs(A[r * n + k]);
                p = r;
            }
        if (best == 0.0) return 1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                cplx t = A[k * n + c];
                A[k * n + c] = A[p * n + c];
                A[p * n + c] = t;
            }
            cplx t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            cplx f = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        cplx s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * b[c];
        b[k] = s / A[k * n + k];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Wilson hopping term H (the M_eo / M_oe of Section 2 times -1/kappa) */
/* ------------------------------------------------------------------ */

/* (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ] * bc.
 * Computed for output sites of parity out_parity (0/1), or all sites (-1);
 * other output sites are set to zero.  nf flavours are hopped identically. */
void orc_hop(const int *L, int t_bc, const cplx *U, const cplx *in, cplx *out, int nf, int out_parity)
{
    init_gammas();
    const long V = vol4(L);
    const int ns = 12 * nf;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        cplx *o = out + i * ns;
        for (int k = 0; k < ns; ++k) o[k] = 0;
        if (out_parity >= 0 && parityof(x) != out_parity) continue;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = +1; dir >= -1; dir -= 2) {
                double sgn;
                long j = neighbour(i, mu, dir, L, t_bc, &sgn);
                cplx link[9];
                if (dir > 0)
                    memcpy(link, U + (i * 4 + mu) * 9, sizeof(link));
                else
                    dag3(U + (j * 4 + mu) * 9, link);
                /* projector P = 1 - dir * gamma_mu */
                cplx P[4][4];
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - dir * GAM[mu][a][b];
                for (int f = 0; f < nf; ++f) {
                    const cplx *src = in + j * ns + 12 * f;
                    /* Upsi[s][a] = sum_b link[a][b] psi[s][b] */
                    cplx up[4][3];
                    for (int s = 0; s < 4; ++s)
                        for (int a = 0; a < 3; ++a) {
                            cplx acc = 0;
                            for (int b = 0; b < 3; ++b) acc += link[3 * a + b] * src[3 * s + b];
                            up[s][a] = acc;
                        }
                    for (int s = 0; s < 4; ++s)
                        for (int a = 0; a < 3; ++a) {
                            cplx acc = 0;
                            for (int t = 0; t < 4; ++t) acc += P[s][t] * up[t][a];
                            o[12 * f + 3 * s + a] += sgn * acc;
                        }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Clover term T (the "clov" part of M_clov, Section 2)                */
/* ------------------------------------------------------------------ */

static const cplx *link_at(const cplx *U, const int *L, const int *x, int mu)
{
    return U + (lexof(x, L) * 4 + mu) * 9;
}

static void shift(const int *x, const int *L, int mu, int d, int *y)
{
    for (int k = 0; k < 4; ++k) y[k] = x[k];
    y[mu] = ((y[mu] + d) % L[mu] + L[mu]) % L[mu];
}

/* Q_{mu nu}(x): sum of the four plaquette leaves around x in the (mu,nu)
 * plane, each starting and ending at x, oriented mu -> nu. */
static void clover_leaves(const cplx *U, const int *L, const int *x, int mu, int nu, cplx *Q)
{
    int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xpmmn[4];
    shift(x, L, mu, +1, xpm);
    shift(x, L, nu, +1, xpn);
    shift(x, L, mu, -1, xmm);
    shift(x, L, nu, -1, xmn);
    shift(xmm, L, nu, +1, xmmpn);
    shift(xmm, L, nu, -1, xmmmn);
    shift(xpm, L, nu, -1, xpmmn);
    cplx a[9], b[9], c[9], d[9], t1[9], t2[9], leaf[9];
    for (int k = 0; k < 9; ++k) Q[k] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
    memcpy(a, link_at(U, L, x, mu), sizeof(a));
    memcpy(b, link_at(U, L, xpm, nu), sizeof(b));
    dag3(link_at(U, L, xpn, mu), c);
    dag3(link_at(U, L, x, nu), d);
    mm3(a, b, t1); mm3(t1, c, t2); mm3(t2, d, leaf);
    for (int k = 0; k < 9; ++k) Q[k] += leaf[k];

    /* U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
    memcpy(a, link_at(U, L, x, nu), sizeof(a));
    dag3(link_at(U, L, xmmpn, mu), b);
    dag3(link_at(U, L, xmm, nu), c);
    memcpy(d, link_at(U, L, xmm, mu), sizeof(d));
    mm3(a, b, t1); mm3(t1, c, t2); mm3(t2, d, leaf);
    for (int k = 0; k < 9; ++k) Q[k] += leaf[k];

    /* U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
    dag3(link_at(U, L, xmm, mu), a);
    dag3(link_at(U, L, xmmmn, nu), b);
    memcpy(c, link_at(U, L, xmmmn, mu), sizeof(c));
    memcpy(d, link_at(U, L, xmn, nu), sizeof(d));
    mm3(a, b, t1); mm3(t1, c, t2); mm3(t2, d, leaf);
    for (int k = 0; k < 9; ++k) Q[k] += leaf[k];

    /* U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+ */
    dag3(link_at(U, L, xmn, nu), a);
    memcpy(b, link_at(U, L, xmn, mu), sizeof(b));
    memcpy(c, link_at(U, L, xpmmn, nu), sizeof(c));
    dag3(link_at(U, L, x, mu), d);
    mm3(a, b, t1); mm3(t1, c, t2); mm3(t2, d, leaf);
    for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
}

/* T(x) = i kappa csw sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x),
 * F = (Q - Q^dagger)/8; stored as a 12x12 matrix per site,
 * row/column index 3*spin + colour.  T: [V][12][12]. */
void orc_clover(const int *L, const cplx *U, double kappa, double csw, cplx *T)
{
    init_gammas();
    const long V = vol4(L);
    const cplx IU = _Complex_I;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        cplx *t = T + i * 144;
        for (int k = 0; k < 144; ++k) t[k] = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx Q[9], F[9];
                clover_leaves(U, L, x, mu, nu, Q);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) F[3 * a + b] = (Q[3 * a + b] - conj(Q[3 * b + a])) / 8.0;
                for (int s = 0; s < 4; ++s)
                    for (int sp = 0; sp < 4; ++sp)
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                t[(3 * s + a) * 12 + 3 * sp + b] += IU * kappa * csw * SIG[mu][nu][s][sp] * F[3 * a + b];
            }
    }
}

/* ------------------------------------------------------------------ */
/* site-diagonal block                                                 */
/* ------------------------------------------------------------------ */

/* Dense site block B (n = 12 nf) of the diagonal part of the operator:
 *   nf = 1: 1 + T + i nu gamma5,                      nu = 2 kappa mu
 *   nf = 2: (1 + T) x 1_f + i nubar gamma5 x tau3 - epst 1 x tau1,
 *           nubar = 2 kappa mubar, epst = 2 kappa epsbar.
 * Index (f, spin, colour) -> 12 f + 3 spin + colour. */
static void site_block(const cplx *Tx, double kappa, double mu, double mubar, double epsbar, int nf, cplx *B)
{
    const cplx IU = _Complex_I;
    const int n = 12 * nf;
    for (int k = 0; k < n * n; ++k) B[k] = 0;
    for (int f = 0; f < nf; ++f)
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) B[(12 * f + r) * n + 12 * f + c] = Tx[r * 12 + c] + (r == c ? 1.0 : 0.0);
    if (nf == 1) {
        double nu = 2.0 * kappa * mu;
        for (int s = 0; s < 4; ++s)
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) B[(3 * s + a) * n + 3 * sp + a] += IU * nu * GAM[4][s][sp];
    } else {
        double nub = 2.0 * kappa * mubar, ept = 2.0 * kappa * epsbar;
        const double tau3[2][2] = {{1, 0}, {0, -1}};
        const double tau1[2][2] = {{0, 1}, {1, 0}};
        for (int f = 0; f < 2; ++f)
            for (int g = 0; g < 2; ++g)
                for (int s = 0; s < 4; ++s)
                    for (int sp = 0; sp < 4; ++sp)
                        for (int a = 0; a < 3; ++a) {
                            cplx v = IU * nub * GAM[4][s][sp] * tau3[f][g];
                            if (s == sp) v -= ept * tau1[f][g];
                            B[(12 * f + 3 * s + a) * n + 12 * g + 3 * sp + a] += v;
                        }
    }
}

/* out(x) = B(x) in(x) on sites of the given parity (or all, -1); zero elsewhere
 * when zero_other is set. */
static void apply_diag(const int *L, const cplx *T, double kappa, double mu, double mubar, double epsbar, int nf,
                       const cplx *in, cplx *out, int parity)
{
    const long V = vol4(L);
    const int n = 12 * nf;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        cplx *o = out + i * n;
        if (parity >= 0 && parityof(x) != parity) {
            for (int k = 0; k < n; ++k) o[k] = 0;
            continue;
        }
        cplx B[576];
        site_block(T + i * 144, kappa, mu, mubar, epsbar, nf, B);
        for (int r = 0; r < n; ++r) {
            cplx s = 0;
            for (int c = 0; c < n; ++c) s += B[r * n + c] * in[i * n + c];
            o[r] = s;
        }
    }
}

/* out(x) = B(x)^{-1} in(x) on sites of the given parity, zero elsewhere. */
static int solve_diag(const int *L, const cplx *T, double kappa, double mu, double mubar, double epsbar, int nf,
                      const cplx *in, cplx *out, int parity)
{
    const long V = vol4(L);
    const int n = 12 * nf;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        cplx *o = out + i * n;
        if (parity >= 0 && parityof(x) != parity) {
            for (int k = 0; k < n; ++k) o[k] = 0;
            continue;
        }
        cplx B[576];
        site_block(T + i * 144, kappa, mu, mubar, epsbar, nf, B);
        for (int k = 0; k < n; ++k) o[k] = in[i * n + k];
        bad |= gauss_solve(B, o, n);
    }
    return bad;
}

/* export: dense site block at lex site i (for tests) */
void orc_site_block(const cplx *T, long i, double kappa, double mu, double mubar, double epsbar, int nf, cplx *B)
{
    init_gammas();
    site_block(T + i * 144, kappa, mu, mubar, epsbar, nf, B);
}

/* ------------------------------------------------------------------ */
/* full-lattice operator D                                              */
/* ------------------------------------------------------------------ */

/* Full Wilson twisted-mass clover operator (equation for Q^{+-} without
 * the leading gamma5; nf = 2 is the two-flavour operator of the equation
 * for Q-hat_h before preconditioning):
 *   out = B(x) in(x) - kappa (H in)(x) */
void orc_apply_D(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
                 double epsbar, int nf, const cplx *in, cplx *out)
{
    init_gammas();
    const long V = vol4(L);
    const long n = 12L * nf * V;
    cplx *h = malloc(sizeof(cplx) * n);
    orc_hop(L, t_bc, U, in, h, nf, -1);
    apply_diag(L, T, kappa, mu, mubar, epsbar, nf, in, out, -1);
    for (long k = 0; k < n; ++k) out[k] -= kappa * h[k];
    free(h);
}

/* ------------------------------------------------------------------ */
/* even-odd Schur complement (equations for Q-hat^{+-} and Q-hat_h)     */
/* ------------------------------------------------------------------ */

static void cb_to_full(const int *L, const cplx *cb, cplx *full, int n, int parity)
{
    const long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        if (parityof(x) == parity)
            memcpy(full + i * n, cb + (i / 2) * n, sizeof(cplx) * n);
        else
            for (int k = 0; k < n; ++k) full[i * n + k] = 0;
    }
}

static void full_to_cb(const int *L, const cplx *full, cplx *cb, int n, int parity)
{
    const long V = vol4(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        int x[4];
        coords(i, L, x);
        if (parityof(x) == parity) memcpy(cb + (i / 2) * n, full + i * n, sizeof(cplx) * n);
    }
}

/* Mhat on odd vectors:
 *   Mhat = M_oo - M_oe M_ee^{-1} M_eo,  M_eo = -kappa H_eo, M_oe = -kappa H_oe,
 *   M_ee/oo = the site block B (with +mu, or -mu when sgn = -1).
 * nf = 1: the bracket of the Q-hat^{+-} equation (sign of i mu gamma5 =
 * sgn); nf = 2: the bracket of the Q-hat_h equation (sgn flips mubar).
 * Returns nonzero if a site block was singular. */
int orc_mhat(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
             double epsbar, int nf, int sgn, const cplx *in_o, cplx *out_o)
{
    init_gammas();
    const long V = vol4(L);
    const int n = 12 * nf;
    const double m = sgn * mu, mb = sgn * mubar;
    cplx *f = malloc(sizeof(cplx) * n * V);
    cplx *g = malloc(sizeof(cplx) * n * V);
    cplx *h = malloc(sizeof(cplx) * n * V);
    cb_to_full(L, in_o, f, n, 1);
    orc_hop(L, t_bc, U, f, g, nf, 0);                          /* g_e = H_eo psi_o */
    int bad = solve_diag(L, T, kappa, m, mb, epsbar, nf, g, h, 0); /* h_e = B_ee^{-1} g_e */
    orc_hop(L, t_bc, U, h, g, nf, 1);                          /* g_o = H_oe h_e */
    apply_diag(L, T, kappa, m, mb, epsbar, nf, f, h, 1);       /* h_o = B_oo psi_o */
    for (long k = 0; k < (long)n * V; ++k) h[k] -= kappa * kappa * g[k];
    full_to_cb(L, h, out_o, n, 1);
    free(f);
    free(g);
    free(h);
    return bad;
}

static void gamma5_cb(const int *L, const cplx *in, cplx *out, int nf)
{
    const long Vh = vol4(L) / 2;
    const int n = 12 * nf;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < Vh; ++i)
        for (int f = 0; f < nf; ++f)
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = 0;
                    for (int t = 0; t < 4; ++t) acc += GAM[4][s][t] * in[i * n + 12 * f + 3 * t + a];
                    out[i * n + 12 * f + 3 * s + a] = acc;
                }
}

/* Mhat^dagger, written through the gamma5-hermiticity of the operator:
 * Mhat(sgn)^dagger = gamma5 Mhat(-sgn) gamma5 (tests pin this against the
 * inner-product definition of the adjoint). */
int orc_mhat_dag(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
                 double epsbar, int nf, int sgn, const cplx *in_o, cplx *out_o)
{
    init_gammas();
    const long n = 12L * nf * vol4(L) / 2;
    cplx *a = malloc(sizeof(cplx) * n);
    cplx *b = malloc(sizeof(cplx) * n);
    gamma5_cb(L, in_o, a, nf);
    int bad = orc_mhat(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, -sgn, a, b);
    gamma5_cb(L, b, out_o, nf);
    free(a);
    free(b);
    return bad;
}

/* Normal operator N = Mhat^dagger Mhat (+ shift) on odd vectors. */
int orc_mdagm(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
              double epsbar, int nf, int sgn, double shift, const cplx *in_o, cplx *out_o)
{
    const long n = 12L * nf * vol4(L) / 2;
    cplx *a = malloc(sizeof(cplx) * n);
    int bad = orc_mhat(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, in_o, a);
    bad |= orc_mhat_dag(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, a, out_o);
    if (shift != 0.0)
        for (long k = 0; k < n; ++k) out_o[k] += shift * in_o[k];
    free(a);
    return bad;
}

/* ------------------------------------------------------------------ */
/* conjugate gradient on N + shift (the plain solver)                   */
/* ------------------------------------------------------------------ */

static double dotr(const cplx *a, const cplx *b, long n) /* Re <a,b> */
{
    double s = 0;
    for (long k = 0; k < n; ++k) s += creal(conj(a[k]) * b[k]);
    return s;
}

/* Textbook Hestenes-Stiefel CG for (Mhat^dagger Mhat + shift) x = b,
 * starting from x = 0, stopping when the recursive residual satisfies
 * |r| <= tol |b|.  Returns the iteration count (negative if maxiter was
 * reached); *relres receives the true residual |b - (N+shift) x| / |b|. */
int orc_cg(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
           double epsbar, int nf, int sgn, double shift, const cplx *b, cplx *x, double tol, int maxiter,
           double *relres)
{
    const long n = 12L * nf * vol4(L) / 2;
    cplx *r = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n);
    for (long k = 0; k < n; ++k) {
        x[k] = 0;
        r[k] = b[k];
        p[k] = b[k];
    }
    const double bb = dotr(b, b, n);
    double rr = bb;
    int it = 0, done = (bb == 0.0);
    while (!done && it < maxiter) {
        orc_mdagm(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, shift, p, q);
        const double alpha = rr / dotr(p, q, n);
        for (long k = 0; k < n; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
        }
        const double rr1 = dotr(r, r, n);
        ++it;
        if (sqrt(rr1) <= tol * sqrt(bb)) done = 1;
        const double beta = rr1 / rr;
        for (long k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        rr = rr1;
    }
    orc_mdagm(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, shift, x, q);
    double e = 0;
    for (long k = 0; k < n; ++k) {
        cplx d = b[k] - q[k];
        e += creal(conj(d) * d);
    }
    if (relres) *relres = (bb == 0.0) ? 0.0 : sqrt(e / bb);
    free(r);
    free(p);
    free(q);
    return done ? it : -it;
}

/* True relative residual |b - (N + shift) x| / |b| with the oracle operator. */
double orc_residual(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu, double mubar,
                    double epsbar, int nf, int sgn, double shift, const cplx *b, const cplx *x)
{
    const long n = 12L * nf * vol4(L) / 2;
    cplx *q = malloc(sizeof(cplx) * n);
    orc_mdagm(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, shift, x, q);
    double e = 0, bb = 0;
    for (long k = 0; k < n; ++k) {
        cplx d = b[k] - q[k];
        e += creal(conj(d) * d);
        bb += creal(conj(b[k]) * b[k]);
    }
    free(q);
    return bb == 0.0 ? sqrt(e) : sqrt(e / bb);
}

/* True relative residual of an Mhat system: |b - Mhat x| / |b|. */
double orc_residual_mhat(const int *L, int t_bc, const cplx *U, const cplx *T, double kappa, double mu,
                         double mubar, double epsbar, int nf, int sgn, int dagger, const cplx *b, const cplx *x)
{
    const long n = 12L * nf * vol4(L) / 2;
    cplx *q = malloc(sizeof(cplx) * n);
    if (dagger)
        orc_mhat_dag(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, x, q);
    else
        orc_mhat(L, t_bc, U, T, kappa, mu, mubar, epsbar, nf, sgn, x, q);
    double e = 0, bb = 0;
    for (long k = 0; k < n; ++k) {
        cplx d = b[k] - q[k];
        e += creal(conj(d) * d);
        bb += creal(conj(b[k]) * b[k]);
    }
    free(q);
    return bb == 0.0 ? sqrt(e) : sqrt(e / bb);
}
