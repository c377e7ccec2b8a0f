/*
 * tmx -- even-odd preconditioned Wilson twisted-mass clover operator and its
 * solvers on AMD MI355X (gfx950).  Plain C ABI.
 *
 * Operators (Section 2 of arXiv:2212.06635, "Even-odd and mass-preconditioned
 * Dirac operators"):
 *
 *   full operator   D     = 1 + T + i nu gamma5 - kappa H,   nu = 2 kappa mu
 *                   (the M_clov + i mu gamma5 inside Q^{+-} = gamma5 D(+-mu),
 *                   hopping normalisation)
 *   two flavours    D_h   = (1 + T) + i nubar gamma5 tau3 - epst tau1 - kappa H,
 *                   nubar = 2 kappa mubar, epst = 2 kappa epsbar
 *   Schur (odd)     Mhat  = A_oo - kappa^2 H_oe A_ee^{-1} H_eo
 *                   (the bracket of the Q-hat^{+-} and Q-hat_h equations, with
 *                   asymmetric odd-odd preconditioning; Q-hat = gamma5 Mhat)
 *   normal          N     = Mhat^dagger Mhat = gamma5 Mhat(-mu) gamma5 Mhat(mu)
 *
 * H is the Wilson hopping term
 *   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)
 * with periodic x,y,z and a factor t_bc on hops across the time boundary;
 * T = i kappa csw sum_{mu<nu} sigma_{mu nu} F_{mu nu} is the clover term with
 * the four-leaf field strength F = (Q - Q^+)/8.  The gamma matrices are in a
 * chiral basis (gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]],
 * gamma5 = diag(1,1,-1,-1)); callers that use another basis convert at the
 * boundary.
 *
 * Canonical (host-facing) layouts, all complex128 = two doubles (re, im):
 *   links      [t][z][y][x][mu 4][row 3][col 3]
 *   full spinor[t][z][y][x][flavour nf][spin 4][colour 3]
 *   odd spinor [cb][flavour][spin][colour] over the odd sites, cb = lex/2,
 *              lex = x + Lx*(y + Ly*(z + Lz*t)), parity = (x+y+z+t) mod 2.
 * Internal layouts (what the apply calls take) are opaque, precision-typed
 * device buffers of tmx_field_bytes() bytes; tmx_pack / tmx_unpack convert.
 *
 * Errors: 0 = TMX_OK; negative = error (the call had no effect on its
 * outputs; tmx_last_error() describes it); TMX_ENOCONV (+1) = a solver hit
 * maxiter or stagnated: x holds its best iterate and info the residual.
 * Nothing aborts or exits.  A context is not thread-safe.  Applies and
 * pack/unpack are asynchronous on the context's stream; solves synchronise
 * (the host takes the convergence decisions).
 */
#ifndef TMX_H
#define TMX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmx_ctx tmx_ctx;

enum {
    TMX_OK = 0,
    TMX_ENOCONV = 1,
    TMX_EINVAL = -1,
    TMX_ENOTLOADED = -2,
    TMX_ENOMEM = -3,
    TMX_EHIP = -4
};

/* storage / arithmetic precision of an apply.  F16 stores IEEE binary16
 * with one FP32 scale per site and computes in FP32. */
enum { TMX_F64 = 0, TMX_F32 = 1, TMX_F16 = 2 };

/* operator selector: degenerate with +mu / -mu, the two-flavour operator, or
 * the mass-preconditioned What^pm(rho) = Qhat^pm pm i rho~ of Section 2 (eq.
 * for W^pm), Qhat^pm = gamma5 Mhat(pm mu), rho~ = 2 kappa rho with rho from
 * tmx_params.  For the W operators tmx_apply_mhat applies What^pm (its adjoint
 * What^-+ with dagger = 1), tmx_apply_mdagm and the CG solvers use
 * (What^pm)^dagger What^pm = What^-+ What^pm; the product is applied as such
 * (the paper's identity What^+ What^- = Qhat^+ Qhat^- + 2 mu rho + rho^2 holds
 * only for the unpreconditioned operator).  Not defined for tmx_apply_D, the
 * learned preconditioner or the autotuner. */
enum { TMX_OP_PLUS = 1, TMX_OP_MINUS = -1, TMX_OP_ND = 2, TMX_OP_WPLUS = 3, TMX_OP_WMINUS = -3 };

/* field kinds for tmx_field_bytes / tmx_pack / tmx_unpack */
enum {
    TMX_FIELD_ODD = 0,  /* one-flavour odd-site spinor */
    TMX_FIELD_ODD_ND = 1,  /* two-flavour odd-site spinor */
    TMX_FIELD_FULL = 2, /* one-flavour full-lattice spinor */
    TMX_FIELD_FULL_ND = 3  /* two-flavour full-lattice spinor */
};

typedef struct {
    double kappa;  /* hopping parameter */
    double csw;    /* clover coefficient */
    double mu;     /* bare light twisted mass (nu = 2 kappa mu) */
    double mubar;  /* two-flavour twisted mass (nubar = 2 kappa mubar) */
    double epsbar; /* two-flavour mass splitting (epst = 2 kappa epsbar) */
    int t_bc;      /* +1 periodic, -1 antiperiodic fermion time boundary */
    double rho;    /* mass-preconditioning mass of TMX_OP_WPLUS / WMINUS, in the
                      normalisation of mu (the operator gets rho~ = 2 kappa rho);
                      the site-block inverses do not depend on it */
} tmx_params;

/* solver kinds */
enum {
    TMX_SOLVER_CG = 0,      /* plain FP64 CG on N */
    TMX_SOLVER_MPCG_F32 = 1,/* CG with FP32 inner iterations, FP64 reliable updates */
    TMX_SOLVER_MPCG_F16 = 2,/* CG with FP16-storage inner iterations, FP64 reliable updates */
    TMX_SOLVER_FGCR_NN = 3, /* two flexible-GCR solves (Mhat^dagger with K^dagger, Mhat with K), restarted;
                               CG acceptance and fallback */
    TMX_SOLVER_PCG_NN = 4,  /* flexible CG on N preconditioned by K K^dagger (learned network), inner
                               precision cfg->inner_prec (F32 / F16) with FP64 reliable updates */
    TMX_SOLVER_PCG_NN_SYM = 5, /* the same with the Hermitian form P = A^dagger A of the network (one
                                  application per iteration; see tmx_pc_apply) */
    TMX_SOLVER_PCG_NN_SYM1 = 6 /* the same with the short Hermitian form P_1 = L_1^dagger L_1 (the
                                  network's one-channel layers only; tmx_pc_apply mode 3) */
};

typedef struct {
    int kind;           /* TMX_SOLVER_* */
    int op;             /* TMX_OP_PLUS / TMX_OP_MINUS / TMX_OP_ND / TMX_OP_WPLUS / TMX_OP_WMINUS */
    double tol;         /* relative 2-norm of the FP64 true residual, e.g. 1e-10 */
    int maxiter;        /* iteration cap (per stage) */
    double delta;       /* reliable-update trigger (0 => 0.01 FP32, 0.03 FP16 iterations) */
    int restart;        /* FGCR restart length m (0 => 16) */
    int use_initial_guess; /* 1: x holds the start vector on entry */
    double inner_tol;   /* multishift: low-precision stage tolerance (0 => 1e-6 / 5e-4) */
    int inner_prec;     /* multishift / FGCR inner precision TMX_F32 or TMX_F16 (default F32) */
} tmx_solver_cfg;

typedef struct {
    int iters;          /* iterations (operator applications of N or Mhat) */
    int reliable_updates;
    int restarts;       /* FGCR restarts or fallbacks; PCG_NN: network applications (K K^dagger) */
    int fallback;       /* 1 if FGCR or PCG_NN fell back to CG */
    double true_residual; /* |b - A x| / |b| recomputed in FP64 at the end */
    double seconds;     /* wall time of the call */
    double gbytes;      /* model bytes moved by operator applications */
} tmx_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context for an Lx*Ly*Lz*Lt lattice (dims = {Lx,Ly,Lz,Lt}, each
 * even and >= 2, volume <= 2^31).  All device work is enqueued on
 * `hip_stream` (a hipStream_t; NULL = the default stream).  The context owns
 * its device buffers; the caller owns every pointer it passes in. */
int tmx_create(const int dims[4], void *hip_stream, tmx_ctx **out);
int tmx_destroy(tmx_ctx *ctx);
const char *tmx_last_error(const tmx_ctx *ctx);
/* Change the stream subsequent work is enqueued on. */
int tmx_set_stream(tmx_ctx *ctx, void *hip_stream);

/* Device allocator of the context.  Every device buffer the library needs
 * from now on (gauge, clover and inverse fields of every precision, solver
 * and network workspaces, reduction buffers, network state) is obtained as
 * alloc(bytes, user) and given back as release(ptr, user) once the library
 * no longer uses it (the context's stream has been synchronised by then).
 * alloc returns a device pointer aligned to at least 256 bytes, or NULL,
 * which the library turns into TMX_ENOMEM for the call that needed it.
 * Buffers that exist when the hook is set stay with the allocator that made
 * them and are released through it (the reduction buffers, which hold no
 * state between calls, move to the new allocator at once).  alloc = release
 * = NULL restores hipMalloc / hipFree; giving only one of them is
 * TMX_EINVAL.  This lets a framework that owns device memory (a caching
 * allocator, a memory pool) serve the library, so that the library only ever
 * computes on memory it is handed.  The named scratch buffers can also be
 * capped in total with the environment variable TMX_WS_LIMIT (bytes, read by
 * tmx_create): a call that would exceed it returns TMX_ENOMEM before
 * launching anything. */
int tmx_set_allocator(tmx_ctx *ctx, void *(*alloc)(size_t bytes, void *user), void (*release)(void *ptr, void *user),
                      void *user);

/* Memory management (library infrastructure, no passage of the paper).
 * Give every scratch buffer of the context back to its allocator: solver
 * fields, network activations, force and tuning workspaces (TMX_WS_LIMIT
 * counts from zero again).  The gauge field, the clover terms
 * and inverses, the network weights and the reduction buffers stay; later
 * calls allocate again what they need.  For a caller that runs a large solve
 * after others on one context, so that the earlier calls' buffers do not sit
 * beside the new ones (the 64^3x128 multishift solve after CG and the
 * network-preconditioned solve).  Waits for the context's stream first.
 * TMX_EINVAL for a null context. */
int tmx_free_workspaces(tmx_ctx *ctx);

/* Parameters.  Changing mu / mubar / epsbar invalidates only the site-block
 * inverses; changing kappa or csw also invalidates the clover term. */
int tmx_set_params(tmx_ctx *ctx, const tmx_params *p);

/* Upload a gauge field from host memory (canonical layout, complex128,
 * copied; the caller keeps ownership).  `gauge_id` labels the field (its
 * position along a trajectory or a configuration number, as the gauge-state
 * tracking of Section 3 does, with the clover term and its inverse following
 * the gauge field's id): a call with the id already loaded is a no-op;
 * a new id invalidates the clover term and its inverses, which are rebuilt
 * lazily on the next use.  Links must be SU(3) (rows 0,1 are stored, row 2
 * is reconstructed as conj(row0 x row1)). */
int tmx_load_gauge(tmx_ctx *ctx, const double *host_links, double gauge_id);
/* Number of host->device gauge uploads performed so far (state tracking). */
int tmx_gauge_uploads(const tmx_ctx *ctx);

/* Clover term T.  host_T == NULL: build it on the device from the links.
 * Otherwise host_T is [lex][chirality 2][6][6] complex128 Hermitian blocks
 * (row/col index = 3*(spin mod 2) + colour within the chirality block);
 * non-Hermitian input (> 1e-12) returns TMX_EINVAL. */
int tmx_load_clover(tmx_ctx *ctx, const double *host_T);
/* Copy the device clover term back as [lex][2][6][6] complex128 (host). */
int tmx_get_clover(tmx_ctx *ctx, double *host_T);

/* ---- layout conversion ------------------------------------------------- */

/* Bytes of one internal field of `kind` in precision `prec`. */
int tmx_field_bytes(const tmx_ctx *ctx, int kind, int prec, size_t *bytes);
/* canonical (device, complex128) -> internal (device, prec); nvec fields,
 * each contiguous at a stride of one field. */
int tmx_pack(tmx_ctx *ctx, void *internal, const double *canonical, int kind, int prec, int nvec);
int tmx_unpack(tmx_ctx *ctx, double *canonical, const void *internal, int kind, int prec, int nvec);

/* ---- operators (device buffers, internal layout, asynchronous) -------- */

/* out = D in (full lattice): the operator M_clov + i mu gamma5 inside
 * Q^{+-} = gamma5 (M_clov +- i mu gamma5) of Section 2 (equation for Q^{+-};
 * D(-mu)^dagger = gamma5 D(mu) gamma5), or its two-flavour form from the
 * equation for Q-hat_h.  op selects +mu, -mu or the two-flavour operator;
 * fields are TMX_FIELD_FULL (or _FULL_ND for op = TMX_OP_ND), device buffers
 * owned by the caller; out and in must differ (TMX_EINVAL). */
int tmx_apply_D(tmx_ctx *ctx, void *out, const void *in, int op, int prec);
/* out = Mhat in or Mhat^dagger in on odd fields: the bracket of the
 * asymmetric even-odd operator Q-hat^{+-} = gamma5 Mhat(+-mu) of Section 2
 * (equation for Q-hat^{+-}; two-flavour: equation for Q-hat_h; W operators:
 * equation for W^{+-}), nrhs <= 32 fields side by side in the multi-vector
 * layout of tmx_pack with nvec = nrhs; device buffers owned by the caller,
 * out != in (TMX_EINVAL); TMX_ENOTLOADED without a gauge field or
 * parameters. */
int tmx_apply_mhat(tmx_ctx *ctx, void *out, const void *in, int op, int prec, int dagger, int nrhs);
/* tmx_apply_mhat without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result (bit for bit) and errors as
 * tmx_apply_mhat; the even-site intermediate field lives in a static device
 * scratch of 256 MiB that the library holds on every GPU it runs on until
 * the process ends (its address is resolved by tmx_create, once per device).
 * Limits: the intermediate, tmx_field_bytes(TMX_FIELD_ODD or _ODD_ND, prec)
 * times nrhs, must fit the 256 MiB (one right-hand side at 32^3x64 in every
 * precision of the one-flavour operator, and in FP32 / FP16 of the
 * two-flavour one), else TMX_EINVAL; the links, clover and site-block
 * inverses of this precision and sector must already be resident (any
 * tmx_apply_mhat in them builds them), else TMX_ENOTLOADED.  Every call on
 * one GPU shares that scratch, which keeps the last call's contents
 * (nothing in it needs clearing: each call overwrites what it reads): calls
 * that overlap on one GPU -- other streams, other contexts, other threads --
 * race and must be serialised by the caller. */
int tmx_apply_mhat_noalloc(tmx_ctx *ctx, void *out, const void *in, int op, int prec, int dagger, int nrhs);
/* out = N in = Mhat^dagger Mhat in, the Hermitian positive operator whose
 * solves the monomials need (Section 2: Q-hat^+ Q-hat^- = Mhat(-)^dagger
 * Mhat(-)); same arguments and errors as tmx_apply_mhat. */
int tmx_apply_mdagm(tmx_ctx *ctx, void *out, const void *in, int op, int prec, int nrhs);

/* Hopping-term force (the link derivative that the fermion force of the
 * rational monomials sums over the shifts, Section 4.3): for odd fields x, y
 * (device, canonical complex128) and S = Re<y, Mhat(op) x> with the clover
 * and twist blocks held fixed, the derivative along U_mu(z) -> exp(i eps T)
 * U_mu(z) (T Hermitian traceless) is Re Tr[i T F_mu(z)], F the traceless
 * anti-Hermitian 3x3 matrix written to force[((lex * 4 + mu) * 3 + i) * 3 + j]
 * (complex128, the canonical link layout of tmx_load_gauge).  force =
 * coeff F, or force += coeff F with accumulate = 1 (summing over shifts).
 * op: TMX_OP_PLUS, TMX_OP_MINUS, or TMX_OP_ND for the two-flavour operator
 * of eq. Q-hat_h (x, y two-flavour odd fields; the hopping term is flavour
 * diagonal, so the outer products are summed over the flavours, with the
 * flavour-mixing site blocks inside the even-site fields).  Enqueued on the
 * context stream. */
int tmx_hop_force(tmx_ctx *ctx, double *force, const double *x, const double *y, int op, double coeff,
                  int accumulate);
/* Clover-term force (Section 4.3, the clover term of Section 2): the same
 * derivative of S = Re<y, Mhat(op) x> taken through the clover term
 * T = i kappa csw sum_{mu<nu} sigma_mu,nu F_mu,nu (F the four-leaf field
 * strength) of both parities, in A_oo and inside A_ee^{-1}, with the hopping
 * matrices held fixed.  Same arguments, layout and accumulation as
 * tmx_hop_force; the full link derivative of S is the sum of the two.
 * TMX_EINVAL if the clover term was loaded with tmx_load_clover (the force
 * needs it built from the links).  Uses 2400 Vh bytes of workspace (the
 * insertions, 864 Vh, and the plaquette loops, 1536 Vh) besides the two
 * even-site fields it shares with tmx_hop_force. */
int tmx_clover_force(tmx_ctx *ctx, double *force, const double *x, const double *y, int op, double coeff,
                     int accumulate);

/* ---- solvers (device buffers, canonical complex128 odd fields) -------- */

/* Solve N x = b (cfg->op selects the operator) for nrhs <= 32 right-hand
 * sides stored contiguously (device, canonical complex128 odd fields, owned
 * by the caller; x also holds the start vector if cfg->use_initial_guess):
 * CG, or the mixed-precision CG with FP64 reliable updates of Sections 1 and
 * 4.1, or the solves preconditioned by the learned network (standing in for
 * the multigrid preconditioner of Section 4.1).  info is an array of nrhs
 * entries (may be NULL).  Each column is solved for b / |b| and the
 * solution scaled back, so any source scale works in every precision.
 * Returns TMX_ENOCONV if any column missed cfg->tol (x then holds the best
 * iterate), TMX_ENOMEM if a workspace could not be allocated (nothing
 * launched), TMX_EINVAL for a source with a NaN or infinite entry (x left as
 * it was). */
int tmx_solve(tmx_ctx *ctx, double *x, const double *b, int nrhs, const tmx_solver_cfg *cfg, tmx_info *info);
/* Solve Mhat x = b (dagger = 0) or Mhat^dagger x = b (dagger = 1), the two
 * inversions of the fermion derivative (Section 4.1), through the normal
 * equations: x = N^{-1} Mhat^dagger b, or x = Mhat N^{-1} b.  One odd field
 * each (device, canonical complex128); errors as tmx_solve. */
int tmx_solve_mhat(tmx_ctx *ctx, double *x, const double *b, int dagger, const tmx_solver_cfg *cfg,
                   tmx_info *info);
/* Solve (N + shifts[k]) x_k = b for k < nshift (<= 32), shifts > 0 or >= 0
 * with shifts[0] the smallest: the mixed-precision multishift solver of the
 * heavy sector (Section 4.2: a low-precision multishift CG, then
 * shift-by-shift refinement).  x is nshift contiguous odd fields.  Low
 * precision multishift CG followed by FP64-reliable refinement per shift
 * (cfg->inner_prec selects F32 or F16 for both stages; TMX_F64 runs the
 * plain FP64 multishift CG).  With cfg->kind = TMX_SOLVER_PCG_NN each
 * shift's refinement is the CG preconditioned by the learned network (set by
 * tmx_pc_set_weights or tmx_pc_train; degenerate op only, TMX_EINVAL
 * otherwise), falling back to mixed-precision CG if it stalls (info fallback
 * = 1); info restarts then counts the network applications.  The source is
 * normalized and the solutions scaled back as in tmx_solve; TMX_EINVAL for a
 * non-finite source. */
int tmx_multishift_solve(tmx_ctx *ctx, double *x, const double *b, const double *shifts, int nshift,
                         const tmx_solver_cfg *cfg, tmx_info *info);
/* Rational function of the normal operator, the partial-fraction form of the
 * rational approximation (Section 4.2):
 *     out = a0 b + sum_{k < nshift} coeffs[k] (N + shifts[k])^{-1} b,
 * N of cfg->op (TMX_OP_ND for the heavy sector).  The solves are those of
 * tmx_multishift_solve (same cfg fields, shifts ascending, nshift <= 32,
 * per-shift accuracy cfg->tol) and the sum is accumulated on the device as
 * each shift's solution is refined; b and out are one odd field each (host
 * arrays coeffs / shifts of nshift doubles, copied).  info has nshift entries
 * (may be NULL).  With the Zolotarev coefficients of x^(-1/2) this applies
 * N^(-1/2) to the relative accuracy of the approximation. */
int tmx_rational_apply(tmx_ctx *ctx, double *out, const double *b, double a0, const double *coeffs,
                       const double *shifts, int nshift, const tmx_solver_cfg *cfg, tmx_info *info);
/* Fermion force of a rational monomial (Sections 4.2 and 4.3: the link
 * derivative that the heavy-sector monomials sum over the shifts of the
 * multishift solve): for S_R = <phi, R(N) phi> with R(N) = a0 + sum_k
 * coeffs[k] (N + shifts[k])^{-1} and x_k = (N + shifts[k])^{-1} phi,
 *     dS_R = -sum_k coeffs[k] <x_k, dN x_k> = Re Tr[i T F_R],
 *     F_R = -2 sum_k coeffs[k] (hop + clover force)(x_k, Mhat x_k)
 * for U_mu(x) -> exp(i eps T) U_mu(x), in the layout and convention of
 * tmx_hop_force (a0 does not enter).  The x_k come from the solves of
 * tmx_multishift_solve (same cfg fields; cfg->op TMX_OP_ND for the heavy
 * sector, TMX_OP_PLUS / MINUS for the degenerate one) and each shift's force
 * is added on the device as soon as its solution is refined.  phi: one odd
 * field (device, canonical); force: V*36 complex128 (device), written
 * (accumulate = 0) or added to.  info has nshift entries (may be NULL).
 * TMX_EINVAL with a host-loaded clover term; TMX_ENOCONV if a shift missed
 * cfg->tol (the force is still complete). */
int tmx_rational_force(tmx_ctx *ctx, double *force, const double *phi, const double *coeffs, const double *shifts,
                       int nshift, const tmx_solver_cfg *cfg, int accumulate, tmx_info *info);
/* Correction term of a rational approximation R(N) ~ N^(-1/2) (Section 4.2;
 * the error of the approximation enters the acceptance step): with
 * Z = N R(N)^2 - 1, det(N)^(1/2) = det(R)^(-1) det(1 + Z)^(1/2), and for a
 * Gaussian eta (density exp(-eta^dagger eta)) det(1 + Z)^(1/2) is the mean of
 * exp(-E) with
 *     E = eta^dagger [(1 + Z)^(-1/2) - 1] eta = sum_{k>=1} binom(-1/2, k) <eta, Z^k eta>.
 * Sums the series until a term is below tol * |E| or maxterms terms; each
 * term applies R twice (as tmx_rational_apply) and N once, all on the device.
 * eta: one odd field (device, canonical); *exponent receives E (real part),
 * *terms (may be NULL) the number of terms.  Returns TMX_ENOCONV (with the
 * partial sum in *exponent) if a solve missed cfg->tol or the series had not
 * reached tol after maxterms terms. */
int tmx_rational_correction(tmx_ctx *ctx, const double *eta, double a0, const double *coeffs, const double *shifts,
                            int nshift, double tol, int maxterms, const tmx_solver_cfg *cfg, double *exponent,
                            int *terms);

/* ---- learned preconditioner ------------------------------------------- */

/* Number of real FP32 parameters of the network (4 layers x 9 paths x
 * (channel matrix + 4x4 spin matrix), complex). */
int tmx_pc_num_params(const tmx_ctx *ctx, size_t *n);
int tmx_pc_set_weights(tmx_ctx *ctx, const float *host_w, size_t n);
int tmx_pc_get_weights(tmx_ctx *ctx, float *host_w, size_t n);
/* out = K in (dagger = 0), K^dagger in (dagger = 1), the Hermitian form
 * P in (dagger = 2) or the short Hermitian form P_1 in (dagger = 3) on
 * canonical odd complex128 device fields.  P = A^dagger A with A = L_2 L_1
 * the network's first two layers (the last two are not used): four stencil
 * layers applied, Hermitian and positive semi-definite by construction, so
 * that one application preconditions CG on N (where K K^dagger takes two);
 * trained with TMX_LOSS_SYM on pairs (b, N^{-1} b).  P_1 = L_1^dagger L_1
 * uses the first layer alone (two one-channel layers, about a third of P's
 * cost); trained with TMX_LOSS_SYM1.  Other values of dagger: TMX_EINVAL. */
int tmx_pc_apply(tmx_ctx *ctx, double *out, const double *in, int dagger);

/* Training loss (loss_kind as in tmx_train_cfg, Mhat of op: TMX_OP_PLUS or
 * TMX_OP_MINUS) over npairs canonical odd device fields and its gradient with
 * respect to the weights (host_grad may be NULL), as used by one training
 * step. */
int tmx_pc_loss_grad(tmx_ctx *ctx, const double *b, const double *x, int npairs, int loss_kind, int op,
                     double *loss, float *host_grad);

typedef struct {
    int epochs;
    int batch;
    float lr;
    float beta1, beta2, eps;
    int seed;
    int loss_kind; /* TMX_LOSS_* (default TMX_LOSS_RESIDUAL) */
    int op;        /* operator the network is trained for: TMX_OP_PLUS (0 = default) or
                      TMX_OP_MINUS (separately trained weights for the Mhat(-mu) solves) */
} tmx_train_cfg;

/* training losses over pairs (b_i, x_i = Mhat^{-1} b_i):
 *   residual: mean_i |Mhat (K b_i - x_i)|^2 / |b_i|^2  = |Mhat K b_i - b_i|^2 / |b_i|^2
 *   solution: mean_i |K b_i - x_i|^2 / |x_i|^2
 * The residual loss controls E = Mhat K - 1 on all modes, which is what a
 * preconditioner needs; the solution loss weights the high modes of Mhat
 * down by Mhat^{-1}. */
enum { TMX_LOSS_RESIDUAL = 0, TMX_LOSS_SOLUTION = 1, TMX_LOSS_SYM = 2, TMX_LOSS_SYM1 = 3 };
/* TMX_LOSS_SYM trains the Hermitian form P (layers 1 and 2) on pairs
 * (b_i, x_i = N^{-1} b_i) with the energy norm of its error,
 *   mean_i <P b_i - x_i, N (P b_i - x_i)> / |b_i|^2 = mean_i |Mhat (P b_i - x_i)|^2 / |b_i|^2,
 * the quantity CG on N minimises; the gradients of layers 3 and 4 are zero.
 * TMX_LOSS_SYM1: the same loss for the short form P_1 (layer 1 only; the
 * gradients of layers 2 to 4 are zero). */

/* One Adam step (Kingma and Ba, with bias correction) on the network weights
 * from a gradient the caller supplies: host_grad holds n FP32 values in the
 * layout of tmx_pc_set_weights (n = tmx_pc_num_params), for instance the
 * gradient of tmx_pc_loss_grad averaged over the batches of several GPUs in
 * data-parallel training.  With t the steps taken since the weights were last
 * set (the moments m, v start at zero then):
 *     m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *     w = w - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * elementwise in FP32.  cfg supplies lr, beta1, beta2, eps (0 selects 1e-3,
 * 0.9, 0.999, 1e-8); its other fields are ignored.  tmx_pc_train takes the
 * same step after each batch.  TMX_EINVAL for a wrong n or non-finite
 * values, TMX_ENOTLOADED before weights are set.  Synchronises. */
int tmx_pc_adam_step(tmx_ctx *ctx, const float *host_grad, size_t n, const tmx_train_cfg *cfg);

/* Train on npairs (b_i, x_i) canonical odd complex128 device fields with
 * the loss selected by cfg->loss_kind and Adam; loss_out[epochs] receives
 * the mean loss of each epoch (host). */
int tmx_pc_train(tmx_ctx *ctx, const double *b, const double *x, int npairs, const tmx_train_cfg *cfg,
                 float *loss_out);

/* ---- autotuner ------------------------------------------------------------ */

/* Time the launch shapes of the two stencil kernels of Mhat for precision
 * prec, operator op and nrhs right-hand sides on this lattice, and keep the
 * fastest for later applies (the operator's kernels, not a model of them;
 * every shape computes each output slot in one thread, so results do not
 * depend on the choice).  Knobs: workgroup size 64 / 128 / 256, plain or
 * XCD-contiguous block order, one or two sites per thread (one right-hand
 * side), and for nrhs > 1 the group size rg (a divisor of nrhs: the operator
 * then runs K1 and K2 on rg right-hand sides at a time, which keeps a group's
 * neighbour spinors within L2), K1 and K2 sharing it.  The internal site
 * order ((z, t) tiles of the planes) is fixed per context by the environment
 * variables TMX_SITE_ZB / TMX_SITE_TB, since the field layout depends on it.
 * If the environment variable TMX_TUNE_CACHE names a file, results are
 * appended there and loaded by tmx_create for the same lattice; with
 * TMX_TUNE_LOG set every timed shape is printed to stderr.  Synchronises. */
int tmx_tune(tmx_ctx *ctx, int prec, int op, int nrhs);
/* Launch shape in use for a kernel key ("K1_f64", "K2_f32_nd_r12", ...):
 * workgroup size, XCD order, sites per thread and right-hand-side group
 * size (0 = all); any pointer may be NULL.  TMX_OK if it was tuned,
 * TMX_ENOCONV if it is the default. */
int tmx_tuned_config(tmx_ctx *ctx, const char *key, int *block, int *xcd, int *spt, int *rg);

/* ---- kernel timing -------------------------------------------------------- */

/* Bracket every stencil kernel launch with HIP events on the context's
 * stream (on != 0) and clear the accumulated statistics; on = 0 stops
 * recording.  Adds one event pair per launch. */
int tmx_kstats_enable(tmx_ctx *ctx, int on);
/* Statistics of kernel idx (0-based, in name order): name ("K1_f64",
 * "K2_f32_nd_r12", ...), launch count and summed duration in ms.
 * Synchronises on the recorded events.  TMX_EINVAL past the last kernel. */
int tmx_kstats_get(tmx_ctx *ctx, int idx, char *name, size_t name_len, long *count, double *total_ms);

/* ---- tracing ------------------------------------------------------------ */

/* Hierarchical timers: push starts a timer at the next level of the call
 * tree with a caller-chosen name; pop stops it and prints
 *   "# TMX: Time for <name> <seconds> s level: <n> <path>"
 * to stdout when tracing is enabled (TMX_TRACE=1 or tmx_trace_enable). */
int tmx_trace_enable(tmx_ctx *ctx, int on);
int tmx_trace_push(tmx_ctx *ctx, const char *name);
int tmx_trace_pop(tmx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TMX_H */
