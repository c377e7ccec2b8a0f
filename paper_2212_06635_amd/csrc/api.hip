// C-ABI entry points, context management and the operator layer.
//
// Gauge-state tracking follows the paper's gauge-id cascade (Section 3):
// a gauge field is identified by a real id; loading the same id again does
// nothing, a new id invalidates every derived field (lower-precision link
// copies, clover term, site inverses), and derived fields are rebuilt lazily
// on the first operation that needs them.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "tmx_ctx.h"
#include "force.h"

using namespace tmx;

namespace tmx {

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int set_err(tmx_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_err(tmx_ctx *c, hipError_t e, const char *where)
{
    if (e == hipSuccess) return TMX_OK;
    return set_err(c, e == hipErrorOutOfMemory ? TMX_ENOMEM : TMX_EHIP,
                   std::string(where) + ": " + hipGetErrorString(e));
}

void *dev_alloc(tmx_ctx *c, size_t bytes)
{
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    AllocRec rec;
    rec.bytes = bytes;
    if (c->alloc_fn) {
        p = c->alloc_fn(bytes, c->alloc_user);
        if (!p) {
            set_err(c, TMX_ENOMEM, "the caller's allocator returned no memory for " + std::to_string(bytes) + " bytes");
            return nullptr;
        }
        rec.release = c->release_fn;
        rec.user = c->alloc_user;
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_err(c, TMX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            return nullptr;
        }
    }
    c->allocs[p] = rec;
    return p;
}

void dev_free(tmx_ctx *c, void *p)
{
    if (!p) return;
    auto it = c->allocs.find(p);
    if (it == c->allocs.end()) return;  // not ours: never released here
    const AllocRec rec = it->second;
    c->allocs.erase(it);
    if (rec.release)
        rec.release(p, rec.user);
    else
        (void)hipFree(p);
}

void *ws_get(tmx_ctx *c, const std::string &name, size_t bytes)
{
    Workspace &w = c->ws[name];
    if (w.bytes >= bytes && w.p) return w.p;
    if (c->ws_limit && c->ws_bytes - w.bytes + bytes > c->ws_limit) {
        set_err(c, TMX_ENOMEM, "workspace '" + name + "' of " + std::to_string(bytes) +
                                   " bytes exceeds the workspace limit (TMX_WS_LIMIT)");
        return nullptr;
    }
    if (w.p) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, w.p);
        c->ws_bytes -= w.bytes;
        w.p = nullptr;
        w.bytes = 0;
    }
    w.p = dev_alloc(c, bytes);
    if (w.p) {
        w.bytes = bytes;
        c->ws_bytes += bytes;
    }
    return w.p;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free Schur operator (tmx_apply_mhat_noalloc): the
// even-site intermediate u = B_ee^{-1} H_eo in.  One copy per GPU, held until
// the process ends; in host code `scratch` names a host-side stand-in, so
// every use goes through the device address resolved per device below.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static std::map<int, void *> scratch_dev;  // device ordinal -> device address of scratch

// device address of `scratch` on the current device (resolved once per
// device); nullptr with the context's error set if it cannot be resolved
static void *scratch_address(tmx_ctx *c)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, TMX_EHIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    auto it = scratch_dev.find(dev);
    if (it != scratch_dev.end()) return it->second;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        set_err(c, TMX_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return nullptr;
    }
    scratch_dev[dev] = p;
    return p;
}

static size_t red_partials_bytes(const tmx_ctx *c) { return sizeof(double) * c->red.max_blocks * MAXR * 4; }
static size_t red_result_bytes() { return sizeof(double) * MAXR * 4; }

static size_t bytes_per_real(int prec) { return prec == F64 ? 8 : (prec == F32 ? 4 : 2); }

double mhat_bytes_per_site(int prec, int nf, int nrhs)
{
    const double bg = (double)bytes_per_real(prec), bs = bg, bc = bg;
    double spin = 120.0 * bs + (prec == F16 ? 20.0 : 0.0);
    return 192.0 * bg + 216.0 * bc + (double)nrhs * nf * spin;
}

int fetch(tmx_ctx *c, int n, double *host)
{
    hipError_t e = hipSuccess;
    if (!c->red.host)
        e = hipMemcpyAsync(c->host_red, c->red.result, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_err(c, e, "reduction readback");
    std::memcpy(host, c->host_red, sizeof(double) * n);
    return TMX_OK;
}

// ---------------------------------------------------------------------------
// derived fields
// ---------------------------------------------------------------------------
static size_t clover_bytes(int prec, long Vh) { return 144 * bytes_per_real(prec) * Vh; }  // both parities
static size_t inv_bytes(int prec, long Vh) { return 144 * bytes_per_real(prec) * Vh; }     // even sites
static size_t invnd_bytes(int prec, long Vh) { return 72 * bytes_per_real(prec) * Vh; }    // even sites
static size_t link_bytes(int prec, long Vh)
{
    return 8 * (size_t)Vh * (prec == F64 ? 96 : (prec == F32 ? 48 : 24));
}

static int ensure_links(tmx_ctx *c, int prec)
{
    if (!c->gauge_loaded) return set_err(c, TMX_ENOTLOADED, "no gauge field loaded");
    if (c->links_ok[prec]) return TMX_OK;
    if (!c->links[prec]) {
        c->links[prec] = dev_alloc(c, link_bytes(prec, c->Vh));
        if (!c->links[prec]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    }
    int r = hip_err(c, launch_convert_links((const double *)c->links[F64], c->links[prec], prec, c->g, c->stream),
                    "convert links");
    if (r) return r;
    c->links_ok[prec] = true;
    return TMX_OK;
}

static int ensure_clover(tmx_ctx *c, int prec)
{
    if (!c->gauge_loaded) return set_err(c, TMX_ENOTLOADED, "no gauge field loaded");
    if (!c->have_params) return set_err(c, TMX_ENOTLOADED, "parameters not set");
    if (!c->clov_ok[F64]) {
        if (!c->clov[F64]) {
            c->clov[F64] = dev_alloc(c, clover_bytes(F64, c->Vh));
            if (!c->clov[F64]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        int r = hip_err(c, launch_clover_build((const double *)c->links[F64], (double *)c->clov[F64], c->g,
                                               c->par.kappa, c->par.csw, c->stream),
                        "clover build");
        if (r) return r;
        c->clov_ok[F64] = true;
        c->clov_kappa = c->par.kappa;
        c->clov_csw = c->par.csw;
        c->clov_ok[F32] = c->clov_ok[F16] = false;
        c->inv_ok[0] = c->inv_ok[1] = c->inv_ok[2] = false;
        c->invnd_ok[0] = c->invnd_ok[1] = c->invnd_ok[2] = false;
    }
    if (prec != F64 && !c->clov_ok[prec]) {
        if (!c->clov[prec]) {
            c->clov[prec] = dev_alloc(c, clover_bytes(prec, c->Vh));
            if (!c->clov[prec]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        int r = hip_err(c, launch_convert_seq((const double *)c->clov[F64], c->clov[prec], prec, 144, c->Vh, c->stream),
                        "convert clover");
        if (r) return r;
        c->clov_ok[prec] = true;
    }
    return TMX_OK;
}

static int ensure_inv(tmx_ctx *c, int prec)
{
    int r = ensure_clover(c, F64);
    if (r) return r;
    const double nu = 2.0 * c->par.kappa * c->par.mu;
    if (c->inv_ok[F64] && c->inv_nu != nu) c->inv_ok[0] = c->inv_ok[1] = c->inv_ok[2] = false;
    if (!c->inv_ok[F64]) {
        if (!c->inv[F64]) {
            c->inv[F64] = dev_alloc(c, inv_bytes(F64, c->Vh));
            if (!c->inv[F64]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        r = hip_err(c, launch_clover_inv((const double *)c->clov[F64], (double *)c->inv[F64], c->g, nu, c->stream),
                    "clover inverse");
        if (r) return r;
        c->inv_ok[F64] = true;
        c->inv_nu = nu;
        c->inv_ok[F32] = c->inv_ok[F16] = false;
    }
    if (prec != F64 && !c->inv_ok[prec]) {
        if (!c->inv[prec]) {
            c->inv[prec] = dev_alloc(c, inv_bytes(prec, c->Vh));
            if (!c->inv[prec]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        r = hip_err(c, launch_convert_seq((const double *)c->inv[F64], c->inv[prec], prec, 144, c->Vh, c->stream),
                    "convert inverse");
        if (r) return r;
        c->inv_ok[prec] = true;
    }
    return TMX_OK;
}

static int ensure_invnd(tmx_ctx *c, int prec)
{
    int r = ensure_clover(c, F64);
    if (r) return r;
    const double nb = 2.0 * c->par.kappa * c->par.mubar, ep = 2.0 * c->par.kappa * c->par.epsbar;
    const double cc = nb * nb - ep * ep;
    if (c->invnd_ok[F64] && c->invnd_c != cc) c->invnd_ok[0] = c->invnd_ok[1] = c->invnd_ok[2] = false;
    if (!c->invnd_ok[F64]) {
        if (!c->invnd[F64]) {
            c->invnd[F64] = dev_alloc(c, invnd_bytes(F64, c->Vh));
            if (!c->invnd[F64]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        r = hip_err(c, launch_clover_inv_nd((const double *)c->clov[F64], (double *)c->invnd[F64], c->g, nb, ep,
                                            c->stream),
                    "nd clover inverse");
        if (r) return r;
        c->invnd_ok[F64] = true;
        c->invnd_c = cc;
        c->invnd_ok[F32] = c->invnd_ok[F16] = false;
    }
    if (prec != F64 && !c->invnd_ok[prec]) {
        if (!c->invnd[prec]) {
            c->invnd[prec] = dev_alloc(c, invnd_bytes(prec, c->Vh));
            if (!c->invnd[prec]) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
        r = hip_err(c, launch_convert_seq((const double *)c->invnd[F64], c->invnd[prec], prec, 72, c->Vh, c->stream),
                    "convert nd inverse");
        if (r) return r;
        c->invnd_ok[prec] = true;
    }
    return TMX_OK;
}

int ensure_ready(tmx_ctx *c, int prec, bool nd)
{
    if (prec < F64 || prec > F16) return set_err(c, TMX_EINVAL, "bad precision");
    int r = ensure_links(c, prec);
    if (!r) r = ensure_clover(c, prec);
    if (!r) r = nd ? ensure_invnd(c, prec) : ensure_inv(c, prec);
    return r;
}

// ---------------------------------------------------------------------------
// operator layer
// ---------------------------------------------------------------------------
static const void *clov_parity(tmx_ctx *c, int prec, int parity)
{
    return static_cast<const char *>(c->clov[prec]) + (size_t)parity * 72 * bytes_per_real(prec) * c->Vh;
}

LaunchCfg launch_cfg(tmx_ctx *c, const std::string &key)
{
    auto it = c->tune.find(key);
    if (it != c->tune.end()) return it->second;
    LaunchCfg d;
    d.block = c->default_block;
    d.xcd = c->xcd_remap;
    return d;
}

static hipEvent_t kev_get(tmx_ctx *c)
{
    if (!c->kpool.empty()) {
        hipEvent_t e = c->kpool.back();
        c->kpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

static void kstat_collect(tmx_ctx *c)
{
    for (auto &k : c->kpending) {
        float ms = 0.f;
        if (k.a && k.b && hipEventSynchronize(k.b) == hipSuccess && hipEventElapsedTime(&ms, k.a, k.b) == hipSuccess) {
            KStat &st = c->kstats[k.name];
            st.count++;
            st.ms += ms;
        } else {
            (void)hipGetLastError();
        }
        if (k.a) c->kpool.push_back(k.a);
        if (k.b) c->kpool.push_back(k.b);
    }
    c->kpending.clear();
}

void kstat_begin(tmx_ctx *c, const std::string &name)
{
    if (!c->kstats_on) return;
    if (c->kpending.size() > 4096) kstat_collect(c);
    KEvent k{name, kev_get(c), nullptr};
    if (k.a) (void)hipEventRecord(k.a, c->stream);
    c->kpending.push_back(k);
}

void kstat_end(tmx_ctx *c)
{
    if (!c->kstats_on || c->kpending.empty()) return;
    KEvent &k = c->kpending.back();
    k.b = kev_get(c);
    if (k.b) (void)hipEventRecord(k.b, c->stream);
}

static std::string kname(const char *k, int prec, bool nd, int nrhs)
{
    static const char *pn[3] = {"f64", "f32", "f16"};
    std::string s = std::string(k) + "_" + pn[prec] + (nd ? "_nd" : "");
    if (nrhs > 1) s += "_r" + std::to_string(nrhs);
    return s;
}

static DslashArgs base_args(tmx_ctx *c, int prec, bool nd, int nrhs)
{
    DslashArgs a{};
    a.g = c->g;
    a.nrhs = nrhs;
    a.U = LinkPtr{c->links[prec], c->Vh};
    a.nu = nd ? 2.0 * c->par.kappa * c->par.mubar : 2.0 * c->par.kappa * c->par.mu;
    a.epst = nd ? 2.0 * c->par.kappa * c->par.epsbar : 0.0;
    a.t_bc = c->par.t_bc;
    return a;
}

// K1: u = B_ee(sgn)^{-1} H_eo in ; K2: out = B_oo(sgn) x - kappa^2 H_oe u
// (with a right-hand-side group size rg < nrhs from the autotuner: K1 then
// K2 on each group of rg right-hand sides, so that a group's neighbour
// spinors stay in L2 between the two halves)
static int schur_pair(tmx_ctx *c, SpinorPtr out, SpinorPtr in, SpinorPtr u, int prec, bool nd, int nrhs, int sgn,
                      int g5in, int g5out, double *nrm = nullptr, double rho = 0.0)
{
    const int nf = nd ? 2 : 1;
    const std::string k1 = kname("K1", prec, nd, nrhs), k2 = kname("K2", prec, nd, nrhs);
    const LaunchCfg l1 = launch_cfg(c, k1), l2 = launch_cfg(c, k2);
    const int rg = (l1.rg > 0 && l1.rg < nrhs && nrhs % l1.rg == 0) ? l1.rg : nrhs;
    DslashArgs a = base_args(c, prec, nd, nrhs);
    a.sgn = sgn;
    a.parity = 0;
    a.out = u;
    a.in = in;
    a.clov = clov_parity(c, prec, 0);
    a.inv = nd ? c->invnd[prec] : c->inv[prec];
    a.g5in = g5in;
    a.xcd = l1.xcd;
    a.spt = l1.spt;
    DslashArgs b = base_args(c, prec, nd, nrhs);
    b.sgn = sgn;
    b.parity = 1;
    b.out = out;
    b.in = u;
    b.x = in;
    b.clov = clov_parity(c, prec, 1);
    b.kfac = c->par.kappa * c->par.kappa;
    b.g5x = g5in;
    b.g5out = g5out;
    b.nrm = nrm;
    b.rho = rho;
    b.xcd = l2.xcd;
    b.spt = l2.spt;
    for (int r0 = 0; r0 < nrhs; r0 += rg) {
        a.r0 = b.r0 = r0;
        a.rg = b.rg = rg;
        kstat_begin(c, k1);
        hipError_t e = launch_dslash(prec, nf, 0, a, c->stream, l1.block);
        kstat_end(c);
        if (e != hipSuccess) return hip_err(c, e, "K1 launch");
        kstat_begin(c, k2);
        e = launch_dslash(prec, nf, 1, b, c->stream, l2.block);
        kstat_end(c);
        if (e != hipSuccess) return hip_err(c, e, "K2 launch");
    }
    return TMX_OK;
}

static int check_op(tmx_ctx *c, int op)
{
    if (op != TMX_OP_PLUS && op != TMX_OP_MINUS && op != TMX_OP_ND && op != TMX_OP_WPLUS && op != TMX_OP_WMINUS)
        return set_err(c, TMX_EINVAL, "bad op");
    return TMX_OK;
}

// the mass-preconditioned What^pm(rho) = g5 Mhat(pm) pm i rho~ (eq. for W^pm)
static bool op_is_w(int op) { return op == TMX_OP_WPLUS || op == TMX_OP_WMINUS; }
// twist sign of the Schur operator behind op
static int op_sign(int op) { return op == TMX_OP_ND ? 1 : (op > 0 ? 1 : -1); }
// i rho~ coefficient of What^s: s rho~, rho~ = 2 kappa rho
static double w_rho(const tmx_ctx *c, int s) { return s * 2.0 * c->par.kappa * c->par.rho; }

// Mhat (or its adjoint) with the even-site intermediate in u (derived fields ready)
static int mhat_with(tmx_ctx *c, SpinorPtr out, SpinorPtr in, SpinorPtr u, int op, int prec, int dagger, int nrhs)
{
    const bool nd = op == TMX_OP_ND;
    const int sgn = op_sign(op);
    if (op_is_w(op)) {
        // What^s = g5 Mhat(s) + i s rho~ ; its adjoint is What^-s
        const int s = dagger ? -sgn : sgn;
        return schur_pair(c, out, in, u, prec, false, nrhs, s, 0, 1, nullptr, w_rho(c, s));
    }
    // Mhat^dagger = g5 Mhat(-sgn) g5
    return schur_pair(c, out, in, u, prec, nd, nrhs, dagger ? -sgn : sgn, dagger, dagger);
}

int op_mhat(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec, int dagger, int nrhs)
{
    int r = check_op(c, op);
    if (r) return r;
    const bool nd = op == TMX_OP_ND;
    r = ensure_ready(c, prec, nd);
    if (r) return r;
    const int nf = nd ? 2 : 1;
    const long stride = c->Vh * nrhs;
    void *ud = ws_get(c, "op_u" + std::to_string(prec), spinor_field_bytes(prec, nf, stride));
    if (!ud) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    return mhat_with(c, out, in, make_spinor(ud, prec, nf, stride), op, prec, dagger, nrhs);
}

int op_mdagm(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec, int nrhs, double *nrm)
{
    int r = check_op(c, op);
    if (r) return r;
    const bool nd = op == TMX_OP_ND;
    r = ensure_ready(c, prec, nd);
    if (r) return r;
    const int nf = nd ? 2 : 1;
    const long stride = c->Vh * nrhs;
    void *ud = ws_get(c, "op_u" + std::to_string(prec), spinor_field_bytes(prec, nf, stride));
    void *vd = ws_get(c, "op_v" + std::to_string(prec), spinor_field_bytes(prec, nf, stride));
    if (!ud || !vd) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    SpinorPtr u = make_spinor(ud, prec, nf, stride), v = make_spinor(vd, prec, nf, stride);
    const int sgn = op_sign(op);
    // v = g5 Mhat(sgn) in ; out = g5 Mhat(-sgn) v = N in (g5 Mhat(-sgn) g5 is the
    // adjoint of Mhat(sgn)), so <in, N in> = |v|^2 per slot if nrm is given.
    // For What: v = What^sgn in, out = What^-sgn v = (What^sgn)^dagger What^sgn in.
    const bool w = op_is_w(op);
    r = schur_pair(c, v, in, u, prec, nd, nrhs, sgn, 0, 1, nrm, w ? w_rho(c, sgn) : 0.0);
    if (r) return r;
    return schur_pair(c, out, v, u, prec, nd, nrhs, -sgn, 0, 1, nullptr, w ? w_rho(c, -sgn) : 0.0);
}

int op_D(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec)
{
    int r = check_op(c, op);
    if (r) return r;
    if (op_is_w(op)) return set_err(c, TMX_EINVAL, "What^pm is defined for the Schur operator only");
    const bool nd = op == TMX_OP_ND;
    r = ensure_links(c, prec);
    if (!r) r = ensure_clover(c, prec);
    if (r) return r;
    const int nf = nd ? 2 : 1;
    const int sgn = nd ? 1 : op;
    for (int p = 0; p < 2; ++p) {
        DslashArgs a = base_args(c, prec, nd, 1);
        a.sgn = sgn;
        a.parity = p;
        a.out = parity_half(out, prec, nf, p);
        a.in = parity_half(in, prec, nf, 1 - p);
        a.x = parity_half(in, prec, nf, p);
        a.clov = clov_parity(c, prec, p);
        a.kfac = c->par.kappa;
        const LaunchCfg l = launch_cfg(c, kname("K2", prec, nd, 1));
        a.xcd = l.xcd;
        hipError_t e = launch_dslash(prec, nf, 1, a, c->stream, l.block);
        if (e != hipSuccess) return hip_err(c, e, "D launch");
    }
    return TMX_OK;
}

// ---------------------------------------------------------------------------
// autotuner: block size x XCD order per stencil kernel key
// ---------------------------------------------------------------------------
static std::string dims_key(const tmx_ctx *c)
{
    return std::to_string(c->dims[0]) + "x" + std::to_string(c->dims[1]) + "x" + std::to_string(c->dims[2]) + "x" +
           std::to_string(c->dims[3]);
}

static void tune_cache_load(tmx_ctx *c)
{
    const char *path = std::getenv("TMX_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char dk[64], kk[64];
    int block, xcd;
    double ms;
    const std::string me = dims_key(c);
    int spt, rg;
    while (std::fscanf(f, "%63s %63s %d %d %d %d %lf", dk, kk, &block, &xcd, &spt, &rg, &ms) == 7) {
        if (me == dk && block >= 64 && block <= 256 && block % 64 == 0 && spt >= 1 && spt <= 8 && rg >= 0)
            c->tune[kk] = LaunchCfg{block, xcd != 0, spt, rg};
    }
    std::fclose(f);
}

static void tune_cache_store(tmx_ctx *c, const std::string &key, const LaunchCfg &l, double ms)
{
    const char *path = std::getenv("TMX_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %s %d %d %d %d %.6f\n", dims_key(c).c_str(), key.c_str(), l.block, l.xcd, l.spt, l.rg, ms);
    std::fclose(f);
}

// time one launch shape of a stencil kernel: every group of its right-hand
// sides once per sweep, two warm-up sweeps, the mean of five (ms per sweep)
static int tune_time(tmx_ctx *c, DslashArgs a, int prec, int nf, int mode, const LaunchCfg &l, hipEvent_t e0,
                     hipEvent_t e1, double *ms_out)
{
    const int nrhs = a.nrhs;
    const int rg = (l.rg > 0 && l.rg < nrhs && nrhs % l.rg == 0) ? l.rg : nrhs;
    a.xcd = l.xcd;
    a.spt = l.spt;
    a.rg = rg;
    auto sweep = [&]() {
        hipError_t e = hipSuccess;
        for (int r0 = 0; r0 < nrhs && e == hipSuccess; r0 += rg) {
            a.r0 = r0;
            e = launch_dslash(prec, nf, mode, a, c->stream, l.block);
        }
        return e;
    };
    hipError_t e = hipSuccess;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = sweep();
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    const int reps = 5;
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = sweep();
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_err(c, e, "tune launch");
    *ms_out = ms / reps;
    return TMX_OK;
}

// the fastest of the candidate launch shapes for one kernel
static int tune_pick(tmx_ctx *c, const DslashArgs &a, int prec, int nf, int mode, const std::vector<LaunchCfg> &cands,
                     hipEvent_t e0, hipEvent_t e1, LaunchCfg *best, double *best_ms)
{
    *best_ms = 1e30;
    const bool log = std::getenv("TMX_TUNE_LOG") != nullptr;
    for (const LaunchCfg &l : cands) {
        double ms;
        int r = tune_time(c, a, prec, nf, mode, l, e0, e1, &ms);
        if (r) return r;
        if (log)
            std::fprintf(stderr, "# TMX: tune %s prec %d nf %d nrhs %d block %d xcd %d spt %d rg %d: %.4f ms\n",
                         mode ? "K2" : "K1", prec, nf, a.nrhs, l.block, l.xcd, l.spt, l.rg, ms);
        if (ms < *best_ms) {
            *best_ms = ms;
            *best = l;
        }
    }
    return TMX_OK;
}
}  // namespace tmx

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int tmx_create(const int dims[4], void *hip_stream, tmx_ctx **out)
{
    if (!out || !dims) return TMX_EINVAL;
    *out = nullptr;
    long V = 1;
    for (int k = 0; k < 4; ++k) {
        if (dims[k] < 2 || dims[k] % 2) return TMX_EINVAL;
        V *= dims[k];
        if (V > (1L << 31)) return TMX_EINVAL;
    }
    tmx_ctx *c = new tmx_ctx();
    for (int k = 0; k < 4; ++k) {
        c->dims[k] = dims[k];
        c->g.L[k] = dims[k];
    }
    c->V = V;
    c->Vh = V / 2;
    c->g.Lxh = dims[0] / 2;
    c->g.Vh = (int)c->Vh;
    // (z, t) plane tiling of the internal site order (see Geom); the
    // defaults come from measurement, TMX_SITE_ZB / TMX_SITE_TB override
    auto pick = [](const char *env, int dflt, int extent) {
        int v = dflt;
        if (const char *e = std::getenv(env)) v = std::atoi(e);
        int sh = 0;
        while ((2 << sh) <= v) ++sh;
        while (sh > 0 && extent % (1 << sh)) --sh;
        return sh;
    };
    c->g.zbs = pick("TMX_SITE_ZB", 2, dims[2]);
    c->g.tbs = pick("TMX_SITE_TB", 8, dims[3]);
    c->stream = static_cast<hipStream_t>(hip_stream);
    // enough workgroups for one slot per thread up to V/2 = 2M sites: a
    // grid-stride loop over several sites serialises their memory latency
    c->red.max_blocks = 8192;
    c->red.partials = static_cast<double *>(dev_alloc(c, red_partials_bytes(c)));
    c->red.result = static_cast<double *>(dev_alloc(c, red_result_bytes()));
    if (!c->red.partials || !c->red.result ||
        hipHostMalloc(&c->host_red, sizeof(double) * MAXR * 4, hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        dev_free(c, c->red.partials);
        dev_free(c, c->red.result);
        delete c;
        return TMX_ENOMEM;
    }
    // reductions also land in the coherent pinned buffer, so a readback is a
    // stream synchronisation without a copy launch (if the mapping is not
    // available the readback copies instead)
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&c->red.host), c->host_red, 0) != hipSuccess) {
        (void)hipGetLastError();
        c->red.host = nullptr;
    }
    // device address of the allocation-free operator's scratch on this
    // device (resolved here, at set-up; a failure only disables that entry point)
    (void)scratch_address(c);
    c->err.clear();
    // cap on the named scratch buffers (bytes), for callers that budget HBM
    if (const char *e = std::getenv("TMX_WS_LIMIT")) c->ws_limit = std::strtoull(e, nullptr, 10);
    const char *tr = std::getenv("TMX_TRACE");
    c->trace = tr && tr[0] == '1';
    tune_cache_load(c);
    // launch-shape overrides for sweeps (the autotuner sets per-kernel values)
    if (const char *e = std::getenv("TMX_DSLASH_BLOCK")) {
        int b = std::atoi(e);
        if (b >= 64 && b <= 256 && b % 64 == 0) c->default_block = b;
    }
    if (const char *e = std::getenv("TMX_DSLASH_XCD")) c->xcd_remap = std::atoi(e) != 0;
    *out = c;
    return TMX_OK;
}

void tmx_pc_free(tmx_ctx *c);  // nn.hip

int tmx_destroy(tmx_ctx *c)
{
    if (!c) return TMX_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    for (int p = 0; p < 3; ++p) {
        dev_free(c, c->links[p]);
        dev_free(c, c->clov[p]);
        dev_free(c, c->inv[p]);
        dev_free(c, c->invnd[p]);
    }
    for (auto &kv : c->ws) dev_free(c, kv.second.p);
    kstat_collect(c);
    for (hipEvent_t e : c->kpool) (void)hipEventDestroy(e);
    dev_free(c, c->red.partials);
    dev_free(c, c->red.result);
    if (c->host_red) (void)hipHostFree(c->host_red);
    tmx_pc_free(c);
    while (!c->allocs.empty()) dev_free(c, c->allocs.begin()->first);
    delete c;
    return TMX_OK;
}

int tmx_free_workspaces(tmx_ctx *c)
{
    if (!c) return TMX_EINVAL;
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_err(c, e, "tmx_free_workspaces");
    for (auto &kv : c->ws) dev_free(c, kv.second.p);
    c->ws.clear();
    c->ws_bytes = 0;
    return TMX_OK;
}

const char *tmx_last_error(const tmx_ctx *c) { return c ? c->err.c_str() : "null context"; }

int tmx_set_stream(tmx_ctx *c, void *s)
{
    if (!c) return TMX_EINVAL;
    c->stream = static_cast<hipStream_t>(s);
    return TMX_OK;
}

int tmx_set_allocator(tmx_ctx *c, void *(*alloc)(size_t, void *), void (*release)(void *, void *), void *user)
{
    if (!c) return TMX_EINVAL;
    if ((alloc == nullptr) != (release == nullptr))
        return set_err(c, TMX_EINVAL, "tmx_set_allocator: give both functions or neither");
    if (hipStreamSynchronize(c->stream) != hipSuccess) (void)hipGetLastError();
    c->alloc_fn = alloc;
    c->release_fn = release;
    c->alloc_user = user;
    // the reduction buffers hold nothing between calls: move them to the new
    // allocator now (everything allocated later comes from it as well; what
    // exists already is released by the allocator that made it)
    double *np = static_cast<double *>(dev_alloc(c, red_partials_bytes(c)));
    double *nr = np ? static_cast<double *>(dev_alloc(c, red_result_bytes())) : nullptr;
    if (!np || !nr) {
        dev_free(c, np);
        return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    }
    dev_free(c, c->red.partials);
    dev_free(c, c->red.result);
    c->red.partials = np;
    c->red.result = nr;
    return TMX_OK;
}

int tmx_set_params(tmx_ctx *c, const tmx_params *p)
{
    if (!c || !p) return TMX_EINVAL;
    if (!(p->kappa > 0) || !std::isfinite(p->kappa) || !std::isfinite(p->csw) || !std::isfinite(p->mu) ||
        !std::isfinite(p->mubar) || !std::isfinite(p->epsbar) || !std::isfinite(p->rho) || (p->t_bc != 1 && p->t_bc != -1))
        return set_err(c, TMX_EINVAL, "invalid parameters");
    if (c->have_params && !c->clover_from_host && (p->kappa != c->par.kappa || p->csw != c->par.csw))
        c->clov_ok[0] = c->clov_ok[1] = c->clov_ok[2] = false;
    if (c->have_params && p->kappa != c->par.kappa) {
        // site inverses depend on 2 kappa mu
        c->inv_ok[0] = c->inv_ok[1] = c->inv_ok[2] = false;
        c->invnd_ok[0] = c->invnd_ok[1] = c->invnd_ok[2] = false;
    }
    c->par = *p;
    c->have_params = true;
    return TMX_OK;
}

int tmx_load_gauge(tmx_ctx *c, const double *host_links, double gauge_id)
{
    if (!c || !host_links) return TMX_EINVAL;
    if (c->gauge_loaded && gauge_id == c->gauge_id) return TMX_OK;
    const size_t bytes = (size_t)c->V * 4 * 9 * 16;
    void *stage = dev_alloc(c, bytes);
    if (!stage) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    if (!c->links[F64]) {
        c->links[F64] = dev_alloc(c, link_bytes(F64, c->Vh));
        if (!c->links[F64]) {
            dev_free(c, stage);
            return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
    }
    hipError_t e = hipMemcpyAsync(stage, host_links, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_pack_links((const double *)stage, (double *)c->links[F64], c->g, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(c, stage);
    if (e != hipSuccess) return hip_err(c, e, "gauge upload");
    c->gauge_loaded = true;
    c->gauge_id = gauge_id;
    c->uploads++;
    // cascade: every derived field is stale now
    for (int p = 0; p < 3; ++p) {
        c->links_ok[p] = p == F64;
        c->clov_ok[p] = false;
        c->inv_ok[p] = false;
        c->invnd_ok[p] = false;
    }
    c->clover_from_host = false;
    return TMX_OK;
}

int tmx_gauge_uploads(const tmx_ctx *c) { return c ? c->uploads : -1; }

int tmx_load_clover(tmx_ctx *c, const double *host_T)
{
    if (!c) return TMX_EINVAL;
    if (!c->gauge_loaded) return set_err(c, TMX_ENOTLOADED, "load a gauge field first");
    if (!host_T) {
        c->clover_from_host = false;
        c->clov_ok[0] = c->clov_ok[1] = c->clov_ok[2] = false;
        int r = ensure_clover(c, F64);
        if (r) return r;
        return hip_err(c, hipStreamSynchronize(c->stream), "clover build");
    }
    // Hermiticity check on the host
    const long n = c->V * 2;
    for (long b = 0; b < n; ++b) {
        const double *m = host_T + b * 72;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                const double re = m[2 * (6 * i + j)], im = m[2 * (6 * i + j) + 1];
                const double re2 = m[2 * (6 * j + i)], im2 = m[2 * (6 * j + i) + 1];
                if (std::fabs(re - re2) > 1e-12 || std::fabs(im + im2) > 1e-12 || !std::isfinite(re) ||
                    !std::isfinite(im))
                    return set_err(c, TMX_EINVAL, "clover block is not Hermitian");
            }
    }
    const size_t bytes = (size_t)c->V * 144 * 8;
    void *stage = dev_alloc(c, bytes);
    if (!stage) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    if (!c->clov[F64]) {
        c->clov[F64] = dev_alloc(c, clover_bytes(F64, c->Vh));
        if (!c->clov[F64]) {
            dev_free(c, stage);
            return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
        }
    }
    hipError_t e = hipMemcpyAsync(stage, host_T, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_clover_from_canonical((const double *)stage, (double *)c->clov[F64], c->g, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(c, stage);
    if (e != hipSuccess) return hip_err(c, e, "clover upload");
    c->clover_from_host = true;
    c->clov_ok[F64] = true;
    c->clov_ok[F32] = c->clov_ok[F16] = false;
    for (int p = 0; p < 3; ++p) c->inv_ok[p] = c->invnd_ok[p] = false;
    return TMX_OK;
}

int tmx_get_clover(tmx_ctx *c, double *host_T)
{
    if (!c || !host_T) return TMX_EINVAL;
    int r = ensure_clover(c, F64);
    if (r) return r;
    const size_t bytes = (size_t)c->V * 144 * 8;
    void *stage = dev_alloc(c, bytes);
    if (!stage) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    hipError_t e = launch_clover_to_canonical((const double *)c->clov[F64], (double *)stage, c->g, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_T, stage, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(c, stage);
    return hip_err(c, e, "clover download");
}

static int kind_nf(int kind) { return (kind == TMX_FIELD_ODD_ND || kind == TMX_FIELD_FULL_ND) ? 2 : 1; }
static bool kind_full(int kind) { return kind == TMX_FIELD_FULL || kind == TMX_FIELD_FULL_ND; }

int tmx_field_bytes(const tmx_ctx *c, int kind, int prec, size_t *bytes)
{
    if (!c || !bytes || kind < 0 || kind > 3 || prec < 0 || prec > 2) return TMX_EINVAL;
    *bytes = (size_t)spinor_field_bytes(prec, kind_nf(kind), c->Vh) * (kind_full(kind) ? 2 : 1);
    return TMX_OK;
}

int tmx_pack(tmx_ctx *c, void *internal, const double *canonical, int kind, int prec, int nvec)
{
    if (!c || !internal || !canonical || kind < 0 || kind > 3 || prec < 0 || prec > 2 || nvec < 1)
        return c ? set_err(c, TMX_EINVAL, "tmx_pack: bad argument") : TMX_EINVAL;
    if (kind_full(kind) && nvec != 1) return set_err(c, TMX_EINVAL, "full fields take nvec = 1");
    SpinorPtr f = make_spinor(internal, prec, kind_nf(kind), c->Vh * nvec);
    return hip_err(c, launch_pack_spinor(canonical, f, prec, kind, c->g, nvec, c->stream), "pack");
}

int tmx_unpack(tmx_ctx *c, double *canonical, const void *internal, int kind, int prec, int nvec)
{
    if (!c || !internal || !canonical || kind < 0 || kind > 3 || prec < 0 || prec > 2 || nvec < 1)
        return c ? set_err(c, TMX_EINVAL, "tmx_unpack: bad argument") : TMX_EINVAL;
    if (kind_full(kind) && nvec != 1) return set_err(c, TMX_EINVAL, "full fields take nvec = 1");
    SpinorPtr f = make_spinor(const_cast<void *>(internal), prec, kind_nf(kind), c->Vh * nvec);
    return hip_err(c, launch_unpack_spinor(canonical, f, prec, kind, c->g, nvec, c->stream), "unpack");
}

int tmx_apply_D(tmx_ctx *c, void *out, const void *in, int op, int prec)
{
    if (!c || !out || !in || out == in) return c ? set_err(c, TMX_EINVAL, "tmx_apply_D: bad argument") : TMX_EINVAL;
    const int nf = op == TMX_OP_ND ? 2 : 1;
    return op_D(c, make_spinor(out, prec, nf, c->Vh), make_spinor(const_cast<void *>(in), prec, nf, c->Vh), op, prec);
}

int tmx_apply_mhat(tmx_ctx *c, void *out, const void *in, int op, int prec, int dagger, int nrhs)
{
    if (!c || !out || !in || out == in || nrhs < 1 || nrhs > MAXR)
        return c ? set_err(c, TMX_EINVAL, "tmx_apply_mhat: bad argument") : TMX_EINVAL;
    const int nf = op == TMX_OP_ND ? 2 : 1;
    const long stride = c->Vh * nrhs;
    return op_mhat(c, make_spinor(out, prec, nf, stride), make_spinor(const_cast<void *>(in), prec, nf, stride), op,
                   prec, dagger ? 1 : 0, nrhs);
}

int tmx_apply_mhat_noalloc(tmx_ctx *c, void *out, const void *in, int op, int prec, int dagger, int nrhs)
{
    if (!c || !out || !in || out == in || nrhs < 1 || nrhs > MAXR || prec < F64 || prec > F16)
        return c ? set_err(c, TMX_EINVAL, "tmx_apply_mhat_noalloc: bad argument") : TMX_EINVAL;
    int r = check_op(c, op);
    if (r) return r;
    const bool nd = op == TMX_OP_ND;
    const int nf = nd ? 2 : 1;
    const long stride = c->Vh * nrhs;
    const size_t need = (size_t)spinor_field_bytes(prec, nf, stride);
    if (need > NOALLOC_SCRATCH_BYTES)
        return set_err(c, TMX_EINVAL, "tmx_apply_mhat_noalloc: the intermediate field needs " + std::to_string(need) +
                                          " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                          "-byte scratch (use tmx_apply_mhat)");
    // every derived field of this precision must exist already (building one
    // would allocate); rebuilding an existing one after new parameters does not
    const bool have = c->gauge_loaded && c->have_params && c->links[prec] && c->clov[F64] && c->clov[prec] &&
                      (nd ? (c->invnd[F64] && c->invnd[prec]) : (c->inv[F64] && c->inv[prec]));
    if (!have)
        return set_err(c, TMX_ENOTLOADED, "tmx_apply_mhat_noalloc: the fields of this precision are not resident "
                                          "(one tmx_apply_mhat in this precision and sector builds them)");
    r = ensure_ready(c, prec, nd);
    if (r) return r;
    void *u = scratch_address(c);
    if (!u) return TMX_EHIP;
    const SpinorPtr O = make_spinor(out, prec, nf, stride), I = make_spinor(const_cast<void *>(in), prec, nf, stride);
    return mhat_with(c, O, I, make_spinor(u, prec, nf, stride), op, prec, dagger ? 1 : 0, nrhs);
}

int tmx_apply_mdagm(tmx_ctx *c, void *out, const void *in, int op, int prec, int nrhs)
{
    if (!c || !out || !in || out == in || nrhs < 1 || nrhs > MAXR)
        return c ? set_err(c, TMX_EINVAL, "tmx_apply_mdagm: bad argument") : TMX_EINVAL;
    const int nf = op == TMX_OP_ND ? 2 : 1;
    const long stride = c->Vh * nrhs;
    return op_mdagm(c, make_spinor(out, prec, nf, stride), make_spinor(const_cast<void *>(in), prec, nf, stride), op,
                    prec, nrhs);
}

}  // extern "C"

namespace tmx {

// Full-lattice fields of the force terms: X, Y odd, u = B_ee(s)^{-1} H_eo X and
// w' = B_ee(-s)^{-1} H_eo g5 Y even (the force kernels apply the outer g5 of
// w); nf flavours each (two for the operator of eq. Q-hat_h, whose site
// blocks B_ee(+-) mix the flavours).
struct ForceFields {
    SpinorPtr X, Y, u, w;
    int nf;
};

// flavour f of an internal FP64 field of nf flavours, as a one-flavour field
static SpinorPtr flavour_view(SpinorPtr a, long stride, int f)
{
    return make_spinor(static_cast<char *>(a.d) + (size_t)f * spinor_field_bytes(F64, 1, stride), F64, 1, stride);
}

// u and w from internal FP64 odd fields X, Y (op: TMX_OP_PLUS / MINUS / ND)
static int force_fields_internal(tmx_ctx *c, SpinorPtr X, SpinorPtr Y, int op, ForceFields &ff)
{
    const bool nd = op == TMX_OP_ND;
    int r = ensure_ready(c, F64, nd);
    if (r) return r;
    const int nf = nd ? 2 : 1;
    const size_t fb = spinor_field_bytes(F64, nf, c->Vh);
    void *pu = ws_get(c, "hf_u", fb), *pw = ws_get(c, "hf_w", fb);
    if (!pu || !pw) return set_err(c, TMX_ENOMEM, "force workspace: out of device memory");
    ff.X = X;
    ff.Y = Y;
    ff.u = make_spinor(pu, F64, nf, c->Vh);
    ff.w = make_spinor(pw, F64, nf, c->Vh);
    ff.nf = nf;
    const int sgn = op_sign(op);
    const LaunchCfg l1 = launch_cfg(c, kname("K1", F64, nd, 1));
    DslashArgs a = base_args(c, F64, nd, 1);
    a.parity = 0;
    a.clov = clov_parity(c, F64, 0);
    a.inv = nd ? c->invnd[F64] : c->inv[F64];
    a.xcd = l1.xcd;
    a.sgn = sgn;
    a.in = ff.X;
    a.out = ff.u;
    hipError_t e = launch_dslash(F64, nf, 0, a, c->stream, l1.block);
    if (e != hipSuccess) return hip_err(c, e, "K1 launch");
    a.sgn = -sgn;
    a.g5in = 1;
    a.in = ff.Y;
    a.out = ff.w;
    e = launch_dslash(F64, nf, 0, a, c->stream, l1.block);
    return e != hipSuccess ? hip_err(c, e, "K1 launch") : TMX_OK;
}

// force (= or +=) coeff * hopping-term force of Re<Y, Mhat X>, per flavour
static int hop_force_fields(tmx_ctx *c, double *force, const ForceFields &ff, double coeff, int accumulate)
{
    for (int fl = 0; fl < ff.nf; ++fl) {
        ForceArgs f{};
        f.g = c->g;
        f.U = LinkPtr{c->links[F64], c->Vh};
        f.X = flavour_view(ff.X, c->Vh, fl);
        f.Y = flavour_view(ff.Y, c->Vh, fl);
        f.u = flavour_view(ff.u, c->Vh, fl);
        f.w = flavour_view(ff.w, c->Vh, fl);
        f.t_bc = c->par.t_bc;
        f.kfac = c->par.kappa * c->par.kappa;
        f.coeff = coeff;
        // the force is linear in the flavour-summed outer products: the
        // second flavour adds its part
        f.accumulate = (accumulate || fl > 0) ? 1 : 0;
        f.out = force;
        f.xcd = c->xcd_remap;
        kstat_begin(c, "HOP_FORCE");
        hipError_t e = launch_hop_force(f, c->stream);
        kstat_end(c);
        if (e != hipSuccess) return hip_err(c, e, "hop force");
    }
    return TMX_OK;
}

// force (= or +=) coeff * clover-term force of Re<Y, Mhat X>: the insertions
// summed over the flavours, then the plaquette loops and the link sums
static int clover_force_fields(tmx_ctx *c, double *force, const ForceFields &ff, double coeff, int accumulate)
{
    if (c->clover_from_host)
        return set_err(c, TMX_EINVAL, "the clover force needs the clover term built from the links");
    void *ph = ws_get(c, "cf_h", (size_t)6 * 9 * 2 * c->Vh * sizeof(double));
    void *pka = ph ? ws_get(c, "cf_ka", (size_t)6 * 16 * 2 * c->Vh * sizeof(double)) : nullptr;
    if (!ph || !pka) return set_err(c, TMX_ENOMEM, "clover force workspace: out of device memory");
    CloverForceArgs f{};
    f.g = c->g;
    f.U = LinkPtr{c->links[F64], c->Vh};
    f.kfac = c->par.kappa * c->par.kappa;
    f.kc8 = c->par.kappa * c->par.csw / 8.0;
    f.coeff = coeff;
    f.accumulate = accumulate ? 1 : 0;
    f.H = static_cast<double *>(ph);
    f.KA = static_cast<double *>(pka);
    f.out = force;
    f.xcd = c->xcd_remap;
    kstat_begin(c, "CLOVER_FORCE");
    hipError_t e = hipSuccess;
    for (int fl = 0; fl < ff.nf && e == hipSuccess; ++fl) {
        f.X = flavour_view(ff.X, c->Vh, fl);
        f.Y = flavour_view(ff.Y, c->Vh, fl);
        f.u = flavour_view(ff.u, c->Vh, fl);
        f.w = flavour_view(ff.w, c->Vh, fl);
        f.h_acc = fl > 0 ? 1 : 0;
        e = launch_clover_insertions(f, c->stream);
    }
    if (e == hipSuccess) e = launch_clover_link_sums(f, c->stream);
    kstat_end(c);
    return hip_err(c, e, "clover force");
}

int force_internal(tmx_ctx *c, double *force, SpinorPtr X, SpinorPtr Y, int op, double coeff, int accumulate,
                   int terms)
{
    ForceFields ff;
    int r = force_fields_internal(c, X, Y, op, ff);
    if (r) return r;
    if (terms & 1) {
        r = hop_force_fields(c, force, ff, coeff, accumulate);
        if (r) return r;
        accumulate = 1;
    }
    if (terms & 2) r = clover_force_fields(c, force, ff, coeff, accumulate);
    return r;
}

}  // namespace tmx

extern "C" {

// the entry points: canonical odd fields x, y (one or two flavours) packed first
static int force_entry(tmx_ctx *c, double *force, const double *x, const double *y, int op, double coeff,
                       int accumulate, int terms, const char *name)
{
    if (!c || !force || !x || !y || !std::isfinite(coeff))
        return c ? set_err(c, TMX_EINVAL, std::string(name) + ": bad argument") : TMX_EINVAL;
    if (op != TMX_OP_PLUS && op != TMX_OP_MINUS && op != TMX_OP_ND)
        return set_err(c, TMX_EINVAL, std::string(name) + ": built for the degenerate and the two-flavour Schur operators");
    if ((terms & 2) && c->clover_from_host)
        return set_err(c, TMX_EINVAL, "the clover force needs the clover term built from the links");
    const int nf = op == TMX_OP_ND ? 2 : 1;
    int r = ensure_ready(c, F64, op == TMX_OP_ND);
    if (r) return r;
    const size_t fb = spinor_field_bytes(F64, nf, c->Vh);
    void *px = ws_get(c, "hf_x", fb), *py = ws_get(c, "hf_y", fb);
    if (!px || !py) return set_err(c, TMX_ENOMEM, "force workspace: out of device memory");
    const SpinorPtr X = make_spinor(px, F64, nf, c->Vh), Y = make_spinor(py, F64, nf, c->Vh);
    const int kind = nf == 2 ? TMX_FIELD_ODD_ND : TMX_FIELD_ODD;
    r = hip_err(c, launch_pack_spinor(x, X, F64, kind, c->g, 1, c->stream), "pack x");
    if (!r) r = hip_err(c, launch_pack_spinor(y, Y, F64, kind, c->g, 1, c->stream), "pack y");
    if (r) return r;
    return force_internal(c, force, X, Y, op, coeff, accumulate, terms);
}

int tmx_hop_force(tmx_ctx *c, double *force, const double *x, const double *y, int op, double coeff, int accumulate)
{
    return force_entry(c, force, x, y, op, coeff, accumulate, 1, "tmx_hop_force");
}

int tmx_clover_force(tmx_ctx *c, double *force, const double *x, const double *y, int op, double coeff,
                     int accumulate)
{
    return force_entry(c, force, x, y, op, coeff, accumulate, 2, "tmx_clover_force");
}

// ---- autotuner -----------------------------------------------------------------
int tmx_tune(tmx_ctx *c, int prec, int op, int nrhs)
{
    if (!c || prec < 0 || prec > 2 || nrhs < 1 || nrhs > MAXR) return c ? set_err(c, TMX_EINVAL, "tmx_tune: bad argument") : TMX_EINVAL;
    if (op != TMX_OP_PLUS && op != TMX_OP_MINUS && op != TMX_OP_ND) return set_err(c, TMX_EINVAL, "bad op");
    const bool nd = op == TMX_OP_ND;
    int r = ensure_ready(c, prec, nd);
    if (r) return r;
    const int nf = nd ? 2 : 1;
    const long stride = c->Vh * nrhs;
    const size_t fb = spinor_field_bytes(prec, nf, stride);
    void *pin = ws_get(c, "tune_in", fb), *pu = ws_get(c, "tune_u", fb), *pout = ws_get(c, "tune_out", fb);
    if (!pin || !pu || !pout) return set_err(c, TMX_ENOMEM, "device buffer: out of device memory");
    r = hip_err(c, hipMemsetAsync(pin, 0, fb, c->stream), "tune fill");
    if (r) return r;
    SpinorPtr in = make_spinor(pin, prec, nf, stride), u = make_spinor(pu, prec, nf, stride),
              out = make_spinor(pout, prec, nf, stride);
    DslashArgs a = base_args(c, prec, nd, nrhs);
    a.sgn = nd ? 1 : op;
    a.parity = 0;
    a.out = u;
    a.in = in;
    a.clov = clov_parity(c, prec, 0);
    a.inv = nd ? c->invnd[prec] : c->inv[prec];
    DslashArgs b = base_args(c, prec, nd, nrhs);
    b.sgn = a.sgn;
    b.parity = 1;
    b.out = out;
    b.in = u;
    b.x = in;
    b.clov = clov_parity(c, prec, 1);
    b.kfac = c->par.kappa * c->par.kappa;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hip_err(c, hipGetLastError(), "tune events");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_err(c, hipGetLastError(), "tune events");
    }
    // knobs: workgroup size, XCD-contiguous block order, sites per thread;
    // several right-hand sides: the group size (a divisor of nrhs), timed as
    // the whole sweep over the groups, K1 and K2 sharing the group size
    std::vector<int> groups;
    for (int g = nrhs; g >= 1; --g)
        if (nrhs % g == 0) groups.push_back(g);
    LaunchCfg best1, best2;
    double best_ms = 1e30, ms1 = 0, ms2 = 0;
    for (int g : groups) {
        std::vector<LaunchCfg> cands;
        for (int xcd = 0; xcd < 2; ++xcd)
            for (int blk : {64, 128, 256})
                for (int spt = 1; spt <= (nrhs == 1 ? 2 : 1); ++spt) cands.push_back(LaunchCfg{blk, xcd, spt, g});
        LaunchCfg c1, c2;
        double t1, t2;
        r = tune_pick(c, a, prec, nf, 0, cands, e0, e1, &c1, &t1);
        if (!r) r = tune_pick(c, b, prec, nf, 1, cands, e0, e1, &c2, &t2);
        if (r) break;
        if (t1 + t2 < best_ms) {
            best_ms = t1 + t2;
            best1 = c1;
            best2 = c2;
            ms1 = t1;
            ms2 = t2;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r) return r;
    const std::string k1 = kname("K1", prec, nd, nrhs), k2 = kname("K2", prec, nd, nrhs);
    c->tune[k1] = best1;
    c->tune[k2] = best2;
    tune_cache_store(c, k1, best1, ms1);
    tune_cache_store(c, k2, best2, ms2);
    return TMX_OK;
}

int tmx_tuned_config(tmx_ctx *c, const char *key, int *block, int *xcd, int *spt, int *rg)
{
    if (!c || !key) return TMX_EINVAL;
    LaunchCfg l = launch_cfg(c, key);
    if (block) *block = l.block;
    if (xcd) *xcd = l.xcd;
    if (spt) *spt = l.spt;
    if (rg) *rg = l.rg;
    return c->tune.count(key) ? TMX_OK : TMX_ENOCONV;
}

// ---- kernel timing -----------------------------------------------------------
int tmx_kstats_enable(tmx_ctx *c, int on)
{
    if (!c) return TMX_EINVAL;
    kstat_collect(c);
    c->kstats.clear();
    c->kstats_on = on != 0;
    return TMX_OK;
}

int tmx_kstats_get(tmx_ctx *c, int idx, char *name, size_t name_len, long *count, double *total_ms)
{
    if (!c || idx < 0) return TMX_EINVAL;
    kstat_collect(c);
    if (idx >= (int)c->kstats.size()) return TMX_EINVAL;
    auto it = c->kstats.begin();
    std::advance(it, idx);
    if (name && name_len) {
        std::strncpy(name, it->first.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    if (count) *count = it->second.count;
    if (total_ms) *total_ms = it->second.ms;
    return TMX_OK;
}

// ---- tracing ---------------------------------------------------------------
int tmx_trace_enable(tmx_ctx *c, int on)
{
    if (!c) return TMX_EINVAL;
    c->trace = on != 0;
    return TMX_OK;
}

int tmx_trace_push(tmx_ctx *c, const char *name)
{
    if (!c || !name) return TMX_EINVAL;
    if (c->trace) (void)hipStreamSynchronize(c->stream);
    c->frames.push_back(TraceFrame{name, now_seconds()});
    return TMX_OK;
}

int tmx_trace_pop(tmx_ctx *c)
{
    if (!c || c->frames.empty()) return TMX_EINVAL;
    if (c->trace) {
        (void)hipStreamSynchronize(c->stream);
        const double dt = now_seconds() - c->frames.back().t0;
        std::string path;
        for (auto &f : c->frames) path += "/" + f.name;
        std::printf("# TMX: Time for %s %.6e s level: %d %s\n", c->frames.back().name.c_str(), dt,
                    (int)c->frames.size(), path.c_str());
        std::fflush(stdout);
    }
    c->frames.pop_back();
    return TMX_OK;
}

}  // extern "C"
