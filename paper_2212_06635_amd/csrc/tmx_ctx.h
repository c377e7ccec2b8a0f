// Library context: device state, lazy derived fields and workspaces.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/tmx.h"
#include "blas.h"
#include "tmx_kernels.h"

namespace tmx {

struct Workspace {
    void *p = nullptr;
    size_t bytes = 0;
};

// one live device allocation: its size and the allocator that made it (the
// caller's hook, or hipMalloc when none was set), so that it is released by
// the same one whatever hook is in place later
struct AllocRec {
    size_t bytes = 0;
    void (*release)(void *, void *) = nullptr;  // null: hipFree
    void *user = nullptr;
};

struct TraceFrame {
    std::string name;
    double t0;
};

// per-kernel timing with HIP events on the context's stream
struct KEvent {
    std::string name;
    hipEvent_t a, b;
};
struct KStat {
    long count = 0;
    double ms = 0;
};

// launch shape of a stencil kernel (chosen by the autotuner): workgroup
// size, XCD-contiguous block order, sites per thread, and for several
// right-hand sides the group size rg (the operator runs K1 then K2 on each
// group of rg right-hand sides in turn; 0 = all at once)
struct LaunchCfg {
    int block = 64;
    int xcd = 1;
    int spt = 1;
    int rg = 0;
};

// learned-preconditioner state (nn.hip)
struct PcState;

}  // namespace tmx

struct tmx_ctx {
    int dims[4];
    tmx::Geom g;
    long V, Vh;
    hipStream_t stream;

    tmx_params par{};
    bool have_params = false;

    // gauge-state tracking: the id of the field on the device
    bool gauge_loaded = false;
    double gauge_id = 0.0;
    int uploads = 0;

    // compressed links per precision (links[F64] is the master)
    void *links[3] = {nullptr, nullptr, nullptr};
    bool links_ok[3] = {false, false, false};

    // A = 1 + T on both parities, Hermitian packed, per precision
    void *clov[3] = {nullptr, nullptr, nullptr};
    bool clov_ok[3] = {false, false, false};
    bool clover_from_host = false;
    double clov_kappa = 0, clov_csw = 0;

    // degenerate site inverse (A_ee + i nu g5)^{-1}, per precision
    void *inv[3] = {nullptr, nullptr, nullptr};
    bool inv_ok[3] = {false, false, false};
    double inv_nu = 0;

    // two-flavour inverse factor (A_ee^2 + nubar^2 - epst^2)^{-1}
    void *invnd[3] = {nullptr, nullptr, nullptr};
    bool invnd_ok[3] = {false, false, false};
    double invnd_c = 0;

    // reductions
    tmx::RedWork red{};
    double *host_red = nullptr;  // pinned

    // named scratch buffers
    std::map<std::string, tmx::Workspace> ws;
    size_t ws_bytes = 0;  // bytes held by the named scratch buffers
    size_t ws_limit = 0;  // cap on ws_bytes (0: none), from TMX_WS_LIMIT

    // device allocator: the caller's hook (tmx_set_allocator) or hipMalloc
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*release_fn)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    std::map<void *, tmx::AllocRec> allocs;  // every live device allocation

    // tracing
    bool trace = false;
    std::vector<tmx::TraceFrame> frames;

    // kernel timing
    bool kstats_on = false;
    std::vector<tmx::KEvent> kpending;
    std::vector<hipEvent_t> kpool;
    std::map<std::string, tmx::KStat> kstats;

    // kernel launch tuning (block size per kernel key)
    std::map<std::string, tmx::LaunchCfg> tune;
    int default_block = 64;
    int xcd_remap = 1;

    tmx::PcState *pc = nullptr;

    std::string err;
};

namespace tmx {

#define HIP_CHECK_RET(c, x, w)               \
    do {                                     \
        int _rr = hip_err((c), (x), (w));    \
        if (_rr) return _rr;                 \
    } while (0)

// error helpers
int set_err(tmx_ctx *c, int code, const std::string &msg);
int hip_err(tmx_ctx *c, hipError_t e, const char *where);

// memory: every device buffer of a context comes from dev_alloc (the
// caller's allocator if one is set, else hipMalloc) and goes back through
// dev_free.  ws_get returns a named scratch buffer of at least `bytes`, or
// nullptr with TMX_ENOMEM recorded (allocation failure or the TMX_WS_LIMIT
// cap): callers check it before launching anything on it.
void *dev_alloc(tmx_ctx *c, size_t bytes);
void dev_free(tmx_ctx *c, void *p);
void *ws_get(tmx_ctx *c, const std::string &name, size_t bytes);

// lazily build everything an apply in `prec` needs
int ensure_ready(tmx_ctx *c, int prec, bool nd);

// operators on internal fields (asynchronous)
int op_mhat(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec, int dagger, int nrhs);
// out = N in = Mhat^dagger Mhat in; if nrm is given it receives <in, N in> = |Mhat in|^2
// of every slot (FP64, Vh * nrhs values)
int op_mdagm(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec, int nrhs, double *nrm = nullptr);
int op_D(tmx_ctx *c, SpinorPtr out, SpinorPtr in, int op, int prec);

// launch shape for a kernel key ("K1_f64", "K2_f32_nd_r12", ...)
LaunchCfg launch_cfg(tmx_ctx *c, const std::string &key);

// reductions: copy device results to the host (synchronises the stream)
int fetch(tmx_ctx *c, int n, double *host);

// model bytes of one Mhat application per odd site
double mhat_bytes_per_site(int prec, int nf, int nrhs);

double now_seconds();

// learned preconditioner: z = K r (dagger = 0) or K^dagger r on odd fields
int pc_apply_internal(tmx_ctx *c, SpinorPtr z, int pz, SpinorPtr r, int pr, int dagger);
// plain / mixed CG on N used as the fallback of the flexible GCR solver
int cg_fallback(tmx_ctx *c, int op, SpinorPtr x, SpinorPtr b, double tol, int maxiter, tmx_info *info);

// link derivative of Re<Y, Mhat(op) X> (internal FP64 odd fields of one or
// two flavours): force (= or +=) coeff F, F the hopping-term (terms & 1)
// plus the clover-term (terms & 2) force, canonical link layout
int force_internal(tmx_ctx *c, double *force, SpinorPtr X, SpinorPtr Y, int op, double coeff, int accumulate,
                   int terms);

// kernel-timing brackets around a launch (no-ops unless enabled)
void kstat_begin(tmx_ctx *c, const std::string &name);
void kstat_end(tmx_ctx *c);

}  // namespace tmx
