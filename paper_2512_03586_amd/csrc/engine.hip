// engine.hip -- host side of the C ABI declared in include/esbgk.h.
//
// Drives Algorithm 1 of the paper on the caller's stream: regime update
// (indicator, transitions, compaction), then per IMEX stage the kinetic stage
// kernel on kinetic cells, the Euler stage on fluid cells and the buffer fill
// (fluid cells inside a kinetic stencil carry the corrected Maxwellian of
// their U), then the final combination.  No device memory is allocated: every
// array is a slice of the caller's workspace.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/esbgk.h"
#include "kernels.h"

using namespace esbgk;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(ESBGK_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes per value of the state arrays (f^n) and of the stage arrays (f^(2), f^(3))
size_t state_elem(int precision) { return precision == ESBGK_FP64 ? 8 : precision == ESBGK_BF16 ? 2 : 4; }
size_t stage_elem(int precision) { return precision == ESBGK_FP64 ? 8 : precision == ESBGK_FP32 ? 4 : 2; }
// whether stage 3 re-evaluates stage 2's Gaussian (and so needs its parameters)
bool stage_gauss_params(int precision) { return stage_elem(precision) == 2 || !ESBGK_QDIFF; }

// IMEX tableaux, 3 stages (Sec. 3.4.2 for ARS(2,3,3); ARS(2,2,2) its
// second-order sibling).  Explicit (At, bt), implicit (A, b).
void tableau(int scheme, double At[9], double bt[3], double A[9], double b[3]) {
    for (int q = 0; q < 9; ++q) At[q] = A[q] = 0.0;
    if (scheme == ESBGK_ARS233) {
        const double al = (3.0 + std::sqrt(3.0)) / 6.0;
        At[3] = al;
        At[6] = al - 1.0; At[7] = 2.0 - 2.0 * al;
        bt[0] = 0.0; bt[1] = 0.5; bt[2] = 0.5;
        A[4] = al;
        A[7] = 1.0 - 2.0 * al; A[8] = al;
        b[0] = 0.0; b[1] = 0.5; b[2] = 0.5;
    } else {
        const double g = 1.0 - 1.0 / std::sqrt(2.0);
        const double d = 1.0 - 1.0 / (2.0 * g);
        At[3] = g;
        At[6] = d; At[7] = 1.0 - d;
        bt[0] = d; bt[1] = 1.0 - d; bt[2] = 0.0;
        A[4] = g;
        A[7] = 1.0 - g; A[8] = g;
        b[0] = 0.0; b[1] = 1.0 - g; b[2] = g;
    }
}

int validate(const esbgk_config *c) {
    if (!c) return fail(ESBGK_EINVAL, "null config");
    if (c->nx < 1 || c->ny < 1) return fail(ESBGK_EINVAL, "nx, ny must be >= 1");
    if ((long long)c->nx * c->ny > (1LL << 28)) return fail(ESBGK_EINVAL, "grid too large");
    if (c->nv < 4 || c->nv > 64 || c->nv % 4 != 0) return fail(ESBGK_EINVAL, "nv must be a multiple of 4 in [4, 64]");
    if (c->scheme != ESBGK_ARS222 && c->scheme != ESBGK_ARS233) return fail(ESBGK_EINVAL, "bad scheme");
    if (c->recon != ESBGK_UPWIND1 && c->recon != ESBGK_MINMOD2) return fail(ESBGK_EINVAL, "bad recon");
    if (c->precision < ESBGK_FP64 || c->precision > ESBGK_MIXED) return fail(ESBGK_EINVAL, "bad precision");
    if (c->precision == ESBGK_MIXED && c->scheme != ESBGK_ARS233)
        return fail(ESBGK_EINVAL, "the mixed storage form needs ARS(2,3,3) (a separate final combination)");
    if (c->indicator != ESBGK_IND_PLAIN && c->indicator != ESBGK_IND_FROZEN && c->indicator != ESBGK_IND_LEARNED)
        return fail(ESBGK_EINVAL, "bad indicator mode");
    if (c->indicator == ESBGK_IND_LEARNED && c->learned_k < 1) return fail(ESBGK_EINVAL, "learned_k must be >= 1");
    if (c->coupling != ESBGK_COUPLE_STAGE && c->coupling != ESBGK_COUPLE_STEP) return fail(ESBGK_EINVAL, "bad coupling");
    if (!(c->lx > 0) || !(c->ly > 0) || !(c->vmax > 0)) return fail(ESBGK_EINVAL, "lx, ly, vmax must be > 0");
    if (!(c->tau > 0)) return fail(ESBGK_EINVAL, "tau must be > 0");
    if (!(c->beta >= -0.5 && c->beta < 1.0)) return fail(ESBGK_EINVAL, "beta must be in [-1/2, 1)");
    if (!(c->dt > 0) && !(c->cfl > 0)) return fail(ESBGK_EINVAL, "need dt > 0 or cfl > 0");
    if (!(c->eta > 0) || !(c->delta >= 0)) return fail(ESBGK_EINVAL, "eta must be > 0, delta >= 0");
    return ESBGK_OK;
}

struct Layout {
    size_t f[3], fP, U[4], D[3], gp, eps, l1, prim, mask, mask_old, cls, kin, buf, newk, blockcounts, counts, err,
        bad, kin_total;
    // learned indicator (indicator == LEARNED only)
    size_t derived, pmask, lcount;
    size_t total;
};

Layout layout(const esbgk_config *c) {
    Layout L;
    const size_t nc = (size_t)c->nx * c->ny, nv2 = (size_t)c->nv * c->nv;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    for (int q = 0; q < 3; ++q) L.f[q] = take(nc * nv2 * (q == 0 ? state_elem(c->precision) : stage_elem(c->precision)));
    // partial sum of the final combination (ARS(2,3,3)), state precision and at least FP32
    L.fP = take(c->scheme == ESBGK_ARS233 ? nc * nv2 * std::max<size_t>(4, state_elem(c->precision)) : 0);
    for (int q = 0; q < 4; ++q) L.U[q] = take(4 * nc * sizeof(double));
    // Euler flux divergences of the step's states, SoA [4][nc]
    for (int q = 0; q < 3; ++q) L.D[q] = take(4 * nc * sizeof(double));
    // Gaussian parameters of stage 2, read by stage 3 when the stage arrays are BF16
    L.gp = take(stage_gauss_params(c->precision) ? (size_t)GP_N * nc * sizeof(double) : 0);
    L.eps = take(nc * sizeof(double));
    L.l1 = take(nc * sizeof(double));
    L.prim = take(4 * nc * sizeof(double));
    L.mask = take(nc);
    L.mask_old = take(nc);
    L.cls = take(nc);
    L.kin = take(nc * sizeof(int));
    L.buf = take(nc * sizeof(int));
    L.newk = take(nc * sizeof(int));
    L.blockcounts = take(3 * (size_t)scan_nblocks(c->nx, c->ny) * sizeof(int));
    L.counts = take(4 * sizeof(int));
    L.err = take(sizeof(int));
    L.bad = take(sizeof(int));
    L.kin_total = take(sizeof(long long));
    const bool learned = c->indicator == ESBGK_IND_LEARNED;
    L.derived = take(learned ? 3 * nc * sizeof(double) : 0);
    L.pmask = take(learned ? nc : 0);
    L.lcount = take(learned ? 4 * sizeof(long long) : 0);
    L.total = off;
    return L;
}

}  // namespace

struct EventPool {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
};

struct esbgk_ctx {
    esbgk_config cfg{};
    int nc = 0, nv2 = 0;
    Geom g{};
    double At[9]{}, bt[3]{}, A[9]{}, b[3]{};
    char *ws = nullptr;
    void *f[3]{};
    void *fP = nullptr;
    double *U[4]{};
    double *gp = nullptr;  // BF16 stage arrays only
    double *D[3]{};        // Euler flux divergences of the step's states
    bool dvalid[3]{};      // D[j] holds the divergence of this step's U^(j)
    double *eps = nullptr, *l1 = nullptr, *prim = nullptr;
    uint8_t *mask = nullptr, *mask_old = nullptr, *cls = nullptr;
    int *kin = nullptr, *buf = nullptr, *newk = nullptr, *blockcounts = nullptr, *counts = nullptr,
        *err = nullptr, *bad = nullptr;
    long long *kin_total = nullptr;
    // learned indicator
    esbgk_mlp *net = nullptr;
    float threshold = 0.0f;
    int dilation = 0;
    double *lderived = nullptr;
    uint8_t *pmask = nullptr;
    long long *lcount = nullptr;
    int64_t steps = 0;
    double time = 0.0;
    bool have_state = false;
    bool timing = false;
    EventPool pool[ESBGK_K_COUNT];
    ~esbgk_ctx() {
        for (auto &p : pool) {
            for (auto e : p.start) (void)hipEventDestroy(e);
            for (auto e : p.stop) (void)hipEventDestroy(e);
        }
    }
};

namespace {

template <class SN, class SS> int run_step(esbgk_ctx *c, hipStream_t st);

// Events bracketing one launch of kernel class k (only while timing is on).
struct TimedLaunch {
    esbgk_ctx *c;
    int k;
    hipStream_t st;
    hipEvent_t stop = nullptr;
    hipError_t err = hipSuccess;
    TimedLaunch(esbgk_ctx *c_, int k_, hipStream_t st_) : c(c_), k(k_), st(st_) {
        if (!c->timing) return;
        EventPool &p = c->pool[k];
        if (p.used == p.start.size()) {
            hipEvent_t a, b;
            if ((err = hipEventCreate(&a)) != hipSuccess) return;
            if ((err = hipEventCreate(&b)) != hipSuccess) return;
            p.start.push_back(a);
            p.stop.push_back(b);
        }
        err = hipEventRecord(p.start[p.used], st);
        stop = p.stop[p.used];
        p.used++;
    }
    hipError_t done() {
        if (err != hipSuccess) return err;
        if (stop) return hipEventRecord(stop, st);
        return hipSuccess;
    }
};

// Lists of the current mask; `total` (may be null) accumulates the kinetic count.
int regime_lists(esbgk_ctx *c, const uint8_t *mask_old, hipStream_t st, long long *total = nullptr) {
    const int radius = c->cfg.recon == ESBGK_MINMOD2 ? 2 : 1;
    HIPCHK(launch_compact(c->mask, mask_old, c->cls, radius, c->cfg.nx, c->cfg.ny, c->blockcounts, c->counts, c->kin,
                          c->buf, c->newk, total, st));
    return ESBGK_OK;
}

template <class S> int fill_list(esbgk_ctx *c, void *f, const double *U, const int *list, const int *count,
                                 hipStream_t st, const void *ref_in = nullptr) {
    FillArgs<S> a;
    a.g = c->g; a.U = U; a.f = (S *)f; a.list = list; a.count = count; a.err = c->err; a.nc = c->nc;
    a.ref_in = (const float *)ref_in;
    TimedLaunch tl(c, ESBGK_K_FILL, st);
    HIPCHK(launch_fill<S>(a, c->nc, st));
    HIPCHK(tl.done());
    return ESBGK_OK;
}

template <class S> int moments_list(esbgk_ctx *c, const void *f, double *U, double *l1, const int *list,
                                    const int *count, hipStream_t st) {
    MomArgs<S> a;
    a.g = c->g; a.f = (const S *)f; a.U = U; a.l1 = l1; a.list = list; a.count = count; a.err = c->err;
    a.nc = c->nc;
    HIPCHK(launch_moments<S>(a, c->nc, st));
    return ESBGK_OK;
}

IndicatorArgs indicator_args(const esbgk_config *cfg) {
    IndicatorArgs a;
    memset(&a, 0, sizeof a);
    a.nx = cfg->nx; a.ny = cfg->ny; a.nc = cfg->nx * cfg->ny;
    const double dx = cfg->lx / cfg->nx, dy = cfg->ly / cfg->ny;
    a.twodx = 2.0 * dx; a.twody = 2.0 * dy;
    a.tau = cfg->tau; a.omb = 1.0 - cfg->beta;
    if (cfg->ce_set == 1) { a.cD = 1.0; a.ck = 2.0; a.cS = 1.0; }
    else { a.cD = 2.0 / 3.0; a.ck = 5.0 / 2.0; a.cS = 2.0 / 3.0; }
    a.eta = cfg->eta; a.delta = cfg->delta;
    return a;
}

// One IMEX stage (i = 1, 2) or the final combination (i = 3) on kinetic cells.
// An implicit term dt A_ij Q'_j of an earlier stage is taken as
// (A_ij / A_jj)(f^(j) - f*_j), f*_j rebuilt from the transport of f^n, which
// for the exact relaxation of stage j equals dt A_ij (tau/eps)(Ghat_j - f^(j)).
// With ARS(2,3,3) the last implicit stage also writes the partial sum
//   P' = f^n - dt sum_{j<3} bt_j L(f^(j)) + dt sum_{j<=3} b_j Q'_j
// (its transport and implicit terms are the ones the stage computes anyway,
// Q'_3 = (f^(3) - f*_3)/(dt A_33) once f^(3) is known), and the final
// combination is f^{n+1} = P' - dt bt_3 L(f^(3)).
template <class SN, class SS> int kinetic_stage(esbgk_ctx *c, int i, hipStream_t st, double *Uout) {
    StageArgs a;
    memset(&a, 0, sizeof a);
    a.g = c->g;
    a.eps = c->eps; a.list = c->kin; a.count = c->counts; a.err = c->err; a.nc = c->nc;
    a.Uout = Uout;
    a.l1out = c->l1;
    const bool partial = c->cfg.scheme == ESBGK_ARS233;
    // mixed form (FP32 state, BF16 stage arrays): increment storage -- f^(2) is
    // stored as f^(2) - f^n; stage 3 writes f^(3) in FP32 into the partial-sum
    // buffer and P - f^(3) into the BF16 array of f^(3)
    const bool inc = !std::is_same<SN, SS>::value;
    if (i < 3) {
        a.fn = c->f[0];
        const double *rowt = &c->At[3 * i], *rowi = &c->A[3 * i];
        for (int j = 0; j < i; ++j)
            if (rowt[j] != 0.0 || (partial && i == 2 && c->bt[j] != 0.0)) {
                a.fl[a.nl] = c->f[j]; a.cl[a.nl] = rowt[j]; a.scl[a.nl] = c->bt[j]; ++a.nl;
            }
        for (int j = 1; j < i; ++j)
            if (rowi[j] != 0.0) {
                // f*_j of stage j = 2 involves f^n only (A_21 = 0)
                if (j != 1 || a.nq != 0 || c->A[3] != 0.0 || !(c->A[4] > 0.0))
                    return fail(ESBGK_EINVAL, "tableau not supported by the kinetic stage kernels");
                a.fq[0] = c->f[j]; a.qa = rowi[j]; a.qd = c->A[3 * j + j]; a.ctn = c->At[3 * j]; ++a.nq;
                a.qb = c->b[j];
                a.pq = c->gp;
            }
        a.aii = c->A[3 * i + i];
        a.fout = c->f[i];
        if (i == 1) a.pout = c->gp;  // null unless the stage arrays are BF16
        if (partial && i == 2) {
            // the one implicit term of stage 3 is that of stage 2
            if (a.nq != 1 || c->b[0] != 0.0) return fail(ESBGK_EINVAL, "tableau not supported by the partial sum");
            a.sout = c->fP;
            a.sfin = c->b[2] / c->A[8];
            if (inc) std::swap(a.fout, a.sout);  // f^(3) in FP32, P' - f^(3) in the BF16 stage array
        }
        // ARS(2,2,2) is stiffly accurate: its last stage is f^{n+1}
        a.emit = (i == 2 && c->cfg.scheme == ESBGK_ARS222) ? 1 : 0;
    } else {
        void *f3 = inc ? c->fP : c->f[2], *part = inc ? c->f[2] : c->fP;
        a.fn = part;
        a.fl[0] = f3; a.cl[0] = c->bt[2]; a.nl = 1;
        a.aii = 0.0;
        a.fout = c->f[0];  // f^n is not read by the final combination
        a.emit = 1;
    }
    TimedLaunch tl(c, i == 1 ? ESBGK_K_STAGE2 : i == 2 ? ESBGK_K_STAGE3 : ESBGK_K_FINAL, st);
    HIPCHK((launch_stage<SN, SS>(a, c->nc, st)));
    HIPCHK(tl.done());
    return ESBGK_OK;
}

int euler_stage(esbgk_ctx *c, int i, hipStream_t st, double *Uout) {
    EulerArgs e;
    memset(&e, 0, sizeof e);
    e.nx = c->cfg.nx; e.ny = c->cfg.ny; e.nc = c->nc; e.recon = c->cfg.recon;
    e.dx = c->g.dx; e.dy = c->g.dy; e.dt = c->g.dt;
    e.Un = c->U[0];
    const double *rowt = i < 3 ? &c->At[3 * i] : c->bt;
    const int nprev = i < 3 ? i : 3;
    // the divergence of the newest state U^(i-1) is formed now and stored;
    // those of earlier states were stored by the earlier stages of this step
    e.jnew = -1;
    for (int j = 0; j < nprev; ++j)
        if (rowt[j] != 0.0) {
            if (j == i - 1) e.jnew = e.nj;
            else if (!c->dvalid[j]) return fail(ESBGK_EINVAL, "tableau not supported by the Euler stage");
            e.Uj[e.nj] = c->U[j]; e.Dj[e.nj] = c->D[j]; e.cj[e.nj] = rowt[j]; ++e.nj;
        }
    e.Dout = c->D[i - 1];
    c->dvalid[i - 1] = true;
    e.Uout = Uout;
    e.mask = c->mask;
    HIPCHK(launch_euler(e, st));
    return ESBGK_OK;
}

// Regime update of a check step of the learned indicator: the plain criterion
// P (the fallback and the judge), and the mask for the next learned_k steps,
// P | (network logit > threshold), or, without a network, P dilated by
// `dilation` cells (the plain-every-K baseline).  Counts the cells where P
// disagrees with the mask that was in use (missed: P and not in use; extra:
// in use and not P).
int learned_update(esbgk_ctx *c, hipStream_t st) {
    if (!c->net && c->dilation < 0) return fail(ESBGK_EINVAL, "learned indicator without a network or dilation");
    HIPCHK(launch_prim(c->U[0], c->prim, c->nc, st));
    std::swap(c->mask_old, c->mask);
    IndicatorArgs ia = indicator_args(&c->cfg);
    ia.U = c->U[0]; ia.eps = c->eps; ia.l1 = c->l1; ia.mask_old = c->mask_old; ia.mask_new = c->pmask;
    HIPCHK(launch_indicator(ia, st));
    long long *counters = c->steps > 0 ? c->lcount : nullptr;
    if (c->net) {
        HIPCHK(launch_learned_mask(c->net, c->cfg.nx, c->cfg.ny, c->cfg.lx, c->cfg.ly, c->prim, c->eps, c->mask_old,
                                   c->lderived, c->pmask, c->threshold, c->mask, counters, st));
    } else {
        HIPCHK(launch_learned_combine(c->pmask, nullptr, 0.0f, c->dilation, c->mask_old, c->mask, c->cls,
                                      c->cfg.nx, c->cfg.ny, counters, st));
    }
    return ESBGK_OK;
}

template <class SN, class SS> int run_step(esbgk_ctx *c, hipStream_t st) {
    const size_t nc = (size_t)c->nc;
    const bool loc = c->cfg.coupling == ESBGK_COUPLE_STEP;
    int rc;
    for (bool &v : c->dvalid) v = false;
    // ---- regime update (Algorithm 1: at the start of every step)
    if (c->cfg.indicator == ESBGK_IND_PLAIN) {
        std::swap(c->mask_old, c->mask);  // the indicator writes the new mask from the previous one
        IndicatorArgs ia = indicator_args(&c->cfg);
        ia.U = c->U[0]; ia.eps = c->eps; ia.l1 = c->l1; ia.mask_old = c->mask_old; ia.mask_new = c->mask;
        HIPCHK(launch_indicator(ia, st));
        if ((rc = regime_lists(c, c->mask_old, st, c->kin_total))) return rc;
        // fluid -> kinetic: f = Mhat(U) (eq. Coupling_FluKin); kinetic -> fluid keeps U = moments(f)
        if ((rc = fill_list<SN>(c, c->f[0], c->U[0], c->newk, c->counts + 2, st))) return rc;
    } else if (c->cfg.indicator == ESBGK_IND_LEARNED && c->steps % c->cfg.learned_k == 0) {
        if ((rc = learned_update(c, st))) return rc;
        if ((rc = regime_lists(c, c->mask_old, st, c->kin_total))) return rc;
        if ((rc = fill_list<SN>(c, c->f[0], c->U[0], c->newk, c->counts + 2, st))) return rc;
    } else {
        HIPCHK(launch_accumulate_count(c->counts, c->kin_total, st));  // the lists are unchanged
    }
    // ---- stage 1 coupling: buffer cells carry Mhat(U^n)
    if ((rc = fill_list<SN>(c, c->f[0], c->U[0], c->buf, c->counts + 1, st))) return rc;
    // ---- stages 2 and 3
    for (int i = 1; i <= 2; ++i) {
        const bool last222 = (i == 2 && c->cfg.scheme == ESBGK_ARS222);
        double *Ukin = c->U[i];
        if (loc) {
            // low-order coupling: fluid cells keep seeing the kinetic cells' U^n
            HIPCHK(hipMemcpyAsync(c->U[i], c->U[0], 4 * nc * sizeof(double), hipMemcpyDeviceToDevice, st));
            if (!last222) Ukin = c->U[3];
        }
        if ((rc = kinetic_stage<SN, SS>(c, i, st, Ukin))) return rc;
        if ((rc = euler_stage(c, i, st, c->U[i]))) return rc;
        if (!last222) {
            const double *Ub = loc ? c->U[0] : c->U[i];
            // mixed form: the BF16 array f^(2) holds f^(2) - f^n; f^(3) is kept in FP32
            // in the partial-sum buffer (see kinetic_stage)
            if (!std::is_same<SN, SS>::value && i == 2) {
                if ((rc = fill_list<SN>(c, c->fP, Ub, c->buf, c->counts + 1, st))) return rc;
            } else if ((rc = fill_list<SS>(c, c->f[i], Ub, c->buf, c->counts + 1, st,
                                           std::is_same<SN, SS>::value ? nullptr : c->f[0]))) {
                return rc;
            }
        }
    }
    if (c->cfg.scheme == ESBGK_ARS233) {
        // ---- final combination (eq. RKEI2 / RKEuler_2), then coupling of U^{n+1}
        if ((rc = kinetic_stage<SN, SS>(c, 3, st, c->U[3]))) return rc;
        if ((rc = euler_stage(c, 3, st, c->U[3]))) return rc;
        std::swap(c->U[0], c->U[3]);
    } else {
        // stiffly accurate: f^{n+1} = f^(3), U^{n+1} = U^(3)
        std::swap(c->f[0], c->f[2]);
        std::swap(c->U[0], c->U[2]);
    }
    return ESBGK_OK;
}

template <class S> int set_f_impl(esbgk_ctx *c, const double *d_f, hipStream_t st) {
    const size_t n = (size_t)c->nc * c->nv2;
    HIPCHK(launch_from_f64<S>(d_f, c->f[0], n, st));
    HIPCHK(hipMemsetAsync(c->mask_old, 0, c->nc, st));
    HIPCHK(hipMemsetAsync(c->mask, 1, c->nc, st));
    int rc = regime_lists(c, nullptr, st);
    if (rc) return rc;
    return moments_list<S>(c, c->f[0], c->U[0], c->l1, c->kin, c->counts, st);
}

template <class S> int set_mask_impl(esbgk_ctx *c, const uint8_t *d_mask, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(c->mask_old, c->mask, c->nc, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->mask, d_mask, c->nc, hipMemcpyDeviceToDevice, st));
    int rc = regime_lists(c, c->mask_old, st);
    if (rc) return rc;
    if ((rc = fill_list<S>(c, c->f[0], c->U[0], c->newk, c->counts + 2, st))) return rc;
    // fresh L1 distances for the kinetic cells
    return moments_list<S>(c, c->f[0], c->U[0], c->l1, c->kin, c->counts, st);
}

int check_ptr(const void *p, size_t align, const char *what) {
    if (!p) return fail(ESBGK_EINVAL, "%s is null", what);
    if ((uintptr_t)p % align) return fail(ESBGK_EINVAL, "%s is not %zu-byte aligned", what, align);
    return ESBGK_OK;
}

}  // namespace

extern "C" {

const char *esbgk_last_error(void) { return g_err; }

int esbgk_workspace_size(const esbgk_config *cfg, size_t *bytes) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!bytes) return fail(ESBGK_EINVAL, "null output");
    *bytes = layout(cfg).total;
    return ESBGK_OK;
}

int esbgk_create(const esbgk_config *cfg, void *d_workspace, size_t bytes, esbgk_ctx **out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(ESBGK_EINVAL, "null output");
    if ((rc = check_ptr(d_workspace, 256, "workspace"))) return rc;
    Layout L = layout(cfg);
    if (bytes < L.total) return fail(ESBGK_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, L.total);
    esbgk_ctx *c = new (std::nothrow) esbgk_ctx();
    if (!c) return fail(ESBGK_EINVAL, "host allocation failed");
    c->cfg = *cfg;
    c->nc = cfg->nx * cfg->ny;
    c->nv2 = cfg->nv * cfg->nv;
    Geom &g = c->g;
    g.nx = cfg->nx; g.ny = cfg->ny; g.nv = cfg->nv; g.nv2 = c->nv2;
    g.dx = cfg->lx / cfg->nx; g.dy = cfg->ly / cfg->ny;
    g.idx = 1.0 / g.dx; g.idy = 1.0 / g.dy;
    g.vmax = cfg->vmax;
    g.dv = 2.0 * cfg->vmax / (double)cfg->nv;
    g.w = g.dv * g.dv;
    g.beta = cfg->beta; g.tau = cfg->tau;
    g.dt = cfg->dt > 0 ? cfg->dt : cfg->cfl * std::min(g.dx, g.dy) / cfg->vmax;
    g.recon = cfg->recon; g.correction = cfg->correction;
    tableau(cfg->scheme, c->At, c->bt, c->A, c->b);
    char *w = (char *)d_workspace;
    c->ws = w;
    for (int q = 0; q < 3; ++q) c->f[q] = w + L.f[q];
    c->fP = w + L.fP;
    for (int q = 0; q < 4; ++q) c->U[q] = (double *)(w + L.U[q]);
    for (int q = 0; q < 3; ++q) c->D[q] = (double *)(w + L.D[q]);
    c->gp = stage_gauss_params(cfg->precision) ? (double *)(w + L.gp) : nullptr;
    c->eps = (double *)(w + L.eps);
    c->l1 = (double *)(w + L.l1);
    c->prim = (double *)(w + L.prim);
    c->mask = (uint8_t *)(w + L.mask);
    c->mask_old = (uint8_t *)(w + L.mask_old);
    c->cls = (uint8_t *)(w + L.cls);
    c->kin = (int *)(w + L.kin);
    c->buf = (int *)(w + L.buf);
    c->newk = (int *)(w + L.newk);
    c->blockcounts = (int *)(w + L.blockcounts);
    c->counts = (int *)(w + L.counts);
    c->err = (int *)(w + L.err);
    c->bad = (int *)(w + L.bad);
    c->kin_total = (long long *)(w + L.kin_total);
    if (cfg->indicator == ESBGK_IND_LEARNED) {
        c->lderived = (double *)(w + L.derived);
        c->pmask = (uint8_t *)(w + L.pmask);
        c->lcount = (long long *)(w + L.lcount);
    }
    *out = c;
    return ESBGK_OK;
}

void esbgk_destroy(esbgk_ctx *ctx) { delete ctx; }

int esbgk_set_state(esbgk_ctx *c, const double *d_rho, const double *d_ux, const double *d_uy,
                    const double *d_T, const double *d_eps, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_rho, 8, "rho")) || (rc = check_ptr(d_ux, 8, "ux")) || (rc = check_ptr(d_uy, 8, "uy")) ||
        (rc = check_ptr(d_T, 8, "T")) || (rc = check_ptr(d_eps, 8, "eps")))
        return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->err, 0, sizeof(int), st));
    HIPCHK(launch_conserved(d_rho, d_ux, d_uy, d_T, d_eps, c->U[0], c->eps, c->nc, c->bad, st));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) return fail(ESBGK_EINVAL, "set_state: non-finite or non-positive rho, T or eps");
    HIPCHK(hipMemsetAsync(c->mask, 0, c->nc, st));
    HIPCHK(hipMemsetAsync(c->mask_old, 0, c->nc, st));
    HIPCHK(hipMemsetAsync(c->l1, 0, c->nc * sizeof(double), st));
    HIPCHK(hipMemsetAsync(c->kin_total, 0, sizeof(long long), st));
    if (c->lcount) HIPCHK(hipMemsetAsync(c->lcount, 0, 4 * sizeof(long long), st));
    if ((rc = regime_lists(c, nullptr, st))) return rc;
    c->steps = 0;
    c->time = 0.0;
    c->have_state = true;
    return ESBGK_OK;
}

int esbgk_set_mask(esbgk_ctx *c, const uint8_t *d_mask, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!c->have_state) return fail(ESBGK_EINVAL, "set_mask before set_state");
    int rc;
    if ((rc = check_ptr(d_mask, 1, "mask"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    switch (c->cfg.precision) {
        case ESBGK_FP64: return set_mask_impl<double>(c, d_mask, st);
        case ESBGK_BF16: return set_mask_impl<bf16_t>(c, d_mask, st);
        default: return set_mask_impl<float>(c, d_mask, st);
    }
}

int esbgk_set_f(esbgk_ctx *c, const double *d_f, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!c->have_state) return fail(ESBGK_EINVAL, "set_f before set_state");
    int rc;
    if ((rc = check_ptr(d_f, 16, "f"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    switch (c->cfg.precision) {
        case ESBGK_FP64: return set_f_impl<double>(c, d_f, st);
        case ESBGK_BF16: return set_f_impl<bf16_t>(c, d_f, st);
        default: return set_f_impl<float>(c, d_f, st);
    }
}

int esbgk_step(esbgk_ctx *c, int nsteps, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!c->have_state) return fail(ESBGK_EINVAL, "step before set_state");
    if (nsteps < 0) return fail(ESBGK_EINVAL, "nsteps < 0");
    hipStream_t st = (hipStream_t)stream;
    for (int n = 0; n < nsteps; ++n) {
        int rc;
        switch (c->cfg.precision) {
            case ESBGK_FP64: rc = run_step<double, double>(c, st); break;
            case ESBGK_FP32: rc = run_step<float, float>(c, st); break;
            case ESBGK_BF16: rc = run_step<bf16_t, bf16_t>(c, st); break;
            default: rc = run_step<float, bf16_t>(c, st); break;
        }
        if (rc) return rc;
        c->steps += 1;
        c->time += c->g.dt;
    }
    return ESBGK_OK;
}

int esbgk_get_moments(esbgk_ctx *c, double *d_rho, double *d_ux, double *d_uy, double *d_T, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    HIPCHK(launch_get_prim(c->U[0], d_rho, d_ux, d_uy, d_T, c->nc, (hipStream_t)stream));
    return ESBGK_OK;
}

int esbgk_get_conserved(esbgk_ctx *c, double *d_U, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_U, 8, "U"))) return rc;
    HIPCHK(hipMemcpyAsync(d_U, c->U[0], 4 * (size_t)c->nc * sizeof(double), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return ESBGK_OK;
}

int esbgk_get_mask(esbgk_ctx *c, uint8_t *d_mask, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_mask, 1, "mask"))) return rc;
    HIPCHK(hipMemcpyAsync(d_mask, c->mask, c->nc, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return ESBGK_OK;
}

int esbgk_get_f(esbgk_ctx *c, double *d_f, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_f, 16, "f"))) return rc;
    const size_t n = (size_t)c->nc * c->nv2;
    hipStream_t st = (hipStream_t)stream;
    switch (c->cfg.precision) {
        case ESBGK_FP64: HIPCHK(launch_to_f64<double>(c->f[0], d_f, n, st)); break;
        case ESBGK_BF16: HIPCHK(launch_to_f64<bf16_t>(c->f[0], d_f, n, st)); break;
        default: HIPCHK(launch_to_f64<float>(c->f[0], d_f, n, st)); break;
    }
    return ESBGK_OK;
}

int esbgk_get_l1(esbgk_ctx *c, double *d_l1, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_l1, 8, "l1"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(d_l1, c->l1, (size_t)c->nc * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_zero_fluid_l1(c->mask, d_l1, c->nc, st));
    return ESBGK_OK;
}

int esbgk_get_kinetic_cells(esbgk_ctx *c, int32_t *d_cells, int32_t *h_count, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    int rc;
    if ((rc = check_ptr(d_cells, 4, "cells")) || (rc = check_ptr(h_count, 4, "count"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(d_cells, c->kin, (size_t)c->nc * sizeof(int), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(h_count, c->counts, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ESBGK_OK;
}

int esbgk_get_stats(esbgk_ctx *c, esbgk_stats *out, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!out) return fail(ESBGK_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    int counts[4] = {0, 0, 0, 0}, err = 0;
    long long total = 0;
    HIPCHK(hipMemcpyAsync(counts, c->counts, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&total, c->kin_total, sizeof(long long), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&err, c->err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memset(out, 0, sizeof *out);
    out->steps = c->steps;
    out->time = c->time;
    out->dt = c->g.dt;
    out->n_kinetic = counts[0];
    out->n_buffer = counts[1];
    out->error_flags = err;
    out->kinetic_cell_steps = total;
    if (err) return fail(ESBGK_ENONPHYS, "non-physical state met during a step (flags 0x%x)", err);
    return ESBGK_OK;
}

int esbgk_set_learned(esbgk_ctx *c, esbgk_mlp *net, float threshold, int dilation) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (c->cfg.indicator != ESBGK_IND_LEARNED) return fail(ESBGK_EINVAL, "context not configured for the learned indicator");
    if (!net && dilation < 0) return fail(ESBGK_EINVAL, "need a network or a dilation radius >= 0");
    if (dilation > 64) return fail(ESBGK_EINVAL, "dilation radius > 64");
    if (!(threshold == threshold)) return fail(ESBGK_EINVAL, "threshold is NaN");
    c->net = net;
    c->threshold = threshold;
    c->dilation = net ? 0 : dilation;
    return ESBGK_OK;
}

int esbgk_get_learned_stats(esbgk_ctx *c, int64_t *h_out, void *stream) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!h_out) return fail(ESBGK_EINVAL, "null output");
    if (!c->lcount) return fail(ESBGK_EINVAL, "context not configured for the learned indicator");
    long long v[4];
    HIPCHK(hipMemcpyAsync(v, c->lcount, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    for (int q = 0; q < 4; ++q) h_out[q] = v[q];
    return ESBGK_OK;
}

int esbgk_set_timing(esbgk_ctx *c, int enable) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    c->timing = enable != 0;
    return ESBGK_OK;
}

int esbgk_kernel_times(esbgk_ctx *c, double *h_ms, int64_t *h_launches, int reset) {
    if (!c) return fail(ESBGK_EINVAL, "null context");
    if (!h_ms || !h_launches) return fail(ESBGK_EINVAL, "null output");
    for (int k = 0; k < ESBGK_K_COUNT; ++k) {
        EventPool &p = c->pool[k];
        double sum = 0.0;
        for (size_t q = 0; q < p.used; ++q) {
            HIPCHK(hipEventSynchronize(p.stop[q]));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, p.start[q], p.stop[q]));
            sum += ms;
        }
        h_ms[k] = sum;
        h_launches[k] = (int64_t)p.used;
        if (reset) p.used = 0;
    }
    return ESBGK_OK;
}

int esbgk_indicator(const esbgk_config *cfg, const double *d_prim, const double *d_eps, const double *d_l1,
                    const uint8_t *d_mask_old, uint8_t *d_mask_new, double *d_lambda, void *stream) {
    int rc = validate(cfg);
    if (rc) return rc;
    if ((rc = check_ptr(d_prim, 8, "prim")) || (rc = check_ptr(d_eps, 8, "eps")) || (rc = check_ptr(d_l1, 8, "l1")) ||
        (rc = check_ptr(d_mask_old, 1, "mask_old")) || (rc = check_ptr(d_mask_new, 1, "mask_new")))
        return rc;
    IndicatorArgs a = indicator_args(cfg);
    a.prim = d_prim; a.eps = d_eps; a.l1 = d_l1; a.mask_old = d_mask_old; a.mask_new = d_mask_new;
    a.lambda = d_lambda;
    HIPCHK(launch_indicator(a, (hipStream_t)stream));
    return ESBGK_OK;
}

}  // extern "C"
