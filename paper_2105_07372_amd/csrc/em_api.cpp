// Host side of libsynchem: argument validation, device buffers, launch sequencing on the caller's
// HIP stream.  Declarations and semantics: include/synchem.h.
#include "synchem.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "em_internal.h"

using namespace sem;

namespace {

thread_local std::string g_err;   // last em_init / em_learn_prior failure on this thread

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

constexpr int kTimingEvents = 512;

}  // namespace

struct em_ctx {
    // problem
    int64_t N = 0;
    int K = 0, Q = 0, D = 0, Dp = 0, L = 0, lo = 0, W = 0, Wp = 0;
    double sigma2 = 0, gamma = 0;
    int update_rho = 1, prec = 0;
    uint64_t flags = 0;
    bool has_gai = false;
    // plan
    int BM = 0, WM = 0, grid = 0, ncols = 0, colsum_grid = 0;
    int LD = 0;           // general pass: 1 = tile double-buffered by direct global-to-LDS copies
    bool ks = false;      // K-split pass (template resident in registers)
    int ksNT = 0, ksKSS = 0;
    bool wide = false;    // wide-row pass (rows streamed through an LDS ring, 128-row tiles)
    int wNTW = 0, wUR = 0;
    bool fac = false;     // factored pass (per-frequency sums; no template)
    bool fs = false;      // ... and its symmetric-window form for the EM and log-likelihood passes
    int fsMTW = 0, fsE = 8;
    size_t fsLds = 0;
    bool kr = false;      // row-stream correlation pass (template in registers, rows via LDS)
    int krNT = 0;
    bool gm = false;      // long-window FP32 pass (GEMM with a posterior / M-step epilogue)
    int gmNT = 0;
    int fWIDE = 0, fKCM = 0, fEPL = 8;
    bool has_angles = false;   // the window is an explicit angle list (em_params.angles)
    int64_t rowbytes = 0;
    size_t lds = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    // device buffers
    uint8_t *V = nullptr;
    float *rowscale = nullptr;
    double *vnorm2 = nullptr;
    double sum_vn2 = 0;
    void *Thi = nullptr, *Tlo = nullptr, *ThiE = nullptr, *TloE = nullptr;
    float *tscale = nullptr, *tscaleE = nullptr;
    float *E2 = nullptr;
    double2 *E64 = nullptr, *phase = nullptr;
    float *logrho32 = nullptr, *logrho32E = nullptr;
    double *logrho64 = nullptr, *logrho64E = nullptr;
    double *a = nullptr, *rho = nullptr, *rho_bar = nullptr, *gai = nullptr;
    double *aE = nullptr, *rhoE = nullptr;
    int64_t *t = nullptr;
    int *stopped = nullptr, *nonfinite = nullptr;
    unsigned *fin_count = nullptr;     // the reduce-and-finalize launch's done counter
    double *ll_last = nullptr, *stats = nullptr, *partials = nullptr, *red = nullptr;
    double *scal = nullptr;  // [0] ll, [1] grad sigma2
    double *lse = nullptr;
    // fwd/bwd state
    bool fwd_valid = false;
    double sigma2E = 0;
    bool etaE = false;
    // timing
    bool timing = false;
    hipEvent_t ev[2 * kTimingEvents] = {};
    int ev_used = 0;
    double pass_ms = 0;
    int64_t pass_count = 0;
    std::vector<void *> allocs;
    std::string err;
};

namespace {

em_status fail(em_ctx *c, em_status s, const std::string &msg) {
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return s;
}

// Waits for a call's work on its stream whatever happened (the call's scratch is freed on
// return) and keeps the first error.
hipError_t finish(hipError_t e, hipStream_t s) {
    const hipError_t se = hipStreamSynchronize(s);
    return e != hipSuccess ? e : se;
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), EM_EDEVICE,                                                     \
                        std::string(#call) + " failed: " + hipGetErrorString(e_));            \
    } while (0)

bool finite_all(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

em_status dev_alloc(em_ctx *c, void **p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, EM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    c->allocs.push_back(*p);
    return EM_OK;
}

template <typename T>
em_status alloc_t(em_ctx *c, T **p, size_t count) {
    return dev_alloc(c, (void **)p, count * sizeof(T));
}

int pow2_floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// Waves over row blocks of the general pass for BM rows per tile: the eight waves split into
// WM row groups x WN window groups (WN a power of two up to the window tiles).
int pass_wm(int prec, int Wp, int BM) {
    const int NT = Wp / 16;
    const int WN = pow2_floor(NT < 8 ? NT : 8);
    int WM = 8 / WN;
    if (WM > BM / 16) WM = BM / 16 > 0 ? BM / 16 : 1;
    if (prec == P_F64) WM = 1;
    return WM;
}

// Choose rows per tile and the wave split of the pass for this problem.
em_status plan(em_ctx *c, size_t lds_max) {
    c->ks = false;
    c->wide = false;
    c->fac = false;
    c->fs = false;
    c->kr = false;
    c->gm = false;
    if (c->flags & EM_FLAG_FACTORED) {
        int WIDE = 0, KCM = 0, EPL = 8, BM = 0;
        size_t lds = 0;
        if (c->prec != P_F64 &&
            fac_plan(c->prec, c->D, c->Q, c->K, c->Wp, c->has_angles ? 0 : c->L, lds_max, &WIDE,
                     &KCM, &EPL, &lds, &BM)) {
            c->fac = true;
            c->BM = BM;
            c->fWIDE = WIDE;
            c->fKCM = KCM;
            c->fEPL = EPL;
            c->WM = 0;
            c->lds = lds;
            int MTW = 0, E = 8;
            size_t fl = 0;
            if (fs_plan(c->prec, c->D, c->Q, c->K, c->L, c->lo, c->W, c->Wp, !c->has_angles,
                        lds_max, &MTW, &E, &fl)) {
                c->fs = true;
                c->fsMTW = MTW;
                c->fsE = E;
                c->fsLds = fl;
            }
            return EM_OK;
        }
        return fail(c, EM_EUNSUPPORTED,
                    "the factored pass needs D = 512 with Q a power-of-two multiple of 8 and a "
                    "matrix-core precision, or D = 2048 in fp16 / bf16 with Q a power-of-two "
                    "multiple of 16");
    }
    const bool one_plane = c->prec == P_F16 || c->prec == P_BF16;
    if (one_plane && (c->flags & EM_FLAG_WIDE_PASS)) {
        int NTW = 0, UR = 0;
        if (wide_plan(c->prec, c->Wp, c->K, lds_max, &NTW, &UR)) {
            c->wide = true;
            c->BM = kWideBM;
            c->wNTW = NTW;
            c->wUR = UR;
            c->WM = 0;
            c->lds = wide_lds_bytes(c->K, c->Wp, NTW, UR);
            return EM_OK;
        }
        return fail(c, EM_EUNSUPPORTED, "no wide-row pass variant for this window and K");
    }
    if (c->prec == P_F32 && !(c->flags & EM_FLAG_GENERAL_PASS)) {
        int NT = 0;
        size_t lds = 0;
        if (gm_plan(c->prec, c->D, c->K, c->Q, c->Wp, lds_max, &NT, &lds)) {
            c->gm = true;
            c->BM = 128;
            c->gmNT = NT;
            c->WM = 0;
            c->lds = lds;
            return EM_OK;
        }
    }
    if (one_plane && !(c->flags & (EM_FLAG_GENERAL_PASS | EM_FLAG_STAGED_PASS))) {
        int NT = 0;
        size_t lds = 0;
        if (kr_plan(c->prec, c->D, c->Dp, c->Q, c->Wp, lds_max, &NT, &lds)) {
            c->kr = true;
            c->BM = 16;
            c->krNT = NT;
            c->WM = 0;
            c->lds = lds;
            return EM_OK;
        }
    }
    if (c->prec != P_F64 && c->prec != P_F32 && !(c->flags & EM_FLAG_GENERAL_PASS)) {
        int BM = 0, NT = 0, KSS = 0;
        if (ks_plan(c->prec, c->Dp, c->Wp, c->K, &BM, &NT, &KSS)) {
            const size_t lds = ks_lds_bytes(c->prec, BM, NT, c->K, c->Dp, c->Wp);
            if (lds <= lds_max && (int64_t)BM * c->K <= 16 * kThreads) {
                c->ks = true;
                c->BM = BM;
                c->ksNT = NT;
                c->ksKSS = KSS;
                c->WM = 0;
                c->lds = lds;
                return EM_OK;
            }
        }
    }
    const int cands_mfma[] = {64, 32, 16};
    const int cands_f64[] = {32, 16, 8};
    const int *cands = c->prec == P_F64 ? cands_f64 : cands_mfma;
    const int ncand = 3;
    c->BM = 0;
    // first choice: double-buffered tiles (rows of whole KiB), then register staging
    for (int LD = (c->rowbytes % 1024 == 0) ? 1 : 0; LD >= 0 && !c->BM; --LD) {
        for (int k = 0; k < ncand; ++k) {
            const int BM = cands[k];
            if (!LD && (int64_t)BM * c->rowbytes > (int64_t)kRegTileChunks * kThreads * 16) continue;
            const size_t lds = pass_lds_bytes(c->prec, BM, c->K, c->Dp, c->Wp, LD);
            if (lds > lds_max) continue;
            if (BM > 16 && (int64_t)BM / 2 >= c->N) continue;          // tiny N: small tiles
            if (BM < 16 && LD) continue;
            const int WM = pass_wm(c->prec, c->Wp, BM);
            if (!pass_variant_exists(c->prec, BM, WM, LD)) continue;   // no kernel built for it
            c->BM = BM;
            c->LD = LD;
            c->WM = WM;
            c->lds = lds;
            break;
        }
    }
    if (!c->BM && one_plane) {
        // rows too long for a tile in LDS: stream them through the wide-row pass
        int NTW = 0, UR = 0;
        if (wide_plan(c->prec, c->Wp, c->K, lds_max, &NTW, &UR)) {
            c->wide = true;
            c->BM = kWideBM;
            c->wNTW = NTW;
            c->wUR = UR;
            c->WM = 0;
            c->lds = wide_lds_bytes(c->K, c->Wp, NTW, UR);
            return EM_OK;
        }
    }
    if (!c->BM)
        return fail(c, EM_EUNSUPPORTED,
                    "no E+M pass fits rows of " + std::to_string(c->rowbytes) +
                        " bytes with this window");
    return EM_OK;
}

em_status check_params(const em_params *p) {
    if (!p) return fail(nullptr, EM_EINVAL, "params is NULL");
    if (p->n_obs < 1) return fail(nullptr, EM_EINVAL, "n_obs must be >= 1");
    if (p->K < 1 || p->Q < 1) return fail(nullptr, EM_EINVAL, "K and Q must be >= 1");
    if (p->L < 1) return fail(nullptr, EM_EINVAL, "L must be >= 1");
    if (p->angles) {
        if (p->window_count < 1) return fail(nullptr, EM_EINVAL, "window_count must be >= 1");
        if (p->window_lo != 0) return fail(nullptr, EM_EINVAL, "window_lo must be 0 with angles");
        if (!finite_all(p->angles, p->window_count))
            return fail(nullptr, EM_EINVAL, "angles must be finite");
    } else if (p->window_count < 1 || p->window_count > p->L) {
        return fail(nullptr, EM_EINVAL, "window_count must be in [1, L]");
    }
    if (!(p->sigma2 > 0) || !std::isfinite(p->sigma2))
        return fail(nullptr, EM_EINVAL, "sigma2 must be positive and finite");
    if (!(p->gamma >= 0) || !std::isfinite(p->gamma))
        return fail(nullptr, EM_EINVAL, "gamma must be >= 0 and finite");
    if (p->update_rho != 0 && p->update_rho != 1)
        return fail(nullptr, EM_EINVAL, "update_rho must be 0 or 1");
    if (p->precision < EM_FP64 || p->precision > EM_BF16)
        return fail(nullptr, EM_EINVAL, "unknown precision");
    if (p->flags & ~(uint64_t)(EM_FLAG_KEEP_LSE | EM_FLAG_TIMING | EM_FLAG_GENERAL_PASS |
                               EM_FLAG_WIDE_PASS | EM_FLAG_FACTORED | EM_FLAG_STAGED_PASS))
        return fail(nullptr, EM_EINVAL, "unknown flag bits");
    if (p->window_lo < -(1 << 30) || p->window_lo > (1 << 30))
        return fail(nullptr, EM_EINVAL, "window_lo out of range");
    const int64_t D = (int64_t)p->K * p->Q;
    if (p->gamma_a_inv) {
        for (int64_t d = 0; d < D; ++d)
            if (!(p->gamma_a_inv[d] >= 0) || !std::isfinite(p->gamma_a_inv[d]))
                return fail(nullptr, EM_EINVAL, "gamma_a_inv entries must be finite and >= 0");
    }
    if (p->a0 && !finite_all(p->a0, 2 * D))
        return fail(nullptr, EM_EINVAL, "a0 must be finite");
    if (D > kMaxD) return fail(nullptr, EM_EUNSUPPORTED, "D = K*Q above 2048");
    if (p->K > kMaxK) return fail(nullptr, EM_EUNSUPPORTED, "K above 512");
    if (p->window_count > kMaxWp) return fail(nullptr, EM_EUNSUPPORTED, "window above 1024");
    if (p->L > (1 << 24)) return fail(nullptr, EM_EUNSUPPORTED, "L above 2^24");
    return EM_OK;
}

em_status check_prior(const double *prior, int W, std::vector<double> &out, em_ctx *c) {
    out.assign(W, 1.0 / W);
    if (!prior) return EM_OK;
    double s = 0;
    for (int i = 0; i < W; ++i) {
        if (!(prior[i] >= 0) || !std::isfinite(prior[i]))
            return fail(c, EM_EINVAL, "prior entries must be finite and >= 0");
        s += prior[i];
    }
    if (!(s > 0)) return fail(c, EM_EINVAL, "prior must have a positive sum");
    for (int i = 0; i < W; ++i) out[i] = prior[i] / s;
    return EM_OK;
}

void logrho_host(const std::vector<double> &rho, int Wp, std::vector<float> &l32,
                 std::vector<double> &l64) {
    l32.assign(Wp, -INFINITY);
    l64.assign(Wp, -INFINITY);
    for (size_t i = 0; i < rho.size(); ++i) {
        const double l = rho[i] > 0 ? std::log(rho[i]) : -INFINITY;
        l32[i] = (float)l;
        l64[i] = l;
    }
}

// One E(+M) pass over rows [r0, r1) with the given template / log-prior buffers.
em_status run_pass(em_ctx *c, int flags, int64_t r0, int64_t r1, const double *a,
                   const void *Thi, const void *Tlo, const float *tscale, const float *lr32,
                   const double *lr64, double coef, float *post, int32_t *argmax, float *margin,
                   bool use_partials, bool timed) {
    PassArgs A{};
    A.a = a;
    A.V = c->V;
    A.rowbytes = c->rowbytes;
    A.rowscale = c->rowscale;
    A.Thi = Thi;
    A.Tlo = Tlo;
    A.tscale = tscale;
    A.logrho32 = lr32;
    A.logrho64 = lr64;
    A.E2 = c->E2;
    A.E64 = c->E64;
    A.phase = c->phase;
    A.L = c->L;
    A.lo = c->lo;
    A.grid = c->has_angles ? 0 : 1;
    A.row_begin = r0;
    A.row_end = r1;
    A.D = c->D;
    A.K = c->K;
    A.Q = c->Q;
    A.Dp = c->Dp;
    A.W = c->W;
    A.Wp = c->Wp;
    A.coef = coef;
    A.flags = flags;
    A.partials = use_partials ? c->partials : nullptr;
    A.ncols = c->ncols;
    A.lse = c->lse;
    A.post = post;
    A.argmax = argmax;
    A.margin = margin;
    A.stopped = c->stopped;
    const int64_t ntiles = (r1 - r0 + c->BM - 1) / c->BM;
    int grid = use_partials ? c->grid : (int)(ntiles < c->grid ? ntiles : c->grid);
    if (grid < 1) grid = 1;
    const bool ev = timed && c->timing && c->ev_used + 2 <= 2 * kTimingEvents;
    if (ev) set_pass_events(c->ev[c->ev_used], c->ev[c->ev_used + 1]);
    hipError_t e;
    if (c->kr)
        e = launch_pass_kr(c->prec, c->krNT, A, grid, c->lds, c->stream);
    else if (c->gm)
        e = launch_pass_gm(c->gmNT, A, grid, c->lds, c->stream);
    else if (c->ks)
        e = launch_pass_ks(c->prec, c->BM, c->ksNT, c->ksKSS, A, grid, c->lds, c->stream);
    else if (c->wide)
        e = launch_pass_wide(c->prec, c->wNTW, c->wUR, A, grid, c->lds, c->stream);
    else if (c->fs && !(flags & (PF_QUERY | PF_STORE_LSE | PF_LOAD_LSE)))
        e = launch_pass_fs(c->prec, c->fsMTW, c->fsE, A, grid, c->fsLds, c->stream);
    else if (c->fac)
        e = launch_pass_fac(c->prec, c->fWIDE, c->fKCM, c->fEPL, A, grid, c->lds, c->stream);
    else
        e = launch_pass(c->prec, c->BM, c->WM, c->LD, A, grid, c->lds, c->stream);
    set_pass_events(nullptr, nullptr);
    if (e != hipSuccess)
        return fail(c, EM_EDEVICE, std::string("E+M pass launch failed: ") + hipGetErrorString(e));
    if (ev) c->ev_used += 2;
    return EM_OK;
}

em_status run_template(em_ctx *c, const double *a, void *Thi, void *Tlo, float *tscale,
                       bool check_stop) {
    TplArgs T{};
    T.a = a;
    T.D = c->D;
    T.K = c->K;
    T.Q = c->Q;
    T.Dp = c->Dp;
    T.W = c->W;
    T.Wp = c->Wp;
    T.prec = c->prec;
    T.E64 = c->E64;
    T.Thi = Thi;
    T.Tlo = Tlo;
    T.tscale = tscale;
    T.stopped = check_stop ? c->stopped : nullptr;
    HIPCHK(c, launch_template(T, c->stream));
    return EM_OK;
}

FinArgs fin_base(em_ctx *c, int mode) {
    FinArgs F{};
    F.mode = mode;
    F.red = c->red;
    F.N = c->N;
    F.D = c->D;
    F.K = c->K;
    F.Q = c->Q;
    F.W = c->W;
    F.Wp = c->Wp;
    F.L = c->L;
    F.sigma2 = c->sigma2;
    F.gamma = c->gamma;
    F.update_rho = c->update_rho;
    F.sum_vn2 = c->sum_vn2;
    F.rho_bar = c->rho_bar;
    F.gai = c->has_gai ? c->gai : nullptr;
    F.phase = c->phase;
    F.a_in = c->a;
    F.rho_in = c->rho;
    F.a = c->a;
    F.rho = c->rho;
    F.t = c->t;
    F.stopped = c->stopped;
    F.ll_last = c->ll_last;
    F.stats = c->stats;
    F.logrho32 = c->logrho32;
    F.logrho64 = c->logrho64;
    F.out = c->scal;
    F.g = 1.0;
    return F;
}

em_status sync(em_ctx *c) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EM_OK;
}

void free_all(em_ctx *c) {
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
}

}  // namespace

extern "C" {

const char *em_version(void) { return "synchem 0.1 (gfx950)"; }

const char *em_last_error(const em_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_err.c_str();
}

em_status em_init(em_ctx **out, const em_params *p, const void *obs_dev, const double *prior,
                  void *stream) {
    g_err.clear();
    if (!out) return fail(nullptr, EM_EINVAL, "out is NULL");
    *out = nullptr;
    em_status st = check_params(p);
    if (st != EM_OK) return st;
    if (!obs_dev) return fail(nullptr, EM_EINVAL, "obs_dev is NULL");
    std::vector<double> rho0;
    st = check_prior(prior, p->window_count, rho0, nullptr);
    if (st != EM_OK) return st;

    em_ctx *c = new em_ctx();
    c->N = p->n_obs;
    c->K = p->K;
    c->Q = p->Q;
    c->D = p->K * p->Q;
    c->Dp = (2 * c->D + 31) / 32 * 32;
    c->L = p->L;
    c->lo = ((p->window_lo % p->L) + p->L) % p->L;
    c->W = p->window_count;
    c->has_angles = p->angles != nullptr;
    c->Wp = (c->W + 15) / 16 * 16;
    c->sigma2 = p->sigma2;
    c->gamma = p->gamma;
    c->update_rho = p->update_rho;
    c->prec = p->precision;
    c->flags = p->flags;
    c->has_gai = p->gamma_a_inv != nullptr;
    c->timing = (p->flags & EM_FLAG_TIMING) != 0;
    c->stream = (hipStream_t)stream;
    c->rowbytes = row_bytes(c->prec, c->Dp);
    c->ncols = 2 * c->D + c->Wp + 4;

    auto bail = [&](em_status s) {
        g_err = c->err;
        free_all(c);
        delete c;
        return s;
    };

    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        c->err = std::string("no HIP device: ") + hipGetErrorString(e);
        return bail(EM_EDEVICE);
    }
    int cus = 0, ldsmax = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&ldsmax, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
            hipSuccess) {
        c->err = "device attribute query failed";
        return bail(EM_EDEVICE);
    }
    if ((st = plan(c, (size_t)ldsmax)) != EM_OK) return bail(st);
    int occ = 1;
    if (c->gm) {
        if (pass_gm_setup(c->gmNT, c->lds, &occ) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
    } else if (c->kr) {
        if (pass_kr_setup(c->prec, c->krNT, c->lds, &occ) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
    } else if (c->ks) {
        if (pass_ks_setup(c->prec, c->BM, c->ksNT, c->ksKSS, c->lds, &occ) != hipSuccess ||
            occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
    } else if (c->wide) {
        if (pass_wide_setup(c->prec, c->wNTW, c->wUR, c->lds, &occ) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
    } else if (c->fac) {
        if (pass_fac_setup(c->prec, c->fWIDE, c->fKCM, c->fEPL, c->lds, &occ) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
        int occ_fs = 1;
        if (c->fs) {   // both kernels fill the same partial rows: the smaller resident grid
            if (pass_fs_setup(c->prec, c->fsMTW, c->fsE, c->fsLds, &occ_fs) != hipSuccess ||
                occ_fs < 1) {
                (void)hipGetLastError();
                occ_fs = 1;
            }
            if (occ_fs < occ) occ = occ_fs;
        }
    } else {
        if (pass_setup(c->prec, c->BM, c->WM, c->LD, c->lds, &occ) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
    }
    const int64_t ntiles = (c->N + c->BM - 1) / c->BM;
    const int64_t gmax = (int64_t)cus * occ;
    c->grid = (int)(ntiles < gmax ? ntiles : gmax);
    {   // workgroups of the set-up column sums: partials of at most 8 MiB
        const int64_t cg = 2 * c->D <= 1024 ? 1024 : 256;
        c->colsum_grid = (int)(c->N < cg ? c->N : cg);
    }

    // buffers
    const int64_t nT = (int64_t)c->Dp * c->Wp;
    const size_t tbytes = c->prec == P_F64 ? nT * 8 : (c->prec == P_F32 ? nT * 4 : nT * 2);
    if ((st = alloc_t(c, &c->V, (size_t)(c->N * c->rowbytes))) != EM_OK) return bail(st);
    if (c->prec != P_F64 && c->prec != P_F32)
        if ((st = alloc_t(c, &c->rowscale, (size_t)c->N)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->vnorm2, (size_t)c->N)) != EM_OK) return bail(st);
    for (void **pp : {&c->Thi, &c->Tlo, &c->ThiE, &c->TloE})
        if ((st = dev_alloc(c, pp, tbytes)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->tscale, 4)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->tscaleE, 4)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->E2, (size_t)c->Wp * 2 * c->K)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->E64, (size_t)c->Wp * c->K)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->phase, (size_t)c->L)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->logrho32, (size_t)c->Wp)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->logrho32E, (size_t)c->Wp)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->logrho64, (size_t)c->Wp)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->logrho64E, (size_t)c->Wp)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->a, (size_t)2 * c->D)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->aE, (size_t)2 * c->D)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->rho, (size_t)c->W)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->rhoE, (size_t)c->W)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->rho_bar, (size_t)c->W)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->gai, (size_t)c->D)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->t, 1)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->stopped, 1)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->fin_count, 1)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->nonfinite, 1)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->ll_last, 1)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->scal, 4)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->stats, (size_t)kStatsCap * EM_STATS_FIELDS)) != EM_OK)
        return bail(st);
    const size_t npart = std::max((size_t)c->grid * c->ncols, (size_t)c->colsum_grid * 2 * c->D);
    if ((st = alloc_t(c, &c->partials, npart)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->red, (size_t)c->ncols)) != EM_OK) return bail(st);
    if ((st = alloc_t(c, &c->lse, (size_t)c->N)) != EM_OK) return bail(st);
    if (c->timing) {
        for (auto &ev : c->ev)
            if (hipEventCreate(&ev) != hipSuccess) {
                c->err = "hipEventCreate failed";
                return bail(EM_EDEVICE);
            }
    }

    // host-side tables: phase e^{+2 pi i m / L}, E = e^{+i k theta_i}, rho_0, log rho_0
    std::vector<double2> ph(c->L);
    for (int m = 0; m < c->L; ++m) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * m / c->L;
        ph[m] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    std::vector<float> e2((size_t)c->Wp * 2 * c->K, 0.f);
    std::vector<double2> e64((size_t)c->Wp * c->K, make_double2(0.0, 0.0));
    for (int i = 0; i < c->W; ++i)
        for (int k = 0; k < c->K; ++k) {
            double2 e;
            if (p->angles) {                          // exp(+i k theta_i) at the given angle
                const long double ang = (long double)k * (long double)p->angles[i];
                e = make_double2((double)cosl(ang), (double)sinl(ang));
            } else {                                  // the exact grid angle 2 pi ((k o_i) mod L) / L
                e = ph[((int64_t)k * (c->lo + i)) % c->L];
            }
            e64[(size_t)i * c->K + k] = e;
            e2[(size_t)i * 2 * c->K + k] = (float)e.x;
            e2[(size_t)i * 2 * c->K + c->K + k] = (float)e.y;
        }
    std::vector<float> l32;
    std::vector<double> l64;
    logrho_host(rho0, c->Wp, l32, l64);
    std::vector<double> gai(c->D, 0.0);
    if (p->gamma_a_inv)
        for (int d = 0; d < c->D; ++d) gai[d] = p->gamma_a_inv[d];
    const int64_t zero64 = 0;
    const int zero = 0;
    std::vector<double> stats0((size_t)kStatsCap * EM_STATS_FIELDS, 0.0);

#define UP(dst, src, bytes)                                                                    \
    do {                                                                                       \
        if (hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, c->stream) !=         \
            hipSuccess) {                                                                      \
            c->err = "host to device copy failed";                                             \
            return bail(EM_EDEVICE);                                                           \
        }                                                                                      \
    } while (0)
    UP(c->phase, ph.data(), ph.size() * sizeof(double2));
    UP(c->E2, e2.data(), e2.size() * sizeof(float));
    UP(c->E64, e64.data(), e64.size() * sizeof(double2));
    UP(c->rho, rho0.data(), rho0.size() * 8);
    UP(c->rho_bar, rho0.data(), rho0.size() * 8);
    UP(c->logrho32, l32.data(), l32.size() * 4);
    UP(c->logrho64, l64.data(), l64.size() * 8);
    UP(c->gai, gai.data(), gai.size() * 8);
    UP(c->t, &zero64, 8);
    UP(c->stopped, &zero, 4);
    UP(c->fin_count, &zero, 4);
    UP(c->nonfinite, &zero, 4);
    UP(c->stats, stats0.data(), stats0.size() * 8);

    // a1: convert the observations
    if (launch_convert(c->prec, obs_dev, c->N, c->D, c->Dp, c->V, c->rowbytes, c->rowscale,
                       c->vnorm2, c->nonfinite, c->stream) != hipSuccess) {
        c->err = "convert launch failed";
        return bail(EM_EDEVICE);
    }
    // sum_j ||v_j||^2 (fixed order) and the initial estimate
    {
        // in the first G entries of the partials buffer (the column sums below come after)
        const int G = (int)std::min<int64_t>(c->N, 256);
        if (launch_sum(c->vnorm2, c->N, c->partials, G, c->scal, c->stream) != hipSuccess) {
            c->err = "reduce launch failed";
            return bail(EM_EDEVICE);
        }
    }
    if (p->a0) {
        UP(c->a, p->a0, (size_t)2 * c->D * 8);
    } else {
        if (launch_colsum(obs_dev, c->prec == P_F64, c->N, c->D, c->partials, c->colsum_grid,
                          c->stream) != hipSuccess ||
            launch_reduce(c->partials, c->colsum_grid, 2 * c->D, c->red, c->stream) !=
                hipSuccess ||
            launch_scale(c->red, c->a, 2 * c->D, 1.0 / (double)c->N, c->stream) != hipSuccess) {
            c->err = "mean launch failed";
            return bail(EM_EDEVICE);
        }
    }
#undef UP
    int nf = 0;
    double svn = 0;
    if (hipMemcpyAsync(&nf, c->nonfinite, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&svn, c->scal, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = "device to host copy failed";
        return bail(EM_EDEVICE);
    }
    if (nf) {
        c->err = "observations contain NaN or Inf";
        return bail(EM_ENONFINITE);
    }
    c->sum_vn2 = svn;
    if ((st = run_template(c, c->a, c->Thi, c->Tlo, c->tscale, false)) != EM_OK)
        return bail(st);
    if ((st = sync(c)) != EM_OK) return bail(st);
    *out = c;
    return EM_OK;
}

em_status em_step(em_ctx *c, int32_t n_iter, double tol, int32_t *iters_done, double *ll_last) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (n_iter < 0) return fail(c, EM_EINVAL, "n_iter must be >= 0");
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(c, EM_EINVAL, "tol must be >= 0");
    int64_t t0 = 0;
    if (iters_done) {
        HIPCHK(c, hipMemcpyAsync(&t0, c->t, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    const double coef = 2.0 / c->sigma2;
    int flags = PF_ACC_M | PF_CHECK_STOP;
    if (c->flags & EM_FLAG_KEEP_LSE) {
        // the per-row LSE buffer is also the adjoint's checkpoint: once an EM pass overwrites it
        // at a_t, it no longer belongs to the last em_loglik_fwd
        flags |= PF_STORE_LSE;
        if (n_iter > 0) c->fwd_valid = false;
    }
    FinArgs F = fin_base(c, FIN_EM);
    F.tol = tol;
    for (int it = 0; it < n_iter; ++it) {
        em_status st = run_pass(c, flags, 0, c->N, c->a, c->Thi, c->Tlo, c->tscale, c->logrho32,
                                c->logrho64, coef, nullptr, nullptr, nullptr, true, true);
        if (st != EM_OK) return st;
        HIPCHK(c, launch_reduce_finalize(F, c->partials, c->grid, c->ncols, c->red, c->fin_count,
                                         c->stream));
        if (!c->ks && !c->fac && !c->kr)   // these passes use a_t itself
            if ((st = run_template(c, c->a, c->Thi, c->Tlo, c->tscale, true)) != EM_OK) return st;
    }
    if (iters_done || ll_last) {
        int64_t t1 = 0;
        double ll = 0;
        HIPCHK(c, hipMemcpyAsync(&t1, c->t, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(&ll, c->ll_last, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (iters_done) *iters_done = (int32_t)(t1 - t0);
        if (ll_last) *ll_last = ll;
    }
    return EM_OK;
}

em_status em_loglik(em_ctx *c, double *ll) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (!ll) return fail(c, EM_EINVAL, "ll is NULL");
    em_status st = run_pass(c, 0, 0, c->N, c->a, c->Thi, c->Tlo, c->tscale, c->logrho32, c->logrho64,
                            2.0 / c->sigma2, nullptr, nullptr, nullptr, true, false);
    if (st != EM_OK) return st;
    FinArgs F = fin_base(c, FIN_LL);
    HIPCHK(c, launch_reduce_finalize(F, c->partials, c->grid, c->ncols, c->red, c->fin_count,
                                         c->stream));
    HIPCHK(c, hipMemcpyAsync(ll, c->scal, 8, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

em_status em_posterior(em_ctx *c, int64_t row0, int64_t nrows, float *w_dev, int32_t *argmax_dev,
                       float *margin_dev) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (row0 < 0 || nrows < 0 || row0 + nrows > c->N)
        return fail(c, EM_EINVAL, "row range outside [0, N)");
    if (nrows == 0) return EM_OK;
    return run_pass(c, PF_QUERY, row0, row0 + nrows, c->a, c->Thi, c->Tlo, c->tscale, c->logrho32,
                    c->logrho64, 2.0 / c->sigma2, w_dev, argmax_dev, margin_dev, false, false);
}

em_status em_get_state(em_ctx *c, double *a, double *rho, int64_t *t) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (a) HIPCHK(c, hipMemcpyAsync(a, c->a, (size_t)2 * c->D * 8, hipMemcpyDeviceToHost, c->stream));
    if (rho) HIPCHK(c, hipMemcpyAsync(rho, c->rho, (size_t)c->W * 8, hipMemcpyDeviceToHost, c->stream));
    if (t) HIPCHK(c, hipMemcpyAsync(t, c->t, 8, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

em_status em_set_state(em_ctx *c, const double *a, const double *rho, int64_t t) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (t < 0) return fail(c, EM_EINVAL, "t must be >= 0");
    if (a && !finite_all(a, 2 * (int64_t)c->D)) return fail(c, EM_EINVAL, "a must be finite");
    std::vector<double> r;
    if (rho) {
        em_status st = check_prior(rho, c->W, r, c);
        if (st != EM_OK) return st;
    }
    const int zero = 0;
    std::vector<float> l32;      // must outlive the asynchronous copies (synchronised below)
    std::vector<double> l64;
    if (a) HIPCHK(c, hipMemcpyAsync(c->a, a, (size_t)2 * c->D * 8, hipMemcpyHostToDevice, c->stream));
    if (rho) {
        logrho_host(r, c->Wp, l32, l64);
        HIPCHK(c, hipMemcpyAsync(c->rho, r.data(), (size_t)c->W * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->logrho32, l32.data(), l32.size() * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->logrho64, l64.data(), l64.size() * 8, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->t, &t, 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->stopped, &zero, 4, hipMemcpyHostToDevice, c->stream));
    em_status st = run_template(c, c->a, c->Thi, c->Tlo, c->tscale, false);
    if (st != EM_OK) return st;
    c->fwd_valid = false;
    return sync(c);
}

em_status em_loglik_fwd(em_ctx *c, const double *a_dev, double sigma2, const double *eta_dev,
                        double *ll) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (!a_dev) return fail(c, EM_EINVAL, "a_dev is NULL");
    if (!ll) return fail(c, EM_EINVAL, "ll is NULL");
    if (!(sigma2 > 0) || !std::isfinite(sigma2))
        return fail(c, EM_EINVAL, "sigma2 must be positive and finite");
    c->fwd_valid = false;
    HIPCHK(c, hipMemcpyAsync(c->aE, a_dev, (size_t)2 * c->D * 8, hipMemcpyDeviceToDevice, c->stream));
    if (eta_dev) {
        HIPCHK(c, launch_softmax(eta_dev, c->rhoE, c->logrho32E, c->logrho64E, c->W, c->Wp, c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(c->rhoE, c->rho, (size_t)c->W * 8, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, launch_logrho(c->rhoE, c->logrho32E, c->logrho64E, c->W, c->Wp, c->stream));
    }
    em_status st = run_template(c, c->aE, c->ThiE, c->TloE, c->tscaleE, false);
    if (st != EM_OK) return st;
    st = run_pass(c, PF_STORE_LSE, 0, c->N, c->aE, c->ThiE, c->TloE, c->tscaleE, c->logrho32E,
                  c->logrho64E, 2.0 / sigma2, nullptr, nullptr, nullptr, true, false);
    if (st != EM_OK) return st;
    FinArgs F = fin_base(c, FIN_LL);
    F.sigma2 = sigma2;
    F.a_in = c->aE;
    F.rho_in = c->rhoE;
    HIPCHK(c, launch_reduce_finalize(F, c->partials, c->grid, c->ncols, c->red, c->fin_count,
                                         c->stream));
    HIPCHK(c, hipMemcpyAsync(ll, c->scal, 8, hipMemcpyDeviceToHost, c->stream));
    if ((st = sync(c)) != EM_OK) return st;
    c->sigma2E = sigma2;
    c->etaE = eta_dev != nullptr;
    c->fwd_valid = true;
    return EM_OK;
}

em_status em_loglik_bwd(em_ctx *c, double g, double *grad_a_dev, double *grad_sigma2,
                        double *grad_eta_dev) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (!c->fwd_valid) return fail(c, EM_ESTATE, "em_loglik_bwd needs a preceding em_loglik_fwd");
    if (!grad_a_dev) return fail(c, EM_EINVAL, "grad_a_dev is NULL");
    if (!std::isfinite(g)) return fail(c, EM_EINVAL, "g must be finite");
    em_status st = run_pass(c, PF_ACC_M | PF_LOAD_LSE, 0, c->N, c->aE, c->ThiE, c->TloE, c->tscaleE,
                            c->logrho32E, c->logrho64E, 2.0 / c->sigma2E, nullptr, nullptr,
                            nullptr, true, false);
    if (st != EM_OK) return st;
    FinArgs F = fin_base(c, FIN_GRAD);
    F.sigma2 = c->sigma2E;
    F.a_in = c->aE;
    F.rho_in = c->rhoE;
    F.g = g;
    F.grad_a = grad_a_dev;
    F.grad_eta = grad_eta_dev;
    HIPCHK(c, launch_reduce_finalize(F, c->partials, c->grid, c->ncols, c->red, c->fin_count,
                                         c->stream));
    double gs = 0;
    HIPCHK(c, hipMemcpyAsync(&gs, c->scal + 1, 8, hipMemcpyDeviceToHost, c->stream));
    if ((st = sync(c)) != EM_OK) return st;
    if (grad_sigma2) *grad_sigma2 = gs;
    return EM_OK;
}

em_status em_get_stats(em_ctx *c, double *buf, int32_t cap, int32_t *n) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (cap < 0 || (cap > 0 && !buf)) return fail(c, EM_EINVAL, "bad buffer");
    int64_t t = 0;
    HIPCHK(c, hipMemcpyAsync(&t, c->t, 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> all((size_t)kStatsCap * EM_STATS_FIELDS);
    HIPCHK(c, hipMemcpyAsync(all.data(), c->stats, all.size() * 8, hipMemcpyDeviceToHost, c->stream));
    em_status st = sync(c);
    if (st != EM_OK) return st;
    const int64_t have = t < kStatsCap ? t : kStatsCap;
    const int64_t cnt = have < cap ? have : cap;
    // oldest first among the last `have` records, then keep the last `cnt`
    for (int64_t r = 0; r < cnt; ++r) {
        const int64_t it = t - cnt + r;
        std::memcpy(buf + r * EM_STATS_FIELDS, all.data() + (it % kStatsCap) * EM_STATS_FIELDS,
                    EM_STATS_FIELDS * sizeof(double));
    }
    if (n) *n = (int32_t)cnt;
    return EM_OK;
}

em_status em_learn_prior(const int32_t *err_dev, int64_t n, int32_t L, int32_t lo, int32_t W,
                         double *rho_bar, int64_t *counts, int64_t *n_in_window, void *stream) {
    g_err.clear();
    if (!err_dev && n > 0) return fail(nullptr, EM_EINVAL, "err_dev is NULL");
    if (n < 0) return fail(nullptr, EM_EINVAL, "n must be >= 0");
    if (L < 1 || L > 16384) return fail(nullptr, EM_EINVAL, "L must be in [1, 16384]");
    if (W < 1 || W > L) return fail(nullptr, EM_EINVAL, "W must be in [1, L]");
    if (!rho_bar) return fail(nullptr, EM_EINVAL, "rho_bar is NULL");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *cnt = nullptr;
    hipError_t e = hipMalloc((void **)&cnt, (size_t)L * 8);
    if (e != hipSuccess) return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    std::vector<unsigned long long> h(L, 0ull);
    e = hipMemcpyAsync(cnt, h.data(), (size_t)L * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n > 0) e = launch_histogram(err_dev, n, L, cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), cnt, (size_t)L * 8, hipMemcpyDeviceToHost, s);
    e = finish(e, s);
    (void)hipFree(cnt);
    if (e != hipSuccess) return fail(nullptr, EM_EDEVICE, std::string("histogram: ") + hipGetErrorString(e));
    const int lom = ((lo % L) + L) % L;
    int64_t inside = 0;
    for (int i = 0; i < W; ++i) inside += (int64_t)h[(lom + i) % L];
    if (counts)
        for (int i = 0; i < L; ++i) counts[i] = (int64_t)h[i];
    if (n_in_window) *n_in_window = inside;
    if (inside == 0) return fail(nullptr, EM_EINVAL, "no draw falls inside the window");
    for (int i = 0; i < W; ++i) rho_bar[i] = (double)h[(lom + i) % L] / (double)inside;
    return EM_OK;
}

// ------------------------------------------------------------------------------------------
// Synchronize and Match (§II-A, §III-A)

namespace {

struct DevBufs {                      // device scratch of one call, freed on every return path
    std::vector<void *> p;
    ~DevBufs() {
        for (void *q : p) (void)hipFree(q);
    }
    bool get(void **out, size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, bytes + 16) != hipSuccess) return false;
        p.push_back(q);
        *out = q;
        return true;
    }
};

em_status sync_shape(int64_t N, int32_t K, int32_t Q) {
    if (N < 1) return fail(nullptr, EM_EINVAL, "the number of observations must be >= 1");
    if (K < 1 || Q < 1) return fail(nullptr, EM_EINVAL, "K and Q must be >= 1");
    if ((int64_t)K * Q > kMaxD) return fail(nullptr, EM_EUNSUPPORTED, "D = K*Q above 2048");
    if (K > kMaxK) return fail(nullptr, EM_EUNSUPPORTED, "K above 512");
    return EM_OK;
}

em_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return EM_OK;
    return fail(nullptr, EM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

em_status em_relative_rotations(const void *obs_dev, int64_t P, int32_t K, int32_t Q, int32_t L,
                                int32_t *rel_dev, float *gap_dev, float *dot_dev, void *stream) {
    g_err.clear();
    em_status st = sync_shape(P, K, Q);
    if (st != EM_OK) return st;
    if (!obs_dev || !rel_dev) return fail(nullptr, EM_EINVAL, "obs_dev and rel_dev are required");
    if (P < 2) return fail(nullptr, EM_EINVAL, "P must be >= 2");
    if (P > kMaxSyncP) return fail(nullptr, EM_EUNSUPPORTED, "P above 8192");
    if (L < 1 || L > kMaxSyncL) return fail(nullptr, EM_EINVAL, "L must be in [1, 4096]");
    hipStream_t s = (hipStream_t)stream;
    // B: Lp rows of [cos(k 2 pi l / L) | sin(k 2 pi l / L) | 0], row stride 64 for the tiled kernel
    const int Lp = (L + 15) / 16 * 16, K2 = relrot_tiled(K, Q, L) ? 64 : (2 * K + 3) / 4 * 4;
    std::vector<float> B((size_t)Lp * K2, 0.f), cs(L), sn(L);
    for (int m = 0; m < L; ++m) {                 // the exact grid angles 2 pi m / L
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * m / L;
        cs[m] = (float)cosl(ang);
        sn[m] = (float)sinl(ang);
    }
    for (int l = 0; l < L; ++l)
        for (int k = 0; k < K; ++k) {
            const int m = (int)(((int64_t)k * l) % L);
            B[(size_t)l * K2 + k] = cs[m];
            B[(size_t)l * K2 + K + k] = sn[m];
        }
    DevBufs buf;
    float *Bd = nullptr, *gap = gap_dev, *dot = dot_dev;
    if (!buf.get((void **)&Bd, B.size() * sizeof(float)) || (!gap && !buf.get((void **)&gap, (size_t)P * P * sizeof(float))) ||
        (!dot && !buf.get((void **)&dot, (size_t)P * P * sizeof(float))))
        return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    hipError_t e = hipMemcpyAsync(Bd, B.data(), B.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_relrot((const float2 *)obs_dev, (int)P, K, Q, L, Bd, rel_dev, gap, dot, s);
    e = finish(e, s);
    return hip_status(e, "relative rotations");
}

em_status em_ppm(const int32_t *rel_dev, int64_t P, int32_t L, int32_t iters, double *theta_dev,
                 void *stream) {
    g_err.clear();
    if (!rel_dev || !theta_dev) return fail(nullptr, EM_EINVAL, "rel_dev and theta_dev are required");
    if (P < 1) return fail(nullptr, EM_EINVAL, "P must be >= 1");
    if (P > kMaxSyncP) return fail(nullptr, EM_EUNSUPPORTED, "P above 8192");
    if (L < 1 || L > kMaxSyncL) return fail(nullptr, EM_EINVAL, "L must be in [1, 4096]");
    if (iters < 0 || iters > 100000) return fail(nullptr, EM_EINVAL, "iters must be in [0, 100000]");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double2> ph(L);
    for (int m = 0; m < L; ++m) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * m / L;
        ph[m] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    DevBufs buf;
    double2 *phd = nullptr, *z0 = nullptr, *z1 = nullptr;
    if (!buf.get((void **)&phd, (size_t)L * sizeof(double2)) || !buf.get((void **)&z0, (size_t)P * sizeof(double2)) || !buf.get((void **)&z1, (size_t)P * sizeof(double2)))
        return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    hipError_t e = hipMemcpyAsync(phd, ph.data(), ph.size() * sizeof(double2),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_ppm(rel_dev, (int)P, L, phd, z0, z1, iters, theta_dev, s);
    e = finish(e, s);
    return hip_status(e, "power method");
}

em_status em_nearest(const void *obs_dev, int64_t N, int32_t K, int32_t Q, int64_t P,
                     int32_t *nn_dev, float *gap_dev, void *stream) {
    g_err.clear();
    em_status st = sync_shape(N, K, Q);
    if (st != EM_OK) return st;
    if (!obs_dev || !nn_dev) return fail(nullptr, EM_EINVAL, "obs_dev and nn_dev are required");
    if (P < 2 || P > N) return fail(nullptr, EM_EINVAL, "P must be in [2, N]");
    if (P > (1 << 30)) return fail(nullptr, EM_EUNSUPPORTED, "P above 2^30");
    if (((int64_t)K * Q) % 8 != 0)
        return fail(nullptr, EM_EUNSUPPORTED, "nearest neighbours need D = K*Q a multiple of 8");
    hipStream_t s = (hipStream_t)stream;
    DevBufs buf;
    float *nrm = nullptr, *gap = gap_dev;
    if (!buf.get((void **)&nrm, (size_t)P * sizeof(float)) || (!gap && !buf.get((void **)&gap, (size_t)N * sizeof(float))))
        return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    hipError_t e = launch_nearest((const float2 *)obs_dev, N, P, K * Q, nrm, nn_dev, gap, s);
    e = finish(e, s);
    return hip_status(e, "nearest neighbours");
}

em_status em_sync_match(const void *obs_dev, int64_t N, int32_t K, int32_t Q, int32_t L,
                        int64_t P, int32_t iters, double *theta_dev, int32_t *nn_dev,
                        void *stream) {
    g_err.clear();
    em_status st = sync_shape(N, K, Q);
    if (st != EM_OK) return st;
    if (!obs_dev || !theta_dev) return fail(nullptr, EM_EINVAL, "obs_dev and theta_dev are required");
    if (P < 2 || P > N) return fail(nullptr, EM_EINVAL, "P must be in [2, N]");
    if (P > kMaxSyncP) return fail(nullptr, EM_EUNSUPPORTED, "P above 8192");
    if (L < 1 || L > kMaxSyncL) return fail(nullptr, EM_EINVAL, "L must be in [1, 4096]");
    if (iters < 0 || iters > 100000) return fail(nullptr, EM_EINVAL, "iters must be in [0, 100000]");
    if (((int64_t)K * Q) % 8 != 0)
        return fail(nullptr, EM_EUNSUPPORTED, "nearest neighbours need D = K*Q a multiple of 8");
    hipStream_t s = (hipStream_t)stream;
    DevBufs buf;
    int32_t *rel = nullptr, *nn = nn_dev;
    double *phi = nullptr;
    if (!buf.get((void **)&rel, (size_t)P * P * sizeof(int32_t)) || !buf.get((void **)&phi, (size_t)P * sizeof(double)) || (!nn && !buf.get((void **)&nn, (size_t)N * sizeof(int32_t))))
        return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    if ((st = em_relative_rotations(obs_dev, P, K, Q, L, rel, nullptr, nullptr, stream)) != EM_OK)
        return st;
    if ((st = em_ppm(rel, P, L, iters, phi, stream)) != EM_OK) return st;
    if ((st = em_nearest(obs_dev, N, K, Q, P, nn, nullptr, stream)) != EM_OK) return st;
    hipError_t e = launch_gather(phi, P, nn, N, theta_dev, s);
    e = finish(e, s);
    return hip_status(e, "gather");
}

em_status em_align(const void *obs_dev, int64_t N, int32_t K, int32_t Q, const double *theta_dev,
                   void *out_dev, void *stream) {
    g_err.clear();
    em_status st = sync_shape(N, K, Q);
    if (st != EM_OK) return st;
    if (!obs_dev || !theta_dev || !out_dev)
        return fail(nullptr, EM_EINVAL, "obs_dev, theta_dev and out_dev are required");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_align((const float2 *)obs_dev, N, K, Q, theta_dev, (float2 *)out_dev, s);
    e = finish(e, s);
    return hip_status(e, "align");
}

em_status em_aligned_mean(const void *obs_dev, int64_t N, int32_t K, int32_t Q,
                          const double *theta_dev, double *mean_dev, void *stream) {
    g_err.clear();
    em_status st = sync_shape(N, K, Q);
    if (st != EM_OK) return st;
    if (!obs_dev || !theta_dev || !mean_dev)
        return fail(nullptr, EM_EINVAL, "obs_dev, theta_dev and mean_dev are required");
    hipStream_t s = (hipStream_t)stream;
    const int D = K * Q;
    const int G = (int)std::min<int64_t>(N, kAlignedMeanBlocks);
    DevBufs buf;
    double *part = nullptr, *sum = nullptr;
    if (!buf.get((void **)&part, (size_t)G * 2 * D * sizeof(double)) ||
        !buf.get((void **)&sum, (size_t)2 * D * sizeof(double)))
        return fail(nullptr, EM_ENOMEM, "hipMalloc failed");
    hipError_t e = launch_aligned_colsum((const float2 *)obs_dev, N, K, Q, theta_dev, part, G, s);
    if (e == hipSuccess) e = launch_reduce(part, G, 2 * D, sum, s);
    if (e == hipSuccess) e = launch_scale(sum, mean_dev, 2 * D, 1.0 / (double)N, s);
    e = finish(e, s);
    return hip_status(e, "aligned mean");
}

em_status em_aligned_mean_noalloc(const void *obs_dev, int64_t N, int32_t K, int32_t Q,
                                  const double *theta_dev, double *mean_dev, void *stream) {
    g_err.clear();
    em_status st = sync_shape(N, K, Q);          // D <= kMaxD: the partials fit the scratch
    if (st != EM_OK) return st;
    if (!obs_dev || !theta_dev || !mean_dev)
        return fail(nullptr, EM_EINVAL, "obs_dev, theta_dev and mean_dev are required");
    const int D = K * Q;
    const int G = (int)std::min<int64_t>(N, kAlignedMeanBlocks);
    double *part = nullptr;
    size_t cap = 0;
    hipError_t e = noalloc_scratch(&part, &cap);
    if (e != hipSuccess) return hip_status(e, "scratch address");
    if ((size_t)G * 2 * D * sizeof(double) > cap)
        return fail(nullptr, EM_EUNSUPPORTED, "partial sums exceed the library's scratch");
    hipStream_t s = (hipStream_t)stream;
    // every partial is written by the column-sum kernel before the reduction reads it; the sum
    // goes straight into mean_dev and is scaled there (the same operations as em_aligned_mean)
    e = launch_aligned_colsum((const float2 *)obs_dev, N, K, Q, theta_dev, part, G, s);
    if (e == hipSuccess) e = launch_reduce(part, G, 2 * D, mean_dev, s);
    if (e == hipSuccess) e = launch_scale(mean_dev, mean_dev, 2 * D, 1.0 / (double)N, s);
    return hip_status(e, "aligned mean");
}

em_status em_error_bins(const double *theta_hat_dev, const double *theta_dev, int64_t N, int32_t L,
                        int32_t lc, int32_t *bins_dev, void *stream) {
    g_err.clear();
    if (!theta_hat_dev || !theta_dev || !bins_dev)
        return fail(nullptr, EM_EINVAL, "theta_hat_dev, theta_dev and bins_dev are required");
    if (N < 1) return fail(nullptr, EM_EINVAL, "N must be >= 1");
    if (L < 1 || L > 16384) return fail(nullptr, EM_EINVAL, "L must be in [1, 16384]");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_error_bins(theta_hat_dev, theta_dev, N, L, lc, bins_dev, s);
    e = finish(e, s);
    return hip_status(e, "error bins");
}

em_status em_set_stream(em_ctx *c, void *stream) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    c->stream = (hipStream_t)stream;
    return EM_OK;
}

em_status em_pass_time(em_ctx *c, double *ms_total, int64_t *launches, int32_t reset) {
    if (!c) return fail(nullptr, EM_EINVAL, "ctx is NULL");
    if (!c->timing) return fail(c, EM_ESTATE, "context was created without EM_FLAG_TIMING");
    em_status st = sync(c);
    if (st != EM_OK) return st;
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->pass_ms += ms;
        c->pass_count += 1;
    }
    c->ev_used = 0;
    if (ms_total) *ms_total = c->pass_ms;
    if (launches) *launches = c->pass_count;
    if (reset) {
        c->pass_ms = 0;
        c->pass_count = 0;
    }
    return EM_OK;
}

em_status em_get_info(const em_ctx *c, em_info *info) {
    if (!c || !info) return EM_EINVAL;
    info->rows_per_tile = c->BM;
    info->grid = c->grid;
    info->threads = kThreads;
    info->window_padded = c->Wp;
    info->bytes_per_row = c->rowbytes;
    info->lds_bytes = (int64_t)(c->fs ? c->fsLds : c->lds);
    std::snprintf(info->kernel, sizeof info->kernel, "%s",
                  c->fs     ? pass_fs_name(c->prec, c->fsMTW, c->fsE)
                  : c->kr   ? pass_kr_name(c->prec, c->krNT)
                  : c->gm   ? pass_gm_name(c->gmNT)
                  : c->ks   ? pass_ks_name(c->prec, c->BM, c->ksNT, c->ksKSS)
                  : c->wide ? pass_wide_name(c->prec, c->wNTW, c->wUR)
                  : c->fac  ? pass_fac_name(c->prec, c->fWIDE, c->fKCM, c->fEPL)
                            : pass_kernel_name(c->prec, c->BM, c->WM, c->LD));
    return EM_OK;
}

void em_destroy(em_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
}

}  // extern "C"
