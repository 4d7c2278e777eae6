// api.hip -- host orchestration and the C ABI declared in include/spmesl.h.
//
// One solve enqueues, on the context's stream:
//   column statistics -> standardised data -> S (matrix cores) ->
//   per-column working-set scaled lasso (two tiers) -> [double polish] ->
//   zero fill + scatter of B, sigma, Omega
// and then reads back one small control block (status flags and counters).
// Nothing else crosses to the host: every loop of the method runs on the
// device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "spmesl.h"
#include "common.hpp"

using namespace spmesl;

namespace {

// Control block shared by the kernels of one solve; zeroed at the start and
// read back at the end.
struct Ctl {
    unsigned long long counters[16];
    int flags;        // colstats: 1 non-finite, 2 zero variance
    int status1;      // status bits of the final phase (the polish in the mixed form)
    int status2;      // status bits of the float phase of the mixed form
    int esc_a;        // escalations of the first solves
    int dirty;        // columns the row-tiled KKT pass flagged
    int esc_c;        // escalations of the flagged columns' re-solves
    int esc_polish;   // escalations of the polish
    int pad[1];
};
static_assert(sizeof(Ctl) % 4 == 0, "Ctl is zeroed as 32-bit words");
static_assert(kNumCounters <= 16, "counter slots");

// Mixed form: the float solve stops at kMixedFloatTol and records the
// near-threshold band of width kMixedBand for the double polish, which then
// meets the caller's tolerance.
constexpr double kMixedBand = 4e-3;
constexpr double kMixedFloatTol = 1e-5;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    int64_t n = 0, p = 0, npad = 0;
    int prec = 0, rchunks = 1;
    size_t mean, scale, partial, xs, xt, hi, lo, S;
    size_t wcnt, widx, wbeta, sigma, lam, cstat, esclist, bandcnt, bandidx;
    size_t suppcnt, suppidx, suppval, pendcnt, pendidx, dirtylist, esclist2, colinfo, polinfo;
    size_t wcnt64, widx64, wbeta64, sigma64, lam64, cstat64, esclist64;
    size_t total = 0;
};

struct Bump {
    size_t cur = 0;
    size_t take(size_t bytes)
    {
        size_t o = cur;
        cur = align_up(cur + std::max<size_t>(bytes, 1), 256);
        return o;
    }
};

Plan make_plan(int64_t n, int64_t p, int prec)
{
    Plan L;
    L.n = n;
    L.p = p;
    L.prec = prec;
    L.rchunks = colstats_rchunks(n, p);
    L.npad = (n + 63) / 64 * 64;
    const size_t P = (size_t)p, N = (size_t)n;
    const size_t tsz = prec == SPMESL_FP64 ? 8 : 4;
    Bump b;
    L.mean = b.take(8 * P);
    L.scale = b.take(8 * P);
    L.partial = b.take(16 * (size_t)L.rchunks * P);
    L.xs = L.xt = L.hi = L.lo = 0;
    if (prec == SPMESL_FP64) L.xs = b.take(8 * N * P);
    if (prec == SPMESL_FP32) L.xs = b.take(4 * N * P);
    if (prec == SPMESL_MIXED) {
        L.xt = b.take(8 * N * P);
        L.hi = b.take(2 * (size_t)L.npad * P);
        L.lo = b.take(2 * (size_t)L.npad * P);
    }
    L.S = b.take(tsz * P * P);
    L.wcnt = b.take(4 * P);
    L.widx = b.take(4 * P * kWMax);
    L.wbeta = b.take(tsz * P * kWMax);
    L.sigma = b.take(8 * P);
    L.lam = b.take(8 * P);
    L.cstat = b.take(4 * P);
    L.esclist = b.take(4 * P);
    L.suppcnt = b.take(4 * P);
    L.suppidx = b.take(4 * P * kWMax);
    L.suppval = b.take(tsz * P * kWMax);
    L.pendcnt = b.take(4 * P);
    L.pendidx = b.take(4 * P * kPendMax);
    L.dirtylist = b.take(4 * P);
    L.esclist2 = b.take(4 * P);
    L.colinfo = b.take(16 * P);
    L.polinfo = prec == SPMESL_MIXED ? b.take(32 * P) : 0;
    L.bandcnt = L.bandidx = 0;
    L.wcnt64 = L.widx64 = L.wbeta64 = L.sigma64 = L.lam64 = L.cstat64 = L.esclist64 = 0;
    if (prec == SPMESL_MIXED) {
        L.bandcnt = b.take(4 * P);
        L.bandidx = b.take(4 * P * kBandMax);
        L.wcnt64 = b.take(4 * P);
        L.widx64 = b.take(4 * P * kWMax);
        L.wbeta64 = b.take(8 * P * kWMax);
        L.sigma64 = b.take(8 * P);
        L.lam64 = b.take(8 * P);
        L.cstat64 = b.take(4 * P);
        L.esclist64 = b.take(4 * P);
    }
    L.total = b.cur;
    return L;
}

struct DevGuard {
    int old = -1;
    bool changed = false;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&old) == hipSuccess && old != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DevGuard()
    {
        if (changed) (void)hipSetDevice(old);
    }
};

} // namespace

struct spmesl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = true;
    Ctl *pinned = nullptr;
    size_t pinned_count = 0;
    hipEvent_t ev[6] = {};
    bool have_events = false;
    std::string err;
};

#define HIPTRY(ctx, x)                                                              \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            (ctx)->err = std::string(#x) + ": " + hipGetErrorString(e_);            \
            return SPMESL_EHIP;                                                     \
        }                                                                           \
    } while (0)

static int fail(spmesl_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

static int ensure_pinned(spmesl_ctx *ctx, size_t count)
{
    if (ctx->pinned_count >= count) return SPMESL_OK;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_count = 0;
    HIPTRY(ctx, hipHostMalloc((void **)&ctx->pinned, count * sizeof(Ctl), hipHostMallocDefault));
    ctx->pinned_count = count;
    return SPMESL_OK;
}

static int ensure_workspace(spmesl_ctx *ctx, size_t bytes)
{
    if (ctx->ws_bytes >= bytes && ctx->ws) return SPMESL_OK;
    if (!ctx->ws_owned)
        return fail(ctx, SPMESL_ENOMEM,
                    "caller workspace of " + std::to_string(ctx->ws_bytes) + " bytes is smaller than the " +
                        std::to_string(bytes) + " bytes this solve needs");
    if (ctx->ws) {
        HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
        HIPTRY(ctx, hipFree(ctx->ws));
    }
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, SPMESL_ENOMEM,
                    "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    ctx->ws = (char *)p;
    ctx->ws_bytes = bytes;
    return SPMESL_OK;
}

static int validate(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt)
{
    if (!prob || !opt) return fail(ctx, SPMESL_EINVAL, "null problem or options");
    if (!prob->X) return fail(ctx, SPMESL_EINVAL, "X is null");
    if (prob->n < 2) return fail(ctx, SPMESL_EINVAL, "n must be >= 2");
    if (prob->p < 2) return fail(ctx, SPMESL_EINVAL, "p must be >= 2");
    if (prob->p > (int64_t)1 << 30) return fail(ctx, SPMESL_EINVAL, "p too large");
    if (prob->ldx < prob->p) return fail(ctx, SPMESL_EINVAL, "ldx must be >= p");
    if (!(opt->lambda0 > 0.0) || !std::isfinite(opt->lambda0))
        return fail(ctx, SPMESL_EINVAL, "lambda0 must be finite and > 0");
    if (!(opt->tol > 0.0) || !std::isfinite(opt->tol))
        return fail(ctx, SPMESL_EINVAL, "tol must be finite and > 0");
    if (opt->precision < SPMESL_FP64 || opt->precision > SPMESL_MIXED)
        return fail(ctx, SPMESL_EINVAL, "unknown precision");
    if (opt->output_scale != SPMESL_SCALE_ORIGINAL && opt->output_scale != SPMESL_SCALE_STANDARDIZED)
        return fail(ctx, SPMESL_EINVAL, "unknown output_scale");
    return SPMESL_OK;
}

// The p regressions: first solves (screen + one working-set solve), the
// escalations, the row-tiled KKT pass over every column, and the re-solves of
// the columns it flagged.  When one row of S does not fit in LDS the first
// solves run their own in-wave KKT passes instead.
template <typename T>
static void enqueue_columns(const Plan &L, char *ws, Ctl *dctl, const spmesl_options *opt,
                            double tol, double band, int max_outer, int max_sweeps, int max_rounds,
                            hipStream_t s)
{
    const int64_t p = L.p;
    const int rj = kkt_rows_per_block(p, sizeof(T), (size_t)80 * 1024) > 0
                       ? kkt_rows_per_block(p, sizeof(T), (size_t)80 * 1024)
                       : kkt_rows_per_block(p, sizeof(T), (size_t)160 * 1024);
    ColArgs<T> a{};
    a.S = (const T *)(ws + L.S);
    a.p = p;
    a.lambda0 = (T)opt->lambda0;
    a.tol = (T)tol;
    a.kkt_tol = (T)tol;
    a.band = (T)band;
    a.max_outer = max_outer;
    a.max_sweeps = max_sweeps;
    a.max_rounds = max_rounds;
    a.w_cnt = (int *)(ws + L.wcnt);
    a.w_idx = (int *)(ws + L.widx);
    a.w_beta = (T *)(ws + L.wbeta);
    a.sigma = (double *)(ws + L.sigma);
    a.lam_used = (double *)(ws + L.lam);
    a.col_status = (int *)(ws + L.cstat);
    a.supp_cnt = (int *)(ws + L.suppcnt);
    a.supp_idx = (int *)(ws + L.suppidx);
    a.supp_val = (T *)(ws + L.suppval);
    a.pend_cnt = (int *)(ws + L.pendcnt);
    a.pend_idx = (int *)(ws + L.pendidx);
    a.band_cnt = band > 0.0 ? (int *)(ws + L.bandcnt) : nullptr;
    a.band_idx = band > 0.0 ? (int *)(ws + L.bandidx) : nullptr;
    a.colinfo = (int *)(ws + L.colinfo);
    a.counters = dctl->counters;
    a.flags = &dctl->flags;
    // first solves
    a.mode = 0;
    a.defer_kkt = rj > 0;
    a.esc_cnt = &dctl->esc_a;
    a.esc_list = (int *)(ws + L.esclist);
    launch_colsolve(a, 0, s);
    a.mode = 1;
    a.work_list = (const int *)(ws + L.esclist);
    a.work_cnt = &dctl->esc_a;
    launch_colsolve(a, 1, s);
    if (rj == 0) return;
    KktArgs<T> k{};
    k.S = a.S;
    k.p = p;
    k.kkt_tol = a.kkt_tol;
    k.band = a.band;
    k.lam_used = a.lam_used;
    k.col_status = a.col_status;
    k.w_cnt = a.w_cnt;
    k.w_idx = a.w_idx;
    k.supp_cnt = a.supp_cnt;
    k.supp_idx = a.supp_idx;
    k.supp_val = a.supp_val;
    k.pend_cnt = a.pend_cnt;
    k.pend_idx = a.pend_idx;
    k.dirty_cnt = &dctl->dirty;
    k.dirty_list = (int *)(ws + L.dirtylist);
    k.band_cnt = a.band_cnt;
    k.band_idx = a.band_idx;
    k.flags = &dctl->flags;
    launch_kkt_rows(k, rj, s);
    // re-solve the flagged columns
    a.work_list = (const int *)(ws + L.dirtylist);
    a.work_cnt = &dctl->dirty;
    a.esc_cnt = &dctl->esc_c;
    a.esc_list = (int *)(ws + L.esclist2);
    launch_colsolve(a, 0, s);
    a.work_list = (const int *)(ws + L.esclist2);
    a.work_cnt = &dctl->esc_c;
    launch_colsolve(a, 1, s);
}

// Enqueue one full solve.  ws: workspace base laid out by `L`; dctl: this
// problem's control block.  Records the phase events when `ev` is non-null.
static int enqueue_solve(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                         const spmesl_result *res, const Plan &L, char *ws, Ctl *dctl,
                         hipEvent_t *ev)
{
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n, p = prob->p;
    const int max_outer = opt->max_outer > 0 ? opt->max_outer : 1000;
    const int max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : 100000;
    const int max_rounds = opt->max_rounds > 0 ? opt->max_rounds : 64;
    double *mean = (double *)(ws + L.mean);
    double *scale = (double *)(ws + L.scale);
    const int original = opt->output_scale == SPMESL_SCALE_ORIGINAL;

    if (ev) HIPTRY(ctx, hipEventRecord(ev[0], s));
    launch_zero_words((uint32_t *)dctl, sizeof(Ctl) / 4, s);
    launch_colstats(prob->X, n, p, prob->ldx, (double *)(ws + L.partial), L.rchunks, mean, scale,
                    &dctl->flags, s);
    if (L.prec == SPMESL_FP64)
        launch_standardize_f64(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xs), s);
    else if (L.prec == SPMESL_FP32)
        launch_standardize_f32(prob->X, n, p, prob->ldx, mean, scale, (float *)(ws + L.xs), s);
    else
        launch_standardize_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                                 (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, s);
    if (ev) HIPTRY(ctx, hipEventRecord(ev[1], s));

    if (L.prec == SPMESL_FP64)
        launch_syrk_f64((const double *)(ws + L.xs), n, p, (double *)(ws + L.S), s);
    else if (L.prec == SPMESL_FP32)
        launch_syrk_f32((const float *)(ws + L.xs), n, p, (float *)(ws + L.S), s);
    else
        launch_syrk_bf16x3((const uint16_t *)(ws + L.hi), (const uint16_t *)(ws + L.lo), n, L.npad,
                           p, (float *)(ws + L.S), s);
    if (ev) HIPTRY(ctx, hipEventRecord(ev[2], s));

    if (L.prec == SPMESL_FP64)
        enqueue_columns<double>(L, ws, dctl, opt, opt->tol, 0.0, max_outer, max_sweeps, max_rounds, s);
    else
        enqueue_columns<float>(L, ws, dctl, opt,
                               std::max(opt->tol, L.prec == SPMESL_MIXED ? kMixedFloatTol
                                                                         : (double)SPMESL_FP32_TOL_FLOOR),
                               L.prec == SPMESL_MIXED ? kMixedBand : 0.0, max_outer, max_sweeps,
                               max_rounds, s);
    if (ev) HIPTRY(ctx, hipEventRecord(ev[3], s));

    if (L.prec == SPMESL_MIXED) {
        PolishArgs q{};
        q.Xt = (const double *)(ws + L.xt);
        q.S32 = (const float *)(ws + L.S);
        q.n = n;
        q.p = p;
        q.lambda0 = opt->lambda0;
        q.tol = opt->tol;
        q.max_outer = max_outer;
        q.max_sweeps = max_sweeps;
        q.max_rounds = max_rounds;
        q.band = (float)kMixedBand;
        q.w_cnt32 = (const int *)(ws + L.wcnt);
        q.w_idx32 = (const int *)(ws + L.widx);
        q.w_beta32 = (const float *)(ws + L.wbeta);
        q.sigma32 = (const double *)(ws + L.sigma);
        q.lam32 = (const double *)(ws + L.lam);
        q.band_cnt = (const int *)(ws + L.bandcnt);
        q.band_idx = (const int *)(ws + L.bandidx);
        q.col_status32 = (const int *)(ws + L.cstat);
        // |S32 - S64| per entry: bfloat16 split (3 * 2^-16) plus float
        // accumulation over n terms; plus float rounding of the gradient
        q.eps = 3.0 * std::ldexp(1.0, -16) + (double)(n + 2) * std::ldexp(1.0, -24) + 1e-6;
        q.esc_cnt = &dctl->esc_polish;
        q.esc_list = (int *)(ws + L.esclist64);
        q.w_cnt = (int *)(ws + L.wcnt64);
        q.w_idx = (int *)(ws + L.widx64);
        q.w_beta = (double *)(ws + L.wbeta64);
        q.sigma = (double *)(ws + L.sigma64);
        q.lam_used = (double *)(ws + L.lam64);
        q.col_status = (int *)(ws + L.cstat64);
        q.polinfo = (int *)(ws + L.polinfo);
        q.flags = &dctl->flags;
        launch_polish(q, s);
    }
    {
        const bool mixed = L.prec == SPMESL_MIXED;
        launch_reduce_stats(p, (const int *)(ws + L.colinfo),
                            mixed ? (const int *)(ws + L.polinfo) : nullptr,
                            (const int *)(ws + (mixed ? L.wcnt64 : L.wcnt)),
                            (const int *)(ws + (mixed ? L.cstat64 : L.cstat)), dctl->counters,
                            &dctl->status1, s);
    }
    if (ev) HIPTRY(ctx, hipEventRecord(ev[4], s));

    if (res->B) launch_fill_zero(res->B, p * p, s);
    if (res->Omega) launch_fill_zero(res->Omega, p * p, s);
    if (L.prec == SPMESL_FP64)
        launch_scatter_outputs<double>(p, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                       (const double *)(ws + L.wbeta), (const double *)(ws + L.sigma),
                                       scale, original, res->B, res->sigma, res->Omega,
                                       &dctl->flags, s);
    else if (L.prec == SPMESL_FP32)
        launch_scatter_outputs<float>(p, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                      (const float *)(ws + L.wbeta), (const double *)(ws + L.sigma),
                                      scale, original, res->B, res->sigma, res->Omega,
                                       &dctl->flags, s);
    else
        launch_scatter_outputs<double>(p, (const int *)(ws + L.wcnt64), (const int *)(ws + L.widx64),
                                       (const double *)(ws + L.wbeta64),
                                       (const double *)(ws + L.sigma64), scale, original, res->B,
                                       res->sigma, res->Omega, &dctl->flags, s);
    if (ev) HIPTRY(ctx, hipEventRecord(ev[5], s));
    HIPTRY(ctx, hipGetLastError());
    return SPMESL_OK;
}

// Status of one finished solve from its control block; fills stats.
static int decode(const Ctl &c, int64_t p, spmesl_stats *st)
{
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->columns = p;
        st->total_outer = (int64_t)c.counters[kCntOuter];
        st->max_outer = (int64_t)c.counters[kCntMaxOuter];
        st->total_sweeps = (int64_t)c.counters[kCntSweeps];
        st->total_updates = (int64_t)c.counters[kCntUpdates];
        st->total_rounds = (int64_t)c.counters[kCntRounds];
        st->max_working_set = (int64_t)c.counters[kCntMaxW];
        st->columns_noconv = (int64_t)c.counters[kCntNoconv];
        st->polish_kkt_checks = (int64_t)c.counters[kCntPolishChecks];
        st->polish_added = (int64_t)c.counters[kCntPolishAdded];
    }
    if (c.flags & 1) return SPMESL_ENONFINITE;
    if (c.flags & 2) return SPMESL_EZEROVAR;
    int bits = c.status1;
    if (bits & 4) return SPMESL_EWORKSET;
    if (bits & 2) return SPMESL_EDEGENERATE;
    if (bits & 1) return SPMESL_ENOCONV;
    return SPMESL_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *spmesl_version(void) { return "spmesl-mi355x 0.1 (gfx950)"; }

int spmesl_create(spmesl_ctx **out, int device, void *hip_stream)
{
    if (!out) return SPMESL_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SPMESL_EINVAL;
    spmesl_ctx *ctx = new (std::nothrow) spmesl_ctx();
    if (!ctx) return SPMESL_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    DevGuard g(device);
    bool ok = true;
    for (int i = 0; i < 6 && ok; ++i) ok = hipEventCreate(&ctx->ev[i]) == hipSuccess;
    ctx->have_events = ok;
    if (!ok || ensure_pinned(ctx, 1) != SPMESL_OK) {
        spmesl_destroy(ctx);
        return SPMESL_EHIP;
    }
    *out = ctx;
    return SPMESL_OK;
}

void spmesl_destroy(spmesl_ctx *ctx)
{
    if (!ctx) return;
    {
        DevGuard g(ctx->device);
        if (ctx->stream || ctx->ws) (void)hipStreamSynchronize(ctx->stream);
        if (ctx->ws && ctx->ws_owned) (void)hipFree(ctx->ws);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        for (int i = 0; i < 6; ++i)
            if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    }
    delete ctx;
}

int spmesl_set_stream(spmesl_ctx *ctx, void *hip_stream)
{
    if (!ctx) return SPMESL_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return SPMESL_OK;
}

const char *spmesl_last_error(const spmesl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int spmesl_workspace_size(const spmesl_problem *prob, const spmesl_options *opt, size_t *bytes)
{
    if (!bytes) return SPMESL_EINVAL;
    int v = validate(nullptr, prob, opt);
    if (v != SPMESL_OK) return v;
    *bytes = make_plan(prob->n, prob->p, opt->precision).total;
    return SPMESL_OK;
}

int spmesl_set_workspace(spmesl_ctx *ctx, void *device_ptr, size_t bytes)
{
    if (!ctx) return SPMESL_EINVAL;
    DevGuard g(ctx->device);
    if (ctx->ws && ctx->ws_owned) {
        HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
        HIPTRY(ctx, hipFree(ctx->ws));
    }
    if (device_ptr) {
        if (((uintptr_t)device_ptr & 255u) != 0)
            return fail(ctx, SPMESL_EINVAL, "workspace must be 256-byte aligned");
        ctx->ws = (char *)device_ptr;
        ctx->ws_bytes = bytes;
        ctx->ws_owned = false;
    } else {
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        ctx->ws_owned = true;
    }
    return SPMESL_OK;
}

int spmesl_solve(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                 spmesl_result *res)
{
    if (!ctx || !res) return SPMESL_EINVAL;
    int v = validate(ctx, prob, opt);
    if (v != SPMESL_OK) return v;
    DevGuard g(ctx->device);
    Plan L = make_plan(prob->n, prob->p, opt->precision);
    size_t ctl_off = align_up(L.total, 256);
    v = ensure_workspace(ctx, ctl_off + sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    v = ensure_pinned(ctx, 1);
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + ctl_off);
    const bool timing = (opt->flags & SPMESL_FLAG_TIMING) && ctx->have_events;
    v = enqueue_solve(ctx, prob, opt, res, L, ctx->ws, dctl, timing ? ctx->ev : nullptr);
    if (v != SPMESL_OK) return v;
    HIPTRY(ctx, hipMemcpyAsync(ctx->pinned, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    int st = decode(ctx->pinned[0], prob->p, res->stats);
    if (res->stats) {
        res->stats->nnz_B = -1;
        if (timing) {
            float ms[5];
            for (int i = 0; i < 5; ++i) HIPTRY(ctx, hipEventElapsedTime(&ms[i], ctx->ev[i], ctx->ev[i + 1]));
            res->stats->ms_standardize = ms[0];
            res->stats->ms_covariance = ms[1];
            res->stats->ms_solve = ms[2];
            res->stats->ms_polish = ms[3];
            res->stats->ms_output = ms[4];
            float tot = 0.f;
            HIPTRY(ctx, hipEventElapsedTime(&tot, ctx->ev[0], ctx->ev[5]));
            res->stats->ms_total = tot;
        }
    }
    if (st == SPMESL_ENONFINITE) ctx->err = "X holds a NaN or Inf";
    else if (st == SPMESL_EZEROVAR) ctx->err = "a column of X has zero variance";
    else if (st == SPMESL_EWORKSET) ctx->err = "a working set exceeded SPMESL_MAX_WORKING_SET";
    else if (st == SPMESL_EDEGENERATE) ctx->err = "a residual variance fell to zero";
    else if (st == SPMESL_ENOCONV) ctx->err = "an iteration cap was reached";
    return st;
}

int spmesl_solve_batch(spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                       const spmesl_options *opt, spmesl_result *res, int *status)
{
    if (!ctx || count < 0 || (count > 0 && (!probs || !res || !status))) return SPMESL_EINVAL;
    if (count == 0) return SPMESL_OK;
    DevGuard g(ctx->device);
    size_t need = 0;
    std::vector<Plan> plans((size_t)count);
    for (int i = 0; i < count; ++i) {
        int v = validate(ctx, &probs[i], opt);
        if (v != SPMESL_OK) {
            ctx->err = "problem " + std::to_string(i) + ": " + ctx->err;
            return v;
        }
        plans[(size_t)i] = make_plan(probs[i].n, probs[i].p, opt->precision);
        need = std::max(need, plans[(size_t)i].total);
    }
    size_t ctl_off = align_up(need, 256);
    int v = ensure_workspace(ctx, ctl_off + (size_t)count * sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    v = ensure_pinned(ctx, (size_t)count);
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + ctl_off);
    for (int i = 0; i < count; ++i) {
        v = enqueue_solve(ctx, &probs[i], opt, &res[i], plans[(size_t)i], ctx->ws, dctl + i, nullptr);
        if (v != SPMESL_OK) return v;
    }
    HIPTRY(ctx, hipMemcpyAsync(ctx->pinned, dctl, (size_t)count * sizeof(Ctl),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    int first = SPMESL_OK;
    for (int i = 0; i < count; ++i) {
        status[i] = decode(ctx->pinned[i], probs[i].p, res[i].stats);
        if (first == SPMESL_OK && status[i] != SPMESL_OK) first = status[i];
    }
    return first;
}

int spmesl_covariance(spmesl_ctx *ctx, const spmesl_problem *prob, int precision, void *S_out,
                      double *mean_out, double *scale_out)
{
    if (!ctx || !S_out) return SPMESL_EINVAL;
    spmesl_options opt{};
    opt.lambda0 = 1.0;
    opt.tol = 1.0;
    opt.precision = precision;
    int v = validate(ctx, prob, &opt);
    if (v != SPMESL_OK) return v;
    DevGuard g(ctx->device);
    Plan L = make_plan(prob->n, prob->p, precision);
    size_t ctl_off = align_up(L.total, 256);
    v = ensure_workspace(ctx, ctl_off + sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    char *ws = ctx->ws;
    Ctl *dctl = (Ctl *)(ws + ctl_off);
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n, p = prob->p;
    double *mean = mean_out ? mean_out : (double *)(ws + L.mean);
    double *scale = scale_out ? scale_out : (double *)(ws + L.scale);
    launch_zero_words((uint32_t *)dctl, sizeof(Ctl) / 4, s);
    launch_colstats(prob->X, n, p, prob->ldx, (double *)(ws + L.partial), L.rchunks, mean, scale,
                    &dctl->flags, s);
    if (precision == SPMESL_FP64) {
        launch_standardize_f64(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xs), s);
        launch_syrk_f64((const double *)(ws + L.xs), n, p, (double *)S_out, s);
    } else if (precision == SPMESL_FP32) {
        launch_standardize_f32(prob->X, n, p, prob->ldx, mean, scale, (float *)(ws + L.xs), s);
        launch_syrk_f32((const float *)(ws + L.xs), n, p, (float *)S_out, s);
    } else {
        launch_standardize_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                                 (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, s);
        launch_syrk_bf16x3((const uint16_t *)(ws + L.hi), (const uint16_t *)(ws + L.lo), n, L.npad, p,
                           (float *)S_out, s);
    }
    HIPTRY(ctx, hipGetLastError());
    v = ensure_pinned(ctx, 1);
    if (v != SPMESL_OK) return v;
    HIPTRY(ctx, hipMemcpyAsync(ctx->pinned, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[0].flags & 1) return fail(ctx, SPMESL_ENONFINITE, "X holds a NaN or Inf");
    if (ctx->pinned[0].flags & 2) return fail(ctx, SPMESL_EZEROVAR, "a column of X has zero variance");
    return SPMESL_OK;
}

int spmesl_symmetrize(spmesl_ctx *ctx, int64_t p, const double *Omega1, double *Omega)
{
    if (!ctx || !Omega1 || !Omega || p < 1) return fail(ctx, SPMESL_EINVAL, "bad symmetrize arguments");
    if (Omega1 == Omega) return fail(ctx, SPMESL_EINVAL, "symmetrize is not in place");
    DevGuard g(ctx->device);
    launch_symmetrize_dense(p, Omega1, Omega, ctx->stream);
    HIPTRY(ctx, hipGetLastError());
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    return SPMESL_OK;
}

} // extern "C"
