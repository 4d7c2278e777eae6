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
#include <mutex>
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
    int dense;        // columns handed to the dense tier
    int dense64;      // columns handed to the dense tier by the polish
    int pool;         // pool entries taken by the dense tier's results
    int pool64;
    int pad[1];
};
static_assert(sizeof(Ctl) % 4 == 0, "Ctl is zeroed as 32-bit words");
static_assert(kNumCounters <= 16, "counter slots");

// Mixed form: the float solve stops at kMixedFloatTol and records the
// near-threshold band of width kMixedBand for the double polish, which then
// meets the caller's tolerance.
constexpr double kMixedBand = 4e-3;
constexpr double kMixedFloatTol = 3e-5;
// Screen factor of the first working sets.  At p = 5000 (block AR(1)) the
// flagged columns fall from 12% to 4% of p against a factor of 1, for 10.6
// instead of 5.3 coordinates per first working set; at 0.7 up to 93% of the
// columns of a scale-free p = 20000 workload would outgrow 32 coordinates.
constexpr int kScreenPermille = 800;
// Rows per block of the dense tier's delayed update, and the largest V whose
// S[V, V] the double dense tier of the mixed form keeps (8 MB).
constexpr int kDenseBlock = 32;
constexpr int64_t kDenseDataMax = 1024;
// Workgroups of the zero fill of the dense outputs (64 blocks of
// nontemporal 16-byte stores write about 5 TB/s beside the covariance kernel).
constexpr int kFillBlocks = 64;

// The launch shapes of a solve: the context's spmesl_tuning with its zero
// fields replaced by the defaults.
struct Tune {
    int dense_block = kDenseBlock;
    int fill_blocks = kFillBlocks;
    int kkt_rows = 0;  // 0: the most that fit
    int screen_permille = kScreenPermille;
    int fill_split = 0;
};
Tune resolve_tune(const spmesl_tuning &t)
{
    Tune u;
    if (t.dense_block > 0) u.dense_block = t.dense_block;
    if (t.fill_blocks > 0) u.fill_blocks = t.fill_blocks;
    if (t.kkt_rows > 0) u.kkt_rows = t.kkt_rows;
    if (t.screen_permille > 0) u.screen_permille = t.screen_permille;
    u.fill_split = t.fill_split;
    return u;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    int64_t n = 0, p = 0, npad = 0;
    int prec = 0, rchunks = 1;
    size_t mean, scale, partial, xs, xt, hi, lo, S;
    size_t wcnt, widx, wbeta, sigma, lam, cstat, esclist, bandcnt, bandidx;
    size_t suppcnt, suppidx, suppval, pendcnt, pendidx, dirtylist, esclist2, colinfo, polinfo;
    size_t wcnt64, widx64, wbeta64, sigma64, lam64, cstat64, esclist64;
    // the dense tier: queues, result offsets into the pools, workspace
    size_t dq, dq64, woff, woff64, dmark, dv, dvold, dr, dbd, dbp, dsk, dsvv, de;
    int64_t pool_cap = 0, svv_cap = 0;
    // the data form (no S): workgroups of its dense tier and rows of V each
    bool data = false;
    int dgroups = 1;
    // workgroups of the S forms' dense tiers (each with its own slice of
    // the dense workspace)
    int sgroups = 1;
    int64_t dvcap = 0;
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

// The data form (SPMESL_FLAG_DATA_FORM, double): no S.  The standardised
// data Xt, the per-column lists, and the dense tier's workspace for
// kDataGroups workgroups whose V holds up to kDataVcap rows.
constexpr int kDataGroups = 128;
constexpr int64_t kDataVcap = 1024;  // V beyond it fails (S_VV of 8 MB per workgroup)

Plan make_plan_data(int64_t n, int64_t p)
{
    Plan L;
    L.n = n;
    L.p = p;
    L.prec = SPMESL_FP64;
    L.data = true;
    L.rchunks = colstats_rchunks(n, p);
    L.npad = (n + 63) / 64 * 64;
    const size_t P = (size_t)p, N = (size_t)n;
    const int64_t groups = (p + 15) / 16;
    L.dgroups = (int)(groups < kDataGroups ? groups : kDataGroups);
    L.dvcap = p < kDataVcap ? p : kDataVcap;
    const size_t G = (size_t)L.dgroups, VC = (size_t)L.dvcap;
    Bump b;
    L.mean = b.take(8 * P);
    L.scale = b.take(8 * P);
    L.partial = b.take(16 * (size_t)L.rchunks * P);
    L.xt = b.take(8 * N * P);
    L.hi = b.take(2 * (size_t)L.npad * P);
    L.lo = b.take(2 * (size_t)L.npad * P);
    L.pool_cap = std::min<int64_t>(p * p, 32 * p + 65536);
    const size_t lists = P * kWMax + (size_t)L.pool_cap;
    L.wcnt = b.take(4 * P);
    L.widx = b.take(4 * lists);
    L.wbeta = b.take(8 * lists);
    L.woff = b.take(4 * P);
    L.sigma = b.take(8 * P);
    L.lam = b.take(8 * P);
    L.cstat = b.take(4 * P);
    L.colinfo = b.take(16 * P);
    L.pendcnt = b.take(4 * P);
    L.dmark = b.take(4 * G * P);
    L.dv = b.take(4 * G * VC);
    L.dvold = b.take(4 * G * VC);
    L.dr = b.take(8 * 16 * G * VC);
    L.dbd = b.take(8 * 16 * G * VC);
    L.dbp = b.take(8 * 16 * G * VC);
    L.dsk = b.take(8 * 16 * G * VC);
    L.svv_cap = L.dvcap;
    L.dsvv = b.take(8 * G * VC * VC);
    L.de = b.take(8 * 16 * N * G);
    L.total = b.cur;
    return L;
}

// The S forms' dense tiers run on G workgroups, each with a slice of the
// dense workspace: the marks, V and its previous copy (p each), R, B, B_prev
// and the screen values (16 p each) and, in the mixed form, S[V, V] and E of
// the double stage.  G is the number of slices that fit a quarter of the
// rest of the plan (at least 16 MB), from 1 to kDenseGroupsMax.
constexpr int kDenseGroupsMax = 32;
constexpr size_t kDenseBudgetFloor = (size_t)16 << 20;
Plan make_plan_g(int64_t n, int64_t p, int prec, int G);

Plan make_plan(int64_t n, int64_t p, int prec, bool data = false)
{
    if (data) return make_plan_data(n, p);
    const Plan one = make_plan_g(n, p, prec, 1);
    const size_t P = (size_t)p;
    size_t slice = 4 * P + 8 * P + 4 * 8 * 16 * P;
    if (prec == SPMESL_MIXED) slice += 8 * (size_t)one.svv_cap * (size_t)one.svv_cap + 8 * 16 * (size_t)n;
    const size_t budget = std::max(kDenseBudgetFloor, one.total / 4);
    const int G = (int)std::min<size_t>(kDenseGroupsMax, std::max<size_t>(1, budget / slice));
    return G == 1 ? one : make_plan_g(n, p, prec, G);
}

Plan make_plan_g(int64_t n, int64_t p, int prec, int G)
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
    // per-column lists hold kWMax entries each; the dense tier's longer
    // results go to a pool after them
    L.pool_cap = std::min<int64_t>(p * p, 32 * p + 65536);
    const size_t lists = P * kWMax + (size_t)L.pool_cap;
    L.wcnt = b.take(4 * P);
    L.widx = b.take(4 * lists);
    L.wbeta = b.take(tsz * lists);
    L.woff = b.take(4 * P);
    L.dq = b.take(4 * P);
    L.sgroups = G;
    const size_t GG = (size_t)G;
    L.dmark = b.take(4 * P * GG);
    L.dv = b.take(4 * P * GG);
    L.dvold = b.take(4 * P * GG);
    L.dr = b.take(8 * 16 * P * GG);
    L.dbd = b.take(8 * 16 * P * GG);
    L.dbp = b.take(8 * 16 * P * GG);
    L.dsk = b.take(8 * 16 * P * GG);
    L.dq64 = L.woff64 = L.dsvv = L.de = 0;
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
        L.widx64 = b.take(4 * lists);
        L.wbeta64 = b.take(8 * lists);
        L.woff64 = b.take(4 * P);
        L.dq64 = b.take(4 * P);
        // S[V, V] of the double dense tier (formed from the data)
        L.svv_cap = p < kDenseDataMax ? p : kDenseDataMax;
        L.dsvv = b.take(8 * (size_t)L.svv_cap * (size_t)L.svv_cap * GG);
        L.de = b.take(8 * 16 * N * GG);
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

// Device memory of spmesl_solve_noalloc: one array per GPU, part of the
// library's code object, held until the process ends.  Host code never uses
// this name as an address (on the host it is only a handle of the symbol):
// the array's device address is looked up once per device with
// hipGetSymbolAddress when the first context on that device is created,
// and kernels receive that address.
static __device__ __align__(256) unsigned char scratch[SPMESL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Address of `scratch` on `device`, which must be the current device;
// nullptr (and the HIP error in *err) when it cannot be found.
char *scratch_address(int device, hipError_t *err)
{
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
        }
        g_scratch_addr[device] = (char *)ptr;
        g_scratch_err[device] = e;
        g_scratch_done[device] = true;
    }
    *err = g_scratch_err[device];
    return g_scratch_addr[device];
}
} // namespace

struct spmesl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = true;
    Ctl *pinned = nullptr;
    size_t pinned_count = 0;
    // host staging of the grouped batch's launch tables
    unsigned char *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t ev[6] = {};
    bool have_events = false;
    // second stream (default priority) for the zero fill of the dense
    // outputs, which overlaps the latency-bound column solves
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t fork2 = nullptr, join2 = nullptr;  // statistics reduction beside the scatter
    // per-launch timing (SPMESL_FLAG_TIMING): events in enqueue order, each
    // with the index of the previous event on its stream
    static constexpr int kMaxMarks = 48;
    hipEvent_t kev[kMaxMarks] = {};
    const char *kname[kMaxMarks] = {};
    int kprev[kMaxMarks] = {};
    int nmarks = 0;
    bool kev_ok = false;
    float kms[kMaxMarks] = {};
    // replay of the last call's whole enqueue sequence as one HIP graph,
    // captured on `cap` (a capturable stream) and launched on `stream`
    hipStream_t cap = nullptr;
    struct CachedGraph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
    };
    static constexpr size_t kMaxGraphs = 4;
    std::vector<CachedGraph> graphs;  // most recently used first
    // device address of this device's no-allocation scratch array (nullptr
    // if the lookup failed; scratch_err then holds the HIP error)
    char *scratch_dev = nullptr;
    hipError_t scratch_err = hipSuccess;
    spmesl_tuning tune = {};     // launch shapes (zero fields: defaults)
    int *tune_status = nullptr;  // device status word of the autotuner's solves
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

// The status code of one finished solve from its control block, on the
// device (the asynchronous entry point's status; the host-side decode()
// below is the same mapping).
__global__ void k_decode_status(const Ctl *c, int *status)
{
    int st = SPMESL_OK;
    const int bits = c->status1;
    if (c->flags & 1) st = SPMESL_ENONFINITE;
    else if (c->flags & 2) st = SPMESL_EZEROVAR;
    else if (bits & 4) st = SPMESL_EWORKSET;
    else if (bits & 2) st = SPMESL_EDEGENERATE;
    else if (bits & 1) st = SPMESL_ENOCONV;
    *status = st;
}

// Bytes that identify a call for graph replay: every pointer, size and
// option the enqueued kernels take, plus the streams.
struct KeyBuf {
    std::vector<unsigned char> b;
    template <typename V> void add(const V &v)
    {
        const unsigned char *q = reinterpret_cast<const unsigned char *>(&v);
        b.insert(b.end(), q, q + sizeof(V));
    }
};

static void key_problem(KeyBuf &k, const spmesl_problem &pr, const spmesl_result &r)
{
    k.add(pr.X);
    k.add(pr.n);
    k.add(pr.p);
    k.add(pr.ldx);
    k.add(pr.B0);
    k.add(pr.sigma0);
    k.add(r.B);
    k.add(r.sigma);
    k.add(r.Omega);
}

static void key_tuning(KeyBuf &k, const spmesl_tuning &t)
{
    k.add(t.dense_block);
    k.add(t.fill_blocks);
    k.add(t.kkt_rows);
    k.add(t.screen_permille);
    k.add(t.fill_split);
}

static void key_options(KeyBuf &k, const spmesl_options &o)
{
    k.add(o.lambda0);
    k.add(o.tol);
    k.add(o.max_outer);
    k.add(o.max_sweeps);
    k.add(o.max_rounds);
    k.add(o.precision);
    k.add(o.output_scale);
    k.add(o.flags & (SPMESL_FLAG_FULL_KKT | SPMESL_FLAG_DATA_FORM));
}

// Records the per-launch events of a timed solve; a null Marker records
// nothing.  mark(s, name) closes the step that ran on s since the previous
// mark on s; a null name opens the stream's first step.
struct Marker {
    spmesl_ctx *ctx;
    hipStream_t streams[2] = {};
    int last[2] = {-1, -1};
    explicit Marker(spmesl_ctx *c) : ctx(c) { ctx->nmarks = 0; }
    void mark(hipStream_t s, const char *name)
    {
        int si = -1;
        for (int i = 0; i < 2 && si < 0; ++i)
            if (streams[i] == s && last[i] >= 0) si = i;
        if (si < 0)
            for (int i = 0; i < 2 && si < 0; ++i)
                if (last[i] < 0) {
                    si = i;
                    streams[i] = s;
                }
        const int e = ctx->nmarks;
        if (si < 0 || e >= spmesl_ctx::kMaxMarks) return;
        if (hipEventRecord(ctx->kev[e], s) != hipSuccess) return;
        ctx->kname[e] = last[si] < 0 ? nullptr : name;
        ctx->kprev[e] = last[si];
        last[si] = e;
        ctx->nmarks = e + 1;
    }
};

static inline void mark(Marker *m, hipStream_t s, const char *name)
{
    if (m) m->mark(s, name);
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
    if ((opt->flags & SPMESL_FLAG_DATA_FORM) && opt->precision != SPMESL_FP64)
        return fail(ctx, SPMESL_EINVAL, "the data form runs in SPMESL_FP64 only");
    return SPMESL_OK;
}

// The zero fill of the dense outputs needs nothing of the solve: it is
// forked onto the context's second stream at a point where the main stream
// leaves HBM to it (chosen per form by the caller), and the scatter waits
// for it.
// `which`: 1 fills B, 2 fills Omega (a solve may fork twice; the second
// fork's join covers both, the second stream being in order).
static int fork_output_fill(spmesl_ctx *ctx, const spmesl_result *res, int64_t p, hipStream_t s, Marker *mk,
                            int which = 3)
{
    const int fb = resolve_tune(ctx->tune).fill_blocks;
    double *B = (which & 1) ? res->B : nullptr;
    double *Om = (which & 2) ? res->Omega : nullptr;
    if (!B && !Om) return SPMESL_OK;
    HIPTRY(ctx, hipEventRecord(ctx->fork, s));
    HIPTRY(ctx, hipStreamWaitEvent(ctx->side, ctx->fork, 0));
    mark(mk, ctx->side, nullptr);
    if (B) {
        launch_fill_zero(B, p * p, ctx->side, fb);
        mark(mk, ctx->side, "fill_B");
    }
    if (Om) {
        launch_fill_zero(Om, p * p, ctx->side, fb);
        mark(mk, ctx->side, "fill_Omega");
    }
    HIPTRY(ctx, hipEventRecord(ctx->join, ctx->side));
    return SPMESL_OK;
}

// The dense tier (dense.hip) for the columns the 128-coordinate tier handed
// over, reading S and writing the columns' results in place.
template <typename T>
static void enqueue_dense(const Plan &L, char *ws, Ctl *dctl, const ColArgs<T> &a, const Tune &tu, hipStream_t s,
                          Marker *mk)
{
    DenseArgs<T> d{};
    d.S = a.S;
    d.Xt = nullptr;
    d.n = L.n;
    d.p = L.p;
    d.pv = a.pv;
    d.lambda0 = a.lambda0;
    d.tol = a.tol;
    d.kkt_tol = a.kkt_tol;
    d.max_outer = a.max_outer;
    d.max_sweeps = a.max_sweeps;
    d.max_rounds = a.max_rounds;
    d.block = tu.dense_block;
    d.queue = a.dense_list;
    d.qcnt = a.dense_cnt;
    d.w_cnt = a.w_cnt;
    d.w_idx = a.w_idx;
    d.w_beta = a.w_beta;
    d.w_off = (int *)(ws + L.woff);
    d.sigma = a.sigma;
    d.lam_used = a.lam_used;
    d.col_status = a.col_status;
    d.pool_cnt = &dctl->pool;
    d.pool_cap = L.pool_cap;
    d.band_cnt = a.band_cnt;
    d.info = a.colinfo;
    d.info_stride = 4;
    d.mark = (int *)(ws + L.dmark);
    d.V = (int *)(ws + L.dv);
    d.Vold = (int *)(ws + L.dvold);
    d.R = (T *)(ws + L.dr);
    d.Bd = (T *)(ws + L.dbd);
    d.Bp = (T *)(ws + L.dbp);
    d.vcap = L.p;
    d.sk = (T *)(ws + L.dsk);
    d.counters = a.counters;
    d.flags = a.flags;
    DenseSrc<T> src{};
    src.cnt = a.w_cnt;
    src.idx = a.w_idx;
    src.beta = a.w_beta;
    src.off = d.w_off;
    src.sigma = a.sigma;
    src.pend_cnt = a.pend_cnt;
    src.pend_idx = a.pend_idx;
    launch_dense<T, T>(d, src, s, L.sgroups);
    mark(mk, s, "dense");
}

// The p regressions: first solves (screen + one working-set solve), the
// escalations, the row-tiled KKT pass over every column, and the re-solves of
// the columns it flagged.  When one row of S does not fit in LDS the first
// solves run their own in-wave KKT passes instead.  With k0 > 0 only the
// columns k0 .. p-1 are solved, each on the predictors 0 .. k0-1 (the scaled
// lassos of responses appended to a design), with in-wave KKT passes.
// Rows of S per tile of the row-tiled KKT pass (0: the pass does not apply).
template <typename T>
static int kkt_rows_for(int64_t p, int64_t k0, const Tune &tu)
{
    int rj = k0 > 0 ? 0 : kkt_rows_per_block(p, sizeof(T), (size_t)160 * 1024);
    if (rj > 0 && tu.kkt_rows > 0 && tu.kkt_rows < rj) rj = tu.kkt_rows >= 2 ? 2 : 1;
    return rj;
}

// The column solves' arguments for one problem (the phase fields mode,
// screened, defer_kkt, work list and escalation queue are set per launch).
template <typename T>
static ColArgs<T> make_col_args(const Plan &L, char *ws, Ctl *dctl, const spmesl_options *opt, double tol,
                                double band, int max_outer, int max_sweeps, int max_rounds, int64_t k0, bool warm)
{
    const int64_t p = L.p;
    ColArgs<T> a{};
    a.S = (const T *)(ws + L.S);
    a.p = p;
    a.k0 = k0;
    a.pv = k0 > 0 ? k0 : p;
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
    a.warm = warm ? 1 : 0;
    a.dense_cnt = &dctl->dense;
    a.dense_list = (int *)(ws + L.dq);
    return a;
}

// The row-tiled KKT pass's arguments for one problem.
template <typename T>
static KktArgs<T> make_kkt_args(const ColArgs<T> &a, const Plan &L, char *ws, Ctl *dctl)
{
    KktArgs<T> k{};
    k.S = a.S;
    k.p = L.p;
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
    return k;
}

template <typename T, typename F>
static int enqueue_columns(const Plan &L, char *ws, Ctl *dctl, const spmesl_options *opt, const Tune &tu,
                           double tol, double band, int max_outer, int max_sweeps, int max_rounds,
                           hipStream_t s, Marker *mk, F &&after_kkt, int64_t k0 = 0, bool warm = false)
{
    const int rj = kkt_rows_for<T>(L.p, k0, tu);
    ColArgs<T> a = make_col_args<T>(L, ws, dctl, opt, tol, band, max_outer, max_sweeps, max_rounds, k0, warm);
    // first solves (their screen lists were written with S).  With the
    // row-tiled pass, the columns they hand to the wide tier join the
    // re-solves' queue: one wide launch after the re-solves finishes both (an
    // escalated column is final after it, and the row-tiled pass examines
    // deferred columns only), which saves a launch that usually finds no work.
    a.mode = 0;
    a.screened = 1;
    a.defer_kkt = rj > 0;
    a.esc_cnt = rj > 0 ? &dctl->esc_c : &dctl->esc_a;
    a.esc_list = (int *)(ws + (rj > 0 ? L.esclist2 : L.esclist));
    launch_colsolve(a, 0, s);
    mark(mk, s, "colsolve_first");
    if (rj == 0) {
        a.mode = 1;
        a.screened = 0;
        a.work_list = (const int *)(ws + L.esclist);
        a.work_cnt = &dctl->esc_a;
        launch_colsolve(a, 1, s);
        mark(mk, s, "colsolve_first_wide");
        if (band == 0.0) enqueue_dense<T>(L, ws, dctl, a, tu, s, mk);
        return after_kkt();
    }
    const KktArgs<T> k = make_kkt_args<T>(a, L, ws, dctl);
    launch_kkt_rows(k, rj, s);
    mark(mk, s, "kkt_rows");
    const int v = after_kkt();
    if (v != SPMESL_OK) return v;
    // re-solve the flagged columns
    a.mode = 1;
    a.screened = 0;
    a.work_list = (const int *)(ws + L.dirtylist);
    a.work_cnt = &dctl->dirty;
    a.esc_cnt = &dctl->esc_c;
    a.esc_list = (int *)(ws + L.esclist2);
    launch_colsolve(a, 0, s);
    mark(mk, s, "colsolve_resume");
    a.work_list = (const int *)(ws + L.esclist2);
    a.work_cnt = &dctl->esc_c;
    launch_colsolve(a, 1, s);
    mark(mk, s, "colsolve_resume_wide");
    // the dense tier; in the mixed form (band > 0) its columns go to the
    // double polish's dense tier instead
    if (band == 0.0) enqueue_dense<T>(L, ws, dctl, a, tu, s, mk);
    return SPMESL_OK;
}

// Column statistics and the standardised copies of X the form needs.
static void enqueue_standardize(const Plan &L, const spmesl_problem *prob, char *ws, Ctl *dctl, hipStream_t s,
                                Marker *mk)
{
    const int64_t n = prob->n, p = prob->p;
    double *mean = (double *)(ws + L.mean);
    double *scale = (double *)(ws + L.scale);
    if (L.prec == SPMESL_MIXED &&
        launch_stats_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                           (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, &dctl->flags,
                           (int *)(ws + L.pendcnt), s)) {
        mark(mk, s, "standardize");
        return;
    }
    launch_colstats(prob->X, n, p, prob->ldx, (double *)(ws + L.partial), L.rchunks, mean, scale,
                    &dctl->flags, (int *)(ws + L.pendcnt), s);
    mark(mk, s, "colstats");
    if (L.prec == SPMESL_FP64)
        launch_standardize_f64(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xs), s);
    else if (L.prec == SPMESL_FP32)
        launch_standardize_f32(prob->X, n, p, prob->ldx, mean, scale, (float *)(ws + L.xs), s);
    else
        launch_standardize_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                                 (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, s);
    mark(mk, s, "standardize");
}

// Tolerance of the column solves: the caller's in double, floored in the
// float and mixed forms.
static double column_tol(const Plan &L, const spmesl_options *opt)
{
    return L.prec == SPMESL_FP64 ? opt->tol
                                 : std::max(opt->tol, L.prec == SPMESL_MIXED ? kMixedFloatTol
                                                                             : (double)SPMESL_FP32_TOL_FLOOR);
}

// The first solves' working sets, {j : |s_jk| > f lambda0 + tol}, are taken
// where S is written.  At beta = 0 the KKT test is |s_jk| > lambda0 + tol; the
// final lambda is sigma lambda0 with sigma < 1, so the lower factor starts
// most columns on their final support (a strong-rule style start: the
// row-tiled KKT pass still checks every column, so the factor changes the
// work, never the result).
static Screen make_screen(const Plan &L, char *ws, const spmesl_options *opt, const Tune &tu, double tol_cols)
{
    const double screen = tu.screen_permille * 1e-3;
    Screen sc;
    sc.thr64 = screen * opt->lambda0 + tol_cols;
    {
        volatile float a = (float)(screen * opt->lambda0), b = (float)tol_cols;
        sc.thr32 = a + b;
    }
    sc.cnt = (int *)(ws + L.pendcnt);  // zeroed by the column statistics
    sc.idx = (int *)(ws + L.pendidx);
    return sc;
}

// The mixed form's double polish of one problem.
static PolishArgs make_polish_args(const Plan &L, char *ws, Ctl *dctl, const spmesl_options *opt, int max_outer,
                                   int max_sweeps, int max_rounds)
{
    const int64_t n = L.n;
    PolishArgs q{};
    q.Xt = (const double *)(ws + L.xt);
    q.S32 = (const float *)(ws + L.S);
    q.n = n;
    q.p = L.p;
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
    q.full_kkt = (opt->flags & SPMESL_FLAG_FULL_KKT) ? 1 : 0;
    q.dense_cnt = &dctl->dense64;
    q.dense_list = (int *)(ws + L.dq64);
    return q;
}

// The columns whose double working sets outgrow the polish's: the dense
// tier in double, from the float solution, with S[V, V] and the gradients
// taken from the standardised data.
static void enqueue_dense64(const PolishArgs &q, const Plan &L, char *ws, Ctl *dctl, const spmesl_options *opt,
                            const Tune &tu, hipStream_t s, Marker *mk)
{
    DenseArgs<double> d{};
    d.S = nullptr;
    d.Xt = q.Xt;
    d.n = L.n;
    d.p = L.p;
    d.pv = L.p;
    d.lambda0 = opt->lambda0;
    d.tol = opt->tol;
    d.kkt_tol = opt->tol;
    d.max_outer = q.max_outer;
    d.max_sweeps = q.max_sweeps;
    d.max_rounds = q.max_rounds;
    d.block = tu.dense_block;
    d.queue = q.dense_list;
    d.qcnt = q.dense_cnt;
    d.w_cnt = q.w_cnt;
    d.w_idx = q.w_idx;
    d.w_beta = q.w_beta;
    d.w_off = (int *)(ws + L.woff64);
    d.sigma = q.sigma;
    d.lam_used = q.lam_used;
    d.col_status = q.col_status;
    d.pool_cnt = &dctl->pool64;
    d.pool_cap = L.pool_cap;
    d.band_cnt = nullptr;
    d.info = q.polinfo;
    d.info_stride = 8;
    d.mark = (int *)(ws + L.dmark);
    d.V = (int *)(ws + L.dv);
    d.Vold = (int *)(ws + L.dvold);
    d.R = (double *)(ws + L.dr);
    d.Bd = (double *)(ws + L.dbd);
    d.Bp = (double *)(ws + L.dbp);
    d.vcap = L.p;
    d.sk = (double *)(ws + L.dsk);
    d.Svv = (double *)(ws + L.dsvv);
    d.svv_cap = L.svv_cap;
    d.E = (double *)(ws + L.de);
    d.counters = dctl->counters;
    d.flags = &dctl->flags;
    DenseSrc<float> src{};
    src.cnt = q.w_cnt32;
    src.idx = q.w_idx32;
    src.beta = q.w_beta32;
    src.off = (const int *)(ws + L.woff);
    src.sigma = q.sigma32;
    src.pend_cnt = (const int *)(ws + L.pendcnt);
    src.pend_idx = (const int *)(ws + L.pendidx);
    launch_dense<double, float>(d, src, s, L.sgroups);
    mark(mk, s, "dense_polish");
}

// The statistics reduction of one problem (reads only the column results).
static void enqueue_reduce_stats(const Plan &L, char *ws, Ctl *dctl, hipStream_t s)
{
    const bool mixed = L.prec == SPMESL_MIXED;
    launch_reduce_stats(L.p, (const int *)(ws + L.colinfo), mixed ? (const int *)(ws + L.polinfo) : nullptr,
                        (const int *)(ws + (mixed ? L.wcnt64 : L.wcnt)),
                        (const int *)(ws + (mixed ? L.cstat64 : L.cstat)), dctl->counters, &dctl->status1, s);
}

// B, sigma and Omega of one problem from its column results.
static void enqueue_scatter(const Plan &L, char *ws, Ctl *dctl, const spmesl_result *res, int original,
                            hipStream_t s)
{
    const int64_t p = L.p;
    const double *scale = (const double *)(ws + L.scale);
    if (L.prec == SPMESL_FP64)
        launch_scatter_outputs<double>(p, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                       (const double *)(ws + L.wbeta), (const int *)(ws + L.woff),
                                       (const double *)(ws + L.sigma), scale, original, res->B, res->sigma,
                                       res->Omega, &dctl->flags, s);
    else if (L.prec == SPMESL_FP32)
        launch_scatter_outputs<float>(p, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                      (const float *)(ws + L.wbeta), (const int *)(ws + L.woff),
                                      (const double *)(ws + L.sigma), scale, original, res->B, res->sigma,
                                      res->Omega, &dctl->flags, s);
    else
        launch_scatter_outputs<double>(p, (const int *)(ws + L.wcnt64), (const int *)(ws + L.widx64),
                                       (const double *)(ws + L.wbeta64), (const int *)(ws + L.woff64),
                                       (const double *)(ws + L.sigma64), scale, original, res->B, res->sigma,
                                       res->Omega, &dctl->flags, s);
}

// Enqueue one full solve.  ws: workspace base laid out by `L`; dctl: this
// problem's control block.  Records the phase events when `ev` is non-null.
static int enqueue_data_form(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                             const spmesl_result *res, const Plan &L, char *ws, Ctl *dctl, hipEvent_t *ev);

static int enqueue_solve(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                         const spmesl_result *res, const Plan &L, char *ws, Ctl *dctl,
                         hipEvent_t *ev)
{
    if (L.data) return enqueue_data_form(ctx, prob, opt, res, L, ws, dctl, ev);
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n, p = prob->p;
    const int max_outer = opt->max_outer > 0 ? opt->max_outer : 1000;
    const int max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : 100000;
    const int max_rounds = opt->max_rounds > 0 ? opt->max_rounds : 64;
    double *scale = (double *)(ws + L.scale);
    const int original = opt->output_scale == SPMESL_SCALE_ORIGINAL;
    const Tune tu = resolve_tune(ctx->tune);

    if (ev) HIPTRY(ctx, hipEventRecord(ev[0], s));
    Marker marker(ctx);
    Marker *mk = ev ? &marker : nullptr;
    mark(mk, s, nullptr);
    launch_zero_words((uint32_t *)dctl, sizeof(Ctl) / 4, s);
    mark(mk, s, "zero_control");
    enqueue_standardize(L, prob, ws, dctl, s, mk);
    // The zero fill of the outputs goes on the second stream under the
    // covariance kernel, which leaves HBM to it (double: MFMA-bound, 290 us at
    // p = 5000; mixed: it slows that kernel from 86 to about 102 us), so that
    // the latency-bound column solves after it run without the fill's 400 MB
    // of writes beside them.  Measured at p = 5000, mixed: 0.262 ms per solve
    // against 0.269 with the fill after the row-tiled KKT pass (which left the
    // polish at 52-57 us instead of 36) and 0.311 with it under the column
    // solves at a low rate (the KKT pass doubled).  The launch shape
    // fill_split moves Omega's fill (1) or both (2) after the row-tiled KKT
    // pass instead.
    const int early = tu.fill_split == 0 ? 3 : (tu.fill_split == 1 ? 1 : 0);
    const int late = 3 & ~early;
    if (early) {
        const int v0 = fork_output_fill(ctx, res, p, s, mk, early);
        if (v0 != SPMESL_OK) return v0;
    }
    if (ev) HIPTRY(ctx, hipEventRecord(ev[1], s));

    const double tol_cols = column_tol(L, opt);
    const Screen sc = make_screen(L, ws, opt, tu, tol_cols);
    // the covariance kernel's span starts here, after the fork and phase events
    mark(mk, s, nullptr);
    if (L.prec == SPMESL_FP64)
        launch_syrk_f64((const double *)(ws + L.xs), n, p, (double *)(ws + L.S), sc, s);
    else if (L.prec == SPMESL_FP32)
        launch_syrk_f32((const float *)(ws + L.xs), n, p, (float *)(ws + L.S), sc, s);
    else
        launch_syrk_bf16x3((const uint16_t *)(ws + L.hi), (const uint16_t *)(ws + L.lo), n, L.npad,
                           p, (float *)(ws + L.S), sc, s);
    mark(mk, s, L.prec == SPMESL_FP64 ? "syrk_f64" : (L.prec == SPMESL_FP32 ? "syrk_f32" : "syrk_bf16x3"));
    if (ev) HIPTRY(ctx, hipEventRecord(ev[2], s));


    const bool fill = res->B || res->Omega;
    auto fork = [&] { return late ? fork_output_fill(ctx, res, p, s, mk, late) : (int)SPMESL_OK; };
    // a warm start: the columns' stored state from B0 and sigma0 (in the
    // scale of the outputs), which the first solves resume from
    const bool warm = prob->B0 || prob->sigma0;
    if (warm) {
        if (L.prec == SPMESL_FP64)
            launch_warm_start<double>(prob->B0, prob->sigma0, p, scale, original, opt->lambda0,
                                      (int *)(ws + L.wcnt), (int *)(ws + L.widx), (double *)(ws + L.wbeta),
                                      (double *)(ws + L.sigma), (double *)(ws + L.lam), (int *)(ws + L.cstat), s);
        else
            launch_warm_start<float>(prob->B0, prob->sigma0, p, scale, original, opt->lambda0,
                                     (int *)(ws + L.wcnt), (int *)(ws + L.widx), (float *)(ws + L.wbeta),
                                     (double *)(ws + L.sigma), (double *)(ws + L.lam), (int *)(ws + L.cstat), s);
        mark(mk, s, "warm_start");
    }
    int vc;
    if (L.prec == SPMESL_FP64)
        vc = enqueue_columns<double>(L, ws, dctl, opt, tu, tol_cols, 0.0, max_outer, max_sweeps, max_rounds, s,
                                     mk, fork, 0, warm);
    else
        vc = enqueue_columns<float>(L, ws, dctl, opt, tu, tol_cols, L.prec == SPMESL_MIXED ? kMixedBand : 0.0,
                                    max_outer, max_sweeps, max_rounds, s, mk, fork, 0, warm);
    if (vc != SPMESL_OK) return vc;
    if (ev) HIPTRY(ctx, hipEventRecord(ev[3], s));

    if (L.prec == SPMESL_MIXED) {
        const PolishArgs q = make_polish_args(L, ws, dctl, opt, max_outer, max_sweeps, max_rounds);
        launch_polish(q, s);
        mark(mk, s, "polish");
        enqueue_dense64(q, L, ws, dctl, opt, tu, s, mk);
    }
    {
        // the statistics reduction reads only the column results: it runs on
        // the second stream (behind the fill it may still hold) while the
        // scatter runs here, and the solve ends when both are done
        HIPTRY(ctx, hipEventRecord(ctx->fork2, s));
        HIPTRY(ctx, hipStreamWaitEvent(ctx->side, ctx->fork2, 0));
        mark(mk, ctx->side, nullptr);
        enqueue_reduce_stats(L, ws, dctl, ctx->side);
        mark(mk, ctx->side, "reduce_stats");
        HIPTRY(ctx, hipEventRecord(ctx->join2, ctx->side));
    }
    if (ev) HIPTRY(ctx, hipEventRecord(ev[4], s));

    if (fill) HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join, 0));
    mark(mk, s, "wait_fill");
    enqueue_scatter(L, ws, dctl, res, original, s);
    mark(mk, s, "scatter");
    HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join2, 0));
    if (ev) HIPTRY(ctx, hipEventRecord(ev[5], s));
    HIPTRY(ctx, hipGetLastError());
    return SPMESL_OK;
}

// The data form (SPMESL_FLAG_DATA_FORM): Algorithm 3 with E = X_K - X_V B
// instead of S.  Every column runs through the dense tier (dense.hip) with
// the standardised data as its source of S: groups of 16 columns, S[V, V]
// formed per group from the data (V = the union of the group's working sets),
// the blocked covariance-form sweeps on V, and the full gradient g = X^T E / n
// for the KKT check.  Memory is O(n p + groups |V|^2), never p^2.
static int enqueue_data_form(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                             const spmesl_result *res, const Plan &L, char *ws, Ctl *dctl, hipEvent_t *ev)
{
    hipStream_t s = ctx->stream;
    const int64_t n = prob->n, p = prob->p;
    const int max_outer = opt->max_outer > 0 ? opt->max_outer : 1000;
    const int max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : 100000;
    const int max_rounds = opt->max_rounds > 0 ? opt->max_rounds : 64;
    double *mean = (double *)(ws + L.mean);
    double *scale = (double *)(ws + L.scale);
    const int original = opt->output_scale == SPMESL_SCALE_ORIGINAL;
    const Tune tu = resolve_tune(ctx->tune);
    if (ev) HIPTRY(ctx, hipEventRecord(ev[0], s));
    Marker marker(ctx);
    Marker *mk = ev ? &marker : nullptr;
    mark(mk, s, nullptr);
    launch_zero_words((uint32_t *)dctl, sizeof(Ctl) / 4, s);
    mark(mk, s, "zero_control");
    if (!launch_stats_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt), (uint16_t *)(ws + L.hi),
                            (uint16_t *)(ws + L.lo), L.npad, &dctl->flags, (int *)(ws + L.pendcnt), s)) {
        launch_colstats(prob->X, n, p, prob->ldx, (double *)(ws + L.partial), L.rchunks, mean, scale,
                        &dctl->flags, (int *)(ws + L.pendcnt), s);
        launch_standardize_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                                 (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, s);
    }
    mark(mk, s, "standardize");
    const int v0 = fork_output_fill(ctx, res, p, s, mk);
    if (v0 != SPMESL_OK) return v0;
    if (ev) HIPTRY(ctx, hipEventRecord(ev[1], s));
    if (ev) HIPTRY(ctx, hipEventRecord(ev[2], s));
    const bool warm = prob->B0 || prob->sigma0;
    if (warm) {
        launch_warm_start<double>(prob->B0, prob->sigma0, p, scale, original, opt->lambda0, (int *)(ws + L.wcnt),
                                  (int *)(ws + L.widx), (double *)(ws + L.wbeta), (double *)(ws + L.sigma),
                                  (double *)(ws + L.lam), (int *)(ws + L.cstat), s);
        mark(mk, s, "warm_start");
    }
    DenseArgs<double> d{};
    d.S = nullptr;
    d.Xt = (const double *)(ws + L.xt);
    d.n = n;
    d.p = p;
    d.pv = p;
    d.lambda0 = opt->lambda0;
    d.tol = opt->tol;
    d.kkt_tol = opt->tol;
    d.max_outer = max_outer;
    d.max_sweeps = max_sweeps;
    d.max_rounds = max_rounds;
    d.block = tu.dense_block;
    d.queue = nullptr;
    d.qcnt = nullptr;
    d.ncols = p;
    d.w_cnt = (int *)(ws + L.wcnt);
    d.w_idx = (int *)(ws + L.widx);
    d.w_beta = (double *)(ws + L.wbeta);
    d.w_off = (int *)(ws + L.woff);
    d.sigma = (double *)(ws + L.sigma);
    d.lam_used = (double *)(ws + L.lam);
    d.col_status = (int *)(ws + L.cstat);
    d.pool_cnt = &dctl->pool;
    d.pool_cap = L.pool_cap;
    d.band_cnt = nullptr;
    d.info = (int *)(ws + L.colinfo);
    d.info_stride = 4;
    d.mark = (int *)(ws + L.dmark);
    d.V = (int *)(ws + L.dv);
    d.Vold = (int *)(ws + L.dvold);
    d.R = (double *)(ws + L.dr);
    d.Bd = (double *)(ws + L.dbd);
    d.Bp = (double *)(ws + L.dbp);
    d.sk = (double *)(ws + L.dsk);
    d.vcap = L.dvcap;
    d.Svv = (double *)(ws + L.dsvv);
    d.svv_cap = L.svv_cap;
    d.E = (double *)(ws + L.de);
    d.counters = dctl->counters;
    d.flags = &dctl->flags;
    DenseSrc<double> src{};
    if (warm) {
        src.cnt = d.w_cnt;
        src.idx = d.w_idx;
        src.beta = d.w_beta;
        src.off = d.w_off;
        src.sigma = d.sigma;
    }
    // the per-column counters start at zero (the tier adds to them)
    launch_zero_words((uint32_t *)(ws + L.colinfo), 4 * p, s);
    launch_dense<double, double>(d, src, s, L.dgroups);
    mark(mk, s, "dense_data_form");
    if (ev) HIPTRY(ctx, hipEventRecord(ev[3], s));
    HIPTRY(ctx, hipEventRecord(ctx->fork2, s));
    HIPTRY(ctx, hipStreamWaitEvent(ctx->side, ctx->fork2, 0));
    mark(mk, ctx->side, nullptr);
    launch_reduce_stats(p, (const int *)(ws + L.colinfo), nullptr, (const int *)(ws + L.wcnt),
                        (const int *)(ws + L.cstat), dctl->counters, &dctl->status1, ctx->side);
    mark(mk, ctx->side, "reduce_stats");
    HIPTRY(ctx, hipEventRecord(ctx->join2, ctx->side));
    if (ev) HIPTRY(ctx, hipEventRecord(ev[4], s));
    if (res->B || res->Omega) HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join, 0));
    mark(mk, s, "wait_fill");
    launch_scatter_outputs<double>(p, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                   (const double *)(ws + L.wbeta), (const int *)(ws + L.woff),
                                   (const double *)(ws + L.sigma), scale, original, res->B, res->sigma, res->Omega,
                                   &dctl->flags, s);
    mark(mk, s, "scatter");
    HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join2, 0));
    if (ev) HIPTRY(ctx, hipEventRecord(ev[5], s));
    HIPTRY(ctx, hipGetLastError());
    return SPMESL_OK;
}

// Enqueue `body` (which enqueues on ctx->stream) as one HIP graph launch on
// the caller's stream.  A call whose key matches the cached graph's replays
// it; otherwise `body` runs under capture on the context's own capturable
// stream (the caller's may be the null stream), and the instantiated graph
// replaces the cached one.  Kernel launches, event records and waits are the
// only stream work `body` does (no memset or copy nodes).
template <typename F>
static int run_graph(spmesl_ctx *ctx, std::vector<unsigned char> &&key, F &&body)
{
    hipStream_t user = ctx->stream;
    auto &gs = ctx->graphs;
    for (size_t i = 0; i < gs.size(); ++i) {
        if (gs[i].key != key) continue;
        std::rotate(gs.begin(), gs.begin() + (std::ptrdiff_t)i, gs.begin() + (std::ptrdiff_t)i + 1);
        HIPTRY(ctx, hipGraphLaunch(gs[0].exec, user));
        return SPMESL_OK;
    }
    if (!ctx->cap) HIPTRY(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    HIPTRY(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    ctx->stream = ctx->cap;
    const int v = body();
    ctx->stream = user;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap, &g);
    if (v != SPMESL_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (v != SPMESL_OK) return v;
        return fail(ctx, SPMESL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess)
        return fail(ctx, SPMESL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    if (gs.size() >= spmesl_ctx::kMaxGraphs) {
        // the least recently used graph may still be executing on the stream
        HIPTRY(ctx, hipStreamSynchronize(user));
        HIPTRY(ctx, hipGraphExecDestroy(gs.back().exec));
        gs.pop_back();
    }
    gs.insert(gs.begin(), spmesl_ctx::CachedGraph{std::move(key), ex});
    HIPTRY(ctx, hipGraphLaunch(ex, user));
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
        st->sum_working_set = (int64_t)c.counters[kCntSumW];
        st->resolved_columns = (int64_t)c.dirty;
        st->escalated_columns = (int64_t)c.counters[kCntEscalated];
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
// The grouped batch (mixed form).  Every step of the path runs once for all
// problems: the covariance tiles, the first solves, the row-tiled KKT pass,
// the re-solves, the escalations and the polish each take one launch whose
// work items span the problems (a table of per-problem arguments, and the
// offsets of each problem's items), so that small problems and the slow
// columns of each fill the chip together instead of one problem's tail at a
// time.  Each problem keeps its own workspace region and control block; a
// column's arithmetic is that of the single solve.
// ---------------------------------------------------------------------------
struct BatchTabs {
    // uploaded from the host: the tables and the host-known offsets
    size_t first, resume, wide, kkt, polish, syrk, col_off, tile_off, kkt_off, upload;
    // written on the device: offsets of the device-counted lists
    size_t dirty_off, esc_off, escp_off;
    size_t bytes;
};

static BatchTabs batch_tabs(int count)
{
    BatchTabs t{};
    Bump b;
    const size_t c = (size_t)count, offs = (c + 1) * sizeof(int64_t);
    const size_t col = std::max(sizeof(ColArgs<float>), sizeof(ColArgs<double>));
    const size_t kkt = std::max(sizeof(KktJob<float>), sizeof(KktJob<double>));
    const size_t syrk = std::max({sizeof(SyrkJob), sizeof(SyrkJobT<float>), sizeof(SyrkJobT<double>)});
    t.first = b.take(c * col);
    t.resume = b.take(c * col);
    t.wide = b.take(c * col);
    t.kkt = b.take(c * kkt);
    t.polish = b.take(c * sizeof(PolishArgs));
    t.syrk = b.take(c * syrk);
    t.col_off = b.take(offs);
    t.tile_off = b.take(offs);
    t.kkt_off = b.take(offs);
    t.upload = b.cur;
    t.dirty_off = b.take(offs);
    t.esc_off = b.take(offs);
    t.escp_off = b.take(offs);
    t.bytes = b.cur;
    return t;
}

// The grouped layout: problem i's workspace at ws_off[i], the control blocks
// at ctl_off, the tables at tab_off.
struct BatchLayout {
    std::vector<size_t> ws_off;
    size_t ctl_off = 0, tab_off = 0, total = 0;
    BatchTabs t{};
};

// Whether these problems run grouped: two or more, the covariance form, no
// warm starts, and a row of every S within the LDS of the row-tiled KKT pass.
static bool batch_grouped(int count, const spmesl_problem *probs, const spmesl_options *opt)
{
    if (count < 2 || (opt->flags & SPMESL_FLAG_DATA_FORM)) return false;
    const size_t elem = opt->precision == SPMESL_FP64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < count; ++i) {
        if (probs[i].B0 || probs[i].sigma0) return false;
        if (kkt_rows_per_block(probs[i].p, elem, (size_t)160 * 1024) <= 0) return false;
    }
    return true;
}

static BatchLayout batch_layout(int count, const std::vector<Plan> &plans)
{
    BatchLayout b;
    b.ws_off.resize((size_t)count);
    size_t o = 0;
    for (int i = 0; i < count; ++i) {
        b.ws_off[(size_t)i] = o;
        o += align_up(plans[(size_t)i].total, 256);
    }
    b.ctl_off = o;
    b.tab_off = align_up(o + (size_t)count * sizeof(Ctl), 256);
    b.t = batch_tabs(count);
    b.total = b.tab_off + b.t.bytes;
    return b;
}

static int ensure_stage(spmesl_ctx *ctx, size_t bytes)
{
    if (ctx->stage_bytes >= bytes) return SPMESL_OK;
    if (ctx->stage) {
        // a previous upload from it may still be in flight
        HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipHostFree(ctx->stage);
    }
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    HIPTRY(ctx, hipHostMalloc((void **)&ctx->stage, bytes, hipHostMallocDefault));
    ctx->stage_bytes = bytes;
    return SPMESL_OK;
}

// Fill the zero of the dense outputs of every problem on the second stream
// (`which` as in fork_output_fill).
static int fork_batch_fill(spmesl_ctx *ctx, int count, const spmesl_result *res, const std::vector<Plan> &plans,
                           hipStream_t s, int which)
{
    const int fb = resolve_tune(ctx->tune).fill_blocks;
    bool any = false;
    for (int i = 0; i < count; ++i) any = any || ((which & 1) && res[i].B) || ((which & 2) && res[i].Omega);
    if (!any) return SPMESL_OK;
    HIPTRY(ctx, hipEventRecord(ctx->fork, s));
    HIPTRY(ctx, hipStreamWaitEvent(ctx->side, ctx->fork, 0));
    for (int i = 0; i < count; ++i) {
        const int64_t p = plans[(size_t)i].p;
        if ((which & 1) && res[i].B) launch_fill_zero(res[i].B, p * p, ctx->side, fb);
        if ((which & 2) && res[i].Omega) launch_fill_zero(res[i].Omega, p * p, ctx->side, fb);
    }
    HIPTRY(ctx, hipEventRecord(ctx->join, ctx->side));
    return SPMESL_OK;
}

// Build the launch tables of a grouped batch into the host staging buffer.
// Returns the grid sizes the launches need.
struct BatchGrids {
    int64_t cols = 0, tiles = 0, kkt_blocks = 0, pmax = 0;
    int rj = 4;
    int syrk_edge = 64;  // covariance tile edge of the double and float forms
};

static void limits_of(const spmesl_options *opt, int *max_outer, int *max_sweeps, int *max_rounds)
{
    *max_outer = opt->max_outer > 0 ? opt->max_outer : 1000;
    *max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : 100000;
    *max_rounds = opt->max_rounds > 0 ? opt->max_rounds : 64;
}

// The first solves' arguments of problem i of a grouped batch.
template <typename T>
static ColArgs<T> batch_col_args(const Plan &L, char *ws, Ctl *c, const spmesl_options *opt)
{
    int mo, ms, mr;
    limits_of(opt, &mo, &ms, &mr);
    const double band = L.prec == SPMESL_MIXED ? kMixedBand : 0.0;
    ColArgs<T> a = make_col_args<T>(L, ws, c, opt, column_tol(L, opt), band, mo, ms, mr, 0, false);
    a.mode = 0;
    a.screened = 1;
    a.defer_kkt = 1;
    a.esc_cnt = &c->esc_c;
    a.esc_list = (int *)(ws + L.esclist2);
    return a;
}

template <typename T>
static BatchGrids build_batch_tables(spmesl_ctx *ctx, int count, const spmesl_options *opts,
                                     const std::vector<Plan> &plans, const BatchLayout &B, unsigned char *h)
{
    const Tune tu = resolve_tune(ctx->tune);
    const BatchTabs &t = B.t;
    char *ws0 = ctx->ws;
    Ctl *dctl = (Ctl *)(ws0 + B.ctl_off);
    BatchGrids gr;
    for (int i = 0; i < count; ++i) gr.rj = std::min(gr.rj, kkt_rows_for<T>(plans[(size_t)i].p, 0, tu));
    if (sizeof(T) == 8) {
        // 128 x 128 double tiles when the batch's tiles of that edge fill the
        // chip (the same rule as one problem's, on the batch's total)
        int64_t t128 = 0;
        for (int i = 0; i < count; ++i) {
            const int64_t e = (plans[(size_t)i].p + 127) / 128;
            t128 += e * (e + 1) / 2;
        }
        gr.syrk_edge = t128 >= 256 ? 128 : 64;
    }
    auto *first = (ColArgs<T> *)(h + t.first);
    auto *resume = (ColArgs<T> *)(h + t.resume);
    auto *wide = (ColArgs<T> *)(h + t.wide);
    auto *kkt = (KktJob<T> *)(h + t.kkt);
    auto *pol = (PolishArgs *)(h + t.polish);
    auto *col_off = (int64_t *)(h + t.col_off);
    auto *tile_off = (int64_t *)(h + t.tile_off);
    auto *kkt_off = (int64_t *)(h + t.kkt_off);
    col_off[0] = tile_off[0] = kkt_off[0] = 0;
    for (int i = 0; i < count; ++i) {
        const Plan &L = plans[(size_t)i];
        const spmesl_options *opt = &opts[i];
        char *ws = ws0 + B.ws_off[(size_t)i];
        Ctl *c = dctl + i;
        const Screen sc = make_screen(L, ws, opt, tu, column_tol(L, opt));
        int64_t tiles = 0, blocks = 0;
        if (L.prec == SPMESL_MIXED)
            ((SyrkJob *)(h + t.syrk))[i] =
                syrk_job_bf16x3((const uint16_t *)(ws + L.hi), (const uint16_t *)(ws + L.lo), L.n, L.npad, L.p,
                                (float *)(ws + L.S), sc, &tiles);
        else
            ((SyrkJobT<T> *)(h + t.syrk))[i] =
                syrk_job_mfma<T>((const T *)(ws + L.xs), L.n, L.p, (T *)(ws + L.S), sc, gr.syrk_edge, &tiles);
        ColArgs<T> a = batch_col_args<T>(L, ws, c, opt);
        first[i] = a;
        kkt[i] = kkt_job<T>(make_kkt_args<T>(a, L, ws, c), gr.rj, &blocks);
        a.mode = 1;
        a.screened = 0;
        a.work_list = (const int *)(ws + L.dirtylist);
        a.work_cnt = &c->dirty;
        resume[i] = a;
        a.work_list = (const int *)(ws + L.esclist2);
        a.work_cnt = &c->esc_c;
        wide[i] = a;
        if (L.prec == SPMESL_MIXED) {
            int mo, ms, mr;
            limits_of(opt, &mo, &ms, &mr);
            pol[i] = make_polish_args(L, ws, c, opt, mo, ms, mr);
        }
        col_off[i + 1] = col_off[i] + L.p;
        tile_off[i + 1] = tile_off[i] + tiles;
        kkt_off[i + 1] = kkt_off[i] + blocks;
        gr.pmax = std::max(gr.pmax, L.p);
    }
    gr.cols = col_off[count];
    gr.tiles = tile_off[count];
    gr.kkt_blocks = kkt_off[count];
    return gr;
}

template <typename T>
static int enqueue_batch_grouped(spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                                 const spmesl_options *opts, const spmesl_result *res, const std::vector<Plan> &plans,
                                 const BatchLayout &B, const BatchGrids &gr)
{
    hipStream_t s = ctx->stream;
    const Tune tu = resolve_tune(ctx->tune);
    const bool mixed = plans[0].prec == SPMESL_MIXED;
    char *ws0 = ctx->ws;
    Ctl *dctl = (Ctl *)(ws0 + B.ctl_off);
    const unsigned char *tb = (const unsigned char *)(ws0 + B.tab_off);
    const BatchTabs &t = B.t;
    const auto *col_off = (const int64_t *)(tb + t.col_off);
    auto *dirty_off = (int64_t *)(tb + t.dirty_off);
    auto *esc_off = (int64_t *)(tb + t.esc_off);
    auto *escp_off = (int64_t *)(tb + t.escp_off);
    const int64_t ctl_words = (int64_t)(sizeof(Ctl) / sizeof(int));
    auto wsi = [&](int i) { return ws0 + B.ws_off[(size_t)i]; };

    launch_zero_words((uint32_t *)dctl, (int64_t)count * (int64_t)(sizeof(Ctl) / 4), s);
    for (int i = 0; i < count; ++i) enqueue_standardize(plans[(size_t)i], &probs[i], wsi(i), dctl + i, s, nullptr);
    const int early = tu.fill_split == 0 ? 3 : (tu.fill_split == 1 ? 1 : 0);
    const int late = 3 & ~early;
    int v = early ? fork_batch_fill(ctx, count, res, plans, s, early) : (int)SPMESL_OK;
    if (v != SPMESL_OK) return v;
    if (mixed)
        launch_syrk_bf16x3_grouped((const SyrkJob *)(tb + t.syrk), (const int64_t *)(tb + t.tile_off), count,
                                   gr.tiles, s);
    else
        launch_syrk_mfma_grouped<T>((const SyrkJobT<T> *)(tb + t.syrk), (const int64_t *)(tb + t.tile_off), count,
                                    gr.tiles, gr.syrk_edge, s);
    launch_colsolve_first_grouped<T>((const ColArgs<T> *)(tb + t.first), col_off, count, gr.cols, s);
    launch_kkt_rows_grouped<T>((const KktJob<T> *)(tb + t.kkt), (const int64_t *)(tb + t.kkt_off), count,
                               gr.kkt_blocks, gr.rj, gr.pmax, s);
    if (late && (v = fork_batch_fill(ctx, count, res, plans, s, late)) != SPMESL_OK) return v;
    // re-solves of the flagged columns, then every escalated column (the
    // first solves' and the re-solves') in the wide tier
    launch_group_offsets(&dctl->dirty, ctl_words, count, dirty_off, s);
    launch_colsolve_list_grouped<T>((const ColArgs<T> *)(tb + t.resume), dirty_off, count, 0, s);
    launch_group_offsets(&dctl->esc_c, ctl_words, count, esc_off, s);
    launch_colsolve_list_grouped<T>((const ColArgs<T> *)(tb + t.wide), esc_off, count, 1, s);
    if (mixed) {
        // the double polish of every column, then its escalations, then the
        // double dense tier of each problem
        const PolishArgs *ptab = (const PolishArgs *)(tb + t.polish);
        launch_polish_grouped(ptab, col_off, count, gr.cols, 0, s);
        launch_group_offsets(&dctl->esc_polish, ctl_words, count, escp_off, s);
        launch_polish_grouped(ptab, escp_off, count, gr.cols, 1, s);
        for (int i = 0; i < count; ++i) {
            int mo, ms, mr;
            limits_of(&opts[i], &mo, &ms, &mr);
            const PolishArgs q = make_polish_args(plans[(size_t)i], wsi(i), dctl + i, &opts[i], mo, ms, mr);
            enqueue_dense64(q, plans[(size_t)i], wsi(i), dctl + i, &opts[i], tu, s, nullptr);
        }
    } else {
        // the dense tier of each problem
        for (int i = 0; i < count; ++i)
            enqueue_dense<T>(plans[(size_t)i], wsi(i), dctl + i,
                             batch_col_args<T>(plans[(size_t)i], wsi(i), dctl + i, &opts[i]), tu, s, nullptr);
    }
    HIPTRY(ctx, hipEventRecord(ctx->fork2, s));
    HIPTRY(ctx, hipStreamWaitEvent(ctx->side, ctx->fork2, 0));
    for (int i = 0; i < count; ++i) enqueue_reduce_stats(plans[(size_t)i], wsi(i), dctl + i, ctx->side);
    HIPTRY(ctx, hipEventRecord(ctx->join2, ctx->side));
    bool fill = false;
    for (int i = 0; i < count; ++i) fill = fill || res[i].B || res[i].Omega;
    if (fill) HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join, 0));
    for (int i = 0; i < count; ++i)
        enqueue_scatter(plans[(size_t)i], wsi(i), dctl + i, &res[i], opts[i].output_scale == SPMESL_SCALE_ORIGINAL,
                        s);
    HIPTRY(ctx, hipStreamWaitEvent(s, ctx->join2, 0));
    HIPTRY(ctx, hipGetLastError());
    return SPMESL_OK;
}

static int solve_batch_grouped(spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                               const std::vector<spmesl_options> &opts, spmesl_result *res, int *status,
                               const std::vector<Plan> &plans)
{
    const BatchLayout B = batch_layout(count, plans);
    int v = ensure_workspace(ctx, B.total);
    if (v != SPMESL_OK) return v;
    if ((v = ensure_pinned(ctx, (size_t)count)) != SPMESL_OK) return v;
    if ((v = ensure_stage(ctx, B.t.upload)) != SPMESL_OK) return v;
    ctx->nmarks = 0;
    // the tables hold workspace addresses: built for this workspace, and
    // uploaded ahead of the solves (outside any graph)
    const bool dbl = plans[0].prec == SPMESL_FP64;
    const BatchGrids gr = dbl ? build_batch_tables<double>(ctx, count, opts.data(), plans, B, ctx->stage)
                              : build_batch_tables<float>(ctx, count, opts.data(), plans, B, ctx->stage);
    HIPTRY(ctx, hipMemcpyAsync(ctx->ws + B.tab_off, ctx->stage, B.t.upload, hipMemcpyHostToDevice, ctx->stream));
    const spmesl_options *opt = &opts[0];
    auto body = [&] {
        return dbl ? enqueue_batch_grouped<double>(ctx, count, probs, opts.data(), res, plans, B, gr)
                   : enqueue_batch_grouped<float>(ctx, count, probs, opts.data(), res, plans, B, gr);
    };
    if (opt->flags & SPMESL_FLAG_EAGER) {
        v = body();
    } else {
        KeyBuf k;
        k.add('G');
        k.add(ctx->ws);
        k.add(count);
        key_tuning(k, ctx->tune);
        for (int i = 0; i < count; ++i) {
            key_problem(k, probs[i], res[i]);
            key_options(k, opts[(size_t)i]);
        }
        v = run_graph(ctx, std::move(k.b), body);
    }
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + B.ctl_off);
    HIPTRY(ctx, hipMemcpyAsync(ctx->pinned, dctl, (size_t)count * sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    int first = SPMESL_OK;
    for (int i = 0; i < count; ++i) {
        status[i] = decode(ctx->pinned[i], probs[i].p, res[i].stats);
        if (first == SPMESL_OK && status[i] != SPMESL_OK) first = status[i];
    }
    return first;
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
    ok = ok && hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ctx->fork2, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ctx->join2, hipEventDisableTiming) == hipSuccess;
    bool kok = ok;
    for (int i = 0; i < spmesl_ctx::kMaxMarks && kok; ++i) kok = hipEventCreate(&ctx->kev[i]) == hipSuccess;
    ctx->kev_ok = kok;
    // the no-allocation entry point's scratch address, with this device current
    ctx->scratch_dev = scratch_address(device, &ctx->scratch_err);
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
        if (ctx->side) {
            (void)hipStreamSynchronize(ctx->side);
            (void)hipStreamDestroy(ctx->side);
        }
        for (auto &cg : ctx->graphs) (void)hipGraphExecDestroy(cg.exec);
        if (ctx->cap) {
            (void)hipStreamSynchronize(ctx->cap);
            (void)hipStreamDestroy(ctx->cap);
        }
        for (int i = 0; i < spmesl_ctx::kMaxMarks; ++i)
            if (ctx->kev[i]) (void)hipEventDestroy(ctx->kev[i]);
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
        if (ctx->join) (void)hipEventDestroy(ctx->join);
        if (ctx->fork2) (void)hipEventDestroy(ctx->fork2);
        if (ctx->join2) (void)hipEventDestroy(ctx->join2);
        if (ctx->ws && ctx->ws_owned) (void)hipFree(ctx->ws);
        if (ctx->tune_status) (void)hipFree(ctx->tune_status);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        if (ctx->stage) (void)hipHostFree(ctx->stage);
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
    // the plan, then the control block spmesl_solve places after it
    *bytes = align_up(make_plan(prob->n, prob->p, opt->precision, opt->flags & SPMESL_FLAG_DATA_FORM).total, 256) +
             sizeof(Ctl);
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
    Plan L = make_plan(prob->n, prob->p, opt->precision, opt->flags & SPMESL_FLAG_DATA_FORM);
    size_t ctl_off = align_up(L.total, 256);
    v = ensure_workspace(ctx, ctl_off + sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    v = ensure_pinned(ctx, 1);
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + ctl_off);
    const bool timing = (opt->flags & SPMESL_FLAG_TIMING) && ctx->have_events && ctx->kev_ok;
    if (timing || (opt->flags & SPMESL_FLAG_EAGER)) {
        v = enqueue_solve(ctx, prob, opt, res, L, ctx->ws, dctl, timing ? ctx->ev : nullptr);
    } else {
        KeyBuf k;
        k.add('s');
        k.add(ctx->ws);
        key_problem(k, *prob, *res);
        key_options(k, *opt);
        key_tuning(k, ctx->tune);
        v = run_graph(ctx, std::move(k.b),
                      [&] { return enqueue_solve(ctx, prob, opt, res, L, ctx->ws, dctl, nullptr); });
    }
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
    if (timing) {
        for (int i = 0; i < ctx->nmarks; ++i) {
            ctx->kms[i] = 0.f;
            if (ctx->kname[i] && ctx->kprev[i] >= 0)
                HIPTRY(ctx, hipEventElapsedTime(&ctx->kms[i], ctx->kev[ctx->kprev[i]], ctx->kev[i]));
        }
    } else {
        ctx->nmarks = 0;
    }
    if (st == SPMESL_ENONFINITE) ctx->err = "X holds a NaN or Inf";
    else if (st == SPMESL_EZEROVAR) ctx->err = "a column of X has zero variance";
    else if (st == SPMESL_EWORKSET) ctx->err = "the dense tier ran out of room for the long working sets";
    else if (st == SPMESL_EDEGENERATE) ctx->err = "a residual variance fell to zero";
    else if (st == SPMESL_ENOCONV) ctx->err = "an iteration cap was reached";
    return st;
}

int spmesl_solve_async(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                       spmesl_result *res, int *status_dev)
{
    if (!ctx || !res || !status_dev) return SPMESL_EINVAL;
    int v = validate(ctx, prob, opt);
    if (v != SPMESL_OK) return v;
    DevGuard g(ctx->device);
    Plan L = make_plan(prob->n, prob->p, opt->precision, opt->flags & SPMESL_FLAG_DATA_FORM);
    size_t ctl_off = align_up(L.total, 256);
    v = ensure_workspace(ctx, ctl_off + sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + ctl_off);
    ctx->nmarks = 0;
    auto body = [&] {
        int vi = enqueue_solve(ctx, prob, opt, res, L, ctx->ws, dctl, nullptr);
        if (vi != SPMESL_OK) return vi;
        hipLaunchKernelGGL(k_decode_status, dim3(1), dim3(1), 0, ctx->stream, dctl, status_dev);
        HIPTRY(ctx, hipGetLastError());
        return (int)SPMESL_OK;
    };
    if (opt->flags & SPMESL_FLAG_EAGER) return body();
    KeyBuf k;
    k.add('a');
    k.add(ctx->ws);
    k.add(status_dev);
    key_problem(k, *prob, *res);
    key_options(k, *opt);
    key_tuning(k, ctx->tune);
    return run_graph(ctx, std::move(k.b), body);
}

int spmesl_solve_noalloc(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                         spmesl_result *res, int *status_dev)
{
    if (!ctx || !res || !status_dev) return SPMESL_EINVAL;
    int v = validate(ctx, prob, opt);
    if (v != SPMESL_OK) return v;
    if (!ctx->scratch_dev)
        return fail(ctx, SPMESL_EHIP,
                    std::string("no device address for the scratch array: ") + hipGetErrorString(ctx->scratch_err));
    const Plan L = make_plan(prob->n, prob->p, opt->precision, opt->flags & SPMESL_FLAG_DATA_FORM);
    const size_t ctl_off = align_up(L.total, 256);
    if (ctl_off + sizeof(Ctl) > (size_t)SPMESL_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, SPMESL_ENOMEM,
                    "this solve needs " + std::to_string(ctl_off + sizeof(Ctl)) +
                        " bytes of scratch; spmesl_solve_noalloc holds " +
                        std::to_string((size_t)SPMESL_NOALLOC_SCRATCH_BYTES));
    DevGuard g(ctx->device);
    char *base = ctx->scratch_dev;
    Ctl *dctl = (Ctl *)(base + ctl_off);
    ctx->nmarks = 0;
    // kernel by kernel (a graph instantiation may allocate); the control
    // block is zeroed by the solve's first kernel
    v = enqueue_solve(ctx, prob, opt, res, L, base, dctl, nullptr);
    if (v != SPMESL_OK) return v;
    hipLaunchKernelGGL(k_decode_status, dim3(1), dim3(1), 0, ctx->stream, dctl, status_dev);
    HIPTRY(ctx, hipGetLastError());
    return SPMESL_OK;
}

int spmesl_set_tuning(spmesl_ctx *ctx, const spmesl_tuning *t)
{
    if (!ctx) return SPMESL_EINVAL;
    if (!t) {
        ctx->tune = spmesl_tuning{};
        return SPMESL_OK;
    }
    if (t->dense_block < 0 || (t->dense_block > 0 && t->dense_block != 16 && t->dense_block != 32 &&
                               t->dense_block != 64))
        return fail(ctx, SPMESL_EINVAL, "dense_block must be 0, 16, 32 or 64");
    if (t->fill_blocks < 0 || t->fill_blocks > 4096)
        return fail(ctx, SPMESL_EINVAL, "fill_blocks must be in 0 .. 4096");
    if (t->kkt_rows < 0 || t->kkt_rows > 4) return fail(ctx, SPMESL_EINVAL, "kkt_rows must be in 0 .. 4");
    if (t->screen_permille < 0 || t->screen_permille > 4000)
        return fail(ctx, SPMESL_EINVAL, "screen_permille must be in 0 .. 4000");
    if (t->fill_split < 0 || t->fill_split > 2) return fail(ctx, SPMESL_EINVAL, "fill_split must be 0, 1 or 2");
    ctx->tune = *t;
    return SPMESL_OK;
}

int spmesl_get_tuning(const spmesl_ctx *ctx, spmesl_tuning *t)
{
    if (!ctx || !t) return SPMESL_EINVAL;
    *t = ctx->tune;
    return SPMESL_OK;
}

// Milliseconds per solve: the fastest of three runs of `reps` asynchronous
// solves back to back (graph replays; the first call captures the graph, is
// checked and is not timed).  The minimum over runs keeps other work on the
// device out of the comparison.
static int time_solves(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                       spmesl_result *res, int reps, double *ms)
{
    spmesl_options o = *opt;
    o.flags &= ~(SPMESL_FLAG_TIMING | SPMESL_FLAG_EAGER);
    int v = spmesl_solve(ctx, prob, &o, res);  // captures the graph, checks the status
    if (v != SPMESL_OK) return v;
    DevGuard g(ctx->device);
    double best = 0.0;
    for (int run = 0; run < 3; ++run) {
        HIPTRY(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
        for (int r = 0; r < reps; ++r) {
            v = spmesl_solve_async(ctx, prob, &o, res, ctx->tune_status);
            if (v != SPMESL_OK) return v;
        }
        HIPTRY(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
        HIPTRY(ctx, hipEventSynchronize(ctx->ev[1]));
        float t = 0.f;
        HIPTRY(ctx, hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
        const double m = (double)t / reps;
        best = run == 0 || m < best ? m : best;
    }
    *ms = best;
    return SPMESL_OK;
}

int spmesl_autotune(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                    spmesl_result *res, int reps, spmesl_tuning *best, double *ms_best)
{
    if (!ctx || !res || reps < 1) return SPMESL_EINVAL;
    int v = validate(ctx, prob, opt);
    if (v != SPMESL_OK) return v;
    if (!ctx->have_events) return fail(ctx, SPMESL_EHIP, "the context has no timing events");
    {
        DevGuard g(ctx->device);
        if (!ctx->tune_status) HIPTRY(ctx, hipMalloc((void **)&ctx->tune_status, sizeof(int)));
    }
    // explicit values for every field, starting from the current shapes
    const Tune d = resolve_tune(ctx->tune);
    spmesl_tuning cur{};
    cur.dense_block = d.dense_block;
    cur.fill_blocks = d.fill_blocks;
    cur.screen_permille = d.screen_permille;
    cur.fill_split = d.fill_split;
    const size_t tsz = opt->precision == SPMESL_FP64 ? 8 : 4;
    const int rj_max = kkt_rows_per_block(prob->p, tsz, (size_t)160 * 1024);
    cur.kkt_rows = d.kkt_rows > 0 && d.kkt_rows < rj_max ? d.kkt_rows : rj_max;
    ctx->tune = cur;
    double tbest = 0.0;
    v = time_solves(ctx, prob, opt, res, reps, &tbest);
    if (v != SPMESL_OK) return v;
    // does the problem reach the dense tier?  (its block size matters only then)
    spmesl_stats st{};
    spmesl_result rs = *res;
    rs.stats = &st;
    v = spmesl_solve(ctx, prob, opt, &rs);
    if (v != SPMESL_OK) return v;
    const bool dense = st.max_working_set > SPMESL_MAX_WORKING_SET || ctx->pinned[0].dense + ctx->pinned[0].dense64 > 0;
    auto search = [&](int32_t spmesl_tuning::*field, std::vector<int> cands) -> int {
        for (int c : cands) {
            if (c == cur.*field) continue;
            spmesl_tuning t = cur;
            t.*field = c;
            ctx->tune = t;
            double ms = 0.0;
            const int r = time_solves(ctx, prob, opt, res, reps, &ms);
            if (r != SPMESL_OK) return r;
            // a candidate replaces the current shapes only when clearly faster
            if (ms < 0.99 * tbest) {
                tbest = ms;
                cur = t;
            }
        }
        ctx->tune = cur;
        return SPMESL_OK;
    };
    if ((v = search(&spmesl_tuning::screen_permille, {700, 800, 900, 1000})) != SPMESL_OK) return v;
    if (rj_max > 0) {
        std::vector<int> kr;
        for (int r = rj_max; r >= 1; r >>= 1) kr.push_back(r);
        if ((v = search(&spmesl_tuning::kkt_rows, kr)) != SPMESL_OK) return v;
    }
    if ((v = search(&spmesl_tuning::fill_blocks, {32, 64, 128, 256})) != SPMESL_OK) return v;
    if ((v = search(&spmesl_tuning::fill_split, {0, 1, 2})) != SPMESL_OK) return v;
    if (dense && (v = search(&spmesl_tuning::dense_block, {16, 32, 64})) != SPMESL_OK) return v;
    ctx->tune = cur;
    // the outputs hold a solve with the chosen shapes
    v = spmesl_solve(ctx, prob, opt, res);
    if (v != SPMESL_OK) return v;
    if (best) *best = cur;
    if (ms_best) *ms_best = tbest;
    return SPMESL_OK;
}

int spmesl_batch_workspace_size(const spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                                const spmesl_options *opt, size_t *bytes)
{
    if (!ctx || !opt || !bytes || count < 0 || (count > 0 && !probs)) return SPMESL_EINVAL;
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        spmesl_options o = *opt;
        o.lambda0 = 1.0;  // the plan does not depend on it
        const int v = validate(nullptr, &probs[i], &o);
        if (v != SPMESL_OK) return v;
        need = std::max(need, make_plan(probs[i].n, probs[i].p, opt->precision,
                                        opt->flags & SPMESL_FLAG_DATA_FORM).total);
    }
    if (batch_grouped(count, probs, opt)) {
        std::vector<Plan> plans((size_t)count);
        for (int i = 0; i < count; ++i) plans[(size_t)i] = make_plan(probs[i].n, probs[i].p, opt->precision);
        *bytes = batch_layout(count, plans).total;
        return SPMESL_OK;
    }
    *bytes = align_up(need, 256) + (size_t)std::max(count, 1) * sizeof(Ctl);
    return SPMESL_OK;
}

int spmesl_solve_batch(spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                       const spmesl_options *opt, const double *lambda0s, spmesl_result *res,
                       int *status)
{
    if (!ctx || !opt || count < 0 || (count > 0 && (!probs || !res || !status))) return SPMESL_EINVAL;
    if (count == 0) return SPMESL_OK;
    DevGuard g(ctx->device);
    size_t need = 0;
    std::vector<Plan> plans((size_t)count);
    std::vector<spmesl_options> opts((size_t)count, *opt);
    for (int i = 0; i < count; ++i) {
        if (lambda0s) opts[(size_t)i].lambda0 = lambda0s[i];
        int v = validate(ctx, &probs[i], &opts[(size_t)i]);
        if (v != SPMESL_OK) {
            ctx->err = "problem " + std::to_string(i) + ": " + ctx->err;
            return v;
        }
        plans[(size_t)i] = make_plan(probs[i].n, probs[i].p, opt->precision, opt->flags & SPMESL_FLAG_DATA_FORM);
        need = std::max(need, plans[(size_t)i].total);
    }
    if (batch_grouped(count, probs, opt)) return solve_batch_grouped(ctx, count, probs, opts, res, status, plans);
    size_t ctl_off = align_up(need, 256);
    int v = ensure_workspace(ctx, ctl_off + (size_t)count * sizeof(Ctl));
    if (v != SPMESL_OK) return v;
    v = ensure_pinned(ctx, (size_t)count);
    if (v != SPMESL_OK) return v;
    Ctl *dctl = (Ctl *)(ctx->ws + ctl_off);
    ctx->nmarks = 0;
    auto body = [&] {
        for (int i = 0; i < count; ++i) {
            int vi = enqueue_solve(ctx, &probs[i], &opts[(size_t)i], &res[i], plans[(size_t)i], ctx->ws,
                                   dctl + i, nullptr);
            if (vi != SPMESL_OK) return vi;
        }
        return (int)SPMESL_OK;
    };
    if (opt->flags & SPMESL_FLAG_EAGER) {
        v = body();
    } else {
        KeyBuf k;
        k.add('b');
        k.add(ctx->ws);
        k.add(count);
        for (int i = 0; i < count; ++i) {
            key_problem(k, probs[i], res[i]);
            key_options(k, opts[(size_t)i]);
            key_tuning(k, ctx->tune);
        }
        v = run_graph(ctx, std::move(k.b), body);
    }
    if (v != SPMESL_OK) return v;
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

int spmesl_kernel_times(const spmesl_ctx *ctx, int cap, const char **names, double *ms)
{
    if (!ctx || cap < 0 || (cap > 0 && (!names || !ms))) return SPMESL_EINVAL;
    int n = 0;
    for (int i = 0; i < ctx->nmarks; ++i) {
        if (!ctx->kname[i]) continue;
        if (n < cap) {
            names[n] = ctx->kname[i];
            ms[n] = (double)ctx->kms[i];
        }
        ++n;
    }
    return n;
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
                    &dctl->flags, nullptr, s);
    if (precision == SPMESL_FP64) {
        launch_standardize_f64(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xs), s);
        launch_syrk_f64((const double *)(ws + L.xs), n, p, (double *)S_out, Screen{}, s);
    } else if (precision == SPMESL_FP32) {
        launch_standardize_f32(prob->X, n, p, prob->ldx, mean, scale, (float *)(ws + L.xs), s);
        launch_syrk_f32((const float *)(ws + L.xs), n, p, (float *)S_out, Screen{}, s);
    } else {
        launch_standardize_split(prob->X, n, p, prob->ldx, mean, scale, (double *)(ws + L.xt),
                                 (uint16_t *)(ws + L.hi), (uint16_t *)(ws + L.lo), L.npad, s);
        launch_syrk_bf16x3((const uint16_t *)(ws + L.hi), (const uint16_t *)(ws + L.lo), n, L.npad, p,
                           (float *)S_out, Screen{}, s);
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

// workspace of spmesl_scaled_lasso: the plan of p + m double variables, the
// packed data [X | Y], and the control block
static size_t lasso_layout(int64_t n, int64_t pa, Plan *L, size_t *xa_off, size_t *ctl_off)
{
    *L = make_plan(n, pa, SPMESL_FP64);
    *xa_off = align_up(L->total, 256);
    *ctl_off = align_up(*xa_off + 8 * (size_t)n * (size_t)pa, 256);
    return *ctl_off + sizeof(Ctl);
}

int spmesl_scaled_lasso_workspace_size(int64_t n, int64_t p, int64_t m, size_t *bytes)
{
    if (!bytes || n < 2 || p < 1 || m < 1 || p > ((int64_t)1 << 30) - m) return SPMESL_EINVAL;
    Plan L;
    size_t xa, ctl;
    *bytes = lasso_layout(n, p + m, &L, &xa, &ctl);
    return SPMESL_OK;
}

int spmesl_scaled_lasso(spmesl_ctx *ctx, const spmesl_problem *prob, const double *Y, int64_t m,
                        int64_t ldy, const spmesl_options *opt, double *beta, double *sigma, int *outer,
                        spmesl_stats *stats)
{
    if (!ctx) return SPMESL_EINVAL;
    if (!prob || !opt) return fail(ctx, SPMESL_EINVAL, "null problem or options");
    if (!prob->X || !Y) return fail(ctx, SPMESL_EINVAL, "X or Y is null");
    if (!beta || !sigma) return fail(ctx, SPMESL_EINVAL, "beta or sigma is null");
    if (prob->p < 1) return fail(ctx, SPMESL_EINVAL, "p must be >= 1");
    if (m < 1) return fail(ctx, SPMESL_EINVAL, "m must be >= 1");
    if (prob->ldx < prob->p) return fail(ctx, SPMESL_EINVAL, "ldx must be >= p");
    if (ldy < m) return fail(ctx, SPMESL_EINVAL, "ldy must be >= m");
    if (prob->p > ((int64_t)1 << 30) - m) return fail(ctx, SPMESL_EINVAL, "p + m too large");
    if (opt->precision != SPMESL_FP64)
        return fail(ctx, SPMESL_EINVAL, "the scaled lasso entry runs in SPMESL_FP64 only");
    if (prob->B0 || prob->sigma0)
        return fail(ctx, SPMESL_EINVAL, "the scaled lasso entry takes no warm start");
    // the design and the responses as one problem of p + m variables
    spmesl_problem aug = *prob;
    aug.p = prob->p + m;
    aug.ldx = aug.p;
    int v = validate(ctx, &aug, opt);
    if (v != SPMESL_OK) return v;
    DevGuard g(ctx->device);
    const int64_t n = prob->n, px = prob->p, pa = aug.p;
    Plan L;
    size_t xa_off, ctl_off;
    v = ensure_workspace(ctx, lasso_layout(n, pa, &L, &xa_off, &ctl_off));
    if (v != SPMESL_OK) return v;
    v = ensure_pinned(ctx, 1);
    if (v != SPMESL_OK) return v;
    char *ws = ctx->ws;
    Ctl *dctl = (Ctl *)(ws + ctl_off);
    double *Xa = (double *)(ws + xa_off);
    double *mean = (double *)(ws + L.mean);
    double *scale = (double *)(ws + L.scale);
    hipStream_t s = ctx->stream;
    const int max_outer = opt->max_outer > 0 ? opt->max_outer : 1000;
    const int max_sweeps = opt->max_sweeps > 0 ? opt->max_sweeps : 100000;
    const int max_rounds = opt->max_rounds > 0 ? opt->max_rounds : 64;
    ctx->nmarks = 0;

    launch_zero_words((uint32_t *)dctl, sizeof(Ctl) / 4, s);
    launch_pack_columns(prob->X, n, px, prob->ldx, Y, m, ldy, Xa, s);
    launch_colstats(Xa, n, pa, pa, (double *)(ws + L.partial), L.rchunks, mean, scale, &dctl->flags,
                    (int *)(ws + L.pendcnt), s);
    launch_standardize_f64(Xa, n, pa, pa, mean, scale, (double *)(ws + L.xs), s);
    // the first working sets from the screen taken with S, as in spmesl_solve,
    // with the design columns j < p as the only candidates
    Screen sc;
    const Tune tu = resolve_tune(ctx->tune);
    sc.thr64 = tu.screen_permille * 1e-3 * opt->lambda0 + opt->tol;
    sc.thr32 = 0.0f;
    sc.cnt = (int *)(ws + L.pendcnt);
    sc.idx = (int *)(ws + L.pendidx);
    sc.pv = px;
    launch_syrk_f64((const double *)(ws + L.xs), n, pa, (double *)(ws + L.S), sc, s);
    v = enqueue_columns<double>(L, ws, dctl, opt, tu, opt->tol, 0.0, max_outer, max_sweeps, max_rounds, s,
                                nullptr, [] { return (int)SPMESL_OK; }, px);
    if (v != SPMESL_OK) return v;
    launch_reduce_stats(m, (const int *)(ws + L.colinfo) + 4 * px, nullptr, (const int *)(ws + L.wcnt) + px,
                        (const int *)(ws + L.cstat) + px, dctl->counters, &dctl->status1, s);
    launch_fill_zero(beta, px * m, s);
    launch_scatter_lasso<double>(px, m, (const int *)(ws + L.wcnt), (const int *)(ws + L.widx),
                                 (const double *)(ws + L.wbeta), (const int *)(ws + L.woff),
                                 (const double *)(ws + L.sigma), scale,
                                 opt->output_scale == SPMESL_SCALE_ORIGINAL, (const int *)(ws + L.colinfo),
                                 beta, sigma, outer, &dctl->flags, s);
    HIPTRY(ctx, hipGetLastError());
    HIPTRY(ctx, hipMemcpyAsync(ctx->pinned, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPTRY(ctx, hipStreamSynchronize(s));
    const int st = decode(ctx->pinned[0], m, stats);
    if (stats) stats->nnz_B = -1;
    if (st == SPMESL_ENONFINITE) ctx->err = "X or Y holds a NaN or Inf";
    else if (st == SPMESL_EZEROVAR) ctx->err = "a column of X or Y has zero variance";
    else if (st == SPMESL_EWORKSET) ctx->err = "the dense tier ran out of room for the long working sets";
    else if (st == SPMESL_EDEGENERATE) ctx->err = "a residual variance fell to zero";
    else if (st == SPMESL_ENOCONV) ctx->err = "an iteration cap was reached";
    return st;
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
