// Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of the
// library's host orchestration, on a real GPU (tests/host_asan/build.sh) or
// against the CPU stand-in of the HIP runtime (tests/host_mock/build.sh,
// where kernels do not run and every device status reads as zero): every
// entry point's host path
// (plans, workspace growth, graph capture, cache and replay, the second
// stream's fork and join events, the timing markers, the batch, the
// asynchronous and no-allocation entry points, warm starts, error paths).
// The device code is the ordinary build; only host code is instrumented.
// Prints one line per step and exits non-zero on an unexpected status.
#include <hip/hip_runtime.h>

#pragma clang diagnostic ignored "-Wunused-result"
#pragma clang diagnostic ignored "-Wunused-value"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "spmesl.h"

static int fails = 0;

// defined by the CPU stand-in of the HIP runtime (tests/host_mock), absent
// from the real one
extern "C" int mock_violations() __attribute__((weak));
extern "C" long mock_launches() __attribute__((weak));
extern "C" long mock_graph_launches() __attribute__((weak));
extern "C" long mock_captures() __attribute__((weak));

#define CHECK(name, got, want)                                                                        \
    do {                                                                                              \
        int g_ = (got);                                                                               \
        std::printf("%-44s status %d (want %d)%s\n", name, g_, (int)(want), g_ == (want) ? "" : "  <-- FAIL"); \
        std::fflush(stdout);                                                                          \
        if (g_ != (want)) ++fails;                                                                    \
    } while (0)

// n x p rows of an AR(0.5) process along the columns (seeded LCG, Box-Muller)
static std::vector<double> make_x(int n, int p, unsigned long long seed)
{
    std::vector<double> x((size_t)n * p);
    unsigned long long s = seed * 6364136223846793005ull + 1442695040888963407ull;
    auto unif = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return ((s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (int i = 0; i < n; ++i) {
        double prev = 0.0;
        for (int j = 0; j < p; ++j) {
            double z = std::sqrt(-2.0 * std::log(unif())) * std::cos(6.283185307179586 * unif());
            prev = j == 0 ? z : 0.5 * prev + std::sqrt(0.75) * z;
            x[(size_t)i * p + j] = prev;
        }
    }
    return x;
}

struct Dev {
    double *X = nullptr, *B = nullptr, *sig = nullptr, *Om = nullptr;
    int n = 0, p = 0;
    Dev(int n_, int p_, unsigned long long seed) : n(n_), p(p_)
    {
        std::vector<double> h = make_x(n, p, seed);
        hipMalloc(&X, h.size() * 8);
        hipMemcpy(X, h.data(), h.size() * 8, hipMemcpyHostToDevice);
        hipMalloc(&B, (size_t)p * p * 8);
        hipMalloc(&sig, (size_t)p * 8);
        hipMalloc(&Om, (size_t)p * p * 8);
    }
    ~Dev()
    {
        hipFree(X);
        hipFree(B);
        hipFree(sig);
        hipFree(Om);
    }
    spmesl_problem prob() const
    {
        spmesl_problem q{};
        q.X = X;
        q.n = n;
        q.p = p;
        q.ldx = p;
        return q;
    }
    spmesl_result res(spmesl_stats *st) const
    {
        spmesl_result r{};
        r.B = B;
        r.sigma = sig;
        r.Omega = Om;
        r.stats = st;
        return r;
    }
};

int main()
{
    spmesl_ctx *ctx = nullptr;
    CHECK("create", spmesl_create(&ctx, 0, nullptr), SPMESL_OK);
    if (!ctx) return 1;
    Dev a(200, 300, 1), b(120, 90, 2);
    int *status_dev = nullptr;
    hipMalloc(&status_dev, sizeof(int));
    spmesl_stats st{};
    for (int prec : {SPMESL_FP64, SPMESL_FP32, SPMESL_MIXED}) {
        spmesl_options o{};
        o.lambda0 = 0.25;
        o.tol = 1e-8;
        o.precision = prec;
        spmesl_problem pa = a.prob(), pb = b.prob();
        spmesl_result ra = a.res(&st), rb = b.res(&st);
        char name[64];
        std::snprintf(name, sizeof name, "solve eager (prec %d)", prec);
        o.flags = SPMESL_FLAG_EAGER;
        CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        o.flags = 0;
        for (int r = 0; r < 3; ++r) {
            std::snprintf(name, sizeof name, "solve graph %d (prec %d)", r, prec);
            CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
            std::snprintf(name, sizeof name, "solve other graph %d (prec %d)", r, prec);
            CHECK(name, spmesl_solve(ctx, &pb, &o, &rb), SPMESL_OK);
        }
        o.flags = SPMESL_FLAG_TIMING;
        std::snprintf(name, sizeof name, "solve timed (prec %d)", prec);
        CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        const char *names[64];
        double ms[64];
        int nk = spmesl_kernel_times(ctx, 64, names, ms);
        std::snprintf(name, sizeof name, "kernel times (prec %d) >= 8 steps", prec);
        CHECK(name, nk >= 8 ? 0 : -1, 0);
        o.flags = 0;
        for (int r = 0; r < 2; ++r) {
            std::snprintf(name, sizeof name, "solve async %d (prec %d)", r, prec);
            CHECK(name, spmesl_solve_async(ctx, &pa, &o, &ra, status_dev), SPMESL_OK);
        }
        hipDeviceSynchronize();
        std::snprintf(name, sizeof name, "solve noalloc (prec %d)", prec);
        CHECK(name, spmesl_solve_noalloc(ctx, &pa, &o, &ra, status_dev), SPMESL_OK);
        hipDeviceSynchronize();
        // warm start from the last outputs
        spmesl_problem pw = pa;
        pw.B0 = a.B;
        pw.sigma0 = a.sig;
        std::snprintf(name, sizeof name, "solve warm (prec %d)", prec);
        CHECK(name, spmesl_solve(ctx, &pw, &o, &ra), SPMESL_OK);
        // a batch of uneven problems, eager and as a graph (twice)
        std::vector<Dev *> ds;
        for (int i = 0; i < 5; ++i) ds.push_back(new Dev(60 + 37 * i, 50 + 61 * i, 10 + i));
        std::vector<spmesl_problem> ps;
        std::vector<spmesl_result> rs;
        std::vector<spmesl_stats> sts(ds.size());
        std::vector<double> lams;
        for (size_t i = 0; i < ds.size(); ++i) {
            ps.push_back(ds[i]->prob());
            rs.push_back(ds[i]->res(&sts[i]));
            lams.push_back(0.2 + 0.02 * (double)i);
        }
        std::vector<int> stat(ds.size(), 99);
        for (int r = 0; r < 3; ++r) {
            o.flags = r == 0 ? SPMESL_FLAG_EAGER : 0;
            std::snprintf(name, sizeof name, "batch %d (prec %d)", r, prec);
            CHECK(name, spmesl_solve_batch(ctx, (int)ds.size(), ps.data(), &o, lams.data(), rs.data(), stat.data()),
                  SPMESL_OK);
        }
        o.flags = 0;
        for (Dev *d : ds) delete d;
        // more distinct calls than the graph cache holds (eviction)
        for (int r = 0; r < 6; ++r) {
            o.lambda0 = 0.2 + 0.01 * r;
            std::snprintf(name, sizeof name, "graph cache churn %d (prec %d)", r, prec);
            CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        }
        o.lambda0 = 0.25;
    }
    {
        // a batch in a caller workspace, eagerly and as graphs, then the
        // autotuner and other launch shapes on the same context
        spmesl_options o{};
        o.lambda0 = 0.25;
        o.tol = 1e-8;
        std::vector<Dev *> ds;
        for (int i = 0; i < 5; ++i) ds.push_back(new Dev(60 + 37 * i, 50 + 61 * i, 20 + i));
        std::vector<spmesl_problem> ps;
        std::vector<spmesl_result> rs;
        std::vector<spmesl_stats> sts(ds.size());
        for (size_t i = 0; i < ds.size(); ++i) {
            ps.push_back(ds[i]->prob());
            rs.push_back(ds[i]->res(&sts[i]));
        }
        std::vector<int> stat(ds.size(), 99);
        char name[80];
        for (int fills : {64, 128}) {
            spmesl_tuning t{};
            t.fill_blocks = fills;
            CHECK("set fill blocks", spmesl_set_tuning(ctx, &t), SPMESL_OK);
            for (int prec : {SPMESL_FP64, SPMESL_MIXED}) {
                o.precision = prec;
                size_t need = 0, need_a = 0;
                CHECK("batch workspace size",
                      spmesl_batch_workspace_size(ctx, (int)ds.size(), ps.data(), &o, &need), SPMESL_OK);
                spmesl_problem pa0 = a.prob();
                CHECK("workspace size", spmesl_workspace_size(&pa0, &o, &need_a), SPMESL_OK);
                need = need > need_a ? need : need_a;  // the single solve below shares it
                char *ws = nullptr;
                hipMalloc(&ws, need);
                CHECK("set batch workspace", spmesl_set_workspace(ctx, ws, need), SPMESL_OK);
                for (int r = 0; r < 3; ++r) {
                    o.flags = r == 0 ? SPMESL_FLAG_EAGER : 0;
                    std::snprintf(name, sizeof name, "batch (fill blocks %d), call %d (prec %d)", fills, r, prec);
                    CHECK(name, spmesl_solve_batch(ctx, (int)ds.size(), ps.data(), &o, nullptr, rs.data(), stat.data()),
                          SPMESL_OK);
                }
                o.flags = 0;
                spmesl_problem pa = a.prob();
                spmesl_result ra = a.res(&st);
                std::snprintf(name, sizeof name, "solve after the batch (prec %d)", prec);
                CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
                CHECK("release batch workspace", spmesl_set_workspace(ctx, nullptr, 0), SPMESL_OK);
                hipFree(ws);
            }
        }
        CHECK("reset tuning", spmesl_set_tuning(ctx, nullptr), SPMESL_OK);
        for (Dev *d : ds) delete d;
        o.precision = SPMESL_MIXED;
        spmesl_problem pa = a.prob();
        spmesl_result ra = a.res(&st);
        spmesl_tuning best{};
        double msb = 0.0;
        CHECK("autotune after the batches", spmesl_autotune(ctx, &pa, &o, &ra, 3, &best, &msb), SPMESL_OK);
        {
            // and on a second context
            spmesl_ctx *tctx = nullptr;
            CHECK("create tuning context", spmesl_create(&tctx, 0, nullptr), SPMESL_OK);
            CHECK("autotune on a fresh context", spmesl_autotune(tctx, &pa, &o, &ra, 3, &best, &msb), SPMESL_OK);
            spmesl_destroy(tctx);
        }
        for (int split : {0, 1, 2}) {
            spmesl_tuning t = best;
            t.fill_split = split;
            t.kkt_rows = 1;
            CHECK("set fill placement", spmesl_set_tuning(ctx, &t), SPMESL_OK);
            std::snprintf(name, sizeof name, "solve with fill placement %d", split);
            CHECK(name, spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        }
        CHECK("reset tuning", spmesl_set_tuning(ctx, nullptr), SPMESL_OK);
        o.precision = SPMESL_FP64;
        o.flags = SPMESL_FLAG_DATA_FORM;
        CHECK("data form", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        o.flags = SPMESL_FLAG_DATA_FORM | SPMESL_FLAG_EAGER;
        CHECK("data form eager", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
        o.precision = SPMESL_MIXED;
        o.flags = SPMESL_FLAG_FULL_KKT;
        CHECK("full KKT pass", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
    }
    // error paths
    spmesl_options o{};
    o.lambda0 = -1.0;
    o.tol = 1e-8;
    spmesl_problem pa = a.prob();
    spmesl_result ra = a.res(&st);
    CHECK("negative lambda0", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_EINVAL);
    o.lambda0 = 0.25;
    spmesl_problem big = pa;
    big.n = 400;
    big.p = 5000;
    big.ldx = 5000;
    CHECK("noalloc beyond its array", spmesl_solve_noalloc(ctx, &big, &o, &ra, status_dev), SPMESL_ENOMEM);
    // a caller workspace, too small and then exact
    size_t need = 0;
    CHECK("workspace size", spmesl_workspace_size(&pa, &o, &need), SPMESL_OK);
    char *ws = nullptr;
    hipMalloc(&ws, need);
    CHECK("set small workspace", spmesl_set_workspace(ctx, ws, need - 256), SPMESL_OK);
    CHECK("solve in small workspace", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_ENOMEM);
    CHECK("set exact workspace", spmesl_set_workspace(ctx, ws, need), SPMESL_OK);
    CHECK("solve in exact workspace", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
    CHECK("release workspace", spmesl_set_workspace(ctx, nullptr, 0), SPMESL_OK);
    hipFree(ws);
    spmesl_tuning t{};
    t.dense_block = 16;
    t.fill_blocks = 128;
    CHECK("set tuning", spmesl_set_tuning(ctx, &t), SPMESL_OK);
    CHECK("solve tuned", spmesl_solve(ctx, &pa, &o, &ra), SPMESL_OK);
    spmesl_tuning best{};
    double msb = 0.0;
    CHECK("autotune", spmesl_autotune(ctx, &pa, &o, &ra, 2, &best, &msb), SPMESL_OK);
    hipFree(status_dev);
    spmesl_destroy(ctx);
    if (mock_violations) {
        std::printf("HIP stand-in: %ld kernel launches, %ld captures, %ld graph launches, %d rule violations\n",
                    mock_launches(), mock_captures(), mock_graph_launches(), mock_violations());
        fails += mock_violations();
    }
    std::printf("host sanitizer run: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
