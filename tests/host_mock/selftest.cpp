// The stand-in's rule checks report what they should: each block below
// breaks one rule of stream capture (or keeps them) and the violation count
// must move by exactly the expected amount.
#include <hip/hip_runtime.h>

#include <cstdio>

extern "C" int mock_violations();

static int bad = 0;
static void expect(const char *what, int before, int added)
{
    const int got = mock_violations() - before;
    std::printf("%-48s %d violation(s) (want %d)%s\n", what, got, added, got == added ? "" : "  <-- FAIL");
    if (got != added) ++bad;
}

int main()
{
    hipStream_t a, b;
    hipEvent_t fork, join;
    hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
    hipEventCreate(&fork);
    hipEventCreate(&join);
    hipGraph_t g = nullptr;
    int v = mock_violations();
    // a fork joined back: no violation
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipEventRecord(fork, a);
    hipStreamWaitEvent(b, fork, 0);
    hipEventRecord(join, b);
    hipStreamWaitEvent(a, join, 0);
    hipStreamEndCapture(a, &g);
    hipGraphDestroy(g);
    expect("fork and join", v, 0);
    // a fork never joined back
    v = mock_violations();
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipEventRecord(fork, a);
    hipStreamWaitEvent(b, fork, 0);
    hipEventRecord(join, b);
    hipStreamEndCapture(a, &g);
    expect("fork not joined", v, 1);
    // work on the forked stream after its join
    v = mock_violations();
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipEventRecord(fork, a);
    hipStreamWaitEvent(b, fork, 0);
    hipEventRecord(join, b);
    hipStreamWaitEvent(a, join, 0);
    hipEventRecord(fork, b);
    hipStreamEndCapture(a, &g);
    expect("work after the join", v, 1);
    // a copy and a synchronisation while capturing
    v = mock_violations();
    int x = 1, y = 0;
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipMemcpyAsync(&y, &x, sizeof x, hipMemcpyDeviceToHost, a);
    hipStreamSynchronize(a);
    hipStreamEndCapture(a, &g);
    hipGraphDestroy(g);
    expect("copy and synchronisation in a capture", v, 2);
    // a launch outside the hardware's limits
    v = mock_violations();
    hipLaunchKernel(nullptr, dim3(0), dim3(64), nullptr, 0, a);
    hipLaunchKernel(nullptr, dim3(1), dim3(2048), nullptr, 0, a);
    hipLaunchKernel(nullptr, dim3(1), dim3(64), nullptr, 200 * 1024, a);
    hipGetLastError();
    expect("launch shapes out of range", v, 3);
    hipEventDestroy(fork);
    hipEventDestroy(join);
    hipStreamDestroy(a);
    hipStreamDestroy(b);
    std::printf("stand-in self-test: %d failed\n", bad);
    return bad ? 1 : 0;
}
