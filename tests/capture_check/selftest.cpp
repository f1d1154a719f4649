// Checks that the recording stand-in (hip_record.cpp) reports each kind of
// broken capture rule it claims to detect, and nothing for a legal fork and
// join.  Runs host only; no library code is involved.  Exit code: the number
// of cases that did not behave as expected.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <functional>
#include <vector>

extern "C" long hiprec_violation_count(void);
extern "C" int hiprec_report(FILE *f);

static void kernel_stub() {}

static void launch(hipStream_t s)
{
    (void)hipLaunchKernel((const void *)&kernel_stub, dim3(4), dim3(256), nullptr, 0, s);
}

int main()
{
    hipStream_t a, b, c;
    hipEvent_t e, f;
    hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
    hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
    hipEventCreateWithFlags(&e, hipEventDisableTiming);
    hipEventCreateWithFlags(&f, hipEventDisableTiming);
    double *dev = nullptr, *pin = nullptr;
    hipMalloc((void **)&dev, 1024);
    hipHostMalloc((void **)&pin, 1024, 0);
    std::vector<double> pageable(128);

    struct Case {
        const char *name;
        long expect; // violations the case must add
        std::function<void()> run;
    };
    auto capture = [&](const std::function<void()> &body) {
        hipGraph_t g = nullptr;
        hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
        body();
        hipStreamEndCapture(a, &g);
        if (g)
            hipGraphDestroy(g);
    };
    const std::vector<Case> cases = {
        {"legal fork and join", 0,
         [&] {
             capture([&] {
                 hipEventRecord(e, a);
                 hipStreamWaitEvent(b, e, 0);
                 launch(a);
                 launch(b);
                 hipMemcpyAsync(pin, dev, 1024, hipMemcpyDeviceToHost, b);
                 hipEventRecord(f, b);
                 hipStreamWaitEvent(a, f, 0);
             });
         }},
        {"forked stream not joined", 1,
         [&] {
             capture([&] {
                 hipEventRecord(e, a);
                 hipStreamWaitEvent(b, e, 0);
                 launch(b);
             });
         }},
        {"work on a stream outside the capture", 1, [&] { capture([&] { launch(c); }); }},
        {"allocation inside the capture", 1,
         [&] {
             capture([&] {
                 void *p = nullptr;
                 hipMalloc(&p, 64);
             });
         }},
        {"wait on an event recorded outside the capture", 1,
         [&] {
             hipEventRecord(e, c);
             capture([&] { hipStreamWaitEvent(a, e, 0); });
         }},
        {"captured copy to pageable memory", 1,
         [&] {
             capture([&] {
                 hipMemcpyAsync(pageable.data(), dev, 64, hipMemcpyDeviceToHost, a);
             });
         }},
        {"copy past the end of an allocation", 1,
         [&] { hipMemcpyAsync(pin, dev, 2048, hipMemcpyDeviceToHost, c); }},
        {"host wait inside the capture", 1, [&] { capture([&] { hipStreamSynchronize(c); }); }},
        {"pinned buffer freed while a graph copies into it", 2,
         [&] {
             hipGraph_t g = nullptr;
             hipGraphExec_t x = nullptr;
             double *tmp = nullptr;
             hipHostMalloc((void **)&tmp, 256, 0);
             hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
             hipMemcpyAsync(tmp, dev, 256, hipMemcpyDeviceToHost, a);
             hipStreamEndCapture(a, &g);
             hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
             hipHostFree(tmp);      // the graph and its executable still copy into it
             hipGraphLaunch(x, a);  // and it is launched afterwards
             hipGraphExecDestroy(x);
             hipGraphDestroy(g);
         }},
        {"invalid launch shape", 1,
         [&] {
             (void)hipLaunchKernel((const void *)&kernel_stub, dim3(0), dim3(256), nullptr, 0, c);
         }},
    };
    int bad = 0;
    for (const Case &k : cases) {
        const long before = hiprec_violation_count();
        k.run();
        const long got = hiprec_violation_count() - before;
        const bool ok = k.expect == 0 ? got == 0 : got >= k.expect;
        std::printf("%-52s expected %s%ld, got %ld: %s\n", k.name, k.expect ? ">= " : "",
                    k.expect, got, ok ? "ok" : "WRONG");
        bad += !ok;
    }
    return bad;
}
