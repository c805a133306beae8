// Autotuner: picks, per problem shape and device, the launch configuration of
// the kernels whose best shape is not known in advance, by timing every
// candidate on the context's own data once (HIP events) and keeping the
// fastest.  Results are kept per process and, when a path is given, in a small
// text file (one "shape nred staged rpt" line per shape) so that later setups of the
// same shape skip the timing.
//
// Tuned:
//   nred, rpt      workgroups of the reducing PCG kernels (64 ... 1024) and vertex
//                  rows per thread in their tiles (1, 4): fewer partials to sum
//                  against more tiles per workgroup, and more loads in flight per
//                  thread against fewer workgroups with work;
//   smooth_staged  smoother: each chain step's blocks staged in LDS by the forward and
//                  again by the backward chains (0), or kept in LDS from the forward
//                  chains for the backward ones (1).
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "common.h"

namespace {

struct TuneRec {
    int nred = 256;
    int staged = 1;
    int rpt = 1;
};

std::mutex g_tune_mu;
std::map<std::string, TuneRec> g_tune;

std::string tune_key(tgms_ctx* c) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "v3/%s/%dx%d/b%dx%d/ov%d/p%d", arch.c_str(), c->nx, c->ny, c->bx, c->by,
                  c->overlap, c->precision);
    return buf;
}

// the cache file: one line per shape, "key nred staged rpt"
void load_cache(const char* path) {
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512], key[256];
    int nred = 0, staged = 0, rpt = 0;
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line, "%255s %d %d %d", key, &nred, &staged, &rpt) != 4) continue;
        if (nred >= 1 && nred <= tgms::nred_max() && staged >= 0 && staged <= 2 && (rpt == 1 || rpt == 4))
            g_tune[key] = TuneRec{nred, staged, rpt};
    }
    std::fclose(f);
}

void save_cache(const char* path) {
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (auto& kv : g_tune)
        std::fprintf(f, "%s %d %d %d\n", kv.first.c_str(), kv.second.nred, kv.second.staged, kv.second.rpt);
    std::fclose(f);
}

template <typename F>
double time_ms(tgms_ctx* c, int reps, F&& body) {
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    body();  // warm-up
    HIP_OK(hipEventRecord(a, c->stream));
    for (int r = 0; r < reps; ++r) body();
    HIP_OK(hipEventRecord(b, c->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

}  // namespace

namespace tgms {

void autotune(tgms_ctx* c, const char* cache_path) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_cache(cache_path);
    const std::string key = tune_key(c);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
        c->nred = it->second.nred;
        c->smooth_staged = it->second.staged;
        c->rpt = it->second.rpt;
        c->tuned = 2;
        return;
    }
    const long long nv = (long long)c->nx * c->ny;
    // scalars that let the PCG kernels run (done flag clear), on zero vectors
    for (int k = 0; k < SC_COUNT; ++k) c->red_h[k] = 0.0;
    c->red_h[SC_MAXIT] = 1e9;
    c->red_h[SC_RTOL2] = 0.0;
    HIP_OK(hipMemcpyAsync(c->sc, c->red_h, SC_COUNT * sizeof(double), hipMemcpyHostToDevice, c->stream));
    zero(c, c->vz, sizeof(double) * nv);
    zero(c, c->vp, sizeof(double) * nv);
    zero(c, c->vg, sizeof(double) * nv);
    TuneRec best;
    double tbest = 1e30;
    for (int nred : {64, 128, 256, 512, 1024})
        for (int rpt : {1, 4}) {
            c->nred = nred;
            c->rpt = rpt;
            const double t = time_ms(c, 5, [&] { dir_apply(c, c->vz, c->vp, c->vp1, c->vq); });
            if (t < tbest) {
                tbest = t;
                best.nred = nred;
                best.rpt = rpt;
            }
        }
    c->nred = best.nred;
    c->rpt = best.rpt;
    // smoother: every step's blocks staged twice (forward and backward chains) or kept
    // in LDS from the forward chains (fewer bytes, fewer workgroups per CU)
    const bool prec32 = c->precision != 0;
    double ts[2] = {1e30, 1e30};
    // timed as whole two-grid applications: the solve's smoothings also form their
    // right-hand sides, which changes the balance between the modes
    (void)prec32;
    for (int st = 0; st < 2; ++st) {
        c->smooth_staged = st;
        ts[st] = time_ms(c, 3, [&] { twogrid_probe(c); });
    }
    best.staged = ts[1] < ts[0] ? 1 : 0;
    c->smooth_staged = best.staged;
    HIP_OK(hipStreamSynchronize(c->stream));
    c->tuned = 1;
    g_tune[key] = best;
    save_cache(cache_path);
}

}  // namespace tgms
