// Launch-configuration autotuner with an on-disk cache.
//
// For a handle, every feasible configuration is timed on the handle's own
// batch (chains: the lane layouts whose capacity covers s without more than
// 4x padding; dense: the VALU, MFMA and split kernels the handle can use).
// The fastest becomes the handle's configuration and is appended to the cache
// file named by OSC_AUTOTUNE_CACHE, one line per key:
//     <kind> <method> <prec> <s> <batch bucket> <arch> <config>
// osc_create applies a cached configuration when one matches.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "osc_internal.h"

namespace osc {
namespace {

std::mutex g_cache_mu;

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// batch bucket: floor(log2(batch))
int bucket(int64_t batch) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= batch) ++b;
    return b;
}

std::string cache_key(const osc_sys *s) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s %s %s %d %d %s", s->kind == OSC_CHAIN ? "chain" : "dense",
                  s->method == OSC_RK4 ? "rk4" : "verlet", s->prec == OSC_F32 ? "f32" : "f64", (int)s->s,
                  bucket(s->batch), arch_name().c_str());
    return buf;
}

osc_status apply(osc_sys *s, int64_t code) {
    return osc_set_config(s, s->kind == OSC_CHAIN ? OSC_CFG_CHAIN_LAYOUT : OSC_CFG_DENSE_KERNEL, code);
}

}  // namespace

// Apply a cached configuration to a freshly created handle (silently keeps
// the default when the cache has no usable entry).
void autotune_apply_cached(osc_sys *s) {
    const char *path = std::getenv("OSC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    const std::string key = cache_key(s);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    long long best = -1;
    while (std::fgets(line, sizeof line, f)) {
        const size_t n = key.size();
        if (std::strncmp(line, key.c_str(), n) == 0 && line[n] == ' ') best = std::atoll(line + n + 1);
    }
    std::fclose(f);
    if (best >= 0) {
        const std::string saved = osc_last_error();
        if (apply(s, best) != OSC_OK) (void)apply(s, 0);
        set_error(saved);
    }
}

}  // namespace osc

using namespace osc;

extern "C" osc_status osc_autotune(osc_sys *s, const void *x0, const void *v0, int64_t probe_steps,
                                   int64_t *chosen) {
    if (!s || !x0 || !v0) return fail(OSC_EINVAL, "handle, x0 and v0 must be non-NULL");
    if (probe_steps < 1) return fail(OSC_EINVAL, "probe_steps must be >= 1");
    // their kernels choose their own layouts, and a time measured on them
    // must not enter the cache under the free system's key
    if (s->driven || s->vdp_mu > 0.0)
        return fail(OSC_ENOTSUP, "osc_autotune tunes the free integrators; damped, driven and Van der Pol "
                                 "handles take fixed layouts");
    if (s->batch == 0) return OSC_OK;
    std::vector<int64_t> cands;
    if (s->kind == OSC_CHAIN) {
        for (int i = 0; i < chain_num_configs(); ++i) {
            const ChainConfig c = chain_config_at(i);
            const long cap = (long)c.lpi * c.dpl;
            if (cap < s->s || cap > 4L * s->s + 4) continue;
            if (s->s > 8 && c.lpi == 1) continue;   // lane-per-instance layouts cover s <= 8 only
            cands.push_back(((int64_t)c.lpi << 16) | c.dpl);
        }
    } else {
        for (int64_t k : {1, 2, 3})
            if (osc_set_config(s, OSC_CFG_DENSE_KERNEL, k) == OSC_OK) cands.push_back(k);
        (void)osc_set_config(s, OSC_CFG_DENSE_KERNEL, 0);
    }
    if (cands.empty()) return fail(OSC_ENOTSUP, "no configuration to tune");
    const size_t bytes = (size_t)s->batch * s->s * (s->prec == OSC_F64 ? 8 : 4);
    void *xe = pool_alloc(bytes), *ve = pool_alloc(bytes);
    if (!xe || !ve) {
        pool_free(xe);
        pool_free(ve);
        return fail(OSC_ENOMEM, "device memory exhausted in osc_autotune");
    }
    hipEvent_t a, b;
    OSC_HIP(hipEventCreate(&a));
    OSC_HIP(hipEventCreate(&b));
    const int64_t saved_spl = s->steps_per_launch;
    s->steps_per_launch = 0;
    double best_ms = 1e300;
    int64_t best = cands[0];
    osc_status r = OSC_OK;
    for (int64_t c : cands) {
        if ((r = apply(s, c)) != OSC_OK) break;
        // warm-up (first launch of a kernel), then the timed probe
        if ((r = osc_integrate(s, x0, v0, 1, 0, nullptr, nullptr, xe, ve)) != OSC_OK) break;
        OSC_HIP(hipEventRecord(a, s->stream));
        if ((r = osc_integrate(s, x0, v0, probe_steps, 0, nullptr, nullptr, xe, ve)) != OSC_OK) break;
        OSC_HIP(hipEventRecord(b, s->stream));
        OSC_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        OSC_HIP(hipEventElapsedTime(&ms, a, b));
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    pool_free(xe);
    pool_free(ve);
    s->steps_per_launch = saved_spl;
    if (r != OSC_OK) return r;
    if ((r = apply(s, best)) != OSC_OK) return r;
    if (chosen) *chosen = best;
    const char *path = std::getenv("OSC_AUTOTUNE_CACHE");
    if (path && *path) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %lld\n", cache_key(s).c_str(), (long long)best);
            std::fclose(f);
        }
    }
    return OSC_OK;
}
