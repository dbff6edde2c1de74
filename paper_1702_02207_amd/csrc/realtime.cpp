// Real-time periodic stepping (osc_rt_*).
//
// The paper proposes the oscillator as a time-critical workload: a model
// stepped in hardware- or software-in-the-loop simulation, and a benchmark of
// periodic hard-deadline threads and of the delay of parallel systems
// (introduction, section 5).  Here one handle's state is held on the device
// and advanced one tick (steps_per_tick steps, one launch) per wall-clock
// period: at each release time the host enqueues the tick, then polls its
// completion event (with a wall-clock cap, so no wait is unbounded) and
// records the latency from release to the result being ready.  A tick is a
// chunk of the handle's chunked integration from the global step count, so
// the periodic trajectory is bit for bit that of one osc_integrate call.
// The resident mode (osc_rt_run_resident, chains) keeps one kernel on the
// device for the whole run instead (resident.hip): the host raises a release
// counter in host-mapped memory and polls the kernel's completion count, so a
// tick costs no launch and no event; both waits are bounded.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "osc_internal.h"

using namespace osc;

struct osc_rt {
    osc_sys *sys = nullptr;
    int64_t k = 1;             // steps per tick
    int64_t n = 0;             // steps taken
    void *x0 = nullptr, *v0 = nullptr;   // device copies of the initial state (read by the first tick)
    void *xo = nullptr, *vo = nullptr;   // output of a tick when the caller gives none
    size_t bytes = 0;          // batch * s elements of the handle's type
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    // resident runs: the host-mapped control block (host and device address)
    osc::RtControl *ctl = nullptr, *ctl_dev = nullptr;
    double idle_s = 0.0;       // 0: max(0.1 s, 50 periods)
    bool broken = false;       // a resident run failed part-way: the held state is undefined
};

namespace {

using clock_type = std::chrono::steady_clock;

double seconds(clock_type::duration d) { return std::chrono::duration<double>(d).count(); }

void rt_release(osc_rt *rt) {
    if (!rt) return;
    if (rt->sys) (void)hipStreamSynchronize(rt->sys->stream);
    for (void *p : {rt->x0, rt->v0, rt->xo, rt->vo}) pool_free(p);
    if (rt->ctl) (void)hipHostFree(rt->ctl);
    if (rt->ev_start) (void)hipEventDestroy(rt->ev_start);
    if (rt->ev_end) (void)hipEventDestroy(rt->ev_end);
    delete rt;
}

// Wait until `e` has completed, polling (the lowest latency), for at most
// `cap` seconds of wall clock.
osc_status wait_event(hipEvent_t e, double cap) {
    const auto t0 = clock_type::now();
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return OSC_OK;
        if (q != hipErrorNotReady) return fail(OSC_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
        if (seconds(clock_type::now() - t0) > cap) return fail(OSC_ETIMEOUT, "a real-time tick did not complete");
    }
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = p / 100.0 * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

osc_rt_stats summarize(const std::vector<double> &lat, const std::vector<double> &launch,
                       const std::vector<double> &gpu, int64_t missed) {
    osc_rt_stats o{};
    o.ticks = (int64_t)lat.size();
    o.missed = missed;
    if (!lat.empty()) {
        double mean = 0.0;
        for (double v : lat) mean += v;
        mean /= (double)lat.size();
        double var = 0.0;
        for (double v : lat) var += (v - mean) * (v - mean);
        o.mean_s = mean;
        o.jitter_s = std::sqrt(var / (double)lat.size());
        o.p50_s = percentile(lat, 50.0);
        o.p99_s = percentile(lat, 99.0);
        o.max_s = *std::max_element(lat.begin(), lat.end());
        o.launch_p99_s = percentile(launch, 99.0);
        o.gpu_p50_s = percentile(gpu, 50.0);
    }
    return o;
}

}  // namespace

extern "C" {

osc_status osc_rt_create(osc_sys *sys, const void *x0, const void *v0, int64_t steps_per_tick, osc_rt **out) {
    set_error("");
    if (!out) return fail(OSC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sys || !x0 || !v0) return fail(OSC_EINVAL, "handle, x0 and v0 must be non-NULL");
    if (steps_per_tick < 1) return fail(OSC_EINVAL, "steps_per_tick must be >= 1");
    if (sys->batch < 1) return fail(OSC_EINVAL, "real-time stepping needs at least one instance");
    osc_status r = sys_rt_supported(sys);
    if (r) return r;
    osc_rt *rt = new (std::nothrow) osc_rt();
    if (!rt) return fail(OSC_ENOMEM, "host allocation failed");
    rt->sys = sys;
    rt->k = steps_per_tick;
    rt->bytes = (size_t)sys->batch * sys->s * (sys->prec == OSC_F64 ? sizeof(double) : sizeof(float));
    rt->x0 = pool_alloc(rt->bytes);
    rt->v0 = pool_alloc(rt->bytes);
    rt->xo = pool_alloc(rt->bytes);
    rt->vo = pool_alloc(rt->bytes);
    if (!rt->x0 || !rt->v0 || !rt->xo || !rt->vo) {
        rt_release(rt);
        return fail(OSC_ENOMEM, "device memory exhausted for the real-time stepper");
    }
    hipError_t e = hipMemcpyAsync(rt->x0, x0, rt->bytes, hipMemcpyDeviceToDevice, sys->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rt->v0, v0, rt->bytes, hipMemcpyDeviceToDevice, sys->stream);
    if (e == hipSuccess) e = hipEventCreate(&rt->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&rt->ev_end);
    if (e == hipSuccess) e = hipStreamSynchronize(sys->stream);
    if (e != hipSuccess) {
        rt_release(rt);
        return fail(OSC_EDEVICE, std::string("osc_rt_create: ") + hipGetErrorString(e));
    }
    *out = rt;
    return OSC_OK;
}

osc_status osc_rt_tick(osc_rt *rt, void *x_out, void *v_out) {
    set_error("");
    if (!rt) return fail(OSC_EINVAL, "stepper is NULL");
    if (rt->broken) return fail(OSC_EDEVICE, "the stepper's state was lost in a failed resident run; destroy it");
    osc_status r = sys_rt_tick(rt->sys, rt->x0, rt->v0, rt->n, rt->k, x_out ? x_out : rt->xo,
                               v_out ? v_out : rt->vo);
    if (r) return r;
    rt->n += rt->k;
    return OSC_OK;
}

int64_t osc_rt_steps(const osc_rt *rt) { return rt ? rt->n : -1; }

osc_status osc_rt_run(osc_rt *rt, double period_s, int64_t nticks, void *x_frames, void *v_frames,
                      double *latencies, osc_rt_stats *stats) {
    set_error("");
    if (!rt) return fail(OSC_EINVAL, "stepper is NULL");
    if (rt->broken) return fail(OSC_EDEVICE, "the stepper's state was lost in a failed resident run; destroy it");
    if (!(period_s > 0.0 && period_s < 60.0)) return fail(OSC_EINVAL, "period_s must be in (0, 60)");
    if (nticks < 0) return fail(OSC_EINVAL, "nticks must be >= 0");
    const hipStream_t st = rt->sys->stream;
    std::vector<double> lat((size_t)nticks), launch((size_t)nticks), gpu((size_t)nticks);
    int64_t missed = 0;
    // wait for queued work first, so the first release is not delayed by it
    if (hipStreamSynchronize(st) != hipSuccess) return fail(OSC_EDEVICE, "hipStreamSynchronize failed");
    const auto period = std::chrono::duration_cast<clock_type::duration>(std::chrono::duration<double>(period_s));
    const auto t0 = clock_type::now() + period;
    const double cap = std::max(10.0, 100.0 * period_s);
    for (int64_t i = 0; i < nticks; ++i) {
        const auto release = t0 + i * period;
        // sleep while the release is far, then spin to it
        for (auto now = clock_type::now(); now < release; now = clock_type::now()) {
            if (release - now > std::chrono::microseconds(300))
                std::this_thread::sleep_for(release - now - std::chrono::microseconds(200));
        }
        const auto t_launch = clock_type::now();
        char *xf = x_frames ? static_cast<char *>(x_frames) + (size_t)i * rt->bytes : nullptr;
        char *vf = v_frames ? static_cast<char *>(v_frames) + (size_t)i * rt->bytes : nullptr;
        if (hipEventRecord(rt->ev_start, st) != hipSuccess) return fail(OSC_EDEVICE, "hipEventRecord failed");
        osc_status r = osc_rt_tick(rt, xf, vf);
        if (r) return r;
        if (hipEventRecord(rt->ev_end, st) != hipSuccess) return fail(OSC_EDEVICE, "hipEventRecord failed");
        if ((r = wait_event(rt->ev_end, cap))) return r;
        const auto t_done = clock_type::now();
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, rt->ev_start, rt->ev_end);
        lat[(size_t)i] = seconds(t_done - release);
        launch[(size_t)i] = seconds(t_launch - release);
        gpu[(size_t)i] = 1e-3 * ms;
        if (t_done > release + period) ++missed;
        if (latencies) latencies[i] = lat[(size_t)i];
    }
    if (stats) *stats = summarize(lat, launch, gpu, missed);
    return OSC_OK;
}

osc_status osc_rt_set_idle_limit(osc_rt *rt, double seconds) {
    set_error("");
    if (!rt) return fail(OSC_EINVAL, "stepper is NULL");
    if (!(seconds >= 0.0 && seconds < 3600.0)) return fail(OSC_EINVAL, "the idle limit must be in [0, 3600) seconds");
    rt->idle_s = seconds;
    return OSC_OK;
}

osc_status osc_rt_run_resident(osc_rt *rt, double period_s, int64_t nticks, void *x_frames, void *v_frames,
                               double *latencies, osc_rt_stats *stats) {
    set_error("");
    if (!rt) return fail(OSC_EINVAL, "stepper is NULL");
    if (rt->broken) return fail(OSC_EDEVICE, "the stepper's state was lost in a failed resident run; destroy it");
    if (!(period_s > 0.0 && period_s < 60.0)) return fail(OSC_EINVAL, "period_s must be in (0, 60)");
    if (nticks < 0) return fail(OSC_EINVAL, "nticks must be >= 0");
    osc_status r = sys_rt_resident_supported(rt->sys);
    if (r) return r;
    const hipStream_t st = rt->sys->stream;
    if (!rt->ctl) {
        void *h = nullptr, *d = nullptr;
        hipError_t e = hipHostMalloc(&h, sizeof(RtControl), hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) return fail(OSC_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        if ((e = hipHostGetDevicePointer(&d, h, 0)) != hipSuccess) {
            (void)hipHostFree(h);
            return fail(OSC_EDEVICE, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
        }
        rt->ctl = static_cast<RtControl *>(h);
        rt->ctl_dev = static_cast<RtControl *>(d);
    }
    std::vector<double> lat((size_t)nticks), launch((size_t)nticks), gpu((size_t)nticks, 0.0);
    int64_t missed = 0;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(OSC_EDEVICE, "hipStreamSynchronize failed");
    if (nticks > 0) {
        RtControl *c = rt->ctl;
        __atomic_store_n(&c->release, (int64_t)0, __ATOMIC_SEQ_CST);
        __atomic_store_n(&c->done, (uint64_t)0, __ATOMIC_SEQ_CST);
        __atomic_store_n(&c->exit_reason, kRtExitRunning, __ATOMIC_SEQ_CST);
        const double idle = rt->idle_s > 0.0 ? rt->idle_s : std::max(0.1, 50.0 * period_s);
        ResidentSpec spec{rt->ctl_dev, nticks, rt->n, rt->k, (int64_t)(idle * 1e8),
                          x_frames, v_frames, rt->xo, rt->vo};
        int64_t blocks = 0;
        if ((r = sys_rt_resident(rt->sys, rt->x0, rt->v0, spec, &blocks))) return r;   // nothing launched
        // from here on the kernel runs: every way out stops it and waits for it
        auto abort_run = [&](osc_status code, const std::string &msg) {
            __atomic_store_n(&c->release, (int64_t)-1, __ATOMIC_SEQ_CST);
            (void)hipStreamSynchronize(st);
            rt->broken = true;
            return fail(code, msg);
        };
        const auto period = std::chrono::duration_cast<clock_type::duration>(std::chrono::duration<double>(period_s));
        const auto t0 = clock_type::now() + period;
        const double cap = std::max(10.0, 100.0 * period_s);
        for (int64_t i = 0; i < nticks; ++i) {
            const auto release = t0 + i * period;
            for (auto now = clock_type::now(); now < release; now = clock_type::now()) {
                if (release - now > std::chrono::microseconds(300))
                    std::this_thread::sleep_for(release - now - std::chrono::microseconds(200));
            }
            __atomic_store_n(&c->release, i + 1, __ATOMIC_SEQ_CST);
            const auto t_raised = clock_type::now();
            const uint64_t want = (uint64_t)(i + 1) * (uint64_t)blocks;
            while (__atomic_load_n(&c->done, __ATOMIC_ACQUIRE) < want) {
                const int reason = __atomic_load_n(&c->exit_reason, __ATOMIC_ACQUIRE);
                if (reason == kRtExitIdle)
                    return abort_run(OSC_ETIMEOUT, "the resident kernel reached its idle limit before a release");
                if (reason == kRtExitStop)
                    return abort_run(OSC_EDEVICE, "the resident kernel ended before the run's last tick");
                if (seconds(clock_type::now() - t_raised) > cap)
                    return abort_run(OSC_ETIMEOUT, "a resident real-time tick did not complete");
            }
            const auto t_done = clock_type::now();
            lat[(size_t)i] = seconds(t_done - release);
            launch[(size_t)i] = seconds(t_raised - release);
            if (t_done > release + period) ++missed;
            if (latencies) latencies[i] = lat[(size_t)i];
        }
        __atomic_store_n(&c->release, (int64_t)-1, __ATOMIC_SEQ_CST);
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            rt->broken = true;
            return fail(OSC_EDEVICE, std::string("resident run: ") + hipGetErrorString(e));
        }
        rt->n += nticks * rt->k;
    }
    if (stats) *stats = summarize(lat, launch, gpu, missed);
    return OSC_OK;
}

void osc_rt_destroy(osc_rt *rt) { rt_release(rt); }

}  // extern "C"
