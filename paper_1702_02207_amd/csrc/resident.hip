// Resident real-time stepping of chains (free, damped and driven, or Van der
// Pol, in the register layouts): one kernel stays on the device for a whole periodic run and advances the state one tick (steps_per_tick steps)
// each time the host raises a release counter in host-mapped memory, instead
// of one launch per tick.  The host writes the counter at each release time
// and polls a completion count that the kernel raises once per workgroup and
// tick, after the tick's results are stored and made visible system-wide.
//
// Each tick runs the chain integrator (chain_run.h) from the global step the
// run has reached, loading the held state and storing it back beside the
// tick's output: the arithmetic and the chunk boundaries are those of
// launching one kernel per tick, so the two modes give bitwise the same
// trajectory.  Instances are independent, so every workgroup waits for the
// release and works on its own; the host only launches grids whose
// workgroups can all be resident at once.
//
// Every wait is bounded: a workgroup gives up when no release arrives within
// the idle limit (measured with the 100 MHz real-time counter, and capped by
// a poll count as well), when the host writes the stop value, or after the
// run's last tick.

#include <cstdint>
#include <string>

#include "chain_run.h"
#include "driven_run.h"
#include "vdp.h"
#include "vdp_run.h"

namespace osc {
namespace {

constexpr int kResidentThreads = 256;

// 1: tick `want` released; 0: stop requested; -1: idle limit reached
__device__ int wait_release(RtControl *ctl, int64_t want, int64_t idle_ticks) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    // each poll takes far more than 40 ns (a system-scope load from host
    // memory plus a sleep), so this count ends the loop only if the
    // real-time counter does not advance
    const int64_t max_polls = idle_ticks / 4 + 1000;
    for (int64_t p = 0; p < max_polls; ++p) {
        const int64_t rel = __hip_atomic_load(&ctl->release, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        if (rel < 0) return 0;
        if (rel >= want) return 1;
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > idle_ticks) return -1;
        __builtin_amdgcn_s_sleep(1);
    }
    return -1;
}

template <typename T, int DPL, int LPI, int METHOD, bool FREE>
__global__ void __launch_bounds__(kResidentThreads) chain_resident_kernel(ChainLaunch<T> a, ResidentRun<T> r) {
    __shared__ int go;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t plane = (size_t)a.batch * a.s;
    int reason = kRtExitTicks;
    for (int64_t i = 0; i < r.nticks; ++i) {
        if (threadIdx.x == 0) go = wait_release(r.ctl, r.first_release + i + 1, r.idle_ticks);
        __syncthreads();
        const int gv = go;
        __syncthreads();   // every thread has read go before it is written again
        if (gv != 1) {
            reason = gv == 0 ? kRtExitStop : kRtExitIdle;
            break;
        }
        ChainLaunch<T> t = a;
        t.n0 = r.n_start + i * r.k;
        t.nsteps = r.k;
        t.out_stride = 0;
        t.load_mode = t.n0 == 0 ? LOAD_USER : LOAD_STATE;
        t.store_mode = STORE_STATE | STORE_USER;
        t.xe = r.xf ? r.xf + (size_t)i * plane : r.xo;
        t.ve = r.vf ? r.vf + (size_t)i * plane : r.vo;
        chain_run<T, DPL, LPI, METHOD, FREE>(t, g / LPI, (int)(g % LPI));
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&r.ctl->done, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // a workgroup that ends early says why (the host then stops the others)
    if (threadIdx.x == 0 && reason != kRtExitTicks)
        __hip_atomic_store(&r.ctl->exit_reason, reason, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Damped, driven chains in the register layouts (driven_run.h), the same
// release protocol.
template <typename T, int DPL, int LPI, int EX>
__global__ void __launch_bounds__(kResidentThreads, (sizeof(T) == 8 && DPL == 16) ? 1 : 2)
    driven_resident_kernel(DrivenLaunch<T> a, ResidentRun<T> r) {
    __shared__ int go;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t plane = (size_t)a.batch * a.s;
    int reason = kRtExitTicks;
    for (int64_t i = 0; i < r.nticks; ++i) {
        if (threadIdx.x == 0) go = wait_release(r.ctl, r.first_release + i + 1, r.idle_ticks);
        __syncthreads();
        const int gv = go;
        __syncthreads();
        if (gv != 1) {
            reason = gv == 0 ? kRtExitStop : kRtExitIdle;
            break;
        }
        DrivenLaunch<T> t = a;
        t.n0 = r.n_start + i * r.k;
        t.nsteps = r.k;
        t.out_stride = 0;
        t.load_mode = t.n0 == 0 ? LOAD_USER : LOAD_STATE;
        t.store_mode = STORE_STATE | STORE_USER;
        t.xe = r.xf ? r.xf + (size_t)i * plane : r.xo;
        t.ve = r.vf ? r.vf + (size_t)i * plane : r.vo;
        driven_chain_run<T, DPL, LPI, EX>(t, g);
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&r.ctl->done, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (threadIdx.x == 0 && reason != kRtExitTicks)
        __hip_atomic_store(&r.ctl->exit_reason, reason, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T, int DPL, int LPI, bool FORCED>
__global__ void __launch_bounds__(kResidentThreads, (sizeof(T) == 8 && DPL == 16) ? 1 : 2)
    vdp_resident_kernel(VdpLaunch<T> a, ResidentRun<T> r) {
    __shared__ int go;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t plane = (size_t)a.batch * a.s;
    int reason = kRtExitTicks;
    for (int64_t i = 0; i < r.nticks; ++i) {
        if (threadIdx.x == 0) go = wait_release(r.ctl, r.first_release + i + 1, r.idle_ticks);
        __syncthreads();
        const int gv = go;
        __syncthreads();
        if (gv != 1) {
            reason = gv == 0 ? kRtExitStop : kRtExitIdle;
            break;
        }
        VdpLaunch<T> t = a;
        t.n0 = r.n_start + i * r.k;
        t.nsteps = r.k;
        t.out_stride = 0;
        t.load_mode = t.n0 == 0 ? LOAD_USER : LOAD_STATE;
        t.store_mode = STORE_STATE | STORE_USER;
        t.xe = r.xf ? r.xf + (size_t)i * plane : r.xo;
        t.ve = r.vf ? r.vf + (size_t)i * plane : r.vo;
        vdp_chain_run<T, DPL, LPI, FORCED>(t, g);
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&r.ctl->done, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (threadIdx.x == 0 && reason != kRtExitTicks)
        __hip_atomic_store(&r.ctl->exit_reason, reason, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Every workgroup must be resident at once: one that waits for a free CU
// would only start when the others end.
osc_status check_resident(const void *f, int64_t blocks, int bs) {
    int dev = 0, cus = 0, per_cu = 0;
    OSC_HIP(hipGetDevice(&dev));
    OSC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    OSC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, bs, 0));
    if (blocks > (int64_t)per_cu * cus)
        return fail(OSC_ENOTSUP, "resident stepping: the batch needs " + std::to_string(blocks) +
                                     " workgroups, more than can be resident at once (" +
                                     std::to_string((int64_t)per_cu * cus) + ")");
    return OSC_OK;
}

template <typename T, int DPL, int LPI>
osc_status launch_driven_layout(const DrivenLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st) {
    const int ex = (a.beta != 0.0 ? 1 : 0) | (a.f ? 2 : 0);
    void (*f)(DrivenLaunch<T>, ResidentRun<T>) =
        ex == 0 ? &driven_resident_kernel<T, DPL, LPI, 0>
                : ex == 1 ? &driven_resident_kernel<T, DPL, LPI, 1>
                          : ex == 2 ? &driven_resident_kernel<T, DPL, LPI, 2> : &driven_resident_kernel<T, DPL, LPI, 3>;
    const int64_t blocks = (a.batch * LPI + kResidentThreads - 1) / kResidentThreads;
    osc_status e = check_resident(reinterpret_cast<const void *>(f), blocks, kResidentThreads);
    if (e) return e;
    hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(kResidentThreads), 0, st, a, r);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T, int METHOD>
using ResidentFn = void (*)(ChainLaunch<T>, ResidentRun<T>);

template <typename T, int METHOD, int... I>
constexpr auto make_resident_table(std::integer_sequence<int, I...>) {
    struct Table {
        ResidentFn<T, METHOD> f[sizeof...(I)];
        ResidentFn<T, METHOD> free_end[sizeof...(I)];
    };
    return Table{{&chain_resident_kernel<T, kConfigs[I].dpl, kConfigs[I].lpi, METHOD, false>...},
                 {&chain_resident_kernel<T, kConfigs[I].dpl, kConfigs[I].lpi, METHOD, kConfigs[I].lpi == 1>...}};
}

template <typename T, int METHOD>
ResidentFn<T, METHOD> resident_lookup(ChainConfig cfg, int s) {
    static const auto t = make_resident_table<T, METHOD>(std::make_integer_sequence<int, kNumConfigs>{});
    const bool free_end = cfg.lpi == 1 && s == cfg.dpl;
    for (int i = 0; i < kNumConfigs; ++i)
        if (kConfigs[i].lpi == cfg.lpi && kConfigs[i].dpl == cfg.dpl) return free_end ? t.free_end[i] : t.f[i];
    return nullptr;
}

template <typename T, int METHOD>
osc_status launch_method(const ChainLaunch<T> &a, ChainConfig cfg, const ResidentRun<T> &r, hipStream_t st) {
    auto f = resident_lookup<T, METHOD>(cfg, a.s);
    if (!f) return fail(OSC_ENOTSUP, "no resident kernel for this chain configuration");
    const int bs = cfg.lpi == 128 ? 128 : kResidentThreads;
    const int64_t blocks = (a.batch * cfg.lpi + bs - 1) / bs;
    osc_status e = check_resident(reinterpret_cast<const void *>(f), blocks, bs);
    if (e) return e;
    hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(bs), 0, st, a, r);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace

template <typename T, int DPL, int LPI>
osc_status launch_vdp_layout(const VdpLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st) {
    void (*f)(VdpLaunch<T>, ResidentRun<T>) =
        a.f ? &vdp_resident_kernel<T, DPL, LPI, true> : &vdp_resident_kernel<T, DPL, LPI, false>;
    const int64_t blocks = (a.batch * LPI + kResidentThreads - 1) / kResidentThreads;
    osc_status e = check_resident(reinterpret_cast<const void *>(f), blocks, kResidentThreads);
    if (e) return e;
    hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(kResidentThreads), 0, st, a, r);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T>
int64_t chain_resident_blocks(const ChainLaunch<T> &a, ChainConfig cfg) {
    const int bs = cfg.lpi == 128 ? 128 : kResidentThreads;
    return (a.batch * cfg.lpi + bs - 1) / bs;
}

template <typename T>
osc_status chain_resident_launch(const ChainLaunch<T> &a, int method, ChainConfig cfg, const ResidentRun<T> &r,
                                 hipStream_t st) {
    if ((long)cfg.lpi * cfg.dpl < a.s) return fail(OSC_EINVAL, "chain configuration too small for s");
    if (a.batch == 0) return fail(OSC_EINVAL, "resident stepping needs at least one instance");
    return method == OSC_RK4 ? launch_method<T, OSC_RK4>(a, cfg, r, st) : launch_method<T, OSC_VERLET>(a, cfg, r, st);
}

template <typename T>
int64_t driven_resident_blocks(const DrivenLaunch<T> &a) {
    int dpl = 0, lpi = 0;
    if (!driven_regs_layout(a.s, &dpl, &lpi)) return 0;
    return (a.batch * lpi + kResidentThreads - 1) / kResidentThreads;
}

template <typename T>
osc_status driven_resident_launch(const DrivenLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st) {
    if (a.batch == 0) return fail(OSC_EINVAL, "resident stepping needs at least one instance");
    const int s = a.s;
    if (s <= 1) return launch_driven_layout<T, 1, 1>(a, r, st);
    if (s <= 2) return launch_driven_layout<T, 2, 1>(a, r, st);
    if (s <= 4) return launch_driven_layout<T, 4, 1>(a, r, st);
    if (s <= 8) return launch_driven_layout<T, 8, 1>(a, r, st);
    if (s <= 64) return launch_driven_layout<T, 1, 64>(a, r, st);
    if (s <= 128) return launch_driven_layout<T, 2, 64>(a, r, st);
    if (s <= 256) return launch_driven_layout<T, 4, 64>(a, r, st);
    if (s <= 512) return launch_driven_layout<T, 8, 64>(a, r, st);
    if (s <= 1024) return launch_driven_layout<T, 16, 64>(a, r, st);
    return fail(OSC_ENOTSUP, "resident stepping of damped or driven chains takes s <= 1024");
}

template <typename T>
int64_t vdp_resident_blocks(const VdpLaunch<T> &a) {
    int dpl = 0, lpi = 0;
    if (!driven_regs_layout(a.s, &dpl, &lpi)) return 0;   // the same layouts
    return (a.batch * lpi + kResidentThreads - 1) / kResidentThreads;
}

template <typename T>
osc_status vdp_resident_launch(const VdpLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st) {
    if (a.batch == 0) return fail(OSC_EINVAL, "resident stepping needs at least one instance");
    const int s = a.s;
    if (s <= 1) return launch_vdp_layout<T, 1, 1>(a, r, st);
    if (s <= 2) return launch_vdp_layout<T, 2, 1>(a, r, st);
    if (s <= 4) return launch_vdp_layout<T, 4, 1>(a, r, st);
    if (s <= 8) return launch_vdp_layout<T, 8, 1>(a, r, st);
    if (s <= 64) return launch_vdp_layout<T, 1, 64>(a, r, st);
    if (s <= 128) return launch_vdp_layout<T, 2, 64>(a, r, st);
    if (s <= 256) return launch_vdp_layout<T, 4, 64>(a, r, st);
    if (s <= 512) return launch_vdp_layout<T, 8, 64>(a, r, st);
    if (s <= 1024) return launch_vdp_layout<T, 16, 64>(a, r, st);
    return fail(OSC_ENOTSUP, "resident stepping of Van der Pol chains takes s <= 1024");
}

template int64_t vdp_resident_blocks<float>(const VdpLaunch<float> &);
template int64_t vdp_resident_blocks<double>(const VdpLaunch<double> &);
template osc_status vdp_resident_launch<float>(const VdpLaunch<float> &, const ResidentRun<float> &, hipStream_t);
template osc_status vdp_resident_launch<double>(const VdpLaunch<double> &, const ResidentRun<double> &, hipStream_t);
template int64_t driven_resident_blocks<float>(const DrivenLaunch<float> &);
template int64_t driven_resident_blocks<double>(const DrivenLaunch<double> &);
template osc_status driven_resident_launch<float>(const DrivenLaunch<float> &, const ResidentRun<float> &,
                                                  hipStream_t);
template osc_status driven_resident_launch<double>(const DrivenLaunch<double> &, const ResidentRun<double> &,
                                                   hipStream_t);
template int64_t chain_resident_blocks<float>(const ChainLaunch<float> &, ChainConfig);
template int64_t chain_resident_blocks<double>(const ChainLaunch<double> &, ChainConfig);
template osc_status chain_resident_launch<float>(const ChainLaunch<float> &, int, ChainConfig,
                                                 const ResidentRun<float> &, hipStream_t);
template osc_status chain_resident_launch<double>(const ChainLaunch<double> &, int, ChainConfig,
                                                  const ResidentRun<double> &, hipStream_t);

}  // namespace osc
