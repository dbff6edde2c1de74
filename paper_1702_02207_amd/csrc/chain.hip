// Launchers of the chain integrator (chain_run.h): one launch per run or per
// chunk of a run, work lists for the server, and the one-step-per-launch
// baseline.

#include <cstdint>
#include <type_traits>

#include "chain_run.h"

namespace osc {
namespace {

template <typename T, int DPL, int LPI, int METHOD, bool FREE>
__global__ void __launch_bounds__(256) chain_kernel(ChainLaunch<T> a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    chain_run<T, DPL, LPI, METHOD, FREE>(a, g / LPI, (int)(g % LPI));
}

// Work list: lane group i integrates items[i] (an instance of any launch
// whose s fits the layout; step ranges may differ between items).
template <typename T, int DPL, int LPI, int METHOD>
__global__ void __launch_bounds__(256) chain_items_kernel(const ChainItem<T> *__restrict__ items, int64_t nitems) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = g / LPI;
    if (i >= nitems) return;   // whole groups only: LPI divides the workgroup
    const ChainLaunch<T> a = items[i].L;
    chain_run<T, DPL, LPI, METHOD>(a, items[i].b, (int)(g % LPI));
}


template <typename T, int METHOD>
using KernelFn = void (*)(ChainLaunch<T>);
template <typename T, int METHOD>
using ItemsFn = void (*)(const ChainItem<T> *, int64_t);

template <typename T, int METHOD, int... I>
constexpr auto make_table(std::integer_sequence<int, I...>) {
    struct Table {
        KernelFn<T, METHOD> f[sizeof...(I)];
        KernelFn<T, METHOD> free_end[sizeof...(I)];   // LPI == 1 layouts with s == DPL
        ItemsFn<T, METHOD> g[sizeof...(I)];
    };
    return Table{{&chain_kernel<T, kConfigs[I].dpl, kConfigs[I].lpi, METHOD, false>...},
                 {&chain_kernel<T, kConfigs[I].dpl, kConfigs[I].lpi, METHOD, kConfigs[I].lpi == 1>...},
                 {&chain_items_kernel<T, kConfigs[I].dpl, kConfigs[I].lpi, METHOD>...}};
}

template <typename T, int METHOD>
const auto &table() {
    static const auto t = make_table<T, METHOD>(std::make_integer_sequence<int, kNumConfigs>{});
    return t;
}

template <typename T, int METHOD>
KernelFn<T, METHOD> lookup(ChainConfig cfg, int s) {
    const bool free_end = cfg.lpi == 1 && s == cfg.dpl;
    for (int i = 0; i < kNumConfigs; ++i)
        if (kConfigs[i].lpi == cfg.lpi && kConfigs[i].dpl == cfg.dpl)
            return free_end ? table<T, METHOD>().free_end[i] : table<T, METHOD>().f[i];
    return nullptr;
}

template <typename T, int METHOD>
ItemsFn<T, METHOD> lookup_items(ChainConfig cfg) {
    for (int i = 0; i < kNumConfigs; ++i)
        if (kConfigs[i].lpi == cfg.lpi && kConfigs[i].dpl == cfg.dpl) return table<T, METHOD>().g[i];
    return nullptr;
}

}  // namespace

int chain_num_configs() { return kNumConfigs; }
ChainConfig chain_config_at(int i) { return ChainConfig{kConfigs[i].lpi, kConfigs[i].dpl}; }

ChainConfig chain_pick_config(int s) {
    if (s <= 8) return ChainConfig{1, s};
    // smallest capacity >= s; among equal capacity prefer more DOFs per lane
    ChainConfig best{0, 0};
    long best_cap = 0;
    for (int i = 0; i < kNumConfigs; ++i) {
        const long cap = (long)kConfigs[i].lpi * kConfigs[i].dpl;
        if (cap < s || kConfigs[i].lpi == 1) continue;
        if (best.lpi == 0 || cap < best_cap || (cap == best_cap && kConfigs[i].dpl > best.dpl)) {
            best = ChainConfig{kConfigs[i].lpi, kConfigs[i].dpl};
            best_cap = cap;
        }
    }
    return best;
}

// Threads per workgroup: 256, except for instances spanning two waves, which
// take a workgroup each (their halo exchange synchronises the workgroup, and
// work-list items differ in their step counts).
static int block_threads(ChainConfig cfg) { return cfg.lpi == 128 ? 128 : 256; }

template <typename T>
osc_status chain_launch(const ChainLaunch<T> &a, int method, ChainConfig cfg, hipStream_t st) {
    if ((long)cfg.lpi * cfg.dpl < a.s)
        return fail(OSC_EINVAL, "chain configuration too small for s");
    if (a.batch == 0) return OSC_OK;
    const int bs = block_threads(cfg);
    const int64_t threads = a.batch * cfg.lpi;
    const int64_t blocks = (threads + bs - 1) / bs;
    if (blocks > 0x7fffffff) return fail(OSC_EINVAL, "batch too large for one launch");
    if (method == OSC_RK4) {
        auto f = lookup<T, OSC_RK4>(cfg, a.s);
        if (!f) return fail(OSC_ENOTSUP, "no chain kernel for this configuration");
        hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(bs), 0, st, a);
    } else {
        auto f = lookup<T, OSC_VERLET>(cfg, a.s);
        if (!f) return fail(OSC_ENOTSUP, "no chain kernel for this configuration");
        hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(bs), 0, st, a);
    }
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template osc_status chain_launch<float>(const ChainLaunch<float> &, int, ChainConfig, hipStream_t);
template osc_status chain_launch<double>(const ChainLaunch<double> &, int, ChainConfig, hipStream_t);

template <typename T>
osc_status chain_launch_items(const ChainItem<T> *items, int64_t nitems, int method, ChainConfig cfg,
                              hipStream_t st) {
    if (nitems == 0) return OSC_OK;
    const int bs = block_threads(cfg);
    const int64_t blocks = (nitems * cfg.lpi + bs - 1) / bs;
    if (blocks > 0x7fffffff) return fail(OSC_EINVAL, "work list too long for one launch");
    if (method == OSC_RK4) {
        auto f = lookup_items<T, OSC_RK4>(cfg);
        if (!f) return fail(OSC_ENOTSUP, "no chain kernel for this configuration");
        hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(bs), 0, st, items, nitems);
    } else {
        auto f = lookup_items<T, OSC_VERLET>(cfg);
        if (!f) return fail(OSC_ENOTSUP, "no chain kernel for this configuration");
        hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(bs), 0, st, items, nitems);
    }
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}
template osc_status chain_launch_items<float>(const ChainItem<float> *, int64_t, int, ChainConfig, hipStream_t);
template osc_status chain_launch_items<double>(const ChainItem<double> *, int64_t, int, ChainConfig, hipStream_t);

// --------------------------------------------------------------------------
// plain baseline: one instance, one step per launch, state in device memory
// --------------------------------------------------------------------------
namespace {

constexpr int kPlainThreads = 1024;
constexpr int kPlainMaxS = 2048;

// One time step of one instance.  Thread t owns DOFs t, t + 1024, ...;
// neighbours are exchanged through LDS.
template <typename T, int METHOD>
__global__ void __launch_bounds__(kPlainThreads) chain_plain_step(ChainLaunch<T> a, int64_t b) {
    constexpr bool COMP = std::is_same<T, float>::value;
    __shared__ T su[kPlainMaxS + 2];
    __shared__ T sv[kPlainMaxS + 2];
    const int s = a.s;
    const size_t plane = (size_t)a.batch * s;
    const size_t base = (size_t)b * s;
    T *X = a.state, *XL = a.state + plane, *W = a.state + 2 * plane, *WL = a.state + 3 * plane;

    auto coef = [&](int d, T &ch, T &rh, T &cl, T &rl) {
        ch = a.c.clh[base + d];
        rh = a.c.crh[base + d];
        cl = COMP ? a.c.cll[base + d] : T(0);
        rl = COMP ? a.c.crl[base + d] : T(0);
    };
    // (B u)_d from an LDS copy of u with su[0] = 0 (wall) and su[s+1] = 0
    auto bop = [&](const T *u, int d, T ch, T rh, T cl, T rl, bool lo) -> T {
        const T el = u[d + 1] - u[d];
        const T er = u[d + 2] - u[d + 1];
        if (lo) return fmat(ch, el, fmat(-rh, er, fmat(cl, el, -rl * er)));
        return fmat(ch, el, -rh * er);
    };

    if (threadIdx.x == 0) {
        su[0] = T(0);
        sv[0] = T(0);
        su[s + 1] = T(0);
        sv[s + 1] = T(0);
    }
    if constexpr (METHOD == OSC_RK4) {
        for (int d = threadIdx.x; d < s; d += kPlainThreads) {
            su[d + 1] = X[base + d];
            sv[d + 1] = W[base + d];
        }
        __syncthreads();
        T P[kPlainMaxS / kPlainThreads], Q[kPlainMaxS / kPlainThreads];
        int q = 0;
        for (int d = threadIdx.x; d < s; d += kPlainThreads, ++q) {
            T ch, rh, cl, rl;
            coef(d, ch, rh, cl, rl);
            P[q] = bop(su, d, ch, rh, cl, rl, COMP);
            Q[q] = bop(sv, d, ch, rh, cl, rl, false);
        }
        __syncthreads();
        q = 0;
        for (int d = threadIdx.x; d < s; d += kPlainThreads, ++q) {
            su[d + 1] = P[q];
            sv[d + 1] = Q[q];
        }
        __syncthreads();
        q = 0;
        for (int d = threadIdx.x; d < s; d += kPlainThreads, ++q) {
            T ch, rh, cl, rl;
            coef(d, ch, rh, cl, rl);
            const T P2 = bop(su, d, ch, rh, cl, rl, false);
            const T Q2 = bop(sv, d, ch, rh, cl, rl, false);
            T x = X[base + d], xl = XL[base + d], w = W[base + d], wl = WL[base + d];
            T yx, yw;
            rk4_increments(w, P[q], Q[q], P2, Q2, yx, yw);
            comp_add(x, xl, yx);
            comp_add(w, wl, yw);
            X[base + d] = x;
            XL[base + d] = xl;
            W[base + d] = w;
            WL[base + d] = wl;
        }
    } else {
        for (int d = threadIdx.x; d < s; d += kPlainThreads) {
            T x = X[base + d], xl = XL[base + d];
            comp_add(x, xl, W[base + d]);
            X[base + d] = x;
            XL[base + d] = xl;
            su[d + 1] = x;
        }
        __syncthreads();
        for (int d = threadIdx.x; d < s; d += kPlainThreads) {
            T ch, rh, cl, rl;
            coef(d, ch, rh, cl, rl);
            const T P = bop(su, d, ch, rh, cl, rl, COMP);
            T w = W[base + d], wl = WL[base + d];
            comp_add(w, wl, -P);
            W[base + d] = w;
            WL[base + d] = wl;
        }
    }
}

}  // namespace

template <typename T>
osc_status chain_plain(const ChainLaunch<T> &a, int method, hipStream_t st) {
    if (a.s > kPlainMaxS) return fail(OSC_ENOTSUP, "plain integrator supports s <= 2048");
    // convert the user state, run single steps, convert back
    ChainLaunch<T> conv = a;
    conv.nsteps = 0;
    conv.out_stride = 0;
    conv.load_mode = LOAD_USER;
    conv.store_mode = STORE_STATE;
    const ChainConfig cfg = chain_pick_config(a.s);
    osc_status r = chain_launch<T>(conv, method, cfg, st);
    if (r != OSC_OK) return r;
    const int threads = a.s < kPlainThreads ? ((a.s + 63) / 64) * 64 : kPlainThreads;
    for (int64_t b = 0; b < a.batch; ++b) {
        for (int64_t n = 0; n < a.nsteps; ++n) {
            if (method == OSC_RK4)
                hipLaunchKernelGGL((chain_plain_step<T, OSC_RK4>), dim3(1), dim3(threads), 0, st, a, b);
            else
                hipLaunchKernelGGL((chain_plain_step<T, OSC_VERLET>), dim3(1), dim3(threads), 0, st, a, b);
        }
        OSC_HIP(hipGetLastError());
    }
    conv.load_mode = LOAD_STATE;
    conv.store_mode = STORE_USER;
    conv.n0 = a.nsteps;
    return chain_launch<T>(conv, method, cfg, st);
}

template osc_status chain_plain<float>(const ChainLaunch<float> &, int, hipStream_t);
template osc_status chain_plain<double>(const ChainLaunch<double> &, int, hipStream_t);

}  // namespace osc
