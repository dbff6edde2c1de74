// Dense instances with large s, split over many workgroups.
//
// One workgroup cannot hold an s = 2048 operator (16 MB in FP32), and one
// workgroup streaming it would take hundreds of microseconds per step.  Here a
// time step is two kernels: rows are spread over workgroups (64 rows each) and
// the k dimension of every product over the workgroup's 16 wavefronts, which
// reduce their partial sums through LDS in a fixed order (results are
// reproducible).  The kernel boundary is the global synchronisation point
// between the products of a step, so no workgroup ever waits for another.  A device-side step counter lets the same two launches
// be replayed (hipGraph) for every step.
//
// RK4 (exact linear Taylor form): phase 1 forms P = B x (split coefficients)
// and Q = B w; phase 2 forms P2 = B P, Q2 = B Q and applies
//   dx = w - P/2 - Q/6 + P2/24,  dw = -P - Q/2 + P2/6 + Q2/24.
// Verlet (kick-drift-kick, P_n = B x_n carried): phase 1 kicks and drifts each
// row, w += -P_n/2, x += w; phase 2 forms P_{n+1} = B x_{n+1} and kicks again.
// FP32 state is compensated as in the other integrators.

#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kRows = 64;     // rows per workgroup (one per lane)
constexpr int kWaves = 16;    // k-split: 16 wavefronts each take 1/16 of the columns
constexpr int kThreads = 64 * kWaves;

template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    if constexpr (std::is_same<T, float>::value) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

template <typename T>
__device__ __forceinline__ void comp_add(T &hi, T &lo, T y) {
    if constexpr (std::is_same<T, float>::value) {
        y = y + lo;
        const T t = hi + y;
        lo = y - (t - hi);
        hi = t;
    } else {
        hi = hi + y;
    }
}

// Partial products of the rows [r0, r0 + 64) over this wave's k-range,
// reduced across the wavefronts.  Returns (for lane = row) up to three sums:
// y1 = Bh u1 (+ Bl u1 when lo), y2 = Bh u2.
template <typename T, bool LO, bool TWO>
__device__ __forceinline__ void rows_product(const DenseSplitLaunch<T> &a, const T *Bh, const T *Bl, const T *u1,
                                             const T *u2, int r0, T &y1, T &y2, T (*red)[kWaves][kRows]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = a.s;
    const int row = r0 + lane;
    const int kper = (s + kWaves - 1) / kWaves;
    const int k0 = wave * kper, k1 = min(s, k0 + kper);
    // four independent partial sums per product keep several loads in flight
    T a1[4] = {T(0), T(0), T(0), T(0)}, a1l[4] = {T(0), T(0), T(0), T(0)}, a2[4] = {T(0), T(0), T(0), T(0)};
    if (row < s) {
        int j = k0;
        for (; j + 4 <= k1; j += 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T bh = Bh[(size_t)(j + q) * s + row];
                const T v1 = u1[j + q];
                a1[q] = fmat(bh, v1, a1[q]);
                if constexpr (LO) a1l[q] = fmat(Bl[(size_t)(j + q) * s + row], v1, a1l[q]);
                if constexpr (TWO) a2[q] = fmat(bh, u2[j + q], a2[q]);
            }
        }
        for (; j < k1; ++j) {
            const T bh = Bh[(size_t)j * s + row];
            const T v1 = u1[j];
            a1[0] = fmat(bh, v1, a1[0]);
            if constexpr (LO) a1l[0] = fmat(Bl[(size_t)j * s + row], v1, a1l[0]);
            if constexpr (TWO) a2[0] = fmat(bh, u2[j], a2[0]);
        }
    }
    const T s1 = (a1[0] + a1[1]) + (a1[2] + a1[3]);
    const T s1l = (a1l[0] + a1l[1]) + (a1l[2] + a1l[3]);
    const T s2 = (a2[0] + a2[1]) + (a2[2] + a2[3]);
    red[0][wave][lane] = s1 + s1l;
    if constexpr (TWO) red[1][wave][lane] = s2;
    __syncthreads();
    y1 = T(0);
    y2 = T(0);
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
        y1 += red[0][v][lane];
        if constexpr (TWO) y2 += red[1][v][lane];
    }
}

// grid: (row blocks, instances); kThreads threads; only wave 0 writes results.
template <typename T, int METHOD>
__global__ void __launch_bounds__(kThreads) split_phase1(DenseSplitLaunch<T> a) {
    __shared__ T red[2][kWaves][kRows];
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const size_t ss = (size_t)s * s;
    const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
    const T *Bl = std::is_same<T, float>::value ? a.Bl + (a.shared ? 0 : b * ss) : nullptr;
    const size_t plane = (size_t)a.batch * s, base = (size_t)b * s;
    const int r0 = blockIdx.x * kRows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) *a.counter += 1;   // the step being taken
    if constexpr (METHOD == OSC_RK4) {
        T P, Q;
        rows_product<T, std::is_same<T, float>::value, true>(a, Bh, Bl, a.state + base, a.state + 2 * plane + base,
                                                             r0, P, Q, red);
        const int row = r0 + lane;
        if (wave == 0 && row < s) {
            a.P[base + row] = P;
            a.Q[base + row] = Q;
        }
    } else {
        // kick with the carried P_n, then drift (own rows only)
        const int row = r0 + threadIdx.x;
        if (threadIdx.x < kRows && row < s) {
            const size_t i = base + row;
            T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
            comp_add(w, wl, T(-0.5) * a.P[i]);
            comp_add(x, xl, w);
            a.state[i] = x;
            a.state[plane + i] = xl;
            a.state[2 * plane + i] = w;
            a.state[3 * plane + i] = wl;
        }
    }
}

template <typename T, int METHOD>
__global__ void __launch_bounds__(kThreads) split_phase2(DenseSplitLaunch<T> a) {
    __shared__ T red[2][kWaves][kRows];
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const size_t ss = (size_t)s * s;
    const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
    const T *Bl = std::is_same<T, float>::value ? a.Bl + (a.shared ? 0 : b * ss) : nullptr;
    const size_t plane = (size_t)a.batch * s, base = (size_t)b * s;
    const int r0 = blockIdx.x * kRows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = r0 + lane;
    const int64_t n = *a.counter;   // steps completed after this one
    const double h = a.h[a.shared ? 0 : b];
    if constexpr (METHOD == OSC_RK4) {
        T P2, Q2;
        rows_product<T, false, true>(a, Bh, Bl, a.P + base, a.Q + base, r0, P2, Q2, red);
        if (wave == 0 && row < s) {
            const size_t i = base + row;
            const T P = a.P[i], Q = a.Q[i];
            T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
            const T yx = fmat(T(1.0 / 24.0), P2, fmat(T(-1.0 / 6.0), Q, fmat(T(-0.5), P, w)));
            const T yw = fmat(T(1.0 / 24.0), Q2, fmat(T(1.0 / 6.0), P2, fmat(T(-0.5), Q, -P)));
            comp_add(x, xl, yx);
            comp_add(w, wl, yw);
            a.state[i] = x;
            a.state[plane + i] = xl;
            a.state[2 * plane + i] = w;
            a.state[3 * plane + i] = wl;
            if (a.out_stride > 0 && n % a.out_stride == 0) {
                const size_t fo = (size_t)(n / a.out_stride) * plane;
                if (a.xf) a.xf[fo + i] = (T)((double)x + (double)xl);
                if (a.vf) a.vf[fo + i] = (T)(((double)w + (double)wl) / h);
            }
        }
    } else {
        T P, unused;
        rows_product<T, std::is_same<T, float>::value, false>(a, Bh, Bl, a.state + base, nullptr, r0, P, unused, red);
        if (wave == 0 && row < s) {
            const size_t i = base + row;
            T w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
            comp_add(w, wl, T(-0.5) * P);
            a.state[2 * plane + i] = w;
            a.state[3 * plane + i] = wl;
            a.P[i] = P;
            if (a.out_stride > 0 && n % a.out_stride == 0) {
                const size_t fo = (size_t)(n / a.out_stride) * plane;
                if (a.xf) a.xf[fo + i] = (T)((double)a.state[i] + (double)a.state[plane + i]);
                if (a.vf) a.vf[fo + i] = (T)(((double)w + (double)wl) / h);
            }
        }
    }
}

// State from the caller's (x0, v0), frame 0, the step counter, and for Verlet
// the carried P_0 = B x_0.
template <typename T, int METHOD>
__global__ void __launch_bounds__(kThreads) split_load(DenseSplitLaunch<T> a) {
    __shared__ T red[2][kWaves][kRows];
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const size_t ss = (size_t)s * s;
    const size_t plane = (size_t)a.batch * s, base = (size_t)b * s;
    const int r0 = blockIdx.x * kRows;
    const double h = a.h[a.shared ? 0 : b];
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) *a.counter = a.n0;
    const int row = r0 + threadIdx.x;
    if (threadIdx.x < kRows && row < s) {
        const size_t i = base + row;
        const double wd = h * (double)a.v0[i];
        const T w = (T)wd;
        a.state[i] = a.x0[i];
        a.state[plane + i] = T(0);
        a.state[2 * plane + i] = w;
        a.state[3 * plane + i] = std::is_same<T, float>::value ? (T)(wd - (double)w) : T(0);
        if (a.out_stride > 0 && a.n0 % a.out_stride == 0) {
            const size_t fo = (size_t)(a.n0 / a.out_stride) * plane;
            if (a.xf) a.xf[fo + i] = a.x0[i];
            if (a.vf) a.vf[fo + i] = a.v0[i];
        }
    }
    if constexpr (METHOD == OSC_VERLET) {
        __syncthreads();
        const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
        const T *Bl = std::is_same<T, float>::value ? a.Bl + (a.shared ? 0 : b * ss) : nullptr;
        // this block's own rows of x were just written by this block, but the
        // product needs all rows: read them from the caller's x0 instead
        T P, unused;
        rows_product<T, std::is_same<T, float>::value, false>(a, Bh, Bl, a.x0 + base, nullptr, r0, P, unused, red);
        if ((threadIdx.x >> 6) == 0 && r0 + (threadIdx.x & 63) < s) a.P[base + r0 + (threadIdx.x & 63)] = P;
    }
}

template <typename T, int METHOD>
__global__ void split_store(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const size_t plane = (size_t)a.batch * s, base = (size_t)b * s;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= s) return;
    const size_t i = base + row;
    const double h = a.h[a.shared ? 0 : b];
    bool ok = true;
    const T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
    ok = __builtin_isfinite(x) && __builtin_isfinite(w);
    if (a.xe) a.xe[i] = (T)((double)x + (double)xl);
    if (a.ve) a.ve[i] = (T)(((double)w + (double)wl) / h);
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

template <typename T, int METHOD>
osc_status split_run_m(const DenseSplitLaunch<T> &a, hipStream_t st, hipGraphExec_t *graph, int64_t *graph_steps,
                       int64_t graph_chunk) {
    const dim3 grid((a.s + kRows - 1) / kRows, (unsigned)a.batch);
    const dim3 block(kThreads);
    if (a.load_mode == LOAD_USER) hipLaunchKernelGGL((split_load<T, METHOD>), grid, block, 0, st, a);
    OSC_HIP(hipGetLastError());
    int64_t left = a.nsteps;
    // replay a captured chunk of steps while whole chunks remain
    if (graph && graph_chunk > 0 && left >= graph_chunk) {
        if (!*graph || *graph_steps != graph_chunk) {
            if (*graph) (void)hipGraphExecDestroy(*graph);
            *graph = nullptr;
            hipGraph_t g = nullptr;
            OSC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int64_t k = 0; k < graph_chunk; ++k) {
                hipLaunchKernelGGL((split_phase1<T, METHOD>), grid, block, 0, st, a);
                hipLaunchKernelGGL((split_phase2<T, METHOD>), grid, block, 0, st, a);
            }
            OSC_HIP(hipStreamEndCapture(st, &g));
            hipError_t e = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(OSC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            *graph_steps = graph_chunk;
        }
        while (left >= graph_chunk) {
            OSC_HIP(hipGraphLaunch(*graph, st));
            left -= graph_chunk;
        }
    }
    for (; left > 0; --left) {
        hipLaunchKernelGGL((split_phase1<T, METHOD>), grid, block, 0, st, a);
        hipLaunchKernelGGL((split_phase2<T, METHOD>), grid, block, 0, st, a);
    }
    OSC_HIP(hipGetLastError());
    if (a.store_mode & STORE_USER) {
        const dim3 g2((a.s + 255) / 256, (unsigned)a.batch);
        hipLaunchKernelGGL((split_store<T, METHOD>), g2, dim3(256), 0, st, a);
        OSC_HIP(hipGetLastError());
    }
    return OSC_OK;
}

}  // namespace

template <typename T>
osc_status dense_split_run(const DenseSplitLaunch<T> &a, int method, hipStream_t st, hipGraphExec_t *graph,
                           int64_t *graph_steps, int64_t graph_chunk) {
    if (a.batch == 0) return OSC_OK;
    if (a.batch > 65535) return fail(OSC_ENOTSUP, "split dense path takes at most 65535 instances per launch");
    return method == OSC_RK4 ? split_run_m<T, OSC_RK4>(a, st, graph, graph_steps, graph_chunk)
                             : split_run_m<T, OSC_VERLET>(a, st, graph, graph_steps, graph_chunk);
}

template osc_status dense_split_run<float>(const DenseSplitLaunch<float> &, int, hipStream_t, hipGraphExec_t *,
                                           int64_t *, int64_t);
template osc_status dense_split_run<double>(const DenseSplitLaunch<double> &, int, hipStream_t, hipGraphExec_t *,
                                            int64_t *, int64_t);

}  // namespace osc
