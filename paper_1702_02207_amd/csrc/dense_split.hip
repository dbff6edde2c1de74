// Dense instances with large s, split over many workgroups.
//
// One workgroup cannot hold an s = 2048 operator (16 MB in FP32), and a few
// workgroups streaming it would use only a few compute units' share of the
// cache bandwidth.  Here every product is split two ways: rows over
// workgroups (64 rows each, one per lane) and the k dimension over G column
// groups of workgroups, and inside a workgroup over its 16 wavefronts.  The
// waves reduce through LDS; the column groups leave partial sums in global
// memory, which their consumers add in a fixed order, so results are
// reproducible and no workgroup ever waits for another: kernel boundaries are
// the only global synchronisation.  A device-side step counter lets the same
// launches be replayed (hipGraph) for every step.
//
// RK4 (exact linear Taylor form), three kernels per step:
//   products 1: partial P = B x (split coefficients), Q = B w;
//   products 2: P, Q of the group's columns summed over the groups, then
//               partial P2 = B P, Q2 = B Q;
//   update:     dx = w - P/2 - Q/6 + P2/24,  dw = -P - Q/2 + P2/6 + Q2/24.
// Verlet (kick-drift-kick, P_n = B x_n carried), three kernels per step:
//   kick-drift: w += -P_n/2, x += w;  product: partial P_{n+1} = B x_{n+1};
//   kick:       w += -P_{n+1}/2, carry P_{n+1}.
// FP32 state is compensated as in the other integrators.

#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kRows = 64;          // rows per workgroup (one per lane)
constexpr int kWaves = 16;         // wavefronts per workgroup, each a share of the group's columns
constexpr int kThreads = 64 * kWaves;
constexpr int kRowThreads = 64;    // per-row kernels: one wavefront per workgroup, many workgroups
enum { kP = 0, kQ = 1, kP2 = 2, kQ2 = 3 };

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

template <typename T>
__device__ __forceinline__ int group_cols(const DenseSplitLaunch<T> &a) {
    return (a.s + a.groups - 1) / a.groups;
}

// partial product q of instance b, column group g, row i
template <typename T>
__device__ __forceinline__ size_t part_at(const DenseSplitLaunch<T> &a, int q, int64_t b, int g, int i) {
    return (((size_t)q * a.batch + b) * a.groups + g) * a.s + i;
}

constexpr int kMaxGroups = 16;

// sum of partial product q over the column groups, in group order (all the
// loads are issued before the first add)
template <typename T>
__device__ __forceinline__ T part_sum(const DenseSplitLaunch<T> &a, int q, int64_t b, int i) {
    T v[kMaxGroups];
    const T *p = a.part + part_at(a, q, b, 0, i);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) v[g] = g < a.groups ? p[(size_t)g * a.s] : T(0);
    T acc = T(0);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) acc += v[g];
    return acc;
}

// Partial products of rows [r0, r0 + 64) over columns [c0, c1), the columns
// divided among the wavefronts and reduced through LDS.  Column j of the
// operands is u1[j - uoff], u2[j - uoff].  Returns (lane = row):
// y1 = Bh u1 (+ Bl u1 when LO), y2 = Bh u2.
// The wave's share of the group's columns: [k0, k1).
__device__ __forceinline__ void wave_cols(int c0, int c1, int &k0, int &k1) {
    const int wave = threadIdx.x >> 6;
    const int per = (c1 - c0 + kWaves - 1) / kWaves;
    k0 = c0 + wave * per;
    k1 = min(c1, k0 + per);
}

// The first (up to) eight operator high parts of the lane's row in the
// wave's columns, loaded ahead (their loads stay in flight while the caller
// prepares the operands: a workgroup barrier waits for LDS traffic only).
template <typename T>
__device__ __forceinline__ void first_cols(const T *Bh, int s, int r0, int c0, int c1, T (&pre)[8]) {
    const int row = r0 + (threadIdx.x & 63);
    int k0, k1;
    wave_cols(c0, c1, k0, k1);
#pragma unroll
    for (int q = 0; q < 8; ++q) pre[q] = (row < s && k0 + q < k1) ? Bh[(size_t)(k0 + q) * s + row] : T(0);
}

template <typename T, bool LO, bool TWO, bool PRE = false>
__device__ __forceinline__ void rows_product(const T *Bh, const T *Bl, int s, const T *u1, const T *u2, int uoff,
                                             int r0, int c0, int c1, T &y1, T &y2, T (*red)[kWaves][kRows],
                                             const T *pre = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = r0 + lane;
    int k0, k1;
    wave_cols(c0, c1, k0, k1);
    // eight independent partial sums per product keep several loads in flight
    T a1[8], a1l[8], a2[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a1[q] = a1l[q] = a2[q] = T(0);
    if (row < s) {
        int j = k0;
        if constexpr (PRE) {
            // the preloaded columns, in the order the loops below would take them
            if (k0 + 8 <= k1) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    a1[q] = fmat(pre[q], u1[k0 + q - uoff], a1[q]);
                    if constexpr (TWO) a2[q] = fmat(pre[q], u2[k0 + q - uoff], a2[q]);
                }
                j = k0 + 8;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (k0 + q < k1) {
                        a1[0] = fmat(pre[q], u1[k0 + q - uoff], a1[0]);
                        if constexpr (TWO) a2[0] = fmat(pre[q], u2[k0 + q - uoff], a2[0]);
                    }
                j = k1;
            }
        }
        for (; j + 8 <= k1; j += 8) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const T bh = Bh[(size_t)(j + q) * s + row];
                const T v1 = u1[j + q - uoff];
                a1[q] = fmat(bh, v1, a1[q]);
                if constexpr (LO) a1l[q] = fmat(Bl[(size_t)(j + q) * s + row], v1, a1l[q]);
                if constexpr (TWO) a2[q] = fmat(bh, u2[j + q - uoff], a2[q]);
            }
        }
        for (; j < k1; ++j) {
            const T bh = Bh[(size_t)j * s + row];
            const T v1 = u1[j - uoff];
            a1[0] = fmat(bh, v1, a1[0]);
            if constexpr (LO) a1l[0] = fmat(Bl[(size_t)j * s + row], v1, a1l[0]);
            if constexpr (TWO) a2[0] = fmat(bh, u2[j - uoff], a2[0]);
        }
    }
    const T s1 = ((a1[0] + a1[1]) + (a1[2] + a1[3])) + ((a1[4] + a1[5]) + (a1[6] + a1[7]));
    const T s1l = ((a1l[0] + a1l[1]) + (a1l[2] + a1l[3])) + ((a1l[4] + a1l[5]) + (a1l[6] + a1l[7]));
    const T s2 = ((a2[0] + a2[1]) + (a2[2] + a2[3])) + ((a2[4] + a2[5]) + (a2[6] + a2[7]));
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

// grid (row blocks, column groups, instances), kThreads threads.
// RK4: partial P = B x, Q = B w, and the step is counted (the update kernel
// of the same step reads the count).  Verlet: partial P = B x.
template <typename T, int METHOD>
__global__ void __launch_bounds__(kThreads) split_products1(DenseSplitLaunch<T> a) {
    __shared__ T red[2][kWaves][kRows];
    const int64_t b = blockIdx.z;
    const int g = blockIdx.y, s = a.s, cg = group_cols(a);
    const size_t ss = (size_t)s * s, plane = (size_t)a.batch * s, base = (size_t)b * s;
    const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
    const T *Bl = std::is_same<T, float>::value ? a.Bl + (a.shared ? 0 : b * ss) : nullptr;
    const int r0 = blockIdx.x * kRows, c0 = g * cg, c1 = min(s, c0 + cg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = r0 + lane;
    constexpr bool LO = std::is_same<T, float>::value;
    if (METHOD == OSC_RK4 && blockIdx.x == 0 && g == 0 && b == 0 && threadIdx.x == 0) *a.counter += 1;
    T y1, y2;
    if constexpr (METHOD == OSC_RK4)
        rows_product<T, LO, true>(Bh, Bl, s, a.state + base, a.state + 2 * plane + base, 0, r0, c0, c1, y1, y2,
                                  red);
    else
        rows_product<T, LO, false>(Bh, Bl, s, a.state + base, nullptr, 0, r0, c0, c1, y1, y2, red);
    if (wave == 0 && row < s) {
        a.part[part_at(a, kP, b, g, row)] = y1;
        if constexpr (METHOD == OSC_RK4) a.part[part_at(a, kQ, b, g, row)] = y2;
    }
}

// RK4: P and Q of the group's columns summed over the groups into LDS, then
// partial P2 = B P, Q2 = B Q (coefficient high parts).
template <typename T>
__global__ void __launch_bounds__(kThreads) split_products2(DenseSplitLaunch<T> a) {
    __shared__ T red[2][kWaves][kRows];
    extern __shared__ unsigned char dyn[];
    const int64_t b = blockIdx.z;
    const int g = blockIdx.y, s = a.s, cg = group_cols(a);
    T *sP = reinterpret_cast<T *>(dyn);
    T *sQ = sP + cg;
    const size_t ss = (size_t)s * s;
    const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
    const int r0 = blockIdx.x * kRows, c0 = g * cg, c1 = min(s, c0 + cg);
    T pre[8];
    first_cols(Bh, s, r0, c0, c1, pre);
    for (int t = threadIdx.x; t < c1 - c0; t += kThreads) {
        sP[t] = part_sum(a, kP, b, c0 + t);
        sQ[t] = part_sum(a, kQ, b, c0 + t);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = r0 + lane;
    T y1, y2;
    rows_product<T, false, true, true>(Bh, nullptr, s, sP, sQ, c0, r0, c0, c1, y1, y2, red, pre);
    if (wave == 0 && row < s) {
        a.part[part_at(a, kP2, b, g, row)] = y1;
        a.part[part_at(a, kQ2, b, g, row)] = y2;
    }
}

template <typename T>
__device__ __forceinline__ void write_frame_row(const DenseSplitLaunch<T> &a, int64_t n, size_t i, T x, T xl, T w,
                                               T wl, double h) {
    if (a.out_stride > 0 && n % a.out_stride == 0) {
        const size_t fo = (size_t)(n / a.out_stride) * ((size_t)a.batch * a.s);
        if (a.xf) a.xf[fo + i] = (T)((double)x + (double)xl);
        if (a.vf) a.vf[fo + i] = (T)(((double)w + (double)wl) / h);
    }
}

// grid (row blocks of 256, instances).  RK4: each row's update from the four
// summed products, and its frame.
template <typename T>
__global__ void __launch_bounds__(kRowThreads) split_update(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const int row = blockIdx.x * kRowThreads + threadIdx.x;
    if (row >= s) return;
    const size_t plane = (size_t)a.batch * s, i = (size_t)b * s + row;
    const int64_t n = *a.counter;   // steps completed after this one
    const double h = a.h[a.shared ? 0 : b];
    const T P = part_sum(a, kP, b, row), Q = part_sum(a, kQ, b, row);
    const T P2 = part_sum(a, kP2, b, row), Q2 = part_sum(a, kQ2, b, row);
    T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
    T yx, yw;
    rk4_increments(w, P, Q, P2, Q2, yx, yw);
    comp_add(x, xl, yx);
    comp_add(w, wl, yw);
    a.state[i] = x;
    a.state[plane + i] = xl;
    a.state[2 * plane + i] = w;
    a.state[3 * plane + i] = wl;
    write_frame_row(a, n, i, x, xl, w, wl, h);
}

// Verlet: half kick with the carried P_n, then drift; counts the step (the
// kick kernel of the same step reads the count).
template <typename T>
__global__ void __launch_bounds__(kRowThreads) split_kick_drift(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const int row = blockIdx.x * kRowThreads + threadIdx.x;
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) *a.counter += 1;   // the step being taken
    if (row >= s) return;
    const size_t plane = (size_t)a.batch * s, i = (size_t)b * s + row;
    T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
    comp_add(w, wl, T(-0.5) * a.P[i]);
    comp_add(x, xl, w);
    a.state[i] = x;
    a.state[plane + i] = xl;
    a.state[2 * plane + i] = w;
    a.state[3 * plane + i] = wl;
}

// Verlet: P_{n+1} summed over the groups and carried; with KICK the second
// half kick and the frame of step n+1.
template <typename T, bool KICK>
__global__ void __launch_bounds__(kRowThreads) split_kick(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const int row = blockIdx.x * kRowThreads + threadIdx.x;
    if (row >= s) return;
    const size_t plane = (size_t)a.batch * s, i = (size_t)b * s + row;
    const T P = part_sum(a, kP, b, row);
    a.P[i] = P;
    if constexpr (KICK) {
        const int64_t n = *a.counter;
        const double h = a.h[a.shared ? 0 : b];
        T w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
        comp_add(w, wl, T(-0.5) * P);
        a.state[2 * plane + i] = w;
        a.state[3 * plane + i] = wl;
        write_frame_row(a, n, i, a.state[i], a.state[plane + i], w, wl, h);
    }
}

// State from the caller's (x0, v0), frame 0 and the step counter.
template <typename T>
__global__ void __launch_bounds__(kRowThreads) split_load(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const int row = blockIdx.x * kRowThreads + threadIdx.x;
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) *a.counter = a.n0;
    if (row >= s) return;
    const size_t plane = (size_t)a.batch * s, i = (size_t)b * s + row;
    const double h = a.h[a.shared ? 0 : b];
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

template <typename T>
__global__ void __launch_bounds__(kRowThreads) split_store(DenseSplitLaunch<T> a) {
    const int64_t b = blockIdx.y;
    const int s = a.s;
    const int row = blockIdx.x * kRowThreads + threadIdx.x;
    if (row >= s) return;
    const size_t plane = (size_t)a.batch * s, i = (size_t)b * s + row;
    const double h = a.h[a.shared ? 0 : b];
    const T x = a.state[i], xl = a.state[plane + i], w = a.state[2 * plane + i], wl = a.state[3 * plane + i];
    const bool ok = __builtin_isfinite(x) && __builtin_isfinite(w);
    if (a.xe) a.xe[i] = (T)((double)x + (double)xl);
    if (a.ve) a.ve[i] = (T)(((double)w + (double)wl) / h);
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

struct Grids {
    dim3 prod, rows;
    size_t prod2_lds;
};

template <typename T>
Grids grids(const DenseSplitLaunch<T> &a) {
    Grids g;
    g.prod = dim3((a.s + kRows - 1) / kRows, (unsigned)a.groups, (unsigned)a.batch);
    g.rows = dim3((a.s + kRowThreads - 1) / kRowThreads, (unsigned)a.batch);
    g.prod2_lds = 2 * (size_t)((a.s + a.groups - 1) / a.groups) * sizeof(T);
    return g;
}

template <typename T, int METHOD>
void launch_step(const DenseSplitLaunch<T> &a, const Grids &g, hipStream_t st) {
    if constexpr (METHOD == OSC_RK4) {
        hipLaunchKernelGGL((split_products1<T, METHOD>), g.prod, dim3(kThreads), 0, st, a);
        hipLaunchKernelGGL((split_products2<T>), g.prod, dim3(kThreads), g.prod2_lds, st, a);
        hipLaunchKernelGGL((split_update<T>), g.rows, dim3(kRowThreads), 0, st, a);
    } else {
        hipLaunchKernelGGL((split_kick_drift<T>), g.rows, dim3(kRowThreads), 0, st, a);
        hipLaunchKernelGGL((split_products1<T, METHOD>), g.prod, dim3(kThreads), 0, st, a);
        hipLaunchKernelGGL((split_kick<T, true>), g.rows, dim3(kRowThreads), 0, st, a);
    }
}

template <typename T, int METHOD>
osc_status split_run_m(const DenseSplitLaunch<T> &a, hipStream_t st, hipGraphExec_t *graph, int64_t *graph_steps,
                       int64_t graph_chunk) {
    const Grids g = grids(a);
    if (a.load_mode == LOAD_USER) {
        hipLaunchKernelGGL((split_load<T>), g.rows, dim3(kRowThreads), 0, st, a);
        if constexpr (METHOD == OSC_VERLET) {
            // P_0 = B x_0, carried into the first kick
            hipLaunchKernelGGL((split_products1<T, METHOD>), g.prod, dim3(kThreads), 0, st, a);
            hipLaunchKernelGGL((split_kick<T, false>), g.rows, dim3(kRowThreads), 0, st, a);
        }
    }
    OSC_HIP(hipGetLastError());
    int64_t left = a.nsteps;
    // replay a captured chunk of steps while whole chunks remain
    if (graph && graph_chunk > 0 && left >= graph_chunk) {
        if (!*graph || *graph_steps != graph_chunk) {
            if (*graph) (void)hipGraphExecDestroy(*graph);
            *graph = nullptr;
            hipGraph_t gr = nullptr;
            OSC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int64_t k = 0; k < graph_chunk; ++k) launch_step<T, METHOD>(a, g, st);
            OSC_HIP(hipStreamEndCapture(st, &gr));
            hipError_t e = hipGraphInstantiate(graph, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return fail(OSC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            *graph_steps = graph_chunk;
        }
        while (left >= graph_chunk) {
            OSC_HIP(hipGraphLaunch(*graph, st));
            left -= graph_chunk;
        }
    }
    for (; left > 0; --left) launch_step<T, METHOD>(a, g, st);
    OSC_HIP(hipGetLastError());
    if (a.store_mode & STORE_USER) {
        hipLaunchKernelGGL((split_store<T>), g.rows, dim3(kRowThreads), 0, st, a);
        OSC_HIP(hipGetLastError());
    }
    return OSC_OK;
}

}  // namespace

int dense_split_groups(int s, int64_t batch) {
    // about two workgroups per compute unit, at least 64 columns per group
    const int64_t rows = (s + kRows - 1) / kRows;
    const int64_t want = (512 + rows * batch - 1) / (rows * batch);
    int64_t gmax = s / 64;
    gmax = gmax < 1 ? 1 : (gmax > kMaxGroups ? kMaxGroups : gmax);
    return (int)(want < 1 ? 1 : (want > gmax ? gmax : want));
}

size_t dense_split_scratch_elems(int s, int64_t batch) {
    // carried P, four partial-product planes per column group
    return (size_t)batch * s * (1 + 4 * (size_t)dense_split_groups(s, batch));
}

template <typename T>
osc_status dense_split_run(const DenseSplitLaunch<T> &a, int method, hipStream_t st, hipGraphExec_t *graph,
                           int64_t *graph_steps, int64_t graph_chunk) {
    if (a.batch == 0) return OSC_OK;
    if (a.batch > 65535) return fail(OSC_ENOTSUP, "split dense path takes at most 65535 instances per launch");
    if (a.groups != dense_split_groups(a.s, a.batch))
        return fail(OSC_EINVAL, "split dense path: column groups do not match the scratch layout");
    return method == OSC_RK4 ? split_run_m<T, OSC_RK4>(a, st, graph, graph_steps, graph_chunk)
                             : split_run_m<T, OSC_VERLET>(a, st, graph, graph_steps, graph_chunk);
}

template osc_status dense_split_run<float>(const DenseSplitLaunch<float> &, int, hipStream_t, hipGraphExec_t *,
                                           int64_t *, int64_t);
template osc_status dense_split_run<double>(const DenseSplitLaunch<double> &, int, hipStream_t, hipGraphExec_t *,
                                            int64_t *, int64_t);

}  // namespace osc
