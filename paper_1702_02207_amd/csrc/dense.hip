// Dense systems of eq. (1): the scaled operator, the stability bound, FP64
// energy, and a generic (VALU) integrator with one workgroup per instance.
// (A = M^-1 K itself is formed in FP64 by the blocked Cholesky path.)
//
// Scaled operator for the integrators: B = h^2 A, stored
// column-major (Bc[j*s + i] = B_ij) so that the lanes of a wave, which own
// consecutive rows, read consecutive addresses.  FP32 keeps B as hi + lo.
//
// Integration uses the same scaled-time arithmetic as the chain kernels:
// RK4 as its exact linear Taylor form (P = Bx, Q = Bw, P2 = BP, Q2 = BQ;
// dx = w - P/2 - Q/6 + P2/24, dw = -P - Q/2 + P2/6 + Q2/24) and Verlet as
// leapfrog on the half-step velocity; FP32 state is compensated and only
// B x uses the low coefficient part.

#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

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

template <int THREADS>
__device__ double block_sum(double v, double *scratch) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < THREADS / 64; ++i) t += scratch[i];
    return t;
}

__device__ __forceinline__ void atomic_max_pos(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr), __double_as_longlong(v));
}

// Scaled operator B = h^2 A, column-major (FP32: hi + lo), one 64x64 tile per
// workgroup, transposed through LDS so that both the row-major read of A and
// the column-major write of B are coalesced.
template <typename T>
__global__ void __launch_bounds__(256) dense_prepare_kernel(int s, const double *__restrict__ A, size_t astride,
                                                            const double *__restrict__ dt, T *Bh, T *Bl,
                                                            size_t bstride, int tiles, int *bad) {
    __shared__ double t[64][65];
    const int64_t sys = blockIdx.x / ((int64_t)tiles * tiles);
    const int tile = (int)(blockIdx.x % ((int64_t)tiles * tiles));
    const int i0 = (tile / tiles) * 64, j0 = (tile % tiles) * 64;
    const double h = dt[sys];
    A += sys * astride;
    bool fine = h > 0.0 && __builtin_isfinite(h);
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int i = idx / 64, j = idx % 64;
        double b = 0.0;
        if (i0 + i < s && j0 + j < s) {
            b = h * h * A[(size_t)(i0 + i) * s + j0 + j];
            fine = fine && __builtin_isfinite(b);
        }
        t[i][j] = b;
    }
    if (!fine) atomicOr(bad, 1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int j = idx / 64, i = idx % 64;
        if (i0 + i < s && j0 + j < s) {
            const double b = t[i][j];
            const size_t o = sys * bstride + (size_t)(j0 + j) * s + i0 + i;
            Bh[o] = (T)b;
            if constexpr (std::is_same<T, float>::value) Bl[o] = (T)(b - (double)Bh[o]);
        }
    }
}

// Row-sum bound theta^2 <= max_i h^2 sum_j |A_ij| (every eigenvalue is
// bounded by any induced norm): one wave per row, each lane summing a fixed
// strided subset in order, then a fixed butterfly, so the bound is the same
// on every run.
__global__ void __launch_bounds__(256) dense_rowsum_kernel(int s, int64_t nsys, const double *__restrict__ A,
                                                           size_t astride, const double *__restrict__ dt,
                                                           double *theta_bound) {
    const int lane = threadIdx.x % 64;
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int64_t sys = row / s;
    const int i = (int)(row % s);
    if (sys >= nsys) return;   // whole waves only: the row index is wave-uniform
    const double h = dt[sys];
    const double *a = A + sys * astride + (size_t)i * s;
    double acc = 0.0;
    for (int j = lane; j < s; j += 64) acc += fabs(h * h * a[j]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) atomic_max_pos(theta_bound + sys, sqrt(acc));
}

// Power iteration for lambda_max of A^T (same spectrum as A), one workgroup;
// writes h * sqrt(lambda) into theta.
__global__ void __launch_bounds__(1024) power_kernel(int s, const double *__restrict__ A, double h, int iters,
                                                     double *theta) {
    extern __shared__ double sm[];
    double *v = sm, *u = sm + s;
    __shared__ double scratch[16];
    for (int i = threadIdx.x; i < s; i += 1024) v[i] = 1.0 + 0.001 * (i % 7);
    __syncthreads();
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        double nrm = 0.0, dot = 0.0;
        for (int j = threadIdx.x; j < s; j += 1024) {
            double acc = 0.0;
            for (int i = 0; i < s; ++i) acc += A[(size_t)i * s + j] * v[i];
            u[j] = acc;
            nrm += acc * acc;
            dot += acc * v[j];
        }
        nrm = block_sum<1024>(nrm, scratch);
        dot = block_sum<1024>(dot, scratch);
        double vv = 0.0;
        for (int j = threadIdx.x; j < s; j += 1024) vv += v[j] * v[j];
        vv = block_sum<1024>(vv, scratch);
        lam = dot / vv;
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        __syncthreads();
        for (int j = threadIdx.x; j < s; j += 1024) v[j] = u[j] * inv;
        __syncthreads();
    }
    if (threadIdx.x == 0) *theta = h * sqrt(lam > 0.0 ? lam : 0.0);
}

// ------------------------------------------------------------------- energy
// E = 1/2 v^T M v + 1/2 x^T K x (M, K symmetric, so (M v)_i = sum_j M_ji v_j
// reads along rows of the lanes); shadow: Q = v^T M v + x^T K x - h^2/4 (Kx)^T (A x).
template <typename T>
__global__ void __launch_bounds__(256) dense_energy_kernel(int s, int shared, const double *__restrict__ M,
                                                           const double *__restrict__ K, const double *__restrict__ A,
                                                           const double *__restrict__ dt, const T *__restrict__ x,
                                                           const T *__restrict__ v, double *E, int shadow) {
    __shared__ double scratch[4];
    const int64_t b = blockIdx.x;
    const size_t ss = (size_t)s * s;
    const size_t mo = shared ? 0 : b * ss;
    const T *xb = x + b * s, *vb = v + b * s;
    double kin = 0.0, pot = 0.0, corr = 0.0;
    for (int i = threadIdx.x; i < s; i += 256) {
        double mv = 0.0, kx = 0.0, ax = 0.0;
        for (int j = 0; j < s; ++j) {
            mv += M[mo + (size_t)j * s + i] * (double)vb[j];
            kx += K[mo + (size_t)j * s + i] * (double)xb[j];
            if (shadow) ax += A[mo + (size_t)i * s + j] * (double)xb[j];
        }
        kin += (double)vb[i] * mv;
        pot += (double)xb[i] * kx;
        corr += kx * ax;
    }
    kin = block_sum<256>(kin, scratch);
    pot = block_sum<256>(pot, scratch);
    corr = block_sum<256>(corr, scratch);
    if (threadIdx.x == 0) {
        if (shadow) {
            const double h = dt[shared ? 0 : b];
            E[b] = kin + pot - 0.25 * h * h * corr;
        } else {
            E[b] = 0.5 * kin + 0.5 * pot;
        }
    }
}

// --------------------------------------------------------- generic integrator
// One workgroup per instance; lane t owns rows t, t + THREADS, ... (RPT rows).
// Operand vectors live in LDS; B streams from L2 (column-major, coalesced).
template <typename T, int METHOD, int THREADS, int RPT>
__device__ __forceinline__ void dense_vec_run(const DenseLaunch<T> &a, const int64_t b) {
    constexpr bool COMP = std::is_same<T, float>::value;
    extern __shared__ unsigned char smem_raw[];
    T *su = reinterpret_cast<T *>(smem_raw);   // operand 1 (x or P)
    T *sv = su + a.s;                          // operand 2 (w or Q)
    const int s = a.s;
    const size_t ss = (size_t)s * s;
    const T *Bh = a.Bh + (a.shared ? 0 : b * ss);
    const T *Bl = COMP ? a.Bl + (a.shared ? 0 : b * ss) : nullptr;
    const double h = a.h[a.shared ? 0 : b];
    const double invh = 1.0 / h;
    const size_t base = (size_t)b * s;
    const size_t plane = (size_t)a.batch * s;

    T x[RPT], xl[RPT], w[RPT], wl[RPT], P[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = threadIdx.x + r * THREADS;
        const bool v = i < s;
        if (a.load_mode == LOAD_USER) {
            x[r] = v ? a.x0[base + i] : T(0);
            xl[r] = T(0);
            const double wd = v ? h * (double)a.v0[base + i] : 0.0;
            w[r] = (T)wd;
            wl[r] = COMP ? (T)(wd - (double)w[r]) : T(0);
        } else {
            x[r] = v ? a.state[base + i] : T(0);
            xl[r] = v ? a.state[plane + base + i] : T(0);
            w[r] = v ? a.state[2 * plane + base + i] : T(0);
            wl[r] = v ? a.state[3 * plane + base + i] : T(0);
        }
        P[r] = T(0);
    }

    // P = B x with split coefficients
    auto bx = [&]() {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = threadIdx.x + r * THREADS;
            if (i < s) su[i] = x[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = threadIdx.x + r * THREADS;
            if (i >= s) continue;
            T acc = T(0), accl = T(0);
            for (int j = 0; j < s; ++j) {
                const T u = su[j];
                acc = fmat(Bh[(size_t)j * s + i], u, acc);
                if constexpr (COMP) accl = fmat(Bl[(size_t)j * s + i], u, accl);
            }
            P[r] = acc + accl;
        }
    };

    if constexpr (METHOD == OSC_VERLET) {
        bx();
        if (a.load_mode == LOAD_USER) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) comp_add(w[r], wl[r], T(-0.5) * P[r]);
        }
    }
    auto vel = [&](int r) -> double {
        double wv = (double)w[r] + (double)wl[r];
        if constexpr (METHOD == OSC_VERLET) wv += 0.5 * (double)P[r];
        return wv * invh;
    };
    const bool untouched = a.load_mode == LOAD_USER;
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = threadIdx.x + r * THREADS;
            if (i >= s) continue;
            if (a.xf) a.xf[fo + base + i] = initial ? a.x0[base + i] : (T)((double)x[r] + (double)xl[r]);
            if (a.vf) a.vf[fo + base + i] = initial ? a.v0[base + i] : (T)vel(r);
        }
    };

    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    const int64_t stride = a.out_stride;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    while (n < nend) {
        int64_t stop = nend;
        if (stride > 0) {
            const int64_t nf = (n / stride + 1) * stride;
            stop = nf < stop ? nf : stop;
        }
        for (int64_t it = n; it < stop; ++it) {
            if constexpr (METHOD == OSC_RK4) {
                T Q[RPT];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = threadIdx.x + r * THREADS;
                    if (i < s) {
                        su[i] = x[r];
                        sv[i] = w[r];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = threadIdx.x + r * THREADS;
                    T ap = T(0), apl = T(0), aq = T(0);
                    if (i < s) {
                        for (int j = 0; j < s; ++j) {
                            const T bh = Bh[(size_t)j * s + i];
                            ap = fmat(bh, su[j], ap);
                            aq = fmat(bh, sv[j], aq);
                            if constexpr (COMP) apl = fmat(Bl[(size_t)j * s + i], su[j], apl);
                        }
                    }
                    P[r] = ap + apl;
                    Q[r] = aq;
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = threadIdx.x + r * THREADS;
                    if (i < s) {
                        su[i] = P[r];
                        sv[i] = Q[r];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = threadIdx.x + r * THREADS;
                    if (i >= s) continue;
                    T p2 = T(0), q2 = T(0);
                    for (int j = 0; j < s; ++j) {
                        const T bh = Bh[(size_t)j * s + i];
                        p2 = fmat(bh, su[j], p2);
                        q2 = fmat(bh, sv[j], q2);
                    }
                    T yx, yw;
                    rk4_increments(w[r], P[r], Q[r], p2, q2, yx, yw);
                    comp_add(x[r], xl[r], yx);
                    comp_add(w[r], wl[r], yw);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r) comp_add(x[r], xl[r], w[r]);
                bx();
#pragma unroll
                for (int r = 0; r < RPT; ++r) comp_add(w[r], wl[r], -P[r]);
            }
        }
        n = stop;
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }
    const bool copy_input = untouched && a.nsteps == 0;
    bool ok = true;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = threadIdx.x + r * THREADS;
        if (i >= s) continue;
        ok = ok && __builtin_isfinite(x[r]) && __builtin_isfinite(w[r]);
        if (a.store_mode & STORE_STATE) {
            a.state[base + i] = x[r];
            a.state[plane + base + i] = xl[r];
            a.state[2 * plane + base + i] = w[r];
            a.state[3 * plane + base + i] = wl[r];
        }
        if (a.store_mode & STORE_USER) {
            if (a.xe) a.xe[base + i] = copy_input ? a.x0[base + i] : (T)((double)x[r] + (double)xl[r]);
            if (a.ve) a.ve[base + i] = copy_input ? a.v0[base + i] : (T)vel(r);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

template <typename T, int METHOD, int THREADS, int RPT>
__global__ void __launch_bounds__(THREADS) dense_vec_kernel(DenseLaunch<T> a) {
    dense_vec_run<T, METHOD, THREADS, RPT>(a, blockIdx.x);
}

template <typename T, int METHOD, int THREADS, int RPT>
__global__ void __launch_bounds__(THREADS) dense_items_kernel(const DenseItem<T> *__restrict__ items) {
    const DenseLaunch<T> a = items[blockIdx.x].L;
    dense_vec_run<T, METHOD, THREADS, RPT>(a, items[blockIdx.x].b);
}

template <typename T, int METHOD, int THREADS, int RPT>
void launch_items(const DenseItem<T> *items, int64_t n, int smax, hipStream_t st) {
    const size_t lds = 2 * (size_t)smax * sizeof(T);
    hipLaunchKernelGGL((dense_items_kernel<T, METHOD, THREADS, RPT>), dim3((unsigned)n), dim3(THREADS), lds, st,
                       items);
}

template <typename T, int METHOD>
osc_status launch_items_m(const DenseItem<T> *items, int64_t n, int smax, hipStream_t st) {
    switch (dense_vec_bucket(smax)) {
        case 0: launch_items<T, METHOD, 64, 1>(items, n, smax, st); break;
        case 1: launch_items<T, METHOD, 256, 1>(items, n, smax, st); break;
        case 2: launch_items<T, METHOD, 256, 2>(items, n, smax, st); break;
        case 3: launch_items<T, METHOD, 256, 4>(items, n, smax, st); break;
        case 4: launch_items<T, METHOD, 256, 8>(items, n, smax, st); break;
        default: return fail(OSC_ENOTSUP, "dense systems support s <= 2048");
    }
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T, int METHOD, int THREADS, int RPT>
void launch_vec(const DenseLaunch<T> &a, hipStream_t st) {
    const size_t lds = 2 * (size_t)a.s * sizeof(T);
    hipLaunchKernelGGL((dense_vec_kernel<T, METHOD, THREADS, RPT>), dim3((unsigned)a.batch), dim3(THREADS), lds, st,
                       a);
}

template <typename T, int METHOD>
osc_status launch_vec_m(const DenseLaunch<T> &a, hipStream_t st) {
    if (a.s <= 64) launch_vec<T, METHOD, 64, 1>(a, st);
    else if (a.s <= 256) launch_vec<T, METHOD, 256, 1>(a, st);
    else if (a.s <= 512) launch_vec<T, METHOD, 256, 2>(a, st);
    else if (a.s <= 1024) launch_vec<T, METHOD, 256, 4>(a, st);
    else if (a.s <= 2048) launch_vec<T, METHOD, 256, 8>(a, st);
    else return fail(OSC_ENOTSUP, "dense systems support s <= 2048");
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace

int dense_vec_bucket(int s) {
    if (s <= 64) return 0;
    if (s <= 256) return 1;
    if (s <= 512) return 2;
    if (s <= 1024) return 3;
    if (s <= 2048) return 4;
    return -1;
}

template <typename T>
osc_status dense_launch_items(const DenseItem<T> *items, int64_t nitems, int smax, int method, hipStream_t st) {
    if (nitems == 0) return OSC_OK;
    if (nitems > 0x7fffffff) return fail(OSC_EINVAL, "work list too long for one launch");
    return method == OSC_RK4 ? launch_items_m<T, OSC_RK4>(items, nitems, smax, st)
                             : launch_items_m<T, OSC_VERLET>(items, nitems, smax, st);
}
template osc_status dense_launch_items<float>(const DenseItem<float> *, int64_t, int, int, hipStream_t);
template osc_status dense_launch_items<double>(const DenseItem<double> *, int64_t, int, int, hipStream_t);

// ------------------------------------------------------------- host helpers

template <typename T>
osc_status dense_prepare(int s, int64_t nsys, const double *A, const double *dt, T *Bh, T *Bl, double *theta,
                         int *bad, hipStream_t st) {
    if (nsys == 0) return OSC_OK;
    const size_t ss = (size_t)s * s;
    const int tiles = (s + 63) / 64;
    const int64_t blocks = nsys * tiles * tiles;
    const int64_t rows = nsys * s;
    if (blocks > 0x7fffffff || (rows + 3) / 4 > 0x7fffffff)
        return fail(OSC_EINVAL, "too many systems for one preparation launch");
    hipLaunchKernelGGL((dense_prepare_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, s, A, ss, dt, Bh, Bl, ss,
                       tiles, bad);
    OSC_HIP(hipGetLastError());
    hipLaunchKernelGGL(dense_rowsum_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, s, nsys, A, ss, dt,
                       theta);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

osc_status dense_power_theta(int s, const double *A, double h, double *theta, hipStream_t st) {
    hipLaunchKernelGGL(power_kernel, dim3(1), dim3(1024), 2 * (size_t)s * sizeof(double), st, s, A, h, 200, theta);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T>
osc_status dense_energy(int64_t batch, int s, int shared, const double *M, const double *K, const double *A,
                        const double *dt, const T *x, const T *v, double *E, bool shadow, hipStream_t st) {
    if (batch == 0) return OSC_OK;
    hipLaunchKernelGGL((dense_energy_kernel<T>), dim3((unsigned)batch), dim3(256), 0, st, s, shared, M, K, A, dt, x,
                       v, E, shadow ? 1 : 0);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T>
osc_status dense_launch_vec(const DenseLaunch<T> &a, int method, hipStream_t st) {
    if (a.batch == 0) return OSC_OK;
    if (a.batch > 0x7fffffff) return fail(OSC_EINVAL, "batch too large for one launch");
    return method == OSC_RK4 ? launch_vec_m<T, OSC_RK4>(a, st) : launch_vec_m<T, OSC_VERLET>(a, st);
}

template osc_status dense_prepare<float>(int, int64_t, const double *, const double *, float *, float *, double *,
                                         int *, hipStream_t);
template osc_status dense_prepare<double>(int, int64_t, const double *, const double *, double *, double *,
                                          double *, int *, hipStream_t);
template osc_status dense_energy<float>(int64_t, int, int, const double *, const double *, const double *,
                                        const double *, const float *, const float *, double *, bool, hipStream_t);
template osc_status dense_energy<double>(int64_t, int, int, const double *, const double *, const double *,
                                         const double *, const double *, const double *, double *, bool,
                                         hipStream_t);
template osc_status dense_launch_vec<float>(const DenseLaunch<float> &, int, hipStream_t);
template osc_status dense_launch_vec<double>(const DenseLaunch<double> &, int, hipStream_t);

}  // namespace osc
