// The integration schemes as matrices (propagator form).
//
// For eq. (1) the first-order system of section 3 is y' = L y with the
// constant matrix L = [[0, I], [-A, 0]], y = (x, v), so both schemes map y
// linearly.  Classic RK4 is y_{n+1} = P y_n with P the degree-4 Taylor
// polynomial of exp(hL); with B = h^2 A,
//   P = [[C, h S], [-(B - B^2/6)/h, C]],   C = I - B/2 + B^2/24,  S = I - B/6,
// and velocity Verlet (kick-drift-kick) has
//   P = [[I - B/2, h I], [-(B - B^2/4)/h, I - B/2]].
// k steps are P^k, formed here in FP64 by repeated squaring.  Uses:
//   * osc_propagator: P^k itself;
//   * frame jumps (OSC_CFG_PROPAGATOR = 1): the state advances from frame to
//     frame by one product with P^out_stride and over the rest of the run by
//     P^r, in FP64;
//   * per-step propagator (OSC_CFG_PROPAGATOR = 2, chains of s <= 2): every
//     step applies P - I, split into FP32 high and low parts, to the
//     compensated state, one lane per instance.
// Systems of s <= 2 keep P in registers, one lane per system; larger ones
// (up to s = 2048) form P^k and apply it by FP64 matrix-core products: the
// squarings and the frame jumps are plain GEMMs (row-major n x n by n x n,
// and batch x n by the transposed n x n), which run through rocBLAS's DGEMM
// with atomics off, so that a result does not depend on the run.

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include <rocblas/rocblas.h>

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kThreads = 256;

// ------------------------------------------------------------- one system
template <int S>
struct Mat {
    double e[S][S];
};

// A = M^-1 K of system `sys`: chains from masses and springs (spring 0 to
// the wall, spring i between bodies i-1 and i, free last body), dense
// systems from the formed operator.
template <int S>
__device__ __forceinline__ Mat<S> system_a(const PropArgs &a, int64_t sys) {
    Mat<S> A;
    if (a.kind == OSC_CHAIN) {
        const double *m = a.m + sys * S, *k = a.k + sys * S;
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const double kr = i + 1 < S ? k[i + 1 < S ? i + 1 : i] : 0.0;
                double v = 0.0;
                if (j == i) v = (k[i] + kr) / m[i];
                else if (j == i - 1) v = -k[i] / m[i];
                else if (j == i + 1) v = -kr / m[i];
                A.e[i][j] = v;
            }
    } else {
        const double *src = a.A + sys * S * S;
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) A.e[i][j] = src[i * S + j];
    }
    return A;
}

template <int N>
__device__ __forceinline__ Mat<N> mul(const Mat<N> &X, const Mat<N> &Y) {
    Mat<N> Z;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int p = 0; p < N; ++p) acc = __builtin_fma(X.e[i][p], Y.e[p][j], acc);
            Z.e[i][j] = acc;
        }
    return Z;
}

template <int N>
__device__ __forceinline__ Mat<N> identity() {
    Mat<N> I;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) I.e[i][j] = i == j ? 1.0 : 0.0;
    return I;
}

// One step of the scheme on (x, v), physical units.
template <int S>
__device__ __forceinline__ Mat<2 * S> step_matrix(const Mat<S> &A, double h, int method) {
    Mat<S> A2;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int p = 0; p < S; ++p) acc = __builtin_fma(A.e[i][p], A.e[p][j], acc);
            A2.e[i][j] = acc;
        }
    const double h2 = h * h, h3 = h2 * h, h4 = h2 * h2;
    Mat<2 * S> P;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            double pxx, pxv, pvx;
            if (method == OSC_RK4) {
                pxx = I - 0.5 * h2 * A.e[i][j] + h4 * A2.e[i][j] / 24.0;
                pxv = h * I - h3 * A.e[i][j] / 6.0;
                pvx = -h * A.e[i][j] + h3 * A2.e[i][j] / 6.0;
            } else {
                pxx = I - 0.5 * h2 * A.e[i][j];
                pxv = h * I;
                pvx = -h * A.e[i][j] + 0.25 * h3 * A2.e[i][j];
            }
            P.e[i][j] = pxx;
            P.e[i][S + j] = pxv;
            P.e[S + i][j] = pvx;
            P.e[S + i][S + j] = pxx;
        }
    return P;
}

// P^k by repeated squaring (k is the same in every lane).
template <int N>
__device__ __forceinline__ Mat<N> power(Mat<N> base, int64_t k) {
    Mat<N> R = identity<N>();
    bool first = true;
    while (k > 0) {
        if (k & 1) {
            R = first ? base : mul(R, base);
            first = false;
        }
        k >>= 1;
        if (k > 0) base = mul(base, base);
    }
    return R;
}

template <int S>
__global__ void __launch_bounds__(kThreads) small_powers_kernel(PropArgs a, int64_t k, double *out) {
    const int64_t sys = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (sys >= a.nsys) return;
    constexpr int N = 2 * S;
    const Mat<N> P = power(step_matrix(system_a<S>(a, sys), a.h[sys], a.method), k);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) out[(sys * N + i) * N + j] = P.e[i][j];
}

// Frame jumps, one lane per instance: y advances by P^stride between frames
// and by P^rest after the last frame (P^nsteps without frames).
template <typename T, int S>
__global__ void __launch_bounds__(kThreads) small_jump_kernel(PropArgs a, PropRun<T> r) {
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= r.batch) return;
    constexpr int N = 2 * S;
    const int64_t sys = a.nsys == 1 ? 0 : b;
    const Mat<N> P1 = step_matrix(system_a<S>(a, sys), a.h[sys], a.method);
    const int64_t nf = r.out_stride > 0 ? r.nsteps / r.out_stride + 1 : 0;
    const int64_t rest = r.out_stride > 0 ? r.nsteps - (nf - 1) * r.out_stride : r.nsteps;
    double y[N];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        y[i] = (double)r.x0[b * S + i];
        y[S + i] = (double)r.v0[b * S + i];
    }
    const size_t plane = (size_t)r.batch * S;
    auto put = [&](T *xd, T *vd) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (xd) xd[b * S + i] = (T)y[i];
            if (vd) vd[b * S + i] = (T)y[S + i];
        }
    };
    if (nf > 0) {
#pragma unroll
        for (int i = 0; i < S; ++i) {   // frame 0 is the caller's state as given
            if (r.xf) r.xf[b * S + i] = r.x0[b * S + i];
            if (r.vf) r.vf[b * S + i] = r.v0[b * S + i];
        }
        const Mat<N> PS = power(P1, r.out_stride);
        for (int64_t f = 1; f < nf; ++f) {
            double z[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int p = 0; p < N; ++p) acc = __builtin_fma(PS.e[i][p], y[p], acc);
                z[i] = acc;
            }
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = z[i];
            put(r.xf ? r.xf + f * plane : nullptr, r.vf ? r.vf + f * plane : nullptr);
        }
    }
    if (rest > 0) {
        const Mat<N> PR = power(P1, rest);
        double z[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int p = 0; p < N; ++p) acc = __builtin_fma(PR.e[i][p], y[p], acc);
            z[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = z[i];
    }
    if (r.nsteps == 0) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (r.xe) r.xe[b * S + i] = r.x0[b * S + i];
            if (r.ve) r.ve[b * S + i] = r.v0[b * S + i];
        }
    } else {
        put(r.xe, r.ve);
    }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; ++i) ok = ok && __builtin_isfinite(y[i]);
    if (!ok && r.nonfinite) atomicOr(r.nonfinite, 1);
}

// ------------------------------------------------------ batched products
// A of every chain of the batch as a dense [batch][s][s] matrix.
__global__ void __launch_bounds__(kThreads) chain_dense_a_kernel(PropArgs a, int s, double *A) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t total = a.nsys * s * s;
    if (idx >= total) return;
    const int64_t sys = idx / ((int64_t)s * s);
    const int i = (int)(idx / s % s), j = (int)(idx % s);
    const double *m = a.m + sys * s, *k = a.k + sys * s;
    const double kr = i + 1 < s ? k[i + 1] : 0.0;
    double v = 0.0;
    if (j == i) v = (k[i] + kr) / m[i];
    else if (j == i - 1) v = -k[i] / m[i];
    else if (j == i + 1) v = -kr / m[i];
    A[idx] = v;
}

// The one-step matrix [nsys][2s][2s] from A and A^2 ([nsys][s][s]).
__global__ void __launch_bounds__(kThreads) assemble_kernel(int64_t nsys, int s, int method, const double *A,
                                                            const double *A2, const double *h, double *P) {
    const int n = 2 * s;
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= nsys * n * n) return;
    const int64_t sys = idx / ((int64_t)n * n);
    const int r = (int)(idx / n % n), c = (int)(idx % n);
    const int i = r % s, j = c % s;
    const size_t o = (size_t)sys * s * s + (size_t)i * s + j;
    const double hh = h[sys], h2 = hh * hh, h3 = h2 * hh, h4 = h2 * h2;
    const double I = i == j ? 1.0 : 0.0, a = A[o], a2 = A2[o];
    double v;
    const bool top = r < s, left = c < s;
    if (method == OSC_RK4) {
        if (top == left) v = I - 0.5 * h2 * a + h4 * a2 / 24.0;
        else if (top) v = hh * I - h3 * a / 6.0;
        else v = -hh * a + h3 * a2 / 6.0;
    } else {
        if (top == left) v = I - 0.5 * h2 * a;
        else if (top) v = hh * I;
        else v = -hh * a + 0.25 * h3 * a2;
    }
    P[idx] = v;
}

__global__ void __launch_bounds__(kThreads) identity_kernel(int64_t nsys, int n, double *P) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= nsys * n * n) return;
    P[idx] = (idx / n % n) == (idx % n) ? 1.0 : 0.0;
}

// Z [batch][2s] = (x0, v0) in FP64; frame 0 is the caller's state as given.
template <typename T>
__global__ void __launch_bounds__(kThreads) load_z_kernel(PropRun<T> r, int s, double *Z) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= r.batch * s) return;
    const int64_t b = idx / s;
    const int i = (int)(idx % s);
    Z[b * 2 * s + i] = (double)r.x0[idx];
    Z[b * 2 * s + s + i] = (double)r.v0[idx];
    if (r.out_stride > 0) {
        if (r.xf) r.xf[idx] = r.x0[idx];
        if (r.vf) r.vf[idx] = r.v0[idx];
    }
    if (r.nsteps == 0) {
        if (r.xe) r.xe[idx] = r.x0[idx];
        if (r.ve) r.ve[idx] = r.v0[idx];
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) store_z_kernel(int64_t batch, int s, const double *Z, T *xd, T *vd,
                                                           int *nonfinite) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= batch * s) return;
    const int64_t b = idx / s;
    const int i = (int)(idx % s);
    const double x = Z[b * 2 * s + i], v = Z[b * 2 * s + s + i];
    if (xd) xd[idx] = (T)x;
    if (vd) vd[idx] = (T)v;
    if (!(__builtin_isfinite(x) && __builtin_isfinite(v)) && nonfinite) atomicOr(nonfinite, 1);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// One rocBLAS handle per device, created on first use; calls set the stream
// and enqueue under the lock (the products run asynchronously on it).
std::mutex blas_mutex;
std::map<int, rocblas_handle> blas_handles;

// C = op(A) B in column-major terms (rocBLAS's convention), strided over nsys
osc_status dgemm(hipStream_t st, bool trans_a, int m, int n, int k, const double *A, int64_t stride_a,
                 const double *B, int64_t stride_b, double *C, int64_t stride_c, int64_t nsys) {
    int dev = 0;
    OSC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(blas_mutex);
    rocblas_handle &h = blas_handles[dev];
    if (!h) {
        if (rocblas_create_handle(&h) != rocblas_status_success) {
            h = nullptr;
            return fail(OSC_EDEVICE, "rocblas_create_handle failed");
        }
        // no atomics: the same products give the same bits on every call
        if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success)
            return fail(OSC_EDEVICE, "rocblas_set_atomics_mode failed");
    }
    if (rocblas_set_stream(h, st) != rocblas_status_success) return fail(OSC_EDEVICE, "rocblas_set_stream failed");
    const double one = 1.0, zero = 0.0;
    const rocblas_operation ta = trans_a ? rocblas_operation_transpose : rocblas_operation_none;
    const rocblas_status r =
        nsys == 1 ? rocblas_dgemm(h, ta, rocblas_operation_none, m, n, k, &one, A, trans_a ? k : m, B, k, &zero, C, m)
                  : rocblas_dgemm_strided_batched(h, ta, rocblas_operation_none, m, n, k, &one, A, trans_a ? k : m,
                                                  stride_a, B, k, stride_b, &zero, C, m, stride_c, (rocblas_int)nsys);
    if (r != rocblas_status_success)
        return fail(OSC_EDEVICE, std::string("rocBLAS DGEMM: ") + rocblas_status_to_string(r));
    return OSC_OK;
}

// C = X Y for every system (row-major n x n), C distinct from X and Y: in
// column-major terms C^T = Y^T X^T.
osc_status square_mul(int64_t nsys, int n, const double *X, const double *Y, double *C, hipStream_t st) {
    const int64_t nn = (int64_t)n * n;
    return dgemm(st, false, n, n, n, Y, nn, X, nn, C, nn, nsys);
}

// Temporaries of one call: returned to the pool only after the stream has
// finished every launch that uses them (also on an error return).
struct DevBufs {
    hipStream_t st;
    void *p[8] = {};
    explicit DevBufs(hipStream_t s) : st(s) {}
    ~DevBufs() {
        bool any = false;
        for (void *q : p) any = any || q;
        if (any) (void)hipStreamSynchronize(st);
        for (void *q : p) pool_free(q);
    }
};

// ------------------------------------------------- per-step propagator
// Chains of s <= 2, one lane per instance.  In scaled units (w = h v,
// B = h^2 A) every step adds (P - I) y to the state:
//   dx = w + Dxx x + Dxw w,   dw = Dwx x + Dww w,
// RK4:    Dxx = Dww = -B/2 + B^2/24,  Dxw = -B/6,  Dwx = -B + B^2/6;
// Verlet: Dxx = Dww = -B/2,           Dxw = 0,     Dwx = -B + B^2/4.
// B comes from the split chain coefficients in FP64.  In FP32 the blocks
// that multiply x are split into high and low parts (those that multiply w
// enter smaller by h omega and use the high part), x and w are kept as
// hi + lo (the low part collects the increments and is folded into the high
// part every 4 steps, at fixed global step indices), and each increment is
// summed from its smallest term up: low parts, w terms, high parts, then w.
template <typename T, int S>
__global__ void __launch_bounds__(kThreads) prop_step_kernel(ChainLaunch<T> a, int method) {
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (b >= a.batch) return;
    constexpr bool COMP = std::is_same<T, float>::value;
    const size_t base = (size_t)b * S, plane = (size_t)a.batch * S;
    const double h = a.c.h[b];
    double Bm[S][S], B2[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const double cl = (double)a.c.clh[base + i] + (COMP ? (double)a.c.cll[base + i] : 0.0);
        const double cr = (double)a.c.crh[base + i] + (COMP ? (double)a.c.crl[base + i] : 0.0);
#pragma unroll
        for (int j = 0; j < S; ++j) Bm[i][j] = j == i ? cl + cr : (j == i - 1 ? -cl : (j == i + 1 ? -cr : 0.0));
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int p = 0; p < S; ++p) acc = __builtin_fma(Bm[i][p], Bm[p][j], acc);
            B2[i][j] = acc;
        }
    T xxh[S][S], xxl[S][S], xw[S][S], wxh[S][S], wxl[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) {
            double dxx, dxw, dwx;
            if (method == OSC_RK4) {
                dxx = -0.5 * Bm[i][j] + B2[i][j] / 24.0;
                dxw = -Bm[i][j] / 6.0;
                dwx = -Bm[i][j] + B2[i][j] / 6.0;
            } else {
                dxx = -0.5 * Bm[i][j];
                dxw = 0.0;
                dwx = -Bm[i][j] + 0.25 * B2[i][j];
            }
            xxh[i][j] = (T)dxx;
            xxl[i][j] = COMP ? (T)(dxx - (double)xxh[i][j]) : T(0);
            xw[i][j] = (T)dxw;
            wxh[i][j] = (T)dwx;
            wxl[i][j] = COMP ? (T)(dwx - (double)wxh[i][j]) : T(0);
        }
    T x[S], xl[S], w[S], wl[S];
    if (a.load_mode == LOAD_USER) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            x[i] = a.x0[base + i];
            xl[i] = T(0);
            const double wd = h * (double)a.v0[base + i];
            w[i] = (T)wd;
            wl[i] = COMP ? (T)(wd - (double)w[i]) : T(0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            x[i] = a.state[base + i];
            xl[i] = a.state[plane + base + i];
            w[i] = a.state[2 * plane + base + i];
            wl[i] = a.state[3 * plane + base + i];
        }
    }
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (a.xf) a.xf[fo + base + i] = initial ? a.x0[base + i] : (T)((double)x[i] + (double)xl[i]);
            if (a.vf) a.vf[fo + base + i] = initial ? a.v0[base + i] : (T)(((double)w[i] + (double)wl[i]) / h);
        }
    };
    auto step = [&]() {
        T xe[S], we[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            xe[i] = COMP ? x[i] + xl[i] : x[i];
            we[i] = COMP ? w[i] + wl[i] : w[i];
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            T tx = T(0), tw = T(0);
            if constexpr (COMP) {
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    tx = fma_t(xxl[i][j], xe[j], tx);
                    tw = fma_t(wxl[i][j], xe[j], tw);
                }
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                tx = fma_t(xw[i][j], we[j], tx);
                tw = fma_t(xxh[i][j], we[j], tw);   // Dww = Dxx
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                tx = fma_t(xxh[i][j], xe[j], tx);
                tw = fma_t(wxh[i][j], xe[j], tw);
            }
            const T dx = we[i] + tx;
            if constexpr (COMP) {
                xl[i] += dx;
                wl[i] += tw;
            } else {
                x[i] += dx;
                w[i] += tw;
            }
        }
    };
    auto fold = [&]() {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            T t = x[i] + xl[i];
            xl[i] = xl[i] - (t - x[i]);
            x[i] = t;
            t = w[i] + wl[i];
            wl[i] = wl[i] - (t - w[i]);
            w[i] = t;
        }
    };
    constexpr int64_t kFold = 4;
    const bool untouched = a.load_mode == LOAD_USER;
    const int64_t stride = a.out_stride;
    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    while (n < nend) {
        int64_t stop = nend;
        if (stride > 0) {
            const int64_t nf = (n / stride + 1) * stride;
            stop = nf < stop ? nf : stop;
        }
        while (n < stop) {
            const int64_t to_fold = COMP ? kFold - n % kFold : stop - n;
            const int cnt = (int)(stop - n < to_fold ? stop - n : to_fold);
            for (int q = 0; q < cnt; ++q) step();
            n += cnt;
            if (COMP && n % kFold == 0) fold();
        }
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < S; ++i) ok = ok && __builtin_isfinite(x[i]) && __builtin_isfinite(w[i]);
    if (a.store_mode & STORE_STATE) {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            a.state[base + i] = x[i];
            a.state[plane + base + i] = xl[i];
            a.state[2 * plane + base + i] = w[i];
            a.state[3 * plane + base + i] = wl[i];
        }
    }
    if (a.store_mode & STORE_USER) {
        const bool copy_input = untouched && a.nsteps == 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (a.xe) a.xe[base + i] = copy_input ? a.x0[base + i] : (T)((double)x[i] + (double)xl[i]);
            if (a.ve) a.ve[base + i] = copy_input ? a.v0[base + i] : (T)(((double)w[i] + (double)wl[i]) / h);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

}  // namespace

bool propagator_small(int s) { return s <= 2; }

template <typename T>
osc_status prop_step_launch(const ChainLaunch<T> &a, int method, hipStream_t st) {
    if (a.batch == 0) return OSC_OK;
    if (a.s < 1 || a.s > 2) return fail(OSC_ENOTSUP, "the per-step propagator takes chains of s <= 2");
    if (a.s == 1)
        hipLaunchKernelGGL((prop_step_kernel<T, 1>), dim3(blocks_for(a.batch)), dim3(kThreads), 0, st, a, method);
    else
        hipLaunchKernelGGL((prop_step_kernel<T, 2>), dim3(blocks_for(a.batch)), dim3(kThreads), 0, st, a, method);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}
template osc_status prop_step_launch<float>(const ChainLaunch<float> &, int, hipStream_t);
template osc_status prop_step_launch<double>(const ChainLaunch<double> &, int, hipStream_t);

// P1 (one step) of every system, [nsys][2s][2s], by batched products.
osc_status propagator_step_matrices(const PropArgs &a, int s, double *P1, hipStream_t st) {
    const int64_t nsys = a.nsys;
    const size_t ss = (size_t)s * s;
    DevBufs tmp(st);
    const double *A = a.A;
    if (a.kind == OSC_CHAIN) {
        tmp.p[0] = pool_alloc(nsys * ss * sizeof(double));
        if (!tmp.p[0]) return fail(OSC_ENOMEM, "device memory exhausted for the chains' operators");
        hipLaunchKernelGGL(chain_dense_a_kernel, dim3(blocks_for(nsys * (int64_t)ss)), dim3(kThreads), 0, st, a, s,
                           static_cast<double *>(tmp.p[0]));
        OSC_HIP(hipGetLastError());
        A = static_cast<const double *>(tmp.p[0]);
    }
    tmp.p[1] = pool_alloc(nsys * ss * sizeof(double));
    if (!tmp.p[1]) return fail(OSC_ENOMEM, "device memory exhausted for A^2");
    double *A2 = static_cast<double *>(tmp.p[1]);
    osc_status r = square_mul(nsys, s, A, A, A2, st);
    if (r) return r;
    const int n = 2 * s;
    hipLaunchKernelGGL(assemble_kernel, dim3(blocks_for(nsys * (int64_t)n * n)), dim3(kThreads), 0, st, nsys, s,
                       a.method, A, A2, a.h, P1);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

// P1^k1 -> out1 and (if out2) P1^k2 -> out2, sharing the squarings.
osc_status propagator_powers(int64_t nsys, int n, const double *P1, int64_t k1, double *out1, int64_t k2,
                             double *out2, hipStream_t st) {
    const size_t nn = (size_t)n * n;
    DevBufs tmp(st);
    for (int i = 0; i < 3; ++i) {
        tmp.p[i] = pool_alloc(nsys * nn * sizeof(double));
        if (!tmp.p[i]) return fail(OSC_ENOMEM, "device memory exhausted for propagator powers");
    }
    double *base = static_cast<double *>(tmp.p[0]), *spare = static_cast<double *>(tmp.p[1]);
    double *t = static_cast<double *>(tmp.p[2]);
    OSC_HIP(hipMemcpyAsync(base, P1, nsys * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
    struct Acc {
        int64_t k;
        double *out;
        bool set;
    } acc[2] = {{k1, out1, false}, {out2 ? k2 : 0, out2, false}};
    for (Acc &q : acc)
        if (q.out && q.k == 0) {
            hipLaunchKernelGGL(identity_kernel, dim3(blocks_for(nsys * (int64_t)nn)), dim3(kThreads), 0, st, nsys, n,
                               q.out);
            OSC_HIP(hipGetLastError());
        }
    int64_t kmax = std::max(acc[0].k, acc[1].k);
    osc_status r;
    for (int bit = 0; (kmax >> bit) > 0; ++bit) {
        for (Acc &q : acc) {
            if (!q.out || !((q.k >> bit) & 1)) continue;
            if (!q.set) {
                OSC_HIP(hipMemcpyAsync(q.out, base, nsys * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
                q.set = true;
            } else {
                if ((r = square_mul(nsys, n, q.out, base, t, st))) return r;
                OSC_HIP(hipMemcpyAsync(q.out, t, nsys * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
            }
        }
        if ((kmax >> (bit + 1)) > 0) {
            if ((r = square_mul(nsys, n, base, base, spare, st))) return r;
            std::swap(base, spare);
        }
    }
    return OSC_OK;
}

osc_status propagator_matrix(const PropArgs &a, int s, int64_t k, double *out, hipStream_t st) {
    if (a.nsys == 0) return OSC_OK;
    if (propagator_small(s)) {
        if (s == 1)
            hipLaunchKernelGGL(small_powers_kernel<1>, dim3(blocks_for(a.nsys)), dim3(kThreads), 0, st, a, k, out);
        else
            hipLaunchKernelGGL(small_powers_kernel<2>, dim3(blocks_for(a.nsys)), dim3(kThreads), 0, st, a, k, out);
        OSC_HIP(hipGetLastError());
        return OSC_OK;
    }
    const int n = 2 * s;
    DevBufs tmp(st);
    tmp.p[0] = pool_alloc(a.nsys * (size_t)n * n * sizeof(double));
    if (!tmp.p[0]) return fail(OSC_ENOMEM, "device memory exhausted for the one-step matrices");
    double *P1 = static_cast<double *>(tmp.p[0]);
    osc_status r = propagator_step_matrices(a, s, P1, st);
    if (r) return r;
    return propagator_powers(a.nsys, n, P1, k, out, 0, nullptr, st);
}

template <typename T>
osc_status propagator_jump(const PropArgs &a, int s, const PropRun<T> &run, hipStream_t st) {
    if (run.batch == 0) return OSC_OK;
    if (propagator_small(s)) {
        if (s == 1)
            hipLaunchKernelGGL((small_jump_kernel<T, 1>), dim3(blocks_for(run.batch)), dim3(kThreads), 0, st, a, run);
        else
            hipLaunchKernelGGL((small_jump_kernel<T, 2>), dim3(blocks_for(run.batch)), dim3(kThreads), 0, st, a, run);
        OSC_HIP(hipGetLastError());
        return OSC_OK;
    }
    const int n = 2 * s;
    const size_t nn = (size_t)n * n;
    const int64_t nf = run.out_stride > 0 ? run.nsteps / run.out_stride + 1 : 0;
    const int64_t rest = run.out_stride > 0 ? run.nsteps - (nf - 1) * run.out_stride : run.nsteps;
    const int64_t kS = nf > 1 ? run.out_stride : 0;
    DevBufs tmp(st);
    tmp.p[0] = pool_alloc(a.nsys * nn * sizeof(double));            // P1
    tmp.p[1] = kS ? pool_alloc(a.nsys * nn * sizeof(double)) : nullptr;   // P^stride
    tmp.p[2] = rest ? pool_alloc(a.nsys * nn * sizeof(double)) : nullptr; // P^rest
    tmp.p[3] = pool_alloc((size_t)run.batch * n * sizeof(double));   // Z
    tmp.p[4] = pool_alloc((size_t)run.batch * n * sizeof(double));   // Z'
    if (!tmp.p[0] || (kS && !tmp.p[1]) || (rest && !tmp.p[2]) || !tmp.p[3] || !tmp.p[4])
        return fail(OSC_ENOMEM, "device memory exhausted for propagator jumps");
    double *P1 = static_cast<double *>(tmp.p[0]), *PS = static_cast<double *>(tmp.p[1]);
    double *PR = static_cast<double *>(tmp.p[2]);
    double *Z = static_cast<double *>(tmp.p[3]), *Z2 = static_cast<double *>(tmp.p[4]);
    osc_status r;
    if ((r = propagator_step_matrices(a, s, P1, st))) return r;
    if (kS || rest) {
        if ((r = propagator_powers(a.nsys, n, P1, kS ? kS : rest, kS ? PS : PR, rest, kS ? PR : nullptr, st)))
            return r;
    }
    hipLaunchKernelGGL((load_z_kernel<T>), dim3(blocks_for(run.batch * s)), dim3(kThreads), 0, st, run, s, Z);
    OSC_HIP(hipGetLastError());
    // Z' = Z P^T, one row per instance: column-major Z'^T = P Z^T, with the
    // row-major P read as its transpose
    auto advance = [&](const double *P) -> osc_status {
        osc_status e = a.nsys == 1 ? dgemm(st, true, n, (int)run.batch, n, P, 0, Z, 0, Z2, 0, 1)
                                   : dgemm(st, true, n, 1, n, P, (int64_t)nn, Z, n, Z2, n, run.batch);
        if (e) return e;
        std::swap(Z, Z2);
        return OSC_OK;
    };
    const size_t plane = (size_t)run.batch * s;
    for (int64_t f = 1; f < nf; ++f) {
        if ((r = advance(PS))) return r;
        hipLaunchKernelGGL((store_z_kernel<T>), dim3(blocks_for(run.batch * s)), dim3(kThreads), 0, st, run.batch, s,
                           Z, run.xf ? run.xf + f * plane : nullptr, run.vf ? run.vf + f * plane : nullptr,
                           run.nonfinite);
        OSC_HIP(hipGetLastError());
    }
    if (rest > 0) {
        if ((r = advance(PR))) return r;
    }
    if (run.nsteps > 0) {
        hipLaunchKernelGGL((store_z_kernel<T>), dim3(blocks_for(run.batch * s)), dim3(kThreads), 0, st, run.batch, s,
                           Z, run.xe, run.ve, run.nonfinite);
        OSC_HIP(hipGetLastError());
    }
    return OSC_OK;
}

template osc_status propagator_jump<float>(const PropArgs &, int, const PropRun<float> &, hipStream_t);
template osc_status propagator_jump<double>(const PropArgs &, int, const PropRun<double> &, hipStream_t);

}  // namespace osc
