// Chain coefficient preparation, stability bound and FP64 energy kernels.
//
// For the fixed-free chain of eq. (2) generalised to s bodies, A = M^-1 K is
// tridiagonal with rows (A x)_i = (k_i (x_i - x_{i-1}) - k_{i+1} (x_{i+1} - x_i)) / m_i.
// In scaled time the integrators need B = h^2 A, i.e. per body
//   cl_i = h^2 k_i / m_i,   cr_i = h^2 k_{i+1} / m_i   (cr_{s-1} = 0),
// formed here in FP64 and, for FP32 state, split into hi + lo parts.

#include <type_traits>

#include <algorithm>

#include "osc_internal.h"

namespace osc {
namespace {

__device__ __forceinline__ void atomic_max_pos(double *addr, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long *>(addr), __double_as_longlong(v));
}

// Grid-stride over the DOFs; the stability bound is reduced per workgroup so
// that only one atomic per workgroup reaches the single bound in memory
// (same-address atomics serialise in the cache).
template <typename T>
__global__ void __launch_bounds__(256) chain_prepare_kernel(int64_t batch, int s, const double *__restrict__ m,
                                                            const double *__restrict__ k, const double *dt, T *clh,
                                                            T *crh, T *cll, T *crl, double *hout,
                                                            double *theta_bound, int *bad) {
    __shared__ double wmax[4];
    double bound = 0.0;
    const int64_t n = batch * (int64_t)s;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / s;
        const int d = (int)(i - b * s);
        const double h = dt[b];
        const double mi = m[i];
        const double kl = k[i];
        const double kr = (d + 1 < s) ? k[i + 1] : 0.0;
        const bool ok = (h > 0.0) && __builtin_isfinite(h) && (mi > 0.0) && __builtin_isfinite(mi) &&
                        (kl >= 0.0) && __builtin_isfinite(kl) && (kr >= 0.0) && __builtin_isfinite(kr);
        if (!ok) {
            atomicOr(bad, 1);
            continue;
        }
        const double cl = h * h * kl / mi;
        const double cr = h * h * kr / mi;
        if (d == 0 && hout) hout[b] = h;
        clh[i] = (T)cl;
        crh[i] = (T)cr;
        if constexpr (std::is_same<T, float>::value) {
            cll[i] = (T)(cl - (double)clh[i]);
            crl[i] = (T)(cr - (double)crh[i]);
        }
        // Gershgorin: every eigenvalue of B lies below the largest row sum
        // |B_ii| + sum_j |B_ij| = 2 (cl_i + cr_i); theta = sqrt(lambda_max(B)) = h omega_max.
        bound = fmax(bound, sqrt(2.0 * (cl + cr)));
    }
    for (int off = 32; off > 0; off >>= 1) bound = fmax(bound, __shfl_xor(bound, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = bound;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        if (mx > 0.0) atomic_max_pos(theta_bound, mx);
    }
}

// Exact stability estimate of one chain per thread.  B = h^2 M^-1 K is
// similar to the symmetric tridiagonal T = M^-1/2 (h^2 K) M^-1/2 with
//   T_ii = cl_i + cr_i,   T_{i,i+1}^2 = cr_i cl_{i+1},
// (cl_i = h^2 k_i / m_i, cr_i = h^2 k_{i+1} / m_i), so h^2 omega_max^2 is the
// largest eigenvalue of T.  Sturm sequence: the number of eigenvalues below
// t equals the number of negative terms of q_0 = T_00 - t,
// q_i = T_ii - t - T_{i-1,i}^2 / q_{i-1}.  Bisection on [0, Gershgorin bound]
// narrows lambda_max to a relative width of 2^-40; the upper end is kept, so
// the estimate never lies below lambda_max.
__global__ void __launch_bounds__(256) chain_sturm_kernel(int64_t batch, int s, const double *__restrict__ m,
                                                          const double *__restrict__ k,
                                                          const double *__restrict__ dt, double *theta) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double h = dt[b];
    const double *mb = m + b * s, *kb = k + b * s;
    auto cl = [&](int i) { return h * h * kb[i] / mb[i]; };
    auto cr = [&](int i) { return i + 1 < s ? h * h * kb[i + 1] / mb[i] : 0.0; };
    double hi = 0.0;
    for (int i = 0; i < s; ++i) hi = fmax(hi, 2.0 * (cl(i) + cr(i)));
    // count of eigenvalues below t
    auto below = [&](double t) {
        int cnt = 0;
        double q = 1.0, e2 = 0.0;
        for (int i = 0; i < s; ++i) {
            const double d = cl(i) + cr(i);
            q = d - t - (i > 0 ? e2 / q : 0.0);
            if (q == 0.0) q = -1e-300;   // t is an eigenvalue of the leading block: count it as passed
            cnt += q < 0.0;
            e2 = i + 1 < s ? cr(i) * cl(i + 1) : 0.0;
        }
        return cnt;
    };
    double lo = 0.0;
    for (int it = 0; it < 200 && hi - lo > 0x1p-40 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == s) hi = mid;   // every eigenvalue lies below mid
        else lo = mid;
    }
    theta[b] = sqrt(hi);
}

// One group of G lanes (power of two <= 64) per instance; FP64 sums reduced
// across the group with xor shuffles.
template <typename T, int G>
__global__ void __launch_bounds__(256) chain_energy_kernel(int64_t batch, int s, const double *__restrict__ m,
                                                           const double *__restrict__ k,
                                                           const double *__restrict__ hh,
                                                           const T *__restrict__ x, const T *__restrict__ v,
                                                           double *E, bool shadow) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = g / G;
    const int l = (int)(g % G);
    const bool active = b < batch;
    double kin = 0.0, pot = 0.0, corr = 0.0;
    if (active) {
        const size_t base = (size_t)b * s;
        for (int d = l; d < s; d += G) {
            const double xd = (double)x[base + d];
            const double xm = d > 0 ? (double)x[base + d - 1] : 0.0;
            const double vd = (double)v[base + d];
            const double e = xd - xm;
            kin += m[base + d] * vd * vd;
            pot += k[base + d] * e * e;
            if (shadow) {
                // (K x)_d = k_d e_d - k_{d+1} e_{d+1}
                double f = k[base + d] * e;
                if (d + 1 < s) f -= k[base + d + 1] * ((double)x[base + d + 1] - xd);
                corr += f * f / m[base + d];
            }
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        kin += __shfl_xor(kin, off, G);
        pot += __shfl_xor(pot, off, G);
        corr += __shfl_xor(corr, off, G);
    }
    if (active && l == 0) {
        if (shadow) {
            const double h = hh[b];
            E[b] = kin + pot - 0.25 * h * h * corr;
        } else {
            E[b] = 0.5 * kin + 0.5 * pot;
        }
    }
}

template <typename T, int G>
void launch_energy(int64_t batch, int s, const double *m, const double *k, const double *h, const T *x,
                   const T *v, double *E, bool shadow, hipStream_t st) {
    const int64_t threads = batch * G;
    const int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL((chain_energy_kernel<T, G>), dim3((unsigned)blocks), dim3(256), 0, st, batch, s, m, k,
                       h, x, v, E, shadow);
}

}  // namespace

template <typename T>
osc_status chain_prepare(int64_t batch, int s, const double *m, const double *k, const double *dt, T *clh,
                         T *crh, T *cll, T *crl, double *h, double *theta_bound, int *bad_param,
                         hipStream_t st) {
    const int64_t n = batch * (int64_t)s;
    if (n == 0) return OSC_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL((chain_prepare_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, batch, s, m, k, dt,
                       clh, crh, cll, crl, h, theta_bound, bad_param);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

osc_status chain_sturm_theta(int64_t batch, int s, const double *m, const double *k, const double *dt,
                             double *theta, hipStream_t st) {
    if (batch == 0) return OSC_OK;
    hipLaunchKernelGGL(chain_sturm_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, batch, s, m,
                       k, dt, theta);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template <typename T>
osc_status chain_energy(int64_t batch, int s, const double *m, const double *k, const double *h, const T *x,
                        const T *v, double *E, bool shadow, hipStream_t st) {
    if (batch == 0) return OSC_OK;
    if (s <= 1) launch_energy<T, 1>(batch, s, m, k, h, x, v, E, shadow, st);
    else if (s <= 2) launch_energy<T, 2>(batch, s, m, k, h, x, v, E, shadow, st);
    else if (s <= 4) launch_energy<T, 4>(batch, s, m, k, h, x, v, E, shadow, st);
    else if (s <= 8) launch_energy<T, 8>(batch, s, m, k, h, x, v, E, shadow, st);
    else if (s <= 16) launch_energy<T, 16>(batch, s, m, k, h, x, v, E, shadow, st);
    else if (s <= 32) launch_energy<T, 32>(batch, s, m, k, h, x, v, E, shadow, st);
    else launch_energy<T, 64>(batch, s, m, k, h, x, v, E, shadow, st);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

template osc_status chain_prepare<float>(int64_t, int, const double *, const double *, const double *, float *,
                                         float *, float *, float *, double *, double *, int *, hipStream_t);
template osc_status chain_prepare<double>(int64_t, int, const double *, const double *, const double *,
                                          double *, double *, double *, double *, double *, double *, int *,
                                          hipStream_t);
template osc_status chain_energy<float>(int64_t, int, const double *, const double *, const double *,
                                        const float *, const float *, double *, bool, hipStream_t);
template osc_status chain_energy<double>(int64_t, int, const double *, const double *, const double *,
                                         const double *, const double *, double *, bool, hipStream_t);

}  // namespace osc
