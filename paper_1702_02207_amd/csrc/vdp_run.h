// Coupled Van der Pol chains: the chain of eq. (2) with a Van der Pol
// element on every body, optionally driven by a harmonic force,
//     m_i x_i'' - mu (1 - x_i^2) x_i' + (K x)_i = F_i cos(Omega t),
// the nonlinear oscillators the paper's section 1 motivates the work with.
//
// Classic RK4 on the first-order system of section 3, in scaled time
// (tau = t/h, w = h v, B = h^2 M^-1 K, g_i = h mu / m_i, f = F / m):
//     x' = w,   w' = -B x + g (1 - x^2) w + h^2 f cos(Omega h tau),
// with the force's phase at the stage times t_n, t_n + h/2 (twice), t_n + h
// taken from the FP64 rotation of the damped, driven kernel, re-anchored
// exactly every 64 global steps, so that chunked runs give the same bits.
// The linear Taylor form of the free chains does not apply (the right-hand
// side is nonlinear), so the four stages are evaluated in turn.  With k_j
// the stages' w-slopes, stage j's argument is (x + d_j, w + c_j) with
// d_2 = w/2, d_3 = w/2 + k_1/4, d_4 = w + k_2/2 and c_2 = k_1/2,
// c_3 = k_2/2, c_4 = k_3, so that
//     B (x + d_j) = B x + B d_j:
// B x takes the split FP32 coefficients once per step, the small offsets
// the high parts only.  The increments are
//     dx = w + (k_1 + k_2 + k_3)/6,   dw = (k_1 + 2 k_2 + 2 k_3 + k_4)/6
// (the x-slopes of RK4 are w plus the offsets).  FP32 keeps x and w as
// renormalised hi + lo pairs: the stages read the high parts, the low parts
// collect the increments as they are formed, and x += w keeps its exact
// rounding error (FP64: a plain update).
//
// Layouts: those of the damped, driven register kernel (one lane per chain
// for s <= 8, one wave per chain beyond, DPP halos, no LDS), s <= 1024.
//
// This header holds the integrator; vdp.hip instantiates the free FP32
// kernels, vdp_forced.hip the forced FP32 ones and vdp_f64.hip both FP64
// sets, each built with the instruction scheduling that suits its register
// pressure.

#pragma once

#include <cstdint>
#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kThreads = 256;

template <typename T, int DPL, int LPI, bool FORCED>
__device__ __forceinline__ void vdp_chain_run(const VdpLaunch<T> &a, const int64_t g) {
    constexpr bool COMP = std::is_same<T, float>::value;
    const int64_t b = g / LPI;
    const int sl = (int)(g % LPI);
    const bool active = b < a.batch;
    const int s = a.s;
    const int d0 = sl * DPL;
    const size_t base = (size_t)(active ? b : 0) * s, plane = (size_t)a.batch * s;
    const double h = active ? a.c.h[b] : 1.0;

    const bool run_whole = active && d0 + DPL <= s;
    auto load = [&](const auto *src, auto (&dst)[DPL]) {
        using U = std::remove_const_t<std::remove_pointer_t<decltype(src)>>;
        constexpr int V = 16 / (int)sizeof(U);
        typedef U vec_t __attribute__((ext_vector_type(V)));
        if (DPL % V == 0 && run_whole && ((uintptr_t)(src + base + d0) % 16) == 0) {
#pragma unroll
            for (int q = 0; q < DPL / V; ++q) {
                const vec_t v = *reinterpret_cast<const vec_t *>(src + base + d0 + q * V);
#pragma unroll
                for (int e = 0; e < V; ++e) dst[q * V + e] = v[e];
            }
        } else {
#pragma unroll
            for (int j = 0; j < DPL; ++j) dst[j] = (active && d0 + j < s) ? src[base + d0 + j] : U(0);
        }
    };
    auto store = [&](T *dst, auto val) {
        constexpr int V = 16 / (int)sizeof(T);
        typedef T vec_t __attribute__((ext_vector_type(V)));
        if (DPL % V == 0 && run_whole && ((uintptr_t)(dst + base + d0) % 16) == 0) {
#pragma unroll
            for (int q = 0; q < DPL / V; ++q) {
                vec_t v;
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = val(q * V + e);
                *reinterpret_cast<vec_t *>(dst + base + d0 + q * V) = v;
            }
        } else {
#pragma unroll
            for (int j = 0; j < DPL; ++j)
                if (active && d0 + j < s) dst[base + d0 + j] = val(j);
        }
    };

    T clh[DPL], crh[DPL], cll[DPL], crl[DPL], gm[DPL], x[DPL], xl[DPL], w[DPL], wl[DPL];
    load(a.c.clh, clh);
    load(a.c.crh, crh);
#pragma unroll
    for (int j = 0; j < DPL; ++j) cll[j] = crl[j] = T(0);
    if constexpr (COMP) {
        load(a.c.cll, cll);
        load(a.c.crl, crl);
    }
    {
        double md[DPL];
        load(a.m, md);
        // zero beyond the chain (padding DOFs stay at rest)
#pragma unroll
        for (int j = 0; j < DPL; ++j) gm[j] = md[j] > 0.0 ? (T)(h * a.mu / md[j]) : T(0);
    }
    T fh[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) fh[j] = T(0);
    Phase ph{};
    if constexpr (FORCED) {
        double fd[DPL];
        load(a.f, fd);
#pragma unroll
        for (int j = 0; j < DPL; ++j) fh[j] = (T)(h * h * fd[j]);
        if (active) ph.start(a.omega[b] * h, a.n0);
    }
    if (a.load_mode == LOAD_USER) {
        T v0[DPL];
        load(a.x0, x);
        load(a.v0, v0);
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            xl[j] = T(0);
            const double wd = h * (double)v0[j];
            w[j] = (T)wd;
            wl[j] = COMP ? (T)(wd - (double)w[j]) : T(0);
        }
    } else {
        load(a.state, x);
        load(a.state + plane, xl);
        load(a.state + 2 * plane, w);
        load(a.state + 3 * plane, wl);
    }

    auto halo = [&](const T (&u)[DPL], T &prev, T &next) {
        if constexpr (LPI == 1) {
            prev = T(0);
            next = T(0);
        } else {
            prev = from_left<true>(u[DPL - 1]);
            next = from_right<true>(u[0]);
        }
    };
    // out = B U (high coefficients; SPLIT: plus the low coefficients' part)
    auto bop = [&](auto split_c, const T (&U)[DPL], T (&out)[DPL]) {
        constexpr bool SPLIT = decltype(split_c)::value && COMP;
        T up, un;
        halo(U, up, un);
        T el = U[0] - up;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const T ur = j + 1 < DPL ? U[j + 1 < DPL ? j + 1 : j] : un;
            const T er = ur - U[j];
            if constexpr (SPLIT) out[j] = fma_t(clh[j], el, fma_t(-crh[j], er, fma_t(cll[j], el, -crl[j] * er)));
            else out[j] = fma_t(clh[j], el, -crh[j] * er);
            el = er;
        }
    };

    auto xval = [&](int j) { return (T)((double)x[j] + (double)xl[j]); };
    auto vval = [&](int j) { return (T)(((double)w[j] + (double)wl[j]) / h); };
    auto copy_out = [&](T *dst, const T *src) {
        T o[DPL];
        load(src, o);
        store(dst, [&](int j) { return o[j]; });
    };
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
        if (a.xf) {
            if (initial) copy_out(a.xf + fo, a.x0);
            else store(a.xf + fo, xval);
        }
        if (a.vf) {
            if (initial) copy_out(a.vf + fo, a.v0);
            else store(a.vf + fo, vval);
        }
    };

    const bool untouched = a.load_mode == LOAD_USER;
    const int64_t stride = a.out_stride;
    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    const std::true_type split{};
    const std::false_type hi_only{};
    // FP32: each step ends with both pairs renormalised (|lo| at most half an
    // ulp of hi), so hi alone is the pair rounded to T: the stages read x and
    // w, and during the step the low parts collect the increments, x's the
    // small part of dx (starting from both low parts), w's dw.
    if constexpr (COMP) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            T t = x[j] + xl[j];
            xl[j] = xl[j] - (t - x[j]);
            x[j] = t;
            t = w[j] + wl[j];
            wl[j] = wl[j] - (t - w[j]);
            w[j] = t;
        }
    }
    while (n < nend) {
        // the force's phase at the stage times (FP64), as scaled weights
        T c0 = T(0), ch = T(0), c1 = T(0);
        if constexpr (FORCED) {
            if (n % kAnchor == 0) ph.set(n);
            c0 = (T)ph.c;
            ph.half();
            ch = (T)ph.c;
            ph.half();
            c1 = (T)ph.c;
        }
        T R[DPL], d[DPL], Bd[DPL], kc[DPL];
        bop(split, x, R);   // B x
        // stage 1 at (x, w)
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            T k = fma_t(gm[j] * fma_t(-x[j], x[j], T(1)), w[j], -R[j]);
            if constexpr (FORCED) k = fma_t(fh[j], c0, k);
            kc[j] = k;
            xl[j] = fma_t(T(1.0 / 6.0), k, xl[j] + wl[j]);
            wl[j] = fma_t(T(1.0 / 6.0), k, wl[j]);
            d[j] = T(0.5) * w[j];   // d_2
        }
        // stages 2 and 3 at (x + d_k, w + k_{k-1}/2)
#pragma unroll
        for (int st = 2; st <= 3; ++st) {
            bop(hi_only, d, Bd);
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const T xt = x[j] + d[j];
                const T wt = fma_t(T(0.5), kc[j], w[j]);
                T k = fma_t(gm[j] * fma_t(-xt, xt, T(1)), wt, -(R[j] + Bd[j]));
                if constexpr (FORCED) k = fma_t(fh[j], ch, k);
                // d_3 = w/2 + k_1/4 = wt/2 (stage 2); d_4 = w + k_2/2 = wt (stage 3)
                d[j] = st == 2 ? T(0.5) * wt : wt;
                kc[j] = k;
                xl[j] = fma_t(T(1.0 / 6.0), k, xl[j]);
                wl[j] = fma_t(T(1.0 / 3.0), k, wl[j]);
            }
        }
        // stage 4 at (x + d_4, w + k_3)
        bop(hi_only, d, Bd);
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const T xt = x[j] + d[j];
            const T wt = w[j] + kc[j];
            T k = fma_t(gm[j] * fma_t(-xt, xt, T(1)), wt, -(R[j] + Bd[j]));
            if constexpr (FORCED) k = fma_t(fh[j], c1, k);
            wl[j] = fma_t(T(1.0 / 6.0), k, wl[j]);
            if constexpr (COMP) {
                // x += w (its exact error kept) + the collected part; renormalise both pairs
                T t = x[j] + w[j];
                xl[j] += w[j] - (t - x[j]);
                x[j] = t;
                t = x[j] + xl[j];
                xl[j] = xl[j] - (t - x[j]);
                x[j] = t;
                t = w[j] + wl[j];
                wl[j] = wl[j] - (t - w[j]);
                w[j] = t;
            } else {
                x[j] += w[j] + xl[j];
                w[j] += wl[j];
                xl[j] = T(0);
                wl[j] = T(0);
            }
        }
        ++n;
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }

    bool ok = true;
    const bool copy_input = untouched && a.nsteps == 0;
#pragma unroll
    for (int j = 0; j < DPL; ++j)
        if (active && d0 + j < s) ok = ok && __builtin_isfinite(x[j]) && __builtin_isfinite(w[j]);
    if (a.store_mode & STORE_STATE) {
        store(a.state, [&](int j) { return x[j]; });
        store(a.state + plane, [&](int j) { return xl[j]; });
        store(a.state + 2 * plane, [&](int j) { return w[j]; });
        store(a.state + 3 * plane, [&](int j) { return wl[j]; });
    }
    if (a.store_mode & STORE_USER) {
        if (a.xe) {
            if (copy_input) copy_out(a.xe, a.x0);
            else store(a.xe, xval);
        }
        if (a.ve) {
            if (copy_input) copy_out(a.ve, a.v0);
            else store(a.ve, vval);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

// Two waves per SIMD; one for FP64 with 16 DOFs per lane (its stage values
// do not fit half the registers).
template <typename T, int DPL, int LPI, bool FORCED>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 8 && DPL == 16) ? 1 : 2) vdp_chain_kernel(VdpLaunch<T> a) {
    vdp_chain_run<T, DPL, LPI, FORCED>(a, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

template <typename T, int DPL, int LPI, bool FORCED>
osc_status launch_layout(const VdpLaunch<T> &a, hipStream_t st) {
    const int64_t threads = a.batch * LPI;
    const unsigned blocks = (unsigned)((threads + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((vdp_chain_kernel<T, DPL, LPI, FORCED>), dim3(blocks), dim3(kThreads), 0, st, a);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace

// The kernels of one precision, with or without the force; each combination
// is instantiated in a file of its own (the forced and free FP32 kernels
// take different instruction schedules).
template <typename T, bool FORCED>
osc_status vdp_launch_as(const VdpLaunch<T> &a, hipStream_t st) {
    if (a.batch == 0) return OSC_OK;
    const int s = a.s;
    if (s <= 1) return launch_layout<T, 1, 1, FORCED>(a, st);
    if (s <= 2) return launch_layout<T, 2, 1, FORCED>(a, st);
    if (s <= 4) return launch_layout<T, 4, 1, FORCED>(a, st);
    if (s <= 8) return launch_layout<T, 8, 1, FORCED>(a, st);
    if (s <= 64) return launch_layout<T, 1, 64, FORCED>(a, st);
    if (s <= 128) return launch_layout<T, 2, 64, FORCED>(a, st);
    if (s <= 256) return launch_layout<T, 4, 64, FORCED>(a, st);
    if (s <= 512) return launch_layout<T, 8, 64, FORCED>(a, st);
    if (s <= 1024) return launch_layout<T, 16, 64, FORCED>(a, st);
    return fail(OSC_ENOTSUP, "Van der Pol chains take s <= 1024");
}

template <typename T>
osc_status vdp_launch(const VdpLaunch<T> &a, hipStream_t st) {
    return a.f ? vdp_launch_as<T, true>(a, st) : vdp_launch_as<T, false>(a, st);
}

}  // namespace osc
