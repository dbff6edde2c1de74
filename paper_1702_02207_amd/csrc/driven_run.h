// The damped, driven chain integrator in registers (the per-lane part of
// driven.hip's register kernel), shared with the resident real-time kernels
// (resident.hip).  The scheme and its arithmetic are described in driven.hip.

#pragma once

#include <cstdint>
#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

// Register layouts of the driven chain kernels: DOFs per lane and lanes per
// instance for s <= 1024 (false beyond).
inline bool driven_regs_layout(int s, int *dpl, int *lpi) {
    static const int caps[][3] = {{1, 1, 1}, {2, 2, 1}, {4, 4, 1}, {8, 8, 1}, {64, 1, 64},
                                  {128, 2, 64}, {256, 4, 64}, {512, 8, 64}, {1024, 16, 64}};
    for (const auto &c : caps)
        if (s <= c[0]) {
            *dpl = c[1];
            *lpi = c[2];
            return true;
        }
    return false;
}

// Chains in registers: one lane per instance (LPI = 1, s <= DPL) or one wave
// per instance (LPI = 64, DPL consecutive DOFs per lane, s <= 64 DPL).  The
// stencil's neighbouring values across lanes come from whole-wave DPP shifts
// (zero outside the wave: the wall, and beyond the free end, whose
// coefficient is zero); no LDS, no barrier.  The step is the recursion above:
// B x with split coefficients, B w, B z1_w, B z2_w and, with stiffness
// damping, B z3_w, four of the five stencils with the high coefficients only.
// The low parts of x and w collect the z terms as they are formed and one
// Kahan step per variable ends the step (FP64: a plain update).  Two waves
// per SIMD except for FP64 with 16 DOFs per lane (one).
// EX: bit 0 Rayleigh beta != 0 (the stiffness-proportional damping term),
// bit 1 a force; fixed per launch, so that each step is one basic block.
template <typename T, int DPL, int LPI, int EX>
__device__ __forceinline__ void driven_chain_run(const DrivenLaunch<T> &a, const int64_t g) {
    constexpr bool COMP = std::is_same<T, float>::value;
    const int64_t b = g / LPI;
    const int sl = (int)(g % LPI);
    const bool active = b < a.batch;
    const int s = a.s;
    const int d0 = sl * DPL;
    const size_t base = (size_t)(active ? b : 0) * s, plane = (size_t)a.batch * s;
    const double h = active ? a.h[b] : 1.0;
    const T dampw = (T)(a.alpha * h), dampb = (T)(a.beta / h);
    constexpr bool use_beta = (EX & 1) != 0, forced = (EX & 2) != 0;

    // A lane's DPL consecutive elements of a [batch][s] plane move as 16-byte
    // vectors when the run is whole and aligned, so that a wave's accesses
    // fill whole cache lines together instead of one element per line per
    // instruction.
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
    // element j of the lane's run is val(j), formed as it is stored
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

    T clh[DPL], crh[DPL], cll[DPL], crl[DPL], fh[DPL], x[DPL], xl[DPL], w[DPL], wl[DPL];
    load(a.c.clh, clh);
    load(a.c.crh, crh);
#pragma unroll
    for (int j = 0; j < DPL; ++j) cll[j] = crl[j] = fh[j] = T(0);
    if constexpr (COMP) {
        load(a.c.cll, cll);
        load(a.c.crl, crl);
    }
    if constexpr (forced) {
        double fd[DPL];
        load(a.f, fd);
#pragma unroll
        for (int j = 0; j < DPL; ++j) fh[j] = (T)(h * h * fd[j]);
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
    if constexpr (COMP) {
        // start from a normalised pair (the high part the rounded state)
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

    // neighbours of the lane's run: the left lane's last and the right lane's first value
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
            // the low coefficients' terms first, the dominant product last
            if constexpr (SPLIT) out[j] = fma_t(clh[j], el, fma_t(-crh[j], er, fma_t(cll[j], el, -crl[j] * er)));
            else out[j] = fma_t(clh[j], el, -crh[j] * er);
            el = er;
        }
    };

    Phase ph{};
    if (forced && active) ph.start(a.omega[b] * h, a.n0);
    auto xval = [&](int j) { return (T)((double)x[j] + (double)xl[j]); };
    auto vval = [&](int j) { return (T)(((double)w[j] + (double)wl[j]) / h); };
    // the caller's x0 / v0 unchanged (frame 0, nsteps = 0)
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
    auto steps = [&](auto beta_c, auto forced_c) {
        constexpr bool BETA = decltype(beta_c)::value, FORCED = decltype(forced_c)::value;
        const std::true_type split{};
        const std::false_type hi_only{};
        while (n < nend) {
            T g1 = T(0), g2 = T(0), g4 = T(0);
            if constexpr (FORCED) {
                if (n % kAnchor == 0) ph.set(n);
                const double c0 = ph.c;
                ph.half();
                const double ch = ph.c;
                ph.half();
                const double c1 = ph.c;
                g1 = (T)c0;
                g2 = (T)(2.0 * (ch - c0));
                g4 = (T)(4.0 * ((c0 - ch) + (c1 - ch)));
            }
            // z_{k+1,w} = -B z_{k,x} - a z_{k,w} - b B z_{k,w} + g e, with
            // z_{k,x} = z_{k-1,w}: Bp holds B z_{k,x}, V the new z_w
            T Bp[DPL], V[DPL], R[DPL];
            bop(split, x, R);     // B x
            bop(hi_only, w, Bp);  // B w = B z1_x
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                T v = fma_t(-dampw, w[j], -R[j]);
                if constexpr (BETA) v = fma_t(-dampb, Bp[j], v);
                if constexpr (FORCED) v = fma_t(fh[j], g1, v);
                V[j] = v;   // z1_w
                xl[j] = fma_t(T(0.5), v, xl[j]);
                wl[j] += v;
            }
            bop(hi_only, V, R);   // B z1_w = B z2_x
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                T v = fma_t(-dampw, V[j], -Bp[j]);
                if constexpr (BETA) v = fma_t(-dampb, R[j], v);
                if constexpr (FORCED) v = fma_t(fh[j], g2, v);
                V[j] = v;   // z2_w
                Bp[j] = R[j];
                xl[j] = fma_t(T(1.0 / 6.0), v, xl[j]);
                wl[j] = fma_t(T(0.5), v, wl[j]);
            }
            bop(hi_only, V, R);   // B z2_w = B z3_x
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                T v = fma_t(-dampw, V[j], -Bp[j]);
                if constexpr (BETA) v = fma_t(-dampb, R[j], v);
                V[j] = v;   // z3_w
                Bp[j] = R[j];
                xl[j] = fma_t(T(1.0 / 24.0), v, xl[j]);
                wl[j] = fma_t(T(1.0 / 6.0), v, wl[j]);
            }
            if constexpr (BETA) bop(hi_only, V, R);   // B z3_w
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                T v = fma_t(-dampw, V[j], -Bp[j]);
                if constexpr (BETA) v = fma_t(-dampb, R[j], v);
                if constexpr (FORCED) v = fma_t(fh[j], g4, v);
                wl[j] = fma_t(T(1.0 / 24.0), v, wl[j]);   // z4_w
                // x += w + (low part), w += (low part)
                const T y = w[j] + xl[j];
                if constexpr (COMP) {
                    T t = x[j] + y;
                    xl[j] = y - (t - x[j]);
                    x[j] = t;
                    t = w[j] + wl[j];
                    wl[j] = wl[j] - (t - w[j]);
                    w[j] = t;
                } else {
                    x[j] += y;
                    w[j] += wl[j];
                    xl[j] = T(0);
                    wl[j] = T(0);
                }
            }
            ++n;
            if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
        }
    };
    steps(std::integral_constant<bool, use_beta>{}, std::integral_constant<bool, forced>{});

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

}  // namespace
}  // namespace osc
