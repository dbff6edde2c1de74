// Batched integration of fixed-free spring chains (eq. (2) generalised to s
// bodies; s = 2 is the two-mass system itself) on gfx950.
//
// Layout.  A group of LPI consecutive lanes holds one instance; each lane
// keeps DPL consecutive degrees of freedom of that instance in registers for
// the whole launch.  LPI = 1 is the instance-per-lane layout (2-DOF
// ensembles), LPI = 64 one instance per 64-wide wavefront (long chains),
// LPI = 128 one instance over the two wavefronts of a workgroup (chains of
// 1025 to 2048 DOFs, which would not fit one wave's registers without
// spilling).  The only cross-lane traffic of the tridiagonal stencil is the
// edge value of each neighbouring lane, fetched with DPP whole-wave shifts
// (wave_shr:1 / wave_shl:1); only the two-wave layout also passes the two
// values across its wave boundary through LDS, with a workgroup barrier per
// product.  Many time steps run per launch; HBM is touched only to load the
// coefficients and state, to write frames and to store the final state.
//
// Arithmetic (scaled time tau = t/h, w = h v, B = h^2 A):
//   RK4.  For a linear autonomous system the classic four-stage RK4 map is
//   exactly the degree-4 Taylor polynomial of exp(hL), L = [[0, I], [-A, 0]]
//   (section 3's first-order form).  With P = Bx, Q = Bw, P2 = BP, Q2 = BQ:
//     dx = w - P/2 - Q/6 + P2/24,   dw = -P - Q/2 + P2/6 + Q2/24.
//   The stage form and this form differ only in rounding; this one keeps the
//   inexact constants 1/6 and 1/24 off the dominant terms.
//   Verlet.  Velocity Verlet written as leapfrog on the half-step velocity:
//     x_{n+1} = x_n + w_{n+1/2},  w_{n+3/2} = w_{n+1/2} - B x_{n+1},
//   with w_{1/2} = w_0 - B x_0 / 2 and w_n = w_{n+1/2} + B x_n / 2 at output.
//
// FP32 precision scheme: x and w are kept as an unevaluated sum hi + lo
// (compensated / Kahan update), and B x uses coefficients split into FP32
// hi + lo parts; the products with w, B x and B w, which enter the update
// multiplied by at least one more power of the small step, use hi only.
// FP64 runs the same code without the low parts.

//
// This header holds the per-lane integrator (chain_run) and the table of
// layouts; chain.hip launches it once per run, resident.hip once per
// real-time tick inside a resident kernel.

#pragma once

#include <cstdint>
#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {


template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    if constexpr (std::is_same<T, float>::value) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// FREE: the lane's last DOF is the chain's free end (LPI == 1 and s == DPL),
// whose right coefficient is exactly zero; its terms are then left out at
// compile time (same results: a product with +-0 added to a finite value).
template <typename T, int DPL, int LPI, bool FREE>
struct Group {
    bool first, last;   // lane is the first / last of its instance's group
    int sl;             // lane within the group
    // LPI == 128 (one instance over the two waves of a 128-thread workgroup):
    // the values across the wave boundary go through LDS, in two slots used
    // in turn, so that a slot is rewritten only after the barrier that
    // follows every read of it
    T *xch;
    mutable int slot;

    // Neighbouring values across the lane boundary: the last DOF of the left
    // lane and the first DOF of the right lane.  Outside the chain the wall
    // (left) is at rest; the free end (right) has a zero coefficient, the 0
    // only keeps the product finite.
    __device__ __forceinline__ void halo(const T (&u)[DPL], T &prev, T &next) const {
        if constexpr (LPI == 1) {
            prev = T(0);
            next = T(0);
        } else if constexpr (LPI == 64) {
            // the group is the whole wave: the shifts already bring in 0
            // (DPP folds into the extension's subtraction; no selects)
            prev = from_left<true>(u[DPL - 1]);
            next = from_right<true>(u[0]);
        } else if constexpr (LPI == 128) {
            T vp, vn;
            halo_pair(u, u, prev, next, vp, vn);
        } else {
            // groups inside the wave
            const T p = from_left<false>(u[DPL - 1]);
            const T n = from_right<false>(u[0]);
            prev = first ? T(0) : p;
            next = last ? T(0) : n;
        }
    }

    // The halos of two vectors at once: for LPI == 128 within each wave as
    // for LPI == 64, and across the boundary between the two waves through
    // LDS with one barrier for both (every lane of the workgroup passes the
    // barrier equally often: all run the same steps); otherwise two halos.
    __device__ __forceinline__ void halo_pair(const T (&u)[DPL], const T (&v)[DPL], T &up, T &un, T &vp,
                                              T &vn) const {
        if constexpr (LPI == 128) {
            up = from_left<true>(u[DPL - 1]);
            un = from_right<true>(u[0]);
            vp = from_left<true>(v[DPL - 1]);
            vn = from_right<true>(v[0]);
            T *const x = xch + 4 * slot;
            slot ^= 1;
            if (sl == 63) {
                x[0] = u[DPL - 1];
                x[2] = v[DPL - 1];
            }
            if (sl == 64) {
                x[1] = u[0];
                x[3] = v[0];
            }
            __syncthreads();
            if (sl == 64) {
                up = x[0];
                vp = x[2];
            }
            if (sl == 63) {
                un = x[1];
                vn = x[3];
            }
        } else {
            halo(u, up, un);
            halo(v, vp, vn);
        }
    }

    // out = B u with one coefficient set: (B u)_j = cl_j e_j - cr_j e_{j+1},
    // e_j = u_j - u_{j-1} the extension of spring j.
    __device__ __forceinline__ void apply(const T (&u)[DPL], const T (&cl)[DPL], const T (&cr)[DPL],
                                          T (&out)[DPL]) const {
        T prev, next;
        halo(u, prev, next);
        apply_h(u, prev, next, cl, cr, out);
    }
    // the same with the halo given
    __device__ __forceinline__ void apply_h(const T (&u)[DPL], const T prev, const T next, const T (&cl)[DPL],
                                            const T (&cr)[DPL], T (&out)[DPL]) const {
        T el = u[0] - prev;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            if (FREE && j == DPL - 1) {
                out[j] = cl[j] * el;
                continue;
            }
            const T un = (j + 1 < DPL) ? u[(j + 1 < DPL) ? j + 1 : j] : next;
            const T er = un - u[j];
            out[j] = fmat(cl[j], el, -cr[j] * er);
            el = er;
        }
    }

    // out = B u with split coefficients (hi + lo), the low products first.
    __device__ __forceinline__ void apply2(const T (&u)[DPL], const T (&clh)[DPL], const T (&crh)[DPL],
                                           const T (&cll)[DPL], const T (&crl)[DPL],
                                           T (&out)[DPL]) const {
        T prev, next;
        halo(u, prev, next);
        apply2_h(u, prev, next, clh, crh, cll, crl, out);
    }
    __device__ __forceinline__ void apply2_h(const T (&u)[DPL], const T prev, const T next,
                                             const T (&clh)[DPL], const T (&crh)[DPL], const T (&cll)[DPL],
                                             const T (&crl)[DPL], T (&out)[DPL]) const {
        T el = u[0] - prev;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            if (FREE && j == DPL - 1) {
                out[j] = fmat(clh[j], el, cll[j] * el);
                continue;
            }
            const T un = (j + 1 < DPL) ? u[(j + 1 < DPL) ? j + 1 : j] : next;
            const T er = un - u[j];
            out[j] = fmat(clh[j], el, fmat(-crh[j], er, fmat(cll[j], el, -crl[j] * er)));
            el = er;
        }
    }
};

// hi + lo <- hi + lo + y (compensated summation); FP64 adds directly.
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
__device__ __forceinline__ bool finite(T v) { return __builtin_isfinite(v); }

// One lane of the group that integrates instance b of launch a (sl = lane
// within the group).  Lanes of an instance outside the batch run on zeros so
// that their group still answers the DPP exchanges of a full wave.
template <typename T, int DPL, int LPI, int METHOD, bool FREE = false>
__device__ __forceinline__ void chain_run(const ChainLaunch<T> &a, const int64_t b, const int sl) {
    static_assert(!FREE || LPI == 1, "the free end is known at compile time only for one lane per instance");
    constexpr bool COMP = std::is_same<T, float>::value;
    const bool active = b < a.batch;
    const int s = a.s;
    const int d0 = sl * DPL;
    T *xch = nullptr;
    if constexpr (LPI == 128) {
        __shared__ T xch_buf[8];
        xch = xch_buf;
    }
    Group<T, DPL, LPI, FREE> grp{sl == 0, sl == LPI - 1, sl, xch, 0};

    T clh[DPL], crh[DPL], cll[DPL], crl[DPL];
    T x[DPL], xl[DPL], w[DPL], wl[DPL];
    const size_t base = (size_t)(active ? b : 0) * s;
    const double h = active ? a.c.h[b] : 1.0;
    const size_t plane = (size_t)a.batch * s;

    // A lane's DPL consecutive elements of a [batch][s] plane move as 16-byte
    // vectors when the run is whole and aligned, so that a wave's accesses
    // to a plane fill whole cache lines together instead of one element per
    // line per instruction (which lets lines leave the cache between the
    // instructions that share them).
    constexpr int V = 16 / (int)sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(V)));
    const bool run_whole = DPL % V == 0 && active && d0 + DPL <= s;
    auto aligned = [&](const T *p) { return run_whole && ((uintptr_t)(p + base + d0) % 16) == 0; };
    auto load = [&](const T *src, T (&dst)[DPL]) {
        if (aligned(src)) {
#pragma unroll
            for (int q = 0; q < DPL / V; ++q) {
                const vec_t v = *reinterpret_cast<const vec_t *>(src + base + d0 + q * V);
#pragma unroll
                for (int e = 0; e < V; ++e) dst[q * V + e] = v[e];
            }
        } else {
#pragma unroll
            for (int j = 0; j < DPL; ++j) dst[j] = (active && d0 + j < s) ? src[base + d0 + j] : T(0);
        }
    };
    auto store = [&](T *dst, const T (&src)[DPL]) {
        if (aligned(dst)) {
#pragma unroll
            for (int q = 0; q < DPL / V; ++q) {
                vec_t v;
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = src[q * V + e];
                *reinterpret_cast<vec_t *>(dst + base + d0 + q * V) = v;
            }
        } else {
#pragma unroll
            for (int j = 0; j < DPL; ++j)
                if (active && d0 + j < s) dst[base + d0 + j] = src[j];
        }
    };

    load(a.c.clh, clh);
    load(a.c.crh, crh);
#pragma unroll
    for (int j = 0; j < DPL; ++j) cll[j] = crl[j] = T(0);
    if constexpr (COMP) {
        load(a.c.cll, cll);
        load(a.c.crl, crl);
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

    const double invh = 1.0 / h;
    T P[DPL];   // Verlet: B x at the current full step
    if constexpr (METHOD == OSC_VERLET) {
        if constexpr (COMP) grp.apply2(x, clh, crh, cll, crl, P);
        else grp.apply(x, clh, crh, P);
        if (a.load_mode == LOAD_USER) {
#pragma unroll
            for (int j = 0; j < DPL; ++j) comp_add(w[j], wl[j], T(-0.5) * P[j]);   // w_{1/2}
        }
    }

    // velocity at the current full step, in FP64 before the final rounding
    auto vel = [&](int j) -> double {
        double wv = (double)w[j] + (double)wl[j];
        if constexpr (METHOD == OSC_VERLET) wv += 0.5 * (double)P[j];
        return wv * invh;
    };
    // the caller's initial state is copied out unchanged (frame 0, nsteps = 0)
    const bool untouched = a.load_mode == LOAD_USER;
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
        T o[DPL];
        if (a.xf) {
            if (initial) load(a.x0, o);
            else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) o[j] = (T)((double)x[j] + (double)xl[j]);
            }
            store(a.xf + fo, o);
        }
        if (a.vf) {
            if (initial) load(a.v0, o);
            else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) o[j] = (T)vel(j);
            }
            store(a.vf + fo, o);
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
        // FP32: the low parts collect the increments and are folded into the
        // high parts every kNorm steps (at fixed global step indices, so any
        // chunking of a run gives the same result); the products read
        // x = hi + lo and w = hi + lo rounded once per step.
        auto step = [&]() {
            T xe[DPL], we[DPL];
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                xe[j] = COMP ? x[j] + xl[j] : x[j];
                we[j] = COMP ? w[j] + wl[j] : w[j];
            }
            if constexpr (METHOD == OSC_RK4) {
                T Q[DPL];
                if constexpr (LPI == 128) {
                    // both halos across one barrier
                    T xprev, xnext, wprev, wnext;
                    grp.halo_pair(xe, we, xprev, xnext, wprev, wnext);
                    if constexpr (COMP) grp.apply2_h(xe, xprev, xnext, clh, crh, cll, crl, P);
                    else grp.apply_h(xe, xprev, xnext, clh, crh, P);
                    grp.apply_h(we, wprev, wnext, clh, crh, Q);
                } else {
                    if constexpr (COMP) grp.apply2(xe, clh, crh, cll, crl, P);
                    else grp.apply(xe, clh, crh, P);
                    grp.apply(we, clh, crh, Q);
                }
                // P2 = B P and Q2 = B Q, formed per DOF as they are consumed
                T pprev, pnext, qprev, qnext;
                grp.halo_pair(P, Q, pprev, pnext, qprev, qnext);
                T epl = P[0] - pprev, eql = Q[0] - qprev;
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const T pn = (j + 1 < DPL) ? P[(j + 1 < DPL) ? j + 1 : j] : pnext;
                    const T qn = (j + 1 < DPL) ? Q[(j + 1 < DPL) ? j + 1 : j] : qnext;
                    T P2, Q2;
                    if (FREE && j == DPL - 1) {
                        P2 = clh[j] * epl;
                        Q2 = clh[j] * eql;
                    } else {
                        const T epr = pn - P[j], eqr = qn - Q[j];
                        P2 = fmat(clh[j], epl, -crh[j] * epr);
                        Q2 = fmat(clh[j], eql, -crh[j] * eqr);
                        epl = epr;
                        eql = eqr;
                    }
                    T yx, yw;
                    rk4_increments(we[j], P[j], Q[j], P2, Q2, yx, yw);
                    if constexpr (COMP) {
                        xl[j] += yx;
                        wl[j] += yw;
                    } else {
                        x[j] += yx;
                        w[j] += yw;
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    if constexpr (COMP) xl[j] += we[j];
                    else x[j] += we[j];
                    xe[j] = COMP ? x[j] + xl[j] : x[j];
                }
                if constexpr (COMP) grp.apply2(xe, clh, crh, cll, crl, P);
                else grp.apply(xe, clh, crh, P);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    if constexpr (COMP) wl[j] -= P[j];
                    else w[j] -= P[j];
                }
            }
        };
        // hi + lo <- the same sum with |lo| below half an ulp of hi (exact)
        auto renorm = [&]() {
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                T t = x[j] + xl[j];
                xl[j] = xl[j] - (t - x[j]);
                x[j] = t;
                t = w[j] + wl[j];
                wl[j] = wl[j] - (t - w[j]);
                w[j] = t;
            }
        };
        // 32-bit trip counts keep the loop test on the scalar unit; two
        // steps per trip halve the loop overhead.  Fold period: the rounding
        // of lo grows with the increments it has collected.  One instance per
        // lane (s <= 8) folds every 4 steps: with so few DOFs nothing averages
        // that rounding out of the energy (two-mass ensemble, 10^4 steps:
        // drift 8.7e-7 against ~1.2e-6 at 8).  Longer chains fold every 8.
        constexpr int64_t kNorm = COMP ? (LPI == 1 ? 4 : 8) : (int64_t(1) << 30);
        int64_t g = n;   // global index of the next step
        for (int64_t left = stop - n; left > 0;) {
            const int64_t to_norm = kNorm - g % kNorm;
            const int cnt = (int)(left < to_norm ? left : to_norm);
            int k = 0;
            for (; k + 2 <= cnt; k += 2) {
                step();
                step();
            }
            if (k < cnt) step();
            g += cnt;
            left -= cnt;
            if (COMP && g % kNorm == 0) renorm();
        }
        n = stop;
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }
    const bool copy_input = untouched && a.nsteps == 0;

    bool ok = true;
#pragma unroll
    for (int j = 0; j < DPL; ++j)
        if (active && d0 + j < s) ok = ok && finite(x[j]) && finite(w[j]);
    if (a.store_mode & STORE_STATE) {
        store(a.state, x);
        store(a.state + plane, xl);
        store(a.state + 2 * plane, w);
        store(a.state + 3 * plane, wl);
    }
    if (a.store_mode & STORE_USER) {
        T o[DPL];
        if (a.xe) {
            if (copy_input) load(a.x0, o);
            else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) o[j] = (T)((double)x[j] + (double)xl[j]);
            }
            store(a.xe, o);
        }
        if (a.ve) {
            if (copy_input) load(a.v0, o);
            else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) o[j] = (T)vel(j);
            }
            store(a.ve, o);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

// --------------------------------------------------------------------------
// configuration table
// --------------------------------------------------------------------------
struct Entry {
    int lpi, dpl;
};
constexpr Entry kConfigs[] = {
    {1, 1}, {1, 2}, {1, 3}, {1, 4}, {1, 5}, {1, 6}, {1, 7}, {1, 8},
    {2, 8}, {4, 8}, {8, 8}, {16, 8}, {32, 8},
    {64, 4}, {64, 8}, {64, 16}, {128, 16},
};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

}  // namespace
}  // namespace osc
