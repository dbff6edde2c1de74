// Damped and driven systems: eq. (1) with Rayleigh damping C = alpha M +
// beta K and a harmonic force F cos(Omega t),
//     M x'' + C x' + K x = F cos(Omega t),
// advanced by classic RK4 on the first-order form of section 3 (stages at
// t_n, t_n + h/2, t_n + h/2, t_n + h).  In scaled time tau = t/h, w = h v,
// B = h^2 A, f = M^-1 F the stage slope of w is
//     kw = -B X - (alpha h) W - (beta / h) B W + h^2 f cos(Omega t).
// One 256-thread workgroup per instance; thread t owns DOFs t, t + 256, ...
// in registers.  Each stage writes its arguments (X, W) to LDS, in two
// buffers used in turn, so that one barrier per stage separates the writes
// from the reads of the products (the buffer written by a stage was last read
// two stages earlier, before the barrier in between).  Chains take the
// three-point stencil from LDS; dense systems stream the column-major operator.
//
// FP32: x and w are kept as hi + lo (Kahan update every step); B X uses the
// operator split into high and low parts, B W the high part (it enters
// smaller by h omega).  The stage arguments are X_s = x + c_s kx, W_s = w +
// c_s kw, and the increments are summed with the dominant term last:
//     dx = w + (kw1 + kw2 + kw3) / 6,   dw = (kw1 + kw4 + 2 (kw2 + kw3)) / 6.
// The force's phase is a rotation in FP64, set exactly (sincos of Omega h n)
// at every global step index divisible by 64 and advanced by half-step
// rotations in between, so that chunked and unchunked runs agree bitwise.
// Chains of s <= 1024 take a register-resident kernel instead (below).

#include <cmath>
#include <type_traits>

#include "osc_internal.h"

namespace osc {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kAnchor = 64;

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

// cos / sin of the force's phase at the current half step
struct Phase {
    double c, s;     // e^{i Omega h tau}
    double rc, rs;   // e^{i Omega h / 2}
    double wh;       // Omega h
    __device__ void set(int64_t n) {
        sincos(wh * (double)n, &s, &c);
    }
    // The rounding is spelled out (one product, then one fused
    // multiply-add) so that every inlined copy, in and out of the step loop,
    // computes bit for bit the same rotation.
    __device__ void half() {
        const double nc = __builtin_fma(c, rc, -(s * rs)), ns = __builtin_fma(s, rc, c * rs);
        c = nc;
        s = ns;
    }
};

template <typename T, int RPT, int KIND>
__global__ void __launch_bounds__(kThreads) driven_kernel(DrivenLaunch<T> a) {
    extern __shared__ unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr bool COMP = std::is_same<T, float>::value;
    const int64_t b = blockIdx.x;
    const int s = a.s;
    const int tid = threadIdx.x;
    const size_t base = (size_t)b * s, plane = (size_t)a.batch * s;
    const int64_t sys = a.shared ? 0 : b;
    const double h = a.h[sys];
    const T dampw = (T)(a.alpha * h), dampb = (T)(a.beta / h);
    const bool use_beta = a.beta != 0.0;
    // LDS: two buffers of [X | W], each s + 2 long (chains read a zero on
    // both sides: the wall, and the free end's coefficient is zero)
    const int pitch = s + 2;
    T *buf[2] = {lds, a.nbuf == 2 ? lds + 2 * pitch : lds};

    // coefficients of the owned rows
    T clh[RPT], crh[RPT], cll[RPT], crl[RPT], fh[RPT];
    T x[RPT], xl[RPT], w[RPT], wl[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = tid + r * kThreads;
        const bool own = i < s;
        clh[r] = crh[r] = cll[r] = crl[r] = T(0);
        if constexpr (KIND == OSC_CHAIN) {
            if (own) {
                clh[r] = a.c.clh[base + i];
                crh[r] = a.c.crh[base + i];
                if constexpr (COMP) {
                    cll[r] = a.c.cll[base + i];
                    crl[r] = a.c.crl[base + i];
                }
            }
        }
        fh[r] = (own && a.f) ? (T)(h * h * a.f[base + i]) : T(0);
        if (a.load_mode == LOAD_USER) {
            x[r] = own ? a.x0[base + i] : T(0);
            xl[r] = T(0);
            const double wd = own ? h * (double)a.v0[base + i] : 0.0;
            w[r] = (T)wd;
            wl[r] = COMP ? (T)(wd - (double)w[r]) : T(0);
        } else {
            x[r] = own ? a.state[base + i] : T(0);
            xl[r] = own ? a.state[plane + base + i] : T(0);
            w[r] = own ? a.state[2 * plane + base + i] : T(0);
            wl[r] = own ? a.state[3 * plane + base + i] : T(0);
        }
    }
    if (tid == 0) {
        for (int q = 0; q < a.nbuf; ++q) {
            buf[q][0] = buf[q][s + 1] = T(0);
            buf[q][pitch] = buf[q][pitch + s + 1] = T(0);
        }
    }

    const T *Bh = KIND == OSC_DENSE ? a.Bh + (size_t)sys * s * s : nullptr;
    const T *Bl = (KIND == OSC_DENSE && COMP) ? a.Bl + (size_t)sys * s * s : nullptr;
    // (B u)_row from LDS u (offset 1); split: hi + lo parts of the operator
    auto bop = [&](const T *u, int r, bool split) -> T {
        const int i = tid + r * kThreads;
        if constexpr (KIND == OSC_CHAIN) {
            const T el = u[i + 1] - u[i], er = u[i + 2] - u[i + 1];
            T p = fma_t(clh[r], el, -crh[r] * er);
            if (COMP && split) p += fma_t(cll[r], el, -crl[r] * er);
            return p;
        } else {
            T hi = T(0), lo = T(0);
            for (int j = 0; j < s; ++j) {
                const T uj = u[j + 1];
                hi = fma_t(Bh[(size_t)j * s + i], uj, hi);
                if (COMP && split) lo = fma_t(Bl[(size_t)j * s + i], uj, lo);
            }
            return hi + lo;
        }
    };

    Phase ph{};
    const bool forced = a.f != nullptr;
    if (forced) {
        const double wh = a.omega[b] * h;
        ph.wh = wh;
        sincos(0.5 * wh, &ph.rs, &ph.rc);
        const int64_t anchor = a.n0 - a.n0 % kAnchor;
        ph.set(anchor);
        for (int64_t q = anchor; q < a.n0; ++q) {
            ph.half();
            ph.half();
        }
    }

    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + r * kThreads;
            if (i >= s) continue;
            if (a.xf) a.xf[fo + base + i] = initial ? a.x0[base + i] : (T)((double)x[r] + (double)xl[r]);
            if (a.vf) a.vf[fo + base + i] = initial ? a.v0[base + i] : (T)(((double)w[r] + (double)wl[r]) / h);
        }
    };

    int cur = 0;   // LDS buffer of the next stage
    const bool single = a.nbuf == 1;
    // one stage: publish (X, W), then kw = F(X, W) at the given force value
    auto stage = [&](const T (&X)[RPT], const T (&W)[RPT], T force, T (&kw)[RPT]) {
        T *ux = buf[cur], *uw = buf[cur] + pitch;
        if (single) __syncthreads();   // one buffer: every read of the previous stage is done
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + r * kThreads;
            if (i < s) {
                ux[i + 1] = X[r];
                uw[i + 1] = W[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + r * kThreads;
            if (i >= s) {
                kw[r] = T(0);
                continue;
            }
            T acc = -bop(ux, r, true);
            if (use_beta) acc = fma_t(-dampb, bop(uw, r, false), acc);
            acc = fma_t(-dampw, W[r], acc);
            if (forced) acc = fma_t(fh[r], force, acc);
            kw[r] = acc;
        }
        if (!single) cur ^= 1;
    };

    const bool untouched = a.load_mode == LOAD_USER;
    const int64_t stride = a.out_stride;
    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    while (n < nend) {
        if (forced && n % kAnchor == 0) ph.set(n);
        const T f0 = (T)ph.c;
        if (forced) ph.half();
        const T fhalf = (T)ph.c;
        if (forced) ph.half();
        const T f1 = (T)ph.c;
        T xe[RPT], we[RPT], X[RPT], W[RPT], k1[RPT], k2[RPT], k3[RPT], k4[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            xe[r] = COMP ? x[r] + xl[r] : x[r];
            we[r] = COMP ? w[r] + wl[r] : w[r];
        }
        stage(xe, we, f0, k1);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            X[r] = fma_t(T(0.5), we[r], xe[r]);
            W[r] = fma_t(T(0.5), k1[r], we[r]);
        }
        stage(X, W, fhalf, k2);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            X[r] = fma_t(T(0.5), W[r], xe[r]);
            W[r] = fma_t(T(0.5), k2[r], we[r]);
        }
        stage(X, W, fhalf, k3);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            X[r] = xe[r] + W[r];
            W[r] = we[r] + k3[r];
        }
        stage(X, W, f1, k4);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const T dx = fma_t(T(1.0 / 6.0), k1[r] + k2[r] + k3[r], we[r]);
            const T dw = (k1[r] + k4[r] + T(2) * (k2[r] + k3[r])) * T(1.0 / 6.0);
            comp_add(x[r], xl[r], dx);
            comp_add(w[r], wl[r], dw);
        }
        ++n;
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }

    bool ok = true;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
        if (tid + r * kThreads < s) ok = ok && __builtin_isfinite(x[r]) && __builtin_isfinite(w[r]);
    const bool copy_input = untouched && a.nsteps == 0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = tid + r * kThreads;
        if (i >= s) continue;
        if (a.store_mode & STORE_STATE) {
            a.state[base + i] = x[r];
            a.state[plane + base + i] = xl[r];
            a.state[2 * plane + base + i] = w[r];
            a.state[3 * plane + base + i] = wl[r];
        }
        if (a.store_mode & STORE_USER) {
            if (a.xe) a.xe[base + i] = copy_input ? a.x0[base + i] : (T)((double)x[r] + (double)xl[r]);
            if (a.ve) a.ve[base + i] = copy_input ? a.v0[base + i] : (T)(((double)w[r] + (double)wl[r]) / h);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

// Chains in registers: one lane per instance (LPI = 1, s <= DPL) or one wave
// per instance (LPI = 64, DPL consecutive DOFs per lane, s <= 64 DPL).  The
// stencil's neighbouring values across lanes come from whole-wave DPP shifts
// (zero outside the wave: the wall, and beyond the free end, whose
// coefficient is zero); no LDS, no barrier.  Same stage form and force phase
// as the workgroup kernel; the state is updated by a Kahan sum every step, so
// its high part is the rounded state itself.
// At least two waves per SIMD except for FP64 with 16 DOFs per lane: the
// FP32 16-DOF kernel then spills ~20 registers to scratch and still runs
// 1.8x faster than at one wave per SIMD; the FP64 one would spill ~370.
// EX: bit 0 Rayleigh beta != 0 (the stiffness-proportional damping term),
// bit 1 a force; fixed per launch, so that each step is one basic block.
template <typename T, int DPL, int LPI, int EX>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 8 && DPL == 16) ? 1 : 2)
    driven_chain_kernel(DrivenLaunch<T> a) {
    constexpr bool COMP = std::is_same<T, float>::value;
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t b = g / LPI;
    const int sl = (int)(g % LPI);
    const bool active = b < a.batch;
    const int s = a.s;
    const int d0 = sl * DPL;
    const size_t base = (size_t)(active ? b : 0) * s, plane = (size_t)a.batch * s;
    const double h = active ? a.h[b] : 1.0;
    const T dampw = (T)(a.alpha * h), dampb = (T)(a.beta / h);
    constexpr bool use_beta = (EX & 1) != 0, forced = (EX & 2) != 0;

    T clh[DPL], crh[DPL], cll[DPL], crl[DPL], fh[DPL], x[DPL], xl[DPL], w[DPL], wl[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const bool own = active && d0 + j < s;
        const size_t i = base + d0 + j;
        clh[j] = own ? a.c.clh[i] : T(0);
        crh[j] = own ? a.c.crh[i] : T(0);
        cll[j] = (own && COMP) ? a.c.cll[i] : T(0);
        crl[j] = (own && COMP) ? a.c.crl[i] : T(0);
        fh[j] = (own && forced) ? (T)(h * h * a.f[i]) : T(0);
        if (a.load_mode == LOAD_USER) {
            x[j] = own ? a.x0[i] : T(0);
            xl[j] = T(0);
            const double wd = own ? h * (double)a.v0[i] : 0.0;
            w[j] = (T)wd;
            wl[j] = COMP ? (T)(wd - (double)w[j]) : T(0);
        } else {
            x[j] = own ? a.state[i] : T(0);
            xl[j] = own ? a.state[plane + i] : T(0);
            w[j] = own ? a.state[2 * plane + i] : T(0);
            wl[j] = own ? a.state[3 * plane + i] : T(0);
        }
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
    // kw = -B X (split) - a W - b B W + f c; BETA and FORCED are fixed for
    // the whole launch and compiled in, so that the step is one basic block
    auto slope = [&](auto beta_c, auto forced_c, const T (&X)[DPL], const T (&W)[DPL], T force, T (&kw)[DPL]) {
        constexpr bool BETA = decltype(beta_c)::value, FORCED = decltype(forced_c)::value;
        T xp, xn;
        halo(X, xp, xn);
        T wp = T(0), wn = T(0);
        if constexpr (BETA) halo(W, wp, wn);
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const T xm = j > 0 ? X[j > 0 ? j - 1 : 0] : xp, xr = j + 1 < DPL ? X[j + 1 < DPL ? j + 1 : j] : xn;
            const T el = X[j] - xm, er = xr - X[j];
            T p = fma_t(clh[j], el, -crh[j] * er);
            if constexpr (COMP) p += fma_t(cll[j], el, -crl[j] * er);
            T acc = -p;
            if constexpr (BETA) {
                const T wm = j > 0 ? W[j > 0 ? j - 1 : 0] : wp, wr = j + 1 < DPL ? W[j + 1 < DPL ? j + 1 : j] : wn;
                const T q = fma_t(clh[j], W[j] - wm, -crh[j] * (wr - W[j]));
                acc = fma_t(-dampb, q, acc);
            }
            acc = fma_t(-dampw, W[j], acc);
            if constexpr (FORCED) acc = fma_t(fh[j], force, acc);
            kw[j] = acc;
        }
    };

    Phase ph{};
    if (forced && active) {
        const double wh = a.omega[b] * h;
        ph.wh = wh;
        sincos(0.5 * wh, &ph.rs, &ph.rc);
        const int64_t anchor = a.n0 - a.n0 % kAnchor;
        ph.set(anchor);
        for (int64_t q = anchor; q < a.n0; ++q) {
            ph.half();
            ph.half();
        }
    }
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * plane;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            if (!(active && d0 + j < s)) continue;
            const size_t i = base + d0 + j;
            if (a.xf) a.xf[fo + i] = initial ? a.x0[i] : (T)((double)x[j] + (double)xl[j]);
            if (a.vf) a.vf[fo + i] = initial ? a.v0[i] : (T)(((double)w[j] + (double)wl[j]) / h);
        }
    };

    const bool untouched = a.load_mode == LOAD_USER;
    const int64_t stride = a.out_stride;
    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    auto steps = [&](auto beta_c, auto forced_c) {
        constexpr bool FORCED = decltype(forced_c)::value;
        while (n < nend) {
            if (FORCED && n % kAnchor == 0) ph.set(n);
            const T f0 = (T)ph.c;
            if (FORCED) ph.half();
            const T fhalf = (T)ph.c;
            if (FORCED) ph.half();
            const T f1 = (T)ph.c;
            if constexpr (COMP) {
                // The stages read only the high parts, so the low parts collect
                // the step's slope terms as they are formed (smallest first):
                //   dx = w + (k1 + k2 + k3) / 6,  dw = (k1 + 2 k2 + 2 k3 + k4) / 6
                // and one Kahan step per variable adds them at the end; no
                // per-DOF partial sums stay live across the stages.
                T X[DPL], W[DPL], k[DPL];
                slope(beta_c, forced_c, x, w, f0, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    X[j] = fma_t(T(0.5), w[j], x[j]);
                    W[j] = fma_t(T(0.5), k[j], w[j]);
                    xl[j] = fma_t(T(1.0 / 6.0), k[j], xl[j]);
                    wl[j] = fma_t(T(1.0 / 6.0), k[j], wl[j]);
                }
                slope(beta_c, forced_c, X, W, fhalf, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    X[j] = fma_t(T(0.5), W[j], x[j]);
                    W[j] = fma_t(T(0.5), k[j], w[j]);
                    xl[j] = fma_t(T(1.0 / 6.0), k[j], xl[j]);
                    wl[j] = fma_t(T(1.0 / 3.0), k[j], wl[j]);
                }
                slope(beta_c, forced_c, X, W, fhalf, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    X[j] = x[j] + W[j];
                    W[j] = w[j] + k[j];
                    xl[j] = fma_t(T(1.0 / 6.0), k[j], xl[j]);
                    wl[j] = fma_t(T(1.0 / 3.0), k[j], wl[j]);
                }
                slope(beta_c, forced_c, X, W, f1, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    wl[j] = fma_t(T(1.0 / 6.0), k[j], wl[j]);
                    const T y = w[j] + xl[j];
                    T t = x[j] + y;
                    xl[j] = y - (t - x[j]);
                    x[j] = t;
                    t = w[j] + wl[j];
                    wl[j] = wl[j] - (t - w[j]);
                    w[j] = t;
                }
            } else {
                T X[DPL], W[DPL], k[DPL], sx[DPL], sw[DPL];
                slope(beta_c, forced_c, x, w, f0, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    sx[j] = k[j];
                    sw[j] = k[j];
                    X[j] = fma_t(T(0.5), w[j], x[j]);
                    W[j] = fma_t(T(0.5), k[j], w[j]);
                }
                slope(beta_c, forced_c, X, W, fhalf, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    sx[j] += k[j];
                    sw[j] = fma_t(T(2), k[j], sw[j]);
                    X[j] = fma_t(T(0.5), W[j], x[j]);
                    W[j] = fma_t(T(0.5), k[j], w[j]);
                }
                slope(beta_c, forced_c, X, W, fhalf, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    sx[j] += k[j];
                    sw[j] = fma_t(T(2), k[j], sw[j]);
                    X[j] = x[j] + W[j];
                    W[j] = w[j] + k[j];
                }
                slope(beta_c, forced_c, X, W, f1, k);
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    x[j] += fma_t(T(1.0 / 6.0), sx[j], w[j]);
                    w[j] += (sw[j] + k[j]) * T(1.0 / 6.0);
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
    for (int j = 0; j < DPL; ++j) {
        if (!(active && d0 + j < s)) continue;
        const size_t i = base + d0 + j;
        ok = ok && __builtin_isfinite(x[j]) && __builtin_isfinite(w[j]);
        if (a.store_mode & STORE_STATE) {
            a.state[i] = x[j];
            a.state[plane + i] = xl[j];
            a.state[2 * plane + i] = w[j];
            a.state[3 * plane + i] = wl[j];
        }
        if (a.store_mode & STORE_USER) {
            if (a.xe) a.xe[i] = copy_input ? a.x0[i] : (T)((double)x[j] + (double)xl[j]);
            if (a.ve) a.ve[i] = copy_input ? a.v0[i] : (T)(((double)w[j] + (double)wl[j]) / h);
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

template <typename T, int DPL, int LPI>
osc_status launch_chain_regs(const DrivenLaunch<T> &a, hipStream_t st) {
    const int64_t threads = a.batch * LPI;
    const unsigned blocks = (unsigned)((threads + kThreads - 1) / kThreads);
    const int ex = (a.beta != 0.0 ? 1 : 0) | (a.f ? 2 : 0);
    if (ex == 0) hipLaunchKernelGGL((driven_chain_kernel<T, DPL, LPI, 0>), dim3(blocks), dim3(kThreads), 0, st, a);
    else if (ex == 1) hipLaunchKernelGGL((driven_chain_kernel<T, DPL, LPI, 1>), dim3(blocks), dim3(kThreads), 0, st, a);
    else if (ex == 2) hipLaunchKernelGGL((driven_chain_kernel<T, DPL, LPI, 2>), dim3(blocks), dim3(kThreads), 0, st, a);
    else hipLaunchKernelGGL((driven_chain_kernel<T, DPL, LPI, 3>), dim3(blocks), dim3(kThreads), 0, st, a);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

// chains of s <= 1024 in registers; 0 when the workgroup kernel takes them
template <typename T>
osc_status launch_chain_regs_for(const DrivenLaunch<T> &a, hipStream_t st, bool *done) {
    *done = true;
    const int s = a.s;
    if (s <= 1) return launch_chain_regs<T, 1, 1>(a, st);
    if (s <= 2) return launch_chain_regs<T, 2, 1>(a, st);
    if (s <= 4) return launch_chain_regs<T, 4, 1>(a, st);
    if (s <= 8) return launch_chain_regs<T, 8, 1>(a, st);
    if (s <= 64) return launch_chain_regs<T, 1, 64>(a, st);
    if (s <= 128) return launch_chain_regs<T, 2, 64>(a, st);
    if (s <= 256) return launch_chain_regs<T, 4, 64>(a, st);
    if (s <= 512) return launch_chain_regs<T, 8, 64>(a, st);
    if (s <= 1024) return launch_chain_regs<T, 16, 64>(a, st);
    *done = false;
    return OSC_OK;
}

template <typename T, int KIND>
osc_status launch_kind(const DrivenLaunch<T> &a, hipStream_t st) {
    const size_t lds = 2 * (size_t)a.nbuf * (a.s + 2) * sizeof(T);
    const dim3 grid((unsigned)a.batch), block(kThreads);
    const int rpt = (a.s + kThreads - 1) / kThreads;
    if (rpt <= 1) hipLaunchKernelGGL((driven_kernel<T, 1, KIND>), grid, block, lds, st, a);
    else if (rpt <= 2) hipLaunchKernelGGL((driven_kernel<T, 2, KIND>), grid, block, lds, st, a);
    else if (rpt <= 4) hipLaunchKernelGGL((driven_kernel<T, 4, KIND>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((driven_kernel<T, 8, KIND>), grid, block, lds, st, a);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

// f = F / m for chains
__global__ void __launch_bounds__(kThreads) chain_force_kernel(int64_t n, const double *F, const double *m,
                                                               double *f) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) f[i] = F[i] / m[i];
}

}  // namespace

template <typename T>
osc_status driven_launch(const DrivenLaunch<T> &in, hipStream_t st) {
    if (in.batch == 0) return OSC_OK;
    if (in.s < 1 || in.s > 2048) return fail(OSC_ENOTSUP, "damped / driven systems take s <= 2048");
    if (in.batch > 0x7fffffff) return fail(OSC_EINVAL, "too many instances for one launch");
    DrivenLaunch<T> a = in;
    if (a.kind == OSC_CHAIN && !a.force_workgroup) {
        bool done = false;
        osc_status r = launch_chain_regs_for<T>(a, st, &done);
        if (r || done) return r;
    }
    // two stage buffers when they fit 64 KB of LDS, else one
    a.nbuf = 4 * (size_t)(a.s + 2) * sizeof(T) <= 65536 ? 2 : 1;
    return a.kind == OSC_CHAIN ? launch_kind<T, OSC_CHAIN>(a, st) : launch_kind<T, OSC_DENSE>(a, st);
}
template osc_status driven_launch<float>(const DrivenLaunch<float> &, hipStream_t);
template osc_status driven_launch<double>(const DrivenLaunch<double> &, hipStream_t);

__global__ void __launch_bounds__(kThreads) eye_kernel(int64_t nsys, int s, double *I) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx < nsys * s * s) I[idx] = (idx / s % s) == (idx % s) ? 1.0 : 0.0;
}

osc_status dense_force(int s, int64_t nsys, int64_t batch, const double *M, const double *F, double *f,
                       int *notspd, hipStream_t st) {
    if (batch == 0) return OSC_OK;
    const size_t ss = (size_t)s * s;
    struct Tmp {
        hipStream_t st;
        void *p[4] = {};
        ~Tmp() {
            (void)hipStreamSynchronize(st);
            for (void *q : p) pool_free(q);
        }
    } t{st};
    t.p[0] = pool_alloc(nsys * ss * sizeof(double));                              // I, then M^-1
    t.p[1] = pool_alloc(nsys * ss * sizeof(double));                              // Cholesky factor
    t.p[2] = pool_alloc(nsys * dense_form_scratch_elems(s) * sizeof(double));     // inverted blocks
    t.p[3] = pool_alloc(nsys * ss * sizeof(double));                              // M^-1
    for (void *q : t.p)
        if (!q) return fail(OSC_ENOMEM, "device memory exhausted for M^-1 F");
    const int64_t total = nsys * (int64_t)ss;
    hipLaunchKernelGGL(eye_kernel, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, nsys,
                       s, static_cast<double *>(t.p[0]));
    OSC_HIP(hipGetLastError());
    osc_status r = dense_form_a(s, nsys, M, static_cast<double *>(t.p[0]), static_cast<double *>(t.p[1]),
                                static_cast<double *>(t.p[2]), static_cast<double *>(t.p[3]), notspd, st);
    if (r) return r;
    // f_b = M^-1 F_b: rows of F times (M^-1)^T
    Gemm64 g{};
    g.overwrite = 1;
    g.n = g.k = s;
    g.A = F, g.a_i = s, g.a_p = 1;
    g.B = static_cast<const double *>(t.p[3]), g.b_p = 1, g.b_j = s;
    g.C = f, g.c_i = s, g.c_j = 1;
    int64_t n = 1;
    if (nsys == 1) {
        g.m = (int)batch;
    } else {
        g.m = 1;
        g.a_sys = g.c_sys = s;
        g.b_sys = ss;
        n = batch;
    }
    return gemm64(g, n, st);
}

osc_status chain_force(int64_t n, const double *F, const double *m, double *f, hipStream_t st) {
    if (n == 0) return OSC_OK;
    hipLaunchKernelGGL(chain_force_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, n,
                       F, m, f);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace osc
