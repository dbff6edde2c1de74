// Damped and driven systems: eq. (1) with Rayleigh damping C = alpha M +
// beta K and a harmonic force F cos(Omega t),
//     M x'' + C x' + K x = F cos(Omega t),
// advanced by classic RK4 on the first-order form of section 3 (stages at
// t_n, t_n + h/2, t_n + h/2, t_n + h).  In scaled time tau = t/h, w = h v,
// B = h^2 A, f = M^-1 F the stage slope of w is
//     kw = -B X - (alpha h) W - (beta / h) B W + h^2 f cos(Omega t).
// The system is linear with constant coefficients (only the force depends on
// t), so the four stages sum to a four-level recursion: with y = (x, w),
// L y = (w, -B x - a w - b B w) (a = alpha h, b = beta / h), e = (0, h^2 f)
// and the force phases c0, ch, ch, c1 of the stages,
//     y_{n+1} = y + z1 + z2/2 + z3/6 + z4/24,   z1 = L y + g1 e,
//     z_k = L z_{k-1} + g_k e,  g1 = c0, g2 = 2 (ch - c0), g3 = 0,
//     g4 = 4 (c0 - 2 ch + c1)
// (expand k1..k4 and match the coefficients of L^j e).  The x-part of z_k is
// the w-part of z_{k-1}, so B of it is already known: a step takes B x (split
// coefficients in FP32: the dominant term), B w and B of three w-parts (the
// last only with stiffness damping) -- five products against the stage
// form's eight.  The g_k are formed in FP64 from the FP64 phase.
//
// Two kernels run this step.  One 256-thread workgroup per instance (dense
// systems and chains of up to 2048 DOFs): thread t owns DOFs t, t + 256, ...
// in registers; each level publishes its operand to LDS, in two buffers used
// in turn, so that one barrier per level separates the writes from the reads
// of the products (the buffer written by a level was last read two levels
// earlier, before the barrier in between); chains take the three-point
// stencil from LDS, dense systems stream the column-major operator.  Chains
// of s <= 1024 take a register-resident kernel instead (below).  Shared dense
// operators in FP32 run on the matrix cores (dense_mfma.hip).
//
// FP32: x and w are kept as hi + lo (Kahan update every step); the low parts
// or per-DOF sums collect the z terms, the dominant term added last.  The
// force's phase is the FP64 rotation of osc_internal.h (Phase), set exactly
// at every global step index divisible by 64, so chunked and unchunked runs
// agree bitwise.

#include <cmath>
#include <type_traits>

#include "driven_run.h"

namespace osc {
namespace {

constexpr int kThreads = 256;

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
    if (forced) ph.start(a.omega[b] * h, a.n0);

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

    int cur = 0;   // LDS buffer of the next publication
    const bool single = a.nbuf == 1;
    // publish U (and V into the buffer's second half when given) for the
    // products of the next level
    auto publish = [&](const T (&U)[RPT], const T *V) {
        T *ux = buf[cur], *uw = buf[cur] + pitch;
        if (single) __syncthreads();   // one buffer: every read of the previous level is done
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + r * kThreads;
            if (i < s) {
                ux[i + 1] = U[r];
                if (V) uw[i + 1] = V[r];
            }
        }
        __syncthreads();
        T *out = buf[cur];
        if (!single) cur ^= 1;
        return out;
    };

    const bool untouched = a.load_mode == LOAD_USER;
    const int64_t stride = a.out_stride;
    int64_t n = a.n0;
    const int64_t nend = a.n0 + a.nsteps;
    if (stride > 0 && untouched && n % stride == 0) write_frame(n / stride, true);
    while (n < nend) {
        // the RK4 map as the four-level recursion of the register kernel
        // below: z1 = L y + g1 e, z_k = L z_{k-1} + g_k e, y += z1 + z2/2 +
        // z3/6 + z4/24, the x-part of each level the w-part of the one before
        T g1 = T(0), g2 = T(0), g4 = T(0);
        if (forced) {
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
        T xe[RPT], we[RPT], Bp[RPT], V[RPT], R[RPT], sx[RPT], sw[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            xe[r] = COMP ? x[r] + xl[r] : x[r];
            we[r] = COMP ? w[r] + wl[r] : w[r];
        }
        const T *u = publish(xe, we);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool own = tid + r * kThreads < s;
            R[r] = own ? bop(u, r, true) : T(0);               // B x
            Bp[r] = own ? bop(u + pitch, r, false) : T(0);     // B w = B z1_x
            T v = fma_t(-dampw, we[r], -R[r]);
            if (use_beta) v = fma_t(-dampb, Bp[r], v);
            if (forced) v = fma_t(fh[r], g1, v);
            V[r] = own ? v : T(0);   // z1_w
            sx[r] = T(0.5) * V[r];
            sw[r] = V[r];
        }
        u = publish(V, nullptr);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool own = tid + r * kThreads < s;
            R[r] = own ? bop(u, r, false) : T(0);   // B z1_w = B z2_x
            T v = fma_t(-dampw, V[r], -Bp[r]);
            if (use_beta) v = fma_t(-dampb, R[r], v);
            if (forced) v = fma_t(fh[r], g2, v);
            V[r] = own ? v : T(0);   // z2_w
            Bp[r] = R[r];
            sx[r] = fma_t(T(1.0 / 6.0), V[r], sx[r]);
            sw[r] = fma_t(T(0.5), V[r], sw[r]);
        }
        u = publish(V, nullptr);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool own = tid + r * kThreads < s;
            R[r] = own ? bop(u, r, false) : T(0);   // B z2_w = B z3_x
            T v = fma_t(-dampw, V[r], -Bp[r]);
            if (use_beta) v = fma_t(-dampb, R[r], v);
            V[r] = own ? v : T(0);   // z3_w
            Bp[r] = R[r];
            sx[r] = fma_t(T(1.0 / 24.0), V[r], sx[r]);
            sw[r] = fma_t(T(1.0 / 6.0), V[r], sw[r]);
        }
        if (use_beta) {
            u = publish(V, nullptr);
#pragma unroll
            for (int r = 0; r < RPT; ++r) R[r] = tid + r * kThreads < s ? bop(u, r, false) : T(0);   // B z3_w
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            T v = fma_t(-dampw, V[r], -Bp[r]);
            if (use_beta) v = fma_t(-dampb, R[r], v);
            if (forced) v = fma_t(fh[r], g4, v);   // z4_w
            const T dx = we[r] + sx[r];
            const T dw = fma_t(T(1.0 / 24.0), v, sw[r]);
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

template <typename T, int DPL, int LPI, int EX>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 8 && DPL == 16) ? 1 : 2) driven_chain_kernel(DrivenLaunch<T> a) {
    driven_chain_run<T, DPL, LPI, EX>(a, (int64_t)blockIdx.x * kThreads + threadIdx.x);
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
