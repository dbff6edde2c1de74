// Dense eq. (1) systems whose A = M^-1 K is shared by many instances: every
// stage product is a true GEMM, (s x s) . (s x instances), run on the gfx950
// matrix cores with v_mfma_f32_16x16x32_f16.
//
// Workgroup: NW wavefronts and 16 instances (one MFMA column tile).  Wave w
// owns rows [16 RT w, 16 RT (w + 1)) of the operator (RT row tiles of 16) and
// the same rows of the 16 instances' state, kept in registers in the MFMA
// accumulator layout (lane l, element r of row tile t: row 16 t + 4 (l/16) + r,
// instance l % 16).  The operator stays resident in registers for the whole
// launch; the right-hand operand of each product goes through a small LDS
// buffer, which also performs the transpose from the accumulator layout to
// the operand layout.  The buffer is laid out [8-row block][instance][8 rows]:
// an operand fragment (8 consecutive rows of one instance per lane) is one
// 16-byte slot, and the 64 lanes of a fragment read, like the 4-row writes of
// the accumulator layout, one contiguous stretch, so no two lanes of an access
// meet in an LDS bank.
//
// Precision.  The FP16 operator B^ = beta h^2 A (beta a power of two with
// ||B^||_inf <= 1) is split into B1 = fp16(B^) and B2 = fp16((B^ - B1) 2^11);
// an FP32 operand u becomes u1 = fp16(u) and u2 = fp16((u - u1) 2^11).  Then
//   B^ u ~ B1 u1 + 2^-11 (B1 u2 + B2 u1)       (three MFMAs, ~2^-22 relative)
// accumulates in FP32.  RK4 (exact linear Taylor form, as for chains) uses
// this three-term product for B x; for B w it leaves out B1 u2: w = h v is
// already a factor h omega <= 0.01 smaller than x, so the rounding of u1,
// which changes from step to step, moves w by about 2^-12 (h omega)^2 |w| / 2
// per step (a random walk of ~1e-6 |w| over 1e4 steps), while B2 u1 stays
// because a fixed error in the operator would shift every frequency.  B P and
// B Q take one term (B1 u1): they enter the update only at third order and
// beyond, where the FP16 rounding moves a frequency by about
// 2^-11 (h omega)^2 / 12.  The state of each
// instance is scaled by a power of two sigma so that |x| < 1 in FP16 terms;
// powers of two keep every scaling exact.
//
// Damped, driven systems (method kMfmaDriven + EX, RK4 only) take the RK4
// map as the four-level recursion y_{n+1} = y + z1 + z2/2 + z3/6 + z4/24,
// z1 = L y + g1 e, z_k = L z_{k-1} + g_k e (L y = (w, -Bx - a w - b Bw),
// a = alpha h, b = beta / h, e = (0, h^2 f), g = (c0, 2 (ch - c0), 0,
// 4 (c0 - 2 ch + c1)) from the force phases at t_n, t_n + h/2, t_n + h).  The
// x-part of each level is the previous level's w-part, so the products are
// B x (three terms), B w (two; three with stiffness damping, whose b B w
// enters the first level), then B of the level w-parts (one term each: they
// enter at third order and beyond, like B P and B Q above).  The level
// w-parts are kept scaled by powers of beta (Z1 = beta sigma z1, Z2 = beta
// sigma z2, Z3 = beta^2 sigma z3, Z4 = beta^2 sigma z4) so that every FP16
// operand is of order one:
//   Z1 = -B^x - a beta w - b B^w + g1 F,   Z2 = -B^w - a Z1 - b ib B^Z1 + g2 F,
//   Z3 = -B^Z1 - a beta Z2 - b B^Z2,        Z4 = -B^Z2 - a Z3 - b ib B^Z3 + beta g4 F,
// with F = beta sigma h^2 f (kept in LDS) and ib = 1 / beta, and
//   sigma dx = w + ib (Z1/2 + Z2/6 + ib Z3/24),
//   sigma dw = ib (Z1 + Z2/2 + ib (Z3/6 + Z4/24)).
// The force's phase is the FP64 rotation of the other driven kernels.

#include <cstdint>

#include "osc_internal.h"

namespace osc {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kNC = 16;   // instances per workgroup
constexpr float kSplit = 2048.0f;
constexpr float kUnsplit = 1.0f / 2048.0f;

__device__ __forceinline__ void comp_add(float &hi, float &lo, float y) {
    y = y + lo;
    const float t = hi + y;
    lo = y - (t - hi);
    hi = t;
}

__device__ __forceinline__ f4 mfma(half8 a, half8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// One workgroup's share of launch a: the 16 instances of column tile `tile`.
template <int RT, int NW, int METHOD>
__device__ __forceinline__ void mfma_run(const DenseMfmaLaunch &a, const int64_t tile) {
    constexpr bool DRIVEN = METHOD >= kMfmaDriven;
    constexpr bool BETA = DRIVEN && (METHOD & 1), FORCED = DRIVEN && (METHOD & 2);
    constexpr int kNW = NW;          // waves per workgroup
    constexpr int SP = 16 * RT * NW; // padded dimension
    constexpr int KS = SP / 32;      // k-steps of 32
    constexpr int NB = SP / 8;       // 8-row blocks of an operand
    // operand buffers: x (hi, lo), w (hi), B x (hi), B w (hi)
    __shared__ __attribute__((aligned(16))) _Float16 bufA[2][NB][kNC][8];
    // w takes its low plane too where the stiffness damping b B w enters the
    // first level (driven launches with beta != 0)
    __shared__ __attribute__((aligned(16))) _Float16 bufB[BETA ? 2 : 1][NB][kNC][8];
    __shared__ __attribute__((aligned(16))) _Float16 bufC[1][NB][kNC][8];
    __shared__ __attribute__((aligned(16))) _Float16 bufD[1][NB][kNC][8];
    __shared__ float smax[kNW][kNC];
    // compensation terms (touched once per step), lane-private slots
    __shared__ float sxl[kNW][RT][4][64];
    __shared__ float swl[kNW][RT][4][64];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, quad = lane >> 4;
    const int64_t b = tile * kNC + col;
    const bool active = b < a.batch;
    const int s = a.s;
    const int row0 = wave * 16 * RT;
    const size_t base = (size_t)(active ? b : 0) * s;
    const size_t plane = (size_t)a.batch * s;
    const double h = a.h;
    const float ib = a.inv_beta;

    // resident operator fragments
    half8 B1r[RT][KS], B2r[RT][KS];
    const half8 *B1 = reinterpret_cast<const half8 *>(a.B1);
    const half8 *B2 = reinterpret_cast<const half8 *>(a.B2);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const size_t idx = ((size_t)(wave * RT + t) * KS + q) * 64 + lane;
            B1r[t][q] = B1[idx];
            B2r[t][q] = B2[idx];
        }

    // state, unscaled first
    float x[RT][4], w[RT][4];
    float(&xl)[RT][4][64] = sxl[wave];
    float(&wl)[RT][4][64] = swl[wave];
    double mx = 0.0;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 16 * t + 4 * quad + r;
            const bool v = active && row < s;
            const size_t i = base + row;
            if (a.load_mode == LOAD_USER) {
                x[t][r] = v ? a.x0[i] : 0.0f;
                xl[t][r][lane] = 0.0f;
                const double wd = v ? h * (double)a.v0[i] : 0.0;
                w[t][r] = (float)wd;
                wl[t][r][lane] = (float)(wd - (double)w[t][r]);
            } else {
                x[t][r] = v ? a.state[i] : 0.0f;
                xl[t][r][lane] = v ? a.state[plane + i] : 0.0f;
                w[t][r] = v ? a.state[2 * plane + i] : 0.0f;
                wl[t][r][lane] = v ? a.state[3 * plane + i] : 0.0f;
            }
            mx = fmax(mx, fmax(fabs((double)x[t][r]), fabs((double)w[t][r])));
        }
    // the force, beta h^2 f (scaled by sigma below), in lane-private LDS
    // slots beside the compensation terms; its size joins the scale choice,
    // as the forced response grows from it
    __shared__ float sfs[kNW][RT][4][64];
    float(&Fs)[RT][4][64] = sfs[wave];
    const double beta_d = 1.0 / (double)ib;
    if constexpr (FORCED) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * t + 4 * quad + r;
                const double fd = (active && row < s) ? beta_d * h * h * a.f[base + row] : 0.0;
                Fs[t][r][lane] = (float)fd;
                mx = fmax(mx, fabs(fd));
            }
    }
    // per-instance power-of-two scale sigma (max |state| sigma in [0.5, 1)),
    // chosen from the initial state and carried with the state across
    // launches so that chunked runs round exactly like unchunked ones
    float m32 = (float)mx;
    m32 = fmaxf(m32, __shfl_xor(m32, 16, 64));
    m32 = fmaxf(m32, __shfl_xor(m32, 32, 64));
    if (quad == 0) smax[wave][col] = m32;
    __syncthreads();
    float mall = 0.0f;
#pragma unroll
    for (int v = 0; v < kNW; ++v) mall = fmaxf(mall, smax[v][col]);
    int e = 0;
    (void)frexpf(mall, &e);
    float sigma = (mall > 0.0f && __builtin_isfinite(mall)) ? ldexpf(1.0f, -e) : 1.0f;
    if (a.load_mode == LOAD_STATE && active) sigma = a.sigma[b];
    if ((a.store_mode & STORE_STATE) && active && wave == 0 && quad == 0) a.sigma[b] = sigma;
    const double inv_sigma = 1.0 / (double)sigma;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            x[t][r] *= sigma;
            xl[t][r][lane] *= sigma;
            w[t][r] *= sigma;
            wl[t][r][lane] *= sigma;
            if constexpr (FORCED) Fs[t][r][lane] *= sigma;
        }
    Phase ph{};
    if (FORCED && active) ph.start(a.omega[b] * h, a.n0);
    const float ka = (float)(a.alpha * h), kab = (float)(a.alpha * h * beta_d);
    const float kb = (float)(a.beta / h), kbi = (float)(a.beta / h * (double)ib);

    // operand u -> LDS (hi plane, optionally the scaled low plane)
    auto put = [&](_Float16 (*buf)[NB][kNC][8], const float (&u)[RT][4], bool two) {
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            half4 hv, lv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const _Float16 hh = (_Float16)u[t][r];
                hv[r] = hh;
                lv[r] = (_Float16)((u[t][r] - (float)hh) * kSplit);
            }
            const int row = row0 + 16 * t + 4 * quad;
            *reinterpret_cast<half4 *>(&buf[0][row / 8][col][row % 8]) = hv;
            if (two) *reinterpret_cast<half4 *>(&buf[1][row / 8][col][row % 8]) = lv;
        }
    };
    auto frag = [&](_Float16 (*buf)[NB][kNC][8], int p, int q) -> half8 {
        return *reinterpret_cast<const half8 *>(&buf[p][4 * q + quad][col][0]);
    };
    // three-term product: out = B^ u with u split in buf
    auto prod3 = [&](_Float16 (*buf)[NB][kNC][8], float (&out)[RT][4]) {
        f4 am[RT], ac[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            am[t] = f4{0.f, 0.f, 0.f, 0.f};
            ac[t] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const half8 uh = frag(buf, 0, q), ul = frag(buf, 1, q);
#pragma unroll
            for (int t = 0; t < RT; ++t) am[t] = mfma(B1r[t][q], uh, am[t]);
#pragma unroll
            for (int t = 0; t < RT; ++t) ac[t] = mfma(B1r[t][q], ul, ac[t]);
#pragma unroll
            for (int t = 0; t < RT; ++t) ac[t] = mfma(B2r[t][q], uh, ac[t]);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[t][r] = __builtin_fmaf(ac[t][r], kUnsplit, am[t][r]);
    };
    // two-term product: out = (B1 + 2^-11 B2) u1, the operand's low plane left out
    auto prod2 = [&](_Float16 (*buf)[NB][kNC][8], float (&out)[RT][4]) {
        f4 am[RT], ac[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            am[t] = f4{0.f, 0.f, 0.f, 0.f};
            ac[t] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const half8 uh = frag(buf, 0, q);
#pragma unroll
            for (int t = 0; t < RT; ++t) am[t] = mfma(B1r[t][q], uh, am[t]);
#pragma unroll
            for (int t = 0; t < RT; ++t) ac[t] = mfma(B2r[t][q], uh, ac[t]);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[t][r] = __builtin_fmaf(ac[t][r], kUnsplit, am[t][r]);
    };
    auto prod1 = [&](_Float16 (*buf)[NB][kNC][8], float (&out)[RT][4]) {
        f4 am[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) am[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const half8 uh = frag(buf, 0, q);
#pragma unroll
            for (int t = 0; t < RT; ++t) am[t] = mfma(B1r[t][q], uh, am[t]);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[t][r] = am[t][r];
    };

    float P[RT][4];   // Verlet: B^ x at the current full step (scaled units)
    if constexpr (METHOD == OSC_VERLET) {
        __syncthreads();
        put(bufA, x, true);
        __syncthreads();
        prod3(bufA, P);
        if (a.load_mode == LOAD_USER) {
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) comp_add(w[t][r], wl[t][r][lane], -0.5f * ib * P[t][r]);
        }
    }
    auto vel = [&](int t, int r) -> double {
        double wv = (double)w[t][r] + (double)wl[t][r][lane];
        if constexpr (METHOD == OSC_VERLET) wv += 0.5 * (double)ib * (double)P[t][r];
        return wv * inv_sigma / h;
    };
    const bool untouched = a.load_mode == LOAD_USER;
    // A lane's four consecutive DOFs of tile t go out as one 16-byte store
    // when they are whole and aligned, so that a wave writes whole lines of
    // each instance instead of one float per line per instruction.
    auto emit = [&](float *dst, int t, auto val) {
        if (!active) return;
        const int row = row0 + 16 * t + 4 * quad;
        float *p = dst + base + row;
        if (row + 4 <= s && ((uintptr_t)p % 16) == 0) {
            *reinterpret_cast<f4 *>(p) = f4{val(t, 0), val(t, 1), val(t, 2), val(t, 3)};
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (row + r < s) p[r] = val(t, r);
        }
    };
    auto xout = [&](int t, int r) { return (float)(((double)x[t][r] + (double)xl[t][r][lane]) * inv_sigma); };
    auto vout = [&](int t, int r) { return (float)vel(t, r); };
    auto xin = [&](int t, int r) { return a.x0[base + row0 + 16 * t + 4 * quad + r]; };
    auto vin = [&](int t, int r) { return a.v0[base + row0 + 16 * t + 4 * quad + r]; };
    auto write_frame = [&](int64_t f, bool initial) {
        const size_t fo = (size_t)f * a.frame_plane;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            if (a.xf) {
                if (initial) emit(a.xf + fo, t, xin);
                else emit(a.xf + fo, t, xout);
            }
            if (a.vf) {
                if (initial) emit(a.vf + fo, t, vin);
                else emit(a.vf + fo, t, vout);
            }
        }
    };

    // RK4 increments (the products are B^ u = beta B u, ib = 1 / beta, a
    // power of two), each summed from its smallest term up and rounded once
    // at the scale of its dominant term:
    //   dx = w - (ib/2) (P + Q/3 - ib P2/12)
    //   dw = -ib (P + (Q - ib P2/3 - ib Q2/12) / 2)
    const float e1 = -ib / 12.0f, e2 = -ib / 3.0f, e3 = -0.5f * ib;

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
            if constexpr (DRIVEN) {
                float g1 = 0.0f, g2 = 0.0f, gb4 = 0.0f;
                if constexpr (FORCED) {
                    if (it % kAnchor == 0) ph.set(it);
                    const double c0 = ph.c;
                    ph.half();
                    const double ch = ph.c;
                    ph.half();
                    const double c1 = ph.c;
                    g1 = (float)c0;
                    g2 = (float)(2.0 * (ch - c0));
                    gb4 = (float)(4.0 * ((c0 - ch) + (c1 - ch)) * beta_d);
                }
                float pk[RT][4], qk[RT][4], Z[RT][4], R[RT][4], sx[RT][4], sw[RT][4];
                __syncthreads();
                put(bufA, x, true);
                put(bufB, w, BETA);
                __syncthreads();
                prod3(bufA, pk);   // B^ x
                if constexpr (BETA) prod3(bufB, qk);   // B^ w, also in b B^ w at the first level
                else prod2(bufB, qk);
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float z = __builtin_fmaf(-kab, w[t][r], -pk[t][r]);
                        if constexpr (BETA) z = __builtin_fmaf(-kb, qk[t][r], z);
                        if constexpr (FORCED) z = __builtin_fmaf(Fs[t][r][lane], g1, z);
                        Z[t][r] = z;   // Z1
                        sx[t][r] = 0.5f * z;
                        sw[t][r] = z;
                    }
                put(bufC, Z, false);
                __syncthreads();
                prod1(bufC, R);   // B^ Z1
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float z = __builtin_fmaf(-ka, Z[t][r], -qk[t][r]);
                        if constexpr (BETA) z = __builtin_fmaf(-kbi, R[t][r], z);
                        if constexpr (FORCED) z = __builtin_fmaf(Fs[t][r][lane], g2, z);
                        Z[t][r] = z;   // Z2
                        pk[t][r] = R[t][r];   // B^ Z1
                        sx[t][r] = __builtin_fmaf(1.0f / 6.0f, z, sx[t][r]);
                        sw[t][r] = __builtin_fmaf(0.5f, z, sw[t][r]);
                    }
                put(bufD, Z, false);
                __syncthreads();
                prod1(bufD, R);   // B^ Z2
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float z = __builtin_fmaf(-kab, Z[t][r], -pk[t][r]);
                        if constexpr (BETA) z = __builtin_fmaf(-kb, R[t][r], z);
                        Z[t][r] = z;   // Z3
                        qk[t][r] = R[t][r];   // B^ Z2
                    }
                if constexpr (BETA) {
                    put(bufC, Z, false);
                    __syncthreads();
                    prod1(bufC, R);   // B^ Z3
                }
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float z = __builtin_fmaf(-ka, Z[t][r], -qk[t][r]);
                        if constexpr (BETA) z = __builtin_fmaf(-kbi, R[t][r], z);
                        if constexpr (FORCED) z = __builtin_fmaf(Fs[t][r][lane], gb4, z);   // Z4
                        const float dxs = __builtin_fmaf(ib, __builtin_fmaf(ib * (1.0f / 24.0f), Z[t][r], sx[t][r]),
                                                         w[t][r]);
                        const float dws = ib * __builtin_fmaf(ib, __builtin_fmaf(1.0f / 24.0f, z, (1.0f / 6.0f) * Z[t][r]),
                                                              sw[t][r]);
                        comp_add(x[t][r], xl[t][r][lane], dxs);
                        comp_add(w[t][r], wl[t][r][lane], dws);
                    }
            } else if constexpr (METHOD == OSC_RK4) {
                // each product is folded into the partial sums and written out
                // as the next operand as soon as it is formed; P, sx and sw
                // stay live until the increments are complete
                float pk[RT][4], sx[RT][4], sw[RT][4], T[RT][4];
                __syncthreads();
                put(bufA, x, true);
                put(bufB, w, false);
                __syncthreads();
                prod3(bufA, pk);   // P = B^ x
                put(bufC, pk, false);
                prod2(bufB, T);   // Q = B^ w
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sx[t][r] = __builtin_fmaf(1.0f / 3.0f, T[t][r], pk[t][r]);
                        sw[t][r] = T[t][r];
                    }
                put(bufD, T, false);
                __syncthreads();
                prod1(bufC, T);   // P2 = B^ P
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sx[t][r] = __builtin_fmaf(e1, T[t][r], sx[t][r]);
                        sw[t][r] = __builtin_fmaf(e2, T[t][r], sw[t][r]);
                        comp_add(x[t][r], xl[t][r][lane], __builtin_fmaf(e3, sx[t][r], w[t][r]));
                    }
                prod1(bufD, T);   // Q2 = B^ Q
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sw[t][r] = __builtin_fmaf(e1, T[t][r], sw[t][r]);
                        comp_add(w[t][r], wl[t][r][lane], -ib * __builtin_fmaf(0.5f, sw[t][r], pk[t][r]));
                    }
            } else {
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) comp_add(x[t][r], xl[t][r][lane], w[t][r]);
                __syncthreads();
                put(bufA, x, true);
                __syncthreads();
                prod3(bufA, P);
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) comp_add(w[t][r], wl[t][r][lane], -ib * P[t][r]);
            }
        }
        n = stop;
        if (stride > 0 && n % stride == 0) write_frame(n / stride, false);
    }

    const bool copy_input = untouched && a.nsteps == 0;
    bool ok = true;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 16 * t + 4 * quad + r;
            if (active && row < s) ok = ok && __builtin_isfinite(x[t][r]) && __builtin_isfinite(w[t][r]);
        }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        if (a.store_mode & STORE_STATE) {
            emit(a.state, t, [&](int tt, int r) { return (float)((double)x[tt][r] * inv_sigma); });
            emit(a.state + plane, t, [&](int tt, int r) { return (float)((double)xl[tt][r][lane] * inv_sigma); });
            emit(a.state + 2 * plane, t, [&](int tt, int r) { return (float)((double)w[tt][r] * inv_sigma); });
            emit(a.state + 3 * plane, t, [&](int tt, int r) { return (float)((double)wl[tt][r][lane] * inv_sigma); });
        }
        if (a.store_mode & STORE_USER) {
            if (a.xe) {
                if (copy_input) emit(a.xe, t, xin);
                else emit(a.xe, t, xout);
            }
            if (a.ve) {
                if (copy_input) emit(a.ve, t, vin);
                else emit(a.ve, t, vout);
            }
        }
    }
    if (!ok && a.nonfinite) atomicOr(a.nonfinite, 1);
}

template <int RT, int NW, int METHOD>
__global__ void __launch_bounds__(64 * NW, 1) dense_mfma_kernel(DenseMfmaLaunch a) {
    mfma_run<RT, NW, METHOD>(a, blockIdx.x);
}

// Work list: workgroup i runs items[i] (a launch of at most 16 instances with
// its own operator, e.g. one served request).
template <int RT, int NW, int METHOD>
__global__ void __launch_bounds__(64 * NW, 1) dense_mfma_items_kernel(const DenseMfmaItem *__restrict__ items) {
    const DenseMfmaLaunch a = items[blockIdx.x].L;
    mfma_run<RT, NW, METHOD>(a, 0);
}

// Operator fragments: for row tile T, k-step q, lane l, element j:
// row = 16 T + l % 16, k = 32 q + 8 (l / 16) + j.
__global__ void dense_mfma_fragments_kernel(int s, int sp, const double *__restrict__ A, double scale,
                                            _Float16 *B1, _Float16 *B2) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ks = sp / 32;
    const int64_t total = (int64_t)(sp / 16) * ks * 64 * 8;
    if (idx >= total) return;
    const int j = (int)(idx % 8);
    const int l = (int)((idx / 8) % 64);
    const int q = (int)((idx / 512) % ks);
    const int T = (int)(idx / (512 * (int64_t)ks));
    const int row = 16 * T + l % 16, k = 32 * q + 8 * (l / 16) + j;
    const double v = (row < s && k < s) ? scale * A[(size_t)row * s + k] : 0.0;
    const _Float16 h1 = (_Float16)(float)v;
    B1[idx] = h1;
    B2[idx] = (_Float16)(float)((v - (double)(float)h1) * 2048.0);
}

template <int RT, int NW>
void launch_rt(const DenseMfmaLaunch &a, int method, hipStream_t st) {
    const unsigned blocks = (unsigned)((a.batch + kNC - 1) / kNC);
    switch (method) {
        case OSC_RK4:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, OSC_RK4>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
        case OSC_VERLET:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, OSC_VERLET>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
        case kMfmaDriven + 0:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, kMfmaDriven + 0>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
        case kMfmaDriven + 1:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, kMfmaDriven + 1>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
        case kMfmaDriven + 2:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, kMfmaDriven + 2>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL((dense_mfma_kernel<RT, NW, kMfmaDriven + 3>), dim3(blocks), dim3(64 * NW), 0, st, a);
            break;
    }
}

template <int RT, int NW>
void launch_items_rt(const DenseMfmaItem *items, int64_t n, int method, hipStream_t st) {
    if (method == OSC_RK4)
        hipLaunchKernelGGL((dense_mfma_items_kernel<RT, NW, OSC_RK4>), dim3((unsigned)n), dim3(64 * NW), 0, st, items);
    else
        hipLaunchKernelGGL((dense_mfma_items_kernel<RT, NW, OSC_VERLET>), dim3((unsigned)n), dim3(64 * NW), 0, st,
                           items);
}

}  // namespace

osc_status dense_mfma_launch_items(const DenseMfmaItem *items, int64_t nitems, int pad, int method,
                                   hipStream_t st) {
    if (nitems == 0) return OSC_OK;
    if (nitems > 0x7fffffff) return fail(OSC_EINVAL, "work list too long for one launch");
    switch (pad / 64) {
        case 1: launch_items_rt<2, 2>(items, nitems, method, st); break;
        case 2: launch_items_rt<2, 4>(items, nitems, method, st); break;
        case 3: launch_items_rt<2, 6>(items, nitems, method, st); break;
        case 4: launch_items_rt<2, 8>(items, nitems, method, st); break;
        default: return fail(OSC_ENOTSUP, "MFMA path needs s <= 256");
    }
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

int dense_mfma_pad(int s) { return s <= 256 ? ((s + 63) / 64) * 64 : 0; }

size_t dense_mfma_fragment_elems(int s) {
    const int sp = dense_mfma_pad(s);
    return (size_t)(sp / 16) * (sp / 32) * 64 * 8;
}

osc_status dense_mfma_fragments(int s, const double *A, double scale, _Float16 *B1, _Float16 *B2, hipStream_t st) {
    const int sp = dense_mfma_pad(s);
    if (!sp) return fail(OSC_ENOTSUP, "MFMA path needs s <= 256");
    const int64_t total = (int64_t)dense_mfma_fragment_elems(s);
    hipLaunchKernelGGL(dense_mfma_fragments_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, s, sp,
                       A, scale, B1, B2);
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

osc_status dense_mfma_launch(const DenseMfmaLaunch &a, int method, hipStream_t st) {
    if (a.batch == 0) return OSC_OK;
    if (method != OSC_RK4 && method != OSC_VERLET && (method < kMfmaDriven || method > kMfmaDriven + 3))
        return fail(OSC_EINVAL, "unknown MFMA method");
    if ((a.batch + kNC - 1) / kNC > 0x7fffffff) return fail(OSC_EINVAL, "batch too large for one launch");
    // 32 rows per wave: the operator takes 128 registers per lane, which
    // leaves room for two waves per SIMD
    switch (dense_mfma_pad(a.s) / 64) {
        case 1: launch_rt<2, 2>(a, method, st); break;
        case 2: launch_rt<2, 4>(a, method, st); break;
        case 3: launch_rt<2, 6>(a, method, st); break;
        case 4: launch_rt<2, 8>(a, method, st); break;
        default: return fail(OSC_ENOTSUP, "MFMA path needs s <= 256");
    }
    OSC_HIP(hipGetLastError());
    return OSC_OK;
}

}  // namespace osc
