// Internal declarations of libosc (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "osc.h"

struct osc_sys;

namespace osc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
osc_status fail(osc_status st, const std::string &msg);
#define OSC_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::osc::fail(OSC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// RK4 increments of the exact linear (Taylor) form of the classic RK4 map in
// scaled time (w = h v, products P = Bx, Q = Bw, P2 = BP, Q2 = BQ):
//   dx = w - P/2 - Q/6 + P2/24 = w  - (P + Q/3 - P2/12) / 2
//   dw = -P - Q/2 + P2/6 + Q2/24 = -P - (Q - P2/3 - Q2/12) / 2
// The small terms are summed before the dominant one (w, resp. P), which is
// added by the last fused multiply-add, so that each increment is rounded
// once at its own scale.  Adding the small terms one at a time to the
// dominant one rounds three times at that scale and loses the fourth-order
// terms below half an ulp; over 10^4 steps of a two-mass ensemble that drifts
// the energy by up to 2e-6 in FP32 (about 5e-7 in this order).  P2 and Q2,
// formed last, enter through two dependent operations each.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
template <typename T>
__device__ __forceinline__ void rk4_increments(T w, T P, T Q, T P2, T Q2, T &dx, T &dw) {
    const T t = fma_t(T(-1.0 / 12.0), P2, fma_t(T(1.0 / 3.0), Q, P));
    dx = fma_t(T(-0.5), t, w);
    const T u = fma_t(T(-1.0 / 12.0), Q2, fma_t(T(-1.0 / 3.0), P2, Q));
    dw = fma_t(T(-0.5), u, -P);
}

// Whole-wave DPP shifts: lane i receives lane i-1 (from_left) or lane i+1
// (from_right); a lane whose source lies outside the wave (lane 0 shifting
// right, lane 63 shifting left) receives 0: with BC (bound_ctrl) set the
// shift itself writes the 0, else the lane keeps the 0 it was given first.
template <bool BC>
__device__ __forceinline__ int shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, BC); }
template <bool BC>
__device__ __forceinline__ int shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, BC); }

template <bool BC>
__device__ __forceinline__ float from_left(float v) { return __builtin_bit_cast(float, shr1<BC>(__builtin_bit_cast(int, v))); }
template <bool BC>
__device__ __forceinline__ float from_right(float v) { return __builtin_bit_cast(float, shl1<BC>(__builtin_bit_cast(int, v))); }
template <bool BC>
__device__ __forceinline__ double from_left(double v) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    unsigned lo = (unsigned)shr1<BC>((int)(unsigned)b), hi = (unsigned)shr1<BC>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <bool BC>
__device__ __forceinline__ double from_right(double v) {
    unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    unsigned lo = (unsigned)shl1<BC>((int)(unsigned)b), hi = (unsigned)shl1<BC>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Phase of a harmonic force, cos and sin of Omega t at the current half step:
// set exactly (sincos of Omega h n) at every global step index divisible by
// kAnchor and advanced by half-step rotations in between, so that chunked and
// unchunked runs agree bitwise.  The rotation's rounding is spelled out (one
// product, then one fused multiply-add) so that every inlined copy, in and
// out of a step loop, computes bit for bit the same values.
constexpr int64_t kAnchor = 64;
struct Phase {
    double c, s;     // e^{i Omega h tau}
    double rc, rs;   // e^{i Omega h / 2}
    double wh;       // Omega h
    __device__ void set(int64_t n) { sincos(wh * (double)n, &s, &c); }
    __device__ void half() {
        const double nc = __builtin_fma(c, rc, -(s * rs)), ns = __builtin_fma(s, rc, c * rs);
        c = nc;
        s = ns;
    }
    // ready for the step that starts at global step n0
    __device__ void start(double omega_h, int64_t n0) {
        wh = omega_h;
        sincos(0.5 * wh, &rs, &rc);
        const int64_t anchor = n0 - n0 % kAnchor;
        set(anchor);
        for (int64_t q = anchor; q < n0; ++q) {
            half();
            half();
        }
    }
};

// ---------------------------------------------------------------------------
// device memory pool with an HBM budget (pool.cpp)
// ---------------------------------------------------------------------------
void *pool_alloc(size_t bytes);          // nullptr when the budget or the device is exhausted
void pool_free(void *p);
size_t pool_in_use();                    // bytes handed out and not yet returned
size_t pool_budget();                    // 0 = unlimited
void pool_set_budget(size_t bytes);
void pool_trim();                        // return cached blocks to the device
size_t pool_size_class(size_t bytes);    // bytes actually reserved for a request of this size

// ---------------------------------------------------------------------------
// chain integration (chain.hip)
// ---------------------------------------------------------------------------
enum : int { LOAD_USER = 1, LOAD_STATE = 2 };
enum : int { STORE_USER = 1, STORE_STATE = 2 };

// Coefficients of a chain batch in scaled time tau = t / h:
//   (B x)_i = cl_i (x_i - x_{i-1}) - cr_i (x_{i+1} - x_i),
//   cl_i = h^2 k_i / m_i,  cr_i = h^2 k_{i+1} / m_i  (cr_{s-1} = 0).
// For FP32 each coefficient is stored as a high part and a low part
// (hi = fl32(c), lo = fl32(c - hi)); FP64 keeps hi only.
template <typename T>
struct ChainCoef {
    const T *clh, *crh, *cll, *crl;   // [batch][s]
    const double *h;                  // [batch] step
};

// One launch of the chain kernel over a contiguous range of instances.
// Internal state layout (LOAD_STATE / STORE_STATE): four planes
// [4][batch][s]: x_hi, x_lo, w_hi, w_lo with w = h * v (RK4) or the
// half-step value w_{n+1/2} (Verlet).
template <typename T>
struct ChainLaunch {
    int64_t batch;
    int32_t s;
    ChainCoef<T> c;
    const T *x0, *v0;          // LOAD_USER
    T *state;                  // LOAD_STATE / STORE_STATE
    int64_t nsteps;            // steps advanced by this launch
    int64_t n0;                // global step number at entry
    int64_t out_stride;        // 0: no frames
    T *xf, *vf;                // frames [nframes][batch][s]
    T *xe, *ve;                // STORE_USER
    int *nonfinite;            // set to 1 if a state is not finite at exit
    int load_mode;
    int store_mode;
};

// One entry of a work list: instance b of launch L.
template <typename T>
struct ChainItem {
    ChainLaunch<T> L;
    int64_t b;
};

struct ChainConfig {
    int lpi;   // lanes per instance (1..64, power of two)
    int dpl;   // degrees of freedom per lane
};

// Choose a lane-group layout for s degrees of freedom.
ChainConfig chain_pick_config(int s);
// Launch one integration pass.  method: OSC_RK4 / OSC_VERLET.
template <typename T>
osc_status chain_launch(const ChainLaunch<T> &a, int method, ChainConfig cfg, hipStream_t st);
// Launch a work list (device array of items, all of whose s fit cfg).
template <typename T>
osc_status chain_launch_items(const ChainItem<T> *items, int64_t nitems, int method, ChainConfig cfg,
                              hipStream_t st);
// Every configuration the chain kernel is built for (for tests and tuning).
int chain_num_configs();
ChainConfig chain_config_at(int i);

// Plain baseline: one instance, one step per launch, state in device memory.
template <typename T>
osc_status chain_plain(const ChainLaunch<T> &a, int method, hipStream_t st);

// Resident real-time stepping (resident.hip).  The control block lives in
// host-mapped memory; each field sits on a line of its own.
struct RtControl {
    alignas(128) int64_t release;   // host: ticks released so far (negative: stop)
    alignas(128) uint64_t done;     // device: workgroups that finished a tick, over all ticks
    alignas(128) int32_t exit_reason;
};
constexpr int kRtExitRunning = 0, kRtExitTicks = 1, kRtExitStop = 2, kRtExitIdle = 3;
template <typename T>
struct ResidentRun {
    RtControl *ctl;          // device address of the control block
    int64_t first_release;   // release count before this run's first tick
    int64_t nticks;          // ticks of this run
    int64_t n_start;         // global step at the first tick
    int64_t k;               // steps per tick
    int64_t idle_ticks;      // 100 MHz counter ticks without a release before a workgroup gives up
    T *xf, *vf;              // per-tick outputs [nticks][batch][s], or nullptr
    T *xo, *vo;              // every tick's output when xf / vf are nullptr
};
// Launch the resident kernel (a: the handle's chain launch without step
// range or outputs).  OSC_ENOTSUP when its workgroups cannot all be resident.
template <typename T>
osc_status chain_resident_launch(const ChainLaunch<T> &a, int method, ChainConfig cfg, const ResidentRun<T> &r,
                                 hipStream_t st);
template <typename T>
int64_t chain_resident_blocks(const ChainLaunch<T> &a, ChainConfig cfg);
// the same for damped, driven chains of s <= 1024 (register layouts)
template <typename T>
struct DrivenLaunch;
template <typename T>
osc_status driven_resident_launch(const DrivenLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st);
template <typename T>
int64_t driven_resident_blocks(const DrivenLaunch<T> &a);

// ---------------------------------------------------------------------------
// coefficient preparation, stability bound and energy (prep.hip)
// ---------------------------------------------------------------------------
template <typename T>
osc_status chain_prepare(int64_t batch, int s, const double *m, const double *k,
                         const double *dt, T *clh, T *crh, T *cll, T *crl, double *h,
                         double *theta_bound, int *bad_param, hipStream_t st);
// h omega_max of every chain (exact up to a relative 2^-40, never below it),
// by Sturm-sequence bisection in FP64; theta: device [batch].
osc_status chain_sturm_theta(int64_t batch, int s, const double *m, const double *k, const double *dt,
                             double *theta, hipStream_t st);
template <typename T>
osc_status chain_energy(int64_t batch, int s, const double *m, const double *k,
                        const double *h, const T *x, const T *v, double *E, bool shadow,
                        hipStream_t st);

// ---------------------------------------------------------------------------
// dense systems (dense.hip)
// ---------------------------------------------------------------------------
// One integration pass over dense instances.  B = h^2 A column-major
// (Bc[j*s + i] = B_ij), [nsys][s][s] with nsys = 1 when shared; FP32 splits
// B into Bh + Bl.  State layout as for chains.
template <typename T>
struct DenseLaunch {
    int64_t batch;
    int32_t s;
    int32_t shared;
    const T *Bh, *Bl;
    const double *h;           // [nsys]
    const T *x0, *v0;
    T *state;
    int64_t nsteps, n0, out_stride;
    T *xf, *vf, *xe, *ve;
    int *nonfinite;
    int load_mode, store_mode;
};

template <typename T>
struct DenseItem {
    DenseLaunch<T> L;
    int64_t b;
};
// Work list of dense instances, one workgroup each; every item's s must be
// <= smax, which selects the kernel shape.
template <typename T>
osc_status dense_launch_items(const DenseItem<T> *items, int64_t nitems, int smax, int method, hipStream_t st);
// kernel shape bucket of the generic dense integrator for s (0..4)
int dense_vec_bucket(int s);

// A = M^-1 K for nsys systems ([nsys][s][s] row-major M, K, A); Lc scratch
// of the same size, Inv scratch of nsys * dense_form_scratch_elems(s)
// doubles; status |= 1 when a Cholesky pivot is not positive and finite.
size_t dense_form_scratch_elems(int s);
osc_status dense_form_a(int s, int64_t nsys, const double *M, const double *K, double *Lc, double *Inv, double *A,
                        int *status, hipStream_t st);
// Batched FP64 product on the matrix cores: C = A B (overwrite) or C -= A B,
// element (i, p) of A at A[i*a_i + p*a_p], (p, j) of B at B[p*b_p + j*b_j],
// (i, j) of C at C[i*c_i + j*c_j]; system z adds z times the *_sys strides.
// C may alias A only when n <= 64, B only when m <= 64.
struct Gemm64 {
    int m, n, k;
    int overwrite;
    const double *A;
    int64_t a_i, a_p;
    size_t a_sys;
    const double *B;
    int64_t b_p, b_j;
    size_t b_sys;
    double *C;
    int64_t c_i, c_j;
    size_t c_sys;
};
osc_status gemm64(const Gemm64 &g, int64_t nsys, hipStream_t st);
// B = h^2 A (column-major, split for FP32) and per-system row-sum bounds
// theta[sys] >= h omega_max.
template <typename T>
osc_status dense_prepare(int s, int64_t nsys, const double *A, const double *dt, T *Bh, T *Bl, double *theta,
                         int *bad, hipStream_t st);
// Power-iteration estimate h sqrt(lambda_max(A)) of one system.
osc_status dense_power_theta(int s, const double *A, double h, double *theta, hipStream_t st);
template <typename T>
osc_status dense_energy(int64_t batch, int s, int shared, const double *M, const double *K, const double *A,
                        const double *dt, const T *x, const T *v, double *E, bool shadow, hipStream_t st);
template <typename T>
osc_status dense_launch_vec(const DenseLaunch<T> &a, int method, hipStream_t st);

// Large-s dense path (dense_split.hip): three kernels per step over many
// workgroups; state planes always in device memory.
template <typename T>
struct DenseSplitLaunch {
    int64_t batch;
    int32_t s;
    int32_t shared;
    int32_t groups;            // column groups: the k dimension of a product is split over this many workgroups
    const T *Bh, *Bl;
    const double *h;
    const T *x0, *v0;
    T *state;                  // [4][batch][s]
    T *P;                      // [batch][s] Verlet: B x at the current step, carried between steps
    T *part;                   // [4][batch][groups][s] partial products of each column group
    int64_t *counter;          // completed steps (device)
    int64_t nsteps, n0, out_stride;
    T *xf, *vf, *xe, *ve;
    int *nonfinite;
    int load_mode, store_mode;
};
// column groups of the split path for s and batch; scratch elements it needs
int dense_split_groups(int s, int64_t batch);
size_t dense_split_scratch_elems(int s, int64_t batch);
template <typename T>
osc_status dense_split_run(const DenseSplitLaunch<T> &a, int method, hipStream_t st, hipGraphExec_t *graph,
                           int64_t *graph_steps, int64_t graph_chunk);

// Shared-operator MFMA path (dense_mfma.hip), FP32 state, s <= 256.
struct DenseMfmaLaunch {
    int64_t batch;
    int32_t s;
    const void *B1, *B2;       // FP16 operator fragments (hi, scaled lo)
    float inv_beta;            // 1 / beta, a power of two
    double h;
    // damped, driven launches (method kMfmaDriven + EX): Rayleigh damping
    // alpha M + beta K and the force M^-1 F cos(Omega t)
    double alpha, beta;
    const double *f;           // [batch][s] M^-1 F, or nullptr
    const double *omega;       // [batch]
    const float *x0, *v0;
    float *state;
    float *sigma;              // [batch] per-instance scale, carried with the state
    int64_t nsteps, n0, out_stride;
    int64_t frame_plane;       // elements between consecutive frames (normally batch * s)
    float *xf, *vf, *xe, *ve;
    int *nonfinite;
    int load_mode, store_mode;
};
struct DenseMfmaItem {
    DenseMfmaLaunch L;         // batch <= 16: one workgroup
};
// Work list of MFMA launches that all pad to `pad` (dense_mfma_pad).
osc_status dense_mfma_launch_items(const DenseMfmaItem *items, int64_t nitems, int pad, int method, hipStream_t st);
int dense_mfma_pad(int s);                       // padded size (multiple of 64), 0 if s > 256
size_t dense_mfma_fragment_elems(int s);         // FP16 elements per operator part
osc_status dense_mfma_fragments(int s, const double *A, double scale, _Float16 *B1, _Float16 *B2, hipStream_t st);
// method: OSC_RK4, OSC_VERLET, or kMfmaDriven + EX (RK4 of a damped, driven
// system; EX bit 0: beta != 0, bit 1: a force)
constexpr int kMfmaDriven = 4;
osc_status dense_mfma_launch(const DenseMfmaLaunch &a, int method, hipStream_t st);

// ---------------------------------------------------------------------------
// the schemes as matrices (propagator.hip)
// ---------------------------------------------------------------------------
struct PropArgs {
    int kind, method;
    int64_t nsys;              // systems: chains and per-instance dense = batch, shared dense = 1
    const double *m, *k;       // chains: [nsys][s] masses and springs
    const double *A;           // dense: [nsys][s][s] A = M^-1 K
    const double *h;           // [nsys]
};
template <typename T>
struct PropRun {
    int64_t batch, nsteps, out_stride;
    const T *x0, *v0;
    T *xf, *vf, *xe, *ve;
    int *nonfinite;
};
bool propagator_small(int s);   // s <= 2: one lane per system, P in registers
// P^k of every system, [nsys][2s][2s] row-major on (x, v), FP64.
osc_status propagator_matrix(const PropArgs &a, int s, int64_t k, double *out, hipStream_t st);
// Frames by P^out_stride, the rest of the run by P^r (FP64 state).
template <typename T>
osc_status propagator_jump(const PropArgs &a, int s, const PropRun<T> &run, hipStream_t st);
// Per-step propagator for chains of s <= 2 (same launch arguments and state
// planes as the chain kernel).
template <typename T>
osc_status prop_step_launch(const ChainLaunch<T> &a, int method, hipStream_t st);

// ---------------------------------------------------------------------------
// damped and driven systems (driven.hip)
// ---------------------------------------------------------------------------
template <typename T>
struct DrivenLaunch {
    int kind;                  // OSC_CHAIN / OSC_DENSE
    int64_t batch;
    int32_t s;
    int32_t shared;            // dense: one operator for every instance
    int32_t nbuf;              // LDS stage buffers (set by driven_launch)
    int32_t force_workgroup;   // chains: 1 = the workgroup kernel even where registers would do (tests)
    ChainCoef<T> c;            // chains
    const T *Bh, *Bl;          // dense: h^2 A column-major, [nsys][s][s]
    const double *h;           // chains [batch], dense [nsys]
    double alpha, beta;        // Rayleigh damping C = alpha M + beta K
    const double *f;           // [batch][s] M^-1 F, or nullptr (no force)
    const double *omega;       // [batch] force frequency
    const T *x0, *v0;
    T *state;                  // [4][batch][s] as for chains
    int64_t nsteps, n0, out_stride;
    T *xf, *vf, *xe, *ve;
    int *nonfinite;
    int load_mode, store_mode;
};
template <typename T>
osc_status driven_launch(const DrivenLaunch<T> &a, hipStream_t st);
// f = F / m (chains, [n] elements)
osc_status chain_force(int64_t n, const double *F, const double *m, double *f, hipStream_t st);

// ---------------------------------------------------------------------------
// coupled Van der Pol chains (vdp.hip): m_i x_i'' - mu (1 - x_i^2) x_i' +
// (K x)_i = F_i cos(Omega t) (force optional), classic RK4 in stage form,
// s <= 1024 (register layouts)
// ---------------------------------------------------------------------------
template <typename T>
struct VdpLaunch {
    int64_t batch;
    int32_t s;
    ChainCoef<T> c;
    const double *m;           // [batch][s] masses
    double mu;
    const T *x0, *v0;
    T *state;                  // [4][batch][s] as for chains
    int64_t nsteps, n0, out_stride;
    T *xf, *vf, *xe, *ve;
    int *nonfinite;
    int load_mode, store_mode;
    const double *f;           // [batch][s] F / m, or nullptr (no force)
    const double *omega;       // [batch] force frequency
};
template <typename T>
osc_status vdp_launch(const VdpLaunch<T> &a, hipStream_t st);
// f_b = M^-1 F_b for dense systems (M^-1 by the Cholesky formation with K = I)
osc_status dense_force(int s, int64_t nsys, int64_t batch, const double *M, const double *F, double *f,
                       int *notspd, hipStream_t st);

// runtime helpers shared by the server (api.hip)
template <typename T>
ChainCoef<T> chain_coef(const osc_sys *s);
bool dense_uses_split(const osc_sys *s);
osc_status sys_ensure_state(osc_sys *s);
osc_status sys_ensure_split_scratch(osc_sys *s);
// the handle's part of a split-path launch (operator, state, scratch layout)
template <typename T>
void split_launch_base(osc_sys *s, DenseSplitLaunch<T> &a);
void autotune_apply_cached(osc_sys *s);   // autotune.hip
// One real-time tick: k steps from global step n0 (LOAD_USER from x0, v0 when
// n0 == 0, else the held state), the new state stored back and written to
// (xe, ve).  OSC_ENOTSUP for paths that keep no per-launch state planes.
osc_status sys_rt_tick(osc_sys *s, const void *x0, const void *v0, int64_t n0, int64_t k, void *xe, void *ve);
osc_status sys_rt_supported(const osc_sys *s);
// Resident stepping of a chain handle: launch the resident kernel for nticks
// ticks of k steps from global step n0 (outputs as in ResidentRun, untyped);
// *blocks receives its workgroup count.  OSC_ENOTSUP for other handles.
struct ResidentSpec {
    RtControl *ctl;
    int64_t nticks, n0, k, idle_ticks;
    void *xf, *vf, *xo, *vo;
};
osc_status sys_rt_resident_supported(const osc_sys *s);
osc_status sys_rt_resident(osc_sys *s, const void *x0, const void *v0, const ResidentSpec &spec, int64_t *blocks);

}  // namespace osc

// Opaque handle (definition shared by the host runtime files).
struct osc_sys {
    osc_kind kind;
    osc_method method;
    osc_prec prec;
    int32_t s;
    int64_t batch;
    int32_t shared;
    hipStream_t stream;
    int device;
    // FP64 parameters kept on the device (energy needs M and K)
    double *m = nullptr, *k = nullptr;   // chain: [batch][s]; dense: M, K [nsys][s][s]
    double *h = nullptr;                 // chain: [batch]; dense: [nsys]
    void *coef = nullptr;                // chain coefficients (4 planes of T)
    double *A = nullptr;                 // dense: A = M^-1 K [nsys][s][s] (FP64)
    void *Bh = nullptr, *Bl = nullptr;   // dense: h^2 A column-major, hi / lo parts
    int64_t nsys = 0;                    // dense: number of distinct systems
    void *F1 = nullptr, *F2 = nullptr;   // dense FP32, s <= 256: MFMA operator fragments [nsys]
    float inv_beta = 1.0f;
    float *inv_betas = nullptr;          // host copy, one per system
    double *h_host = nullptr;            // host copy of each system's step
    void *mfma_items = nullptr;          // device work list (per-instance operators)
    size_t mfma_items_bytes = 0;
    double h_shared = 0.0;
    // configuration (osc_set_config)
    int dense_kernel = 0;                // 0 auto, 1 VALU, 2 MFMA, 3 split
    int64_t graph_steps = 64;            // steps per captured hipGraph (split path), 0 = eager
    void *split_scratch = nullptr;       // carried P, partial products and the step counter
    hipGraphExec_t split_graph = nullptr;
    int64_t split_graph_len = 0;
    unsigned char split_key[256] = {};   // launch arguments the graph was captured with
    int64_t steps_per_launch = 0;        // 0: whole run in one launch
    void *state = nullptr;               // internal state planes for chunked runs
    size_t state_bytes = 0;
    int *flag = nullptr;                 // device non-finite flag
    void *plain_state = nullptr;         // state planes of the plain baseline
    double theta_max = 0.0;              // largest dt * omega bound over the batch
    osc::ChainConfig cfg{1, 1};
    // osc_integrate_static: for the length of one call the chunked-run state
    // and the split path's buffers are parts of the library's static device
    // scratch instead of the handle's own (allocated on demand), and no graph
    // is captured
    int propagator = 0;                  // OSC_CFG_PROPAGATOR: 0 off, 1 frame jumps, 2 per-step (chains s <= 2)
    // osc_set_excitation: Rayleigh damping and harmonic force (RK4 only)
    bool driven = false;
    double alpha = 0.0, beta = 0.0;
    double *force = nullptr;             // [batch][s] M^-1 F (device), or nullptr
    double *omega = nullptr;             // [batch] (device)
    // osc_set_van_der_pol: a Van der Pol element on every body (chains, RK4)
    double vdp_mu = 0.0;
    // real-time stepping (osc_rt_tick): the next integration is one launch
    // from global step rt_n0 that loads the held state (or the given initial
    // state when rt_load == LOAD_USER) and stores it back beside the output
    bool rt_chunk = false;
    int64_t rt_n0 = 0;
    int rt_load = 0;
    bool static_call = false;
    void *scratch_state = nullptr;
    void *scratch_split = nullptr;
};
