/*
 * osc.h -- C ABI of libosc, a gfx950 (MI355X) integrator for coupled linear
 * oscillators.
 *
 * The systems are those of eq. (1) of Al-Oraiqat, "Parallel implementation
 * of the coupled harmonic oscillator" (arXiv 1702.02207):
 *     sum_j (m_ij x_j'' + k_ij x_j) = 0,   i.e.   x'' = -A x,  A = M^-1 K,
 * reduced to the first-order system x' = v, v' = -A x (section 3) and advanced
 * with a fixed step by classic four-stage Runge-Kutta (RK4) or by velocity
 * Verlet.  Many independent instances are integrated at once.
 *
 * Two kinds of system are accepted:
 *   OSC_CHAIN  the fixed-free spring chain of eq. (2) / Fig. 1 generalised to
 *              s bodies: diagonal M (masses m_i) and tridiagonal K.  Spring 0
 *              ties body 0 to the wall, spring i (i >= 1) joins bodies i-1 and
 *              i, the last body is free.  s = 2 is exactly eq. (2) with
 *              C1 = k[0], C2 = k[1].
 *   OSC_DENSE  a general eq. (1) system: M symmetric positive definite and K
 *              symmetric, both full s x s.  A = M^-1 K is formed on the GPU in
 *              FP64 through the Cholesky factor of M.
 *
 * Conventions shared by every entry point
 *   - All functions return an osc_status; no exception or abort crosses the
 *     ABI.  On failure, osc_last_error() returns a thread-local message.
 *   - State arrays are instance-major, row-major [batch][s].  Their element
 *     type follows the precision: double for OSC_F64, float for OSC_F32.
 *   - Frames are the states at steps n = 0, out_stride, 2*out_stride, ...
 *     (n <= nsteps), stored [nframes][batch][s] with
 *     nframes = nsteps / out_stride + 1; out_stride == 0 means no frames.
 *     The time of frame f is t = f * out_stride * dt, formed in FP64 from
 *     the integer step count.
 *   - Device arrays are owned by the caller; the library never frees them and
 *     keeps no pointer to them after the call's work has been enqueued.
 *   - Work is enqueued on the stream given at creation (a hipStream_t; NULL
 *     is the null stream).  osc_integrate and osc_energy are asynchronous:
 *     they validate their arguments and return at once.  Errors found on the
 *     device (a non-finite state) are reported by osc_sync.
 *   - A handle may be used by one host thread at a time.
 */
#ifndef OSC_H
#define OSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OSC_ABI_VERSION 1

typedef enum {
    OSC_OK = 0,
    OSC_EINVAL = 1,      /* invalid argument (null pointer, size, enum, dt <= 0, ...) */
    OSC_ENOTSPD = 2,     /* the Cholesky factorisation of M failed: M is not SPD */
    OSC_EUNSTABLE = 3,   /* dt * omega_max lies outside the scheme's stability interval */
    OSC_ENOMEM = 4,      /* device memory (or the configured HBM budget) exhausted */
    OSC_EDEVICE = 5,     /* a HIP runtime call failed */
    OSC_ENONFINITE = 6,  /* a state became NaN or infinite (reported by osc_sync) */
    OSC_ENOTSUP = 7,     /* a combination this build does not provide */
    OSC_ETIMEOUT = 8,    /* a wait ran out of time */
    OSC_EBUSY = 9        /* the server is full / shutting down */
} osc_status;

typedef enum { OSC_CHAIN = 0, OSC_DENSE = 1 } osc_kind;
typedef enum { OSC_RK4 = 0, OSC_VERLET = 1 } osc_method;
typedef enum { OSC_F64 = 0, OSC_F32 = 1 } osc_prec;
typedef enum { OSC_MEM_HOST = 0, OSC_MEM_DEVICE = 1 } osc_mem;

/*
 * Description of a batch of systems.
 *
 * OSC_CHAIN:  M = masses  [batch][s] (> 0),  K = springs [batch][s] (>= 0,
 *             K[b][0] > 0 is the wall spring),  dt = [batch] (> 0).
 * OSC_DENSE:  shared != 0: M, K are [s][s] row-major, used by every instance,
 *             dt = [1];  shared == 0: M, K are [batch][s][s], dt = [batch].
 * param_mem tells whether M, K and dt are host or device pointers.  They are
 * read during osc_create only; the caller may free them afterwards.
 *
 * prec = OSC_F32 keeps the state in FP32 with compensated (two-term) updates
 * and coefficients split into FP32 high + low parts; dense products with a
 * shared operator (s <= 256) run on MFMA with the operator and operands split
 * into FP16 high and scaled low parts (three terms for B x, two for B w, one
 * for the higher-order products; FP32 accumulation); results stay within the
 * FP32 tolerance of the FP64 reference.
 * prec = OSC_F64 runs everything in double.
 */
typedef struct osc_desc {
    osc_kind kind;
    osc_method method;
    osc_prec prec;
    int32_t s;            /* degrees of freedom per instance, >= 1 */
    int64_t batch;        /* number of instances, >= 0 (0: every call is a no-op) */
    int32_t shared;       /* dense only */
    osc_mem param_mem;
    const double *M;
    const double *K;
    const double *dt;
} osc_desc;

typedef struct osc_sys osc_sys;

/*
 * osc_create -- validate a description and prepare the device-side system
 * (eq. (1)): for chains, the per-body coefficients of A = M^-1 K scaled by
 * dt^2; for dense systems, A = M^-1 K by FP64 Cholesky and its scaled split
 * operands.  Checks positive definiteness (OSC_ENOTSPD) and stability: the
 * step is rejected (OSC_EUNSTABLE) when dt * omega_bound exceeds 2.78 for
 * RK4 (the imaginary-axis limit is 2*sqrt(2)) or 1.99 for Verlet (limit 2).
 * omega_bound is first a cheap upper bound (Gershgorin for chains, the
 * largest absolute row sum of A for dense systems); when that exceeds the
 * limit it is replaced by an estimate of the largest frequency itself: for
 * chains the exact value (Sturm-sequence bisection on the symmetric
 * tridiagonal M^-1/2 K M^-1/2, FP64) with a 1 % margin, for dense systems
 * power iteration (which approaches it from below) with a 2 % margin.
 * Blocks until the preparation has finished.
 * stream: hipStream_t or NULL.  *out receives a new handle on success.
 */
osc_status osc_create(const osc_desc *desc, void *stream, osc_sys **out);

/*
 * osc_integrate -- advance every instance nsteps steps from (x0, v0).
 * x0, v0:            device [batch][s] initial state (read only).
 * x_frames, v_frames: device [nframes][batch][s] or NULL to skip.
 * x_end, v_end:      device [batch][s] final state, or NULL to skip.
 * nsteps = 0 copies the initial state out.  Asynchronous on the handle's
 * stream.  The result of an instance does not depend on the batch it sits
 * in or on the launch configuration chosen.
 */
osc_status osc_integrate(osc_sys *sys, const void *x0, const void *v0, int64_t nsteps,
                         int64_t out_stride, void *x_frames, void *v_frames, void *x_end,
                         void *v_end);

/*
 * osc_integrate_static -- osc_integrate for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, and bit for bit the same results,
 * as osc_integrate with the handle's configuration.  Every device buffer the
 * run needs beyond the caller's inputs and outputs (the compensated state
 * carried between launches when OSC_CFG_STEPS_PER_LAUNCH splits the run; the
 * split dense path's state, carried product, partial sums and step counter)
 * is taken from one scratch array of OSC_STATIC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and
 * captures no graph: its kernels are enqueued directly on the handle's stream,
 * so that a caller may capture them.  The first call on a device looks up the
 * array's address there (hipGetSymbolAddress).  Nothing in the scratch needs
 * to start at zero: every value is written before it is read.
 * Errors: OSC_ENOMEM (with the size needed) when the run needs more scratch
 * than the maximum (a chunked run needs 4 * batch * s elements plus one float
 * per instance; the split path that plus (1 + 4 * column groups) * batch * s
 * elements); OSC_ENOTSUP for dense systems with per-instance operators on the
 * matrix-core path (their work list is uploaded per call).
 * Every call on one device shares that device's scratch: calls that overlap
 * in time on one device (on different streams or host threads) race, and the
 * caller must order them.
 */
#define OSC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
osc_status osc_integrate_static(osc_sys *sys, const void *x0, const void *v0, int64_t nsteps,
                                int64_t out_stride, void *x_frames, void *v_frames, void *x_end,
                                void *v_end);

/*
 * osc_integrate_plain -- the same result as osc_integrate with no frames,
 * computed the plain way: one instance at a time and one time step per kernel
 * launch, with the state kept in device memory between launches.  It exists
 * as the per-instance baseline that the batched path is measured against.
 */
osc_status osc_integrate_plain(osc_sys *sys, const void *x0, const void *v0, int64_t nsteps,
                               void *x_end, void *v_end);

/*
 * osc_energy -- E[b] = 1/2 v^T M v + 1/2 x^T K x for every instance, in FP64
 * on the device (chain: 1/2 sum m_i v_i^2 + 1/2 sum k_i (x_i - x_{i-1})^2).
 * x, v: device [batch][s] in the handle's precision; E: device double [batch].
 */
osc_status osc_energy(osc_sys *sys, const void *x, const void *v, double *E);

/*
 * osc_shadow_energy -- the quantity velocity Verlet conserves exactly:
 * Q[b] = v^T M v + x^T K x - (dt^2/4) (K x)^T M^-1 (K x), FP64 on the device.
 * Same arguments as osc_energy.
 */
osc_status osc_shadow_energy(osc_sys *sys, const void *x, const void *v, double *Q);

/*
 * osc_set_excitation -- damp and drive every instance of the handle: eq. (1)
 * with Rayleigh damping C = alpha M + beta K and a harmonic force,
 *     M x'' + C x' + K x = F cos(Omega t),
 * integrated by classic RK4 on the first-order form of section 3 (stages at
 * t_n, t_n + dt/2, t_n + dt/2, t_n + dt; t_n = n dt from the integer step).
 * alpha, beta >= 0 (same for every instance).  F: forces [batch][s] (host or
 * device per mem), or NULL for no force; Omega: [batch] frequencies (rad per
 * unit time), required with F.  Dense systems take f = M^-1 F on the GPU (FP64,
 * by the Cholesky factor of M).  alpha = beta = 0 and F = NULL make the
 * handle free again.  Afterwards osc_integrate (and osc_integrate_static) run
 * the damped / driven integrator: chains of s <= 1024 in registers, one
 * operator shared by many instances (FP32, s <= 256) on the matrix cores, the
 * others one workgroup per instance (s <= 2048);
 * osc_integrate_plain and the propagator modes return OSC_ENOTSUP; osc_energy
 * still returns 1/2 v^T M v + 1/2 x^T K x (no longer conserved).
 * OSC_ENOTSUP for a Verlet handle (the velocity-dependent force would make the
 * scheme implicit), and for damping on a Van der Pol chain (osc_set_van_der_pol;
 * a force alone drives it).  OSC_EUNSTABLE when dt * max(omega_max, alpha + beta
 * omega_max^2) exceeds 2.5: every mode's |lambda| is at most that, and RK4's
 * stability region holds the left half-disk of radius 2.6156.  Synchronous.
 */
osc_status osc_set_excitation(osc_sys *sys, double alpha, double beta, const double *F, const double *Omega,
                              osc_mem mem);

/*
 * osc_set_van_der_pol -- put a Van der Pol element on every body of a chain
 * (section 1 names the Van der Pol system as the standard model of nonlinear
 * oscillation):
 *     m_i x_i'' - mu (1 - x_i^2) x_i' + (K x)_i = 0,
 * the spring chain of eq. (2) with each body pumped while |x_i| < 1 and
 * damped beyond.  mu >= 0, finite, the same for every instance; mu = 0 makes
 * the handle linear again.  Afterwards osc_integrate (and osc_integrate_static
 * and both real-time steppers) run classic RK4 in stage form on the
 * first-order system of section 3, in registers.  The linear stability
 * check of osc_create still applies; the nonlinear term is not bounded by it
 * (a step too long for the amplitude reached shows as OSC_ENONFINITE from
 * osc_sync).  osc_energy returns 1/2 v^T M v + 1/2 x^T K x (not conserved).
 * A force set by osc_set_excitation (alpha = beta = 0) drives the Van der Pol
 * chain: m_i x_i'' - mu (1 - x_i^2) x_i' + (K x)_i = F_i cos(Omega t), the
 * forced Van der Pol oscillator, with the force's phase as in the damped,
 * driven integrator.
 * OSC_EINVAL for a negative or non-finite mu; OSC_ENOTSUP for dense handles,
 * Verlet handles, s > 1024, a handle with Rayleigh damping, or a propagator
 * mode.  The plain baseline, osc_propagator and osc_autotune
 * return OSC_ENOTSUP while mu > 0.  Synchronous, host only.
 */
osc_status osc_set_van_der_pol(osc_sys *sys, double mu);

/*
 * osc_propagator -- the matrix of k steps of the handle's scheme.  For
 * eq. (1) the first-order system of section 3 is y' = L y with the constant
 * L = [[0, I], [-A, 0]], y = (x, v), so k steps of either scheme are one
 * matrix: y_{n+k} = P_k y_n.  One RK4 step is the degree-4 Taylor polynomial
 * of exp(hL): with B = h^2 A, C = I - B/2 + B^2/24, S = I - B/6,
 *   P_1 = [[C, h S], [-(B - B^2/6)/h, C]];
 * one velocity Verlet step is P_1 = [[I - B/2, h I], [-(B - B^2/4)/h, I - B/2]].
 * P_k = P_1^k by repeated squaring, all in FP64 on the GPU.
 * P: device double [nsys][2s][2s] row-major, positions first (nsys = batch
 * for chains and per-instance dense systems, 1 for a shared operator).
 * Any s up to 2048; for s > 2 the call takes device temporaries of four
 * [nsys][2s][2s] FP64 matrices (OSC_ENOMEM when they do not fit).  k = 0
 * gives the identity.  Ordered on the handle's stream; for s > 2 the call
 * waits for its own temporaries.
 */
osc_status osc_propagator(osc_sys *sys, int64_t k, double *P);

/*
 * osc_dense_operator -- copy A = M^-1 K of a dense handle, formed on the GPU
 * in FP64 by Cholesky (eq. (1)), to the device array A ([nsys][s][s]
 * row-major, nsys = 1 when shared, else batch).  Asynchronous.  OSC_EINVAL
 * for a chain handle.
 */
osc_status osc_dense_operator(osc_sys *sys, double *A);

/*
 * Launch configuration of a handle.  None of these changes a result beyond
 * the rounding differences stated here; they exist for tuning and testing.
 *   OSC_CFG_CHAIN_LAYOUT      chains: (lanes_per_instance << 16) | dofs_per_lane,
 *                             one of the layouts the library is built for
 *                             (0 = automatic).  Results are bitwise identical
 *                             across layouts.
 *   OSC_CFG_DENSE_KERNEL      dense: 0 automatic, 1 VALU, one workgroup per
 *                             instance (any s), 2 MFMA (FP32, shared operator,
 *                             s <= 256), 3 split (each step three kernels over
 *                             many workgroups; for few instances of large s).
 *                             Damped / driven chains: 0 automatic (registers
 *                             for s <= 1024), 1 one workgroup per instance.
 *                             Damped / driven dense systems: 0 and 2 the
 *                             matrix cores where MFMA applies, 1 one
 *                             workgroup per instance.
 *   OSC_CFG_STEPS_PER_LAUNCH  maximum time steps per kernel launch (0 = the
 *                             whole run).  The state between launches keeps its
 *                             compensation terms, so chunked and unchunked runs
 *                             agree bitwise.
 *   OSC_CFG_GRAPH_STEPS       split dense path: steps per captured hipGraph
 *                             that is replayed (0 = launch eagerly; default 64).
 *   OSC_CFG_PROPAGATOR        the scheme applied as its matrix (osc_propagator):
 *                             0 off (default); 1 frame jumps: osc_integrate
 *                             forms P^out_stride and advances from frame to
 *                             frame by one product with it, the rest of the run
 *                             by P^r (r = nsteps - last frame step; P^nsteps
 *                             when out_stride == 0), with the state in FP64
 *                             (any s; for s > 2 six [nsys][2s][2s] FP64
 *                             temporaries, OSC_ENOMEM from osc_integrate when
 *                             they do not fit): the scheme's own trajectory at the
 *                             frames, rounded differently and not computed at
 *                             the steps in between; 2 per-step propagator for
 *                             chains of s <= 2: each step applies P - I (FP32:
 *                             split into high and low parts) to the compensated
 *                             state.
 * Returns OSC_EINVAL for an unknown key or value, OSC_ENOTSUP for a layout or
 * kernel this handle cannot use.
 */
typedef enum {
    OSC_CFG_CHAIN_LAYOUT = 1,
    OSC_CFG_DENSE_KERNEL = 2,
    OSC_CFG_STEPS_PER_LAUNCH = 3,
    OSC_CFG_GRAPH_STEPS = 4,
    OSC_CFG_PROPAGATOR = 5
} osc_config;
osc_status osc_set_config(osc_sys *sys, osc_config key, int64_t value);

/*
 * osc_autotune -- time every feasible launch configuration of the handle on
 * its own batch (chains: the lane layouts; dense: the VALU / MFMA / split
 * kernels), probe_steps steps each starting from (x0, v0) (device arrays as
 * for osc_integrate; nothing is written to them), and keep the fastest.
 * *chosen (may be NULL) receives the configuration value, as accepted by
 * osc_set_config.  When the environment variable OSC_AUTOTUNE_CACHE names a
 * file, the choice is appended to it, and osc_create applies the cached
 * choice for the same kind, method, precision, s, batch size class and GPU.
 * Synchronous.  Chain layouts give bitwise-identical results; dense kernels
 * agree within the FP32 tolerance.  OSC_ENOTSUP for handles with damping,
 * a force or Van der Pol elements (their kernels take fixed layouts).
 */
osc_status osc_autotune(osc_sys *sys, const void *x0, const void *v0, int64_t probe_steps, int64_t *chosen);

/* osc_sync -- wait for the handle's stream; returns OSC_ENONFINITE if any
 * integration since the last osc_sync produced a non-finite state. */
osc_status osc_sync(osc_sys *sys);

/* osc_destroy -- release the handle (waits for its queued work).  NULL is a no-op. */
void osc_destroy(osc_sys *sys);

/* osc_last_error -- description of the last failure on this thread ("" if none). */
const char *osc_last_error(void);

/* osc_abi_version -- OSC_ABI_VERSION of the loaded library. */
int osc_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Real-time periodic stepping.                                              */
/* ------------------------------------------------------------------------ */
/*
 * The paper proposes the oscillator model as a time-critical workload for
 * hardware- and software-in-the-loop simulation and as a benchmark of the
 * delay of parallel systems and of periodic hard-deadline threads
 * (introduction, section 5).  A real-time stepper holds one handle's state on
 * the device and advances it by one tick (steps_per_tick steps, one kernel
 * launch) at a time.  A tick continues the handle's integration from the
 * global step count with its compensation terms, so the states after the
 * ticks are bit for bit the frames of one osc_integrate call with
 * out_stride = steps_per_tick.  Supported: chains, dense systems on the VALU
 * and shared-operator MFMA paths, damped / driven systems, the per-step
 * propagator; OSC_ENOTSUP for frame jumps, the split dense path and
 * per-instance dense operators on the matrix cores.  The handle must outlive
 * the stepper and not be integrated in between.
 */
typedef struct osc_rt osc_rt;

/* osc_rt_create -- a stepper at step 0 from (x0, v0) (device [batch][s], copied). */
osc_status osc_rt_create(osc_sys *sys, const void *x0, const void *v0, int64_t steps_per_tick, osc_rt **out);

/* osc_rt_tick -- advance one tick, asynchronously on the handle's stream; the
 * new state goes to x_out, v_out (device [batch][s]; NULL: kept internally). */
osc_status osc_rt_tick(osc_rt *rt, void *x_out, void *v_out);

/* osc_rt_steps -- steps taken so far (-1 for NULL). */
int64_t osc_rt_steps(const osc_rt *rt);

typedef struct osc_rt_stats {
    int64_t ticks;         /* periods run */
    int64_t missed;        /* ticks whose result was ready only after the next release */
    double p50_s, p99_s, max_s, mean_s;   /* latency: release time -> result ready (host clock) */
    double jitter_s;       /* standard deviation of the latency */
    double launch_p99_s;   /* release -> tick enqueued, 99th percentile */
    double gpu_p50_s;      /* device time of a tick (events around its launch), median */
} osc_rt_stats;

/*
 * osc_rt_run -- the periodic loop: nticks periods of period_s seconds (0 <
 * period_s < 60) on the host's steady clock.  At each release time one tick
 * is enqueued and its completion event polled (at most max(10 s, 100 periods)
 * per tick: OSC_ETIMEOUT beyond); the latency is release -> completion seen
 * by the host, and a tick misses its deadline when that exceeds one period.
 * x_frames, v_frames: device [nticks][batch][s] for the state after each tick,
 * or NULL; latencies: host double [nticks] or NULL; stats may be NULL.
 * Blocks for about nticks * period_s.
 */
osc_status osc_rt_run(osc_rt *rt, double period_s, int64_t nticks, void *x_frames, void *v_frames,
                      double *latencies, osc_rt_stats *stats);

/*
 * osc_rt_run_resident -- the same periodic loop with one kernel resident on
 * the device for the whole run instead of one launch per tick (chain handles,
 * damped or driven ones with s <= 1024 on the register kernels, not in a
 * propagator mode: OSC_ENOTSUP otherwise, also when the batch needs more
 * workgroups than the device holds at once).  At each release the host raises a counter in host-mapped memory;
 * every workgroup of the kernel polls it, advances its instances one tick,
 * stores the tick's result (x_frames / v_frames as for osc_rt_run, else the
 * stepper's own output buffers) and raises a completion count the host polls.
 * The trajectory is bitwise that of osc_rt_run / osc_rt_tick.  A workgroup
 * that sees no release for the idle limit (osc_rt_set_idle_limit; default
 * max(0.1 s, 50 periods)) ends the kernel: the host then returns
 * OSC_ETIMEOUT, as it does when a tick takes longer than max(10 s, 100
 * periods).  After any error of this call the stepper's held state is
 * undefined: later calls on it return OSC_EDEVICE; destroy it.  gpu_p50_s is
 * 0 (no per-tick events); launch_p99_s is release -> counter raised.
 */
osc_status osc_rt_run_resident(osc_rt *rt, double period_s, int64_t nticks, void *x_frames, void *v_frames,
                               double *latencies, osc_rt_stats *stats);

/* osc_rt_set_idle_limit -- idle limit of osc_rt_run_resident in seconds (> 0;
 * 0 restores the default). */
osc_status osc_rt_set_idle_limit(osc_rt *rt, double seconds);

/* osc_rt_destroy -- release the stepper (waits for its queued ticks).  NULL is a no-op. */
void osc_rt_destroy(osc_rt *rt);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of single-instance integration requests.     */
/* ------------------------------------------------------------------------ */
/*
 * The paper proposes the oscillator model as a time-critical workload for
 * hardware- and software-in-the-loop simulation and as a delay benchmark of
 * parallel systems (introduction and conclusion).  A server runs many such
 * integrations at once: requests of either kind, any s and step count are
 * admitted, first come first served, while the bytes they hold on the device
 * fit the HBM budget and a slot is free.  A worker thread then advances every
 * admitted request by one chunk of time steps per scheduler iteration,
 * batching requests of the same kernel shape into one work-list launch; a
 * request that arrives while others run joins at the next iteration, and a
 * finished one frees its memory and slot for the queue.  Chunk lengths depend
 * only on the request itself, so every result is bitwise the same whether the
 * request ran alone or in a mix.  Parameters and results are host arrays.
 */
typedef struct osc_server osc_server;

typedef struct osc_server_config {
    size_t hbm_budget;        /* device bytes the admitted requests may hold (0 = unlimited) */
    int32_t max_slots;        /* requests admitted at once (>= 1) */
    int32_t chunk_us;         /* target GPU time of one request chunk, microseconds (0 = 2000) */
    int32_t fake_executor;    /* 1: no device work; chunks take simulated time (scheduler tests) */
    int32_t frame_jumps;      /* 1: a dense request whose frames cost much less to reach by powers
                                 of its one-step matrix (OSC_CFG_PROPAGATOR = 1, FP64) than by
                                 stepping is served that way, whole, by the admitting thread;
                                 0: every request is stepped */
} osc_server_config;

typedef struct osc_request_info {
    osc_status status;        /* OSC_OK or the error that ended the request */
    double queue_s;           /* submit -> admitted */
    double latency_s;         /* submit -> results ready */
    int64_t bytes;            /* device bytes accounted to the request */
    int64_t iterations;       /* scheduler iterations the request took part in */
    int32_t frame_jumps;      /* 1 if the request was served by frame jumps */
} osc_request_info;

typedef struct osc_server_counters {
    int64_t submitted, completed, failed, queued, active;
    int64_t iterations;
    size_t hbm_in_use, hbm_peak;   /* accounted device bytes of admitted requests */
    double setup_s;                /* worker time spent admitting (allocation, operator formation) */
    double iterate_s;              /* worker time spent in scheduler iterations (launch to sync) */
} osc_server_counters;

/* osc_server_create -- start a server (and its worker thread) on the current
 * device.  cfg is copied. */
osc_status osc_server_create(const osc_server_config *cfg, osc_server **out);

/*
 * osc_server_submit -- queue one integration.  desc describes one instance
 * (batch must be 1; dense systems are given by their own M, K, shared = 1),
 * with host parameters (param_mem = OSC_MEM_HOST); x0, v0 are host arrays of
 * s elements of the request's precision.  Everything is copied before the call
 * returns.  *ticket identifies the request.  OSC_ENOMEM if the request alone
 * exceeds the budget, OSC_EBUSY after shutdown began.
 */
osc_status osc_server_submit(osc_server *srv, const osc_desc *desc, const void *x0, const void *v0,
                             int64_t nsteps, int64_t out_stride, uint64_t *ticket);

/*
 * osc_server_wait -- wait up to timeout_s seconds (< 0: forever) for a
 * request; on completion copy its results to the host arrays given (any may
 * be NULL): frames [nframes][s], final state [s], and fill *info.  The request
 * is forgotten after a successful wait.  OSC_ETIMEOUT if it is not done yet;
 * the request's own error status otherwise.
 */
osc_status osc_server_wait(osc_server *srv, uint64_t ticket, double timeout_s, void *x_frames, void *v_frames,
                           void *x_end, void *v_end, osc_request_info *info);

/* osc_server_stats -- counters of the server so far. */
osc_status osc_server_stats(osc_server *srv, osc_server_counters *out);

/* osc_server_destroy -- finish the admitted requests, fail the queued ones,
 * stop the worker and release everything.  NULL is a no-op. */
void osc_server_destroy(osc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* OSC_H */
