// Host runtime behind the C ABI declared in include/osc.h.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "osc_internal.h"
#include "vdp.h"

// Device scratch of the allocation-free entry point (osc_integrate_static):
// each device that runs the library holds its own copy from the library's
// load on that device until the process ends.  In host code `scratch` names
// a host-side stand-in, never the device memory: kernels and copies take the
// per-device address that static_scratch() obtains from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[OSC_STATIC_SCRATCH_BYTES];

namespace osc {

namespace {
thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on `device`, looked up once per device with that
// device current (the caller's current device is restored).
osc_status static_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return fail(OSC_EDEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        OSC_HIP(hipGetDevice(&cur));
        if (cur != device) OSC_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(OSC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return OSC_OK;
}

// Stability limits on the imaginary axis with a small margin: RK4 is stable
// for h omega <= 2 sqrt(2) = 2.828, velocity Verlet for h omega < 2.
constexpr double kRk4Limit = 2.78;
constexpr double kVerletLimit = 1.99;
// safety factor on an exact (chains) largest frequency
constexpr double kStabilityMargin = 1.01;

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { pool_free(p); }
};

osc_status copy_in(void *dst, const void *src, size_t bytes, osc_mem where, hipStream_t st) {
    if (bytes == 0) return OSC_OK;
    OSC_HIP(hipMemcpyAsync(dst, src, bytes, where == OSC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           st));
    return OSC_OK;
}

void release(osc_sys *s) {
    if (!s) return;
    for (void *p : {(void *)s->m, (void *)s->k, (void *)s->h, s->coef, (void *)s->flag, s->plain_state,
                    (void *)s->A, s->Bh, s->Bl, s->F1, s->F2, s->state, s->split_scratch, (void *)s->force,
                    (void *)s->omega})
        pool_free(p);
    pool_free(s->mfma_items);
    if (s->split_graph) (void)hipGraphExecDestroy(s->split_graph);
    delete[] s->inv_betas;
    delete[] s->h_host;
    delete s;
}

size_t elem(const osc_sys *s) { return s->prec == OSC_F64 ? sizeof(double) : sizeof(float); }

// State planes [4][batch][s] followed by one float per instance (the MFMA
// path's operand scale).
size_t state_bytes(const osc_sys *s) { return 4 * (size_t)s->batch * s->s * elem(s) + (size_t)s->batch * sizeof(float); }

void *state_buf(const osc_sys *s) { return s->static_call ? s->scratch_state : s->state; }
void *split_buf(const osc_sys *s) { return s->static_call ? s->scratch_split : s->split_scratch; }

osc_status ensure_state(osc_sys *s) {
    if (s->static_call)
        return s->scratch_state ? OSC_OK : fail(OSC_EINVAL, "internal: no static scratch for the chunked state");
    const size_t need = state_bytes(s);
    if (s->state && s->state_bytes >= need) return OSC_OK;
    pool_free(s->state);
    s->state = pool_alloc(need);
    s->state_bytes = s->state ? need : 0;
    if (!s->state) return fail(OSC_ENOMEM, "device memory exhausted for the chunked-run state");
    return OSC_OK;
}

template <typename L>
void set_sigma(L &, osc_sys *) {}
void set_sigma(DenseMfmaLaunch &a, osc_sys *s) {
    a.sigma = reinterpret_cast<float *>(static_cast<char *>(state_buf(s)) + 4 * (size_t)s->batch * s->s * sizeof(float));
}

// Advance [0, nsteps) in launches of at most steps_per_launch steps, passing
// the compensated state through device memory between launches.
template <typename L, typename F>
osc_status run_chunks(osc_sys *s, L base, int64_t nsteps, F &&launch) {
    if (s->rt_chunk) {
        // one real-time tick
        osc_status r = ensure_state(s);
        if (r) return r;
        base.n0 = s->rt_n0;
        base.nsteps = nsteps;
        base.load_mode = s->rt_load;
        base.store_mode = STORE_STATE | STORE_USER;
        base.state = static_cast<decltype(base.state)>(state_buf(s));
        set_sigma(base, s);
        return launch(base);
    }
    const int64_t chunk = s->steps_per_launch > 0 ? s->steps_per_launch : nsteps;
    if (nsteps <= chunk) {
        base.n0 = 0;
        base.nsteps = nsteps;
        base.load_mode = LOAD_USER;
        base.store_mode = STORE_USER;
        return launch(base);
    }
    osc_status r = ensure_state(s);
    if (r) return r;
    for (int64_t n0 = 0; n0 < nsteps; n0 += chunk) {
        L a = base;
        a.n0 = n0;
        a.nsteps = chunk < nsteps - n0 ? chunk : nsteps - n0;
        a.load_mode = n0 == 0 ? LOAD_USER : LOAD_STATE;
        a.store_mode = n0 + a.nsteps == nsteps ? STORE_USER : STORE_STATE;
        a.state = static_cast<decltype(a.state)>(state_buf(s));
        set_sigma(a, s);
        if ((r = launch(a))) return r;
    }
    return OSC_OK;
}

// ------------------------------------------------------------------ chains

template <typename T>
ChainCoef<T> coef_of(const osc_sys *s) {
    const size_t n = (size_t)s->batch * s->s;
    T *base = static_cast<T *>(s->coef);
    ChainCoef<T> c;
    c.clh = base;
    c.crh = base + n;
    c.cll = std::is_same<T, float>::value ? base + 2 * n : nullptr;
    c.crl = std::is_same<T, float>::value ? base + 3 * n : nullptr;
    c.h = s->h;
    return c;
}

template <typename T>
osc_status create_chain(osc_sys *s, const osc_desc *d) {
    const size_t n = (size_t)s->batch * s->s;
    const hipStream_t st = s->stream;
    s->m = static_cast<double *>(pool_alloc(n * sizeof(double)));
    s->k = static_cast<double *>(pool_alloc(n * sizeof(double)));
    s->h = static_cast<double *>(pool_alloc((size_t)s->batch * sizeof(double)));
    const int planes = std::is_same<T, float>::value ? 4 : 2;
    s->coef = pool_alloc(planes * n * sizeof(T));
    s->flag = static_cast<int *>(pool_alloc(64));
    DevBuf scratch;   // [theta bound (double)][bad flag (int)]
    scratch.p = pool_alloc(64);
    if (!s->m || !s->k || !s->h || !s->coef || !s->flag || !scratch.p)
        return fail(OSC_ENOMEM, "device memory / HBM budget exhausted in osc_create");
    osc_status r;
    if ((r = copy_in(s->m, d->M, n * sizeof(double), d->param_mem, st))) return r;
    if ((r = copy_in(s->k, d->K, n * sizeof(double), d->param_mem, st))) return r;
    if ((r = copy_in(s->h, d->dt, (size_t)s->batch * sizeof(double), d->param_mem, st))) return r;
    OSC_HIP(hipMemsetAsync(s->flag, 0, 64, st));
    OSC_HIP(hipMemsetAsync(scratch.p, 0, 64, st));
    double *theta = static_cast<double *>(scratch.p);
    int *bad = reinterpret_cast<int *>(static_cast<char *>(scratch.p) + 8);
    T *base = static_cast<T *>(s->coef);
    r = chain_prepare<T>(s->batch, s->s, s->m, s->k, s->h, base, base + n, planes == 4 ? base + 2 * n : nullptr,
                         planes == 4 ? base + 3 * n : nullptr, /*hout=*/nullptr, theta, bad, st);
    if (r) return r;
    struct {
        double theta;
        int bad;
        int pad;
    } host{};
    OSC_HIP(hipMemcpyAsync(&host, scratch.p, 16, hipMemcpyDeviceToHost, st));
    OSC_HIP(hipStreamSynchronize(st));
    if (host.bad) return fail(OSC_EINVAL, "chain parameters need m > 0, k >= 0 and finite dt > 0");
    const double lim = s->method == OSC_RK4 ? kRk4Limit : kVerletLimit;
    double est = host.theta;   // Gershgorin bound: accepted as it is when within the limit
    if (!(est <= lim)) {
        // The bound can exceed h omega_max by up to sqrt(2) (unequal masses
        // across a stiff spring): decide on the exact largest frequency of
        // each chain instead, with a 1 % margin.
        DevBuf th;
        th.p = pool_alloc((size_t)s->batch * sizeof(double));
        if (!th.p) return fail(OSC_ENOMEM, "device memory exhausted for the stability estimate");
        if ((r = chain_sturm_theta(s->batch, s->s, s->m, s->k, s->h, static_cast<double *>(th.p), st))) return r;
        std::vector<double> all((size_t)s->batch);
        OSC_HIP(hipMemcpyAsync(all.data(), th.p, all.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        OSC_HIP(hipStreamSynchronize(st));
        est = 0.0;
        for (double t : all) est = std::max(est, kStabilityMargin * t);
    }
    s->theta_max = est;
    if (!(est <= lim))
        return fail(OSC_EUNSTABLE, "dt * omega_max (with a 1 % margin) " + std::to_string(est) + " exceeds " +
                                       std::to_string(lim));
    s->cfg = chain_pick_config(s->s);
    return OSC_OK;
}

template <typename T>
osc_status integrate_chain(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                           void *xf, void *vf, void *xe, void *ve) {
    ChainLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.c = coef_of<T>(s);
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.nonfinite = s->flag;
    return run_chunks(s, a, nsteps,
                      [&](const ChainLaunch<T> &c) { return chain_launch<T>(c, s->method, s->cfg, s->stream); });
}

template <typename T>
osc_status plain_chain(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, void *xe, void *ve) {
    const size_t n = (size_t)s->batch * s->s;
    if (!s->plain_state) {
        s->plain_state = pool_alloc(4 * n * sizeof(T));
        if (!s->plain_state) return fail(OSC_ENOMEM, "device memory exhausted in osc_integrate_plain");
    }
    ChainLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.c = coef_of<T>(s);
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.state = static_cast<T *>(s->plain_state);
    a.nsteps = nsteps;
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.nonfinite = s->flag;
    return chain_plain<T>(a, s->method, s->stream);
}

// ------------------------------------------------------------------ dense

// Plain baseline for dense systems: one instance at a time and one time step
// per launch of the generic (VALU) integrator, the compensated state kept in
// device memory between launches.
template <typename T>
osc_status plain_dense(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, void *xe, void *ve) {
    const int64_t n = s->s;
    const size_t ss = (size_t)n * n;
    if (!s->plain_state) {
        s->plain_state = pool_alloc(4 * (size_t)s->batch * n * sizeof(T));
        if (!s->plain_state) return fail(OSC_ENOMEM, "device memory exhausted in osc_integrate_plain");
    }
    for (int64_t b = 0; b < s->batch; ++b) {
        DenseLaunch<T> a{};
        a.batch = 1;
        a.s = s->s;
        a.shared = 1;   // the instance's own operator, addressed directly
        a.Bh = static_cast<const T *>(s->Bh) + (s->shared ? 0 : b * ss);
        a.Bl = s->Bl ? static_cast<const T *>(s->Bl) + (s->shared ? 0 : b * ss) : nullptr;
        a.h = s->h + (s->shared ? 0 : b);
        a.nonfinite = s->flag;
        a.x0 = static_cast<const T *>(x0) + b * n;
        a.v0 = static_cast<const T *>(v0) + b * n;
        a.state = static_cast<T *>(s->plain_state) + 4 * b * n;
        a.xe = xe ? static_cast<T *>(xe) + b * n : nullptr;
        a.ve = ve ? static_cast<T *>(ve) + b * n : nullptr;
        for (int64_t k = 0; k < nsteps || k == 0; ++k) {
            a.n0 = k;
            a.nsteps = nsteps > 0 ? 1 : 0;
            a.load_mode = k == 0 ? LOAD_USER : LOAD_STATE;
            a.store_mode = k + 1 >= nsteps ? STORE_USER : STORE_STATE;
            osc_status r = dense_launch_vec<T>(a, s->method, s->stream);
            if (r) return r;
        }
    }
    return OSC_OK;
}


template <typename T>
osc_status create_dense(osc_sys *s, const osc_desc *d) {
    const hipStream_t st = s->stream;
    const int n = s->s;
    const int64_t nsys = s->shared ? 1 : s->batch;
    s->nsys = nsys;
    const size_t ss = (size_t)n * n;
    const size_t mbytes = nsys * ss * sizeof(double);
    s->m = static_cast<double *>(pool_alloc(mbytes));
    s->k = static_cast<double *>(pool_alloc(mbytes));
    s->A = static_cast<double *>(pool_alloc(mbytes));
    s->h = static_cast<double *>(pool_alloc(nsys * sizeof(double)));
    s->Bh = pool_alloc(nsys * ss * sizeof(T));
    s->Bl = std::is_same<T, float>::value ? pool_alloc(nsys * ss * sizeof(T)) : nullptr;
    s->flag = static_cast<int *>(pool_alloc(64));
    DevBuf Lc, Inv, scratch, theta;
    Lc.p = pool_alloc(mbytes);
    Inv.p = pool_alloc(nsys * dense_form_scratch_elems(n) * sizeof(double));
    scratch.p = pool_alloc(64);
    theta.p = pool_alloc(nsys * sizeof(double));
    if (!s->m || !s->k || !s->A || !s->h || !s->Bh || (std::is_same<T, float>::value && !s->Bl) || !s->flag ||
        !Lc.p || !Inv.p || !scratch.p || !theta.p)
        return fail(OSC_ENOMEM, "device memory / HBM budget exhausted in osc_create");
    osc_status r;
    if ((r = copy_in(s->m, d->M, mbytes, d->param_mem, st))) return r;
    if ((r = copy_in(s->k, d->K, mbytes, d->param_mem, st))) return r;
    if ((r = copy_in(s->h, d->dt, nsys * sizeof(double), d->param_mem, st))) return r;
    OSC_HIP(hipMemsetAsync(s->flag, 0, 64, st));
    OSC_HIP(hipMemsetAsync(scratch.p, 0, 64, st));
    OSC_HIP(hipMemsetAsync(theta.p, 0, nsys * sizeof(double), st));
    int *notspd = static_cast<int *>(scratch.p);
    int *bad = notspd + 1;
    if ((r = dense_form_a(n, nsys, s->m, s->k, static_cast<double *>(Lc.p), static_cast<double *>(Inv.p), s->A,
                          notspd, st)))
        return r;
    if ((r = dense_prepare<T>(n, nsys, s->A, s->h, static_cast<T *>(s->Bh), static_cast<T *>(s->Bl),
                              static_cast<double *>(theta.p), bad, st)))
        return r;
    int flags[2] = {0, 0};
    OSC_HIP(hipMemcpyAsync(flags, scratch.p, sizeof(flags), hipMemcpyDeviceToHost, st));
    std::vector<double> th(nsys), hh(nsys);
    OSC_HIP(hipMemcpyAsync(th.data(), theta.p, nsys * sizeof(double), hipMemcpyDeviceToHost, st));
    OSC_HIP(hipMemcpyAsync(hh.data(), s->h, nsys * sizeof(double), hipMemcpyDeviceToHost, st));
    OSC_HIP(hipStreamSynchronize(st));
    if (flags[0]) return fail(OSC_ENOTSPD, "Cholesky factorisation of M failed (M is not positive definite)");
    if (flags[1]) return fail(OSC_EINVAL, "dense parameters need finite M, K and finite dt > 0");
    const double lim = s->method == OSC_RK4 ? kRk4Limit : kVerletLimit;
    double worst = 0.0;
    for (int64_t i = 0; i < nsys; ++i) {
        double t = th[i];   // sqrt of the largest row sum of |h^2 A|: an upper bound of h omega_max
        if (!(t <= lim)) {
            // the norm bound is loose: refine with power iteration, 2 % margin on omega
            if ((r = dense_power_theta(n, s->A + i * ss, hh[i], static_cast<double *>(theta.p) + i, st))) return r;
            OSC_HIP(hipMemcpyAsync(&t, static_cast<double *>(theta.p) + i, sizeof(double), hipMemcpyDeviceToHost,
                                   st));
            OSC_HIP(hipStreamSynchronize(st));
            t *= 1.02;
        }
        worst = t > worst ? t : worst;
        if (!(t <= lim))
            return fail(OSC_EUNSTABLE,
                        "dt * omega estimate " + std::to_string(t) + " exceeds " + std::to_string(lim));
    }
    s->theta_max = worst;
    s->h_shared = hh[0];
    s->h_host = new (std::nothrow) double[nsys];
    if (!s->h_host) return fail(OSC_ENOMEM, "host allocation failed");
    for (int64_t i = 0; i < nsys; ++i) s->h_host[i] = hh[i];
    if (std::is_same<T, float>::value && dense_mfma_pad(n) > 0) {
        // FP16 operator fragments of B^ = beta h^2 A with ||B^||_inf in [1/2, 1), per system
        const size_t fe = dense_mfma_fragment_elems(n);
        s->F1 = pool_alloc(nsys * fe * sizeof(_Float16));
        s->F2 = pool_alloc(nsys * fe * sizeof(_Float16));
        s->inv_betas = new (std::nothrow) float[nsys];
        if (!s->F1 || !s->F2 || !s->inv_betas)
            return fail(OSC_ENOMEM, "memory exhausted for MFMA operator fragments");
        for (int64_t i = 0; i < nsys; ++i) {
            const double rowsum = th[i] * th[i];
            int e = 0;
            (void)std::frexp(rowsum > 0.0 ? rowsum : 1.0, &e);
            const double beta = std::ldexp(1.0, -e);
            s->inv_betas[i] = (float)std::ldexp(1.0, e);
            if ((r = dense_mfma_fragments(n, s->A + i * ss, beta * hh[i] * hh[i],
                                          static_cast<_Float16 *>(s->F1) + i * fe,
                                          static_cast<_Float16 *>(s->F2) + i * fe, st)))
                return r;
        }
        s->inv_beta = s->inv_betas[0];
        OSC_HIP(hipStreamSynchronize(st));
    }
    return OSC_OK;
}

bool use_mfma(const osc_sys *s) {
    const bool can = s->prec == OSC_F32 && s->F1 != nullptr;
    return (s->dense_kernel == 0 || s->dense_kernel == 2) ? can : false;
}

// Split path by default for few instances of large s: one workgroup per
// instance would leave most of the GPU idle.
bool use_split(const osc_sys *s) {
    if (s->dense_kernel == 3) return true;
    if (s->dense_kernel != 0) return false;
    return s->s > 256 && s->batch * ((s->s + 63) / 64) <= 1024;
}

template <typename T>
osc_status integrate_split(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                           void *xf, void *vf, void *xe, void *ve) {
    osc_status r = ensure_state(s);
    if (r) return r;
    if ((r = sys_ensure_split_scratch(s))) return r;
    DenseSplitLaunch<T> a{};
    split_launch_base(s, a);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    if (!s->static_call) {
        // the graph replays phase kernels only: key on what they read
        static_assert(sizeof(DenseSplitLaunch<T>) <= sizeof(s->split_key), "graph key too small");
        unsigned char key[sizeof(s->split_key)] = {};
        std::memcpy(key, &a, sizeof(a));
        if (std::memcmp(key, s->split_key, sizeof(key)) != 0 && s->split_graph) {
            (void)hipGraphExecDestroy(s->split_graph);
            s->split_graph = nullptr;
        }
        std::memcpy(s->split_key, key, sizeof(key));
    }
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.n0 = 0;
    a.nsteps = nsteps;
    a.load_mode = LOAD_USER;
    a.store_mode = STORE_USER;
    // no capture on the null stream, nor in an allocation-free call (whose
    // launches a caller may itself be capturing)
    const int64_t gsteps = (s->stream && !s->static_call) ? s->graph_steps : 0;
    if (s->static_call) return dense_split_run<T>(a, s->method, s->stream, nullptr, nullptr, 0);
    return dense_split_run<T>(a, s->method, s->stream, &s->split_graph, &s->split_graph_len, gsteps);
}

// Per-instance operators on the matrix cores: one work-list item (one
// workgroup) per instance, each with its own fragments and scale; chunked
// state is kept per instance ([batch][4][s] plus one scale each).
osc_status integrate_mfma_items(osc_sys *s, const DenseMfmaLaunch &base, int64_t nsteps) {
    const int64_t B = s->batch, n = s->s;
    const size_t fe = dense_mfma_fragment_elems((int)n);
    const int64_t chunk = s->steps_per_launch > 0 ? s->steps_per_launch : (nsteps > 0 ? nsteps : 1);
    const bool chunked = nsteps > chunk;
    osc_status r;
    if (chunked && (r = ensure_state(s))) return r;
    const size_t bytes = B * sizeof(DenseMfmaItem);
    if (s->mfma_items_bytes < bytes) {
        pool_free(s->mfma_items);
        s->mfma_items = pool_alloc(bytes);
        s->mfma_items_bytes = s->mfma_items ? bytes : 0;
        if (!s->mfma_items) return fail(OSC_ENOMEM, "device memory exhausted for the MFMA work list");
    }
    std::vector<DenseMfmaItem> items(B);
    float *st = static_cast<float *>(s->state);
    for (int64_t n0 = 0; n0 < nsteps || n0 == 0; n0 += chunk) {
        const int64_t cnt = std::min(chunk, nsteps - n0);
        for (int64_t b = 0; b < B; ++b) {
            DenseMfmaLaunch a = base;
            a.batch = 1;
            a.B1 = static_cast<const _Float16 *>(s->F1) + b * fe;
            a.B2 = static_cast<const _Float16 *>(s->F2) + b * fe;
            a.inv_beta = s->inv_betas[b];
            a.h = s->h_host[b];
            a.x0 = base.x0 + b * n;
            a.v0 = base.v0 + b * n;
            a.xf = base.xf ? base.xf + b * n : nullptr;
            a.vf = base.vf ? base.vf + b * n : nullptr;
            a.xe = base.xe ? base.xe + b * n : nullptr;
            a.ve = base.ve ? base.ve + b * n : nullptr;
            a.n0 = n0;
            a.nsteps = cnt;
            a.load_mode = n0 == 0 ? LOAD_USER : LOAD_STATE;
            a.store_mode = n0 + cnt == nsteps ? STORE_USER : STORE_STATE;
            a.state = chunked ? st + b * 4 * n : nullptr;
            a.sigma = chunked ? st + 4 * B * n + b : nullptr;
            items[b].L = a;
        }
        OSC_HIP(hipMemcpyAsync(s->mfma_items, items.data(), bytes, hipMemcpyHostToDevice, s->stream));
        if ((r = dense_mfma_launch_items(static_cast<const DenseMfmaItem *>(s->mfma_items), B,
                                         dense_mfma_pad((int)n), s->method, s->stream)))
            return r;
        // the host vector is reused for the next chunk: the copy must have been consumed
        if (n0 + chunk < nsteps) OSC_HIP(hipStreamSynchronize(s->stream));
        if (nsteps == 0) break;
    }
    return OSC_OK;
}

template <typename T>
osc_status integrate_dense(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                           void *xf, void *vf, void *xe, void *ve) {
    if (!use_mfma(s) && use_split(s)) return integrate_split<T>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    if constexpr (std::is_same<T, float>::value) {
        if (use_mfma(s)) {
            DenseMfmaLaunch a{};
            a.batch = s->batch;
            a.s = s->s;
            a.B1 = s->F1;
            a.B2 = s->F2;
            a.inv_beta = s->inv_beta;
            a.h = s->h_shared;
            a.x0 = static_cast<const float *>(x0);
            a.v0 = static_cast<const float *>(v0);
            a.out_stride = out_stride;
            a.frame_plane = s->batch * (int64_t)s->s;
            a.xf = static_cast<float *>(xf);
            a.vf = static_cast<float *>(vf);
            a.xe = static_cast<float *>(xe);
            a.ve = static_cast<float *>(ve);
            a.nonfinite = s->flag;
            if (s->shared)
                return run_chunks(s, a, nsteps,
                                  [&](const DenseMfmaLaunch &c) { return dense_mfma_launch(c, s->method, s->stream); });
            return integrate_mfma_items(s, a, nsteps);
        }
    }
    DenseLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.shared = s->shared ? 1 : 0;
    a.Bh = static_cast<const T *>(s->Bh);
    a.Bl = static_cast<const T *>(s->Bl);
    a.h = s->h;
    a.nonfinite = s->flag;
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    return run_chunks(s, a, nsteps,
                      [&](const DenseLaunch<T> &c) { return dense_launch_vec<T>(c, s->method, s->stream); });
}

PropArgs prop_args(const osc_sys *s) {
    PropArgs a{};
    a.kind = s->kind;
    a.method = s->method;
    a.nsys = s->kind == OSC_CHAIN ? s->batch : s->nsys;
    a.m = s->kind == OSC_CHAIN ? s->m : nullptr;
    a.k = s->kind == OSC_CHAIN ? s->k : nullptr;
    a.A = s->kind == OSC_DENSE ? s->A : nullptr;
    a.h = s->h;
    return a;
}

// Frames by powers of the one-step matrix (OSC_CFG_PROPAGATOR = 1).
template <typename T>
osc_status integrate_jump(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride, void *xf,
                          void *vf, void *xe, void *ve) {
    PropRun<T> run{};
    run.batch = s->batch;
    run.nsteps = nsteps;
    run.out_stride = out_stride;
    run.x0 = static_cast<const T *>(x0);
    run.v0 = static_cast<const T *>(v0);
    run.xf = static_cast<T *>(xf);
    run.vf = static_cast<T *>(vf);
    run.xe = static_cast<T *>(xe);
    run.ve = static_cast<T *>(ve);
    run.nonfinite = s->flag;
    return propagator_jump<T>(prop_args(s), s->s, run, s->stream);
}

// One application of the one-step matrix per step (OSC_CFG_PROPAGATOR = 2).
template <typename T>
osc_status integrate_prop_step(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                               void *xf, void *vf, void *xe, void *ve) {
    ChainLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.c = coef_of<T>(s);
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.nonfinite = s->flag;
    return run_chunks(s, a, nsteps,
                      [&](const ChainLaunch<T> &c) { return prop_step_launch<T>(c, s->method, s->stream); });
}

// Damped and driven systems (osc_set_excitation): stage-form RK4, one
// workgroup per instance.
template <typename T>
osc_status integrate_driven(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                            void *xf, void *vf, void *xe, void *ve) {
    if (s->propagator)
        return fail(OSC_ENOTSUP, "the propagator modes take free (undamped, undriven) systems");
    if constexpr (std::is_same<T, float>::value) {
        // one operator shared by many instances: the matrix-core integrator
        if (s->kind == OSC_DENSE && s->shared && use_mfma(s)) {
            DenseMfmaLaunch a{};
            a.batch = s->batch;
            a.s = s->s;
            a.B1 = s->F1;
            a.B2 = s->F2;
            a.inv_beta = s->inv_beta;
            a.h = s->h_shared;
            a.alpha = s->alpha;
            a.beta = s->beta;
            a.f = s->force;
            a.omega = s->omega;
            a.x0 = static_cast<const float *>(x0);
            a.v0 = static_cast<const float *>(v0);
            a.out_stride = out_stride;
            a.frame_plane = s->batch * (int64_t)s->s;
            a.xf = static_cast<float *>(xf);
            a.vf = static_cast<float *>(vf);
            a.xe = static_cast<float *>(xe);
            a.ve = static_cast<float *>(ve);
            a.nonfinite = s->flag;
            const int method = kMfmaDriven + (s->beta != 0.0 ? 1 : 0) + (s->force ? 2 : 0);
            return run_chunks(s, a, nsteps,
                              [&](const DenseMfmaLaunch &c) { return dense_mfma_launch(c, method, s->stream); });
        }
    }
    DrivenLaunch<T> a{};
    a.kind = s->kind;
    a.batch = s->batch;
    a.s = s->s;
    a.shared = s->kind == OSC_DENSE ? s->shared : 0;
    if (s->kind == OSC_CHAIN) a.c = coef_of<T>(s);
    a.Bh = static_cast<const T *>(s->Bh);
    a.Bl = static_cast<const T *>(s->Bl);
    a.h = s->h;
    a.alpha = s->alpha;
    a.beta = s->beta;
    a.f = s->force;
    a.omega = s->omega;
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.nonfinite = s->flag;
    a.force_workgroup = s->dense_kernel == 1 ? 1 : 0;
    return run_chunks(s, a, nsteps, [&](const DrivenLaunch<T> &c) { return driven_launch<T>(c, s->stream); });
}

// Van der Pol chains (osc_set_van_der_pol): stage-form RK4 in registers.
template <typename T>
osc_status integrate_vdp(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride, void *xf,
                         void *vf, void *xe, void *ve) {
    VdpLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.c = coef_of<T>(s);
    a.m = s->m;
    a.mu = s->vdp_mu;
    a.f = s->force;
    a.omega = s->omega;
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.out_stride = out_stride;
    a.xf = static_cast<T *>(xf);
    a.vf = static_cast<T *>(vf);
    a.xe = static_cast<T *>(xe);
    a.ve = static_cast<T *>(ve);
    a.nonfinite = s->flag;
    return run_chunks(s, a, nsteps, [&](const VdpLaunch<T> &c) { return vdp_launch<T>(c, s->stream); });
}

}  // namespace

template <typename T>
ChainCoef<T> chain_coef(const osc_sys *s) {
    return coef_of<T>(s);
}
template ChainCoef<float> chain_coef<float>(const osc_sys *);
template ChainCoef<double> chain_coef<double>(const osc_sys *);

bool dense_uses_split(const osc_sys *s) { return use_split(s); }

osc_status sys_ensure_state(osc_sys *s) { return ensure_state(s); }

osc_status sys_ensure_split_scratch(osc_sys *s) {
    if (s->static_call)
        return s->scratch_split ? OSC_OK : fail(OSC_EINVAL, "internal: no static scratch for the split path");
    const size_t e = s->prec == OSC_F64 ? 8 : 4;
    if (!s->split_scratch) {
        s->split_scratch = pool_alloc(dense_split_scratch_elems(s->s, s->batch) * e + 64);
        if (!s->split_scratch) return fail(OSC_ENOMEM, "device memory exhausted for the split dense path");
    }
    return OSC_OK;
}

template <typename T>
void split_launch_base(osc_sys *s, DenseSplitLaunch<T> &a) {
    const size_t n = (size_t)s->batch * s->s;
    a.batch = s->batch;
    a.s = s->s;
    a.shared = s->shared ? 1 : 0;
    a.groups = dense_split_groups(s->s, s->batch);
    a.Bh = static_cast<const T *>(s->Bh);
    a.Bl = static_cast<const T *>(s->Bl);
    a.h = s->h;
    a.state = static_cast<T *>(state_buf(s));
    a.P = static_cast<T *>(split_buf(s));
    a.part = a.P + n;
    a.counter = reinterpret_cast<int64_t *>(a.part + 4 * (size_t)a.groups * n);
    a.nonfinite = s->flag;
}
template void split_launch_base<float>(osc_sys *, DenseSplitLaunch<float> &);
template void split_launch_base<double>(osc_sys *, DenseSplitLaunch<double> &);

void set_error(const std::string &msg) { g_last_error = msg; }

osc_status fail(osc_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

}  // namespace osc

using namespace osc;

extern "C" {

int osc_abi_version(void) { return OSC_ABI_VERSION; }

const char *osc_last_error(void) { return g_last_error.c_str(); }

osc_status osc_create(const osc_desc *d, void *stream, osc_sys **out) {
    g_last_error.clear();
    if (!out) return fail(OSC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(OSC_EINVAL, "desc is NULL");
    if (d->kind != OSC_CHAIN && d->kind != OSC_DENSE) return fail(OSC_EINVAL, "unknown kind");
    if (d->method != OSC_RK4 && d->method != OSC_VERLET) return fail(OSC_EINVAL, "unknown method");
    if (d->prec != OSC_F64 && d->prec != OSC_F32) return fail(OSC_EINVAL, "unknown precision");
    if (d->param_mem != OSC_MEM_HOST && d->param_mem != OSC_MEM_DEVICE)
        return fail(OSC_EINVAL, "unknown param_mem");
    if (d->s < 1) return fail(OSC_EINVAL, "s must be >= 1");
    if (d->batch < 0) return fail(OSC_EINVAL, "batch must be >= 0");
    if (!d->M || !d->K || !d->dt) return fail(OSC_EINVAL, "M, K and dt must be non-NULL");
    if ((double)d->batch * d->s > 4.0e9) return fail(OSC_EINVAL, "batch * s too large");
    if (d->s > 2048) return fail(OSC_ENOTSUP, "this build supports s <= 2048");
    if (d->kind == OSC_DENSE && !d->shared && (double)d->batch * d->s * d->s > 2.0e9)
        return fail(OSC_EINVAL, "batch * s * s too large for per-instance dense systems");

    osc_sys *s = new (std::nothrow) osc_sys();
    if (!s) return fail(OSC_ENOMEM, "host allocation failed");
    s->kind = d->kind;
    s->method = d->method;
    s->prec = d->prec;
    s->s = d->s;
    s->batch = d->batch;
    s->shared = d->kind == OSC_DENSE ? (d->shared ? 1 : 0) : 0;
    s->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(OSC_EDEVICE, "no HIP device");
    }
    osc_status r;
    if (d->kind == OSC_CHAIN) r = d->prec == OSC_F32 ? create_chain<float>(s, d) : create_chain<double>(s, d);
    else r = d->prec == OSC_F32 ? create_dense<float>(s, d) : create_dense<double>(s, d);
    if (r != OSC_OK) {
        (void)hipStreamSynchronize(s->stream);
        release(s);
        return r;
    }
    autotune_apply_cached(s);
    *out = s;
    return OSC_OK;
}

osc_status osc_set_config(osc_sys *s, osc_config key, int64_t value) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    switch (key) {
        case OSC_CFG_CHAIN_LAYOUT: {
            if (s->kind != OSC_CHAIN) return fail(OSC_EINVAL, "layout applies to chains");
            if (value == 0) {
                s->cfg = chain_pick_config(s->s);
                return OSC_OK;
            }
            const ChainConfig c{(int)(value >> 16), (int)(value & 0xffff)};
            for (int i = 0; i < chain_num_configs(); ++i) {
                const ChainConfig k = chain_config_at(i);
                if (k.lpi == c.lpi && k.dpl == c.dpl) {
                    if ((long)c.lpi * c.dpl < s->s) return fail(OSC_ENOTSUP, "layout holds fewer than s DOFs");
                    s->cfg = c;
                    return OSC_OK;
                }
            }
            return fail(OSC_ENOTSUP, "no kernel built for this layout");
        }
        case OSC_CFG_DENSE_KERNEL:
            if (s->kind == OSC_CHAIN && (value == 0 || value == 1)) {
                // damped / driven chains: 1 = the one-workgroup-per-instance kernel
                s->dense_kernel = (int)value;
                return OSC_OK;
            }
            if (s->kind != OSC_DENSE) return fail(OSC_EINVAL, "kernel choice applies to dense systems");
            if (value < 0 || value > 3) return fail(OSC_EINVAL, "dense kernel must be 0, 1, 2 or 3");
            if (value == 2 && !(s->prec == OSC_F32 && s->F1))
                return fail(OSC_ENOTSUP, "MFMA path needs FP32, a shared operator and s <= 256");
            s->dense_kernel = (int)value;
            return OSC_OK;
        case OSC_CFG_STEPS_PER_LAUNCH:
            if (value < 0) return fail(OSC_EINVAL, "steps per launch must be >= 0");
            s->steps_per_launch = value;
            return OSC_OK;
        case OSC_CFG_GRAPH_STEPS:
            if (value < 0 || value > 4096) return fail(OSC_EINVAL, "graph steps must be in [0, 4096]");
            s->graph_steps = value;
            return OSC_OK;
        case OSC_CFG_PROPAGATOR:
            if (value < 0 || value > 2) return fail(OSC_EINVAL, "propagator mode must be 0, 1 or 2");
            if (value != 0 && s->vdp_mu > 0.0)
                return fail(OSC_ENOTSUP, "the propagator modes take linear systems, not Van der Pol chains");
            if (value == 2 && !(s->kind == OSC_CHAIN && s->s <= 2))
                return fail(OSC_ENOTSUP, "the per-step propagator takes chains of s <= 2");
            s->propagator = (int)value;
            return OSC_OK;
    }
    return fail(OSC_EINVAL, "unknown configuration key");
}

static osc_status integrate_checks(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                                   const void *xf, const void *vf) {
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(OSC_EINVAL, "nsteps must be >= 0");
    if (out_stride < 0) return fail(OSC_EINVAL, "out_stride must be >= 0");
    if (out_stride == 0 && (xf || vf)) return fail(OSC_EINVAL, "frames requested with out_stride == 0");
    if (s->batch > 0 && (!x0 || !v0)) return fail(OSC_EINVAL, "x0 and v0 must be non-NULL");
    return OSC_OK;
}

static osc_status integrate_any(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                                void *xf, void *vf, void *xe, void *ve) {
    if (s->vdp_mu > 0.0)
        return s->prec == OSC_F32 ? integrate_vdp<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                                  : integrate_vdp<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    if (s->driven)
        return s->prec == OSC_F32 ? integrate_driven<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                                  : integrate_driven<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    if (s->propagator == 1)
        return s->prec == OSC_F32 ? integrate_jump<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                                  : integrate_jump<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    if (s->propagator == 2)
        return s->prec == OSC_F32 ? integrate_prop_step<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                                  : integrate_prop_step<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    if (s->kind == OSC_DENSE)
        return s->prec == OSC_F32 ? integrate_dense<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                                  : integrate_dense<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    return s->prec == OSC_F32 ? integrate_chain<float>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve)
                              : integrate_chain<double>(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
}

osc_status osc_integrate(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride, void *xf,
                         void *vf, void *xe, void *ve) {
    g_last_error.clear();
    osc_status r = integrate_checks(s, x0, v0, nsteps, out_stride, xf, vf);
    if (r || s->batch == 0) return r;
    return integrate_any(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
}

osc_status osc_integrate_static(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, int64_t out_stride,
                                void *xf, void *vf, void *xe, void *ve) {
    g_last_error.clear();
    osc_status r = integrate_checks(s, x0, v0, nsteps, out_stride, xf, vf);
    if (r || s->batch == 0) return r;
    // device memory the run needs beyond its inputs and outputs
    size_t need_state = 0, need_split = 0;
    if (s->propagator == 1 && !propagator_small(s->s) && !s->driven)
        return fail(OSC_ENOTSUP, "osc_integrate_static: frame jumps of systems with s > 2 form their matrix powers "
                                 "in per-call buffers; use osc_integrate");
    if (s->propagator == 0 && s->kind == OSC_DENSE && use_mfma(s) && !s->shared && !s->driven)
        return fail(OSC_ENOTSUP, "osc_integrate_static: per-instance operators on the matrix cores take a work "
                                 "list built per call; use osc_integrate");
    if (s->driven) {
        if (s->steps_per_launch > 0 && nsteps > s->steps_per_launch) need_state = state_bytes(s);
    } else if (s->propagator == 1) {
        // one kernel per call, no scratch
    } else if (s->propagator == 0 && s->kind == OSC_DENSE && !use_mfma(s) && use_split(s)) {
        need_state = state_bytes(s);
        need_split = dense_split_scratch_elems(s->s, s->batch) * elem(s) + 64;
    } else if (s->steps_per_launch > 0 && nsteps > s->steps_per_launch) {
        need_state = state_bytes(s);
    }
    const size_t off = (need_state + 255) / 256 * 256;
    const size_t need = off + need_split;
    if (need > OSC_STATIC_SCRATCH_BYTES)
        return fail(OSC_ENOMEM, "osc_integrate_static: the run needs " + std::to_string(need) +
                                    " bytes of device scratch; the maximum is " +
                                    std::to_string((size_t)OSC_STATIC_SCRATCH_BYTES) +
                                    " (fewer instances per call, or osc_integrate)");
    void *base = nullptr;
    if (need > 0 && (r = static_scratch(s->device, &base))) return r;
    s->static_call = true;
    s->scratch_state = need_state ? base : nullptr;
    s->scratch_split = need_split ? static_cast<char *>(base) + off : nullptr;
    r = integrate_any(s, x0, v0, nsteps, out_stride, xf, vf, xe, ve);
    s->static_call = false;
    s->scratch_state = s->scratch_split = nullptr;
    return r;
}

osc_status osc_integrate_plain(osc_sys *s, const void *x0, const void *v0, int64_t nsteps, void *xe, void *ve) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    if (s->driven || s->vdp_mu > 0.0)
        return fail(OSC_ENOTSUP, "the plain baseline takes free (undamped, undriven, linear) systems");
    if (nsteps < 0) return fail(OSC_EINVAL, "nsteps must be >= 0");
    if (s->batch == 0) return OSC_OK;
    if (!x0 || !v0) return fail(OSC_EINVAL, "x0 and v0 must be non-NULL");
    if (s->kind == OSC_DENSE)
        return s->prec == OSC_F32 ? plain_dense<float>(s, x0, v0, nsteps, xe, ve)
                                  : plain_dense<double>(s, x0, v0, nsteps, xe, ve);
    return s->prec == OSC_F32 ? plain_chain<float>(s, x0, v0, nsteps, xe, ve)
                              : plain_chain<double>(s, x0, v0, nsteps, xe, ve);
}

static osc_status energy_common(osc_sys *s, const void *x, const void *v, double *E, bool shadow) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    if (s->batch == 0) return OSC_OK;
    if (!x || !v || !E) return fail(OSC_EINVAL, "x, v and E must be non-NULL");
    if (s->kind == OSC_DENSE) {
        if (s->prec == OSC_F32)
            return dense_energy<float>(s->batch, s->s, s->shared, s->m, s->k, s->A, s->h,
                                       static_cast<const float *>(x), static_cast<const float *>(v), E, shadow,
                                       s->stream);
        return dense_energy<double>(s->batch, s->s, s->shared, s->m, s->k, s->A, s->h,
                                    static_cast<const double *>(x), static_cast<const double *>(v), E, shadow,
                                    s->stream);
    }
    if (s->prec == OSC_F32)
        return chain_energy<float>(s->batch, s->s, s->m, s->k, s->h, static_cast<const float *>(x),
                                   static_cast<const float *>(v), E, shadow, s->stream);
    return chain_energy<double>(s->batch, s->s, s->m, s->k, s->h, static_cast<const double *>(x),
                                static_cast<const double *>(v), E, shadow, s->stream);
}

osc_status osc_energy(osc_sys *s, const void *x, const void *v, double *E) { return energy_common(s, x, v, E, false); }

osc_status osc_shadow_energy(osc_sys *s, const void *x, const void *v, double *Q) {
    return energy_common(s, x, v, Q, true);
}

osc_status osc_set_excitation(osc_sys *s, double alpha, double beta, const double *F, const double *Omega,
                              osc_mem mem) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    if (!(alpha >= 0.0 && std::isfinite(alpha)) || !(beta >= 0.0 && std::isfinite(beta)))
        return fail(OSC_EINVAL, "alpha and beta must be finite and >= 0");
    if (mem != OSC_MEM_HOST && mem != OSC_MEM_DEVICE) return fail(OSC_EINVAL, "unknown mem");
    if (F && !Omega) return fail(OSC_EINVAL, "a force needs its frequencies Omega");
    const bool on = alpha != 0.0 || beta != 0.0 || F != nullptr;
    if (on && s->method != OSC_RK4)
        return fail(OSC_ENOTSUP, "damped / driven systems are integrated by RK4 only");
    if (s->vdp_mu > 0.0 && (alpha != 0.0 || beta != 0.0))
        return fail(OSC_ENOTSUP, "a Van der Pol chain takes a force but no Rayleigh damping");
    const hipStream_t st = s->stream;
    const int64_t nh = s->kind == OSC_CHAIN ? s->batch : s->nsys;
    if ((alpha != 0.0 || beta != 0.0) && nh > 0) {
        // per mode |lambda| <= max(omega, alpha + beta omega^2); RK4's
        // stability region holds the left half-disk of radius 2.6156
        std::vector<double> hh((size_t)nh);
        OSC_HIP(hipMemcpyAsync(hh.data(), s->h, nh * sizeof(double), hipMemcpyDeviceToHost, st));
        OSC_HIP(hipStreamSynchronize(st));
        const double hmin = *std::min_element(hh.begin(), hh.end()), hmax = *std::max_element(hh.begin(), hh.end());
        const double th = s->theta_max, gh = alpha * hmax + beta * th * th / hmin;
        const double lim = 2.5;
        if (!(std::max(th, gh) <= lim))
            return fail(OSC_EUNSTABLE, "dt * max(omega_max, alpha + beta omega_max^2) = " +
                                           std::to_string(std::max(th, gh)) + " exceeds " + std::to_string(lim));
    }
    pool_free(s->force);
    pool_free(s->omega);
    s->force = s->omega = nullptr;
    s->driven = false;
    if (F && s->batch > 0) {
        const size_t n = (size_t)s->batch * s->s;
        DevBuf Fdev, flag;
        s->force = static_cast<double *>(pool_alloc(n * sizeof(double)));
        s->omega = static_cast<double *>(pool_alloc((size_t)s->batch * sizeof(double)));
        flag.p = pool_alloc(64);
        const double *Fp = F;
        if (mem == OSC_MEM_HOST) {
            Fdev.p = pool_alloc(n * sizeof(double));
            if (Fdev.p) OSC_HIP(hipMemcpyAsync(Fdev.p, F, n * sizeof(double), hipMemcpyHostToDevice, st));
            Fp = static_cast<const double *>(Fdev.p);
        }
        if (!s->force || !s->omega || !flag.p || !Fp) {
            OSC_HIP(hipStreamSynchronize(st));
            return fail(OSC_ENOMEM, "device memory exhausted for the force");
        }
        osc_status r = copy_in(s->omega, Omega, (size_t)s->batch * sizeof(double), mem, st);
        if (r) return r;
        OSC_HIP(hipMemsetAsync(flag.p, 0, 64, st));
        r = s->kind == OSC_CHAIN ? chain_force((int64_t)n, Fp, s->m, s->force, st)
                                 : dense_force(s->s, s->nsys, s->batch, s->m, Fp, s->force,
                                               static_cast<int *>(flag.p), st);
        if (r) return r;
        OSC_HIP(hipStreamSynchronize(st));   // the staged force is released below
    }
    s->alpha = alpha;
    s->beta = beta;
    s->driven = on;
    return OSC_OK;
}

osc_status osc_set_van_der_pol(osc_sys *s, double mu) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(OSC_EINVAL, "mu must be finite and >= 0");
    if (mu > 0.0) {
        if (s->kind != OSC_CHAIN) return fail(OSC_ENOTSUP, "Van der Pol elements are on chains only");
        if (s->method != OSC_RK4) return fail(OSC_ENOTSUP, "Van der Pol chains are integrated by RK4 only");
        if (s->s > 1024) return fail(OSC_ENOTSUP, "Van der Pol chains take s <= 1024");
        if (s->alpha != 0.0 || s->beta != 0.0)
            return fail(OSC_ENOTSUP, "a Van der Pol chain takes a force but no Rayleigh damping");
        if (s->propagator) return fail(OSC_ENOTSUP, "the propagator modes take linear systems, not Van der Pol chains");
    }
    s->vdp_mu = mu;
    return OSC_OK;
}

osc_status osc_propagator(osc_sys *s, int64_t k, double *P) {
    g_last_error.clear();
    if (!s || !P) return fail(OSC_EINVAL, "handle and P must be non-NULL");
    if (k < 0) return fail(OSC_EINVAL, "k must be >= 0");
    if (s->vdp_mu > 0.0) return fail(OSC_ENOTSUP, "a Van der Pol chain has no step matrix (nonlinear)");
    if (s->batch == 0) return OSC_OK;
    return propagator_matrix(prop_args(s), s->s, k, P, s->stream);
}

osc_status osc_dense_operator(osc_sys *s, double *A) {
    g_last_error.clear();
    if (!s || !A) return fail(OSC_EINVAL, "handle and A must be non-NULL");
    if (s->kind != OSC_DENSE) return fail(OSC_EINVAL, "not a dense handle");
    OSC_HIP(hipMemcpyAsync(A, s->A, (size_t)s->nsys * s->s * s->s * sizeof(double), hipMemcpyDeviceToDevice,
                           s->stream));
    return OSC_OK;
}

osc_status osc_sync(osc_sys *s) {
    g_last_error.clear();
    if (!s) return fail(OSC_EINVAL, "handle is NULL");
    OSC_HIP(hipStreamSynchronize(s->stream));
    int flag = 0;
    OSC_HIP(hipMemcpy(&flag, s->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        OSC_HIP(hipMemset(s->flag, 0, sizeof(int)));
        return fail(OSC_ENONFINITE, "a state became non-finite");
    }
    return OSC_OK;
}

void osc_destroy(osc_sys *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    release(s);
}

}  // extern "C"

namespace osc {

osc_status sys_rt_supported(const osc_sys *s) {
    if (s->propagator == 1) return fail(OSC_ENOTSUP, "real-time stepping takes the stepping integrators, not frame jumps");
    if (s->kind == OSC_DENSE && !s->driven) {
        if (use_mfma(s) && !s->shared)
            return fail(OSC_ENOTSUP, "real-time stepping: per-instance operators on the matrix cores are not supported");
        if (!use_mfma(s) && use_split(s))
            return fail(OSC_ENOTSUP, "real-time stepping: the split dense path (large s, few instances) is not supported");
    }
    return OSC_OK;
}

osc_status sys_rt_resident_supported(const osc_sys *s) {
    if (s->kind != OSC_CHAIN) return fail(OSC_ENOTSUP, "resident real-time stepping takes chains only");
    if (s->driven && (s->s > 1024 || s->dense_kernel == 1))
        return fail(OSC_ENOTSUP, "resident real-time stepping of damped or driven chains takes the register "
                                 "kernels (s <= 1024)");
    if (s->propagator != 0) return fail(OSC_ENOTSUP, "resident real-time stepping takes the stepping integrators");
    return OSC_OK;
}

template <typename T>
osc_status rt_resident(osc_sys *s, const void *x0, const void *v0, const ResidentSpec &spec, int64_t *blocks) {
    ResidentRun<T> r{};
    r.ctl = spec.ctl;
    r.first_release = 0;
    r.nticks = spec.nticks;
    r.n_start = spec.n0;
    r.k = spec.k;
    r.idle_ticks = spec.idle_ticks;
    r.xf = static_cast<T *>(spec.xf);
    r.vf = static_cast<T *>(spec.vf);
    r.xo = static_cast<T *>(spec.xo);
    r.vo = static_cast<T *>(spec.vo);
    if (s->vdp_mu > 0.0) {
        VdpLaunch<T> d{};
        d.batch = s->batch;
        d.s = s->s;
        d.c = coef_of<T>(s);
        d.m = s->m;
        d.mu = s->vdp_mu;
        d.f = s->force;
        d.omega = s->omega;
        d.x0 = static_cast<const T *>(x0);
        d.v0 = static_cast<const T *>(v0);
        d.state = static_cast<T *>(state_buf(s));
        d.nonfinite = s->flag;
        *blocks = vdp_resident_blocks<T>(d);
        return vdp_resident_launch<T>(d, r, s->stream);
    }
    if (s->driven) {
        DrivenLaunch<T> d{};
        d.kind = OSC_CHAIN;
        d.batch = s->batch;
        d.s = s->s;
        d.c = coef_of<T>(s);
        d.h = s->h;
        d.alpha = s->alpha;
        d.beta = s->beta;
        d.f = s->force;
        d.omega = s->omega;
        d.x0 = static_cast<const T *>(x0);
        d.v0 = static_cast<const T *>(v0);
        d.state = static_cast<T *>(state_buf(s));
        d.nonfinite = s->flag;
        *blocks = driven_resident_blocks<T>(d);
        return driven_resident_launch<T>(d, r, s->stream);
    }
    ChainLaunch<T> a{};
    a.batch = s->batch;
    a.s = s->s;
    a.c = coef_of<T>(s);
    a.x0 = static_cast<const T *>(x0);
    a.v0 = static_cast<const T *>(v0);
    a.state = static_cast<T *>(state_buf(s));
    a.nonfinite = s->flag;
    *blocks = chain_resident_blocks<T>(a, s->cfg);
    return chain_resident_launch<T>(a, s->method, s->cfg, r, s->stream);
}

osc_status sys_rt_resident(osc_sys *s, const void *x0, const void *v0, const ResidentSpec &spec, int64_t *blocks) {
    osc_status r = sys_rt_resident_supported(s);
    if (r) return r;
    if ((r = ensure_state(s))) return r;
    return s->prec == OSC_F32 ? rt_resident<float>(s, x0, v0, spec, blocks)
                              : rt_resident<double>(s, x0, v0, spec, blocks);
}

osc_status sys_rt_tick(osc_sys *s, const void *x0, const void *v0, int64_t n0, int64_t k, void *xe, void *ve) {
    osc_status r = sys_rt_supported(s);
    if (r) return r;
    s->rt_chunk = true;
    s->rt_n0 = n0;
    s->rt_load = n0 == 0 ? LOAD_USER : LOAD_STATE;
    r = integrate_any(s, x0, v0, k, 0, nullptr, nullptr, xe, ve);
    s->rt_chunk = false;
    return r;
}

}  // namespace osc
