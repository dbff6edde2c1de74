// Continuous-batching server for single-instance integration requests.
//
// A worker thread owns the scheduling.  Each scheduler iteration it
//   1. admits queued requests first come first served while the accounted
//      device bytes stay within the HBM budget and a slot is free; a setup
//      thread then allocates, uploads and forms the operator on a stream of
//      its own, concurrently with the running iterations, and hands the
//      request to the worker when it is ready;
//   2. advances every admitted request by one chunk of time steps: chains and
//      small dense systems go into work-list launches, one per kernel shape,
//      spread over four streams; large dense systems run their split path
//      (captured step graphs) on a stream of their own;
//   3. retires finished requests: results are copied to host memory, device
//      memory and the slot are released, and waiters are woken.
// Every kernel computes an instance independently of its neighbours in a
// launch, and a run split into chunks gives bitwise the result of one launch
// (the compensated state and every schedule of the integrators are tied to
// global step indices), so results do not depend on what else is in flight
// nor on where the chunks end.  Chunk lengths aim at a fixed GPU time per
// iteration; seconds per step come from a per-shape estimate that each
// iteration updates from events around its launches (a fixed formula until a
// shape has been seen).
// With frame jumps enabled, a dense request whose frames cost much less to
// reach by powers of its one-step matrix (the scheme's own trajectory at the
// frames, formed and applied in FP64) than by stepping is served whole by
// the setup thread and never joins an iteration.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "osc_internal.h"

namespace osc {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum class RState { QUEUED, ACTIVE, DONE, FAILED };

struct Req {
    uint64_t ticket = 0;
    osc_desc desc{};
    std::vector<double> M, K, dt;
    std::vector<unsigned char> x0, v0;
    int64_t nsteps = 0, out_stride = 0, nframes = 0;
    size_t elem = 4;
    int64_t bytes = 0;
    RState st = RState::QUEUED;
    osc_status status = OSC_OK;
    std::string error;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t iterations = 0;
    // device side (worker thread only)
    osc_sys *sys = nullptr;
    void *dx0 = nullptr, *dv0 = nullptr, *dxf = nullptr, *dvf = nullptr, *dxe = nullptr, *dve = nullptr;
    bool split = false, mfma = false;
    bool jump = false;           // served whole by frame jumps at admission
    int64_t done = 0, chunk = 0;
    // results
    std::vector<unsigned char> hxf, hvf, hxe, hve;
};

constexpr int kStreams = 4;

// Conservative device bytes of a request: every allocation rounded to the
// pool's size classes.
int64_t estimate_bytes(const osc_desc &d, int64_t nframes, bool jump) {
    const size_t e = d.prec == OSC_F64 ? 8 : 4;
    const size_t s = (size_t)d.s;
    size_t b = 0;
    auto add = [&](size_t n) { b += pool_size_class(n); };
    add(s * e); add(s * e); add(s * e); add(s * e);              // x0, v0, x_end, v_end
    if (nframes > 0) { add(nframes * s * e); add(nframes * s * e); }
    add(4 * s * e + 4);                                          // chunked-run state
    add(64);                                                     // non-finite flag
    if (d.kind == OSC_CHAIN) {
        add(s * 8); add(s * 8); add(8);                          // m, k, h
        add((d.prec == OSC_F32 ? 4 : 2) * s * e);                // coefficients
        add(64);                                                 // create scratch
    } else {
        const size_t ss = s * s;
        add(ss * 8); add(ss * 8); add(ss * 8); add(8);           // M, K, A, h
        add(ss * e); if (d.prec == OSC_F32) add(ss * e);         // B hi / lo
        add(ss * 8); add(ss * 8); add(64); add(8);               // create temporaries
        if (d.prec == OSC_F32 && s <= 256) {                     // MFMA fragments
            const size_t fe = dense_mfma_fragment_elems((int)s) * 2;
            add(fe); add(fe);
        }
        add(dense_split_scratch_elems((int)s, 1) * e + 64);      // split scratch
        if (jump) {                                              // frame jumps: A^2, six 2s x 2s
            add(ss * 8);                                         // matrices, two states (FP64)
            for (int i = 0; i < 6; ++i) add(4 * ss * 8);
            add(2 * s * 8); add(2 * s * 8);
        }
    }
    return (int64_t)b;
}

// Whether a dense request's frames cost much less by frame jumps than by
// stepping.  Jumps: FP64 products of 2s x 2s matrices (A^2, squarings and
// multiplications for P^out_stride and the remainder power) at about 35
// TFLOP/s, 20 us per frame, 1 ms of set-up.  Stepping: seconds per step of
// the path the request would take (one instance: the split path beyond
// s = 256, matrix cores for FP32 up to 256, else the vector kernel), as
// measured for a lone instance.  Jumps are taken below half the stepping time.
bool jumps_pay(const osc_desc &d, int64_t nsteps, int64_t out_stride) {
    if (d.kind != OSC_DENSE || nsteps <= 0) return false;
    const double s = d.s;
    const int64_t nf = out_stride > 0 ? nsteps / out_stride + 1 : 0;
    const int64_t k = std::max<int64_t>(1, out_stride > 0 ? out_stride : nsteps);
    int bits = 0;
    while ((k >> bits) > 0) ++bits;
    const double gemm_s = 2.0 * (2 * s) * (2 * s) * (2 * s) / 35e12;
    const double jump_s = (1 + 2 * bits + 2) * gemm_s + 20e-6 * (double)nf + 1e-3;
    double step_s;
    if (s > 256) step_s = 1.0e-5 + 1.8e-12 * s * s;
    else if (d.prec == OSC_F32) step_s = 1e-6 + 8e-11 * s * s;
    else step_s = 2e-6 + 1.2e-9 * s * s;
    return jump_s < 0.5 * step_s * (double)nsteps;
}

// First guess of the seconds per step of one instance, before its shape's
// launches have been timed; used only to size chunks.
double step_seconds_guess(const Req &r) {
    const double s = r.desc.s;
    if (r.desc.kind == OSC_CHAIN) return 2e-7 + 4e-9 * s;
    if (r.split) return 2.0e-5 + 8e-12 * s * s;
    if (r.mfma) return 1e-6 + 2e-11 * s * s;
    return 2e-6 + 1.2e-9 * s * s;
}

// The launch shape a request's chunks run in: path, method, precision and
// the size class that selects the kernel.
uint64_t shape_key(const Req &r) {
    uint64_t path, cls;
    const osc_sys *sy = r.sys;
    if (r.desc.kind == OSC_CHAIN) {
        path = 0;
        cls = sy ? (((uint64_t)sy->cfg.lpi << 16) | (uint64_t)sy->cfg.dpl) : (uint64_t)r.desc.s;
    } else if (r.split) {
        path = 3;
        cls = (uint64_t)((r.desc.s + 63) / 64);
    } else if (r.mfma) {
        path = 1;
        cls = (uint64_t)dense_mfma_pad(r.desc.s);
    } else {
        path = 2;
        cls = (uint64_t)dense_vec_bucket(r.desc.s);
    }
    return (path << 56) | ((uint64_t)r.desc.method << 48) | ((uint64_t)r.desc.prec << 40) | cls;
}

struct Server {
    osc_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::condition_variable cv_setup;
    std::deque<Req *> queue;
    std::deque<Req *> preparing;   // admitted, waiting for or in setup
    std::vector<Req *> active;     // ready: part of every iteration
    std::map<uint64_t, Req *> all;
    std::atomic<uint64_t> next_ticket{1};
    bool stopping = false;
    size_t in_use = 0, peak = 0;
    int64_t submitted = 0, completed = 0, failed = 0, iterations = 0;
    double setup_s = 0.0, iterate_s = 0.0;
    std::thread worker, setup_worker;
    hipStream_t streams[kStreams] = {};
    hipStream_t setup_stream = nullptr;
    int64_t in_setup = 0;
    void *stage = nullptr;       // pinned host staging of work lists
    size_t stage_bytes = 0;
    void *items = nullptr;       // device copy of work lists
    size_t items_bytes = 0;

    // One iteration's work lists of both precisions: every list is appended
    // to one host image at its own 256-byte aligned offset, the image goes to
    // the device in one copy, and each launch reads its list at that offset
    // once the copy has completed.
    // seconds per step of each launch shape (exponential average of timed launches)
    std::map<uint64_t, double> step_est;
    std::vector<hipEvent_t> event_pool;   // reused timing events
    size_t events_used = 0;
    struct Timed {
        hipEvent_t a, b;
        uint64_t key;
        int64_t steps;   // the longest chunk in the launch
    };
    std::vector<Timed> timed;
    hipEvent_t event();                   // next event of the pool (nullptr if none could be made)
    double step_seconds(const Req &r) const {
        auto it = step_est.find(shape_key(r));
        return it != step_est.end() ? it->second : step_seconds_guess(r);
    }
    int64_t chunk_of(const Req &r) const {
        int64_t c = std::max<int64_t>(16, (int64_t)(cfg.chunk_us * 1e-6 / step_seconds(r)));
        if (r.split) c = std::max<int64_t>(64, c / 64 * 64);   // whole captured graphs
        return c;
    }

    struct WorkLists {
        std::vector<unsigned char> image;
        std::vector<std::function<void(const char *dev, hipStream_t st)>> launches;
        std::vector<std::pair<uint64_t, int64_t>> shapes;   // per launch: shape key, longest chunk
        size_t append(const void *src, size_t bytes) {
            const size_t off = image.size();
            image.resize(off + (bytes + 255) / 256 * 256);
            std::memcpy(image.data() + off, src, bytes);
            return off;
        }
    };

    void loop();
    void setup_loop();
    bool setup(Req *r);   // false: the request has been finished (failed, or served by jumps) and may be gone
    bool serve_by_jumps(Req *r);
    void run_iteration(std::vector<Req *> &act);
    void finish(Req *r, osc_status st, const std::string &msg);
    void release_device(Req *r);
    template <typename T>
    void collect_groups(std::vector<Req *> &act, std::vector<int64_t> &cnt, WorkLists &wl, int &next_stream);
    void launch_lists(WorkLists &wl, std::vector<Req *> &act, int &next_stream);
};

void Server::release_device(Req *r) {
    for (void *p : {r->dx0, r->dv0, r->dxf, r->dvf, r->dxe, r->dve}) pool_free(p);
    r->dx0 = r->dv0 = r->dxf = r->dvf = r->dxe = r->dve = nullptr;
    if (r->sys) osc_destroy(r->sys);
    r->sys = nullptr;
}

void Server::finish(Req *r, osc_status st, const std::string &msg) {
    if (!cfg.fake_executor) release_device(r);
    std::lock_guard<std::mutex> lk(mu);
    r->status = st;
    r->error = msg;
    r->t_done = now_s();
    r->st = st == OSC_OK ? RState::DONE : RState::FAILED;
    in_use -= (size_t)r->bytes;
    if (st == OSC_OK) ++completed;
    else ++failed;
    active.erase(std::remove(active.begin(), active.end(), r), active.end());
    cv_done.notify_all();
}

hipEvent_t Server::event() {
    if (events_used < event_pool.size()) return event_pool[events_used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    event_pool.push_back(e);
    ++events_used;
    return e;
}

bool Server::setup(Req *r) {
    const size_t s = (size_t)r->desc.s;
    r->hxe.assign(s * r->elem, 0);
    r->hve.assign(s * r->elem, 0);
    r->hxf.assign(r->nframes * s * r->elem, 0);
    r->hvf.assign(r->nframes * s * r->elem, 0);
    if (cfg.fake_executor) {
        r->chunk = chunk_of(*r);
        return true;
    }
    osc_desc d = r->desc;
    d.M = r->M.data();
    d.K = r->K.data();
    d.dt = r->dt.data();
    d.param_mem = OSC_MEM_HOST;
    osc_status st = osc_create(&d, setup_stream, &r->sys);
    if (st != OSC_OK) {
        finish(r, st, osc_last_error());
        return false;
    }
    r->dx0 = pool_alloc(s * r->elem);
    r->dv0 = pool_alloc(s * r->elem);
    r->dxe = pool_alloc(s * r->elem);
    r->dve = pool_alloc(s * r->elem);
    if (r->nframes > 0) {
        r->dxf = pool_alloc(r->nframes * s * r->elem);
        r->dvf = pool_alloc(r->nframes * s * r->elem);
    }
    r->split = r->desc.kind == OSC_DENSE && dense_uses_split(r->sys);
    r->mfma = r->desc.kind == OSC_DENSE && r->desc.prec == OSC_F32 && r->sys->F1 != nullptr;
    st = r->jump ? OSC_OK : sys_ensure_state(r->sys);
    if (st == OSC_OK && r->split && !r->jump) st = sys_ensure_split_scratch(r->sys);
    if (st != OSC_OK || !r->dx0 || !r->dv0 || !r->dxe || !r->dve || (r->nframes > 0 && (!r->dxf || !r->dvf))) {
        finish(r, OSC_ENOMEM, "device memory exhausted while admitting a request");
        return false;
    }
    if (hipMemcpyAsync(r->dx0, r->x0.data(), s * r->elem, hipMemcpyHostToDevice, setup_stream) != hipSuccess ||
        hipMemcpyAsync(r->dv0, r->v0.data(), s * r->elem, hipMemcpyHostToDevice, setup_stream) != hipSuccess ||
        hipStreamSynchronize(setup_stream) != hipSuccess) {
        finish(r, OSC_EDEVICE, "upload of the initial state failed");
        return false;
    }
    if (r->jump) return serve_by_jumps(r);
    r->chunk = chunk_of(*r);
    // the setup stream is drained; from here on the handle's own stream is
    // one the worker drains every iteration, so the completion path never
    // waits behind another request's setup
    r->sys->stream = streams[0];
    return true;
}

// A request served whole by frame jumps on the setup stream (powers of its
// one-step matrix in FP64, one product per frame) and its results
// downloaded; it is finished here and never joins an iteration.
bool Server::serve_by_jumps(Req *r) {
    const size_t s = (size_t)r->desc.s, bytes = s * r->elem;
    osc_status st = osc_set_config(r->sys, OSC_CFG_PROPAGATOR, 1);
    if (st == OSC_OK)
        st = osc_integrate(r->sys, r->dx0, r->dv0, r->nsteps, r->out_stride, r->dxf, r->dvf, r->dxe, r->dve);
    std::string msg = st == OSC_OK ? std::string() : std::string(osc_last_error());
    if (st == OSC_OK) {
        bool ok = hipMemcpyAsync(r->hxe.data(), r->dxe, bytes, hipMemcpyDeviceToHost, setup_stream) == hipSuccess &&
                  hipMemcpyAsync(r->hve.data(), r->dve, bytes, hipMemcpyDeviceToHost, setup_stream) == hipSuccess;
        if (r->nframes > 0)
            ok = ok &&
                 hipMemcpyAsync(r->hxf.data(), r->dxf, r->nframes * bytes, hipMemcpyDeviceToHost, setup_stream) ==
                     hipSuccess &&
                 hipMemcpyAsync(r->hvf.data(), r->dvf, r->nframes * bytes, hipMemcpyDeviceToHost, setup_stream) ==
                     hipSuccess;
        ok = ok && hipStreamSynchronize(setup_stream) == hipSuccess;
        if (!ok) {
            st = OSC_EDEVICE;
            msg = "download of the results failed";
        } else if ((st = osc_sync(r->sys)) != OSC_OK) {
            msg = osc_last_error();
        }
    }
    finish(r, st, msg);
    return false;
}

// Build the work lists of one precision into wl (split-path requests, which
// take no work list, are launched here directly).
template <typename T>
void Server::collect_groups(std::vector<Req *> &act, std::vector<int64_t> &cnt, WorkLists &wl, int &next_stream) {
    std::map<std::pair<int, int64_t>, std::vector<ChainItem<T>>> chains;   // (method, layout)
    std::map<std::pair<int, int>, std::vector<DenseItem<T>>> denses;       // (method, smax bucket)
    std::map<std::pair<int, int>, int> dense_smax;
    std::map<std::pair<int, int>, std::vector<DenseMfmaItem>> mfmas;       // (method, padded s)
    std::map<std::pair<int, int64_t>, std::pair<uint64_t, int64_t>> chain_shape;   // shape key, longest chunk
    std::map<std::pair<int, int>, std::pair<uint64_t, int64_t>> dense_shape, mfma_shape;
    auto note = [](std::pair<uint64_t, int64_t> &sh, const Req *r, int64_t c) {
        sh.first = shape_key(*r);
        sh.second = std::max(sh.second, c);
    };
    const size_t want_elem = sizeof(T);
    for (size_t i = 0; i < act.size(); ++i) {
        Req *r = act[i];
        if (r->elem != want_elem || !r->sys) continue;
        const int64_t n0 = r->done, c = cnt[i];
        const int load = n0 == 0 ? LOAD_USER : LOAD_STATE;
        const int store = n0 + c == r->nsteps ? STORE_USER : STORE_STATE;
        osc_sys *sy = r->sys;
        if (r->desc.kind == OSC_CHAIN) {
            ChainItem<T> it{};
            it.L.batch = 1;
            it.L.s = sy->s;
            it.L.c = chain_coef<T>(sy);
            it.L.x0 = static_cast<const T *>(r->dx0);
            it.L.v0 = static_cast<const T *>(r->dv0);
            it.L.state = static_cast<T *>(sy->state);
            it.L.nsteps = c;
            it.L.n0 = n0;
            it.L.out_stride = r->out_stride;
            it.L.xf = static_cast<T *>(r->dxf);
            it.L.vf = static_cast<T *>(r->dvf);
            it.L.xe = static_cast<T *>(r->dxe);
            it.L.ve = static_cast<T *>(r->dve);
            it.L.nonfinite = sy->flag;
            it.L.load_mode = load;
            it.L.store_mode = store;
            it.b = 0;
            const int64_t key = ((int64_t)sy->cfg.lpi << 16) | sy->cfg.dpl;
            chains[{(int)sy->method, key}].push_back(it);
            note(chain_shape[{(int)sy->method, key}], r, c);
        } else if (std::is_same<T, float>::value && sy->F1) {
            // matrix cores, one workgroup per request (operator resident in registers)
            DenseMfmaItem it{};
            DenseMfmaLaunch &a = it.L;
            a.batch = 1;
            a.s = sy->s;
            a.B1 = sy->F1;
            a.B2 = sy->F2;
            a.inv_beta = sy->inv_beta;
            a.h = sy->h_shared;
            a.x0 = static_cast<const float *>(r->dx0);
            a.v0 = static_cast<const float *>(r->dv0);
            a.state = static_cast<float *>(sy->state);
            a.sigma = static_cast<float *>(sy->state) + 4 * (size_t)sy->s;
            a.nsteps = c;
            a.n0 = n0;
            a.out_stride = r->out_stride;
            a.frame_plane = sy->s;
            a.xf = static_cast<float *>(r->dxf);
            a.vf = static_cast<float *>(r->dvf);
            a.xe = static_cast<float *>(r->dxe);
            a.ve = static_cast<float *>(r->dve);
            a.nonfinite = sy->flag;
            a.load_mode = load;
            a.store_mode = store;
            mfmas[{(int)sy->method, dense_mfma_pad(sy->s)}].push_back(it);
            note(mfma_shape[{(int)sy->method, dense_mfma_pad(sy->s)}], r, c);
        } else if (!r->split) {
            DenseItem<T> it{};
            it.L.batch = 1;
            it.L.s = sy->s;
            it.L.shared = 1;
            it.L.Bh = static_cast<const T *>(sy->Bh);
            it.L.Bl = static_cast<const T *>(sy->Bl);
            it.L.h = sy->h;
            it.L.x0 = static_cast<const T *>(r->dx0);
            it.L.v0 = static_cast<const T *>(r->dv0);
            it.L.state = static_cast<T *>(sy->state);
            it.L.nsteps = c;
            it.L.n0 = n0;
            it.L.out_stride = r->out_stride;
            it.L.xf = static_cast<T *>(r->dxf);
            it.L.vf = static_cast<T *>(r->dvf);
            it.L.xe = static_cast<T *>(r->dxe);
            it.L.ve = static_cast<T *>(r->dve);
            it.L.nonfinite = sy->flag;
            it.L.load_mode = load;
            it.L.store_mode = store;
            it.b = 0;
            const std::pair<int, int> key{(int)sy->method, dense_vec_bucket(sy->s)};
            denses[key].push_back(it);
            dense_smax[key] = std::max(dense_smax[key], (int)sy->s);
            note(dense_shape[key], r, c);
        } else {
            DenseSplitLaunch<T> a{};
            split_launch_base(sy, a);
            a.out_stride = r->out_stride;
            a.xf = static_cast<T *>(r->dxf);
            a.vf = static_cast<T *>(r->dvf);
            a.x0 = static_cast<const T *>(r->dx0);
            a.v0 = static_cast<const T *>(r->dv0);
            a.xe = static_cast<T *>(r->dxe);
            a.ve = static_cast<T *>(r->dve);
            a.n0 = n0;
            a.nsteps = c;
            a.load_mode = load;
            a.store_mode = store;
            // the step graph's arguments do not change between chunks of a request
            hipStream_t sst = streams[next_stream];
            hipEvent_t e0 = event(), e1 = event();
            if (e0) (void)hipEventRecord(e0, sst);
            osc_status st = dense_split_run<T>(a, sy->method, sst, &sy->split_graph, &sy->split_graph_len, 64);
            if (e0 && e1 && hipEventRecord(e1, sst) == hipSuccess) timed.push_back({e0, e1, shape_key(*r), c});
            next_stream = (next_stream + 1) % kStreams;
            if (st != OSC_OK) r->status = st;
        }
    }
    for (auto &g : chains) {
        const size_t off = wl.append(g.second.data(), g.second.size() * sizeof(ChainItem<T>));
        const int64_t n = (int64_t)g.second.size();
        const int method = g.first.first;
        const ChainConfig cfgc{(int)(g.first.second >> 16), (int)(g.first.second & 0xffff)};
        wl.launches.push_back([=](const char *dev, hipStream_t st) {
            (void)chain_launch_items<T>(reinterpret_cast<const ChainItem<T> *>(dev + off), n, method, cfgc, st);
        });
        wl.shapes.push_back(chain_shape[g.first]);
    }
    for (auto &g : denses) {
        const size_t off = wl.append(g.second.data(), g.second.size() * sizeof(DenseItem<T>));
        const int64_t n = (int64_t)g.second.size();
        const int method = g.first.first, smax = dense_smax[g.first];
        wl.launches.push_back([=](const char *dev, hipStream_t st) {
            (void)dense_launch_items<T>(reinterpret_cast<const DenseItem<T> *>(dev + off), n, smax, method, st);
        });
        wl.shapes.push_back(dense_shape[g.first]);
    }
    for (auto &g : mfmas) {
        const size_t off = wl.append(g.second.data(), g.second.size() * sizeof(DenseMfmaItem));
        const int64_t n = (int64_t)g.second.size();
        const int method = g.first.first, pad = g.first.second;
        wl.launches.push_back([=](const char *dev, hipStream_t st) {
            (void)dense_mfma_launch_items(reinterpret_cast<const DenseMfmaItem *>(dev + off), n, pad, method, st);
        });
        wl.shapes.push_back(mfma_shape[g.first]);
    }
}

// Upload every work list of the iteration in one copy and launch the lists
// across the streams, each after the copy.  The worker drains all streams at
// the end of every iteration, so neither buffer is in use by an earlier copy
// or kernel when it is rewritten or replaced here.
void Server::launch_lists(WorkLists &wl, std::vector<Req *> &act, int &next_stream) {
    const size_t bytes = wl.image.size();
    if (bytes == 0) return;
    if (bytes > stage_bytes) {
        if (stage) (void)hipHostFree(stage);
        pool_free(items);
        stage = nullptr;
        items = nullptr;
        stage_bytes = items_bytes = 0;
        if (hipHostMalloc(&stage, bytes * 2, 0) != hipSuccess) stage = nullptr;
        items = pool_alloc(bytes * 2);
        if (!stage || !items) {
            if (stage) (void)hipHostFree(stage);
            pool_free(items);
            stage = nullptr;
            items = nullptr;
            for (Req *r : act) r->status = OSC_ENOMEM;
            return;
        }
        stage_bytes = items_bytes = bytes * 2;
    }
    std::memcpy(stage, wl.image.data(), bytes);
    hipEvent_t ready;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) {
        for (Req *r : act) r->status = OSC_EDEVICE;
        return;
    }
    if (hipMemcpyAsync(items, stage, bytes, hipMemcpyHostToDevice, streams[0]) != hipSuccess ||
        hipEventRecord(ready, streams[0]) != hipSuccess) {
        (void)hipEventDestroy(ready);
        for (Req *r : act) r->status = OSC_EDEVICE;
        return;
    }
    for (size_t i = 0; i < wl.launches.size(); ++i) {
        hipStream_t st = streams[next_stream];
        next_stream = (next_stream + 1) % kStreams;
        (void)hipStreamWaitEvent(st, ready, 0);
        hipEvent_t e0 = event(), e1 = event();
        if (e0) (void)hipEventRecord(e0, st);
        wl.launches[i](static_cast<const char *>(items), st);
        if (e0 && e1 && hipEventRecord(e1, st) == hipSuccess)
            timed.push_back({e0, e1, wl.shapes[i].first, wl.shapes[i].second});
    }
    (void)hipEventDestroy(ready);
}

void Server::run_iteration(std::vector<Req *> &act) {
    std::vector<int64_t> cnt(act.size());
    double sim = 0.0;
    timed.clear();
    events_used = 0;
    for (size_t i = 0; i < act.size(); ++i) {
        act[i]->chunk = chunk_of(*act[i]);
        cnt[i] = std::min(act[i]->chunk, act[i]->nsteps - act[i]->done);
        sim = std::max(sim, cnt[i] * step_seconds_guess(*act[i]));
    }
    if (cfg.fake_executor) {
        std::this_thread::sleep_for(std::chrono::duration<double>(std::min(sim, 0.002)));
    } else {
        WorkLists wl;
        int next_stream = 0;
        collect_groups<float>(act, cnt, wl, next_stream);
        collect_groups<double>(act, cnt, wl, next_stream);
        launch_lists(wl, act, next_stream);
        for (auto &st : streams) (void)hipStreamSynchronize(st);
        // seconds per step of each shape from this iteration's launches
        for (const Timed &t : timed) {
            float ms = 0.0f;
            if (t.steps <= 0 || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess || !(ms > 0.0f)) continue;
            const double per_step = 1e-3 * (double)ms / (double)t.steps;
            auto it = step_est.find(t.key);
            if (it == step_est.end()) step_est[t.key] = per_step;
            else it->second = 0.5 * it->second + 0.5 * per_step;
        }
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        ++iterations;
    }
    for (size_t i = 0; i < act.size(); ++i) {
        Req *r = act[i];
        r->done += cnt[i];
        ++r->iterations;
        if (r->status != OSC_OK) {
            finish(r, r->status, "a launch of this request failed");
            continue;
        }
        if (r->done < r->nsteps) continue;
        osc_status st = OSC_OK;
        std::string msg;
        if (!cfg.fake_executor) {
            const size_t s = (size_t)r->desc.s;
            bool ok = hipMemcpy(r->hxe.data(), r->dxe, s * r->elem, hipMemcpyDeviceToHost) == hipSuccess &&
                      hipMemcpy(r->hve.data(), r->dve, s * r->elem, hipMemcpyDeviceToHost) == hipSuccess;
            if (r->nframes > 0)
                ok = ok &&
                     hipMemcpy(r->hxf.data(), r->dxf, r->nframes * s * r->elem, hipMemcpyDeviceToHost) == hipSuccess &&
                     hipMemcpy(r->hvf.data(), r->dvf, r->nframes * s * r->elem, hipMemcpyDeviceToHost) == hipSuccess;
            if (!ok) {
                st = OSC_EDEVICE;
                msg = "download of the results failed";
            } else {
                st = osc_sync(r->sys);
                if (st != OSC_OK) msg = osc_last_error();
            }
        } else {
            std::memcpy(r->hxe.data(), r->x0.data(), r->x0.size());
            std::memcpy(r->hve.data(), r->v0.data(), r->v0.size());
        }
        finish(r, st, msg);
    }
}

void Server::setup_loop() {
    if (!cfg.fake_executor) (void)hipSetDevice(device);
    for (;;) {
        Req *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_setup.wait(lk, [&] { return stopping || !preparing.empty(); });
            if (preparing.empty()) {
                if (stopping) break;
                continue;
            }
            r = preparing.front();
            preparing.pop_front();
            ++in_setup;
        }
        const double t0 = now_s();
        const bool ok = setup(r);   // a failed or jump-served request is finished there; r must not be touched after
        const double t1 = now_s();
        std::lock_guard<std::mutex> lk(mu);
        --in_setup;
        setup_s += t1 - t0;
        if (ok) active.push_back(r);
        cv_work.notify_all();
    }
}

void Server::loop() {
    if (!cfg.fake_executor) (void)hipSetDevice(device);
    for (;;) {
        std::vector<Req *> act;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool admitted = false;
            while (!queue.empty() && (int64_t)(active.size() + preparing.size()) + in_setup < cfg.max_slots) {
                Req *r = queue.front();
                if (cfg.hbm_budget && in_use + (size_t)r->bytes > cfg.hbm_budget) break;   // wait for memory
                queue.pop_front();
                in_use += (size_t)r->bytes;
                peak = std::max(peak, in_use);
                r->st = RState::ACTIVE;
                r->t_admit = now_s();
                preparing.push_back(r);
                admitted = true;
            }
            if (admitted) cv_setup.notify_all();
            if (active.empty()) {
                if (stopping && queue.empty() && preparing.empty() && in_setup == 0) break;
                cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
            act = active;
        }
        const double t1 = now_s();
        run_iteration(act);
        const double t2 = now_s();
        std::lock_guard<std::mutex> lk(mu);
        iterate_s += t2 - t1;
    }
}

}  // namespace
}  // namespace osc

struct osc_server {
    osc::Server impl;
};

using namespace osc;

extern "C" {

osc_status osc_server_create(const osc_server_config *cfg, osc_server **out) {
    if (!out) return fail(OSC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(OSC_EINVAL, "config is NULL");
    if (cfg->max_slots < 1) return fail(OSC_EINVAL, "max_slots must be >= 1");
    if (cfg->chunk_us < 0) return fail(OSC_EINVAL, "chunk_us must be >= 0");
    osc_server *srv = new (std::nothrow) osc_server();
    if (!srv) return fail(OSC_ENOMEM, "host allocation failed");
    Server &S = srv->impl;
    S.cfg = *cfg;
    if (S.cfg.chunk_us == 0) S.cfg.chunk_us = 2000;
    if (!S.cfg.fake_executor) {
        if (hipGetDevice(&S.device) != hipSuccess) {
            delete srv;
            return fail(OSC_EDEVICE, "no HIP device");
        }
        bool ok = hipStreamCreateWithFlags(&S.setup_stream, hipStreamNonBlocking) == hipSuccess;
        for (auto &st : S.streams) ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (!ok) {
            for (auto &t : S.streams)
                if (t) (void)hipStreamDestroy(t);
            if (S.setup_stream) (void)hipStreamDestroy(S.setup_stream);
            delete srv;
            return fail(OSC_EDEVICE, "stream creation failed");
        }
    }
    S.setup_worker = std::thread([&S] { S.setup_loop(); });
    S.worker = std::thread([&S] { S.loop(); });
    *out = srv;
    return OSC_OK;
}

osc_status osc_server_submit(osc_server *srv, const osc_desc *d, const void *x0, const void *v0, int64_t nsteps,
                             int64_t out_stride, uint64_t *ticket) {
    if (!srv || !d || !x0 || !v0 || !ticket) return fail(OSC_EINVAL, "NULL argument");
    if (d->batch != 1) return fail(OSC_EINVAL, "a request is one instance (batch = 1)");
    if (d->param_mem != OSC_MEM_HOST) return fail(OSC_EINVAL, "request parameters must be host arrays");
    if (d->s < 1 || d->s > 2048) return fail(OSC_EINVAL, "s must be in [1, 2048]");
    if (d->kind != OSC_CHAIN && d->kind != OSC_DENSE) return fail(OSC_EINVAL, "unknown kind");
    if (d->method != OSC_RK4 && d->method != OSC_VERLET) return fail(OSC_EINVAL, "unknown method");
    if (d->prec != OSC_F64 && d->prec != OSC_F32) return fail(OSC_EINVAL, "unknown precision");
    if (!d->M || !d->K || !d->dt) return fail(OSC_EINVAL, "M, K and dt must be non-NULL");
    if (nsteps < 0 || out_stride < 0) return fail(OSC_EINVAL, "nsteps and out_stride must be >= 0");
    Server &S = srv->impl;
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(OSC_ENOMEM, "host allocation failed");
    const size_t s = (size_t)d->s;
    r->desc = *d;
    r->desc.shared = d->kind == OSC_DENSE ? 1 : 0;
    const size_t np = d->kind == OSC_CHAIN ? s : s * s;
    r->M.assign(d->M, d->M + np);
    r->K.assign(d->K, d->K + np);
    r->dt.assign(d->dt, d->dt + 1);
    r->elem = d->prec == OSC_F64 ? 8 : 4;
    r->x0.assign(static_cast<const unsigned char *>(x0), static_cast<const unsigned char *>(x0) + s * r->elem);
    r->v0.assign(static_cast<const unsigned char *>(v0), static_cast<const unsigned char *>(v0) + s * r->elem);
    r->nsteps = nsteps;
    r->out_stride = out_stride;
    r->nframes = out_stride > 0 ? nsteps / out_stride + 1 : 0;
    r->jump = S.cfg.frame_jumps != 0 && !S.cfg.fake_executor && jumps_pay(r->desc, nsteps, out_stride);
    r->bytes = estimate_bytes(r->desc, r->nframes, r->jump);
    if (r->jump && S.cfg.hbm_budget && (size_t)r->bytes > S.cfg.hbm_budget) {   // stepping needs less
        r->jump = false;
        r->bytes = estimate_bytes(r->desc, r->nframes, false);
    }
    if (S.cfg.hbm_budget && (size_t)r->bytes > S.cfg.hbm_budget) {
        delete r;
        return fail(OSC_ENOMEM, "request needs more device memory than the whole budget");
    }
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stopping) {
        delete r;
        return fail(OSC_EBUSY, "server is shutting down");
    }
    r->ticket = S.next_ticket++;
    r->t_submit = now_s();
    S.queue.push_back(r);
    S.all[r->ticket] = r;
    ++S.submitted;
    *ticket = r->ticket;
    S.cv_work.notify_one();
    return OSC_OK;
}

osc_status osc_server_wait(osc_server *srv, uint64_t ticket, double timeout_s, void *xf, void *vf, void *xe,
                           void *ve, osc_request_info *info) {
    if (!srv) return fail(OSC_EINVAL, "server is NULL");
    Server &S = srv->impl;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(OSC_EINVAL, "unknown ticket");
    Req *r = it->second;
    auto done = [&] { return r->st == RState::DONE || r->st == RState::FAILED; };
    if (timeout_s < 0) S.cv_done.wait(lk, done);
    else if (!S.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
        return fail(OSC_ETIMEOUT, "request not finished yet");
    if (info) {
        info->status = r->status;
        info->queue_s = r->t_admit > 0 ? r->t_admit - r->t_submit : r->t_done - r->t_submit;
        info->latency_s = r->t_done - r->t_submit;
        info->bytes = r->bytes;
        info->iterations = r->iterations;
        info->frame_jumps = r->jump ? 1 : 0;
    }
    const osc_status st = r->status;
    if (st == OSC_OK) {
        if (xf && !r->hxf.empty()) std::memcpy(xf, r->hxf.data(), r->hxf.size());
        if (vf && !r->hvf.empty()) std::memcpy(vf, r->hvf.data(), r->hvf.size());
        if (xe) std::memcpy(xe, r->hxe.data(), r->hxe.size());
        if (ve) std::memcpy(ve, r->hve.data(), r->hve.size());
    }
    const std::string msg = r->error;
    S.all.erase(it);
    delete r;
    if (st != OSC_OK) return fail(st, msg.empty() ? "request failed" : msg);
    return OSC_OK;
}

osc_status osc_server_stats(osc_server *srv, osc_server_counters *out) {
    if (!srv || !out) return fail(OSC_EINVAL, "NULL argument");
    Server &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    out->submitted = S.submitted;
    out->completed = S.completed;
    out->failed = S.failed;
    out->queued = (int64_t)S.queue.size();
    out->active = (int64_t)(S.active.size() + S.preparing.size()) + S.in_setup;
    out->iterations = S.iterations;
    out->hbm_in_use = S.in_use;
    out->hbm_peak = S.peak;
    out->setup_s = S.setup_s;
    out->iterate_s = S.iterate_s;
    return OSC_OK;
}

void osc_server_destroy(osc_server *srv) {
    if (!srv) return;
    Server &S = srv->impl;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stopping = true;
        for (Req *r : S.queue) {
            r->st = RState::FAILED;
            r->status = OSC_EBUSY;
            r->error = "server shut down before the request was admitted";
            r->t_done = now_s();
            ++S.failed;
        }
        S.queue.clear();
        S.cv_work.notify_all();
        S.cv_setup.notify_all();
        S.cv_done.notify_all();
    }
    if (S.worker.joinable()) S.worker.join();
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.cv_setup.notify_all();
    }
    if (S.setup_worker.joinable()) S.setup_worker.join();
    for (auto &kv : S.all) delete kv.second;
    S.all.clear();
    for (hipEvent_t e : S.event_pool) (void)hipEventDestroy(e);
    if (S.stage) (void)hipHostFree(S.stage);
    pool_free(S.items);
    for (auto &st : S.streams)
        if (st) (void)hipStreamDestroy(st);
    if (S.setup_stream) (void)hipStreamDestroy(S.setup_stream);
    delete srv;
}

}  // extern "C"
