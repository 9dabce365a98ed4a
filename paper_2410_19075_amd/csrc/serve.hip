// Continuous-batching server (nd_server_* in include/nd.h).
//
// Requests are queued FIFO with their arrival time.  Each pump admits queued
// requests while their device footprint fits the HBM budget and a slot is free,
// enqueues one chunk of RK4 steps for every admitted request that has steps
// left, and retires the requests whose last chunk has completed.  Admitted
// requests are grouped by kernel class (model, topology, precision, tile
// shape); every class owns a fixed-capacity descriptor table and work map in
// device memory and one chunk graph captured once with a persistent grid.
// Between chunks only the table contents change (double-buffered pinned host
// staging, async copies on the pump's stream), so the same graph is replayed
// whatever the mix of requests.  A request's kernels and tile decomposition
// depend on its own problem only, so its arithmetic is identical alone and in
// any mix.
//
// The device is kept busy across pumps: a pump enqueues chunk k+1 before it
// waits for chunk k, so admission, retirement and the host's table updates run
// while the device works.  Admission allocates from the device's stream-ordered
// pool and uploads the initial state on a copy stream of the server (the
// compute stream waits on an event before the request's first chunk);
// retirement downloads results on the copy stream and frees on it, so neither
// synchronises the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace nd {

#define HIPC(expr)                                        \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

using ClassKey = std::tuple<int, int, int, int, int, int, int>;

static ClassKey class_key(const Net* n) {
    const int h = n->prob.topo == ND_CUBE3D || n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D
                      ? (int)n->prob.radius : 0;
    const int bs = (n->prob.topo == ND_BALL3D || n->prob.topo == ND_DISK2D) ? n->cfg.block : 0;
    return ClassKey(n->prob.model, n->prob.topo, n->prob.precision, n->cfg.tile, n->cfg.tile_y, h, bs);
}

struct Request {
    nd_req id = 0;
    int sidx = -1;            // pinned status word of the server
    int64_t last_seq = -1;    // last chunk that includes the request
    hipEvent_t ready = nullptr;  // recorded on the copy stream behind the admission uploads
    bool waited = false;      // the compute stream waits on `ready` before the first chunk
    nd_problem prob{};
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> weight, per_elem, y0, y, R;
    double dt = 0.0;
    int64_t steps = 0;
    nd_observe obs{0, -1};
    int64_t footprint = 0;
    int32_t state = ND_REQ_QUEUED;
    nd_status status = ND_OK;
    double arrival = 0.0, admitted = -1.0, finished = -1.0;
    Net* net = nullptr;
    int cls = -1, slot = -1;
    bool cancel = false;
};

struct ClassTable {
    ClassKey key;
    Group g{};
    int cap_desc = 0, cap_work = 0;
    void* dev = nullptr;  // desc | work | nwork
    // host staging, double-buffered by chunk parity: the copies of chunk k read
    // buffer k & 1 while the host fills the other for chunk k + 1
    NetDesc* h_desc[2] = {nullptr, nullptr};
    int2* h_work[2] = {nullptr, nullptr};
    int* h_nwork[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // without / with mean-velocity kernels
    std::vector<Request*> slots;

    ~ClassTable() {
        for (auto& e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        if (dev) (void)hipFree(dev);
        for (int b = 0; b < 2; ++b) {
            if (h_desc[b]) (void)hipHostFree(h_desc[b]);
            if (h_work[b]) (void)hipHostFree(h_work[b]);
            if (h_nwork[b]) (void)hipHostFree(h_nwork[b]);
        }
    }
    int active() const {
        int c = 0;
        for (auto* r : slots) c += r != nullptr;
        return c;
    }
};

// A chunk in flight: its sequence number and the timing events around it.
struct Inflight {
    int64_t seq;
    hipEvent_t start, end;
};

struct Server {
    nd_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::map<nd_req, std::unique_ptr<Request>> reqs;
    std::deque<Request*> queue;
    std::vector<Request*> running;
    std::vector<std::unique_ptr<ClassTable>> classes;
    int64_t next_id = 1;
    nd_server_counters st{};
    hipStream_t cs = nullptr;        // copy stream: admission uploads, result downloads, frees
    int32_t* h_status = nullptr;     // pinned status words, one per running request
    std::vector<int> free_sidx;
    std::deque<Inflight> inflight;   // chunks enqueued and not yet seen complete, oldest first
    std::vector<hipEvent_t> ev_pool;
    int64_t next_seq = 0, done_seq = -1;
    double last_pump = -1.0;  // server clock at the previous pump

    ~Server();
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    nd_status init();
    nd_status table_for(Request* r, ClassTable** out);
    nd_status grow_work(ClassTable* t, int need);
    nd_status admit(Request* r);
    void release(Request* r, int32_t state, nd_status why);
    nd_status launch(hipStream_t st, bool* launched);
    nd_status finish_oldest(bool wait, bool* done);
    nd_status drain();
    nd_status retire();
    nd_status pump(hipStream_t st, int64_t* pending);
};

nd_status Server::init() {
    HIPC(hipHostMalloc((void**)&h_status, (size_t)cfg.max_slots * sizeof(int32_t)));
    for (int i = cfg.max_slots - 1; i >= 0; --i) free_sidx.push_back(i);
    HIPC(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    return ND_OK;
}

Server::~Server() {
    // wait for the chunks still in flight (their end events) and the copy stream,
    // not for the whole device
    for (auto& f : inflight) (void)hipEventSynchronize(f.end);
    if (cs) (void)hipStreamSynchronize(cs);
    for (Request* r : running) {
        if (r->net) delete r->net;
        if (r->ready) (void)hipEventDestroy(r->ready);
    }
    classes.clear();
    if (cs) {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamDestroy(cs);
    }
    for (auto& f : inflight) {
        (void)hipEventDestroy(f.start);
        (void)hipEventDestroy(f.end);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (h_status) (void)hipHostFree(h_status);
}

static void set_empty(NetDesc& d) {
    std::memset(&d, 0, sizeof d);
    d.r_every = 1;
}

nd_status Server::grow_work(ClassTable* t, int need) {
    if (need <= t->cap_work && t->dev) return ND_OK;
    // the device tables and the staging are replaced: no chunk may still use them
    nd_status s = drain();
    if (s) return s;
    int cap = std::max(need, std::max(1024, 2 * t->cap_work));
    for (auto& e : t->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    if (t->dev) (void)hipFree(t->dev);
    t->dev = nullptr;
    for (int b = 0; b < 2; ++b) {
        if (t->h_work[b]) (void)hipHostFree(t->h_work[b]);
        t->h_work[b] = nullptr;
    }
    const size_t bd = (size_t)t->cap_desc * sizeof(NetDesc), bw = (size_t)cap * sizeof(int2);
    HIPC(hipMalloc(&t->dev, bd + bw + 64));
    for (int b = 0; b < 2; ++b) HIPC(hipHostMalloc((void**)&t->h_work[b], bw));
    t->cap_work = cap;
    t->g.desc = (NetDesc*)t->dev;
    t->g.work = (int2*)((char*)t->dev + bd);
    t->g.nwork = (int*)((char*)t->dev + bd + bw);
    return ND_OK;
}

nd_status Server::table_for(Request* r, ClassTable** out) {
    const ClassKey key = class_key(r->net);
    for (auto& t : classes)
        if (t->key == key) {
            *out = t.get();
            return ND_OK;
        }
    auto t = std::make_unique<ClassTable>();
    t->key = key;
    t->cap_desc = cfg.max_slots;
    t->slots.assign(cfg.max_slots, nullptr);
    Group& g = t->g;
    g.model = std::get<0>(key);
    g.topo = std::get<1>(key);
    g.prec = std::get<2>(key);
    g.tile = std::get<3>(key);
    g.tile_y = std::get<4>(key);
    g.h = std::get<5>(key);
    g.block = std::get<6>(key);
    g.ndesc = t->cap_desc;
    g.grid = cfg.grid;
    for (int b = 0; b < 2; ++b) {
        HIPC(hipHostMalloc((void**)&t->h_desc[b], (size_t)t->cap_desc * sizeof(NetDesc)));
        HIPC(hipHostMalloc((void**)&t->h_nwork[b], 64));
    }
    nd_status s = grow_work(t.get(), 1024);
    if (s) return s;
    *out = t.get();
    classes.push_back(std::move(t));
    return ND_OK;
}

nd_status Server::admit(Request* r) {
    nd_status s;
    if (!cs && (s = init())) return s;  // device resources at the first admission (the rest stays host-only)
    Net* n = new (std::nothrow) Net();
    if (!n) return fail(ND_ERR_OUT_OF_MEMORY, "host allocation failed");
    const int sidx = free_sidx.back();
    n->astream = cs;
    n->own_status_host = false;
    n->status_host = h_status + sidx;
    s = n->create(&r->prob);
    if (!s) s = n->begin_run(r->dt, r->steps, &r->obs);
    hipError_t e = hipSuccess;
    if (!s) {
        e = hipMemcpyAsync(n->tmpl.y[n->ypar], r->y0.data(), r->y0.size() * 8, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r->ready, cs);
        if (e != hipSuccess) s = hip_fail(e, "admission upload");
    }
    if (s) {
        delete n;
        if (r->ready) (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
        return s;
    }
    free_sidx.pop_back();
    r->sidx = sidx;
    r->net = n;
    st.bytes_in_use += r->footprint;
    ClassTable* t = nullptr;
    if ((s = table_for(r, &t))) {
        release(r, ND_REQ_FAILED, s);
        return s;
    }
    const int slot = (int)(std::find(t->slots.begin(), t->slots.end(), nullptr) - t->slots.begin());
    t->slots[slot] = r;
    r->cls = (int)(std::find_if(classes.begin(), classes.end(), [&](auto& c) { return c.get() == t; }) -
                   classes.begin());
    r->slot = slot;
    r->state = ND_REQ_RUNNING;
    r->admitted = now();
    running.push_back(r);
    return ND_OK;
}

// Called only once every chunk that includes r has completed.
void Server::release(Request* r, int32_t state, nd_status why) {
    if (r->slot >= 0) classes[r->cls]->slots[r->slot] = nullptr;
    r->slot = -1;
    if (r->net) {
        delete r->net;  // frees ordered on the copy stream
        r->net = nullptr;
        st.bytes_in_use -= r->footprint;
    }
    if (r->ready) {
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
    }
    r->y0.clear();  // the admission upload read it; every chunk after it has completed
    r->y0.shrink_to_fit();
    if (r->sidx >= 0) {
        free_sidx.push_back(r->sidx);
        r->sidx = -1;
    }
    r->state = state;
    r->status = why;
    r->finished = now();
    if (state == ND_REQ_DONE) ++st.completed;
    if (state == ND_REQ_FAILED) ++st.failed;
    if (state == ND_REQ_CANCELLED) ++st.cancelled;
}

// Enqueue one chunk on strm for every running request with steps left (not
// cancelled, not failed); host progress advances here, at enqueue time.
nd_status Server::launch(hipStream_t strm, bool* launched) {
    *launched = false;
    const int K = cfg.chunk_steps;
    const int b = (int)(next_seq & 1);
    auto live = [](const Request* r) {
        return r && !r->cancel && r->net->run_done < r->net->run_total && !*r->net->status_host;
    };
    nd_status s;
    hipEvent_t ev0 = nullptr;
    for (auto& tp : classes) {
        ClassTable* t = tp.get();
        int nw = 0;
        bool mv = false, any = false;
        for (Request* r : t->slots)
            if (live(r)) {
                any = true;
                nw += (int)r->net->work_items();
                mv = mv || r->net->mv_start >= 0;
            }
        if (!any) continue;
        if ((s = grow_work(t, nw))) return s;
        if (!ev0) {
            if (ev_pool.size() < 2)
                for (int q = 0; q < 2; ++q) {
                    hipEvent_t e;
                    HIPC(hipEventCreate(&e));
                    ev_pool.push_back(e);
                }
            ev0 = ev_pool.back();
            ev_pool.pop_back();
            HIPC(hipEventRecord(ev0, strm));
        }
        int w = 0;
        for (int sl = 0; sl < t->cap_desc; ++sl) {
            Request* r = t->slots[sl];
            if (live(r)) {
                if (!r->waited) {  // the admission uploads precede the first chunk
                    HIPC(hipStreamWaitEvent(strm, r->ready, 0));
                    r->waited = true;
                }
                t->h_desc[b][sl] = r->net->chunk_desc();
                const int64_t m = r->net->work_items();
                for (int64_t q = 0; q < m; ++q) t->h_work[b][w++] = make_int2(sl, (int)q);
            } else {
                set_empty(t->h_desc[b][sl]);
            }
        }
        *t->h_nwork[b] = w;
        HIPC(hipMemcpyAsync(t->g.desc, t->h_desc[b], (size_t)t->cap_desc * sizeof(NetDesc), hipMemcpyHostToDevice,
                            strm));
        HIPC(hipMemcpyAsync(t->g.work, t->h_work[b], (size_t)std::max(w, 1) * sizeof(int2), hipMemcpyHostToDevice,
                            strm));
        HIPC(hipMemcpyAsync(t->g.nwork, t->h_nwork[b], sizeof(int), hipMemcpyHostToDevice, strm));
        t->g.mv = mv;
        if (graphs_enabled()) {
            hipGraphExec_t& ex = t->exec[mv ? 1 : 0];
            if (!ex && (s = capture_chunk(t->g, K, &ex))) return s;
            HIPC(hipGraphLaunch(ex, strm));
        } else if ((s = enqueue_chunk(t->g, K, strm))) {
            return s;
        }
    }
    if (!ev0) return ND_OK;
    // status words behind the chunk (a non-finite state fails the request at the
    // chunk boundary), progress, and the chunk's end event
    const int64_t seq = next_seq++;
    for (Request* r : running) {
        if (!live(r)) continue;
        Net* n = r->net;
        HIPC(hipMemcpyAsync(n->status_host, n->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost, strm));
        const int64_t done = std::min<int64_t>(K, n->run_total - n->run_done);
        n->run_done += done;
        n->ypar ^= (int)(done & 1);
        st.osc_steps += done * n->prob.n;
        r->last_seq = seq;
    }
    hipEvent_t ev1 = ev_pool.back();
    ev_pool.pop_back();
    HIPC(hipEventRecord(ev1, strm));
    inflight.push_back({seq, ev0, ev1});
    ++st.chunks;
    *launched = true;
    return ND_OK;
}

// The oldest chunk in flight: wait for it (or only test it), count its device
// time and mark its requests' work as complete.
nd_status Server::finish_oldest(bool wait, bool* done) {
    *done = false;
    if (inflight.empty()) return ND_OK;
    Inflight f = inflight.front();
    if (wait) {
        HIPC(hipEventSynchronize(f.end));
    } else {
        const hipError_t q = hipEventQuery(f.end);
        if (q == hipErrorNotReady) return ND_OK;
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, f.start, f.end) == hipSuccess) st.gpu_seconds += 1e-3 * ms;
    inflight.pop_front();
    ev_pool.push_back(f.start);
    ev_pool.push_back(f.end);
    done_seq = f.seq;
    *done = true;
    return ND_OK;
}

nd_status Server::drain() {
    bool d = true;
    nd_status s;
    while (!inflight.empty())
        if ((s = finish_oldest(true, &d))) return s;
    return ND_OK;
}

// Retire the requests none of whose chunks is still in flight: cancelled, failed
// (non-finite state) or finished (results downloaded on the copy stream).
nd_status Server::retire() {
    std::vector<Request*> still;
    for (Request* r : running) {
        Net* n = r->net;
        if (r->last_seq > done_seq) {
            still.push_back(r);
        } else if (r->cancel) {
            release(r, ND_REQ_CANCELLED, ND_OK);
        } else if (*n->status_host) {
            release(r, ND_REQ_FAILED, fail(ND_ERR_NUMERIC, "request %lld: the state turned non-finite",
                                           (long long)r->id));
        } else if (n->run_done >= n->run_total) {
            r->y.resize((size_t)nvars_of(r->prob.model) * r->prob.n);
            hipError_t e = hipMemcpyAsync(r->y.data(), n->tmpl.y[n->ypar], r->y.size() * 8, hipMemcpyDeviceToHost, cs);
            if (e == hipSuccess && n->r_every > 0) {
                r->R.resize(n->run_total / n->r_every + 1);
                e = hipMemcpyAsync(r->R.data(), n->R_dev, r->R.size() * 8, hipMemcpyDeviceToHost, cs);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(cs);  // the copy stream only
            if (e != hipSuccess) {
                release(r, ND_REQ_FAILED, hip_fail(e, "result download"));
            } else {
                bool finite = true;
                for (double v : r->y) finite = finite && std::isfinite(v);
                release(r, finite ? ND_REQ_DONE : ND_REQ_FAILED, finite ? ND_OK : ND_ERR_NUMERIC);
            }
        } else {
            still.push_back(r);
        }
    }
    running.swap(still);
    return ND_OK;
}

nd_status Server::pump(hipStream_t strm, int64_t* pending) {
    nd_status s;
    const double t = now();
    if (last_pump >= 0.0 && (!running.empty() || !inflight.empty())) st.active_seconds += t - last_pump;
    last_pump = t;
    bool d = true;
    // ---- chunks that completed meanwhile, and the requests they finish
    while (d)
        if ((s = finish_oldest(false, &d))) return s;
    if ((s = retire())) return s;
    // ---- admission: FIFO while the head fits the budget and a slot is free
    while (!queue.empty()) {
        Request* r = queue.front();
        if (r->cancel) {
            queue.pop_front();
            release(r, ND_REQ_CANCELLED, ND_OK);
            continue;
        }
        if ((int)running.size() >= cfg.max_slots) break;
        if (st.bytes_in_use + r->footprint > cfg.hbm_budget_bytes) break;
        queue.pop_front();
        if ((s = admit(r))) {
            if (r->state == ND_REQ_QUEUED) release(r, ND_REQ_FAILED, s);
        }
    }
    // ---- the next chunk, queued behind the one the device is running
    bool launched = false;
    if ((s = launch(strm, &launched))) return s;
    // ---- keep one chunk queued behind the running one; with nothing new to
    // launch, wait for the oldest so that progress is made
    while (inflight.size() > 1 || (!launched && !inflight.empty()))
        if ((s = finish_oldest(true, &d))) return s;
    if ((s = retire())) return s;
    if (pending) *pending = (int64_t)(queue.size() + running.size());
    return ND_OK;
}

}  // namespace nd

using namespace nd;

extern "C" {

nd_status nd_server_create(const nd_server_config* cfg, nd_server_h* out) {
    if (!cfg || !out) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->reserved != 0) return fail(ND_ERR_INVALID_ARG, "reserved must be 0");
    if (cfg->hbm_budget_bytes <= 0) return fail(ND_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
    if (cfg->max_slots < 1 || cfg->max_slots > 4096) return fail(ND_ERR_INVALID_ARG, "max_slots in [1, 4096]");
    if (cfg->chunk_steps < 1) return fail(ND_ERR_INVALID_ARG, "chunk_steps must be >= 1");
    if (cfg->grid < 0 || (cfg->grid % 8) != 0) return fail(ND_ERR_INVALID_ARG, "grid must be a multiple of 8");
    Server* s = new (std::nothrow) Server();
    if (!s) return fail(ND_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->cfg = *cfg;
    if (s->cfg.grid == 0) s->cfg.grid = 2048;
    s->t0 = std::chrono::steady_clock::now();
    *out = reinterpret_cast<nd_server_h>(s);
    return ND_OK;
}

static Server* as_server(nd_server_h h) { return reinterpret_cast<Server*>(h); }

nd_status nd_server_now(nd_server_h h, double* seconds) {
    Server* s = as_server(h);
    if (!s || !seconds) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    *seconds = s->now();
    return ND_OK;
}

nd_status nd_server_submit(nd_server_h h, const nd_problem* p, const double* y0, int64_t len, double dt,
                           int64_t steps, const nd_observe* obs, double arrival, nd_req* id) {
    Server* s = as_server(h);
    if (!s || !id || !y0) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    nd_status st = validate_problem(p);
    if (st) return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ND_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (steps < 1) return fail(ND_ERR_INVALID_ARG, "steps must be >= 1");
    const int64_t want = nvars_of(p->model) * p->n;
    if (len != want) return fail(ND_ERR_INVALID_ARG, "state length %lld, expected %lld", (long long)len,
                                 (long long)want);
    if (obs) {
        if (obs->record_every < 0 || obs->mv_start_step < -1 || obs->mv_start_step >= steps)
            return fail(ND_ERR_INVALID_ARG, "bad observation settings");
        if ((obs->record_every > 0 || obs->mv_start_step >= 0) && p->model == ND_HH)
            return fail(ND_ERR_INVALID_ARG, "R and mean phase velocity are not defined for HH");
    }
    for (int64_t i = 0; i < len; ++i)
        if (!std::isfinite(y0[i])) return fail(ND_ERR_NUMERIC, "initial state holds a non-finite value at %lld",
                                               (long long)i);
    auto r = std::make_unique<Request>();
    r->prob = *p;
    if (p->topo == ND_CSR || p->topo == ND_LINKS) {
        r->row_ptr.assign(p->row_ptr, p->row_ptr + p->n + 1);
        r->col.assign(p->col, p->col + p->nnz);
        r->prob.row_ptr = r->row_ptr.data();
        r->prob.col = r->col.data();
        if (p->topo == ND_CSR) {
            r->weight.assign(p->weight, p->weight + p->nnz);
            r->prob.weight = r->weight.data();
        }
    }
    if (p->per_elem) {
        r->per_elem.assign(p->per_elem, p->per_elem + p->n);
        r->prob.per_elem = r->per_elem.data();
    }
    r->y0.assign(y0, y0 + len);
    r->dt = dt;
    r->steps = steps;
    if (obs) r->obs = *obs;
    r->footprint = footprint_bytes(p, config_for(p));
    if (r->obs.record_every > 0) r->footprint += (steps / r->obs.record_every + 1) * 8;
    if (r->obs.mv_start_step >= 0) r->footprint += p->n * 8;
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->footprint > s->cfg.hbm_budget_bytes)
        return fail(ND_ERR_INVALID_ARG, "request footprint %lld exceeds the HBM budget %lld",
                    (long long)r->footprint, (long long)s->cfg.hbm_budget_bytes);
    r->id = s->next_id++;
    r->arrival = arrival >= 0.0 ? arrival : s->now();
    *id = r->id;
    s->queue.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    ++s->st.submitted;
    return ND_OK;
}

nd_status nd_server_pump(nd_server_h h, void* stream, int64_t* pending) {
    Server* s = as_server(h);
    if (!s) return fail(ND_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    return s->pump((hipStream_t)stream, pending);
}

nd_status nd_server_info(nd_server_h h, nd_req id, nd_request_info* info) {
    Server* s = as_server(h);
    if (!s || !info) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(ND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    const Request* r = it->second.get();
    info->state = r->state;
    info->status = r->status;
    info->steps_done = r->net ? r->net->run_done : (r->state == ND_REQ_DONE ? r->steps : 0);
    info->arrival = r->arrival;
    info->admitted = r->admitted;
    info->finished = r->finished;
    return ND_OK;
}

nd_status nd_server_result(nd_server_h h, nd_req id, double* y, int64_t len, double* R, int64_t r_len) {
    Server* s = as_server(h);
    if (!s) return fail(ND_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(ND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    const Request* r = it->second.get();
    if (r->state != ND_REQ_DONE) return fail(ND_ERR_NOT_READY, "request %lld is not done", (long long)id);
    if (y) {
        if (len != (int64_t)r->y.size()) return fail(ND_ERR_INVALID_ARG, "state length mismatch");
        std::memcpy(y, r->y.data(), len * 8);
    }
    if (R) {
        if (r_len != (int64_t)r->R.size()) return fail(ND_ERR_INVALID_ARG, "R length mismatch");
        std::memcpy(R, r->R.data(), r_len * 8);
    }
    return ND_OK;
}

nd_status nd_server_cancel(nd_server_h h, nd_req id) {
    Server* s = as_server(h);
    if (!s) return fail(ND_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(ND_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    Request* r = it->second.get();
    if (r->state == ND_REQ_QUEUED || r->state == ND_REQ_RUNNING) r->cancel = true;
    return ND_OK;
}

nd_status nd_server_stats(nd_server_h h, nd_server_counters* out) {
    Server* s = as_server(h);
    if (!s || !out) return fail(ND_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)s->running.size();
    return ND_OK;
}

nd_status nd_server_destroy(nd_server_h h) {
    Server* s = as_server(h);
    if (!s) return fail(ND_ERR_INVALID_ARG, "NULL server");
    delete s;
    return ND_OK;
}

}  // extern "C"
