// Serving runtime: continuous batching of independent implicit simulations
// on one device.
//
// One device arena is allocated at creation and carved into per-request
// ranges by a first-fit allocator with coalescing.  Worker threads, each
// owning a non-blocking HIP stream and a pinned read-back area, take the
// oldest waiting request whose range fits; once a request has been passed
// over 4 times per worker nothing passes it any more, so large requests are
// not starved by a stream of small ones.  An admitted request creates its
// problem inside its range (state, Krylov basis and preconditioner resident
// for the request's life), runs its implicit steps on the worker's stream and
// releases the range.  Concurrent requests overlap on the device through
// their streams; each request issues the same kernels and takes the same host
// decisions as it would alone, so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/jfnk.h"
#include "admission.hpp"
#include "problem.hpp"

namespace {

constexpr size_t kRangeAlign = 4096;
constexpr int kMaxActive = 64;
// a waiting request passed over this many times (per worker) blocks later arrivals
constexpr int kMaxSkipsPerWorker = 4;

enum { REQ_WAITING = 0, REQ_RUNNING = 1, REQ_DONE = 2 };

struct Request {
    long long id = 0;
    jfnk_problem_desc desc{};
    jfnk_solver_opts opts{};
    std::vector<double> u;  // initial state, then the final state
    int nsteps = 0;
    size_t bytes = 0;
    int state = REQ_WAITING;
    int skips = 0;
    jfnk_request_stats st{};
    std::vector<double> step_ms;
};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct jfnk_server {
    int device = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    jfnk::RangeAllocator ranges;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> waiting;
    std::map<long long, std::unique_ptr<Request>> reqs;
    std::vector<std::thread> workers;
    int nworkers = 0;
    bool stop = false;
    long long next_id = 1;
    std::chrono::steady_clock::time_point t0;

    // called with mu held: choose the request to admit and its range
    bool pick(Request** r, size_t* off) {
        return jfnk::pick_request(waiting, ranges, kMaxSkipsPerWorker * nworkers, r, off);
    }

    void run(Request* r, void* range, hipStream_t stream, void* pinned) {
        jfnk_problem* p = nullptr;
        int rc = jfnk::create_problem_in(&r->desc, &r->opts, r->u.data(), 0, stream, range, r->bytes, pinned, &p);
        if (rc != 0) {
            r->st.status = rc;
            return;
        }
        for (int k = 0; k < r->nsteps; ++k) {
            jfnk_step_stats ss;
            rc = jfnk_implicit_step(p, &ss);
            r->step_ms.push_back(ss.wall_ms);
            r->st.newton_its += ss.newton_its;
            r->st.gmres_its += ss.gmres_its;
            r->st.rejections += ss.rejections;
            if (rc != 0) {
                r->st.status = rc;
                break;
            }
            r->st.steps_done++;
            r->st.sim_time = ss.t;
        }
        rc = jfnk_get_state(p, r->u.data(), 0);
        if (rc != 0 && r->st.status == 0) r->st.status = rc;
        jfnk_destroy_problem(p);
    }

    void worker() {
        hipStream_t stream = nullptr;
        void* pinned = nullptr;
        bool ok = hipSetDevice(device) == hipSuccess &&
                  hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
                  hipHostMalloc(&pinned, jfnk::kPinnedBytes, hipHostMallocDefault) == hipSuccess;
        for (;;) {
            Request* r = nullptr;
            size_t off = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return pick(&r, &off) || (stop && waiting.empty()); });
                if (!r) break;
                r->state = REQ_RUNNING;
                r->st.t_admit_ms = ms_since(t0);
            }
            if (ok) {
                run(r, arena + off, stream, pinned);
                // every path out of run(), a failed creation included, may have
                // left copies or kernels on the stream that write into the
                // range: drain them before the range can go to another request
                if (hipStreamSynchronize(stream) != hipSuccess && r->st.status == 0) r->st.status = -3;
            } else {
                r->st.status = -3;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                ranges.release(off, r->bytes);
                r->state = REQ_DONE;
                r->st.t_done_ms = ms_since(t0);
            }
            cv_work.notify_all();
            cv_done.notify_all();
        }
        if (stream) (void)hipStreamDestroy(stream);
        if (pinned) (void)hipHostFree(pinned);
    }
};

extern "C" {

int jfnk_server_create(size_t hbm_bytes, int max_active, jfnk_server** out) {
    if (!out || hbm_bytes == 0 || max_active < 1 || max_active > kMaxActive)
        return jfnk::set_error(-1, "server: need an output pointer, hbm_bytes > 0 and 1 <= max_active <= 64");
    jfnk_server* s = new (std::nothrow) jfnk_server();
    if (!s) return jfnk::set_error(-2, "server: host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return jfnk::set_error(-3, "server: no HIP device");
    }
    s->arena_bytes = hbm_bytes / kRangeAlign * kRangeAlign;
    void* a = nullptr;
    if (hipMalloc(&a, s->arena_bytes) != hipSuccess) {
        delete s;
        return jfnk::set_error(-2, "server: arena allocation failed");
    }
    s->arena = (char*)a;
    s->ranges.init(s->arena_bytes);
    s->t0 = std::chrono::steady_clock::now();
    s->nworkers = max_active;
    for (int i = 0; i < max_active; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return 0;
}

int jfnk_server_submit(jfnk_server* s, const jfnk_problem_desc* desc, const jfnk_solver_opts* opts,
                       const double* u0, int nsteps, long long* id) {
    if (!s || !desc || !opts || !u0 || !id || nsteps < 0) return jfnk::set_error(-1, "server_submit: bad argument");
    size_t fp = 0;
    int rc = jfnk_footprint_bytes(desc, opts, &fp);
    if (rc) return rc;
    const size_t bytes = (jfnk::problem_range_bytes(desc, opts) + kRangeAlign - 1) / kRangeAlign * kRangeAlign;
    if (bytes > s->arena_bytes) return jfnk::set_error(-1, "server_submit: request larger than the arena");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return jfnk::set_error(-2, "server_submit: host allocation failed");
    r->desc = *desc;
    r->opts = *opts;
    const size_t nvec = (size_t)(2 + desc->ndim) * desc->n[0] * desc->n[1] * (desc->ndim > 2 ? desc->n[2] : 1);
    r->u.assign(u0, u0 + nvec);
    r->nsteps = nsteps;
    r->bytes = bytes;
    r->step_ms.reserve((size_t)nsteps);
    r->st.cells = (double)desc->n[0] * desc->n[1] * (desc->ndim > 2 ? desc->n[2] : 1);
    r->st.footprint_bytes = (double)fp;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return jfnk::set_error(-1, "server_submit: server is stopping");
        r->id = s->next_id++;
        r->st.t_submit_ms = ms_since(s->t0);
        *id = r->id;
        s->waiting.push_back(r.get());
        s->reqs[r->id] = std::move(r);
    }
    s->cv_work.notify_all();
    return 0;
}

int jfnk_server_poll(jfnk_server* s, long long id) {
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    return it == s->reqs.end() ? -1 : it->second->state;
}

int jfnk_server_wait(jfnk_server* s, long long id, double* u_out, jfnk_request_stats* st, double* step_ms,
                     int cap, int* nsteps_out) {
    if (!s) return jfnk::set_error(-1, "server_wait: null server");
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return jfnk::set_error(-1, "server_wait: unknown request");
        Request* q = it->second.get();
        s->cv_done.wait(lk, [&] { return q->state == REQ_DONE; });
        r = std::move(it->second);
        s->reqs.erase(it);
    }
    if (u_out) std::memcpy(u_out, r->u.data(), sizeof(double) * r->u.size());
    if (st) *st = r->st;
    const int n = (int)r->step_ms.size();
    if (step_ms && cap > 0) std::memcpy(step_ms, r->step_ms.data(), sizeof(double) * (size_t)std::min(n, cap));
    if (nsteps_out) *nsteps_out = n;
    return 0;
}

int jfnk_server_destroy(jfnk_server* s) {
    if (!s) return 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    if (s->arena) (void)hipFree(s->arena);
    delete s;
    return 0;
}

}  // extern "C"
