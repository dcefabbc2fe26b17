// Continuous-batching server of libgapd.so (include/gapd.h, "serving").
//
// Jobs (all-pairs or multi-source propagations on an image) queue first come
// first served.  A job is admitted when a slot is free and its bytes (image,
// weights, workspace and result) fit in the caller's device arena; admitted
// jobs run concurrently, one HIP stream per slot, so work from different
// requests overlaps on the device.  A finished job keeps its result in the
// arena until gapd_serve_release returns the bytes, which lets waiting jobs in.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gapd.h"
#include "capi_internal.h"
#include "gapd_internal.h"

using namespace gapd;

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing free list (offsets).
class Arena {
  public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = al256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = al256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

enum class JState { Queued, Running, Done, Failed };

struct JobRec {
    gapd_job spec{};
    std::vector<uint8_t> image;
    std::vector<int32_t> sources;
    JState state = JState::Queued;
    int status = GAPD_OK;
    size_t bytes = 0, off = 0;
    size_t elems = 0;
    int64_t n_prop = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t *dev_out = nullptr;
};

// Bytes of a job in the arena: image, weights, control block, workspace,
// sources and result.
size_t job_bytes(const gapd_job &j, size_t *elems) {
    const size_t N = (size_t)j.H * j.W;
    size_t b = al256(N * j.C) + weight_block_bytes(j.H, j.W) + al256(sizeof(FrCtl));
    if (j.kind == GAPD_JOB_ALL_PAIRS) {
        if (j.mode != GAPD_MODE_NAIVE) b += fr_workspace_bytes((int)N, true);
        *elems = N * N;
    } else {
        b += al256(sizeof(int32_t) * (size_t)j.K);
        *elems = (size_t)j.K * N;
    }
    b += al256(*elems * sizeof(int32_t));
    return b;
}

}  // namespace

struct gapd_server {
    char *arena_dev = nullptr;
    size_t arena_bytes = 0;
    int device = 0;
    Arena arena{0};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<JobRec>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::atomic<bool> poisoned{false};  // a device error happened: no more jobs run
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void worker_loop();
    int run_job(JobRec &j, hipStream_t st);
};

int gapd_server::run_job(JobRec &j, hipStream_t st) {
    const gapd_job &s = j.spec;
    const int N = s.H * s.W;
    char *p = arena_dev + j.off;
    uint8_t *img = (uint8_t *)p;
    p += al256((size_t)N * s.C);
    GImgW w = weight_block_layout(p, s.H, s.W, s.conn);
    p += weight_block_bytes(s.H, s.W);
    FrCtl *ctl = (FrCtl *)p;
    p += al256(sizeof(FrCtl));
    std::string err;
    bool poisoned = false;
    hipError_t e = hipMemcpyAsync(img, j.image.data(), j.image.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(w.wr, 0, weight_block_bytes(s.H, s.W), st);
    if (e == hipSuccess) e = launch_prep(w, img, s.C, s.weight_mode, st);
    if (e != hipSuccess) return GAPD_EDEVICE;
    const GImg g = as_const(w);
    const int max_rounds = max_rounds_for(N);
    if (s.kind == GAPD_JOB_ALL_PAIRS) {
        if (s.mode != GAPD_MODE_NAIVE) {
            FrState fs = fr_workspace_layout(p, N, true);
            p += fr_workspace_bytes(N, true);
            fs.H = s.H;
            fs.W = s.W;
            fs.rule = s.mode == GAPD_MODE_TREE_FILL_EXTREMA ? kRuleExtrema : kRuleFilling;
            fs.D = (int32_t *)p;
            j.dev_out = fs.D;
            FrCtl hc{};
            const int r = run_filling_rate(g, fs, max_rounds, st, nullptr, hc, err, poisoned);
            j.n_prop = hc.n_prop;
            return r;
        }
        j.dev_out = (int32_t *)p;
        j.n_prop = N;
        return run_rows(g, nullptr, 0, N, j.dev_out, max_rounds, ctl, st, err, poisoned);
    }
    int32_t *src = (int32_t *)p;
    p += al256(sizeof(int32_t) * (size_t)s.K);
    j.dev_out = (int32_t *)p;
    j.n_prop = s.K;
    e = hipMemcpyAsync(src, j.sources.data(), sizeof(int32_t) * s.K, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return GAPD_EDEVICE;
    return run_rows(g, src, 0, s.K, j.dev_out, max_rounds, ctl, st, err, poisoned);
}

void gapd_server::worker_loop() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        JobRec *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) break;
                if (!queue.empty()) {
                    JobRec &head = *jobs[queue.front()];
                    size_t off = 0;
                    if (arena.alloc(head.bytes, &off)) {
                        head.off = off;
                        head.state = JState::Running;
                        head.t_admit = now();
                        j = &head;
                        queue.pop_front();
                        break;
                    }
                }
                cv_work.wait(lk);
            }
            if (!j) break;
        }
        int r = poisoned.load() ? GAPD_EDEVICE : run_job(*j, st);
        // Whatever run_job returned, nothing of this job may still be queued
        // on the slot's stream once its arena range can be released.  A device
        // error poisons the server: every later job fails at once.
        const hipError_t se = hipStreamSynchronize(st);
        if (se != hipSuccess || r == GAPD_EDEVICE) {
            poisoned.store(true);
            r = GAPD_EDEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            j->t_done = now();
            j->status = r;
            j->state = r == GAPD_OK ? JState::Done : JState::Failed;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
}

extern "C" {

int gapd_server_create(void *arena_dev, size_t arena_bytes, int max_slots, gapd_server **out) {
    if (!out) return GAPD_EINVAL;
    *out = nullptr;
    if (!arena_dev || arena_bytes == 0 || max_slots < 1 || max_slots > 64) return GAPD_EINVAL;
    if ((uintptr_t)arena_dev & 255) return GAPD_EINVAL;
    gapd_server *s = new gapd_server();
    s->arena_dev = (char *)arena_dev;
    s->arena_bytes = arena_bytes & ~size_t(255);
    s->arena = Arena(s->arena_bytes);
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return GAPD_EDEVICE; }
    for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s] { s->worker_loop(); });
    *out = s;
    return GAPD_OK;
}

int gapd_serve_submit(gapd_server *srv, const gapd_job *job, uint64_t *ticket) {
    if (!srv || !job || !ticket) return GAPD_EINVAL;
    if (job->kind != GAPD_JOB_ALL_PAIRS && job->kind != GAPD_JOB_MULTI_SOURCE) return GAPD_EINVAL;
    std::string why;
    int st = validate_image(job->image, job->H, job->W, job->C, job->conn, job->weight_mode, why);
    if (st != GAPD_OK) { g_create_error = why; return st; }
    const int N = job->H * job->W;
    if (job->kind == GAPD_JOB_ALL_PAIRS) {
        if (job->mode != GAPD_MODE_NAIVE && job->mode != GAPD_MODE_TREE_FILL_FR &&
            job->mode != GAPD_MODE_TREE_FILL_EXTREMA)
            return GAPD_EINVAL;
        if (job->mode != GAPD_MODE_NAIVE && !tree_methods_fit(job->H, job->W)) {
            g_create_error = "tree-method jobs need both image sides <= 192 (distance field in LDS)";
            return GAPD_EINVAL;
        }
    } else {
        if (job->K < 1 || !job->sources) return GAPD_EINVAL;
        for (int k = 0; k < job->K; ++k)
            if (job->sources[k] < 0 || job->sources[k] >= N) return GAPD_EINVAL;
    }
    auto rec = std::make_unique<JobRec>();
    rec->spec = *job;
    rec->image.assign(job->image, job->image + (size_t)N * job->C);
    if (job->kind == GAPD_JOB_MULTI_SOURCE) rec->sources.assign(job->sources, job->sources + job->K);
    rec->spec.image = nullptr;
    rec->spec.sources = nullptr;
    rec->bytes = job_bytes(*job, &rec->elems);
    if (al256(rec->bytes) > srv->arena_bytes) {
        g_create_error = "job larger than the whole arena";
        return GAPD_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        rec->t_submit = srv->now();
        const uint64_t t = srv->next_ticket++;
        srv->jobs[t] = std::move(rec);
        srv->queue.push_back(t);
        *ticket = t;
    }
    srv->cv_work.notify_all();
    return GAPD_OK;
}

static int fill_result(const JobRec &j, gapd_result *res) {
    if (j.state == JState::Queued || j.state == JState::Running) return GAPD_PENDING;
    if (j.state == JState::Failed) return j.status;
    if (res) {
        res->dev_out = j.dev_out;
        res->elems = j.elems;
        res->n_prop = j.n_prop;
        res->t_submit = j.t_submit;
        res->t_admit = j.t_admit;
        res->t_done = j.t_done;
    }
    return GAPD_OK;
}

int gapd_serve_poll(gapd_server *srv, uint64_t ticket, gapd_result *res) {
    if (!srv) return GAPD_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return GAPD_ENOTFOUND;
    return fill_result(*it->second, res);
}

int gapd_serve_wait(gapd_server *srv, uint64_t ticket, gapd_result *res) {
    if (!srv) return GAPD_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end()) return GAPD_ENOTFOUND;
        const int st = fill_result(*it->second, res);
        if (st != GAPD_PENDING) return st;
        if (srv->stop) return GAPD_EBUSY;
        srv->cv_done.wait(lk);
    }
}

int gapd_serve_release(gapd_server *srv, uint64_t ticket) {
    if (!srv) return GAPD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(ticket);
        if (it == srv->jobs.end()) return GAPD_ENOTFOUND;
        JobRec &j = *it->second;
        if (j.state == JState::Queued || j.state == JState::Running) return GAPD_EBUSY;
        srv->arena.release(j.off, j.bytes);
        srv->jobs.erase(it);
    }
    srv->cv_work.notify_all();
    return GAPD_OK;
}

void gapd_server_destroy(gapd_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (auto &t : srv->workers) t.join();
    delete srv;
}

}  // extern "C"
