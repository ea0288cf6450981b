// Continuous-batching job server.
//
// Jobs are queued in arrival order.  When a stream is free, the first queued
// job whose device footprint (workspace + tables of its task, as computed by
// footprint_bytes) fits in the budget next to the jobs already running is
// admitted, so a small job does not wait behind a large one that does not fit
// yet.  Each time a job is passed over that way it counts one bypass; a job
// passed over kMaxBypass times stops later jobs from passing it, so it runs as
// soon as memory frees up (no starvation).  Admitted jobs run concurrently,
// one per HIP stream, so the kernels of several jobs overlap on the device.
// Each job runs the same code path as fabx_score with its own task and
// workspace, so its result does not depend on what else is running; a job
// that fails leaves the others untouched.  When a job ends, its device
// memory (workspace and task tables) goes back to the context's pool; the
// result keeps the per-cell counts on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "internal.h"

namespace fabx {
namespace {

using Clock = std::chrono::steady_clock;

enum class JobState { Queued, Running, Done, Failed, Cancelled };

// Times a queued job may be passed over by later jobs that fit before it.
constexpr int kMaxBypass = 8;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Job {
    std::shared_ptr<TaskImpl> task;
    ScoreParams params{};
    int64_t footprint = 0;
    JobState state = JobState::Queued;
    std::shared_ptr<ResultImpl> result;
    int code = FABX_OK;
    std::string msg;
    int bypassed = 0;
    // submit entry, end of the task build (queued), admission, completion
    Clock::time_point t_submit, t_queued, t_admit, t_done;
    // recorded on the context's stream at submit: the job's stream waits for it,
    // so the job reads features produced there before the submit call
    hipEvent_t ready = nullptr;
};

}  // namespace

struct ServerImpl {
    std::shared_ptr<CtxImpl> ctx;
    int64_t budget = 0;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Job> jobs;
    uint64_t next_id = 1;
    int64_t in_use = 0, high_water = 0;
    int64_t submitted = 0, completed = 0, cancelled = 0, failed = 0, running = 0;
    // per completed job: completion - submit entry, and its parts
    std::vector<double> latencies_ms, build_ms, queue_ms, run_ms;
    bool stop = false;

    // The queued job to admit now, or queue.end(): the first that fits, unless
    // a job before it has been passed over kMaxBypass times already.  Called
    // with mu held.
    std::deque<uint64_t>::iterator pick() {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            Job &j = jobs[*it];
            if (j.footprint <= budget - in_use) return it;
            if (j.bypassed >= kMaxBypass) break;
        }
        return queue.end();
    }

    void drop_event(Job &j) {
        if (j.ready) ctx->events.put(j.ready);
        j.ready = nullptr;
    }

    void worker(size_t k) {
        (void)hipSetDevice(ctx->device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            std::deque<uint64_t>::iterator chosen;
            cv.wait(lk, [&] {
                if (stop) return true;
                chosen = pick();
                return chosen != queue.end();
            });
            if (stop && queue.empty()) return;
            if (stop) {
                // cancel what is still queued
                for (uint64_t id : queue) {
                    jobs[id].state = JobState::Cancelled;
                    drop_event(jobs[id]);
                    ++cancelled;
                }
                queue.clear();
                cv.notify_all();
                return;
            }
            const uint64_t id = *chosen;
            for (auto it = queue.begin(); it != chosen; ++it) ++jobs[*it].bypassed;
            queue.erase(chosen);
            Job &job = jobs[id];
            job.state = JobState::Running;
            job.t_admit = Clock::now();
            in_use += job.footprint;
            high_water = std::max(high_water, in_use);
            ++running;
            auto task = job.task;
            auto params = job.params;
            const hipEvent_t ready = job.ready;
            lk.unlock();
            std::shared_ptr<ResultImpl> res;
            int code = FABX_OK;
            std::string msg;
            try {
                FABX_HIP(hipStreamWaitEvent(streams[k], ready, 0));
                res = run_score(task, params, streams[k]);
            } catch (const Error &e) {
                code = e.code;
                msg = e.msg;
            } catch (const std::exception &e) {
                code = FABX_ENOMEM;
                msg = e.what();
            }
            // nothing of the job may still run on the stream (a failed call can leave
            // launches behind) before its memory and its event are reused
            (void)hipStreamSynchronize(streams[k]);
            // the result keeps per-cell counts on the host; give the device memory
            // (workspace, task tables, column plans) back to the context's pool
            release_device(*task);
            lk.lock();
            Job &j2 = jobs[id];
            drop_event(j2);
            j2.t_done = Clock::now();
            in_use -= j2.footprint;
            --running;
            j2.task.reset();  // the result (if any) keeps the task's host tables
            if (code == FABX_OK) {
                j2.state = JobState::Done;
                j2.result = res;
                ++completed;
                latencies_ms.push_back(ms_between(j2.t_submit, j2.t_done));
                build_ms.push_back(ms_between(j2.t_submit, j2.t_queued));
                queue_ms.push_back(ms_between(j2.t_queued, j2.t_admit));
                run_ms.push_back(ms_between(j2.t_admit, j2.t_done));
            } else {
                j2.state = JobState::Failed;
                j2.code = code;
                j2.msg = msg;
                ++failed;
            }
            cv.notify_all();
        }
    }
};

}  // namespace fabx

struct fabx_server {
    std::unique_ptr<fabx::ServerImpl> p;
};

using namespace fabx;

namespace fabx {
template <typename F>
int guarded_server(F &&f) {
    try {
        f();
        set_last_error("");
        return FABX_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FABX_ENOMEM;
    }
}
}  // namespace fabx

extern "C" {

int fabx_server_create(fabx_ctx *ctx, int64_t budget, int32_t n_streams, fabx_server **out) {
    return guarded_server([&] {
        if (!ctx || !out) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        if (ctx->p->device < 0) fail(FABX_EINVAL, "server needs a device context");
        if (budget <= 0 || n_streams < 1 || n_streams > 16) fail(FABX_EINVAL, "bad budget or n_streams");
        auto s = std::make_unique<ServerImpl>();
        s->ctx = ctx->p;
        s->budget = budget;
        FABX_HIP(hipSetDevice(ctx->p->device));
        for (int i = 0; i < n_streams; ++i) {
            hipStream_t st;
            FABX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            s->streams.push_back(st);
        }
        ServerImpl *raw = s.get();
        for (int i = 0; i < n_streams; ++i) raw->workers.emplace_back([raw, i] { raw->worker(size_t(i)); });
        *out = new fabx_server{std::move(s)};
    });
}

void fabx_server_destroy(fabx_server *srv) {
    if (!srv) return;
    ServerImpl &s = *srv->p;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        s.stop = true;
    }
    s.cv.notify_all();
    for (auto &w : s.workers) w.join();
    for (auto st : s.streams) (void)hipStreamDestroy(st);
    delete srv;
}

int fabx_server_submit(fabx_server *srv, fabx_dataset *ds, int32_t on, const int32_t *by, int32_t n_by,
                       const int32_t *across, int32_t n_across, const fabx_score_opts *opts,
                       uint64_t *job_id) {
    return guarded_server([&] {
        const Clock::time_point t_entry = Clock::now();
        if (!srv || !ds || !job_id) fail(FABX_EINVAL, "null argument");
        ServerImpl &s = *srv->p;
        if (ds->p->ctx->device != s.ctx->device) fail(FABX_EINVAL, "dataset is on another device");
        Job job;
        job.t_submit = t_entry;
        job.params = resolve_opts(opts, *ds->p);
        job.task = build_task(ds->p, on, by, n_by, across, n_across);
        job.footprint = footprint_bytes(*job.task, job.params);
        if (job.footprint > s.budget)
            fail(FABX_ENOMEM, "job footprint " + std::to_string(job.footprint) +
                                  " bytes exceeds the server budget");
        prepack_tables(*job.task);
        FABX_HIP(hipSetDevice(s.ctx->device));
        job.ready = s.ctx->events.get();
        if (hipEventRecord(job.ready, s.ctx->stream) != hipSuccess) {
            (void)hipGetLastError();
            s.ctx->events.put(job.ready);
            fail(FABX_EHIP, "recording the submit event on the context's stream failed");
        }
        job.t_queued = Clock::now();
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.stop) {
            s.drop_event(job);
            fail(FABX_ECANCELED, "server is stopping");
        }
        const uint64_t id = s.next_id++;
        s.jobs.emplace(id, std::move(job));
        s.queue.push_back(id);
        ++s.submitted;
        *job_id = id;
        s.cv.notify_all();
    });
}

static int server_result(ServerImpl &s, uint64_t id, fabx_result **out, bool wait) {
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.jobs.find(id);
    if (it == s.jobs.end()) {
        set_last_error("unknown job id (or its result was already fetched)");
        return FABX_ENOTFOUND;
    }
    if (wait)
        s.cv.wait(lk, [&] {
            auto st = it->second.state;
            return st != JobState::Queued && st != JobState::Running;
        });
    Job &j = it->second;
    int rc = FABX_OK;
    switch (j.state) {
        case JobState::Queued:
        case JobState::Running:
            set_last_error("job not finished");
            return FABX_EAGAIN;
        case JobState::Cancelled:
            set_last_error("job was cancelled");
            rc = FABX_ECANCELED;
            break;
        case JobState::Failed:
            set_last_error(j.msg);
            rc = j.code;
            break;
        case JobState::Done:
            if (out) *out = new fabx_result{j.result};
            set_last_error("");
            break;
    }
    // the outcome has been handed over: the server keeps nothing of the job
    s.jobs.erase(it);
    return rc;
}

int fabx_server_poll(fabx_server *srv, uint64_t job_id, fabx_result **out) {
    if (!srv) return FABX_EINVAL;
    return server_result(*srv->p, job_id, out, false);
}

int fabx_server_wait(fabx_server *srv, uint64_t job_id, fabx_result **out) {
    if (!srv) return FABX_EINVAL;
    return server_result(*srv->p, job_id, out, true);
}

int fabx_server_cancel(fabx_server *srv, uint64_t job_id) {
    if (!srv) return FABX_EINVAL;
    ServerImpl &s = *srv->p;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.jobs.find(job_id);
    if (it == s.jobs.end()) {
        set_last_error("unknown job id");
        return FABX_ENOTFOUND;
    }
    if (it->second.state != JobState::Queued) {
        set_last_error("job already running or finished");
        return FABX_EAGAIN;
    }
    s.queue.erase(std::find(s.queue.begin(), s.queue.end(), job_id));
    it->second.state = JobState::Cancelled;
    s.drop_event(it->second);
    ++s.cancelled;
    s.cv.notify_all();
    return FABX_OK;
}

int fabx_server_stats_get(fabx_server *srv, fabx_server_stats *st) {
    if (!srv || !st) return FABX_EINVAL;
    ServerImpl &s = *srv->p;
    std::lock_guard<std::mutex> lk(s.mu);
    st->submitted = s.submitted;
    st->completed = s.completed;
    st->cancelled = s.cancelled;
    st->failed = s.failed;
    st->queued = int64_t(s.queue.size());
    st->running = s.running;
    st->hbm_in_use = s.in_use;
    st->hbm_high_water = s.high_water;
    std::vector<double> l = s.latencies_ms;
    std::sort(l.begin(), l.end());
    // nearest-rank percentile of a sorted vector
    auto pct = [](const std::vector<double> &v, double q) {
        if (v.empty()) return 0.0;
        const double r = std::max(1.0, std::ceil(q * double(v.size())));
        return v[size_t(std::min<double>(double(v.size()), r)) - 1];
    };
    st->p50_ms = pct(l, 0.50);
    st->p99_ms = pct(l, 0.99);
    std::vector<double> q = s.queue_ms;
    std::sort(q.begin(), q.end());
    st->p50_queue_ms = pct(q, 0.50);
    st->p99_queue_ms = pct(q, 0.99);
    auto mean = [](const std::vector<double> &v) {
        double a = 0.0;
        for (double x : v) a += x;
        return v.empty() ? 0.0 : a / double(v.size());
    };
    st->mean_build_ms = mean(s.build_ms);
    st->mean_queue_ms = mean(s.queue_ms);
    st->mean_run_ms = mean(s.run_ms);
    return FABX_OK;
}

}  // extern "C"
