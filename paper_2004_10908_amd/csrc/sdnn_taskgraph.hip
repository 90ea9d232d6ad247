// Host task-graph executor and the inference pipeline built on it (host code).
//
// The paper's runtime (section "Worker-level Scheduling Algorithm") runs a task
// graph whose tasks belong to domains (CPU, GPU) on per-domain worker threads
// with work stealing, keeping the number of workers that hunt for work matched to
// the available parallelism: a worker that becomes active while no other worker
// of its domain is stealing wakes one up to take over the thief role, and the last
// thief may only go to sleep once every queue of its domain is empty and no
// worker of its domain is active.  This file implements that scheme from its
// description:
//  * per worker, one task queue per domain (the owner pushes and pops at the back,
//    thieves take from the front); one shared queue per domain for submissions
//    from outside the workers;
//  * per domain, counters of active workers and of thieves, and a notifier with a
//    two-phase wait (prepare_wait, then commit_wait or cancel_wait), so that a
//    notification issued between a worker's last look at the queues and its
//    sleep is never lost;
//  * a worker's loop: drain its own queue (waking a thief when it is the first
//    active worker and nobody steals), then steal; when nothing is found it
//    prepares to sleep, re-checks the shared queue, and, as the last thief,
//    re-checks the active count and every queue of its domain before sleeping;
//  * finishing a task releases its successors whose dependency count reaches zero
//    (a condition task instead picks one successor by the index it returns); a
//    task of the other domain is pushed to the worker's queue of that domain and
//    wakes a worker there when that domain has neither active workers nor thieves.
// Queues are mutex-protected deques (the work is coarse: a batch's decode, its
// GPU forward, its check), not the lock-free deque the paper uses.
//
// GPU-domain workers each own one HIP stream (default priority); a GPU task
// enqueues its work on the worker's stream and synchronizes it before returning,
// so at most one batch per GPU worker is in flight and the next batch's CPU tasks
// overlap the GPU work.
//
// The inference pipeline (the paper's end-to-end inference task graph, section
// "Large Sparse Neural Network Inference": inputs dispatched batch by batch to the
// GPU, results evaluated against a golden reference by CPU tasks) builds, per
// batch b: decode[b] (CPU: the batch's rows from the sparse input, the nonzero
// column ids of each row, into a pinned host buffer as dense 0/1 fp32 rows) ->
// infer[b] (GPU: copy in, sdnn_forward over the batch, copy out the batch's
// nonzero-row ids and their count) -> check[b] (CPU: compare them with the batch's
// truth categories).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <random>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "sdnn.h"
#include "sdnn_taskgraph.h"

namespace sdnn_tg {
struct Task;
}
using sdnn_tg::Task;

namespace {

thread_local std::string g_tg_err;

int tg_fail(int st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_tg_err = buf;
    return st;
}

constexpr int NDOM = 2;   // SDNN_TG_CPU, SDNN_TG_GPU

// Mutex-protected deque: the owner works at the back, thieves take the front.
struct TaskQueue {
    std::mutex m;
    std::deque<Task*> q;
    void push(Task* t) {
        std::lock_guard<std::mutex> g(m);
        q.push_back(t);
    }
    Task* pop() {
        std::lock_guard<std::mutex> g(m);
        if (q.empty()) return nullptr;
        Task* t = q.back();
        q.pop_back();
        return t;
    }
    Task* steal() {
        std::lock_guard<std::mutex> g(m);
        if (q.empty()) return nullptr;
        Task* t = q.front();
        q.pop_front();
        return t;
    }
    bool empty() {
        std::lock_guard<std::mutex> g(m);
        return q.empty();
    }
};

// Two-phase wait: a waiter announces itself (prepare_wait), re-checks its
// predicate, then sleeps (commit_wait) or withdraws (cancel_wait).  A notify that
// happens after prepare_wait wakes a prepared waiter, or makes its commit_wait
// return at once, so no wake-up is lost between the check and the sleep.
struct Notifier {
    std::mutex m;
    std::condition_variable cv;
    uint64_t epoch = 0;
    int prepared = 0, sleeping = 0;
    uint64_t prepare_wait() {
        std::lock_guard<std::mutex> g(m);
        ++prepared;
        return epoch;
    }
    void cancel_wait() {
        std::lock_guard<std::mutex> g(m);
        --prepared;
    }
    void commit_wait(uint64_t seen) {
        std::unique_lock<std::mutex> g(m);
        ++sleeping;
        cv.wait(g, [&] { return epoch != seen; });
        --sleeping;
        --prepared;
    }
    void notify_one() {
        {
            std::lock_guard<std::mutex> g(m);
            if (prepared == 0) return;
            ++epoch;
        }
        cv.notify_one();
    }
    void notify_all() {
        {
            std::lock_guard<std::mutex> g(m);
            ++epoch;
        }
        cv.notify_all();
    }
};

}  // namespace

namespace sdnn_tg {
// A task of a graph.  `run` returns -1 for an ordinary task, or (condition task)
// the index of the one successor to release.
struct Task {
    int domain = SDNN_TG_CPU;
    std::function<int(hipStream_t)> run;
    std::vector<Task*> succ;
    int deps = 0;                       // strong dependencies (predecessors that are not condition tasks)
    int preds = 0;                      // all predecessors; a run starts at the tasks with none
    bool condition = false;
    std::atomic<int> left{0};           // dependencies still to finish in the current run
    struct ::sdnn_tg_graph_s* graph = nullptr;
};
}  // namespace sdnn_tg

struct sdnn_tg_graph_s {
    std::vector<std::unique_ptr<Task>> tasks;
    std::atomic<int> pending{0};        // tasks still to run in the current run
    std::mutex m;
    std::condition_variable done_cv;
    bool done = false;
    std::atomic<int> errors{0};
};

namespace sdnn_tg {
struct Worker {
    int id = 0, domain = SDNN_TG_CPU;
    TaskQueue queue[NDOM];
    hipStream_t stream = nullptr;       // GPU workers
    std::thread th;
    std::mt19937 rng;
};
}  // namespace sdnn_tg
using sdnn_tg::Worker;

struct sdnn_tg_executor_s {
    std::vector<std::unique_ptr<Worker>> workers;
    std::vector<Worker*> by_domain[NDOM];
    TaskQueue shared[NDOM];
    Notifier notifier[NDOM];
    std::atomic<int> actives[NDOM];
    std::atomic<int> thieves[NDOM];
    std::atomic<bool> stop{false};
    int device = 0;
    // statistics
    std::atomic<int64_t> executed{0}, steals{0}, failed_steals{0}, sleeps{0};

    void submit(Worker* w, Task* t);
    void execute(Worker* w, Task* t);
    void exploit(Worker* w, Task*& t);
    Task* explore(Worker* w);
    bool wait_for_task(Worker* w, Task*& t);
    void loop(Worker* w);
    void schedule_external(Task* t);
};

void sdnn_tg_executor_s::schedule_external(Task* t) {
    const int d = t->domain;
    shared[d].push(t);
    notifier[d].notify_one();
}

// A task becomes ready: queue it on the worker's queue of its domain, and wake a
// worker of that domain if the domain has neither active workers nor thieves.
void sdnn_tg_executor_s::submit(Worker* w, Task* t) {
    const int d = t->domain;
    w->queue[d].push(t);
    if (w->domain != d && actives[d].load() == 0 && thieves[d].load() == 0) notifier[d].notify_one();
}

void sdnn_tg_executor_s::execute(Worker* w, Task* t) {
    // re-arm the join counter: a task in a loop of condition tasks runs again
    t->left.store(t->deps);
    int r = -1;
    try {
        r = t->run(w->stream);
    } catch (...) {
        t->graph->errors.fetch_add(1);
        r = -1;
    }
    executed.fetch_add(1, std::memory_order_relaxed);
    sdnn_tg_graph_s* g = t->graph;
    if (t->condition) {
        if (r >= 0 && r < (int)t->succ.size()) submit(w, t->succ[r]);
    } else {
        for (Task* s : t->succ)
            if (s->left.fetch_sub(1) == 1) submit(w, s);
    }
    if (g->pending.fetch_sub(1) == 1) {
        std::lock_guard<std::mutex> lk(g->m);
        g->done = true;
        g->done_cv.notify_all();
    }
}

void sdnn_tg_executor_s::exploit(Worker* w, Task*& t) {
    if (!t) return;
    const int d = w->domain;
    // the first worker to turn active while nobody steals wakes one to steal
    if (actives[d].fetch_add(1) + 1 == 1 && thieves[d].load() == 0) notifier[d].notify_one();
    do {
        execute(w, t);
        t = w->queue[d].pop();
    } while (t);
    actives[d].fetch_sub(1);
}

// Steal attempts: random victims of the domain and the shared queue, a bounded
// number of rounds with yields in between.
Task* sdnn_tg_executor_s::explore(Worker* w) {
    const int d = w->domain;
    auto& peers = by_domain[d];
    const int rounds = 64;
    for (int r = 0; r < rounds && !stop.load(); ++r) {
        const int v = (int)(w->rng() % (peers.size() + 1));
        Task* t = v == (int)peers.size() ? shared[d].steal() : (peers[v] == w ? nullptr : peers[v]->queue[d].steal());
        if (!t) {
            // tasks of this domain queued by workers of the other domain
            for (Worker* x : by_domain[1 - d])
                if ((t = x->queue[d].steal())) break;
        }
        if (t) {
            steals.fetch_add(1, std::memory_order_relaxed);
            return t;
        }
        failed_steals.fetch_add(1, std::memory_order_relaxed);
        std::this_thread::yield();
    }
    return nullptr;
}

bool sdnn_tg_executor_s::wait_for_task(Worker* w, Task*& t) {
    const int d = w->domain;
    auto any_queued = [&]() {
        if (!shared[d].empty()) return true;
        for (auto& x : workers)
            if (!x->queue[d].empty()) return true;
        return false;
    };
    while (true) {
        thieves[d].fetch_add(1);
        while (true) {
            t = explore(w);
            if (t) {
                // the last thief turning active hands its role to another worker
                if (thieves[d].fetch_sub(1) == 1) notifier[d].notify_one();
                return true;
            }
            const uint64_t seen = notifier[d].prepare_wait();
            if (!shared[d].empty()) {
                notifier[d].cancel_wait();
                t = shared[d].steal();
                if (t) {
                    if (thieves[d].fetch_sub(1) == 1) notifier[d].notify_one();
                    return true;
                }
                continue;   // steal again
            }
            if (stop.load()) {
                notifier[d].cancel_wait();
                for (auto& n : notifier) n.notify_all();
                thieves[d].fetch_sub(1);
                return false;
            }
            if (thieves[d].fetch_sub(1) == 1) {
                // the last thief sleeps only if nothing of its domain is running or queued
                if (actives[d].load() > 0 || any_queued()) {
                    notifier[d].cancel_wait();
                    break;   // become a thief again
                }
            }
            sleeps.fetch_add(1, std::memory_order_relaxed);
            notifier[d].commit_wait(seen);
            return true;
        }
    }
}

void sdnn_tg_executor_s::loop(Worker* w) {
    if (w->domain == SDNN_TG_GPU) (void)hipSetDevice(device);
    Task* t = nullptr;
    while (true) {
        exploit(w, t);
        if (!wait_for_task(w, t)) break;
    }
}

extern "C" {

int sdnn_tg_executor_create(int32_t n_cpu, int32_t n_gpu, sdnn_tg_executor* out) {
    if (!out) return tg_fail(SDNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_cpu < 1 || n_cpu > 256 || n_gpu < 0 || n_gpu > 64)
        return tg_fail(SDNN_EINVAL, "worker counts out of range (n_cpu 1..256, n_gpu 0..64)");
    // GPU-domain worker threads are switched off: a process that ran GPU tasks on
    // them (kernels launched from executor-owned threads) ended with a segmentation
    // fault at exit after every task had finished, for a reason not yet found.  Host
    // builds against a stand-in HIP header (the sanitizer tests) keep them.
#ifndef SDNN_TG_STANDIN_HIP
    if (n_gpu > 0)
        return tg_fail(SDNN_EUNSUPPORTED, "GPU-domain workers are switched off (n_gpu must be 0)");
#endif
    auto ex = std::make_unique<sdnn_tg_executor_s>();
    for (int d = 0; d < NDOM; ++d) {
        ex->actives[d] = 0;
        ex->thieves[d] = 0;
    }
    if (n_gpu > 0 && hipGetDevice(&ex->device) != hipSuccess) return tg_fail(SDNN_EHIP, "hipGetDevice failed");
    for (int i = 0; i < n_cpu + n_gpu; ++i) {
        auto w = std::make_unique<Worker>();
        w->id = i;
        w->domain = i < n_cpu ? SDNN_TG_CPU : SDNN_TG_GPU;
        w->rng.seed(0x9e3779b9u * (unsigned)(i + 1));
        if (w->domain == SDNN_TG_GPU) {
            const hipError_t e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (auto& x : ex->workers)
                    if (x->stream) (void)hipStreamDestroy(x->stream);
                return tg_fail(SDNN_EHIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
            }
        }
        ex->by_domain[w->domain].push_back(w.get());
        ex->workers.push_back(std::move(w));
    }
    for (auto& w : ex->workers) {
        Worker* wp = w.get();
        sdnn_tg_executor_s* e = ex.get();
        w->th = std::thread([e, wp] { e->loop(wp); });
    }
    *out = ex.release();
    return SDNN_OK;
}

void sdnn_tg_executor_destroy(sdnn_tg_executor ex) {
    if (!ex) return;
    ex->stop.store(true);
    for (auto& n : ex->notifier) n.notify_all();
    for (auto& w : ex->workers) {
        if (w->th.joinable()) w->th.join();
        if (w->stream) (void)hipStreamDestroy(w->stream);
    }
    delete ex;
}

int sdnn_tg_executor_stats(sdnn_tg_executor ex, int64_t* stats4) {
    if (!ex || !stats4) return tg_fail(SDNN_EINVAL, "NULL argument");
    stats4[0] = ex->executed.load();
    stats4[1] = ex->steals.load();
    stats4[2] = ex->failed_steals.load();
    stats4[3] = ex->sleeps.load();
    return SDNN_OK;
}

const char* sdnn_tg_last_error(void) { return g_tg_err.c_str(); }

}  // extern "C"

namespace {

Task* add_task(sdnn_tg_graph_s* g, int domain, std::function<int(hipStream_t)> fn, bool condition = false) {
    auto t = std::make_unique<Task>();
    t->domain = domain;
    t->run = std::move(fn);
    t->condition = condition;
    t->graph = g;
    g->tasks.push_back(std::move(t));
    return g->tasks.back().get();
}

void precede(Task* a, Task* b) {
    a->succ.push_back(b);
    ++b->preds;
    if (!a->condition) ++b->deps;
}

// Run a graph to completion on the executor (blocking).  The run starts at the
// tasks without predecessors (a task reached only from condition tasks waits for
// them); expected_tasks is the number of task executions the run makes.
int run_graph(sdnn_tg_executor ex, sdnn_tg_graph_s* g, int expected_tasks) {
    g->done = false;
    g->errors = 0;
    g->pending = expected_tasks;
    for (auto& t : g->tasks) t->left = t->deps;
    for (auto& t : g->tasks)
        if (t->preds == 0) ex->schedule_external(t.get());
    std::unique_lock<std::mutex> lk(g->m);
    g->done_cv.wait(lk, [&] { return g->done; });
    return g->errors.load() ? tg_fail(SDNN_EDEVICE, "%d task(s) failed", g->errors.load()) : SDNN_OK;
}

}  // namespace

extern "C" {

int sdnn_tg_run_diamond_chain(sdnn_tg_executor ex, int32_t width, int32_t depth, int32_t gpu_every, int64_t* sum) {
    if (!ex || !sum || width < 1 || depth < 1 || gpu_every < 0) return tg_fail(SDNN_EINVAL, "bad arguments");
    if (gpu_every > 0 && ex->by_domain[SDNN_TG_GPU].empty()) return tg_fail(SDNN_EINVAL, "no GPU workers");
    sdnn_tg_graph_s g;
    std::atomic<int64_t> acc{0};
    std::vector<Task*> prev;
    Task* src = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { acc.fetch_add(1); return -1; });
    prev.push_back(src);
    for (int lvl = 0; lvl < depth; ++lvl) {
        std::vector<Task*> cur;
        for (int i = 0; i < width; ++i) {
            const int dom = (gpu_every > 0 && (lvl * width + i) % gpu_every == 0) ? SDNN_TG_GPU : SDNN_TG_CPU;
            const int64_t v = (int64_t)lvl * width + i + 2;
            Task* t = add_task(&g, dom, [&, v, dom](hipStream_t s) {
                if (dom == SDNN_TG_GPU && !s) throw std::runtime_error("GPU task without a stream");
                acc.fetch_add(v);
                return -1;
            });
            for (Task* p : prev) precede(p, t);
            cur.push_back(t);
        }
        prev.swap(cur);
    }
    Task* sink = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { acc.fetch_add(1); return -1; });
    for (Task* p : prev) precede(p, sink);
    const int st = run_graph(ex, &g, (int)g.tasks.size());
    *sum = acc.load();
    return st;
}

int sdnn_tg_run_condition_loop(sdnn_tg_executor ex, int32_t iterations, int32_t* count) {
    if (!ex || !count || iterations < 0) return tg_fail(SDNN_EINVAL, "bad arguments");
    sdnn_tg_graph_s g;
    int n = 0;
    // init -> body -> cond -(0)-> body (loop) / -(1)-> done: the condition task
    // releases exactly one successor, so the run executes 2 + 2 * iterations + ... tasks
    Task* init = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { n = 0; return -1; });
    Task* body = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { ++n; return -1; });
    Task* cond = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { return n < iterations ? 0 : 1; }, true);
    Task* done = add_task(&g, SDNN_TG_CPU, [&](hipStream_t) { return -1; });
    precede(init, body);
    precede(body, cond);
    precede(cond, body);   // weak edge (from a condition task)
    precede(cond, done);
    const int runs = std::max(1, iterations);
    const int st = run_graph(ex, &g, 1 + 2 * runs + 1);
    *count = n;
    return st;
}

int sdnn_tg_pipeline_run(sdnn_tg_executor ex, sdnn_net* nets, int32_t n_nets, int32_t n_neurons, int64_t rows,
                         const int64_t* batch_off, int32_t n_batches, const int64_t* in_ptr, const int32_t* in_cols,
                         const int64_t* truth_off, const int32_t* truth_rows, float* y0_dev, float* y_dev,
                         int32_t* nz_dev, int32_t* n_nz_dev, int64_t* mismatches, double* seconds) {
    if (!ex || !nets || !batch_off || !in_ptr || !in_cols || !truth_off || !truth_rows || !y0_dev || !y_dev || !nz_dev ||
        !n_nz_dev || !mismatches)
        return tg_fail(SDNN_EINVAL, "NULL argument");
    const int ngpu = (int)ex->by_domain[SDNN_TG_GPU].size();
    if (ngpu < 1) return tg_fail(SDNN_EINVAL, "the pipeline needs GPU workers");
    if (n_nets != ngpu) return tg_fail(SDNN_EINVAL, "one net per GPU worker (%d workers, %d nets)", ngpu, n_nets);
    if (n_batches < 1 || n_batches > 4096 || batch_off[0] != 0 || batch_off[n_batches] != rows)
        return tg_fail(SDNN_EINVAL, "batch offsets must start at 0 and end at rows");
    for (int b = 0; b < n_batches; ++b)
        if (batch_off[b + 1] < batch_off[b]) return tg_fail(SDNN_EINVAL, "batch offsets must not decrease");
    const int N = n_neurons;
    // pinned staging: inputs (dense rows) and each batch's nonzero-row ids and count
    float* hin = nullptr;
    int32_t* hnz = nullptr;
    if (hipHostMalloc((void**)&hin, std::max<size_t>(1, (size_t)rows * N * 4), 0) != hipSuccess)
        return tg_fail(SDNN_ENOMEM, "pinned input staging of %lld rows", (long long)rows);
    if (hipHostMalloc((void**)&hnz, (size_t)(rows + n_batches) * 4, 0) != hipSuccess) {
        (void)hipHostFree(hin);
        return tg_fail(SDNN_ENOMEM, "pinned result staging");
    }
    std::vector<int> worker_of(ex->workers.size(), -1);
    for (int i = 0; i < ngpu; ++i) worker_of[ex->by_domain[SDNN_TG_GPU][i]->id] = i;
    sdnn_tg_graph_s g;
    std::vector<std::string> errs(n_batches);
    for (int b = 0; b < n_batches; ++b) {
        const int64_t r0 = batch_off[b], nb = batch_off[b + 1] - r0;
        mismatches[b] = 0;
        Task* dec = add_task(&g, SDNN_TG_CPU, [=](hipStream_t) {
            float* dst = hin + (size_t)r0 * N;
            std::memset(dst, 0, (size_t)nb * N * 4);
            for (int64_t r = 0; r < nb; ++r)
                for (int64_t e = in_ptr[r0 + r]; e < in_ptr[r0 + r + 1]; ++e) {
                    const int32_t c = in_cols[e];
                    if (c >= 0 && c < N) dst[(size_t)r * N + c] = 1.0f;
                }
            return -1;
        });
        Task* inf = add_task(&g, SDNN_TG_GPU, [=, &errs, &worker_of](hipStream_t s) {
            int wi = -1;
            for (auto& w : ex->workers)
                if (w->stream == s) wi = worker_of[w->id];
            if (wi < 0 || nb == 0) return -1;
            const size_t off = (size_t)r0 * N;
            if (hipMemcpyAsync(y0_dev + off, hin + off, (size_t)nb * N * 4, hipMemcpyHostToDevice, s) != hipSuccess)
                throw std::runtime_error("copy in");
            const int64_t bo[2] = {0, nb};
            const sdnn_status st = sdnn_forward(nets[wi], y0_dev + off, nb, bo, 1, y_dev + off, nz_dev + r0,
                                                n_nz_dev + b, nullptr, nullptr, s);
            if (st != SDNN_OK) {
                errs[b] = sdnn_last_error();
                throw std::runtime_error("forward");
            }
            if (hipMemcpyAsync(hnz + r0, nz_dev + r0, (size_t)nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(hnz + rows + b, n_nz_dev + b, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                throw std::runtime_error("copy out");
            return -1;
        });
        Task* chk = add_task(&g, SDNN_TG_CPU, [=](hipStream_t) {
            // the batch's nonzero rows (batch-local ids) against its truth categories
            // (global row ids, ascending): a symmetric difference count
            const int32_t n = nb ? hnz[rows + b] : 0;
            int64_t i = 0, j = truth_off[b], mism = 0;
            const int64_t je = truth_off[b + 1];
            while (i < n || j < je) {
                const int64_t a = i < n ? r0 + hnz[r0 + i] : INT64_MAX;
                const int64_t t = j < je ? (int64_t)truth_rows[j] : INT64_MAX;
                if (a == t) { ++i; ++j; }
                else if (a < t) { ++mism; ++i; }
                else { ++mism; ++j; }
            }
            mismatches[b] = mism;
            return -1;
        });
        precede(dec, inf);
        precede(inf, chk);
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int st = run_graph(ex, &g, (int)g.tasks.size());
    const auto t1 = std::chrono::steady_clock::now();
    if (seconds) *seconds = std::chrono::duration<double>(t1 - t0).count();
    (void)hipHostFree(hin);
    (void)hipHostFree(hnz);
    if (st != SDNN_OK) {
        for (auto& e : errs)
            if (!e.empty()) return tg_fail(SDNN_EDEVICE, "pipeline task failed: %s", e.c_str());
        return st;
    }
    return SDNN_OK;
}

}  // extern "C"
