// Continuous-batching solve server.  Several operators (BF + ULV factors) stay
// resident; requests (a block of right-hand sides for one operator) arrive at
// any time and are queued.  A dispatcher forms a batch whenever a stream slot
// is free: it takes the oldest waiting request and adds later requests for the
// same operator in arrival order while the batch's memory (batch input and
// output blocks plus the solve workspace for its width) fits the slot's arena,
// gathers their columns into the arena, runs one fio_approx_solve on the batch
// (optionally replayed from a captured hipGraph) and scatters the solutions
// back.  Batches on different slots overlap on the device.
//
// Memory: each slot owns one device arena, shared by all operators (a slot runs
// one batch at a time), allocated when serving starts: mem_budget / streams
// bytes, or, with no budget, the largest batch of any operator.  A batch of
// width w for operator op lays out U at offset 0, F next, the workspace last, so
// the addresses depend only on (slot, op, w) and captured graphs stay valid.
// The widest batch an operator can take is the widest that fits the arena:
// that is the memory-based admission, and the device memory the server holds
// never exceeds the budget.  Every column of a batch is solved independently
// by the kernels, so with a fixed refinement step count a request's result does
// not depend on the batch it travels in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <tuple>

#include "bf.h"

struct hss_ulv_s;

namespace fio {
size_t ulv_ws_bytes_pub(const hss_ulv_s *f, int nrhs);
}

namespace {

using clk = std::chrono::steady_clock;

struct Operator {
    fio_bf_t bf;
    hss_ulv_t ulv;
    fio_solve_opts opts;
    long n;
    int max_width;       // widest batch that fits a slot's arena (set when serving starts)
};

struct Request {
    long long id;
    int op;
    const double2 *U;
    long ldu;
    double2 *F;
    long ldf;
    int nrhs;
    double t_submit = 0, t_start = 0, t_done = 0;
    int batch = -1;
    int status = 1;      // 1 pending, 0 done, < 0 error
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    fio::DevBuf *arena = nullptr;              // U, F and workspace of the running batch
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (op, nrhs) -> captured solve
    bool busy = false;
    std::vector<long long> reqs;
    size_t bytes = 0;
    int batch_id = -1;
    int op = -1;
    int nrhs = 0;
};

}  // namespace

struct fio_server_s {
    int max_batch = 64;
    int bucket = 1;                   // batch widths are rounded up to a multiple of this
    size_t budget = 0;
    size_t slot_bytes = 0;            // arena bytes per slot
    bool graphs = false;
    clk::time_point t0;
    std::vector<Operator> ops;
    std::vector<Slot> slots;
    std::map<long long, Request> reqs;
    std::deque<long long> queue;
    std::mutex mu;
    std::condition_variable cv;       // dispatcher wake-up
    std::condition_variable cv_done;  // waiters
    std::thread dispatcher;
    std::vector<std::thread> completers;
    std::vector<std::deque<int>> slot_batches;   // per slot: a launched batch awaiting completion
    std::vector<std::unique_ptr<std::condition_variable>> slot_cv;
    bool stop = false;
    bool started = false;
    long long next_id = 1;
    int next_batch = 0;
    size_t in_flight = 0, peak_bytes = 0;
    long completed = 0, batches = 0;
    size_t max_queue = 0;
    int error = 0;

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
};

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// arena layout of a batch of `nrhs` columns: U at 0, F at f_off, workspace at ws_off
struct Layout {
    size_t f_off, ws_off, ws, total;
};

Layout layout(const Operator &op, int nrhs) {
    Layout l;
    const size_t blk = align256((size_t)op.n * nrhs * sizeof(double2));
    l.ws = 0;
    fio_solve_workspace_size(op.bf, op.ulv, nrhs, &op.opts, &l.ws);
    l.f_off = blk;
    l.ws_off = 2 * blk;
    l.total = 2 * blk + align256(l.ws);
    return l;
}

size_t batch_bytes(const Operator &op, int nrhs) { return layout(op, nrhs).total; }

double2 *u_of(Slot &s) { return s.arena->as<double2>(); }
double2 *f_of(Slot &s, const Operator &o, int nrhs) {
    return reinterpret_cast<double2 *>(static_cast<char *>(s.arena->p) + layout(o, nrhs).f_off);
}

// Runs (or replays) the batched solve of `s` on its stream.
fio_status run_solve(fio_server_s *S, Slot &s, int op, int nrhs, bool capture_only = false) {
    Operator &o = S->ops[op];
    const Layout l = layout(o, nrhs);
    char *base = static_cast<char *>(s.arena->p);
    auto call = [&]() {
        return fio_approx_solve(o.bf, o.ulv, base, o.n, base + l.f_off, o.n, nrhs, &o.opts, nullptr,
                                base + l.ws_off, l.ws, s.stream);
    };
    if (!S->graphs) return call();
    auto key = std::make_pair(op, nrhs);
    auto it = s.graphs.find(key);
    if (it == s.graphs.end()) {
        hipGraph_t g;
        if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return FIO_ERR_HIP;
        fio_status st = call();
        if (hipStreamEndCapture(s.stream, &g) != hipSuccess || st != FIO_OK) return st != FIO_OK ? st : FIO_ERR_HIP;
        hipGraphExec_t ge;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return FIO_ERR_HIP;
        }
        (void)hipGraphDestroy(g);
        it = s.graphs.emplace(key, ge).first;
    }
    if (capture_only) return FIO_OK;
    return hipGraphLaunch(it->second, s.stream) == hipSuccess ? FIO_OK : FIO_ERR_HIP;
}

void dispatcher_loop(fio_server_s *S) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv.wait(lk, [&] {
            if (S->stop) return true;
            if (S->queue.empty()) return false;
            for (auto &s : S->slots)
                if (!s.busy) return true;
            return false;
        });
        if (S->stop) return;
        int si = -1;
        for (size_t i = 0; i < S->slots.size(); ++i)
            if (!S->slots[i].busy) {
                si = (int)i;
                break;
            }
        // batch: the oldest request and later ones for the same operator
        const long long head = S->queue.front();
        const int op = S->reqs[head].op;
        std::vector<long long> take;
        int cols = 0;
        // memory-based admission: the batch (rounded up to the width bucket) must fit the slot's
        // arena, i.e. at most max_width columns; submit() rejects requests wider than that
        const int wmax = S->ops[op].max_width;
        for (long long id : S->queue) {
            Request &r = S->reqs[id];
            if (r.op != op) continue;
            const int w = ((cols + r.nrhs + S->bucket - 1) / S->bucket) * S->bucket;
            if (w > wmax) continue;
            take.push_back(id);
            cols += r.nrhs;
        }
        for (long long id : take)
            for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
                if (*it == id) {
                    S->queue.erase(it);
                    break;
                }
        Slot &s = S->slots[si];
        const int width = ((cols + S->bucket - 1) / S->bucket) * S->bucket;
        s.busy = true;
        s.reqs = take;
        s.op = op;
        s.nrhs = width;
        s.bytes = batch_bytes(S->ops[op], width);
        s.batch_id = S->next_batch++;
        S->in_flight += s.bytes;
        S->peak_bytes = S->in_flight > S->peak_bytes ? S->in_flight : S->peak_bytes;
        S->batches++;
        const double ts = S->now();
        // launch outside the lock (stream work only)
        std::vector<Request> local;
        for (long long id : take) {
            Request &r = S->reqs[id];
            r.t_start = ts;
            r.batch = s.batch_id;
            local.push_back(r);
        }
        lk.unlock();
        const long n = S->ops[op].n;
        fio_status st = FIO_OK;
        int c = 0;
        double2 *Ub = u_of(s), *Fb = f_of(s, S->ops[op], width);
        for (auto &r : local) {
            if (hipMemcpy2DAsync(Ub + (size_t)c * n, n * sizeof(double2), r.U,
                                 r.ldu * sizeof(double2), n * sizeof(double2), r.nrhs, hipMemcpyDeviceToDevice,
                                 s.stream) != hipSuccess)
                st = FIO_ERR_HIP;
            c += r.nrhs;
        }
        if (st == FIO_OK && width > cols &&
            hipMemsetAsync(Ub + (size_t)cols * n, 0, (size_t)(width - cols) * n * sizeof(double2),
                           s.stream) != hipSuccess)
            st = FIO_ERR_HIP;
        if (st == FIO_OK) st = run_solve(S, s, op, width);
        c = 0;
        for (auto &r : local) {
            if (st == FIO_OK &&
                hipMemcpy2DAsync(r.F, r.ldf * sizeof(double2), Fb + (size_t)c * n,
                                 n * sizeof(double2), n * sizeof(double2), r.nrhs, hipMemcpyDeviceToDevice,
                                 s.stream) != hipSuccess)
                st = FIO_ERR_HIP;
            c += r.nrhs;
        }
        if (st == FIO_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = FIO_ERR_HIP;
        lk.lock();
        if (st != FIO_OK) S->error = st;
        S->slot_batches[si].push_back(st == FIO_OK ? 0 : (int)st);
        S->slot_cv[si]->notify_one();
    }
}

void completer_loop(fio_server_s *S, int si) {
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->slot_cv[si]->wait(lk, [&] { return S->stop || !S->slot_batches[si].empty(); });
        if (S->slot_batches[si].empty() && S->stop) return;
        const int st = S->slot_batches[si].front();
        S->slot_batches[si].pop_front();
        Slot &s = S->slots[si];
        lk.unlock();
        hipError_t e = st == 0 ? hipEventSynchronize(s.done) : hipSuccess;
        const double td = S->now();
        lk.lock();
        for (long long id : s.reqs) {
            Request &r = S->reqs[id];
            r.t_done = td;
            r.status = (st == 0 && e == hipSuccess) ? 0 : (st != 0 ? st : FIO_ERR_HIP);
            S->completed++;
        }
        s.reqs.clear();
        S->in_flight -= s.bytes;
        s.busy = false;
        S->cv.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace

using namespace fio;

extern "C" fio_status fio_server_create(const fio_server_opts *o, fio_server_t *out) {
    FIO_CHECK_ARG(o && out && o->max_batch_rhs >= 1 && o->streams >= 1 && o->streams <= 8);
    FIO_CHECK_ARG(o->width_bucket >= 0 && (o->width_bucket <= 1 || o->max_batch_rhs % o->width_bucket == 0));
    fio_server_s *S = new fio_server_s();
    S->max_batch = o->max_batch_rhs;
    S->bucket = o->width_bucket > 1 ? o->width_bucket : 1;
    S->budget = o->mem_budget;
    S->graphs = o->use_graphs != 0;
    S->t0 = clk::now();
    S->slots.resize(o->streams);
    for (auto &s : S->slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
            delete S;
            return FIO_ERR_HIP;
        }
    }
    *out = S;
    return FIO_OK;
}

extern "C" fio_status fio_server_add_operator(fio_server_t S, fio_bf_t bf, hss_ulv_t ulv, const fio_solve_opts *opts,
                                              int *op_id) {
    FIO_CHECK_ARG(S && bf && ulv && opts && op_id && !S->started);
    FIO_CHECK_ARG(opts->mode == FIO_SOLVE_DIRECT || (opts->mode == FIO_SOLVE_IR && opts->rel_res_tol <= 0.0));
    Operator o{bf, ulv, *opts, bf->N, 0};
    size_t ws = 0;
    fio_status st = fio_solve_workspace_size(bf, ulv, S->max_batch, opts, &ws);
    if (st != FIO_OK) return st;
    *op_id = (int)S->ops.size();
    S->ops.push_back(o);
    return FIO_OK;
}

// Sizes and allocates the slot arenas and fixes each operator's widest batch (once, at the
// first submission).  Returns FIO_ERR_ARG when the budget cannot hold a one-column batch of
// some operator.
static fio_status start(fio_server_s *S) {
    if (S->started) return FIO_OK;
    if (S->ops.empty()) return FIO_ERR_ARG;
    const int step = S->bucket;
    size_t widest = 0;
    for (auto &o : S->ops) widest = std::max(widest, batch_bytes(o, S->max_batch));
    S->slot_bytes = S->budget ? S->budget / S->slots.size() : widest;
    for (auto &o : S->ops) {
        o.max_width = 0;
        for (int w = step; w <= S->max_batch; w += step)
            if (batch_bytes(o, w) <= S->slot_bytes) o.max_width = w;
        if (o.max_width == 0) return FIO_ERR_ARG;
    }
    fio_status st = guarded([&] {
        for (auto &s : S->slots) s.arena = new DevBuf(S->slot_bytes);
        return FIO_OK;
    });
    if (st != FIO_OK) return st;
    S->started = true;
    if (S->graphs && S->bucket > 1) {
        // capture every (slot, operator, bucketed width) up front: nothing is captured while serving
        for (auto &s : S->slots)
            for (int op = 0; op < (int)S->ops.size(); ++op)
                for (int w = step; w <= S->ops[op].max_width; w += step)
                    if (run_solve(S, s, op, w, true) != FIO_OK) S->error = FIO_ERR_HIP;
    }
    S->slot_batches.assign(S->slots.size(), {});
    for (size_t i = 0; i < S->slots.size(); ++i) S->slot_cv.emplace_back(new std::condition_variable());
    S->dispatcher = std::thread(dispatcher_loop, S);
    for (size_t i = 0; i < S->slots.size(); ++i) S->completers.emplace_back(completer_loop, S, (int)i);
    return FIO_OK;
}

extern "C" fio_status fio_server_submit(fio_server_t S, int op, const void *U, long ldu, void *F, long ldf, int nrhs,
                                        long long *req_id) {
    FIO_CHECK_ARG(S && U && F && req_id && op >= 0 && op < (int)S->ops.size());
    FIO_CHECK_ARG(nrhs >= 1 && nrhs <= S->max_batch && ldu >= S->ops[op].n && ldf >= S->ops[op].n);
    std::lock_guard<std::mutex> lk(S->mu);
    const fio_status st = start(S);
    if (st != FIO_OK) return st;
    // a request wider than the widest batch that fits a slot's share of the budget
    FIO_CHECK_ARG(((nrhs + S->bucket - 1) / S->bucket) * S->bucket <= S->ops[op].max_width);
    Request r;
    r.id = S->next_id++;
    r.op = op;
    r.U = (const double2 *)U;
    r.ldu = ldu;
    r.F = (double2 *)F;
    r.ldf = ldf;
    r.nrhs = nrhs;
    r.t_submit = S->now();
    S->reqs[r.id] = r;
    S->queue.push_back(r.id);
    S->max_queue = S->queue.size() > S->max_queue ? S->queue.size() : S->max_queue;
    *req_id = r.id;
    S->cv.notify_all();
    return FIO_OK;
}

extern "C" fio_status fio_server_wait_all(fio_server_t S) {
    FIO_CHECK_ARG(S);
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] {
        if (!S->queue.empty()) return false;
        for (auto &s : S->slots)
            if (s.busy) return false;
        return true;
    });
    return S->error ? (fio_status)S->error : FIO_OK;
}

extern "C" fio_status fio_server_request_info(fio_server_t S, long long id, double *t_submit, double *t_start,
                                              double *t_done, int *batch, int *status) {
    FIO_CHECK_ARG(S);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return FIO_ERR_ARG;
    const Request &r = it->second;
    if (t_submit) *t_submit = r.t_submit;
    if (t_start) *t_start = r.t_start;
    if (t_done) *t_done = r.t_done;
    if (batch) *batch = r.batch;
    if (status) *status = r.status;
    return FIO_OK;
}

extern "C" fio_status fio_server_stats(fio_server_t S, long *completed, long *batches, long *max_queue,
                                       size_t *peak_bytes) {
    FIO_CHECK_ARG(S);
    std::lock_guard<std::mutex> lk(S->mu);
    if (completed) *completed = S->completed;
    if (batches) *batches = S->batches;
    if (max_queue) *max_queue = (long)S->max_queue;
    if (peak_bytes) *peak_bytes = S->peak_bytes;
    return FIO_OK;
}

extern "C" double fio_server_now(fio_server_t S) { return S ? S->now() : 0.0; }

extern "C" void fio_server_destroy(fio_server_t S) {
    if (!S) return;
    if (S->started) {
        fio_server_wait_all(S);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
            for (auto &c : S->slot_cv) c->notify_all();
        }
        S->dispatcher.join();
        for (auto &t : S->completers) t.join();
    }
    for (auto &s : S->slots) {
        for (auto &kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
        delete s.arena;
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    delete S;
}
