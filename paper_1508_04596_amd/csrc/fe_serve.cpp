// Continuous-batching solve server.
//
// Two modes.  Default: each running request's whole Newton solve runs on its
// worker's stream.  Batched (FE_SERVE_BATCHED): the workers run set-up and line
// searches, and hand every linear solve to a lockstep engine (fe_batch.cpp)
// whose FGMRES steps launch each kernel once over all its running requests.
// There is one engine per size class of the grids (by DOF count, each class
// three times the last), each with its own thread and stream: requests batch
// with requests of similar size, a small request never waits for the steps of
// a large one, and the classes' steps overlap on the device.
//
// One device arena of hbm_budget_bytes is allocated at creation.  An admitted
// request takes one contiguous block of the arena, sized by its predicted
// footprint, and its whole working set (problem handle, solver workspace,
// multigrid hierarchy, design, source and state) is carved from that block in
// order, so admission is decided by memory footprint, requests cannot fragment
// each other's memory, and no device allocation or free (and no implicit device
// synchronisation) happens while requests run.  max_active worker threads, each
// with its own HIP stream, take requests from the queue in arrival order as
// soon as the arena has a free block for them; a request therefore starts
// while others are still on the GPU, and the kernels of all running requests
// overlap on the device.  When the head request does not fit the largest free
// block, the first later request that fits is admitted instead, until the head
// has been passed over max_active times; then admission waits for the head, so
// a large request is delayed by at most that many smaller ones.  A finished request returns its block and
// wakes the admission of the next.  Each request runs the same deterministic
// kernels as a standalone newton_solve, so its result does not depend on what
// else is running.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fe_internal.h"

using namespace fe;

namespace {

// First-fit free list over [0, size) with coalescing of neighbouring free ranges.
class FreeList {
  public:
    void reset(size_t size)
    {
        std::lock_guard<std::mutex> lk(mu_);
        free_.clear();
        used_.clear();
        if (size) free_[0] = size;
    }
    // offset of a range of n bytes (n a multiple of 256), or false if none is free
    bool take(size_t n, size_t *off)
    {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[o + n] = sz - n;
            used_[o] = n;
            *off = o;
            return true;
        }
        return false;
    }
    void give(size_t off)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, n = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + n) {
            n += next->second;
            free_.erase(next);
        }
        auto it = free_.lower_bound(start);
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == start) {
                start = prev->first;
                n += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = n;
    }
    size_t largest()
    {
        std::lock_guard<std::mutex> lk(mu_);
        size_t m = 0;
        for (const auto &f : free_) m = std::max(m, f.second);
        return m;
    }

  private:
    std::mutex mu_;
    std::map<size_t, size_t> free_;            // offset -> size of free ranges
    std::unordered_map<size_t, size_t> used_;  // offset -> size of live ranges
};

// Pinned host memory for the requests' host staging (Krylov scalars, coarse
// factorisation buffers): copies to and from it are direct DMA, where pageable
// memory goes through the runtime's staging copy.  Allocated once; a request
// whose staging does not fit takes pageable memory instead.
class HostPool {
  public:
    hipError_t init(size_t bytes)
    {
        size_ = bytes / 256 * 256;
        if (!size_) return hipSuccess;
        hipError_t e = hipHostMalloc(&base_, size_);
        if (e != hipSuccess) {
            base_ = nullptr;
            size_ = 0;
        }
        fl_.reset(size_);
        return e;
    }
    ~HostPool()
    {
        if (base_) (void)hipHostFree(base_);
    }
    void *alloc(size_t n)
    {
        n = std::max<size_t>(256, (n + 255) / 256 * 256);
        size_t off = 0;
        if (!base_ || !fl_.take(n, &off)) return nullptr;
        return static_cast<char *>(base_) + off;
    }
    bool owns(const void *p) const
    {
        const char *c = static_cast<const char *>(p), *b = static_cast<const char *>(base_);
        return base_ && c >= b && c < b + size_;
    }
    void release(void *p) { fl_.give(static_cast<char *>(p) - static_cast<char *>(base_)); }

  private:
    void *base_ = nullptr;
    size_t size_ = 0;
    FreeList fl_;
};

class Arena final : public Allocator {
  public:
    hipError_t init(size_t bytes)
    {
        size_ = bytes / 256 * 256;
        const char *pz = std::getenv("FE_ARENA_POISON");
        poison_ = pz && pz[0] == '1';
        hipError_t e = hipMalloc(&base_, size_);
        if (e == hipSuccess) fl_.reset(size_);
        return e;
    }
    ~Arena() override
    {
        if (base_) (void)hipFree(base_);
    }
    hipError_t dev_alloc(void **p, size_t n) override
    {
        n = std::max<size_t>(256, (n + 255) / 256 * 256);
        size_t off = 0;
        if (!fl_.take(n, &off)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
        *p = static_cast<char *>(base_) + off;
        return hipSuccess;
    }
    void dev_free(void *p) override
    {
        if (p) fl_.give(static_cast<char *>(p) - static_cast<char *>(base_));
    }
    hipError_t host_alloc(void **p, size_t n) override
    {
        *p = std::aligned_alloc(64, (n + 63) / 64 * 64);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void host_free(void *p) override { std::free(p); }
    size_t size() const { return size_; }
    bool poison() const { return poison_; }
    size_t largest_free() { return fl_.largest(); }

  private:
    void *base_ = nullptr;
    size_t size_ = 0;
    bool poison_ = false;
    FreeList fl_;
};

// One request's block of the arena: allocations are carved from it in order
// (256-byte aligned); frees are ignored, the block returns to the arena when
// the request ends.
class Block final : public Allocator {
  public:
    Block(void *base, size_t size, bool poison, HostPool *pool)
        : base_(static_cast<char *>(base)), size_(size), poison_(poison), pool_(pool)
    {
    }
    hipError_t dev_alloc(void **p, size_t n) override
    {
        n = std::max<size_t>(256, (n + 255) / 256 * 256);
        if (n > size_ - used_) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
        *p = base_ + used_;
        used_ += n;
        // debugging aid: fill fresh blocks with NaN bytes so that a read
        // before the first write shows up as a non-finite result
        if (poison_) return hipMemset(*p, 0xFF, n);
        return hipSuccess;
    }
    void dev_free(void *) override {}
    // host staging: the server's pinned pool, pageable memory when it is full
    // (neither allocating nor freeing synchronises the device)
    hipError_t host_alloc(void **p, size_t n) override
    {
        *p = pool_ ? pool_->alloc(n) : nullptr;
        if (!*p) *p = std::aligned_alloc(64, (n + 63) / 64 * 64);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void host_free(void *p) override
    {
        if (pool_ && pool_->owns(p))
            pool_->release(p);
        else
            std::free(p);
    }

  private:
    char *base_;
    size_t size_, used_ = 0;
    bool poison_;
    HostPool *pool_;
};

enum ReqState { Q_WAITING = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    uint64_t ticket = 0;
    fe_grid grid;
    fe_phys phys;
    fe_solve_opts opts;
    std::vector<double> gamma, s, x, x0;  // x0: initial vector (empty: zero)
    size_t footprint = 0;  // bytes of the request's block
    void *block = nullptr;
    ReqState state = Q_WAITING;
    int status = FE_PENDING;
    fe_solve_report rep;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int bypassed = 0;  // later requests admitted while this one waited at the head
    std::string error;
};

}  // namespace

struct fe_server {
    Arena arena;
    HostPool host_pool;
    size_t budget = 0;
    int max_active = 1;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    size_t reserved = 0;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;
    // batched mode: lockstep FGMRES engines by grid size class
    static constexpr int N_ENGINES = 4;
    fe::BatchEngine *engine[N_ENGINES] = {};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Engine of a request in batched mode: classes of DOF count below 50,000, below
// 150,000, below 450,000 and above (16^3, 24^3, 32^3 and 48^3 grids, 24,565 to
// 588,245 DOF, fall in one class each).
int engine_class(int64_t ndof)
{
    int c = 0;
    for (int64_t lim = 50000; c < fe_server::N_ENGINES - 1 && ndof >= lim; lim *= 3) ++c;
    return c;
}

size_t request_footprint(const fe_grid &g, const fe_solve_opts &o)
{
    const int64_t ws = fe_solve_footprint_bytes(&g, &o);
    const int64_t ne = (int64_t)g.nx * g.ny * g.nz;
    const int64_t ndof = (int64_t)NF * (g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    auto r = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t b = ws + 2 * r(8 * ne) + r(8 * ndof) + 64 * 256;
    // margin for the allocations' own rounding
    return (size_t)r(b + b / 256 + ((int64_t)1 << 20));
}

int run_request(fe_server *S, Request *r, hipStream_t st)
{
    Block mem(r->block, r->footprint, S->arena.poison(), &S->host_pool);
    fe_problem *p = nullptr;
    int rc = problem_create_ex(&r->grid, &r->phys, nullptr, MASK_WALLS_PIN, &mem, st, &p);
    if (rc) return rc;
    p->batch = S->engine[engine_class(p->ndof)];
    const int64_t ne = p->ne, ndof = p->ndof;
    double *g = nullptr, *s = nullptr, *x = nullptr;
    hipError_t e = dalloc(p, &g, sizeof(double) * ne);
    if (e == hipSuccess) e = dalloc(p, &s, sizeof(double) * ne);
    if (e == hipSuccess) e = dalloc(p, &x, sizeof(double) * ndof);
    if (e == hipSuccess) e = hipMemcpyAsync(g, r->gamma.data(), sizeof(double) * ne, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s, r->s.data(), sizeof(double) * ne, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (r->x0.empty())
            e = hipMemsetAsync(x, 0, sizeof(double) * ndof, st);
        else
            e = hipMemcpyAsync(x, r->x0.data(), sizeof(double) * ndof, hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) {
        rc = hip_fail(e, "serve: request set-up");
    } else {
        rc = newton_solve(p, g, s, x, &r->opts, &r->rep, st);
        r->x.resize(ndof);
        e = hipMemcpyAsync(r->x.data(), x, sizeof(double) * ndof, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess && rc >= 0) rc = hip_fail(e, "serve: result copy");
    }
    dfree(p, g);
    dfree(p, s);
    dfree(p, x);
    fe_problem_destroy(p);
    return rc;
}

// The queued request to admit next (under S->mu): the head if it fits the
// largest free block of the arena, else the first later one that fits, as
// long as the head has been passed over fewer than max_active times; queue end
// if none.
std::deque<Request *>::iterator admissible(fe_server *S)
{
    if (S->queue.empty()) return S->queue.end();
    const size_t room = S->arena.largest_free();
    auto head = S->queue.begin();
    if ((*head)->footprint <= room) return head;
    if ((*head)->bypassed >= S->max_active) return S->queue.end();
    for (auto it = std::next(head); it != S->queue.end(); ++it)
        if ((*it)->footprint <= room) return it;
    return S->queue.end();
}

void worker_main(fe_server *S)
{
    (void)hipSetDevice(S->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            std::deque<Request *>::iterator pick;
            S->cv.wait(lk, [&] {
                if (S->stop) return true;
                pick = admissible(S);
                return pick != S->queue.end();
            });
            if (S->stop) break;
            r = *pick;
            if (pick != S->queue.begin()) S->queue.front()->bypassed++;
            S->queue.erase(pick);
            // the arena changes only here and at a request's end, both under S->mu,
            // so the block found free above is still free
            if (S->arena.dev_alloc(&r->block, r->footprint) != hipSuccess) {
                r->status = r->rep.status = FE_ENOMEM;
                r->error = "serve: no arena block for the request";
                r->state = Q_DONE;
                r->t_admit = r->t_done = S->now();
                continue;
            }
            S->reserved += r->footprint;
            r->state = Q_RUNNING;
            r->t_admit = S->now();
            // idle workers all wait for the same condition, so one is woken per
            // event; it passes the wake-up on while more requests are admissible
            if (admissible(S) != S->queue.end()) S->cv.notify_one();
        }
        int rc = run_request(S, r, st);
        // the request's kernels and copies have finished (run_request ends with a
        // stream synchronisation), so its block can be handed out again
        (void)hipStreamSynchronize(st);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.dev_free(r->block);
            r->block = nullptr;
            S->reserved -= r->footprint;
            r->status = rc;
            if (rc < 0) r->rep.status = rc;
            if (rc != FE_OK) r->error = fe_last_error();
            r->state = Q_DONE;
            r->t_done = S->now();
        }
        S->cv.notify_one();
    }
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

int serve_create(size_t hbm_budget_bytes, int max_active, fe_server **out)
{
    return serve_create_ex(hbm_budget_bytes, max_active, 0, out);
}

int serve_create_ex(size_t hbm_budget_bytes, int max_active, int flags, fe_server **out)
{
    const bool batched = (flags & FE_SERVE_BATCHED) != 0;
    const int cap = batched ? 256 : 64;
    if (!out || max_active < 1 || max_active > cap || hbm_budget_bytes < ((size_t)1 << 20) ||
        (flags & ~FE_SERVE_BATCHED)) {
        set_error("serve_create: need out != NULL, 1 <= max_active <= 64 (256 batched), "
                  "budget >= 1 MiB, known flags");
        return FE_EINVAL;
    }
    *out = nullptr;
    auto *S = new (std::nothrow) fe_server();
    if (!S) return FE_ENOMEM;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        set_error("serve_create: no device");
        return FE_EHIP;
    }
    hipError_t e = S->arena.init(hbm_budget_bytes);
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "serve_create: arena allocation");
    }
    S->budget = S->arena.size();
    S->max_active = max_active;
    // pinned host staging: 4 MiB per worker slot within [64 MiB, 512 MiB]
    // (requests of 16^3 to 48^3 take 1.1 to 2.9 MiB, mostly the coarsest
    // level's probing products and band factors; past the pool, pageable memory)
    const size_t pool = std::min<size_t>(std::max<size_t>((size_t)max_active << 22, (size_t)64 << 20),
                                         (size_t)512 << 20);
    if (S->host_pool.init(pool) != hipSuccess) (void)hipGetLastError();  // pageable only
    if (batched) {
        for (auto &E : S->engine) {
            const int rc = batch_engine_create(S->device, &E);
            if (rc) {
                for (auto &F : S->engine) batch_engine_destroy(F);
                delete S;
                return rc;
            }
        }
    }
    S->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < max_active; ++i) S->workers.emplace_back(worker_main, S);
    *out = S;
    return FE_OK;
}

int serve_submit(fe_server *S, const fe_grid *grid, const fe_phys *phys, const double *gamma_host,
                 const double *s_host, const fe_solve_opts *opts, uint64_t *ticket)
{
    return serve_submit_x0(S, grid, phys, gamma_host, s_host, nullptr, opts, ticket);
}

int serve_submit_x0(fe_server *S, const fe_grid *grid, const fe_phys *phys,
                    const double *gamma_host, const double *s_host, const double *x0_host,
                    const fe_solve_opts *opts, uint64_t *ticket)
{
    if (!S || !grid || !phys || !gamma_host || !s_host || !ticket) {
        set_error("serve_submit_x0: NULL argument");
        return FE_EINVAL;
    }
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->h > 0)) {
        set_error("serve_submit: bad grid");
        return FE_EINVAL;
    }
    auto r = std::make_unique<Request>();
    r->grid = *grid;
    r->phys = *phys;
    fe_solve_opts_default(&r->opts);
    if (opts) r->opts = *opts;
    r->opts.verbose = 0;
    // batched mode: levels up to 1,000 nodes assembled (by default 10,000).  Over a
    // batch, an assembled level's 675 stencil values per node make its products
    // bandwidth-bound where the element pass reads about ten values per node
    // (256 requests of 16^3 at 1000/s: 324 -> 832 solves/s); alone, the stencil
    // is the faster of the two at that size.
    if (S->engine[0] && r->opts.mg_assembled_nodes < 0) r->opts.mg_assembled_nodes = 1000;
    const int64_t ne = (int64_t)grid->nx * grid->ny * grid->nz;
    r->gamma.assign(gamma_host, gamma_host + ne);
    r->s.assign(s_host, s_host + ne);
    if (x0_host) {
        const int64_t ndof = (int64_t)NF * (grid->nx + 1) * (grid->ny + 1) * (grid->nz + 1);
        r->x0.assign(x0_host, x0_host + ndof);
    }
    std::memset(&r->rep, 0, sizeof(r->rep));
    r->footprint = request_footprint(r->grid, r->opts);
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    r->t_submit = S->now();
    *ticket = r->ticket;
    Request *raw = r.get();
    if (r->footprint > S->budget) {
        r->state = Q_DONE;
        r->status = FE_ENOMEM;
        r->rep.status = FE_ENOMEM;
        r->t_admit = r->t_done = r->t_submit;
        S->reqs[raw->ticket] = std::move(r);
        set_error("serve_submit: request footprint exceeds the server's memory budget");
        return FE_ENOMEM;
    }
    S->reqs[raw->ticket] = std::move(r);
    S->queue.push_back(raw);
    S->cv.notify_one();
    return FE_OK;
}

int serve_poll(fe_server *S, uint64_t ticket, double *x_host_out, fe_solve_report *report)
{
    if (!S) {
        set_error("serve_poll: NULL server");
        return FE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("serve_poll: unknown ticket");
        return FE_EINVAL;
    }
    Request *r = it->second.get();
    if (r->state != Q_DONE) return FE_PENDING;
    if (x_host_out && !r->x.empty()) std::memcpy(x_host_out, r->x.data(), sizeof(double) * r->x.size());
    if (report) *report = r->rep;
    return r->status;
}

int serve_times(fe_server *S, uint64_t ticket, double *t_submit, double *t_admit, double *t_done)
{
    if (!S) {
        set_error("serve_times: NULL server");
        return FE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("serve_times: unknown ticket");
        return FE_EINVAL;
    }
    const Request *r = it->second.get();
    if (t_submit) *t_submit = r->t_submit;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    return r->state == Q_DONE ? FE_OK : FE_PENDING;
}

const char *serve_error(fe_server *S, uint64_t ticket)
{
    if (!S) return "";
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->state != Q_DONE) return "";
    return it->second->error.c_str();
}

int serve_destroy(fe_server *S)
{
    if (!S) return FE_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &E : S->engine) batch_engine_destroy(E);
    delete S;
    return FE_OK;
}

int serve_engine_stats(fe_server *S, uint64_t *steps, uint64_t *launches)
{
    if (!S) {
        set_error("serve_engine_stats: NULL server");
        return FE_EINVAL;
    }
    uint64_t st = 0, la = 0;
    for (auto *E : S->engine) {
        uint64_t a = 0, b = 0;
        batch_engine_stats(E, &a, &b);
        st += a;
        la += b;
    }
    if (steps) *steps = st;
    if (launches) *launches = la;
    return FE_OK;
}

}  // extern "C"
