// Solve server: continuous batching of independent exponential-DG solves on
// one device (a serving pattern on top of the method of Section 2).
//
// Each request runs the same controller coroutines as expdg_step
// (controller.h) under the server's executor.  The executor does not launch
// an Arnoldi step at once: it records it and suspends the solve.  Once per
// tick the server resumes every solve whose results are there, then launches
// what they recorded as grouped kernels -- one linear-operator launch per
// (equation, degree) and one launch per Gram-Schmidt pass over all solves --
// and all recorded Krylov checks as one batched small-exponential launch on a
// second stream, which overlaps the next tick's Arnoldi work.  Everything a
// solve does outside its Arnoldi steps (residuals, norms, the combine, state
// updates) is launched at once on the main stream, in the solve's own order.
//
// Memory: the HBM budget is one device allocation (the arena) made at
// creation; a request is admitted, in arrival order, when its workspace and
// its two states fit the arena and fewer than max_active solves run.  The
// workspace returns to the arena when the solve ends and the device is done
// with it; the state when it is fetched or cancelled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "controller.h"
#include "runtime.h"

using namespace expdg;

namespace {

// ---- device arena (first fit, coalescing free list) ----
class Arena {
  public:
    static constexpr size_t kAlign = 256;

    void init(char *base, size_t size) {
        base_ = base;
        size_ = size;
        free_.clear();
        free_[0] = size;
        used_ = peak_ = 0;
    }
    char *base() const { return base_; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

    static size_t round(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    bool alloc(size_t n, size_t *off) {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }

    void release(size_t off, size_t n) {
        n = round(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        // merge with the next and the previous block
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

  private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req;

// One tick's records.
struct IterRec {
    Req *r;
    OpArgs<double> a;
    GsItem g;
};
struct CheckRec {
    Req *r;
    ExpmItem e;
};

constexpr int kRing = 16;  // ticks in flight (staging buffers and events)
// A blocking tick waits for earlier ticks while fewer than this share of the
// running solves is ready.  Without it the host ran many ticks ahead of the
// device, each carrying the ~12 % of solves whose results were back; on the
// 2000-request mix at 200/s (max_active 256) waiting for 90 % took the solves
// per tick from 30 to 91 Arnoldi steps and the throughput from 123 to 141
// solves/s (p50 3.36 -> 2.48 s, p99 7.9 -> 6.0 s; 75 % and 100 % measured
// 140/s).
constexpr int kGatherPercent = 90;

struct Batch {
    long long tick = -1;
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    char *host = nullptr;  // pinned staging of the descriptor tables
    char *dev = nullptr;   // their device copy
};

enum class Wait { None, Tick, Event, Check };

}  // namespace

struct expdg_server;

namespace {

// The executor of one served solve.
struct ServeExec {
    // a solve decides a check one Arnoldi step after the one that launched it
    static constexpr int kLookahead = 1;
    expdg_server *sv = nullptr;
    Req *r = nullptr;

    struct Await {
        Req *r;
        bool ready;
        int rc;
        bool await_ready() const noexcept { return ready; }
        void await_suspend(std::coroutine_handle<> h) noexcept;
        int await_resume() const noexcept;
    };

    hipStream_t stream() const;
    Await iterate(expdg_mesh *m, const OpArgs<double> &a, int k, int naug_nz, const CheckReq *cr,
                  Check *c, bool iop);
    Await check(expdg_mesh *m, const CheckReq &q, Check *c);
    Await wait_check(expdg_mesh *m, const Check &c);
    int after_check(expdg_mesh *m, const Check &c);
    Await readback(expdg_mesh *m);
    Await finish(expdg_mesh *) { return Await{r, true, EXPDG_OK}; }
};

struct Req {
    long long id = 0;
    expdg_request rq{};
    std::vector<double> q0;
    int state = EXPDG_REQ_QUEUED;
    int error = EXPDG_OK;
    int steps_done = 0;
    double dt = 0.0;
    expdg_krylov_opts opts{};
    expdg_krylov_stats stats{};
    double t_submit = -1.0, t_admit = -1.0, t_done = -1.0;
    size_t ws_bytes = 0, st_bytes = 0;

    // while admitted
    expdg_mesh mesh;
    size_t ws_off = 0, st_off = 0;
    bool has_ws = false, has_st = false;
    double *q = nullptr, *qp = nullptr;
    int pin_slot = -1;
    hipEvent_t ev = nullptr;  // readback fence
    ServeExec x;
    Task<int> task;
    std::coroutine_handle<> resume;
    Wait wait = Wait::None;
    long long wait_tick = 0;  // Tick: runnable from this tick; Check: the batch waited on;
                              // Event: the tick the fence was recorded in
    int rc_in = EXPDG_OK;     // status handed to the resumed await
    long long release_tick = -1;  // workspace returns once this batch is done
    bool drop_state = false;      // the state returns with the workspace
    bool dropped = false;         // forgotten (fetched or cancelled) once memory is back
};

void ServeExec::Await::await_suspend(std::coroutine_handle<> h) noexcept { r->resume = h; }
int ServeExec::Await::await_resume() const noexcept { return ready ? rc : r->rc_in; }

// Device memory of a request: Krylov workspace, then the two FP64 states.
bool request_sizes(const expdg_request *r, size_t *ws, size_t *st, const char **why) {
    if (!r) return *why = "request is NULL", false;
    expdg_mesh_desc d = r->mesh;
    d.device = 0;
    if (!desc_ok(&d, why)) return false;
    if (d.precision != EXPDG_FP64) return *why = "served solves are FP64", false;
    if (d.has_source) return *why = "served solves take no source term", false;
    if (d.equation == EXPDG_EULER3D) return *why = "served solves are 1D or 2D", false;
    if (r->scheme != EXPDG_EPI2 && r->scheme != EXPDG_EPI3)
        return *why = "scheme must be EXPDG_EPI2 or EXPDG_EPI3", false;
    if (r->nsteps < 1) return *why = "nsteps must be >= 1", false;
    if (!std::isfinite(r->dt)) return *why = "dt must be finite", false;
    if (!(r->dt > 0.0) && !(r->cfl > 0.0 && std::isfinite(r->cfl)))
        return *why = "need dt > 0 or cfl > 0", false;
    if (!(r->tol > 0.0) || !std::isfinite(r->tol)) return *why = "tol must be > 0", false;
    if (r->m_min < 1 || r->m_max < r->m_min || r->m_max > d.m_max)
        return *why = "need 1 <= m_min <= m_max <= mesh.m_max", false;
    if (r->check_every < 1) return *why = "check_every must be >= 1", false;
    if (r->iop < 0 || r->iop > kMaxM) return *why = "iop must be in 0..64", false;
    if (r->adapt != 0 && r->adapt != 1) return *why = "adapt must be 0 or 1", false;
    const Sizes sz = sizes_of(&d);
    *ws = Arena::round(sz.total);
    *st = Arena::round(sz.stride * 8) * 2;
    return true;
}

}  // namespace

struct expdg_server {
    int device = 0;
    int max_active = 0;
    hipStream_t s = nullptr, side = nullptr;
    void *arena_mem = nullptr;
    Arena arena;
    double *pin_pool = nullptr, *pin_pool_dev = nullptr;  // max_active x kPinSize
    std::vector<int> free_pins;
    std::vector<hipEvent_t> free_events;
    std::unordered_map<long long, std::unique_ptr<Req>> reqs;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::vector<Req *> zombies;   // ended, workspace not yet released
    std::vector<long long> finished;
    long long next_id = 1;
    long long tick = 0;       // ticks started
    long long done_tick = 0;  // every batch <= done_tick has completed on both streams
    Batch ring[kRing];
    size_t stage_cap = 0;
    std::vector<IterRec> iters;
    std::vector<CheckRec> checks;
    expdg_server_stats st{};
    std::chrono::steady_clock::time_point t0;
    bool broken = false;  // a device error ended the server

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

hipStream_t ServeExec::stream() const { return sv->s; }

ServeExec::Await ServeExec::iterate(expdg_mesh *m, const OpArgs<double> &a, int k, int naug_nz,
                                    const CheckReq *cr, Check *c, bool iop) {
    (void)naug_nz;
    IterRec rec;
    rec.r = r;
    rec.a = a;
    const size_t L = m->n + (size_t)a.naug;
    const RowPartition rp = row_partition(L);
    const KrylovDev &kd = m->kd;
    GsItem &g = rec.g;
    g.V = (const double *)m->V;
    g.x = (double *)m->V + (size_t)(k - 1) * m->stride;
    g.w = a.out;
    g.stride = m->stride;
    g.L = L;
    g.rpb = rp.rpb;
    g.nrb = rp.nrb;
    g.nrb1 = a.dots ? a.dnb : 0;  // 0: a separate dot pass
    g.nfold = fold_chunks(g.nrb1);
    g.fold = kd.fold;
    g.k = k;
    g.nv = a.nv;
    g.k0 = k - 1 - a.nv;
    g.iop = iop ? 1 : 0;
    g.part = kd.part;
    g.S = kd.S;
    g.H = kd.H;
    g.coefA = kd.coefA;
    g.coefB = kd.coefB;
    g.flags = kd.flags;
    sv->iters.push_back(rec);
    if (cr) {
        c->j = cr->j;
        c->slot = cr->slot;
        c->tick = sv->tick;
        sv->checks.push_back(CheckRec{r, ExpmItem{kd.H, kd.S, kd.res, kd.flags,
                                                  m->slots + cr->slot * kSlotSize,
                                                  m->pin_dev + kPinSlots + cr->slot * 8, cr->dtau,
                                                  cr->j}});
    }
    r->wait = Wait::Tick;
    r->wait_tick = sv->tick + 1;
    return Await{r, false, EXPDG_OK};
}

ServeExec::Await ServeExec::check(expdg_mesh *m, const CheckReq &q, Check *c) {
    const KrylovDev &kd = m->kd;
    c->j = q.j;
    c->slot = q.slot;
    c->tick = sv->tick;
    sv->checks.push_back(CheckRec{r, ExpmItem{kd.H, kd.S, kd.res, kd.flags,
                                              m->slots + q.slot * kSlotSize,
                                              m->pin_dev + kPinSlots + q.slot * 8, q.dtau, q.j}});
    r->wait = Wait::Tick;
    r->wait_tick = sv->tick + 1;
    return Await{r, false, EXPDG_OK};
}

bool batch_done(expdg_server *sv, long long t) {
    if (t <= sv->done_tick) return true;
    const Batch &b = sv->ring[t % kRing];
    if (b.tick != t) return false;  // not launched yet
    return hipEventQuery(b.ev_side) == hipSuccess && hipEventQuery(b.ev_main) == hipSuccess;
}

ServeExec::Await ServeExec::wait_check(expdg_mesh *, const Check &c) {
    if (batch_done(sv, c.tick)) return Await{r, true, EXPDG_OK};
    r->wait = Wait::Check;
    r->wait_tick = c.tick;
    return Await{r, false, EXPDG_OK};
}

int ServeExec::after_check(expdg_mesh *, const Check &c) {
    if (c.tick <= sv->done_tick) return EXPDG_OK;
    const Batch &b = sv->ring[c.tick % kRing];
    if (b.tick != c.tick) return fail(EXPDG_EDEVICE, "check batch %lld not launched", c.tick);
    HIPTRY(hipStreamWaitEvent(sv->s, b.ev_side, 0));
    return EXPDG_OK;
}

ServeExec::Await ServeExec::readback(expdg_mesh *) {
    if (hipEventRecord(r->ev, sv->s) != hipSuccess)
        return Await{r, true, fail(EXPDG_EDEVICE, "hipEventRecord failed")};
    r->wait = Wait::Event;
    r->wait_tick = sv->tick;
    return Await{r, false, EXPDG_OK};
}

// The whole served solve: optional CFL step from q0, then nsteps steps.
Task<int> serve_co(ServeExec &x, Req *r) {
    expdg_mesh *m = &r->mesh;
    hipStream_t s = x.stream();
    if (!(r->rq.dt > 0.0)) {
        const size_t npts = (size_t)m->K * m->Np;
        const int nblk = max_speed_blocks(npts);
        CO_HIPTRY(launch_max_speed(m->d.equation, r->q, npts, m->d.gamma, m->spart, nblk, s));
        CO_HIPTRY(
            hipMemcpyAsync(m->pin + kPinSpeed, m->spart, nblk * 8, hipMemcpyDeviceToHost, s));
        CO_TRY(co_await x.readback(m));
        double c = 0.0;
        for (int b = 0; b < nblk; ++b) c = std::max(c, m->pin[kPinSpeed + b]);
        if (!std::isfinite(c) || !(c > 0.0))
            co_return fail(EXPDG_ENONFINITE, "wave speed of q0 is not a positive number");
        r->dt = r->rq.cfl * m->dxmin / c;
    } else {
        r->dt = r->rq.dt;
    }
    // the history: EPI3, and the entropy viscosity's q^{n-1}
    double *qp = (r->rq.scheme == EXPDG_EPI3 || m->d.ev_ce > 0.0) ? r->qp : nullptr;
    for (int k = 0; k < r->rq.nsteps; ++k) {
        CO_AWAIT_TASK((step_co<double, ServeExec>(x, m, r->rq.scheme, r->dt, r->q, qp, k > 0,
                                                  &r->opts, &r->stats)));
        r->steps_done = k + 1;
    }
    // the final state is complete on the device
    CO_TRY(co_await x.readback(m));
    co_return EXPDG_OK;
}

void return_workspace(expdg_server *sv, Req *r) {
    std::vector<double>().swap(r->q0);
    if (r->has_ws) sv->arena.release(r->ws_off, r->ws_bytes);
    r->has_ws = false;
    if (r->pin_slot >= 0) sv->free_pins.push_back(r->pin_slot);
    r->pin_slot = -1;
    if (r->ev) sv->free_events.push_back(r->ev);
    r->ev = nullptr;
}

void return_state(expdg_server *sv, Req *r) {
    if (r->has_st) sv->arena.release(r->st_off, r->st_bytes);
    r->has_st = false;
    r->q = r->qp = nullptr;
}

bool is_zombie(const expdg_server *sv, const Req *r) {
    return std::find(sv->zombies.begin(), sv->zombies.end(), r) != sv->zombies.end();
}

// A running solve ended (finished, failed or cancelled): its frames go now,
// its workspace once every batch launched so far has completed (a speculative
// check may still run).  The state of a failed or cancelled solve goes with it.
void end_solve(expdg_server *sv, Req *r, int rc, bool cancelled) {
    r->task = Task<int>();
    r->resume = nullptr;
    auto it = std::find(sv->active.begin(), sv->active.end(), r);
    if (it != sv->active.end()) sv->active.erase(it);
    r->release_tick = sv->tick;
    sv->zombies.push_back(r);
    if (cancelled) {
        r->drop_state = true;
        r->dropped = true;
        return;
    }
    r->t_done = sv->now();
    r->state = (rc == EXPDG_OK) ? EXPDG_REQ_DONE : EXPDG_REQ_FAILED;
    r->error = rc;
    r->drop_state = rc != EXPDG_OK;  // nothing to fetch
    sv->finished.push_back(r->id);
}

// Forgets a request that is not running, now or once its workspace is back.
void forget(expdg_server *sv, Req *r) {
    if (is_zombie(sv, r)) {
        r->drop_state = true;
        r->dropped = true;
        return;
    }
    return_state(sv, r);
    sv->reqs.erase(r->id);
}

// Moves done_tick forward and returns the workspaces no batch can touch any more.
void advance(expdg_server *sv) {
    while (sv->done_tick < sv->tick) {
        const long long t = sv->done_tick + 1;
        const Batch &b = sv->ring[t % kRing];
        if (b.tick != t) break;
        if (hipEventQuery(b.ev_side) != hipSuccess || hipEventQuery(b.ev_main) != hipSuccess)
            break;
        sv->done_tick = t;
    }
    for (size_t k = 0; k < sv->zombies.size();) {
        Req *r = sv->zombies[k];
        if (r->release_tick <= sv->done_tick) {
            return_workspace(sv, r);
            if (r->drop_state) return_state(sv, r);
            sv->zombies[k] = sv->zombies.back();
            sv->zombies.pop_back();
            if (r->dropped) sv->reqs.erase(r->id);
        } else {
            ++k;
        }
    }
}

// Admits queued requests in order while they fit.
int admit(expdg_server *sv) {
    while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active &&
           !sv->free_pins.empty()) {
        Req *r = sv->queue.front();
        size_t ws_off = 0, st_off = 0;
        if (!sv->arena.alloc(r->ws_bytes, &ws_off)) break;
        if (!sv->arena.alloc(r->st_bytes, &st_off)) {
            sv->arena.release(ws_off, r->ws_bytes);
            break;
        }
        if (sv->free_events.empty()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                sv->arena.release(ws_off, r->ws_bytes);
                sv->arena.release(st_off, r->st_bytes);
                return fail(EXPDG_EDEVICE, "hipEventCreate failed");
            }
            sv->free_events.push_back(e);
        }
        sv->queue.pop_front();
        r->ws_off = ws_off;
        r->st_off = st_off;
        r->has_ws = r->has_st = true;
        r->ev = sv->free_events.back();
        sv->free_events.pop_back();
        r->pin_slot = sv->free_pins.back();
        sv->free_pins.pop_back();

        expdg_mesh_desc d = r->rq.mesh;
        d.device = sv->device;
        mesh_setup(&r->mesh, &d);
        char *ws = sv->arena.base() + ws_off;
        mesh_carve(&r->mesh, ws);
        r->mesh.pin = sv->pin_pool + (size_t)r->pin_slot * kPinSize;
        r->mesh.pin_dev = sv->pin_pool_dev + (size_t)r->pin_slot * kPinSize;
        char *stb = sv->arena.base() + st_off;
        r->q = (double *)stb;
        r->qp = (double *)(stb + r->st_bytes / 2);
        // a fresh workspace (vector padding zero) and the initial state
        HIPTRY(hipMemsetAsync(ws, 0, r->ws_bytes, sv->s));
        // (q0 stays allocated until the workspace returns: the copy reads it
        // asynchronously)
        HIPTRY(hipMemcpyAsync(r->q, r->q0.data(), r->mesh.n * 8, hipMemcpyHostToDevice, sv->s));
        r->opts = expdg_krylov_opts{r->rq.tol, r->rq.m_min, r->rq.m_max, r->rq.check_every,
                                    nullptr, 0, r->rq.iop, r->rq.adapt, 0};
        r->state = EXPDG_REQ_ACTIVE;
        r->t_admit = sv->now();
        r->x.sv = sv;
        r->x.r = r;
        r->task = serve_co(r->x, r);
        if (!r->task.valid()) {
            end_solve(sv, r, fail(EXPDG_ENOMEM, "coroutine frame allocation failed"), false);
            continue;
        }
        r->wait = Wait::None;
        r->resume = nullptr;
        sv->active.push_back(r);
    }
    return EXPDG_OK;
}

// Whether a solve can run in the current tick (sv->tick).
bool ready(expdg_server *sv, Req *r) {
    switch (r->wait) {
        case Wait::None: return true;
        case Wait::Tick: return sv->tick >= r->wait_tick;
        case Wait::Event: return hipEventQuery(r->ev) == hipSuccess;
        case Wait::Check: return batch_done(sv, r->wait_tick);
    }
    return false;
}

// Resumes every ready solve once; returns how many ran.
int resume_ready(expdg_server *sv, int *finished) {
    int ran = 0;
    std::vector<Req *> now(sv->active);  // solves may end while we go
    for (Req *r : now) {
        if (!ready(sv, r)) continue;
        ++ran;
        r->wait = Wait::None;
        if (r->resume)
            r->resume.resume();
        else
            r->task.start();
        r->rc_in = EXPDG_OK;
        if (r->task.done()) {
            end_solve(sv, r, r->task.result(), false);
            if (finished) ++*finished;
        }
    }
    return ran;
}

// Blocks until some running solve is ready.
int wait_any(expdg_server *sv) {
    Req *best = nullptr;
    for (Req *r : sv->active) {
        if (ready(sv, r)) return EXPDG_OK;
        if (!best || r->wait_tick < best->wait_tick) best = r;
    }
    if (!best) return EXPDG_OK;
    if (best->wait == Wait::Event) {
        HIPTRY(hipEventSynchronize(best->ev));
    } else if (best->wait == Wait::Check) {
        const Batch &b = sv->ring[best->wait_tick % kRing];
        if (b.tick == best->wait_tick) {
            HIPTRY(hipEventSynchronize(b.ev_side));
            HIPTRY(hipEventSynchronize(b.ev_main));
        }
    }
    advance(sv);
    return EXPDG_OK;
}

template <typename T>
T *stage(Batch &b, size_t &used, size_t cap, const T *src, size_t count, T **dev) {
    used = (used + 15) / 16 * 16;
    const size_t bytes = count * sizeof(T);
    if (used + bytes > cap) return nullptr;
    std::memcpy(b.host + used, src, bytes);
    *dev = (T *)(b.dev + used);
    used += bytes;
    return (T *)(b.host + used - bytes);
}

// Launches the tick's grouped Arnoldi steps and its batched checks.
int launch_batch(expdg_server *sv) {
    Batch &b = sv->ring[sv->tick % kRing];
    size_t used = 0;
    const size_t cap = sv->stage_cap;
    const int n = (int)sv->iters.size();
    // linear operator: one grouped launch per (equation, degree, viscous or not)
    struct Group {
        int eq, p;
        bool visc;
        std::vector<OpArgs<double>> items;
        std::vector<int> bstart;
        OpArgs<double> *d_items = nullptr;
        int *d_bstart = nullptr;
    };
    std::vector<Group> groups;
    for (const IterRec &it : sv->iters) {
        const int eq = it.r->mesh.d.equation, p = it.r->mesh.d.p;
        // viscous Burgers, or Euler 2D with entropy viscosity
        const bool visc = it.r->mesh.d.kappa != 0.0 || it.r->mesh.d.ev_ce > 0.0;
        Group *g = nullptr;
        for (auto &x : groups)
            if (x.eq == eq && x.p == p && x.visc == visc) g = &x;
        if (!g) {
            groups.push_back(Group{eq, p, visc, {}, {0}});
            g = &groups.back();
        }
        g->items.push_back(it.a);
        g->bstart.push_back(g->bstart.back() + dg_blocks(eq, p, it.r->mesh.K));
    }
    std::vector<GsItem> gs(n);
    for (int k = 0; k < n; ++k) gs[k] = sv->iters[k].g;
    std::vector<int> gb((size_t)kGroupLaunches * (n + 1));
    int totals[kGroupLaunches] = {};
    if (n > 0) arnoldi_group_layout(gs.data(), n, gb.data(), totals);
    std::vector<ExpmItem> ex;
    ex.reserve(sv->checks.size());
    for (const CheckRec &c : sv->checks) ex.push_back(c.e);

    GsItem *d_gs = nullptr;
    int *d_gb = nullptr;
    ExpmItem *d_ex = nullptr;
    bool ok = true;
    for (auto &g : groups) {
        ok = ok && stage(b, used, cap, g.items.data(), g.items.size(), &g.d_items);
        ok = ok && stage(b, used, cap, g.bstart.data(), g.bstart.size(), &g.d_bstart);
    }
    if (n > 0) {
        ok = ok && stage(b, used, cap, gs.data(), gs.size(), &d_gs);
        ok = ok && stage(b, used, cap, gb.data(), gb.size(), &d_gb);
    }
    if (!ex.empty()) ok = ok && stage(b, used, cap, ex.data(), ex.size(), &d_ex);
    if (!ok) return fail(EXPDG_EDEVICE, "tick staging overflow (%zu bytes)", cap);

    if (used) HIPTRY(hipMemcpyAsync(b.dev, b.host, used, hipMemcpyHostToDevice, sv->s));
    for (auto &g : groups) {
        HIPTRY(launch_dg_op_group(g.eq, g.p, true, g.visc, g.d_items, g.d_bstart,
                                  (int)g.items.size(), g.bstart.back(), sv->s));
        sv->st.grouped_launches += 1;
    }
    if (n > 0) {
        HIPTRY(launch_arnoldi_group(d_gs, d_gb, totals, n, sv->s));
        // the separate dot pass (if any item needs it), the finish, the update
        sv->st.grouped_launches += (totals[0] > 0 ? 1 : 0) + 2;
        sv->st.arnoldi_items += n;
    }
    HIPTRY(hipEventRecord(b.ev_main, sv->s));
    HIPTRY(hipStreamWaitEvent(sv->side, b.ev_main, 0));
    if (!ex.empty()) {
        HIPTRY(launch_hess_expm_group(d_ex, (int)ex.size(), sv->side));
        sv->st.batched_checks += 1;
        sv->st.check_items += (long long)ex.size();
    }
    HIPTRY(hipEventRecord(b.ev_side, sv->side));
    b.tick = sv->tick;
    if (n > 0 || !ex.empty()) sv->st.ticks += 1;
    sv->iters.clear();
    sv->checks.clear();
    return EXPDG_OK;
}

void destroy_all(expdg_server *sv) {
    if (sv->s) (void)hipStreamSynchronize(sv->s);
    if (sv->side) (void)hipStreamSynchronize(sv->side);
    for (auto &kv : sv->reqs)
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    sv->reqs.clear();  // frames of running solves go with their requests
    for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
    sv->free_events.clear();
    for (Batch &b : sv->ring) {
        if (b.ev_main) (void)hipEventDestroy(b.ev_main);
        if (b.ev_side) (void)hipEventDestroy(b.ev_side);
        if (b.host) (void)hipHostFree(b.host);
        if (b.dev) (void)hipFree(b.dev);
        b = Batch{};
    }
    if (sv->pin_pool) (void)hipHostFree(sv->pin_pool);
    if (sv->arena_mem) (void)hipFree(sv->arena_mem);
    if (sv->s) (void)hipStreamDestroy(sv->s);
    if (sv->side) (void)hipStreamDestroy(sv->side);
}

Req *find(expdg_server *sv, long long id) {
    auto it = sv->reqs.find(id);
    return it == sv->reqs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" size_t expdg_request_bytes(const expdg_request *r) {
    size_t ws = 0, st = 0;
    const char *why = "";
    if (!request_sizes(r, &ws, &st, &why)) return 0;
    return ws + st;
}

extern "C" int expdg_server_create(int device, size_t hbm_budget, int max_active,
                                   expdg_server **out) {
    if (!out) return fail(EXPDG_EINVAL, "out is NULL");
    if (max_active < 1 || max_active > 4096) return fail(EXPDG_EINVAL, "max_active must be in 1..4096");
    if (hbm_budget < ((size_t)1 << 20)) return fail(EXPDG_EINVAL, "hbm_budget below 1 MiB");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(EXPDG_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(EXPDG_EINVAL, "device %d out of range", device);
    DeviceGuard g(device);
    if (!g.ok) return fail(EXPDG_EDEVICE, "hipSetDevice(%d) failed", device);
    expdg_server *sv = new (std::nothrow) expdg_server();
    if (!sv) return fail(EXPDG_ENOMEM, "host allocation failed");
    sv->device = device;
    sv->max_active = max_active;
    sv->t0 = std::chrono::steady_clock::now();
    int rc = EXPDG_OK;
    auto chk = [&](bool good, int code, const char *what) {
        if (rc == EXPDG_OK && !good) {
            (void)hipGetLastError();
            rc = fail(code, "%s failed", what);
        }
    };
    hbm_budget = hbm_budget / Arena::kAlign * Arena::kAlign;
    chk(hipMalloc(&sv->arena_mem, hbm_budget) == hipSuccess, EXPDG_ENOMEM, "hipMalloc of the HBM budget");
    if (rc == EXPDG_OK) sv->arena.init((char *)sv->arena_mem, hbm_budget);
    chk(hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking) == hipSuccess, EXPDG_EDEVICE,
        "hipStreamCreate");
    chk(hipStreamCreateWithFlags(&sv->side, hipStreamNonBlocking) == hipSuccess, EXPDG_EDEVICE,
        "hipStreamCreate");
    if (rc == EXPDG_OK) {
        chk(hipHostMalloc((void **)&sv->pin_pool, (size_t)max_active * kPinSize * 8,
                          hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess,
            EXPDG_ENOMEM, "pinned host allocation");
        if (rc == EXPDG_OK)
            chk(hipHostGetDevicePointer((void **)&sv->pin_pool_dev, sv->pin_pool, 0) ==
                    hipSuccess,
                EXPDG_EDEVICE, "hipHostGetDevicePointer");
    }
    for (int k = max_active - 1; k >= 0; --k) sv->free_pins.push_back(k);
    // descriptor tables of one tick: at most one Arnoldi step and one check per solve
    sv->stage_cap = (size_t)max_active * (sizeof(OpArgs<double>) + sizeof(GsItem) +
                                          sizeof(ExpmItem) + (kGroupLaunches + 2) * sizeof(int) +
                                          64) +
                    64 * 1024;
    for (Batch &b : sv->ring) {
        if (rc != EXPDG_OK) break;
        chk(hipEventCreateWithFlags(&b.ev_main, hipEventDisableTiming) == hipSuccess,
            EXPDG_EDEVICE, "hipEventCreate");
        chk(hipEventCreateWithFlags(&b.ev_side, hipEventDisableTiming) == hipSuccess,
            EXPDG_EDEVICE, "hipEventCreate");
        chk(hipHostMalloc((void **)&b.host, sv->stage_cap, hipHostMallocDefault) == hipSuccess,
            EXPDG_ENOMEM, "pinned staging allocation");
        chk(hipMalloc((void **)&b.dev, sv->stage_cap) == hipSuccess, EXPDG_ENOMEM,
            "device staging allocation");
    }
    if (rc != EXPDG_OK) {
        destroy_all(sv);
        delete sv;
        return rc;
    }
    sv->st.arena_bytes = hbm_budget;
    *out = sv;
    return EXPDG_OK;
}

extern "C" int expdg_server_destroy(expdg_server *sv) {
    if (!sv) return fail(EXPDG_EINVAL, "server is NULL");
    DeviceGuard g(sv->device);
    destroy_all(sv);
    delete sv;
    return EXPDG_OK;
}

extern "C" int expdg_server_submit(expdg_server *sv, const expdg_request *r, const double *q0,
                                   long long *id) {
    if (!sv || !r || !q0 || !id) return fail(EXPDG_EINVAL, "NULL argument");
    size_t ws = 0, st = 0;
    const char *why = "";
    if (!request_sizes(r, &ws, &st, &why)) return fail(EXPDG_EINVAL, "invalid request: %s", why);
    if (ws + st > sv->arena.size())
        return fail(EXPDG_EINVAL, "request needs %zu bytes, the HBM budget is %zu", ws + st,
                    sv->arena.size());
    auto req = std::unique_ptr<Req>(new (std::nothrow) Req());
    if (!req) return fail(EXPDG_ENOMEM, "host allocation failed");
    req->rq = *r;
    req->ws_bytes = ws;
    req->st_bytes = st;
    expdg_mesh_desc d = r->mesh;
    d.device = sv->device;
    const size_t n = sizes_of(&d).n;
    try {
        req->q0.assign(q0, q0 + n);
    } catch (...) {
        return fail(EXPDG_ENOMEM, "host allocation failed");
    }
    req->id = sv->next_id++;
    req->t_submit = sv->now();
    Req *p = req.get();
    sv->reqs.emplace(p->id, std::move(req));
    sv->queue.push_back(p);
    *id = p->id;
    return EXPDG_OK;
}

extern "C" int expdg_server_tick(expdg_server *sv, int block, int *finished) {
    if (!sv) return fail(EXPDG_EINVAL, "server is NULL");
    if (finished) *finished = 0;
    if (sv->broken) return fail(EXPDG_EDEVICE, "server stopped after a device error");
    DeviceGuard g(sv->device);
    auto device_error = [&](int rc) {
        sv->broken = true;
        return rc;
    };
    advance(sv);
    int rc = admit(sv);
    if (rc != EXPDG_OK) return device_error(rc);
    if (sv->active.empty()) return EXPDG_OK;
    // a new tick: its staging buffer must be free (the batch kRing ticks ago is done)
    const long long t = sv->tick + 1;
    Batch &b = sv->ring[t % kRing];
    if (b.tick >= 0 && b.tick > sv->done_tick) {
        if (hipEventSynchronize(b.ev_main) != hipSuccess ||
            hipEventSynchronize(b.ev_side) != hipSuccess)
            return device_error(fail(EXPDG_EDEVICE, "batch wait failed"));
        advance(sv);
    }
    sv->tick = t;
    if (block) {
        auto count_ready = [&] {
            int k = 0;
            for (Req *r : sv->active) k += ready(sv, r) ? 1 : 0;
            return k;
        };
        int nready = count_ready();
        // Few solves ready while earlier ticks are still on the device: wait
        // for the oldest of them, so this tick carries the solves it releases
        // instead of launching a thin batch far ahead of the device.
        while ((long long)nready * 100 < (long long)kGatherPercent * (long long)sv->active.size() &&
               sv->done_tick < t - 1) {
            const Batch &ob = sv->ring[(sv->done_tick + 1) % kRing];
            if (ob.tick != sv->done_tick + 1) break;
            if (hipEventSynchronize(ob.ev_main) != hipSuccess ||
                hipEventSynchronize(ob.ev_side) != hipSuccess)
                return device_error(fail(EXPDG_EDEVICE, "batch wait failed"));
            advance(sv);
            nready = count_ready();
        }
        if (nready == 0) {
            rc = wait_any(sv);
            if (rc != EXPDG_OK) return device_error(rc);
        }
    }
    resume_ready(sv, finished);
    rc = launch_batch(sv);
    if (rc != EXPDG_OK) return device_error(rc);
    advance(sv);
    // solves that ended free memory: admit again without waiting for the next call
    rc = admit(sv);
    if (rc != EXPDG_OK) return device_error(rc);
    return EXPDG_OK;
}

extern "C" int expdg_server_finished(expdg_server *sv, long long *ids, int cap) {
    if (!sv || (!ids && cap > 0) || cap < 0) return fail(EXPDG_EINVAL, "bad argument");
    const int k = std::min(cap, (int)sv->finished.size());
    for (int i = 0; i < k; ++i) ids[i] = sv->finished[i];
    sv->finished.erase(sv->finished.begin(), sv->finished.begin() + k);
    return k;
}

extern "C" int expdg_server_poll(expdg_server *sv, long long id, expdg_request_info *info) {
    if (!sv || !info) return fail(EXPDG_EINVAL, "NULL argument");
    Req *r = find(sv, id);
    if (!r || r->dropped) return fail(EXPDG_EINVAL, "unknown request %lld", id);
    info->state = r->state;
    info->error = r->error;
    info->steps_done = r->steps_done;
    info->dt = r->dt;
    info->stats = r->stats;
    info->stats.log = nullptr;
    info->stats.log_cap = 0;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_done = r->t_done;
    info->bytes = r->ws_bytes + r->st_bytes;
    return EXPDG_OK;
}

extern "C" int expdg_server_fetch(expdg_server *sv, long long id, double *q_out) {
    if (!sv || !q_out) return fail(EXPDG_EINVAL, "NULL argument");
    Req *r = find(sv, id);
    if (!r || r->dropped) return fail(EXPDG_EINVAL, "unknown request %lld", id);
    if (r->state != EXPDG_REQ_DONE) return fail(EXPDG_EINVAL, "request %lld is not done", id);
    DeviceGuard g(sv->device);
    HIPTRY(hipMemcpy(q_out, r->q, r->mesh.n * 8, hipMemcpyDeviceToHost));
    advance(sv);
    // the solve's last work on its state has completed (its final fence was
    // read), so the state returns at once
    return_state(sv, r);
    auto fi = std::find(sv->finished.begin(), sv->finished.end(), id);
    if (fi != sv->finished.end()) sv->finished.erase(fi);
    forget(sv, r);
    return EXPDG_OK;
}

extern "C" int expdg_server_cancel(expdg_server *sv, long long id) {
    if (!sv) return fail(EXPDG_EINVAL, "server is NULL");
    Req *r = find(sv, id);
    if (!r) return fail(EXPDG_EINVAL, "unknown request %lld", id);
    DeviceGuard g(sv->device);
    if (r->dropped) return fail(EXPDG_EINVAL, "unknown request %lld", id);
    if (r->state == EXPDG_REQ_ACTIVE) {
        // state and workspace return once the device is done with them
        end_solve(sv, r, EXPDG_OK, true);
        return EXPDG_OK;
    }
    auto qi = std::find(sv->queue.begin(), sv->queue.end(), r);
    if (qi != sv->queue.end()) sv->queue.erase(qi);
    auto fi = std::find(sv->finished.begin(), sv->finished.end(), id);
    if (fi != sv->finished.end()) sv->finished.erase(fi);
    if (r->state == EXPDG_REQ_DONE && !is_zombie(sv, r)) return_state(sv, r);
    forget(sv, r);
    return EXPDG_OK;
}

extern "C" int expdg_server_get_stats(expdg_server *sv, expdg_server_stats *out) {
    if (!sv || !out) return fail(EXPDG_EINVAL, "NULL argument");
    DeviceGuard g(sv->device);
    advance(sv);  // memory of solves the device is done with returns first
    *out = sv->st;
    out->active = (int)sv->active.size();
    out->queued = (int)sv->queue.size();
    int done = 0;
    for (const auto &kv : sv->reqs)
        if (kv.second->state == EXPDG_REQ_DONE && !kv.second->dropped) ++done;
    out->done = done;
    out->arena_bytes = sv->arena.size();
    out->arena_used = sv->arena.used();
    out->arena_peak = sv->arena.peak();
    return EXPDG_OK;
}

extern "C" int expdg_server_sync(expdg_server *sv) {
    if (!sv) return fail(EXPDG_EINVAL, "server is NULL");
    DeviceGuard g(sv->device);
    HIPTRY(hipStreamSynchronize(sv->s));
    HIPTRY(hipStreamSynchronize(sv->side));
    advance(sv);
    return EXPDG_OK;
}

extern "C" double expdg_server_clock(const expdg_server *sv) { return sv ? sv->now() : 0.0; }
