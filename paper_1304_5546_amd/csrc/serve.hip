// Request server: continuous batching of independent 2D cavity solves on one
// device.
//
// Threads: one scheduler owns the device's step loop; a pool of host workers
// does per-request set-up (FP64 geometry, upload, field initialisation) and
// finalisation (FP64 energy / error reductions, field download, release).
//
// Request states: pending (queued, not admitted) -> setup (admitted: slot and
// footprint reserved, a worker is building it) -> ready -> running (in the
// batch) -> done.  Admission is in arrival order, while a slot is free and the
// summed footprints stay within the HBM budget.
//
// The step loop issues chunks: the running requests are grouped by (order,
// material class, alpha); each group gets a descriptor table (per request its
// buffers, first tile, ping-pong parity and dt) and a tile -> request table,
// and one batched stage launch per group and stage covers all its tiles.
// Groups run on their own streams, so small groups overlap.  A chunk ends at
// the earliest finishing request (or after max_chunk_steps): there finished
// requests leave, cancelled ones are dropped and newly set-up ones join.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/dgw.h"
#include "device.hpp"
#include "solver.hpp"

namespace {

using Clock = std::chrono::steady_clock;

enum class St { Pending, Setup, Ready, Running, Done };

struct Req {
    uint64_t id = 0;
    // inputs (copied at submit)
    int64_t nv = 0, K = 0;
    std::vector<double> vx, vy, eps, mu, q0;
    std::vector<int32_t> ev;
    int order = 1;
    int32_t mode[3] = {1, 1, 0};
    double t_final = 0, alpha = 1;
    int prec = DGW_FP32;
    bool keep = false, material = false, uniform = true;
    int64_t footprint = 0;
    // state
    St st = St::Pending;
    bool cancel = false;
    dgw_solver *s = nullptr;
    int64_t steps_left = 0;
    double dt = 0;
    dgw_result res{};
    std::vector<double> fields;
};

// Device-side tables of one (order, material, alpha) group.
struct Group {
    int order = 1;
    bool material = false;
    double alpha = 1;
    int per_cu = 1;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    dgw::BatchDesc *desc_h = nullptr, *desc_d = nullptr;
    int *tiles_h = nullptr, *tiles_d = nullptr;
    size_t cap_desc = 0, cap_tiles = 0;
    float *opsfrag_d = nullptr;  // fragment-ordered operator of this order (group-owned copy)
};

using GroupKey = std::tuple<int, bool, double>;

}  // namespace

struct dgw_server {
    dgw_server_opts opts{};
    int ncu = 256;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_work;
    std::deque<Req *> pending, ready;
    std::vector<Req *> running;
    std::unordered_map<uint64_t, Req *> reqs;
    std::deque<std::function<void()>> tasks;
    std::vector<std::thread> workers;
    std::thread sched;
    std::map<GroupKey, Group> groups;  // scheduler thread only
    uint64_t next_id = 1;
    int64_t reserved = 0;
    int slots_used = 0;
    int setups_in_flight = 0;
    bool stop = false, stop_workers = false;
    int64_t completed = 0;
    double dof_updates = 0, busy_s = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void push_task(dgw_server *S, std::function<void()> fn) {
    S->tasks.push_back(std::move(fn));
    S->cv_work.notify_one();
}

void finalize(dgw_server *S, Req *r, int status);

// Finish a request that never reached the device (under the lock).
void end_locked(dgw_server *S, Req *r, int status) {
    r->st = St::Done;
    r->res.status = status;
    r->res.t_finish = S->now();
    S->cv_done.notify_all();
}

void setup(dgw_server *S, Req *r);

// Admit pending requests in arrival order while slots and memory allow.
void admit_locked(dgw_server *S) {
    while (!S->pending.empty()) {
        Req *r = S->pending.front();
        if (r->cancel || S->stop) {
            S->pending.pop_front();
            end_locked(S, r, DGW_ECANCELLED);
            continue;
        }
        if (S->slots_used >= S->opts.max_slots || S->reserved + r->footprint > S->opts.hbm_budget_bytes) break;
        // queue the set-up first (it may throw; the worker waits for this
        // lock before it looks at the request)
        push_task(S, [S, r] { setup(S, r); });
        S->pending.pop_front();
        S->slots_used++;
        S->reserved += r->footprint;
        S->setups_in_flight++;
        r->st = St::Setup;
        r->res.t_admit = S->now();
    }
}

// Admission that never throws: a failed task allocation leaves the queue as
// it was, admission is retried at the next event.
void admit_nothrow(dgw_server *S) {
    try {
        admit_locked(S);
    } catch (...) {
    }
}

void setup(dgw_server *S, Req *r) {
    hipSetDevice(S->opts.device);
    int rc = DGW_OK;
    dgw_solver *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (r->cancel || S->stop) rc = DGW_ECANCELLED;
    }
    if (rc == DGW_OK) {
        dgw_mesh m{};
        m.dim = 2;
        m.n_verts = r->nv;
        m.vx = r->vx.data();
        m.vy = r->vy.data();
        m.n_elems = r->K;
        m.elem_verts = r->ev.data();
        m.eps = r->eps.empty() ? nullptr : r->eps.data();
        m.mu = r->mu.empty() ? nullptr : r->mu.data();
        dgw_opts o;
        dgw_opts_default(&o);
        o.alpha = r->alpha;
        o.prec = r->prec;
        o.device = S->opts.device;
        o.kernel = dgw::kVariantMfma;  // the batched launches run the fused-operand kernel on its buffers
        rc = dgw_create(&m, r->order, &o, &s);
        if (rc == DGW_OK) rc = r->q0.empty() ? dgw_set_cavity_mode(s, r->mode) : dgw_set_fields(s, r->q0.data());
        if (rc == DGW_OK) {
            int64_t n;
            double dt;
            dgw::steps_for(r->t_final, s->dt_cfl, &n, &dt);
            r->steps_left = n;
            r->dt = dt;
            r->res.steps = n;
            r->res.dt = dt;
        }
    }
    r->s = s;
    std::unique_lock<std::mutex> lk(S->mu);
    S->setups_in_flight--;
    if (rc == DGW_OK && !r->cancel && !S->stop) {
        r->st = St::Ready;
        S->ready.push_back(r);
    } else {
        lk.unlock();
        finalize(S, r, rc == DGW_OK ? DGW_ECANCELLED : rc);
        lk.lock();
    }
    S->cv_sched.notify_all();
}

// Reductions and download of a finished request, release of its memory.
void finalize(dgw_server *S, Req *r, int status) {
    hipSetDevice(S->opts.device);
    if (status == DGW_OK && r->s) {
        double e = 0;
        int rc = dgw_energy(r->s, &e);
        r->res.energy = e;
        r->res.rel_l2_mode = std::numeric_limits<double>::quiet_NaN();
        if (rc == DGW_OK && r->q0.empty() && r->uniform) {
            double err = 0;
            rc = dgw_cavity_error(r->s, r->mode, r->t_final, &err);
            r->res.rel_l2_mode = err;
        }
        if (rc == DGW_OK && r->keep) {
            try {
                r->fields.resize((size_t)3 * r->K * r->s->Np);
                rc = dgw_get_fields(r->s, r->fields.data());
            } catch (const std::bad_alloc &) {
                rc = DGW_ENOMEM;
            }
        }
        if (rc == DGW_OK && !std::isfinite(r->res.energy)) rc = DGW_ENONFINITE;
        status = rc;
    }
    if (r->s) {
        dgw_destroy(r->s);
        r->s = nullptr;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->reserved -= r->footprint;
    S->slots_used--;
    if (status == DGW_OK) S->completed++;
    end_locked(S, r, status);
    admit_nothrow(S);
    S->cv_sched.notify_all();
}

void worker_loop(dgw_server *S) {
    hipSetDevice(S->opts.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [&] { return S->stop_workers || !S->tasks.empty(); });
        if (S->tasks.empty()) return;  // stop_workers and drained
        auto fn = std::move(S->tasks.front());
        S->tasks.pop_front();
        lk.unlock();
        fn();  // tasks catch their own exceptions
        lk.lock();
    }
}

template <typename T>
int grow_pinned(T **h, T **d, size_t *cap, size_t n) {
    if (n <= *cap) return DGW_OK;
    size_t c = std::max<size_t>(n, 2 * *cap);
    if (*h) hipHostFree(*h);
    if (*d) hipFree(*d);
    *h = nullptr;
    *d = nullptr;
    *cap = 0;
    if (hipHostMalloc((void **)h, c * sizeof(T), hipHostMallocDefault) != hipSuccess) return DGW_ENOMEM;
    if (hipMalloc((void **)d, c * sizeof(T)) != hipSuccess) return DGW_ENOMEM;
    *cap = c;
    return DGW_OK;
}

// Issue `chunk` steps for every request of `batch` and wait for them.
int run_chunk(dgw_server *S, const std::vector<Req *> &batch, int64_t chunk) {
    std::map<GroupKey, std::vector<Req *>> by;
    for (Req *r : batch) by[GroupKey(r->order, r->s->material, r->alpha)].push_back(r);
    std::vector<std::pair<Group *, int>> launch;  // group, total tiles
    for (auto &kv : by) {
        Group &g = S->groups[kv.first];
        if (!g.stream) {
            g.order = std::get<0>(kv.first);
            g.material = std::get<1>(kv.first);
            g.alpha = std::get<2>(kv.first);
            // the fused-operand batched kernel at every order (a batched form
            // of the derivative-first kernel, which looks the owning request
            // up once per 16-element unit on its critical path, measured
            // slower in the serving mix: 4.07e10 against 4.47e10
            // DOF-updates/s, 96 requests in a burst)
            g.per_cu = dgw::blocks_per_cu_2d_batch(g.order, g.material);
            if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
                return dgw::set_error(DGW_EDEVICE, "stream creation failed");
        }
        if (!g.opsfrag_d) {
            // the operator depends on the order only: copy it from the first
            // solve of the group (its upload completed in dgw_create)
            const dgw_solver *s0 = kv.second.front()->s;
            const size_t n = (size_t)dgw::opsfrag2d(g.order, nullptr, nullptr, nullptr, nullptr);
            const float *src = s0->opsfrag_d;
            if (!src) return dgw::set_error(DGW_EINVAL, "internal: operator fragments missing");
            if (hipMalloc((void **)&g.opsfrag_d, n * sizeof(float)) != hipSuccess) {
                g.opsfrag_d = nullptr;
                return dgw::set_error(DGW_ENOMEM, "operator table allocation failed");
            }
            if (hipMemcpyAsync(g.opsfrag_d, src, n * sizeof(float), hipMemcpyDeviceToDevice, g.stream) != hipSuccess)
                return dgw::set_error(DGW_EDEVICE, "operator table copy failed");
        }
        auto &rs = kv.second;
        std::sort(rs.begin(), rs.end(), [](const Req *a, const Req *b) { return a->id < b->id; });
        size_t tiles = 0;
        for (Req *r : rs) tiles += (size_t)(r->s->Kp / dgw::kTile);
        if (grow_pinned(&g.desc_h, &g.desc_d, &g.cap_desc, rs.size()) ||
            grow_pinned(&g.tiles_h, &g.tiles_d, &g.cap_tiles, tiles))
            return dgw::set_error(DGW_ENOMEM, "batch table allocation failed");
        int t0 = 0;
        for (size_t i = 0; i < rs.size(); ++i) {
            dgw_solver *s = rs[i]->s;
            dgw::BatchDesc &d = g.desc_h[i];
            d.q[0] = s->q[0];
            d.q[1] = s->q[1];
            d.res = s->res;
            d.geo = s->geo_d;
            d.fgeo = s->fgeo_d;
            d.nbr = s->nbr_d;
            d.tile0 = t0;
            d.cur0 = s->cur;
            d.dt = (float)rs[i]->dt;
            d.pad_ = 0.f;
            const int nt = (int)(s->Kp / dgw::kTile);
            for (int t = 0; t < nt; ++t) g.tiles_h[t0 + t] = (int)i;
            t0 += nt;
        }
        if (hipMemcpyAsync(g.desc_d, g.desc_h, rs.size() * sizeof(dgw::BatchDesc), hipMemcpyHostToDevice,
                           g.stream) != hipSuccess ||
            hipMemcpyAsync(g.tiles_d, g.tiles_h, tiles * sizeof(int), hipMemcpyHostToDevice, g.stream) != hipSuccess)
            return dgw::set_error(DGW_EDEVICE, "batch table upload failed");
        launch.emplace_back(&g, (int)tiles);
    }
    for (int64_t st = 0; st < chunk; ++st)
        for (int k = 0; k < 5; ++k)
            for (auto &gl : launch) {
                Group &g = *gl.first;
                dgw::StageArgs a{};
                a.batch = g.desc_d;
                a.tile_req = g.tiles_d;
                a.opsfrag = g.opsfrag_d;
                a.parity = (int)((5 * st + k) & 1);
                a.ntiles = gl.second;
                int ng = std::max(1, S->ncu) * g.per_cu;
                ng = std::min(ng, (gl.second + 7) / 8 * 8);
                a.ngroups = std::max(8, ng / 8 * 8);
                a.a = (float)dgw::kRkA[k];
                a.b = (float)dgw::kRkB[k];
                a.alpha = (float)g.alpha;
                hipError_t e = dgw::launch_stage2d_batch(g.order, g.material, a, g.stream);
                if (e != hipSuccess) return dgw::set_error(DGW_EDEVICE, hipGetErrorString(e));
            }
    for (auto &gl : launch) {
        if (hipEventRecord(gl.first->done, gl.first->stream) != hipSuccess ||
            hipEventSynchronize(gl.first->done) != hipSuccess)
            return dgw::set_error(DGW_EDEVICE, "batch synchronisation failed");
    }
    return DGW_OK;
}

void sched_loop(dgw_server *S) {
    hipSetDevice(S->opts.device);
    std::unique_lock<std::mutex> lk(S->mu);
    // hand a request that leaves the device to a worker (or finish it here
    // if the task cannot be queued)
    auto hand_off = [&](Req *r, int st) {
        try {
            push_task(S, [S, r, st] { finalize(S, r, st); });
        } catch (...) {
            lk.unlock();
            finalize(S, r, st);
            lk.lock();
        }
    };
    for (;;) {
        S->cv_sched.wait(lk, [&] {
            return !S->ready.empty() || !S->running.empty() || (S->stop && S->setups_in_flight == 0);
        });
        // newcomers join; cancelled or (on stop) all requests leave
        const double now = S->now();
        std::vector<Req *> leaving;
        for (Req *r : S->ready) {
            r->st = St::Running;
            r->res.t_start = now;
            S->running.push_back(r);
        }
        S->ready.clear();
        for (size_t i = 0; i < S->running.size();) {
            Req *r = S->running[i];
            if (r->cancel || S->stop) {
                leaving.push_back(r);
                S->running.erase(S->running.begin() + i);
            } else {
                ++i;
            }
        }
        for (Req *r : leaving) hand_off(r, DGW_ECANCELLED);
        if (S->running.empty()) {
            if (S->stop && S->setups_in_flight == 0 && S->ready.empty()) return;
            continue;
        }
        int64_t chunk = S->opts.max_chunk_steps;
        for (Req *r : S->running) chunk = std::min(chunk, r->steps_left);
        std::vector<Req *> batch = S->running;
        lk.unlock();
        const auto c0 = Clock::now();
        int rc = chunk > 0 ? run_chunk(S, batch, chunk) : DGW_OK;
        const double el = std::chrono::duration<double>(Clock::now() - c0).count();
        lk.lock();
        S->busy_s += el;
        for (size_t i = 0; i < S->running.size();) {
            Req *r = S->running[i];
            bool leave = false;
            if (rc != DGW_OK) {
                leave = true;
            } else {
                S->dof_updates += 3.0 * (double)r->K * r->s->Np * (double)chunk;
                r->steps_left -= chunk;
                if (chunk & 1) r->s->cur ^= 1;
                r->s->t += chunk * r->dt;
                leave = r->steps_left == 0;
            }
            if (leave) {
                hand_off(r, rc);
                S->running.erase(S->running.begin() + i);
            } else {
                ++i;
            }
        }
    }
}

}  // namespace

extern "C" {

int dgw_footprint(const dgw_mesh *mesh, int32_t order, const dgw_opts *opts, int64_t *bytes) {
    if (!mesh || !bytes) return dgw::set_error(DGW_EINVAL, "NULL argument");
    if (mesh->dim != 2 && mesh->dim != 3) return dgw::set_error(DGW_EINVAL, "dim must be 2 or 3");
    if (order < 1 || order > (mesh->dim == 2 ? 8 : 4))
        return dgw::set_error(DGW_EORDER, "order must be in 1..8 (2D) or 1..4 (3D)");
    if (mesh->n_elems <= 0) return dgw::set_error(DGW_EINVAL, "empty mesh");
    bool material = false;
    for (int64_t k = 0; k < mesh->n_elems && !material; ++k)
        material = (mesh->eps && mesh->eps[k] != 1.0) || (mesh->mu && mesh->mu[k] != 1.0);
    const int prec = opts ? opts->prec : DGW_FP32;
    *bytes = dgw::solver_footprint(mesh->dim, order, mesh->n_elems, material, prec);
    return DGW_OK;
}

int dgw_server_create(const dgw_server_opts *opts, dgw_server **out) {
    if (!out) return dgw::set_error(DGW_EINVAL, "NULL output handle");
    *out = nullptr;
    dgw_server *S = new (std::nothrow) dgw_server();
    if (!S) return dgw::set_error(DGW_ENOMEM, "host allocation failed");
    if (opts) S->opts = *opts;
    if (S->opts.max_slots <= 0) S->opts.max_slots = 64;
    if (S->opts.setup_threads <= 0) S->opts.setup_threads = 4;
    if (S->opts.max_chunk_steps <= 0) S->opts.max_chunk_steps = 64;
    if (hipSetDevice(S->opts.device) != hipSuccess ||
        hipDeviceGetAttribute(&S->ncu, hipDeviceAttributeMultiprocessorCount, S->opts.device) != hipSuccess) {
        delete S;
        return dgw::set_error(DGW_EDEVICE, "cannot use the requested device");
    }
    if (S->opts.hbm_budget_bytes <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete S;
            return dgw::set_error(DGW_EDEVICE, "hipMemGetInfo failed");
        }
        S->opts.hbm_budget_bytes = (int64_t)(0.8 * (double)fr);
    }
    S->t0 = Clock::now();
    try {
        for (int i = 0; i < S->opts.setup_threads; ++i) S->workers.emplace_back(worker_loop, S);
        S->sched = std::thread(sched_loop, S);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->stop_workers = true;
        }
        S->cv_sched.notify_all();
        S->cv_work.notify_all();
        if (S->sched.joinable()) S->sched.join();
        for (auto &w : S->workers)
            if (w.joinable()) w.join();
        delete S;
        return dgw::set_error(DGW_ENOMEM, "thread creation failed");
    }
    *out = S;
    return DGW_OK;
}

int dgw_submit(dgw_server *S, const dgw_request *q, uint64_t *ticket) {
    if (!S || !q || !ticket) return dgw::set_error(DGW_EINVAL, "NULL argument");
    const dgw_mesh &m = q->mesh;
    if (m.dim != 2) return dgw::set_error(DGW_EINVAL, "the server runs 2D solves");
    if (!m.vx || !m.vy || !m.elem_verts || m.n_verts <= 0 || m.n_elems <= 0)
        return dgw::set_error(DGW_EINVAL, "empty mesh or NULL mesh array");
    if (m.n_elems >= (int64_t(1) << 26)) return dgw::set_error(DGW_ETOOBIG, "more than 2^26 elements");
    if (q->order < 1 || q->order > 8) return dgw::set_error(DGW_EORDER, "order must be in 1..8");
    if (!dgw::fits_index32_2d(q->order, m.n_elems))
        return dgw::set_error(DGW_ETOOBIG, "2D field arrays are limited to 2^32 values (32-bit partner-trace indices)");
    if (!(q->t_final > 0) || !std::isfinite(q->t_final)) return dgw::set_error(DGW_EINVAL, "t_final must be > 0");
    if (!(q->alpha >= 0.0 && q->alpha <= 1.0)) return dgw::set_error(DGW_EINVAL, "alpha must be in [0, 1]");
    if (q->prec != DGW_FP32) return dgw::set_error(DGW_EINVAL, "the server runs the FP32 path");
    Req *r = new (std::nothrow) Req();
    if (!r) return dgw::set_error(DGW_ENOMEM, "host allocation failed");
    try {
        r->nv = m.n_verts;
        r->K = m.n_elems;
        r->vx.assign(m.vx, m.vx + m.n_verts);
        r->vy.assign(m.vy, m.vy + m.n_verts);
        r->ev.assign(m.elem_verts, m.elem_verts + 3 * m.n_elems);
        if (m.eps) r->eps.assign(m.eps, m.eps + m.n_elems);
        if (m.mu) r->mu.assign(m.mu, m.mu + m.n_elems);
        const int Np = (q->order + 1) * (q->order + 2) / 2;
        if (q->q0) r->q0.assign(q->q0, q->q0 + (size_t)3 * m.n_elems * Np);
    } catch (const std::bad_alloc &) {
        delete r;
        return dgw::set_error(DGW_ENOMEM, "host allocation failed");
    }
    for (int64_t k = 0; k < r->K; ++k) {
        const double e = r->eps.empty() ? 1.0 : r->eps[k], u = r->mu.empty() ? 1.0 : r->mu[k];
        if (e != 1.0 || u != 1.0) r->material = true;
        if (k > 0 && (e != (r->eps.empty() ? 1.0 : r->eps[0]) || u != (r->mu.empty() ? 1.0 : r->mu[0])))
            r->uniform = false;
    }
    r->order = q->order;
    std::memcpy(r->mode, q->mode, sizeof(r->mode));
    r->t_final = q->t_final;
    r->alpha = q->alpha;
    r->prec = q->prec;
    r->keep = q->keep_fields != 0;
    r->footprint = dgw::solver_footprint(2, r->order, r->K, r->material, r->prec);
    r->res.order = r->order;
    r->res.K = r->K;
    r->res.footprint_bytes = r->footprint;
    r->res.rel_l2_mode = std::numeric_limits<double>::quiet_NaN();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        return dgw::set_error(DGW_ECANCELLED, "server is shutting down");
    }
    try {
        S->reqs.reserve(S->reqs.size() + 1);
    } catch (const std::bad_alloc &) {
        delete r;
        return dgw::set_error(DGW_ENOMEM, "host allocation failed");
    }
    if (r->footprint > S->opts.hbm_budget_bytes) {
        const int64_t fp = r->footprint;
        delete r;
        return dgw::set_error(DGW_ETOOBIG, "request footprint " + std::to_string(fp) + " B exceeds the HBM budget");
    }
    r->id = S->next_id++;
    r->res.t_arrival = S->now();
    try {
        S->reqs[r->id] = r;
        S->pending.push_back(r);
    } catch (const std::bad_alloc &) {
        S->reqs.erase(r->id);
        delete r;
        return dgw::set_error(DGW_ENOMEM, "host allocation failed");
    }
    *ticket = r->id;
    admit_nothrow(S);  // may queue set-up tasks
    return DGW_OK;
}

int dgw_poll(dgw_server *S, uint64_t ticket, int32_t *done) {
    if (!S || !done) return dgw::set_error(DGW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return dgw::set_error(DGW_ENOTFOUND, "unknown ticket");
    *done = it->second->st == St::Done ? 1 : 0;
    return DGW_OK;
}

int dgw_wait(dgw_server *S, uint64_t ticket, double *q_out, dgw_result *res) {
    if (!S) return dgw::set_error(DGW_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return dgw::set_error(DGW_ENOTFOUND, "unknown ticket");
    if (q_out && !it->second->keep) return dgw::set_error(DGW_EINVAL, "fields requested but keep_fields was 0");
    // look the ticket up again on every wake-up: another thread waiting on
    // the same ticket may have collected it meanwhile
    S->cv_done.wait(lk, [&] {
        it = S->reqs.find(ticket);
        return it == S->reqs.end() || it->second->st == St::Done;
    });
    if (it == S->reqs.end()) return dgw::set_error(DGW_ENOTFOUND, "ticket collected by another caller");
    Req *r = it->second;
    if (res) *res = r->res;
    if (q_out && r->res.status == DGW_OK) std::copy(r->fields.begin(), r->fields.end(), q_out);
    const int status = r->res.status;
    S->reqs.erase(it);
    delete r;
    if (status != DGW_OK && status != DGW_ECANCELLED) dgw::set_error(status, "request failed");
    return status;
}

int dgw_cancel(dgw_server *S, uint64_t ticket) {
    if (!S) return dgw::set_error(DGW_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return dgw::set_error(DGW_ENOTFOUND, "unknown ticket");
    Req *r = it->second;
    if (r->st == St::Done) return DGW_OK;
    r->cancel = true;
    if (r->st == St::Pending) {
        S->pending.erase(std::find(S->pending.begin(), S->pending.end(), r));
        end_locked(S, r, DGW_ECANCELLED);
        admit_nothrow(S);
    }
    S->cv_sched.notify_all();
    return DGW_OK;
}

int dgw_server_stats(dgw_server *S, int64_t *completed, double *dof_updates, double *busy_s) {
    if (!S) return dgw::set_error(DGW_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (completed) *completed = S->completed;
    if (dof_updates) *dof_updates = S->dof_updates;
    if (busy_s) *busy_s = S->busy_s;
    return DGW_OK;
}

void dgw_server_destroy(dgw_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto &kv : S->reqs) kv.second->cancel = true;
        admit_nothrow(S);  // ends every pending request as cancelled (no task is queued on stop)
    }
    S->cv_sched.notify_all();
    if (S->sched.joinable()) S->sched.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop_workers = true;
    }
    S->cv_work.notify_all();
    for (auto &w : S->workers)
        if (w.joinable()) w.join();
    hipSetDevice(S->opts.device);
    for (auto &kv : S->groups) {
        Group &g = kv.second;
        if (g.desc_h) hipHostFree(g.desc_h);
        if (g.tiles_h) hipHostFree(g.tiles_h);
        if (g.desc_d) hipFree(g.desc_d);
        if (g.tiles_d) hipFree(g.tiles_d);
        if (g.opsfrag_d) hipFree(g.opsfrag_d);
        if (g.done) hipEventDestroy(g.done);
        if (g.stream) hipStreamDestroy(g.stream);
    }
    for (auto &kv : S->reqs) {
        if (kv.second->s) dgw_destroy(kv.second->s);
        delete kv.second;
    }
    delete S;
}

}  // extern "C"
