// Serving runtime: concurrent geodesic queries over resident meshes.
//
// A server owns n_slots worker threads, each with its own HIP stream
// (default priority).  Submitted queries wait in a FIFO; a free worker takes
// the first one that can be admitted and runs the whole query on its stream
// with a workspace from the query mesh's pool.  So queries that arrive while
// others are running start as soon as a slot and memory are free, and their
// kernels overlap on the device with the running ones (continuous admission;
// each query's arithmetic is the same as alone, since workspaces are private
// and the mesh data is read-only).
//
// Admission by device memory: workspaces are pooled per mesh and kept for
// later queries on that mesh.  A query whose mesh has a free workspace is
// admitted at once; otherwise a new workspace is created only if the bytes
// held by all workspaces plus the estimate for the new one stay within the
// budget.  For the oldest waiting query, idle workspaces of other meshes are
// released (least recently used first) to make room; later queries that
// fit may go ahead of it meanwhile.  When nothing is running, the oldest
// query is always admitted, so one query larger than the budget completes.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "hgeo_internal.h"

namespace hg {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Upper estimate of a query workspace (bytes), from the buffers the stages
// allocate: breadth-first sets and pairing, two (v, e) copies, 1/D, log u,
// h, the form's double-buffered ADMM state, outputs, integration pairs and
// pointer-jumping parents, plus the source paths (bounded by nsrc * depth).
uint64_t work_estimate(const Mesh& m, int form, int nsrc) {
    const uint64_t nv = m.nv, nf = m.nf, ne = m.ne;
    uint64_t b = 24 * nv          // level, parent, pedge, two frontiers, counters
                 + 24 * nv + 8 * nv + 8 * nv   // v0, v1, invD; e0, e1; logu
                 + 12 * nf + 4 * ne           // h, target sums
                 + 4 * ne + 12 * nf           // xe, gf
                 + 16 * nv + 8 * nv + 4 * nv  // shi/slo pairs, jp0/jp1, dprev
                 + 6 * (uint64_t)m.n_patches  // tile marks of the tiled search, ADMM tile flags
                 + nv / 256 + 1               // per vertex block: its share of a check
                 + 18 * (uint64_t)std::max(1, m.n_comp);   // per component: check maxima, flags
    if (form == HG_FORM_EDGE)
        b += 36 * nf;                          // zeta per slot (double-buffered) and S per slot
    else
        b += 48 * ne + 24 * nf;                // z copies and g, double-buffered
    if (nsrc > 1) b += (uint64_t)nsrc * 4096 * 64 + 8 * ne;
    return b + (1u << 20);
}

struct Request {
    int64_t ticket;
    Mesh* mesh;
    std::vector<int32_t> src;
    double t;
    hg_opts opts;
    bool has_opts;
    float* d_dev;
    double t_submit;
};

struct Server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<hg_result> done;
    struct Pooled {
        std::unique_ptr<Work> w;
        uint64_t bytes;
        uint64_t last_use;
    };
    std::map<Mesh*, std::vector<Pooled>> free_ws;   // idle workspaces per mesh
    uint64_t held_bytes = 0;    // workspaces alive (idle or in use: the larger of their
                                // admission estimate and their size after their last query),
                                // plus mesh_growth
    uint64_t mesh_growth = 0;   // schedules that served queries added to their meshes
    uint64_t use_clock = 0;
    uint64_t budget = 0;
    int running = 0;
    int64_t next_ticket = 1;
    bool stop = false;
    int device = 0;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    uint64_t idle_bytes() const {
        uint64_t b = 0;
        for (auto& kv : free_ws)
            for (auto& p : kv.second) b += p.bytes;
        return b;
    }

    // moves the least recently used idle workspace into *out; false if none
    bool evict_one(std::vector<std::unique_ptr<Work>>* out) {
        Mesh* best = nullptr;
        size_t bi = 0;
        uint64_t bu = ~0ull;
        for (auto& kv : free_ws)
            for (size_t i = 0; i < kv.second.size(); ++i)
                if (kv.second[i].last_use < bu) {
                    bu = kv.second[i].last_use;
                    best = kv.first;
                    bi = i;
                }
        if (!best) return false;
        auto& v = free_ws[best];
        held_bytes -= v[bi].bytes;
        out->push_back(std::move(v[bi].w));
        v.erase(v.begin() + bi);
        return true;
    }

    // index of the first admissible pending request, -1 if none.  *reuse:
    // a pooled workspace is available for it; *need: bytes of a new one.
    // Idle workspaces released for the oldest request go to *evicted (freed
    // by the caller outside the lock).
    int pick(bool* reuse, uint64_t* need, std::vector<std::unique_ptr<Work>>* evicted) {
        for (size_t i = 0; i < pending.size(); ++i) {
            Request& r = pending[i];
            auto it = free_ws.find(r.mesh);
            if (it != free_ws.end() && !it->second.empty()) {
                *reuse = true;
                return (int)i;
            }
            const int form = r.has_opts ? r.opts.formulation : HG_FORM_EDGE;
            *need = work_estimate(*r.mesh, form, (int)r.src.size());
            *reuse = false;
            if (held_bytes + *need <= budget) return (int)i;
            if (i == 0) {
                const bool fits_after = held_bytes - idle_bytes() + *need <= budget;
                if (fits_after || running == 0) {
                    while (held_bytes + *need > budget && evict_one(evicted)) {
                    }
                    return 0;
                }
            }
        }
        return -1;
    }

    void worker(int slot) {
        (void)hipSetDevice(device);
        hipStream_t s = streams[slot];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool reuse = false;
            uint64_t need = 0;
            int idx = -1;
            std::vector<std::unique_ptr<Work>> evicted;
            cv_work.wait(lk, [&] {
                return (idx = pick(&reuse, &need, &evicted)) >= 0 || (stop && pending.empty());
            });
            if (idx < 0) return;   // stopping, nothing left
            Request r = std::move(pending[idx]);
            pending.erase(pending.begin() + idx);
            Pooled w;
            if (reuse) {
                auto& v = free_ws[r.mesh];
                w = std::move(v.back());
                v.pop_back();
            } else {
                held_bytes += need;
                w.w.reset(new Work());
                w.bytes = need;
            }
            ++running;
            lk.unlock();
            evicted.clear();   // frees the released workspaces' device memory

            hg_result res;
            std::memset(&res, 0, sizeof(res));
            res.ticket = r.ticket;
            res.t_submit = r.t_submit;
            res.t_start = now_s();
            const uint64_t mesh_before = r.mesh->mesh_bytes();
            try {
                (void)hipSetDevice(r.mesh->device);
                QueryOutcome q = solve_query(*r.mesh, *w.w, r.src.data(), (int32_t)r.src.size(), r.t,
                                             r.has_opts ? &r.opts : nullptr, r.d_dev, s, &res.info);
                res.status = q.status;
            } catch (const Error& e) {
                res.status = e.code;
            } catch (const std::bad_alloc&) {
                res.status = HG_E_OOM;
            } catch (...) {
                res.status = HG_E_DEVICE;
            }
            res.t_end = now_s();

            // what the query really holds: a pooled workspace grows past the
            // estimate it was admitted with when a larger query (more
            // sources, the other form) reuses it, and a query may build
            // schedules the mesh keeps (the blocked-ADMM face tiles, the
            // face form's slot geometry); both count against the budget
            const uint64_t actual = std::max<uint64_t>(w.bytes, w.w->bytes());
            const uint64_t mesh_after = r.mesh->mesh_bytes();
            lk.lock();
            held_bytes += actual - w.bytes;
            w.bytes = actual;
            if (mesh_after > mesh_before) {
                held_bytes += mesh_after - mesh_before;
                mesh_growth += mesh_after - mesh_before;
            }
            --running;
            w.last_use = ++use_clock;
            free_ws[r.mesh].push_back(std::move(w));
            done.push_back(res);
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

}  // namespace hg

using namespace hg;

extern "C" {

hg_status hg_server_create(int32_t n_slots, uint64_t workspace_budget, hg_server_t* out) {
    if (!out || n_slots <= 0 || n_slots > 64) return HG_E_INVALID_ARG;
    *out = nullptr;
    try {
        std::unique_ptr<Server> sv(new Server());
        if (hipGetDevice(&sv->device) != hipSuccess) return HG_E_DEVICE;
        if (workspace_budget == 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return HG_E_DEVICE;
            workspace_budget = fr / 2;
        }
        sv->budget = workspace_budget;
        for (int i = 0; i < n_slots; ++i) {
            hipStream_t s;
            if (hipStreamCreate(&s) != hipSuccess) {
                for (auto x : sv->streams) (void)hipStreamDestroy(x);
                return HG_E_DEVICE;
            }
            sv->streams.push_back(s);
        }
        Server* raw = sv.get();
        for (int i = 0; i < n_slots; ++i) sv->workers.emplace_back([raw, i] { raw->worker(i); });
        *out = reinterpret_cast<hg_server_t>(sv.release());
        return HG_OK;
    } catch (...) {
        return HG_E_DEVICE;
    }
}

hg_status hg_server_submit(hg_server_t server, hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t,
                           const hg_opts* opts, float* d_dev, int64_t* ticket) {
    if (!server || !mesh || !src || nsrc <= 0 || !d_dev) return HG_E_INVALID_ARG;
    auto* sv = reinterpret_cast<Server*>(server);
    auto* m = reinterpret_cast<Mesh*>(mesh);
    for (int32_t i = 0; i < nsrc; ++i)
        if (src[i] < 0 || src[i] >= m->nv) return HG_E_INVALID_ARG;
    Request r;
    r.mesh = m;
    r.src.assign(src, src + nsrc);
    r.t = t;
    r.has_opts = opts != nullptr;
    if (opts) r.opts = *opts;
    r.d_dev = d_dev;
    r.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return HG_E_INVALID_ARG;
        r.ticket = sv->next_ticket++;
        if (ticket) *ticket = r.ticket;
        sv->pending.push_back(std::move(r));
    }
    sv->cv_work.notify_all();
    return HG_OK;
}

hg_status hg_server_wait(hg_server_t server, hg_result* out, int32_t timeout_ms) {
    if (!server || !out) return HG_E_INVALID_ARG;
    auto* sv = reinterpret_cast<Server*>(server);
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return !sv->done.empty(); };
    if (timeout_ms < 0)
        sv->cv_done.wait(lk, ready);
    else
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (sv->done.empty()) {
        std::memset(out, 0, sizeof(*out));
        out->ticket = -1;
        return HG_OK;
    }
    *out = sv->done.front();
    sv->done.pop_front();
    return HG_OK;
}

hg_status hg_server_stats(hg_server_t server, hg_server_stats_t* st) {
    if (!server || !st) return HG_E_INVALID_ARG;
    auto* sv = reinterpret_cast<Server*>(server);
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(st, 0, sizeof(*st));
    st->pending = (int32_t)sv->pending.size();
    st->running = sv->running;
    st->completed_unread = (int32_t)sv->done.size();
    st->n_slots = (int32_t)sv->workers.size();
    st->workspace_bytes_held = sv->held_bytes;
    st->workspace_budget = sv->budget;
    int nw = 0;
    for (auto& kv : sv->free_ws) nw += (int)kv.second.size();
    st->workspace_bytes_idle = sv->idle_bytes();
    st->workspaces_idle = nw;
    return HG_OK;
}

double hg_server_clock(void) { return now_s(); }

void hg_server_destroy(hg_server_t server) {
    if (!server) return;
    auto* sv = reinterpret_cast<Server*>(server);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto& th : sv->workers) th.join();
    for (auto s : sv->streams) (void)hipStreamDestroy(s);
    delete sv;
}

}  // extern "C"
