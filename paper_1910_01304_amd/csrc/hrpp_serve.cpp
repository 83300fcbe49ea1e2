// Serving loop of the HRPP library: continuous batching of ray-query
// requests against device-resident BVHs and predictor tables.
//
// A scheduler thread admits queued requests when (1) their rays and results
// fit in the device pool the caller provided (the HBM budget for in-flight
// requests), (2) a stream slot is free, and (3) a predictor replica of the
// request's (scene, query kind) is free.  An admitted request is copied in,
// traced and copied back on its slot's stream; completion is observed with
// a HIP event.  Requests on different slots run concurrently on the device,
// and new requests are admitted as slots and pool space free up.
//
// Only queries whose results do not depend on the table are served: any-hit
// and EXACT closest-hit.  A request's results are therefore the same alone
// and in any mix, while the tables (which persist across requests and make
// later requests cheaper) evolve with the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hrpp.h"
#include "hrpp_internal.h"
#include "pool_alloc.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id;
    uint32_t scene, query, n;
    const hrpp_ray *h_rays;
    void *h_out;
    size_t ray_bytes, out_bytes;
    Clock::time_point t_submit, t_admit, t_done;
    // while running
    int slot = -1;
    int replica = -1;
    size_t pool_off = 0;
    hipEvent_t done_event = nullptr;
    bool done = false;
    hrpp_status status = HRPP_OK;
};

}  // namespace

struct hrpp_server {
    struct Scene {
        const hrpp_bvh *bvh;
        std::vector<hrpp_predictor *> preds[2];   // [0] hit-any, [1] hit-all
        std::vector<bool> busy[2];
        bool removed = false;                     // no new requests; slot kept so indices stay stable
    };

    // Requests of `scene` still queued or running (caller holds mu).
    bool scene_busy(uint32_t scene) const {
        for (const Request *r : queue)
            if (r->scene == scene) return true;
        for (const Request *r : running)
            if (r->scene == scene) return true;
        return false;
    }
    std::vector<Scene> scenes;
    std::vector<hipStream_t> streams;
    std::vector<bool> slot_busy;
    char *d_pool = nullptr;
    hrpp::PoolAllocator pool;
    std::deque<Request *> queue;
    std::vector<Request *> running;
    // every request not yet retired: queued, running, or done and not yet
    // read by its final poll
    std::map<uint64_t, Request *> all;
    hrpp_status first_error = HRPP_OK;   // first failed request since creation
    uint64_t next_id = 1;
    size_t peak_pool = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<bool> stop{false};
    std::thread worker;
    int device = 0;

    explicit hrpp_server(size_t pool_bytes) : pool(pool_bytes) {}

    bool admit_one(Request *r) {
        Scene &sc = scenes[r->scene];
        const int kind = r->query == 0 ? 0 : 1;
        int slot = -1, rep = -1;
        for (size_t i = 0; i < slot_busy.size(); i++)
            if (!slot_busy[i]) { slot = (int)i; break; }
        for (size_t i = 0; i < sc.busy[kind].size(); i++)
            if (!sc.busy[kind][i]) { rep = (int)i; break; }
        if (slot < 0 || rep < 0) return false;
        size_t off = 0;
        if (!pool.alloc(r->ray_bytes + hrpp::align256(r->out_bytes) + 256, off)) return false;
        peak_pool = std::max(peak_pool, pool.used());
        slot_busy[slot] = true;
        sc.busy[kind][rep] = true;
        r->slot = slot;
        r->replica = rep;
        r->pool_off = off;
        r->t_admit = Clock::now();
        hipStream_t s = streams[slot];
        char *d_rays = d_pool + off;
        char *d_out = d_rays + hrpp::align256(r->ray_bytes);
        hipError_t e = hipMemcpyAsync(d_rays, r->h_rays, r->ray_bytes, hipMemcpyHostToDevice, s);
        hrpp_status st = e == hipSuccess ? HRPP_OK : HRPP_EDEVICE;
        hrpp_predictor *p = sc.preds[kind][rep];
        if (st == HRPP_OK) {
            if (r->query == 0)
                st = hrpp_trace_anyhit(sc.bvh, p, reinterpret_cast<const hrpp_ray *>(d_rays), r->n,
                                       reinterpret_cast<uint8_t *>(d_out), nullptr, s);
            else
                st = hrpp_trace_closest(sc.bvh, p, reinterpret_cast<const hrpp_ray *>(d_rays), r->n,
                                        HRPP_CLOSEST_EXACT, reinterpret_cast<hrpp_hit *>(d_out), nullptr, s);
        }
        if (st == HRPP_OK && hipMemcpyAsync(r->h_out, d_out, r->out_bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = HRPP_EDEVICE;
        if (st == HRPP_OK && (hipEventCreateWithFlags(&r->done_event, hipEventDisableTiming) != hipSuccess ||
                              hipEventRecord(r->done_event, s) != hipSuccess))
            st = HRPP_EDEVICE;
        r->status = st;
        running.push_back(r);
        return true;
    }

    void finish(Request *r) {
        Scene &sc = scenes[r->scene];
        const int kind = r->query == 0 ? 0 : 1;
        if (r->status != HRPP_OK) {
            // a failed request may have copies or kernels in flight on its
            // slot: let them end before its pool region, slot and replica are
            // reused, and reset the replica if its trace did not launch
            hipStream_t s = streams[r->slot];
            (void)hipStreamSynchronize(s);
            hrpp_predictor *p = sc.preds[kind][r->replica];
            if (p->scratch_dirty && hrpp_predictor_reset(p, s) == HRPP_OK) (void)hipStreamSynchronize(s);
            if (first_error == HRPP_OK) first_error = r->status;
        }
        slot_busy[r->slot] = false;
        sc.busy[kind][r->replica] = false;
        pool.release(r->pool_off, r->ray_bytes + hrpp::align256(r->out_bytes) + 256);
        if (r->done_event) (void)hipEventDestroy(r->done_event);
        r->done_event = nullptr;
        r->t_done = Clock::now();
        r->done = true;
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool progress = false;
            // completions
            for (size_t i = 0; i < running.size();) {
                Request *r = running[i];
                const bool failed = r->status != HRPP_OK;
                if (failed || !r->done_event || hipEventQuery(r->done_event) == hipSuccess) {
                    finish(r);
                    running[i] = running.back();
                    running.pop_back();
                    progress = true;
                } else {
                    i++;
                }
            }
            // admissions: in arrival order; a request blocked only by a busy
            // replica does not hold back the ones behind it, one blocked by pool
            // space does (so large requests cannot starve)
            for (auto it = queue.begin(); it != queue.end();) {
                Request *r = *it;
                const int kind = r->query == 0 ? 0 : 1;
                bool replica_free = false;
                for (bool b : scenes[r->scene].busy[kind]) replica_free |= !b;
                bool slot_free = false;
                for (bool b : slot_busy) slot_free |= !b;
                if (!slot_free) break;
                if (!replica_free) { ++it; continue; }
                if (!admit_one(r)) break;   // pool full
                it = queue.erase(it);
                progress = true;
            }
            if (progress) cv.notify_all();
            if (stop && queue.empty() && running.empty()) break;
            if (!progress) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(running.empty() && queue.empty() ? 200 : 10));
                lk.lock();
            }
        }
    }
};

namespace {

// Validates one scene description: a device-resident BVH, at least one
// predictor per query kind, each bound to this BVH and not yet used (in
// `seen`, which it extends).
hrpp_status make_scene(const hrpp_serve_scene &s, std::vector<const hrpp_predictor *> &seen,
                       hrpp_server::Scene &sc) {
    if (!s.bvh || !s.bvh->d_nodes || s.n_any == 0 || s.n_closest == 0 || !s.any_preds || !s.closest_preds)
        return HRPP_EINVAL;
    sc.bvh = s.bvh;
    for (int kind = 0; kind < 2; kind++) {
        const uint32_t cnt = kind == 0 ? s.n_any : s.n_closest;
        hrpp_predictor *const *ps = kind == 0 ? s.any_preds : s.closest_preds;
        for (uint32_t k = 0; k < cnt; k++) {
            hrpp_predictor *p = ps[k];
            if (!p || p->bvh_uid != s.bvh->uid || std::find(seen.begin(), seen.end(), p) != seen.end())
                return HRPP_EINVAL;   // a predictor serves exactly one scene and one replica slot
            seen.push_back(p);
            sc.preds[kind].push_back(p);
            sc.busy[kind].push_back(false);
        }
    }
    return HRPP_OK;
}

}  // namespace

extern "C" {

hrpp_status hrpp_serve_create(const hrpp_serve_scene *scenes, uint32_t nscenes, uint32_t slots, void *d_pool,
                              size_t pool_bytes, hrpp_server **out) {
    if (!scenes || nscenes == 0 || slots == 0 || slots > 64 || !d_pool || pool_bytes < 4096 || !out)
        return HRPP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_pool) % 256) return HRPP_EINVAL;
    *out = nullptr;
    hrpp_server *sv = new (std::nothrow) hrpp_server(pool_bytes);
    if (!sv) return HRPP_ENOMEM;
    std::vector<const hrpp_predictor *> seen;
    for (uint32_t i = 0; i < nscenes; i++) {
        hrpp_server::Scene sc;
        if (make_scene(scenes[i], seen, sc) != HRPP_OK) {
            delete sv;
            return HRPP_EINVAL;
        }
        sv->scenes.push_back(sc);
    }
    (void)hipGetDevice(&sv->device);
    for (uint32_t i = 0; i < slots; i++) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
            delete sv;
            return HRPP_EDEVICE;
        }
        sv->streams.push_back(st);
        sv->slot_busy.push_back(false);
    }
    sv->d_pool = static_cast<char *>(d_pool);
    sv->worker = std::thread([sv] { sv->loop(); });
    *out = sv;
    return HRPP_OK;
}

hrpp_status hrpp_serve_add_scene(hrpp_server *sv, const hrpp_serve_scene *scene, uint32_t *index) {
    if (!sv || !scene || !index) return HRPP_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return HRPP_EINVAL;
    std::vector<const hrpp_predictor *> seen;
    for (const auto &sc : sv->scenes)
        if (!sc.removed)
            for (int kind = 0; kind < 2; kind++) seen.insert(seen.end(), sc.preds[kind].begin(), sc.preds[kind].end());
    hrpp_server::Scene sc;
    if (make_scene(*scene, seen, sc) != HRPP_OK) return HRPP_EINVAL;
    sv->scenes.push_back(sc);
    *index = (uint32_t)(sv->scenes.size() - 1);
    return HRPP_OK;
}

hrpp_status hrpp_serve_remove_scene(hrpp_server *sv, uint32_t index) {
    if (!sv) return HRPP_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (index >= sv->scenes.size() || sv->scenes[index].removed) return HRPP_EINVAL;
    sv->scenes[index].removed = true;
    sv->cv.wait(lk, [sv, index] { return !sv->scene_busy(index); });
    return HRPP_OK;
}

hrpp_status hrpp_serve_submit(hrpp_server *sv, uint32_t scene, uint32_t query, const hrpp_ray *h_rays, uint32_t n,
                              void *h_out, uint64_t *request_id) {
    if (!sv || !request_id || query > 1 || n == 0 || n >= (1u << 31) || !h_rays || !h_out) return HRPP_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return HRPP_ENOMEM;
    r->scene = scene;
    r->query = query;
    r->n = n;
    r->h_rays = h_rays;
    r->h_out = h_out;
    r->ray_bytes = (size_t)n * sizeof(hrpp_ray);
    r->out_bytes = query == 0 ? (size_t)n : (size_t)n * sizeof(hrpp_hit);
    if (r->ray_bytes + hrpp::align256(r->out_bytes) + 256 > sv->pool.size()) {
        delete r;
        return HRPP_EBUSY;   // can never fit the budget
    }
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop || scene >= sv->scenes.size() || sv->scenes[scene].removed) { delete r; return HRPP_EINVAL; }
    r->id = sv->next_id++;
    sv->all[r->id] = r;
    sv->queue.push_back(r);
    *request_id = r->id;
    return HRPP_OK;
}

hrpp_status hrpp_serve_poll(hrpp_server *sv, uint64_t request_id, hrpp_request_info *info) {
    if (!sv || !info) return HRPP_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(request_id);
    if (it == sv->all.end()) return HRPP_EINVAL;
    Request *r = it->second;
    std::memset(info, 0, sizeof(*info));
    info->state = r->done ? 2u : (r->slot >= 0 ? 1u : 0u);
    info->status = r->status;
    auto ms = [](Clock::time_point a, Clock::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    if (r->slot >= 0) info->queue_ms = ms(r->t_submit, r->t_admit);
    if (r->done) {
        info->latency_ms = ms(r->t_submit, r->t_done);
        info->service_ms = ms(r->t_admit, r->t_done);
        // the final poll retires the request: its record is freed and its id
        // is unknown from now on
        sv->all.erase(it);
        delete r;
    }
    return HRPP_OK;
}

hrpp_status hrpp_serve_wait_all(hrpp_server *sv) {
    if (!sv) return HRPP_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [sv] { return sv->queue.empty() && sv->running.empty(); });
    return sv->first_error;
}

hrpp_status hrpp_serve_held(hrpp_server *sv, uint64_t *held) {
    if (!sv || !held) return HRPP_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *held = sv->all.size();
    return HRPP_OK;
}

hrpp_status hrpp_serve_pool_peak(hrpp_server *sv, size_t *peak_bytes) {
    if (!sv || !peak_bytes) return HRPP_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *peak_bytes = sv->peak_pool;
    return HRPP_OK;
}

void hrpp_serve_destroy(hrpp_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    if (sv->worker.joinable()) sv->worker.join();
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    for (auto &kv : sv->all) delete kv.second;
    delete sv;
}

}  // extern "C"
