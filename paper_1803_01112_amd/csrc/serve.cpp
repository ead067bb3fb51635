// serve.cpp -- continuous-batching server of reconstruction requests.
//
// Requests (a grid, histories, parameters, K cycles) queue in arrival order.
// A request is admitted when a slot is free and its device-memory footprint
// estimate fits under the server's HBM budget together with the requests
// already running; admission is strictly first-in first-out, so a large
// request at the head is never starved by smaller ones behind it.  Every
// admitted request runs on its own context and HIP stream (one worker thread
// per slot), so the kernels of different requests overlap on the device, and
// a request that arrives while others run is admitted as soon as a slot and
// memory free up.  A failing request (invalid input, out of memory, device
// error) fails alone.
//
// The executor can be simulated (no device work, a sleep proportional to
// the request's history-cycles) to exercise the scheduling policy without a
// GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

#include "../../include/tvs.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    int64_t id = 0;
    tvs_request r{};
    std::vector<float> x0;
    tvs_request_info info{};
    std::vector<float> image;
    std::string err;
};

// Bounds on a request's row entries and row segments (a row's run of
// entries inside one 16 x 16 tile) from its histories' straight entry-exit
// lines.  The most likely path is taken to stay within a margin of that
// line: kMargin mm plus half the line's length times the entry and exit
// slopes (the path bends from the entry ray towards the exit ray); a row
// then crosses at most (extent along an axis + 2 margins) / voxel size + 2
// planes of each axis, and tile boundaries 16 times fewer in x and y; each
// history's bound is also held below the grid-wide ones (row_cap, seg_cap).
// A host pass over the borrowed arrays, on several threads for large
// requests; without histories the grid-wide bounds are used.
constexpr double kMargin = 10.0;

struct LineSums {
    double rows = 0.0, segs = 0.0;
};

LineSums line_bounds(const tvs_request &r, double row_cap, double seg_cap)
{
    LineSums tot;
    const int64_t n = std::max<int64_t>(r.n, 0);
    const tvs_histories &h = r.h;
    if (!h.ex || !h.ey || !h.ez || !h.qx || !h.qy || !h.qz || !h.eth || !h.eps || !h.qth ||
        !h.qps) {
        tot.rows = row_cap * (double)n;
        tot.segs = seg_cap * (double)n;
        return tot;
    }
    const tvs_grid &g = r.grid;
    const double ext[3] = {g.nx * g.vx, g.ny * g.vy, g.nz * g.vz};
    auto part = [&](int64_t i0, int64_t i1, LineSums *out) {
        LineSums t;
        for (int64_t i = i0; i < i1; i++) {
            const double d[3] = {std::fabs((double)h.qx[i] - h.ex[i]),
                                 std::fabs((double)h.qy[i] - h.ey[i]),
                                 std::fabs((double)h.qz[i] - h.ez[i])};
            const double len = std::hypot(d[0], d[1]);
            const double mt = kMargin + 0.5 * len * (std::fabs((double)h.eth[i]) +
                                                     std::fabs((double)h.qth[i]));
            const double mv = kMargin + 0.5 * len * (std::fabs((double)h.eps[i]) +
                                                     std::fabs((double)h.qps[i]));
            const double m[3] = {mt, mt, mv};
            double e[3];
            for (int a = 0; a < 3; a++) {
                e[a] = std::min(d[a] + 2.0 * m[a], ext[a]);
                if (!(e[a] >= 0.0)) e[a] = ext[a];   // NaN input: the grid's extent
            }
            const double rows = e[0] / g.vx + e[1] / g.vy + e[2] / g.vz + 6.0;
            const double segs = e[0] / (16.0 * g.vx) + e[1] / (16.0 * g.vy) + e[2] / g.vz + 6.0;
            t.rows += std::min(rows, row_cap);
            t.segs += std::min(segs, seg_cap);
        }
        *out = t;
    };
    const int64_t per = 1 << 20;
    const int nt = (int)std::min<int64_t>(16, (n + per - 1) / per);
    if (nt <= 1) {
        part(0, n, &tot);
        return tot;
    }
    std::vector<LineSums> sums((size_t)nt);
    std::vector<std::thread> th;
    for (int q = 0; q < nt; q++)
        th.emplace_back(part, n * q / nt, n * (q + 1) / nt, &sums[(size_t)q]);
    for (auto &t : th) t.join();
    for (const auto &t : sums) {
        tot.rows += t.rows;
        tot.segs += t.segs;
    }
    return tot;
}

uint64_t footprint(const tvs_request &r, int64_t chunk)
{
    // device bytes of one context (see tvs_server_footprint)
    // image words in the device's tiled layout (16 x 16 tiles, padding included)
    const uint64_t nvox = (uint64_t)(((r.grid.nx + 15) / 16) * 16) *
                          (uint64_t)(((r.grid.ny + 15) / 16) * 16) * (uint64_t)r.grid.nz;
    const uint64_t ntiles = nvox / 256;
    const double vmin = std::min(r.grid.vx, r.grid.vy);
    const double span = (r.grid.nx * r.grid.vx + r.grid.ny * r.grid.vy) / vmin;
    const double row_cap = (double)((uint64_t)(0.8 * span) + (uint64_t)r.grid.nz + 8);
    const double seg_cap = row_cap / 4 + 2;
    const uint64_t n = (uint64_t)std::max<int64_t>(r.n, 0);
    const LineSums ls = line_bounds(r, row_cap, seg_cap);
    const uint64_t B = (uint64_t)(r.block_size > 0 ? r.block_size : 3200);
    const uint64_t nblocks = (n + B - 1) / B;
    // entries: 32-bit tag + chord (float32, or 16 bits for the f16 / q16 stores)
    const uint64_t entry =
        (r.path_mode == TVS_PATH_STORE_F16 || r.path_mode == TVS_PATH_STORE_Q16) ? 6 : 8;
    double entries;
    if (r.path_mode == TVS_PATH_ON_THE_FLY) {
        // a ring of three chunks of the longest rows the request can have
        const uint64_t held = 3 * std::min<uint64_t>(n, (uint64_t)chunk);
        entries = (double)held * row_cap;
    } else {
        entries = ls.rows;
    }
    const double per_hist = 52 /* streams */ + 8 + 4 + 8 + 4 /* row_off, norm2, seg_off, order */ +
                            8 /* load-time counts */;
    // list starts and the load-time list lengths by (block, tile) and by
    // (block, dispatch slot), live together at the peak
    const double lists = 16.0 * (double)(nblocks * ntiles + 1);
    const double bytes = per_hist * (double)n + 8.0 * ls.segs /* segment places */ + lists +
                         entries * (double)entry + 40.0 * (double)nvox + 24.0 * (double)B +
                         (double)(64ull << 20);
    return (uint64_t)bytes;
}

}  // namespace

struct tvs_server {
    tvs_server_config cfg{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_admit, cv_done;
    std::deque<Req *> queue;
    std::map<int64_t, std::unique_ptr<Req>> all;
    std::vector<std::thread> workers;
    uint64_t budget = 0, in_use = 0, peak = 0;
    int active = 0, peak_active = 0;
    int64_t next_id = 1, completed = 0, failed = 0, admitted = 0;
    bool stop = false;
    int64_t chunk = 262144;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    }
};

namespace {

int run_on_device(tvs_server *sv, Req *q)
{
    const tvs_request &r = q->r;
    tvs_config cfg;
    tvs_config_default(&cfg);
    cfg.block_size = r.block_size > 0 ? r.block_size : 3200;
    cfg.path_mode = r.path_mode;
    cfg.device = sv->cfg.device;
    cfg.hbm_budget_bytes = q->info.bytes;
    cfg.chunk_histories = sv->chunk;
    tvs_ctx *ctx = nullptr;
    int rc = tvs_create(&r.grid, &cfg, &ctx);
    if (rc) {
        q->err = "tvs_create failed";
        return rc;
    }
    rc = tvs_load_histories(ctx, r.n, &r.h, 0, nullptr);
    if (!rc && !q->x0.empty()) rc = tvs_set_image(ctx, q->x0.data(), 0, nullptr);
    if (!rc) rc = tvs_iterate(ctx, &r.params, r.K, nullptr);
    if (!rc) {
        q->image.resize((size_t)r.grid.nx * r.grid.ny * r.grid.nz);
        rc = tvs_get_image(ctx, q->image.data(), 0, nullptr);
    }
    if (rc) q->err = tvs_last_error(ctx);
    tvs_destroy(ctx);
    return rc;
}

int run_simulated(tvs_server *sv, Req *q)
{
    const double us = sv->cfg.sim_ns_per_history_cycle * 1e-3 * (double)q->r.n * q->r.K;
    std::this_thread::sleep_for(std::chrono::microseconds((int64_t)us));
    if (q->r.K < 0 || q->r.n < 0) return TVS_EINVAL;
    q->image.assign((size_t)q->r.grid.nx * q->r.grid.ny * q->r.grid.nz, (float)q->id);
    return TVS_OK;
}

void worker(tvs_server *sv)
{
    if (!sv->cfg.simulate) (void)hipSetDevice(sv->cfg.device);
    for (;;) {
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_admit.wait(lk, [&] {
                if (sv->stop) return true;
                if (sv->queue.empty()) return false;
                Req *h = sv->queue.front();
                return sv->in_use + h->info.bytes <= sv->budget;
            });
            if (sv->stop && sv->queue.empty()) return;
            if (sv->stop) {
                // cancel what never started
                while (!sv->queue.empty()) {
                    Req *c = sv->queue.front();
                    sv->queue.pop_front();
                    c->info.state = 3;
                    c->info.status = TVS_ESTATE;
                    c->err = "server stopped before admission";
                    c->info.done_ms = sv->now_ms();
                    sv->failed++;
                }
                sv->cv_done.notify_all();
                return;
            }
            q = sv->queue.front();
            sv->queue.pop_front();
            sv->in_use += q->info.bytes;
            sv->peak = std::max(sv->peak, sv->in_use);
            sv->active++;
            sv->peak_active = std::max(sv->peak_active, sv->active);
            sv->admitted++;
            q->info.state = 1;
            q->info.admit_ms = sv->now_ms();
            q->info.admit_order = sv->admitted;
        }
        int rc = sv->cfg.simulate ? run_simulated(sv, q) : run_on_device(sv, q);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->in_use -= q->info.bytes;
            sv->active--;
            q->info.status = rc;
            q->info.state = rc ? 3 : 2;
            q->info.done_ms = sv->now_ms();
            if (rc) sv->failed++;
            else sv->completed++;
        }
        sv->cv_admit.notify_all();
        sv->cv_done.notify_all();
    }
}

bool finite_grid(const tvs_grid &g)
{
    return g.nx > 0 && g.ny > 0 && g.nz > 0 && g.vx > 0 && g.vy > 0 && g.vz > 0 &&
           (int64_t)g.nx * g.ny * g.nz < ((int64_t)1 << 31);
}

}  // namespace

extern "C" {

void tvs_server_config_default(tvs_server_config *c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->max_active = 3;
    c->chunk_histories = 262144;
}

int tvs_server_create(const tvs_server_config *cfg, tvs_server **out)
{
    if (!cfg || !out) return TVS_EINVAL;
    *out = nullptr;
    if (cfg->max_active < 1 || cfg->max_active > 16) return TVS_EINVAL;
    if (cfg->simulate && cfg->hbm_budget_bytes == 0) return TVS_EINVAL;
    auto *sv = new tvs_server();
    sv->cfg = *cfg;
    sv->t0 = Clock::now();
    if (cfg->chunk_histories > 0) sv->chunk = cfg->chunk_histories;
    if (cfg->simulate) {
        sv->budget = cfg->hbm_budget_bytes;
    } else {
        size_t fr = 0, tot = 0;
        if (hipSetDevice(cfg->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete sv;
            return TVS_EDEVICE;
        }
        sv->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (uint64_t)(0.8 * (double)fr);
    }
    for (int q = 0; q < cfg->max_active; q++) sv->workers.emplace_back(worker, sv);
    *out = sv;
    return TVS_OK;
}

uint64_t tvs_server_footprint(const tvs_server *sv, const tvs_request *r)
{
    if (!sv || !r) return 0;
    return footprint(*r, sv->chunk);
}

int tvs_server_submit(tvs_server *sv, const tvs_request *r, int64_t *id)
{
    if (!sv || !r || !id) return TVS_EINVAL;
    if (!finite_grid(r->grid) || r->n < 0 || r->K < 0) return TVS_EINVAL;
    if (r->path_mode < 0 || r->path_mode > 3) return TVS_EINVAL;
    auto q = std::make_unique<Req>();
    q->r = *r;
    if (r->x0) {
        const size_t nv = (size_t)r->grid.nx * r->grid.ny * r->grid.nz;
        q->x0.assign(r->x0, r->x0 + nv);
        q->r.x0 = nullptr;
    }
    q->info.bytes = footprint(*r, sv->chunk);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return TVS_ESTATE;
    if (q->info.bytes > sv->budget) return TVS_ENOMEM;
    q->id = sv->next_id++;
    q->info.state = 0;
    q->info.submit_ms = sv->now_ms();
    *id = q->id;
    sv->queue.push_back(q.get());
    sv->all[q->id] = std::move(q);
    sv->cv_admit.notify_all();
    return TVS_OK;
}

int tvs_server_query(tvs_server *sv, int64_t id, tvs_request_info *info)
{
    if (!sv || !info) return TVS_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return TVS_ERANGE;
    *info = it->second->info;
    return TVS_OK;
}

int tvs_server_wait(tvs_server *sv, int64_t id, float *image, int64_t image_len,
                    tvs_request_info *info)
{
    if (!sv) return TVS_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return TVS_ERANGE;
    Req *q = it->second.get();
    sv->cv_done.wait(lk, [&] { return q->info.state >= 2; });
    if (info) *info = q->info;
    if (q->info.state == 2 && image) {
        if ((size_t)image_len < q->image.size()) return TVS_ERANGE;
        std::memcpy(image, q->image.data(), sizeof(float) * q->image.size());
    }
    return q->info.state == 2 ? TVS_OK : q->info.status;
}

int tvs_server_get_counters(tvs_server *sv, tvs_server_counters *out)
{
    if (!sv || !out) return TVS_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    out->budget_bytes = sv->budget;
    out->in_use_bytes = sv->in_use;
    out->peak_bytes = sv->peak;
    out->active = sv->active;
    out->peak_active = sv->peak_active;
    out->queued = (int32_t)sv->queue.size();
    out->completed = sv->completed;
    out->failed = sv->failed;
    return TVS_OK;
}

void tvs_server_destroy(tvs_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_admit.notify_all();
    for (auto &t : sv->workers) t.join();
    delete sv;
}

}  // extern "C"
