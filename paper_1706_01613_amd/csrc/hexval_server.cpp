// Request queue with continuous batching (hexval_server_* of hexval.h).
//
// max_slots worker threads, each with its own HIP stream and its own
// workspace (subdivision queue and lists, and the tables of a batch of up to
// kMaxBatch meshes, allocated once, at creation, and counted against the HBM
// budget).  A worker that becomes free admits the oldest waiting request if
// its device footprint (the mesh bytes the server must upload, zero for a
// device-resident mesh) fits what is left of the budget.  When that request
// is device-resident, the worker also takes the device-resident requests
// queued right behind it, up to kMaxBatch of them and kBatchHexes elements
// in all, and runs them as one batched call: under load the per-call launch
// and synchronisation costs are shared.  Admitted work runs concurrently on
// the slots' streams, so requests arriving while others are on the GPU join
// as soon as a slot and memory are free.  The arithmetic of an element never
// depends on the batch it runs in.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <string>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "hexval.h"
#include "hexval_runtime.hpp"

using Clock = std::chrono::steady_clock;

namespace hexval {

constexpr int kMaxBatch = 64;                 // requests per batched call
constexpr int64_t kBatchHexes = 1ll << 24;    // elements per batched call

struct ServerRequest {
    uint64_t ticket = 0;
    hexval_request_t req{};
    uint64_t upload_bytes = 0;
    Clock::time_point t_submit, t_done;
    bool done = false;
    int status = HEXVAL_OK;
    std::string error;
};

struct Slot {
    hipStream_t stream = nullptr;
    Workspace* ws = nullptr;
    double* up_points = nullptr;
    int32_t* up_conn = nullptr;
    uint64_t up_points_cap = 0, up_conn_cap = 0;
    std::thread worker;
};

}  // namespace hexval

struct hexval_server {
    hexval_opts_t opts{};
    int device = 0;
    int64_t budget = 0;
    int64_t reserved = 0;      // workspaces
    int64_t in_use = 0;        // uploads of admitted requests
    uint64_t next_ticket = 1;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<hexval::ServerRequest*> pending;
    std::map<uint64_t, std::unique_ptr<hexval::ServerRequest>> all;
    std::vector<std::unique_ptr<hexval::Slot>> slots;
};

namespace hexval {

static uint64_t upload_bytes(const hexval_request_t& r)
{
    uint64_t b = 0;
    const hexval_mesh_t& m = r.mesh;
    if (r.host_points) b += (m.connectivity || r.host_conn ? (uint64_t)m.n_points * 3 : (uint64_t)m.n * 24) * 8;
    if (r.host_conn) b += (uint64_t)m.n * 8 * 4;
    return (b + 255) & ~255ull;
}

static int run_one(hexval_server* sv, Slot& sl, ServerRequest& rq)
{
    hexval_request_t r = rq.req;
    hexval_mesh_t m = r.mesh;
    if (r.host_points) {
        const bool shared = m.connectivity || r.host_conn;
        const uint64_t np = shared ? (uint64_t)m.n_points * 3 : (uint64_t)m.n * 24;
        if (np > sl.up_points_cap) {
            if (sl.up_points) hipFree(sl.up_points);
            sl.up_points = nullptr;
            sl.up_points_cap = 0;
            if (hipMalloc(&sl.up_points, np * 8) != hipSuccess)
                return fail(HEXVAL_E_NOMEM, "server upload buffer of %llu bytes", (unsigned long long)(np * 8));
            sl.up_points_cap = np;
        }
        if (hipMemcpyAsync(sl.up_points, r.host_points, np * 8, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return fail(HEXVAL_E_HIP, "server upload of points failed");
        m.points = sl.up_points;
    }
    if (r.host_conn) {
        const uint64_t nc = (uint64_t)m.n * 8;
        if (nc > sl.up_conn_cap) {
            if (sl.up_conn) hipFree(sl.up_conn);
            sl.up_conn = nullptr;
            sl.up_conn_cap = 0;
            if (hipMalloc(&sl.up_conn, nc * 4) != hipSuccess)
                return fail(HEXVAL_E_NOMEM, "server upload buffer of %llu bytes", (unsigned long long)(nc * 4));
            sl.up_conn_cap = nc;
        }
        if (hipMemcpyAsync(sl.up_conn, r.host_conn, nc * 4, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return fail(HEXVAL_E_HIP, "server upload of connectivity failed");
        m.connectivity = sl.up_conn;
    }
    hexval_opts_t o = sv->opts;
    o.stream = sl.stream;
    o.stats = nullptr;
    // shapes are timed by direct calls only: timing one here would stall the slot
    return run_check_ws(&m, 1, false, &o, &r.verdicts, &r.min_coeffs, sl.ws, false);
}

// Device-resident requests as one batched call.
static int run_batch(hexval_server* sv, Slot& sl, const std::vector<ServerRequest*>& batch)
{
    std::vector<hexval_mesh_t> meshes;
    std::vector<uint8_t*> verdicts;
    std::vector<double*> mins;
    for (ServerRequest* rq : batch) {
        meshes.push_back(rq->req.mesh);
        verdicts.push_back(rq->req.verdicts);
        mins.push_back(rq->req.min_coeffs);
    }
    hexval_opts_t o = sv->opts;
    o.stream = sl.stream;
    o.stats = nullptr;
    return run_check_ws(meshes.data(), (int)meshes.size(), true, &o, verdicts.data(), mins.data(), sl.ws, false);
}

static void worker_loop(hexval_server* sv, Slot* sl)
{
    // a worker that cannot select the server's device fails what it takes
    const bool device_ok = hipSetDevice(sv->device) == hipSuccess;
    for (;;) {
        std::vector<ServerRequest*> batch;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] {
                if (sv->stop && sv->pending.empty()) return true;
                if (sv->pending.empty()) return false;
                return sv->in_use + (int64_t)sv->pending.front()->upload_bytes <= sv->budget - sv->reserved;
            });
            if (sv->pending.empty()) return;
            ServerRequest* rq = sv->pending.front();
            sv->pending.pop_front();
            sv->in_use += (int64_t)rq->upload_bytes;
            batch.push_back(rq);
            // device-resident requests queued behind it join its call (in
            // order: the first one that needs an upload, or would overflow
            // the batch, stops the batch)
            int64_t hexes = rq->req.mesh.n;
            if (rq->upload_bytes == 0 && hexes <= kBatchHexes) {
                while (!sv->pending.empty() && (int)batch.size() < kMaxBatch) {
                    ServerRequest* nx = sv->pending.front();
                    if (nx->upload_bytes != 0 || hexes + nx->req.mesh.n > kBatchHexes) break;
                    sv->pending.pop_front();
                    batch.push_back(nx);
                    hexes += nx->req.mesh.n;
                }
            }
        }
        std::vector<int> status(batch.size(), HEXVAL_OK);
        std::vector<std::string> error(batch.size());
        bool alone = batch.size() == 1;
        if (!device_ok) {
            for (size_t k = 0; k < batch.size(); ++k) {
                status[k] = fail(HEXVAL_E_HIP, "server worker could not select device %d", sv->device);
                error[k] = last_error();
            }
            alone = false;
        } else if (!alone && run_batch(sv, *sl, batch) != HEXVAL_OK) {
            alone = true;   // one bad request must not fail the others: run each by itself
        }
        if (alone) {
            for (size_t k = 0; k < batch.size(); ++k) {
                status[k] = run_one(sv, *sl, *batch[k]);
                if (status[k]) error[k] = last_error();
            }
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            const auto now = Clock::now();
            for (size_t k = 0; k < batch.size(); ++k) {
                ServerRequest* rq = batch[k];
                sv->in_use -= (int64_t)rq->upload_bytes;
                rq->status = status[k];
                rq->error = error[k];
                rq->t_done = now;
                rq->done = true;
            }
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
}

}  // namespace hexval

using namespace hexval;

extern "C" {

int hexval_server_create(const hexval_opts_t* opts, int64_t hbm_budget_bytes, int32_t max_slots,
                         hexval_server_t** server)
{
    if (!server) return fail(HEXVAL_E_ARG, "server is NULL");
    *server = nullptr;
    hexval_opts_t o;
    if (opts) o = *opts;
    else default_opts(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (hbm_budget_bytes <= 0) return fail(HEXVAL_E_ARG, "hbm_budget_bytes must be > 0");
    if (max_slots < 1 || max_slots > 64) return fail(HEXVAL_E_ARG, "max_slots must be in 1..64");
    int dev, cus;
    if ((rc = current_device(&dev, &cus))) return rc;
    const uint64_t node_cap = o.queue_capacity ? (uint64_t)o.queue_capacity : (1ull << 20);
    const uint64_t list_cap = o.precision == HEXVAL_FP32_FILTER ? (1ull << 22) : std::max<uint64_t>(node_cap, 1u << 16);
    // batch tables: tiles of at least 64 elements, one partial tile per mesh
    const uint64_t batch_tiles = (uint64_t)(kBatchHexes / 64 + kMaxBatch);
    const int64_t per_slot = (int64_t)Workspace::footprint(node_cap, list_cap, kMaxBatch, batch_tiles);
    if (per_slot * max_slots > hbm_budget_bytes)
        return fail(HEXVAL_E_ARG, "budget %lld B is below the %d slot workspaces (%lld B each)",
                    (long long)hbm_budget_bytes, max_slots, (long long)per_slot);
    std::unique_ptr<hexval_server> sv(new hexval_server());
    sv->opts = o;
    sv->device = dev;
    sv->budget = hbm_budget_bytes;
    sv->reserved = per_slot * max_slots;
    for (int i = 0; i < max_slots; ++i) {
        std::unique_ptr<Slot> sl(new Slot());
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess)
            return fail(HEXVAL_E_HIP, "hipStreamCreate failed");
        sl->ws = new Workspace();
        sl->ws->device = dev;
        if ((rc = sl->ws->init()) || (rc = sl->ws->ensure(node_cap, list_cap, kMaxBatch, batch_tiles))) {
            delete sl->ws;
            hipStreamDestroy(sl->stream);
            return rc;
        }
        sv->slots.push_back(std::move(sl));
    }
    for (auto& sl : sv->slots) sl->worker = std::thread(worker_loop, sv.get(), sl.get());
    *server = sv.release();
    return HEXVAL_OK;
}

int hexval_server_submit(hexval_server_t* sv, const hexval_request_t* request, uint64_t* ticket)
{
    if (!sv || !request || !ticket) return fail(HEXVAL_E_ARG, "NULL argument");
    const hexval_mesh_t& m = request->mesh;
    if (m.n < 0) return fail(HEXVAL_E_ARG, "n < 0");
    if (m.n > 0 && (!request->verdicts || (!m.points && !request->host_points)))
        return fail(HEXVAL_E_ARG, "verdicts or points is NULL");
    if ((request->host_conn || m.connectivity) && request->host_points && m.n_points <= 0)
        return fail(HEXVAL_E_ARG, "uploading a shared-vertex mesh needs n_points");
    std::unique_ptr<ServerRequest> rq(new ServerRequest());
    rq->req = *request;
    rq->upload_bytes = upload_bytes(*request);
    if ((int64_t)rq->upload_bytes > sv->budget - sv->reserved)
        return fail(HEXVAL_E_BUSY, "request needs %llu B of uploads, more than the budget leaves",
                    (unsigned long long)rq->upload_bytes);
    rq->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(HEXVAL_E_ARG, "server is shutting down");
        rq->ticket = sv->next_ticket++;
        *ticket = rq->ticket;
        sv->pending.push_back(rq.get());
        sv->all[rq->ticket] = std::move(rq);
    }
    sv->cv_work.notify_all();
    return HEXVAL_OK;
}

static int finish(hexval_server_t* sv, ServerRequest* rq, double* latency_ms)
{
    if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(rq->t_done - rq->t_submit).count();
    if (rq->status) fail(rq->status, "%s", rq->error.c_str());
    return rq->status;
}

int hexval_server_poll(hexval_server_t* sv, uint64_t ticket, int* done, double* latency_ms)
{
    if (!sv || !done) return fail(HEXVAL_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return fail(HEXVAL_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second->done ? 1 : 0;
    if (!*done) return HEXVAL_OK;
    return finish(sv, it->second.get(), latency_ms);
}

int hexval_server_wait(hexval_server_t* sv, uint64_t ticket, double* latency_ms)
{
    if (!sv) return fail(HEXVAL_E_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return fail(HEXVAL_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    ServerRequest* rq = it->second.get();
    sv->cv_done.wait(lk, [&] { return rq->done; });
    return finish(sv, rq, latency_ms);
}

int hexval_server_destroy(hexval_server_t* sv)
{
    if (!sv) return fail(HEXVAL_E_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto& sl : sv->slots)
        if (sl->worker.joinable()) sl->worker.join();
    for (auto& sl : sv->slots) {
        hipSetDevice(sv->device);
        delete sl->ws;
        if (sl->up_points) hipFree(sl->up_points);
        if (sl->up_conn) hipFree(sl->up_conn);
        hipStreamDestroy(sl->stream);
    }
    delete sv;
    return HEXVAL_OK;
}

}  // extern "C"
