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
//
// Uploads go to one buffer per slot that is kept between requests.  The
// bytes a slot has reserved for it count against the budget for as long as
// the slot holds them; a free slot that holds some gives them back when the
// oldest request does not fit, so the budget bounds what the server holds,
// not only what is in flight.
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
    int waiters = 0;   // threads in hexval_server_wait on this ticket
    int status = HEXVAL_OK;
    std::string error;
};

struct Slot {
    hipStream_t stream = nullptr;
    Workspace* ws = nullptr;
    uint8_t* up = nullptr;      // upload buffer: points, then connectivity
    uint64_t up_cap = 0;        // bytes allocated in up (<= up_reserved)
    uint64_t up_reserved = 0;   // bytes of the budget this slot holds for up (under the lock)
    std::thread worker;
    ~Slot()
    {
        delete ws;
        if (up) hipFree(up);
        if (stream) hipStreamDestroy(stream);
    }
};

}  // namespace hexval

struct hexval_server {
    hexval_opts_t opts{};
    int device = 0;
    int64_t budget = 0;
    int64_t reserved = 0;      // workspaces
    int64_t in_use = 0;        // upload bytes reserved by the slots
    uint64_t next_ticket = 1;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<hexval::ServerRequest*> pending;
    std::map<uint64_t, std::unique_ptr<hexval::ServerRequest>> all;
    std::vector<std::unique_ptr<hexval::Slot>> slots;
};

namespace hexval {

// Byte offset of the connectivity in a slot's upload buffer.
static uint64_t points_bytes(const hexval_request_t& r)
{
    const hexval_mesh_t& m = r.mesh;
    if (!r.host_points) return 0;
    const uint64_t np = m.connectivity || r.host_conn ? (uint64_t)m.n_points * 3 : (uint64_t)m.n * 24;
    return (np * 8 + 255) & ~255ull;
}

static uint64_t upload_bytes(const hexval_request_t& r)
{
    uint64_t b = points_bytes(r);
    if (r.host_conn) b += (uint64_t)r.mesh.n * 8 * 4;
    return (b + 255) & ~255ull;
}

// Upload bytes the slot would add to the server's total by taking rq.
static int64_t growth(const Slot& sl, const ServerRequest& rq)
{
    return rq.upload_bytes > sl.up_reserved ? (int64_t)(rq.upload_bytes - sl.up_reserved) : 0;
}

static int run_one(hexval_server* sv, Slot& sl, ServerRequest& rq)
{
    hexval_request_t r = rq.req;
    hexval_mesh_t m = r.mesh;
    if (rq.upload_bytes > sl.up_cap) {
        // the bytes are reserved already (admission); the slot's stream is idle
        if (sl.up) hipFree(sl.up);
        sl.up = nullptr;
        sl.up_cap = 0;
        if (hipMalloc(&sl.up, rq.upload_bytes) != hipSuccess) {
            sl.up = nullptr;
            return fail(HEXVAL_E_NOMEM, "server upload buffer of %llu bytes", (unsigned long long)rq.upload_bytes);
        }
        sl.up_cap = rq.upload_bytes;
    }
    if (r.host_points) {
        const bool shared = m.connectivity || r.host_conn;
        const uint64_t np = shared ? (uint64_t)m.n_points * 3 : (uint64_t)m.n * 24;
        if (hipMemcpyAsync(sl.up, r.host_points, np * 8, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return fail(HEXVAL_E_HIP, "server upload of points failed");
        m.points = reinterpret_cast<const double*>(sl.up);
    }
    if (r.host_conn) {
        int32_t* conn = reinterpret_cast<int32_t*>(sl.up + points_bytes(r));
        if (hipMemcpyAsync(conn, r.host_conn, (uint64_t)m.n * 32, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return fail(HEXVAL_E_HIP, "server upload of connectivity failed");
        m.connectivity = conn;
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
        bool give_back = false;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            const int64_t room = sv->budget - sv->reserved;
            sv->cv_work.wait(lk, [&] {
                if (sv->pending.empty()) return sv->stop;
                // a slot that holds upload bytes the oldest request needs elsewhere gives them back
                return sv->in_use + growth(*sl, *sv->pending.front()) <= room || sl->up_reserved > 0;
            });
            if (sv->pending.empty()) return;
            ServerRequest* rq = sv->pending.front();
            if (sv->in_use + growth(*sl, *rq) > room) {
                sv->in_use -= (int64_t)sl->up_reserved;
                sl->up_reserved = 0;
                give_back = true;
            } else {
                sv->pending.pop_front();
                sv->in_use += growth(*sl, *rq);
                sl->up_reserved = std::max(sl->up_reserved, rq->upload_bytes);
                batch.push_back(rq);
            }
            // device-resident requests queued behind it join its call (in
            // order: the first one that needs an upload, or would overflow
            // the batch, stops the batch)
            int64_t hexes = rq->req.mesh.n;
            if (!give_back && rq->upload_bytes == 0 && hexes <= kBatchHexes) {
                while (!sv->pending.empty() && (int)batch.size() < kMaxBatch) {
                    ServerRequest* nx = sv->pending.front();
                    if (nx->upload_bytes != 0 || hexes + nx->req.mesh.n > kBatchHexes) break;
                    sv->pending.pop_front();
                    batch.push_back(nx);
                    hexes += nx->req.mesh.n;
                }
            }
        }
        if (give_back) {
            // nothing of this slot is on its stream: the last request it ran has completed
            if (sl->up) hipFree(sl->up);
            sl->up = nullptr;
            sl->up_cap = 0;
            sv->cv_work.notify_all();
            continue;
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
        // a call that failed part-way may have left copies or kernels on the
        // stream: none may touch the caller's buffers once a request is done
        if (device_ok) hipStreamSynchronize(sl->stream);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            const auto now = Clock::now();
            for (size_t k = 0; k < batch.size(); ++k) {
                ServerRequest* rq = batch[k];
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
        // on failure the slots made so far are freed with sv (no worker runs yet)
        std::unique_ptr<Slot> sl(new Slot());
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            sl->stream = nullptr;
            return fail(HEXVAL_E_HIP, "hipStreamCreate failed");
        }
        sl->ws = new Workspace();
        sl->ws->device = dev;
        if ((rc = sl->ws->init()) || (rc = sl->ws->ensure(node_cap, list_cap, kMaxBatch, batch_tiles)))
            return rc;
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

// Reports a finished request (under the lock) and forgets its ticket once no
// other thread waits on it.
static int finish(hexval_server_t* sv, ServerRequest* rq, double* latency_ms)
{
    if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(rq->t_done - rq->t_submit).count();
    const int status = rq->status;
    if (status) fail(status, "%s", rq->error.c_str());
    if (rq->waiters == 0) sv->all.erase(rq->ticket);
    return status;
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
    ++rq->waiters;
    sv->cv_done.wait(lk, [&] { return rq->done; });
    --rq->waiters;
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
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    hipSetDevice(sv->device);
    delete sv;   // the slots free their workspaces, upload buffers and streams
    if (prev >= 0) hipSetDevice(prev);
    return HEXVAL_OK;
}

}  // extern "C"
