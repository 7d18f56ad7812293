// Host runtime and C ABI of libhexval: argument checks, device check,
// workspace pool, launch planning, the pass/round loop and the hand-off of
// uncertifiable elements to the exact tier.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hexval.h"
#include "hexval_exact.hpp"
#include "hexval_internal.hpp"
#include "hexval_kernels.hpp"
#include "hexval_runtime.hpp"

namespace hexval {

static thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

const char* last_error() { return g_error.c_str(); }

#define HX_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(HEXVAL_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- devices

struct DeviceInfo {
    bool checked = false;
    bool ok = false;
    int cus = 0;
    char arch[64] = {0};
};
static std::mutex g_dev_mu;
static DeviceInfo g_dev[64];

int current_device(int* dev, int* cus)
{
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess || d < 0 || d >= 64) {
        hipGetLastError();
        return fail(HEXVAL_E_HIP, "no HIP device available (%s)", hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo& di = g_dev[d];
    if (!di.checked) {
        hipDeviceProp_t p;
        e = hipGetDeviceProperties(&p, d);
        if (e != hipSuccess) return fail(HEXVAL_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
        snprintf(di.arch, sizeof di.arch, "%s", p.gcnArchName);
        di.ok = strncmp(p.gcnArchName, "gfx950", 6) == 0;
        di.cus = p.multiProcessorCount;
        di.checked = true;
    }
    if (!di.ok) return fail(HEXVAL_E_HIP, "device %d is %s; libhexval is built for gfx950 only", d, di.arch);
    *dev = d;
    if (cus) *cus = di.cus;
    return HEXVAL_OK;
}

// ---------------------------------------------------------------- workspace

template <class T>
static int dalloc(T** p, uint64_t n)
{
    if (hipMalloc((void**)p, std::max<uint64_t>(n, 1) * sizeof(T)) != hipSuccess) {
        hipGetLastError();
        *p = nullptr;
        return fail(HEXVAL_E_NOMEM, "hipMalloc of %llu bytes failed", (unsigned long long)(n * sizeof(T)));
    }
    return HEXVAL_OK;
}

template <class T>
static int halloc(T** p, uint64_t n)
{
    if (hipHostMalloc((void**)p, std::max<uint64_t>(n, 1) * sizeof(T), hipHostMallocDefault) != hipSuccess) {
        hipGetLastError();
        *p = nullptr;
        return fail(HEXVAL_E_NOMEM, "hipHostMalloc of %llu bytes failed", (unsigned long long)(n * sizeof(T)));
    }
    return HEXVAL_OK;
}

template <class T>
static void dfree(T*& p)
{
    if (p) hipFree((void*)p);
    p = nullptr;
}

template <class T>
static void hfree(T*& p)
{
    if (p) hipHostFree((void*)p);
    p = nullptr;
}

constexpr uint64_t kExactCap = 1ull << 16;

Workspace::~Workspace()
{
    int prev = -1;
    hipGetDevice(&prev);
    hipSetDevice(device);
    release_queue();
    release_list();
    dfree(cnt);
    hfree(hcnt);
    dfree(exact_elem);
    dfree(exact_mesh);
    dfree(exact_pts);
    dfree(exact_v);
    hfree(h_exact_pts);
    hfree(h_exact_v);
    dfree(meshes);
    hfree(h_meshes);
    dfree(tile_mesh);
    for (auto& e : ev)
        if (e) hipEventDestroy(e);
    if (prev >= 0) hipSetDevice(prev);
}

void Workspace::release_queue()
{
    dfree(nodes);
    dfree(sub_elem);
    dfree(sub_mesh);
    dfree(sub_flags);
    node_cap = 0;
}

void Workspace::release_list()
{
    dfree(list_elem);
    dfree(list_mesh);
    list_cap = 0;
}

int Workspace::init()
{
    int rc;
    if ((rc = dalloc(&cnt, 1)) || (rc = halloc(&hcnt, 1))) return rc;
    if ((rc = dalloc(&exact_elem, kExactCap)) || (rc = dalloc(&exact_mesh, kExactCap)) ||
        (rc = dalloc(&exact_pts, kExactCap * 24)) || (rc = dalloc(&exact_v, kExactCap)) ||
        (rc = halloc(&h_exact_pts, kExactCap * 24)) || (rc = halloc(&h_exact_v, kExactCap)))
        return rc;
    exact_cap = kExactCap;
    for (auto& e : ev) HX_HIP(hipEventCreate(&e));
    return HEXVAL_OK;
}

int Workspace::ensure(uint64_t want_nodes, uint64_t want_list, uint64_t want_meshes, uint64_t want_tiles)
{
    int rc;
    if (want_nodes > node_cap) {
        release_queue();
        if ((rc = dalloc(&nodes, want_nodes)) || (rc = dalloc(&sub_elem, want_nodes)) ||
            (rc = dalloc(&sub_mesh, want_nodes)) || (rc = dalloc(&sub_flags, want_nodes))) {
            release_queue();
            return rc;
        }
        // nodes[].ready holds the epoch of the pass that wrote the node;
        // fresh memory may hold anything, so clear it once here.
        if (hipMemset(nodes, 0, want_nodes * sizeof(Node)) != hipSuccess) {
            release_queue();
            return fail(HEXVAL_E_HIP, "hipMemset of the subdivision queue failed");
        }
        node_cap = want_nodes;
    }
    if (want_list > list_cap) {
        release_list();
        if ((rc = dalloc(&list_elem, want_list)) || (rc = dalloc(&list_mesh, want_list))) {
            release_list();
            return rc;
        }
        list_cap = want_list;
    }
    if (want_meshes > mesh_cap) {
        dfree(meshes);
        hfree(h_meshes);
        mesh_cap = 0;
        if ((rc = dalloc(&meshes, want_meshes)) || (rc = halloc(&h_meshes, want_meshes))) return rc;
        mesh_cap = want_meshes;
    }
    if (want_tiles > tile_cap) {
        dfree(tile_mesh);
        tile_cap = 0;
        if ((rc = dalloc(&tile_mesh, want_tiles))) return rc;
        tile_cap = want_tiles;
    }
    return HEXVAL_OK;
}

uint64_t Workspace::footprint(uint64_t nodes, uint64_t list, uint64_t meshes, uint64_t tiles)
{
    return nodes * (sizeof(Node) + 16) + list * 12 + meshes * sizeof(MeshDev) + tiles * 4 +
           kExactCap * (12 + 24 * 8 + 1) + sizeof(Counters);
}

QueueDev Workspace::queue() const
{
    QueueDev q;
    q.nodes = nodes;
    q.node_cap = node_cap;
    q.sub_elem = sub_elem;
    q.sub_mesh = sub_mesh;
    q.sub_flags = sub_flags;
    q.exact_elem = exact_elem;
    q.exact_mesh = exact_mesh;
    q.exact_cap = exact_cap;
    q.list_elem = list_elem;
    q.list_mesh = list_mesh;
    q.list_cap = list_cap;
    q.cnt = cnt;
    q.epoch = epoch;
    return q;
}

static std::mutex g_pool_mu;
static std::vector<std::unique_ptr<Workspace>> g_pool;

int acquire_workspace(int device, Workspace** out)
{
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (size_t i = 0; i < g_pool.size(); ++i)
            if (g_pool[i]->device == device) {
                *out = g_pool[i].release();
                g_pool.erase(g_pool.begin() + i);
                return HEXVAL_OK;
            }
    }
    std::unique_ptr<Workspace> w(new Workspace());
    w->device = device;
    int rc = w->init();
    if (rc) return rc;
    *out = w.release();
    return HEXVAL_OK;
}

void release_workspace(Workspace* w)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.emplace_back(w);
}

struct WorkspaceGuard {
    Workspace* w = nullptr;
    ~WorkspaceGuard()
    {
        if (w) release_workspace(w);
    }
};

// ---------------------------------------------------------------- options

void default_opts(hexval_opts_t* o)
{
    memset(o, 0, sizeof *o);
    o->precision = HEXVAL_FP64;
    o->max_depth = 6;
}

int check_opts(const hexval_opts_t* o)
{
    if (o->precision != HEXVAL_FP64 && o->precision != HEXVAL_FP32_FILTER)
        return fail(HEXVAL_E_ARG, "precision must be HEXVAL_FP64 or HEXVAL_FP32_FILTER");
    if (o->max_depth < 0 || o->max_depth > 20) return fail(HEXVAL_E_ARG, "max_depth must be in 0..20");
    if (o->block_threads != 0 && (o->block_threads < 64 || o->block_threads > 256 || o->block_threads % 64))
        return fail(HEXVAL_E_ARG, "block_threads must be 0 or a multiple of 64 in 64..256");
    if (o->queue_capacity < 0) return fail(HEXVAL_E_ARG, "queue_capacity must be >= 0");
    if (o->grid_blocks < 0 || o->grid_blocks > (1ll << 30)) return fail(HEXVAL_E_ARG, "grid_blocks out of range");
    return HEXVAL_OK;
}

int check_mesh(const hexval_mesh_t* m, const void* verdicts, int validate, int idx)
{
    if (m->n < 0) return fail(HEXVAL_E_ARG, "mesh %d: n < 0", idx);
    if (m->n == 0) return HEXVAL_OK;
    if (!m->points) return fail(HEXVAL_E_ARG, "mesh %d: points is NULL", idx);
    if (!verdicts) return fail(HEXVAL_E_ARG, "mesh %d: verdicts is NULL", idx);
    if (m->connectivity && validate && (m->n_points <= 0 || m->n_points > (1ll << 31)))
        return fail(HEXVAL_E_ARG, "mesh %d: index validation needs 0 < n_points <= 2^31", idx);
    if (!m->connectivity && m->n > (1ll << 56)) return fail(HEXVAL_E_ARG, "mesh %d: n too large", idx);
    return HEXVAL_OK;
}

static uint64_t pow2_ceil(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// ---------------------------------------------------------------- exact tier

static void run_exact_host(const double* pts, uint8_t* out, int64_t n, int max_depth)
{
    if (n <= 0) return;
    const int64_t nt = std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
    const int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t lo = t * per, hi = std::min(n, lo + per);
        if (lo >= hi) break;
        th.emplace_back([=] {
            for (int64_t i = lo; i < hi; ++i) out[i] = exact_verdict(pts + 24 * i, max_depth);
        });
    }
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------- main loop

int run_check(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts,
              uint8_t* const* verdicts, double* const* mins)
{
    return run_check_ws(meshes, n_meshes, batched, opts, verdicts, mins, nullptr);
}

int run_check_ws(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts_in,
                 uint8_t* const* verdicts, double* const* mins, Workspace* fixed)
{
    hexval_opts_t o;
    if (opts_in) o = *opts_in;
    else default_opts(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (n_meshes < 0) return fail(HEXVAL_E_ARG, "n_meshes < 0");
    if (n_meshes > 0 && (!meshes || !verdicts)) return fail(HEXVAL_E_ARG, "meshes or verdicts is NULL");
    int64_t total = 0;
    for (int i = 0; i < n_meshes; ++i) {
        if ((rc = check_mesh(&meshes[i], verdicts[i], o.validate_indices, i))) return rc;
        total += meshes[i].n;
    }
    hexval_stats_t* st = o.stats;
    if (st) {
        const int timing = st->timing;
        memset(st, 0, sizeof *st);
        st->timing = timing;
    }
    if (total == 0) return HEXVAL_OK;

    int dev, cus;
    if ((rc = current_device(&dev, &cus))) return rc;
    hipStream_t s = (hipStream_t)o.stream;

    const int block = o.block_threads ? o.block_threads : 256;
    // Automatic queue size: 1/32 of the elements, at least 2^19 nodes (any
    // single element's tree at the default cap fits), and room for a tree
    // whose ambiguous region is a surface (4^level live sub-boxes) at the
    // requested cap; at most 2^26 nodes (17 GiB).
    uint64_t want = std::max<uint64_t>(total / 32, 1u << 19);
    if (o.max_depth > 6) want = std::max<uint64_t>(want, 2ull << (2 * o.max_depth));
    uint64_t node_cap = o.queue_capacity ? (uint64_t)o.queue_capacity
                                         : pow2_ceil(std::min<uint64_t>(want, 1ull << 26));
    uint64_t list_cap = o.precision == HEXVAL_FP32_FILTER
                            ? pow2_ceil(std::min<uint64_t>(std::max<uint64_t>(total / 8, 1u << 16), 1u << 27))
                            : std::max<uint64_t>(node_cap, 1u << 16);
    // tiles
    std::vector<int64_t> tile_begin(n_meshes);
    int64_t n_tiles = 0;
    for (int i = 0; i < n_meshes; ++i) {
        tile_begin[i] = n_tiles;
        n_tiles += (meshes[i].n + block - 1) / block;
    }

    WorkspaceGuard wg;
    if (!fixed && (rc = acquire_workspace(dev, &wg.w))) return rc;
    Workspace& w = fixed ? *fixed : *wg.w;
    if (fixed) node_cap = list_cap = 0;   // a fixed workspace keeps its capacities
    if ((rc = w.ensure(node_cap, list_cap, batched ? n_meshes : 1, batched ? n_tiles : 1))) return rc;
    QueueDev q = w.queue();
    // a pooled workspace may be larger than this call asked for
    if (node_cap) q.node_cap = std::min<uint64_t>(q.node_cap, node_cap);
    if (list_cap) q.list_cap = std::min<uint64_t>(q.list_cap, list_cap);

    MeshDev single{};
    std::vector<MeshDev> md(n_meshes);
    for (int i = 0; i < n_meshes; ++i) {
        MeshDev& m = md[i];
        m.points = meshes[i].points;
        m.conn = meshes[i].connectivity;
        m.n = meshes[i].n;
        m.n_points = meshes[i].n_points;
        m.verdict = verdicts[i];
        m.min_coeff = mins ? mins[i] : nullptr;
        m.tile_begin = tile_begin[i];
        m.validate = (o.validate_indices && m.conn) ? 1 : 0;
    }
    const MeshDev* dmeshes = nullptr;
    if (batched) {
        memcpy(w.h_meshes, md.data(), n_meshes * sizeof(MeshDev));
        HX_HIP(hipMemcpyAsync(w.meshes, w.h_meshes, n_meshes * sizeof(MeshDev), hipMemcpyHostToDevice, s));
        launch_tile_table(w.meshes, n_meshes, block, w.tile_mesh, s);
        dmeshes = w.meshes;
    } else {
        single = md[0];
    }

    const bool timing = st && st->timing;
    const int xcds = 8;
    int64_t grid = o.grid_blocks;
    if (!grid) grid = batched ? std::min<int64_t>(n_tiles, (int64_t)cus * 8) : n_tiles;
    grid = std::max<int64_t>(xcds, (grid + xcds - 1) / xcds * xcds);
    grid = std::min<int64_t>(grid, (1ll << 30));
    const int list_grid = cus * 8;
    const int drain_grid = cus;

    uint64_t prev_remaining = 0;
    for (int round = 0;; ++round) {
        ++w.epoch;
        q.epoch = w.epoch;
        launch_reset(w.cnt, s);
        TopArgs ta{};
        ta.mesh = single;
        ta.meshes = dmeshes;
        ta.tile_mesh = w.tile_mesh;
        ta.n_tiles = n_tiles;
        ta.list_count = &w.cnt->n_list;
        ta.q = q;
        ta.max_depth = o.max_depth;
        ta.xcds = xcds;
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[0], s));
        if (round == 0) {
            launch_top_range(ta, batched, (int)grid, block, s);
        } else {
            CollectArgs ca{q, single, dmeshes, batched ? n_meshes : 1};
            launch_collect_deferred(ca, list_grid, s);
            launch_top_list(ta, batched, list_grid, block, s);
        }
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[1], s));
        RootArgs ra{q, single, dmeshes};
        launch_roots(ra, cus * 2, s);
        DrainArgs da{q, o.max_depth};
        launch_drain(da, drain_grid, s);
        FoldArgs fa{q, single, dmeshes};
        launch_fold(fa, cus * 2, s);
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[2], s));
        HX_HIP(hipGetLastError());
        HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HX_HIP(hipStreamSynchronize(s));
        const Counters c = *w.hcnt;
        if (c.error) return fail(HEXVAL_E_QUEUE, "subdivision drain stalled (error bits %u)", c.error);
        if (st) {
            st->n_subdivided += (int64_t)std::min<uint64_t>(c.n_sub, q.node_cap);
            st->n_nodes += (int64_t)c.n_nodes;
            st->max_level = std::max<int32_t>(st->max_level, (int32_t)c.max_level);
            st->n_rounds = round + 1;
            if (round == 0) {
                st->n_elements = total;
                if (timing) {
                    hipEventElapsedTime(&st->ms_first_pass, w.ev[0], w.ev[1]);
                    hipEventElapsedTime(&st->ms_subdivision, w.ev[1], w.ev[2]);
                    hipEventElapsedTime(&st->ms_total, w.ev[0], w.ev[2]);
                }
            }
        }
        const int64_t n_ex = (int64_t)std::min<uint64_t>(c.n_exact, q.exact_cap);
        if (n_ex > 0) {
            GatherArgs ga{q, single, dmeshes, n_ex, w.exact_pts};
            launch_gather_exact(ga, s);
            HX_HIP(hipMemcpyAsync(w.h_exact_pts, w.exact_pts, n_ex * 24 * sizeof(double), hipMemcpyDeviceToHost, s));
            HX_HIP(hipStreamSynchronize(s));
            run_exact_host(w.h_exact_pts, w.h_exact_v, n_ex, o.max_depth);
            HX_HIP(hipMemcpyAsync(w.exact_v, w.h_exact_v, n_ex, hipMemcpyHostToDevice, s));
            ScatterArgs sa{q, single, dmeshes, n_ex, w.exact_v};
            launch_scatter_exact(sa, s);
            HX_HIP(hipGetLastError());
            HX_HIP(hipStreamSynchronize(s));
            if (st) st->n_exact += n_ex;
        }
        // Elements deferred by a full queue are checked again, from their own
        // list and with an empty queue, until none is left.
        uint64_t remaining;
        if (round == 0) {
            remaining = c.n_deferred;
        } else {
            const uint64_t listed = std::min<uint64_t>(prev_remaining, q.list_cap);
            if (c.n_deferred >= listed)
                return fail(HEXVAL_E_QUEUE, "subdivision queue of %llu nodes too small to make progress",
                            (unsigned long long)q.node_cap);
            remaining = prev_remaining - listed + c.n_deferred;
        }
        if (remaining == 0) break;
        prev_remaining = remaining;
    }
    return HEXVAL_OK;
}

int run_coefficients(const hexval_mesh_t* mesh, void* stream, double* coeffs)
{
    if (!mesh) return fail(HEXVAL_E_ARG, "mesh is NULL");
    if (mesh->n < 0) return fail(HEXVAL_E_ARG, "n < 0");
    if (mesh->n == 0) return HEXVAL_OK;
    if (!mesh->points || !coeffs) return fail(HEXVAL_E_ARG, "points or coeffs is NULL");
    int dev, cus, rc;
    if ((rc = current_device(&dev, &cus))) return rc;
    MeshDev m{};
    m.points = mesh->points;
    m.conn = mesh->connectivity;
    m.n = mesh->n;
    m.n_points = mesh->n_points;
    hipStream_t s = (hipStream_t)stream;
    launch_coefficients(m, coeffs, s);
    HX_HIP(hipGetLastError());
    HX_HIP(hipStreamSynchronize(s));
    return HEXVAL_OK;
}

}  // namespace hexval

// ---------------------------------------------------------------- C ABI

using namespace hexval;

extern "C" {

void hexval_opts_default(hexval_opts_t* opts)
{
    if (opts) default_opts(opts);
}

int hexval_check(const double* points, const int32_t* connectivity, int64_t n, uint8_t* verdicts,
                 double* min_coeffs)
{
    hexval_mesh_t m{points, 0, connectivity, n};
    return run_check(&m, 1, false, nullptr, &verdicts, &min_coeffs);
}

int hexval_check_ex(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts, double* min_coeffs)
{
    if (!mesh) return fail(HEXVAL_E_ARG, "mesh is NULL");
    return run_check(mesh, 1, false, opts, &verdicts, &min_coeffs);
}

int hexval_check_batched(const hexval_mesh_t* meshes, int32_t n_meshes, const hexval_opts_t* opts,
                         uint8_t* const* verdicts, double* const* min_coeffs)
{
    return run_check(meshes, n_meshes, true, opts, verdicts, min_coeffs);
}

int hexval_coefficients(const hexval_mesh_t* mesh, void* stream, double* coeffs)
{
    return run_coefficients(mesh, stream, coeffs);
}

const char* hexval_last_error(void) { return last_error(); }

}  // extern "C"
