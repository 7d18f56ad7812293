// Host runtime and C ABI of libhexval: argument checks, device check,
// workspace pool, launch planning, the pass/round loop and the hand-off of
// uncertifiable elements to the exact tier.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hexval.h"
#include "hexval_exact.hpp"
#include "hexval_exact_dev.hpp"
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

const char* device_arch(int dev)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return g_dev[dev].arch;
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
    if (borrowed) return;
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
    dfree(minj);
    dfree(minj_defer);
    dfree(tile_mesh);
    dfree(walk_meshes);
    dfree(walk_tile_mesh);
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
        dfree(walk_meshes);
        mesh_cap = 0;
        if ((rc = dalloc(&meshes, want_meshes)) || (rc = halloc(&h_meshes, want_meshes)) ||
            (rc = dalloc(&walk_meshes, want_meshes)))
            return rc;
        mesh_cap = want_meshes;
    }
    if (want_tiles > tile_cap) {
        dfree(tile_mesh);
        dfree(walk_tile_mesh);
        tile_cap = 0;
        if ((rc = dalloc(&tile_mesh, want_tiles)) || (rc = dalloc(&walk_tile_mesh, want_tiles))) return rc;
        tile_cap = want_tiles;
    }
    return HEXVAL_OK;
}

int Workspace::ensure_minj(uint64_t slots, uint64_t elements)
{
    int rc;
    if (slots > minj_cap) {
        dfree(minj);
        minj_cap = 0;
        if ((rc = dalloc(&minj, 5 * slots))) return rc;
        minj_cap = slots;
    }
    if (elements > defer_cap) {
        dfree(minj_defer);
        defer_cap = 0;
        if ((rc = dalloc(&minj_defer, 2 * elements))) return rc;
        defer_cap = elements;
    }
    return HEXVAL_OK;
}

uint64_t Workspace::footprint(uint64_t nodes, uint64_t list, uint64_t meshes, uint64_t tiles)
{
    return nodes * (sizeof(Node) + 16) + list * 12 + meshes * (sizeof(MeshDev) + sizeof(WalkMesh)) + tiles * 8 +
           kExactCap * (12 + 24 * 8 + 1) + sizeof(Counters);
}

QueueDev Workspace::queue() const
{
    QueueDev q;
    q.nodes = nodes;
    q.node_cap = node_cap;
    q.root_cap = node_cap;
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
    if (o->max_depth < 0 || o->max_depth > kMaxDepth) return fail(HEXVAL_E_ARG, "max_depth must be in 0..20");
    if (o->block_threads != 0 && (o->block_threads < 64 || o->block_threads > 256 || o->block_threads % 64))
        return fail(HEXVAL_E_ARG, "block_threads must be 0 or a multiple of 64 in 64..256");
    if (o->queue_capacity < 0) return fail(HEXVAL_E_ARG, "queue_capacity must be >= 0");
    if (o->grid_blocks < 0 || o->grid_blocks > (1ll << 30)) return fail(HEXVAL_E_ARG, "grid_blocks out of range");
    if (o->walk_layers < -1 || o->walk_layers > 64) return fail(HEXVAL_E_ARG, "walk_layers must be in -1..64");
    if (o->reserved != 0) return fail(HEXVAL_E_ARG, "reserved must be 0");
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

// Kinds of exact decisions: pts hold 24 doubles per element (hexahedra) or 8
// (quadrangles).
enum class ExactKind { kVerdict, kCornerTest, kQuad };

// Device exact tier over the n gathered elements in `pts` (device), then the
// host tier for those it leaves (coordinate spans beyond its integers, or
// exact subdivision when the store has no room for a path); results in `v`
// (device) and `hv`
// (host).  Returns the number settled on the host.
static int exact_tier(Workspace& w, const double* pts, uint8_t* v, uint8_t* hv, double* hpts, int64_t n,
                      int per, ExactKind kind, int max_depth, hipStream_t s, int64_t* host_count)
{
    launch_exact_device(pts, v, n, kind == ExactKind::kQuad ? 2 : kind == ExactKind::kCornerTest ? 1 : 0,
                        max_depth, s);
    if (kind == ExactKind::kVerdict && max_depth > 0) {
        // exact subdivision on the device, the paths in the (idle) subdivision store
        const int64_t per_lane = (int64_t)(max_depth + 1) * kExactDfsWords * (int64_t)sizeof(IW);
        const int64_t lanes = (int64_t)(w.node_cap * sizeof(Node)) / per_lane;
        if (lanes > 0) launch_exact_dfs(pts, v, n, max_depth, w.nodes, lanes, s);
    }
    HX_HIP(hipGetLastError());
    HX_HIP(hipMemcpyAsync(hv, v, n, hipMemcpyDeviceToHost, s));
    HX_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> left;
    for (int64_t i = 0; i < n; ++i)
        if (hv[i] == kHostExact || hv[i] == kExactSubdivide) left.push_back(i);
    *host_count = (int64_t)left.size();
    if (left.empty()) return HEXVAL_OK;
    HX_HIP(hipMemcpyAsync(hpts, pts, n * per * sizeof(double), hipMemcpyDeviceToHost, s));
    HX_HIP(hipStreamSynchronize(s));
    const int64_t m = (int64_t)left.size();
    const int64_t nt = std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
    const int64_t chunk = (m + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min(m, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([&, lo, hi] {
            for (int64_t k = lo; k < hi; ++k) {
                const int64_t i = left[k];
                hv[i] = kind == ExactKind::kQuad         ? exact_quad(hpts + 8 * i)
                        : kind == ExactKind::kCornerTest ? exact_corner_test(hpts + 24 * i)
                                                         : exact_verdict(hpts + 24 * i, max_depth);
            }
        });
    }
    for (auto& x : th) x.join();
    HX_HIP(hipMemcpyAsync(v, hv, n, hipMemcpyHostToDevice, s));
    return HEXVAL_OK;
}

// ---------------------------------------------------------------- autotuner
// Launch shape of the first-pass kernel: threads per block (= elements per
// tile), a persistent grid of k blocks per CU (4, 8, 16 or 32) taking tiles
// at run time and, where the input may walk (a single mesh with trusted
// connectivity, or an FP64 batch of them), the column walk's layers per tile
// (0: plain tiles, or kWalkLayers).  Picked by timing every candidate twice
// on the call's own input (the better time counts; a walking candidate's
// time includes its stride search), cached per (device architecture,
// precision, gather mode, batched, log2 size bucket) and optionally persisted
// in the file named by HEXVAL_TUNE_CACHE (keys of version v4: earlier files
// recorded no walk choice for batches).  The per-element arithmetic never
// depends on the launch shape.

struct TuneChoice {
    int block = 256;
    int per_cu = 4;    // persistent grid of per_cu blocks per CU (tiles are handed out at run time)
    int walk = kWalkLayers;   // layers per column tile of the walking pass, 0 = plain tiles
};

static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(const char* arch, int precision, int gather, bool batched, int64_t total)
{
    int bucket = 0;
    while ((1ll << (bucket + 1)) <= total) ++bucket;
    char buf[128];
    snprintf(buf, sizeof buf, "v4/%s/p%d/g%d/b%d/n%d", arch, precision, gather, batched ? 1 : 0, bucket);
    return buf;
}

static void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("HEXVAL_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[128];
    int block, per_cu, walk;
    while (fscanf(f, "%127s %d %d %d", key, &block, &per_cu, &walk) == 4) {
        TuneChoice c;
        c.block = block;
        c.per_cu = per_cu;
        c.walk = walk;
        g_tune[key] = c;
    }
    fclose(f);
}

static void tune_store_locked(const std::string& key, const TuneChoice& c)
{
    g_tune[key] = c;
    const char* path = getenv("HEXVAL_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d\n", key.c_str(), c.block, c.per_cu, c.walk);
    fclose(f);
}

static int64_t grid_for(const TuneChoice& c, int64_t n_tiles, int cus)
{
    int64_t g = std::min<int64_t>(n_tiles, (int64_t)cus * std::max(c.per_cu, 1));
    return std::min<int64_t>(std::max<int64_t>(8, (g + 7) / 8 * 8), 1ll << 30);
}

bool autotune_enabled()
{
    const char* e = getenv("HEXVAL_AUTOTUNE");
    return !(e && e[0] == '0');
}

// ---------------------------------------------------------------- main loop

int run_check(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts,
              uint8_t* const* verdicts, double* const* mins)
{
    return run_check_ws(meshes, n_meshes, batched, opts, verdicts, mins, nullptr);
}

// Calls of at least this many elements launch subdivision without first
// reading the counters back.
constexpr int64_t kEagerSubdivision = 1ll << 20;

int run_check_ws(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts_in,
                 uint8_t* const* verdicts, double* const* mins, Workspace* fixed, bool tune)
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

    // Launch shape of the first pass: explicit options, else the tuning cache,
    // else (autotuning on) measured below on this input, else defaults.
    TuneChoice choice;
    bool tuned = false;   // choice from the tuning cache or measured on this call
    // a batch whose non-empty meshes all have trusted connectivity takes the
    // prefetching first pass (its own tuning key)
    bool batch_conn = batched && !o.validate_indices;
    for (int i = 0; batch_conn && i < n_meshes; ++i)
        if (meshes[i].n > 0 && !meshes[i].connectivity) batch_conn = false;
    const int gather = batched ? (batch_conn ? 4 : 0) : !meshes[0].connectivity ? 1 : (o.validate_indices ? 3 : 2);
    std::string key;
    bool need_tune = false;
    if (o.block_threads || o.grid_blocks) {
        if (o.block_threads) choice.block = o.block_threads;
    } else {
        key = tune_key(device_arch(dev), o.precision, gather, batched, total);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            choice = it->second;
            tuned = true;
        }
        else need_tune = tune && autotune_enabled();
    }
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
    auto count_tiles = [&](int blk) {
        int64_t t = 0;
        for (int i = 0; i < n_meshes; ++i) t += (meshes[i].n + blk - 1) / blk;
        return t;
    };

    WorkspaceGuard wg;
    if (!fixed && (rc = acquire_workspace(dev, &wg.w))) return rc;
    Workspace& w = fixed ? *fixed : *wg.w;
    if (fixed) {
        // a fixed workspace keeps its capacities; queue_capacity may only narrow the store
        node_cap = o.queue_capacity ? std::min<uint64_t>((uint64_t)o.queue_capacity, fixed->node_cap) : 0;
        list_cap = 0;
    }
    const int64_t max_tiles = count_tiles(need_tune ? 64 : choice.block);
    if ((rc = w.ensure(node_cap, list_cap, batched ? n_meshes : 1, batched ? max_tiles : 1))) return rc;
    QueueDev q = w.queue();
    // a pooled workspace may be larger than this call asked for
    if (node_cap) q.node_cap = std::min<uint64_t>(q.node_cap, node_cap);
    q.root_cap = q.node_cap;
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
        m.validate = (o.validate_indices && m.conn) ? 1 : 0;
    }
    const MeshDev* dmeshes = batched ? w.meshes : nullptr;
    int64_t n_tiles = 0;
    int tile_block = 0;
    // Tiles of `blk` elements; for a batch the mesh table and the
    // tile -> mesh table are rebuilt on the device.
    auto setup_tiles = [&](int blk) -> int {
        tile_block = blk;
        n_tiles = 0;
        for (int i = 0; i < n_meshes; ++i) {
            md[i].tile_begin = n_tiles;
            n_tiles += (meshes[i].n + blk - 1) / blk;
        }
        if (batched) {
            HX_HIP(hipStreamSynchronize(s));   // h_meshes may still be in use
            memcpy(w.h_meshes, md.data(), n_meshes * sizeof(MeshDev));
            HX_HIP(hipMemcpyAsync(w.meshes, w.h_meshes, n_meshes * sizeof(MeshDev), hipMemcpyHostToDevice, s));
            launch_tile_table(w.meshes, n_meshes, blk, w.tile_mesh, s);
        } else {
            single = md[0];
        }
        return HEXVAL_OK;
    };
    const bool timing = st && st->timing && w.ev[0];   // workspaces without events do not time
    const int xcds = 8;
    // A single mesh with trusted connectivity, or a batch of them, may walk
    // columns of stacked elements (k_top_f64_walk, k_filter_f32_walk,
    // k_top_f64_batch_walk): the tuned choice, unless the options fix it
    // (meshes of fewer than 8 layers of the smallest stride walked are not
    // searched: the search costs more than the walk could save there)
    // (batches walk in FP64 only, see k_top_f64_batch_walk)
    bool walk_able = !batched && gather == 2 && total >= 8 * kWalkMinStride;
    for (int i = 0; batched && batch_conn && o.precision == HEXVAL_FP64 && i < n_meshes && !walk_able; ++i)
        walk_able = meshes[i].n >= 8 * kWalkMinStride;
    if (o.walk_layers) choice.walk = o.walk_layers > 0 ? o.walk_layers : 0;
    // an untuned batch (the server's calls) checks in plain tiles: the
    // per-mesh stride search costs more than the walk saves on most batches
    // of small meshes
    else if (batched && !tuned && !need_tune) choice.walk = 0;
    int walk_now = walk_able ? choice.walk : 0;   // layers of the pass being launched
    bool walk = walk_now > 0;
    auto first_args = [&]() {
        TopArgs ta{};
        ta.mesh = single;
        ta.meshes = dmeshes;
        ta.tile_mesh = batched && walk ? w.walk_tile_mesh : w.tile_mesh;
        ta.walk_meshes = batched && walk ? w.walk_meshes : nullptr;
        ta.n_tiles = n_tiles;
        ta.list_count = &w.cnt->n_list;
        ta.q = q;
        ta.max_depth = o.max_depth;
        ta.xcds = xcds;
        ta.batch_conn = batch_conn ? 1 : 0;
        ta.walk_layers = walk ? walk_now : 0;
        ta.walk_limit = walk && !batched ? std::min<int64_t>(total, kWalkSearch) : 0;
        return ta;
    };
    // the column walk needs the stack stride of this mesh (of each mesh of a
    // batch, and the batch's walking tiles), found after each counter reset
    // (the walking pass reads them on the device)
    auto reset = [&]() {
        launch_reset(w.cnt, s);
        if (walk && batched)
            launch_batch_walk(w.meshes, n_meshes, tile_block, walk_now, w.walk_meshes, w.walk_tile_mesh, w.cnt, s);
        else if (walk)
            launch_walk_detect(single.conn, total, std::min<int64_t>(total, kWalkSearch), w.cnt, s);
    };
    auto launch_first = [&](const TopArgs& ta, int64_t g, int blk) {
        if (o.precision == HEXVAL_FP32_FILTER) launch_filter_range(ta, batched, (int)g, blk, s);
        else launch_top_range(ta, batched, (int)g, blk, s);
    };
    if (need_tune) {
        static const int kBlocks[3] = {64, 128, 256};
        static const int kPerCu[4] = {4, 8, 16, 32};
        const int n_walk = walk_able && !o.walk_layers ? 2 : 1;
        const TuneChoice fixed_walk = choice;
        float best = 1e30f;
        for (int blk : kBlocks) {
            if ((rc = setup_tiles(blk))) return rc;
            for (int k = 0; k < 4 * n_walk; ++k) {
                TuneChoice c;
                c.block = blk;
                c.per_cu = kPerCu[k % 4];
                c.walk = n_walk == 2 ? (k < 4 ? 0 : kWalkLayers) : fixed_walk.walk;
                walk_now = walk_able ? c.walk : 0;
                walk = walk_now > 0;
                const int64_t g = grid_for(c, n_tiles, cus);
                float ms = 0.0f;
                for (int rep = 0; rep < 2; ++rep) {
                    // the walk's stride search is part of what a candidate costs
                    HX_HIP(hipEventRecord(w.ev[0], s));
                    reset();
                    launch_first(first_args(), g, blk);
                    HX_HIP(hipEventRecord(w.ev[1], s));
                    HX_HIP(hipGetLastError());
                    HX_HIP(hipEventSynchronize(w.ev[1]));
                    HX_HIP(hipEventElapsedTime(&ms, w.ev[0], w.ev[1]));
                }
                if (ms < best) {
                    best = ms;
                    choice = c;
                }
            }
        }
        walk_now = walk_able ? choice.walk : 0;
        walk = walk_now > 0;
        if (!o.walk_layers) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_store_locked(key, choice);
        }
    }
    if ((rc = setup_tiles(choice.block))) return rc;
    const int block = choice.block;
    int64_t grid = o.grid_blocks ? std::max<int64_t>(8, (o.grid_blocks + 7) / 8 * 8) : grid_for(choice, n_tiles, cus);
    grid = std::min<int64_t>(grid, 1ll << 30);
    if (st) {
        st->block_threads = block;
        st->grid_blocks = grid;
        st->walk_layers = walk_now;
    }
    const int list_grid = cus * 8;
    // 4 blocks per CU: empty levels cost less to launch than at 8, and large
    // levels run as fast (2 per CU was 17% slower on them)
    const int level_grid = cus * 4;

    uint64_t prev_remaining = 0;
    // Once a round listing a single element still overflows the store, the
    // elements left are decided depth first, one lane each, with their path
    // of sub-boxes in the store (k_dfs): bounded memory, the same verdicts.
    bool dfs_round = false;
    const int64_t dfs_lanes = (int64_t)(q.node_cap / (uint64_t)(o.max_depth + 1));
    for (int round = 0;; ++round) {
        if (round == 0) reset();
        else launch_reset(w.cnt, s);
        const TopArgs ta = first_args();
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[0], s));
        const bool filter = round == 0 && o.precision == HEXVAL_FP32_FILTER;
        if (filter) {
            launch_filter_range(ta, batched, (int)grid, block, s);
            if (timing) HX_HIP(hipEventRecord(w.ev[3], s));
            launch_top_list(ta, batched, list_grid, block, s);
        } else if (round == 0) {
            launch_top_range(ta, batched, (int)grid, block, s);
        } else {
            CollectArgs ca{q, single, dmeshes, batched ? n_meshes : 1};
            launch_collect_deferred(ca, list_grid, s);
            if (dfs_round) {
                DfsArgs da{q, single, dmeshes, dfs_lanes, o.max_depth, 0};
                launch_dfs(da, s);
            } else {
                launch_top_list(ta, batched, list_grid, block, s);
            }
        }
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[1], s));
        HX_HIP(hipGetLastError());
        // Subdivision: its kernels read the list sizes on the device and do
        // nothing when the list is empty.  Large calls launch it right away
        // (a host round trip costs more than the launches, and such meshes
        // usually list some element); small ones read the counters first and
        // skip it when nothing was listed.
        bool subdivide = !dfs_round;
        if (subdivide && total < kEagerSubdivision) {
            HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HX_HIP(hipStreamSynchronize(s));
            subdivide = w.hcnt->n_sub > 0;
        }
        if (subdivide) {
            RootArgs ra{q, single, dmeshes};
            launch_roots(ra, cus * 2, s);
            for (int L = 0; L < o.max_depth; ++L) {
                LevelArgs la{q, L, o.max_depth};
                launch_level(la, level_grid, s);
            }
            FoldArgs fa{q, single, dmeshes};
            launch_fold(fa, cus * 2, s);
            HX_HIP(hipGetLastError());
            HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        } else if (dfs_round) {
            HX_HIP(hipGetLastError());
            HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        }
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[2], s));
        HX_HIP(hipStreamSynchronize(s));
        const Counters c = *w.hcnt;
        if (st) {
            st->n_subdivided += (int64_t)std::min<uint64_t>(c.n_sub, q.root_cap);
            // children evaluated: 8 per stored sub-box of levels 0..max_depth-1
            uint64_t base = 0;
            for (int L = 0; L < o.max_depth && c.n_sub > 0; ++L) {
                const uint64_t cnt_l = std::min<uint64_t>(c.lvl[L], q.node_cap - base);
                base += cnt_l;
                st->n_nodes += 8 * (int64_t)cnt_l;
                if (cnt_l) st->max_level = std::max<int32_t>(st->max_level, L + 1);
            }
            st->n_rounds = round + 1;
            if (round == 0) {
                st->n_elements = total;
                if (walk && !batched && c.walk_code) {
                    // the stride the walking pass used (it walks none below kWalkMinStride)
                    const int64_t stride = std::min<int64_t>(total, kWalkSearch) - (int64_t)c.walk_code;
                    st->walk_stride = stride >= kWalkMinStride && stride < total ? stride : 0;
                }
                if (o.precision == HEXVAL_FP32_FILTER)
                    st->n_recheck = (int64_t)std::min<uint64_t>(c.n_list, q.list_cap) + (int64_t)c.n_rechecked;
                if (timing && o.precision == HEXVAL_FP32_FILTER) {
                    hipEventElapsedTime(&st->ms_first_pass, w.ev[0], w.ev[3]);
                    hipEventElapsedTime(&st->ms_recheck, w.ev[3], w.ev[1]);
                    hipEventElapsedTime(&st->ms_subdivision, w.ev[1], w.ev[2]);
                    hipEventElapsedTime(&st->ms_total, w.ev[0], w.ev[2]);
                } else if (timing) {
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
            int64_t on_host = 0;
            if ((rc = exact_tier(w, w.exact_pts, w.exact_v, w.h_exact_v, w.h_exact_pts, n_ex, 24,
                                 ExactKind::kVerdict, o.max_depth, s, &on_host)))
                return rc;
            if (st) st->n_exact_host += (int32_t)on_host;
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
            if (c.n_deferred >= listed) {
                // nothing completed: the listed elements' trees crowded each
                // other out; list fewer per round, down to one at a time,
                // then go depth first
                if (dfs_round || (q.root_cap <= 1 && dfs_lanes < 1))
                    return fail(HEXVAL_E_QUEUE, "subdivision queue of %llu nodes too small to make progress",
                                (unsigned long long)q.node_cap);
                if (q.root_cap <= 1) dfs_round = true;
                q.root_cap = std::max<uint64_t>(1, q.root_cap / 8);
            }
            remaining = prev_remaining - listed + c.n_deferred;
        }
        if (remaining == 0) break;
        prev_remaining = remaining;
    }
    return HEXVAL_OK;
}

// Certified bounds of min J: first pass (root bounds), then one launch per
// level for the elements whose bounds are not yet within the tolerance.
int run_min_jacobian(const hexval_mesh_t* mesh, const hexval_opts_t* opts_in, double rtol, double* lo, double* hi,
                     uint8_t* status)
{
    hexval_opts_t o;
    if (opts_in) o = *opts_in;
    else default_opts(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (o.precision != HEXVAL_FP64) return fail(HEXVAL_E_ARG, "hexval_min_jacobian computes in FP64 only");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(HEXVAL_E_ARG, "rtol must be finite and > 0");
    if (!mesh) return fail(HEXVAL_E_ARG, "mesh is NULL");
    if (mesh->n > 0 && (!lo || !hi)) return fail(HEXVAL_E_ARG, "lo or hi is NULL");
    if ((rc = check_mesh(mesh, lo, o.validate_indices, 0))) return rc;
    hexval_stats_t* st = o.stats;
    if (st) {
        const int timing = st->timing;
        memset(st, 0, sizeof *st);
        st->timing = timing;
    }
    const int64_t n = mesh->n;
    if (n == 0) return HEXVAL_OK;
    int dev, cus;
    if ((rc = current_device(&dev, &cus))) return rc;
    hipStream_t s = (hipStream_t)o.stream;

    // Every split box stores its 8 children: room for as many boxes as
    // elements by default (at least 2^19, at most 2^26 = 17 GiB).
    const uint64_t node_cap = o.queue_capacity
                                  ? (uint64_t)o.queue_capacity
                                  : pow2_ceil(std::min<uint64_t>(std::max<uint64_t>((uint64_t)n, 1u << 19), 1ull << 26));
    WorkspaceGuard wg;
    if ((rc = acquire_workspace(dev, &wg.w))) return rc;
    Workspace& w = *wg.w;
    if ((rc = w.ensure(node_cap, 0, 1, 1))) return rc;
    QueueDev q = w.queue();
    q.node_cap = std::min<uint64_t>(q.node_cap, node_cap);
    q.root_cap = q.node_cap;
    if ((rc = w.ensure_minj(q.node_cap, (uint64_t)n))) return rc;

    MinjArgs a{};
    a.q = q;
    a.mesh.points = mesh->points;
    a.mesh.conn = mesh->connectivity;
    a.mesh.n = n;
    a.mesh.n_points = mesh->n_points;
    a.mesh.validate = (o.validate_indices && mesh->connectivity) ? 1 : 0;
    for (int k = 0; k < 3; ++k) a.mj.u[k] = w.minj + (uint64_t)k * w.minj_cap;
    a.mj.ufinal = w.minj + 3 * w.minj_cap;
    a.mj.lb = w.minj + 4 * w.minj_cap;
    a.mj.rtol = rtol;
    a.mj.lo = lo;
    a.mj.hi = hi;
    a.mj.status = status;
    a.max_depth = o.max_depth;
    a.xcds = 8;
    const bool timing = st && st->timing;
    // the first round over a trusted mesh walks columns of stacked elements
    // (k_minj_top_walk) unless the options ask for plain tiles
    const bool walk = mesh->connectivity && !o.validate_indices && o.walk_layers >= 0 && n >= 8 * kWalkMinStride;
    const int64_t walk_limit = std::min<int64_t>(n, kWalkSearch);

    // Rounds: a round subdivides at most root_cap elements (a quarter of the
    // store, the rest being room for their boxes); elements past it, or that
    // run out of room, are redone from scratch in the next round.  When a
    // round completes nothing, root_cap shrinks; at one element, the next
    // round is final: that element reports QUEUE_FULL if it still does not
    // fit, and root_cap starts over.
    int64_t* lists[2] = {w.minj_defer, w.minj_defer + w.defer_cap};
    int64_t count = n;
    bool final_round = false;
    const uint64_t root_cap0 = std::max<uint64_t>(1, q.node_cap / 4);
    uint64_t root_cap = root_cap0;
    uint64_t tot_sub = 0, tot_nodes = 0;
    int max_level = 0;
    for (int round = 0;; ++round) {
        a.in_list = round == 0 ? nullptr : lists[(round + 1) & 1];
        a.in_count = round == 0 ? 0 : count;
        a.out_list = lists[round & 1];
        a.final_round = final_round ? 1 : 0;
        a.root_cap = root_cap;
        a.n_tiles = (count + 255) / 256;
        a.walk_layers = round == 0 && walk ? (o.walk_layers > 0 ? o.walk_layers : kWalkLayers) : 0;
        a.walk_limit = walk_limit;
        launch_reset(w.cnt, s);
        if (a.walk_layers) launch_walk_detect(mesh->connectivity, n, walk_limit, w.cnt, s);
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[0], s));
        launch_minj_top(a, cus * 4, s);   // 4 blocks per CU: 2-3% faster than 8 on the 400^3 lattice
        if (timing && round == 0) HX_HIP(hipEventRecord(w.ev[1], s));
        HX_HIP(hipGetLastError());
        // subdivision follows on the device (empty lists do nothing)
        {
            launch_minj_roots(a, cus * 2, s);
            for (int L = 0; L <= o.max_depth; ++L) {
                a.level = L;
                launch_minj_level(a, cus * 8, s);
            }
            launch_minj_fold(a, cus * 2, s);
            HX_HIP(hipGetLastError());
            HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        }
        HX_HIP(hipStreamSynchronize(s));
        const Counters& c = *w.hcnt;
        tot_sub += std::min<uint64_t>(c.n_sub, root_cap);
        // boxes stored below the roots, and the deepest level holding any
        uint64_t base = 0;
        for (int L = 0; L <= o.max_depth + 1 && L < kMaxDepth + 4 && c.n_sub > 0; ++L) {
            const uint64_t room = L == 0 ? q.node_cap - base : (q.node_cap - base) & ~7ull;
            const uint64_t cnt_l = std::min<uint64_t>(c.lvl[L], room);
            base += cnt_l;
            if (L > 0) tot_nodes += cnt_l;
            if (cnt_l) max_level = std::max(max_level, L);
        }
        if (st) st->n_rounds = round + 1;
        if (c.n_deferred == 0) break;
        if (final_round) {
            final_round = false;
            root_cap = root_cap0;
        } else if (c.n_deferred == (uint64_t)count) {   // nothing completed
            if (root_cap > 1) root_cap = std::max<uint64_t>(1, root_cap / 8);
            else final_round = true;
        }
        count = (int64_t)c.n_deferred;
    }
    if (timing) {
        HX_HIP(hipEventRecord(w.ev[2], s));
        HX_HIP(hipEventSynchronize(w.ev[2]));
    }
    if (st) {
        st->n_elements = n;
        st->n_subdivided = (int64_t)tot_sub;
        st->n_nodes = (int64_t)tot_nodes;
        st->max_level = max_level;
        st->walk_layers = walk ? (o.walk_layers > 0 ? o.walk_layers : kWalkLayers) : 0;
        if (timing) {
            hipEventElapsedTime(&st->ms_first_pass, w.ev[0], w.ev[1]);
            hipEventElapsedTime(&st->ms_subdivision, w.ev[1], w.ev[2]);
            hipEventElapsedTime(&st->ms_total, w.ev[0], w.ev[2]);
        }
    }
    return HEXVAL_OK;
}

// Corner-only test and corner quality, or linear quadrangles: one pass, then
// the exact tier for the elements whose signs are not certified (in batches
// of the exact list's capacity).
static int run_corner_or_quad(const hexval_mesh_t* mesh, const hexval_opts_t* opts_in, uint8_t* test1,
                              double* quality, bool quad)
{
    hexval_opts_t o;
    if (opts_in) o = *opts_in;
    else default_opts(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (!mesh) return fail(HEXVAL_E_ARG, "mesh is NULL");
    if ((rc = check_mesh(mesh, test1, o.validate_indices, 0))) return rc;
    hexval_stats_t* st = o.stats;
    if (st) {
        const int timing = st->timing;
        memset(st, 0, sizeof *st);
        st->timing = timing;
    }
    const int64_t n = mesh->n;
    if (n == 0) return HEXVAL_OK;
    int dev, cus;
    if ((rc = current_device(&dev, &cus))) return rc;
    hipStream_t s = (hipStream_t)o.stream;
    WorkspaceGuard wg;
    if ((rc = acquire_workspace(dev, &wg.w))) return rc;
    Workspace& w = *wg.w;
    if ((rc = w.ensure(0, 0, 1, 1))) return rc;
    CornerArgs a{};
    a.q = w.queue();
    a.mesh.points = mesh->points;
    a.mesh.conn = mesh->connectivity;
    a.mesh.n = n;
    a.mesh.n_points = mesh->n_points;
    a.mesh.validate = (o.validate_indices && mesh->connectivity) ? 1 : 0;
    a.mesh.verdict = test1;
    a.quality = quality;
    a.n_tiles = (n + 255) / 256;
    a.xcds = 8;
    // quadrangles with trusted connectivity walk their rows (k_quad_walk)
    // unless the options ask for plain tiles
    const bool walk = quad && mesh->connectivity && !o.validate_indices && o.walk_layers >= 0 &&
                      n >= 8 * kWalkMinStride;
    a.walk_layers = walk ? (o.walk_layers > 0 ? o.walk_layers : kWalkLayers) : 0;
    a.walk_limit = std::min<int64_t>(n, kWalkSearch);
    const bool timing = st && st->timing;
    launch_reset(w.cnt, s);
    if (walk) launch_quad_walk_detect(mesh->connectivity, n, a.walk_limit, w.cnt, s);
    if (timing) HX_HIP(hipEventRecord(w.ev[0], s));
    // 8 blocks per CU, 7 for the quadrangle walk (70 VGPRs: 7 waves per SIMD)
    const int grid = o.grid_blocks ? (int)std::max<int64_t>(8, (o.grid_blocks + 7) / 8 * 8) : cus * (walk ? 7 : 8);
    if (quad) launch_quad_check(a, grid, s);
    else launch_corner_test(a, grid, s);
    if (timing) HX_HIP(hipEventRecord(w.ev[1], s));
    HX_HIP(hipGetLastError());
    HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HX_HIP(hipStreamSynchronize(s));
    uint64_t pending = w.hcnt->n_exact, settled = 0;
    const uint64_t walk_code = w.hcnt->walk_code;
    int64_t on_host = 0;
    while (pending > 0) {
        const int64_t k = (int64_t)std::min<uint64_t>(pending, w.exact_cap);
        if (quad) {
            launch_quad_gather(a, k, w.exact_pts, s);
        } else {
            GatherArgs ga{a.q, a.mesh, nullptr, k, w.exact_pts};
            launch_gather_exact(ga, s);
        }
        int64_t on_host_k = 0;
        if ((rc = exact_tier(w, w.exact_pts, w.exact_v, w.h_exact_v, w.h_exact_pts, k, quad ? 8 : 24,
                             quad ? ExactKind::kQuad : ExactKind::kCornerTest, 0, s, &on_host_k)))
            return rc;
        on_host += on_host_k;
        MeshDev sm = a.mesh;
        sm.min_coeff = nullptr;
        ScatterArgs sa{a.q, sm, nullptr, k, w.exact_v};
        launch_scatter_exact(sa, s);
        settled += (uint64_t)k;
        if (pending == (uint64_t)k) break;
        launch_reset(w.cnt, s);
        launch_corner_collect(a, cus * 8, s);
        HX_HIP(hipGetLastError());
        HX_HIP(hipMemcpyAsync(w.hcnt, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HX_HIP(hipStreamSynchronize(s));
        pending = w.hcnt->n_exact;
    }
    if (timing) HX_HIP(hipEventRecord(w.ev[2], s));
    HX_HIP(hipStreamSynchronize(s));
    if (st) {
        st->n_elements = n;
        st->n_exact = (int64_t)settled;
        st->n_exact_host = (int32_t)on_host;
        st->n_rounds = 1;
        st->walk_layers = a.walk_layers;
        if (walk && walk_code) {
            // the row stride the walking pass used (it walks none below kWalkMinStride)
            const int64_t stride = a.walk_limit - (int64_t)walk_code;
            st->walk_stride = stride >= kWalkMinStride && stride < n ? stride : 0;
        }
        if (timing) {
            hipEventElapsedTime(&st->ms_first_pass, w.ev[0], w.ev[1]);
            hipEventElapsedTime(&st->ms_total, w.ev[0], w.ev[2]);
        }
    }
    return HEXVAL_OK;
}

int run_corner_test(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* test1, double* quality)
{
    return run_corner_or_quad(mesh, opts, test1, quality, false);
}

int run_quad_check(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts, double* min_j)
{
    return run_corner_or_quad(mesh, opts, verdicts, min_j, true);
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

// ---------------------------------------------------------------- allocation-free check
// hexval_check_noalloc runs on buffers carved from `scratch`, a fixed device
// array of this library, and on fixed host arrays: the call allocates no
// device or pinned host memory.  Capacities: a subdivision store of 2^17
// sub-boxes (it holds one element's tree whose ambiguous region is a surface
// up to depth 8, the deepest such a call accepts), a recheck/deferred list of
// 2^17 entries and exact-tier staging for 2^13 elements; elements past these
// are checked in later rounds, as with any workspace.  Every call on a device
// uses that device's one copy: concurrent calls on one device race.

constexpr uint64_t kNaNodes = 1ull << 17;
constexpr uint64_t kNaList = 1ull << 17;
constexpr uint64_t kNaExact = 1ull << 13;
constexpr int kNaMaxDepth = 8;
constexpr int kNaMaxDevices = 16;

constexpr uint64_t na_align(uint64_t x) { return (x + 255) & ~255ull; }
constexpr uint64_t kNaOffCnt = 0;
constexpr uint64_t kNaOffNodes = na_align(kNaOffCnt + sizeof(Counters));
constexpr uint64_t kNaOffSubElem = na_align(kNaOffNodes + kNaNodes * sizeof(Node));
constexpr uint64_t kNaOffSubMesh = na_align(kNaOffSubElem + kNaNodes * sizeof(int64_t));
constexpr uint64_t kNaOffSubFlags = na_align(kNaOffSubMesh + kNaNodes * sizeof(int32_t));
constexpr uint64_t kNaOffListElem = na_align(kNaOffSubFlags + kNaNodes * sizeof(uint32_t));
constexpr uint64_t kNaOffListMesh = na_align(kNaOffListElem + kNaList * sizeof(int64_t));
constexpr uint64_t kNaOffExactElem = na_align(kNaOffListMesh + kNaList * sizeof(int32_t));
constexpr uint64_t kNaOffExactMesh = na_align(kNaOffExactElem + kNaExact * sizeof(int64_t));
constexpr uint64_t kNaOffExactPts = na_align(kNaOffExactMesh + kNaExact * sizeof(int32_t));
constexpr uint64_t kNaOffExactV = na_align(kNaOffExactPts + kNaExact * 24 * sizeof(double));
constexpr uint64_t kScratchBytes = na_align(kNaOffExactV + kNaExact);

// One copy per device (loaded with the library's code object on that
// device).  Host code must not use this name as an address: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Host staging of the allocation-free path (counters read back, exact-tier
// points and verdicts), one per device.
struct NoAllocHost {
    Counters cnt;
    double pts[kNaExact * 24];
    uint8_t v[kNaExact];
};
static NoAllocHost g_na_host[kNaMaxDevices];

struct NoAllocDevice {
    std::once_flag once;
    int rc = HEXVAL_OK;
    char msg[256] = {0};
    Workspace ws;
};
static NoAllocDevice g_na[kNaMaxDevices];

// Set-up on the first call on device dev (that device current): the address
// of this device's scratch array, and a workspace whose buffers point into it.
static int noalloc_workspace(int dev, Workspace** out)
{
    if (dev >= kNaMaxDevices)
        return fail(HEXVAL_E_ARG, "hexval_check_noalloc supports devices 0..%d, not %d", kNaMaxDevices - 1, dev);
    NoAllocDevice& d = g_na[dev];
    std::call_once(d.once, [&] {
        unsigned char* p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hipGetLastError();
            d.rc = HEXVAL_E_HIP;
            snprintf(d.msg, sizeof d.msg, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                     hipGetErrorString(e));
            return;
        }
        Workspace& w = d.ws;
        NoAllocHost& h = g_na_host[dev];
        w.borrowed = true;
        w.device = dev;
        w.cnt = reinterpret_cast<Counters*>(p + kNaOffCnt);
        w.nodes = reinterpret_cast<Node*>(p + kNaOffNodes);
        w.sub_elem = reinterpret_cast<int64_t*>(p + kNaOffSubElem);
        w.sub_mesh = reinterpret_cast<int32_t*>(p + kNaOffSubMesh);
        w.sub_flags = reinterpret_cast<uint32_t*>(p + kNaOffSubFlags);
        w.list_elem = reinterpret_cast<int64_t*>(p + kNaOffListElem);
        w.list_mesh = reinterpret_cast<int32_t*>(p + kNaOffListMesh);
        w.exact_elem = reinterpret_cast<int64_t*>(p + kNaOffExactElem);
        w.exact_mesh = reinterpret_cast<int32_t*>(p + kNaOffExactMesh);
        w.exact_pts = reinterpret_cast<double*>(p + kNaOffExactPts);
        w.exact_v = p + kNaOffExactV;
        w.hcnt = &h.cnt;
        w.h_exact_pts = h.pts;
        w.h_exact_v = h.v;
        w.node_cap = kNaNodes;
        w.list_cap = kNaList;
        w.exact_cap = kNaExact;
        w.mesh_cap = 1;   // single-mesh calls only: the mesh and tile tables stay unused
        w.tile_cap = 1;
    });
    if (d.rc) return fail(d.rc, "%s", d.msg);
    *out = &d.ws;
    return HEXVAL_OK;
}

int run_check_noalloc(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts, double* mins)
{
    if (!mesh) return fail(HEXVAL_E_ARG, "mesh is NULL");
    hexval_opts_t o;
    if (opts) o = *opts;
    else default_opts(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (o.max_depth > kNaMaxDepth)
        return fail(HEXVAL_E_ARG, "hexval_check_noalloc: max_depth %d exceeds %d, the deepest its fixed store of "
                    "%llu sub-boxes is sized for", o.max_depth, kNaMaxDepth, (unsigned long long)kNaNodes);
    if ((uint64_t)o.queue_capacity > kNaNodes)
        return fail(HEXVAL_E_ARG, "hexval_check_noalloc: queue_capacity %lld exceeds its fixed store of %llu sub-boxes",
                    (long long)o.queue_capacity, (unsigned long long)kNaNodes);
    if ((rc = check_mesh(mesh, verdicts, o.validate_indices, 0))) return rc;
    if (mesh->n == 0) {
        if (o.stats) {
            const int timing = o.stats->timing;
            memset(o.stats, 0, sizeof *o.stats);
            o.stats->timing = timing;
        }
        return HEXVAL_OK;
    }
    int dev;
    if ((rc = current_device(&dev, nullptr))) return rc;
    Workspace* w = nullptr;
    if ((rc = noalloc_workspace(dev, &w))) return rc;
    return run_check_ws(mesh, 1, false, &o, &verdicts, &mins, w, false);
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

int hexval_corner_test(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* test1, double* quality)
{
    return run_corner_test(mesh, opts, test1, quality);
}

int hexval_quad_check(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts, double* min_j)
{
    return run_quad_check(mesh, opts, verdicts, min_j);
}

int hexval_min_jacobian(const hexval_mesh_t* mesh, const hexval_opts_t* opts, double rtol, double* lo, double* hi,
                        uint8_t* status)
{
    return run_min_jacobian(mesh, opts, rtol, lo, hi, status);
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

int hexval_check_noalloc(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts,
                         double* min_coeffs)
{
    return run_check_noalloc(mesh, opts, verdicts, min_coeffs);
}

const char* hexval_last_error(void) { return last_error(); }

}  // extern "C"
