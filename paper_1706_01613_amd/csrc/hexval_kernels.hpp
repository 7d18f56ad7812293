// Kernel argument blocks and host-side launchers (defined in hexval_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "hexval_internal.hpp"

namespace hexval {

struct TopArgs {
    MeshDev mesh;                         // single-mesh calls
    const MeshDev* meshes;                // batched calls (device array) or nullptr
    const int32_t* tile_mesh;             // batched: global tile -> mesh
    int64_t n_tiles;                      // range mode
    const unsigned long long* list_count; // list mode: number of entries
    QueueDev q;
    int32_t max_depth;
    int32_t xcds;                         // tile chunks (1 or 8)
    int32_t batch_conn;                   // batched: every mesh with tiles has trusted connectivity
    int32_t walk_layers;                  // trusted connectivity: layers per column tile (0: no walk)
    int64_t walk_limit;                   // elements searched for the stack stride (see k_walk_detect)
    const WalkMesh* walk_meshes;          // batched walk: per-mesh strides and tile ranges
};

struct LevelArgs {
    QueueDev q;
    int32_t level;       // level of the stored sub-boxes expanded
    int32_t max_depth;
};

struct RootArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
};

struct FoldArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
};

// Depth-first subdivision of listed elements in bounded memory: lane i keeps
// its path of sub-boxes in nodes [i (max_depth+1), (i+1) (max_depth+1)) of
// the store.
struct DfsArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
    int64_t lanes;        // stacks that fit in the store
    int32_t max_depth;
    int32_t pad;
};

struct CollectArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
    int32_t n_meshes;
};

struct GatherArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
    int64_t n;
    double* out;   // [n,24]
};

struct ScatterArgs {
    QueueDev q;
    MeshDev mesh;
    const MeshDev* meshes;
    int64_t n;
    const uint8_t* verdicts;  // [n]
};

// Minimum of J to a tolerance: per subdivided element (slot) arrays of
// doubles kept in an order-preserving unsigned encoding (atomicMin).
struct MinjDev {
    uint64_t* u[3];      // [node_cap] smallest corner value up to a level (rotating by level)
    uint64_t* ufinal;    // [node_cap] smallest corner value met at any level
    uint64_t* lb;        // [node_cap] smallest lower bound of a retired box
    double rtol;
    double* lo;          // [n] outputs
    double* hi;
    uint8_t* status;     // [n] or nullptr
};

struct MinjArgs {
    QueueDev q;
    MeshDev mesh;
    MinjDev mj;
    int64_t n_tiles;
    const int64_t* in_list;   // later rounds: the elements to redo (nullptr: all n)
    int64_t in_count;
    int64_t* out_list;        // elements deferred to the next round (room for n)
    uint64_t root_cap;        // elements subdivided in this round at most (the rest are deferred)
    int32_t final_round;      // 1: an element out of room reports QUEUE_FULL instead of deferral
    int32_t level;
    int32_t max_depth;
    int32_t xcds;
    int32_t walk_layers;      // first round over a trusted mesh: layers per column tile (0: no walk)
    int64_t walk_limit;       // elements searched for the stack stride
};

// Corner-only test and corner quality (hexval_corner_test).
struct CornerArgs {
    QueueDev q;
    MeshDev mesh;        // mesh.verdict = the test1 output
    double* quality;     // [n] or nullptr
    int64_t n_tiles;
    int32_t xcds;
    int32_t walk_layers; // quadrangles with trusted connectivity: rows per column tile (0: plain tiles)
    int64_t walk_limit;  // quads searched for the row stride
};

void launch_corner_test(const CornerArgs& a, int grid, hipStream_t s);
// Linear quadrangles (hexval_quad_check): mesh.points are 2D, mesh.conn [n,4];
// `quality` carries min_j.
void launch_quad_check(const CornerArgs& a, int grid, hipStream_t s);
void launch_quad_gather(const CornerArgs& a, int64_t n, double* out, hipStream_t s);
// Row stride of a quadrangle mesh with trusted connectivity (the smallest
// r < limit with quad r's corners 0, 1 = quad 0's corners 3, 2) and the
// first row whose quad 0 does not sit on the row below, into c->walk_code /
// c->walk_break as launch_walk_detect does for hexahedra (after launch_reset).
void launch_quad_walk_detect(const int32_t* conn, int64_t n, int64_t limit, Counters* c, hipStream_t s);
void launch_corner_collect(const CornerArgs& a, int grid, hipStream_t s);

void launch_minj_top(const MinjArgs& a, int grid, hipStream_t s);
void launch_minj_roots(const MinjArgs& a, int grid, hipStream_t s);
void launch_minj_level(const MinjArgs& a, int grid, hipStream_t s);
void launch_minj_fold(const MinjArgs& a, int grid, hipStream_t s);

void launch_top_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
// Column walk of the first pass over a single mesh with trusted
// connectivity: the stack stride is searched among the first kWalkSearch
// elements, and the layers it holds for counted (launch_walk_detect, after
// launch_reset; the walking pass reads both from the Counters); a tile spans
// kWalkLayers layers.
constexpr int64_t kWalkSearch = 1ll << 22;
constexpr int kWalkLayers = 16;
// Smallest stride walked (below it a column tile would leave too many lanes
// idle).
constexpr int64_t kWalkMinStride = 4096;
void launch_walk_detect(const int32_t* conn, int64_t n, int64_t limit, Counters* c, hipStream_t s);
// The same for every mesh of a batch of trusted meshes (each searched among
// its first n / 8 elements, at most kWalkSearch; meshes below
// 8 * kWalkMinStride elements are not walked), then the walking pass's tiles
// of `block` columns and `layers` layers: per-mesh ranges in wm, the
// tile -> mesh table in tile_mesh (at most one entry per plain tile of
// `block` elements: a mesh that would need more tiles walking is checked in
// plain tiles), their count in c->walk_tiles.  After launch_reset.
void launch_batch_walk(const MeshDev* meshes, int n_meshes, int block, int layers, WalkMesh* wm,
                       int32_t* tile_mesh, Counters* c, hipStream_t s);
void launch_filter_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
void launch_top_list(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
void launch_level(const LevelArgs& a, int grid, hipStream_t s);
void launch_roots(const RootArgs& a, int grid, hipStream_t s);
void launch_fold(const FoldArgs& a, int grid, hipStream_t s);
void launch_reset(Counters* c, hipStream_t s);
void launch_tile_table(const MeshDev* meshes, int n_meshes, int tile, int32_t* tile_mesh, hipStream_t s);
void launch_collect_deferred(const CollectArgs& a, int grid, hipStream_t s);
// Decides the listed elements (Q.list_elem, n_list entries) with a
// depth-first subdivision per lane: verdicts final, or kExact with the element
// on the exact list, or kDeferred when that list is full.
void launch_dfs(const DfsArgs& a, hipStream_t s);
void launch_gather_exact(const GatherArgs& a, hipStream_t s);
void launch_scatter_exact(const ScatterArgs& a, hipStream_t s);
void launch_coefficients(const MeshDev& m, double* out, hipStream_t s);
// Device exact tier over gathered points (mode 0 verdict, 1 corner-only test,
// 2 quadrangle); out[i] = result, or 0xFE where the host tier must decide.
void launch_exact_device(const double* pts, uint8_t* out, int64_t n, int mode, int max_depth, hipStream_t s);
// Exact subdivision of the elements launch_exact_device marked 0xFC, with
// `lanes` paths of (max_depth + 1) levels in `stack` (device memory of
// lanes * (max_depth + 1) * 28 * 48 bytes); results replace the marks.
void launch_exact_dfs(const double* pts, uint8_t* out, int64_t n, int max_depth, void* stack, int64_t lanes,
                      hipStream_t s);

}  // namespace hexval
