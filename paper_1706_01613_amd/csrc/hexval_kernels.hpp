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

void launch_top_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
void launch_filter_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
void launch_top_list(const TopArgs& a, bool batched, int grid, int block, hipStream_t s);
void launch_level(const LevelArgs& a, int grid, hipStream_t s);
void launch_roots(const RootArgs& a, int grid, hipStream_t s);
void launch_fold(const FoldArgs& a, int grid, hipStream_t s);
void launch_reset(Counters* c, hipStream_t s);
void launch_tile_table(const MeshDev* meshes, int n_meshes, int tile, int32_t* tile_mesh, hipStream_t s);
void launch_collect_deferred(const CollectArgs& a, int grid, hipStream_t s);
void launch_gather_exact(const GatherArgs& a, hipStream_t s);
void launch_scatter_exact(const ScatterArgs& a, hipStream_t s);
void launch_coefficients(const MeshDev& m, double* out, hipStream_t s);

}  // namespace hexval
