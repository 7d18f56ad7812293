// Host runtime internals shared by the C ABI and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexval.h"
#include "hexval_internal.hpp"

namespace hexval {

int fail(int code, const char* fmt, ...);
const char* last_error();
int current_device(int* dev, int* cus);
const char* device_arch(int dev);
void default_opts(hexval_opts_t* o);
int check_opts(const hexval_opts_t* o);

// Device buffers of one in-flight call: subdivision queue, exact-tier
// staging, check lists, mesh table.  Pooled per device; a call owns one
// workspace from start to finish.
struct Workspace {
    int device = 0;
    bool borrowed = false;   // buffers owned elsewhere (never freed here)
    uint64_t node_cap = 0, exact_cap = 0, list_cap = 0, mesh_cap = 0, tile_cap = 0;
    Node* nodes = nullptr;
    int64_t* sub_elem = nullptr;
    int32_t* sub_mesh = nullptr;
    uint32_t* sub_flags = nullptr;
    int64_t* exact_elem = nullptr;
    int32_t* exact_mesh = nullptr;
    double* exact_pts = nullptr;
    uint8_t* exact_v = nullptr;
    double* h_exact_pts = nullptr;
    uint8_t* h_exact_v = nullptr;
    int64_t* list_elem = nullptr;
    int32_t* list_mesh = nullptr;
    Counters* cnt = nullptr;
    Counters* hcnt = nullptr;
    MeshDev* meshes = nullptr;
    MeshDev* h_meshes = nullptr;
    int32_t* tile_mesh = nullptr;
    WalkMesh* walk_meshes = nullptr;   // [mesh_cap] batched column walk: per-mesh strides and tiles
    int32_t* walk_tile_mesh = nullptr; // [tile_cap] its tile -> mesh table
    uint64_t* minj = nullptr;     // min-J arrays: 5 x minj_cap (u[0..2], ufinal, lb)
    uint64_t minj_cap = 0;
    int64_t* minj_defer = nullptr;   // min-J deferred-element lists: 2 x defer_cap
    uint64_t defer_cap = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

    ~Workspace();
    int init();
    int ensure(uint64_t nodes, uint64_t list, uint64_t meshes, uint64_t tiles);
    int ensure_minj(uint64_t slots, uint64_t elements);
    void release_queue();
    void release_list();
    QueueDev queue() const;
    // device bytes held by a workspace with these capacities
    static uint64_t footprint(uint64_t nodes, uint64_t list, uint64_t meshes, uint64_t tiles);
};

int acquire_workspace(int device, Workspace** out);
void release_workspace(Workspace* w);

// The whole check of n_meshes meshes on opts->stream; returns when final.
int run_check(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts,
              uint8_t* const* verdicts, double* const* mins);

// Same, on a caller-owned workspace (nullptr: one from the pool).  tune:
// whether a launch shape not in the tuning cache may be timed on this call
// (else the default shape is used).
int run_check_ws(const hexval_mesh_t* meshes, int n_meshes, bool batched, const hexval_opts_t* opts,
                 uint8_t* const* verdicts, double* const* mins, Workspace* ws, bool tune = true);

// Corner-only test and corner quality (hexval_corner_test).
int run_corner_test(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* test1, double* quality);

// Linear quadrangles (hexval_quad_check).
int run_quad_check(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts, double* min_j);

// Certified bounds of min J (hexval_min_jacobian).
int run_min_jacobian(const hexval_mesh_t* mesh, const hexval_opts_t* opts, double rtol, double* lo, double* hi,
                     uint8_t* status);

}  // namespace hexval
