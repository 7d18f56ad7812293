// Device data structures shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hexval {

// Sentinel verdicts used while a call is in progress (never returned).
constexpr uint8_t kPending = 0xFE;   // sent to subdivision, folded later
constexpr uint8_t kExact = 0xFD;     // waiting for the exact tier
constexpr uint8_t kDeferred = 0xFF;  // queue full: handled in a later pass

// Flags of an element in subdivision (one word per subdivided element).
constexpr uint32_t kFlagInvalid = 1u;    // a sub-box corner certainly <= 0
constexpr uint32_t kFlagUndecided = 2u;  // a sub-box at the cap certainly ambiguous
constexpr uint32_t kFlagExact = 4u;      // a decision could not be certified
constexpr uint32_t kFlagOverflow = 8u;   // a child did not fit in the queue

// Largest depth cap accepted (levels 0..kMaxDepth).
constexpr int kMaxDepth = 20;

// One element of one mesh, as the kernels see it.
struct MeshDev {
    const double* points;       // [n,8,3] or vertices [n_points,3]
    const int32_t* conn;        // [n,8] or nullptr
    int64_t n;
    int64_t n_points;
    uint8_t* verdict;
    double* min_coeff;          // may be nullptr
    int64_t tile_begin;         // first global tile of this mesh (batched)
    int32_t validate;
    int32_t pad;
};

// A stored sub-box of the subdivision: 27 coefficients in tensor order,
// possibly mirrored (see `orient`), the element's bound scale, the index of
// the element in the subdivided list and the level.  256 bytes, so that eight
// lanes load one node as a single 256-byte span.
struct alignas(256) Node {
    double b[27];
    double scale;
    int64_t slot;      // index into the subdivided-element arrays
    int32_t level;
    int32_t orient;    // bit d set: axis d stored mirrored
    uint64_t pad[2];
};

// Counters of one pass.
struct alignas(256) Counters {
    // lvl[l]: sub-boxes of level l reserved (l = 0: the roots).  Stored
    // sub-boxes of level l occupy nodes[base_l, base_l + min(lvl[l], cap -
    // base_l)) with base_0 = 0 and base_{l+1} = base_l + that count.
    unsigned long long lvl[kMaxDepth + 4];
    unsigned long long n_sub;         // subdivided elements (slots used)
    unsigned long long n_exact;       // elements listed for the exact tier
    unsigned long long n_deferred;    // elements deferred to a later pass
    unsigned long long n_list;        // entries in the FP64 (re)check list
    unsigned long long walk_code;     // stack stride of a single mesh: limit - stride, 0 = none
    unsigned long long walk_break;    // 2^62 - first layer whose column 0 breaks the stack, 0 = none
    unsigned long long n_rechecked;   // FP32 filter: elements redone in FP64 inside the pass
    unsigned long long walk_tiles;    // tiles of a batched walking pass (set on the device)
    // first-pass tile counters, one per XCD chunk, each on a 256-byte line
    unsigned long long tile_next[8 * 32];
};

// Column walk of one mesh of a batch (set on the device before the walking
// pass): stride s (0: the mesh is checked in plain tiles), layers walked, and
// the mesh's first tile and tile count in the walking pass's numbering.
struct WalkMesh {
    int64_t s;
    int64_t nl;
    int64_t tile_begin;
    int64_t n_tiles;
};

struct QueueDev {
    Node* nodes;
    uint64_t node_cap;
    uint64_t root_cap;     // subdivided elements a round may list (<= node_cap)
    int64_t* sub_elem;     // [node_cap] element id of subdivided slot
    int32_t* sub_mesh;     // [node_cap] mesh index
    uint32_t* sub_flags;   // [node_cap]
    int64_t* exact_elem;   // [exact_cap]
    int32_t* exact_mesh;
    uint64_t exact_cap;
    int64_t* list_elem;    // FP64 (re)check list: recheck / deferred
    int32_t* list_mesh;
    uint64_t list_cap;
    Counters* cnt;
};

}  // namespace hexval
