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

// Error bits reported by kernels.
constexpr uint32_t kErrSpinTimeout = 1u;

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

// A sub-box waiting in the subdivision queue: 27 coefficients in tensor
// order, possibly mirrored (see `orient`), the element's bound scale, the
// index of the element in the subdivided list and the level.  256 bytes.
struct alignas(256) Node {
    double b[27];
    double scale;
    int64_t slot;      // index into the subdivided-element arrays
    int32_t level;
    int32_t orient;    // bit d set: axis d stored mirrored
    uint64_t pad;
    uint64_t ready;    // written last (release): the epoch of the pass that wrote the node
};

struct Counters {
    unsigned long long node_tail;     // node slots reserved
    unsigned long long node_head;     // node slots claimed by the drain
    unsigned long long outstanding;   // nodes queued or in process
    unsigned long long n_sub;         // subdivided elements (slots used)
    unsigned long long n_exact;       // elements listed for the exact tier
    unsigned long long n_deferred;    // elements deferred to a later pass
    unsigned long long n_nodes;       // sub-boxes evaluated
    unsigned long long n_recheck;     // FP32 filter: elements listed for FP64
    unsigned long long n_list;        // entries in the FP64 (re)check list
    unsigned int max_level;
    unsigned int error;
    unsigned long long pad[5];
};

struct QueueDev {
    Node* nodes;
    uint64_t node_cap;
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
    uint64_t epoch;        // pass number; a node is ready when node.ready == epoch
};

}  // namespace hexval
