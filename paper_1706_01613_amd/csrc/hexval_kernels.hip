// HIP kernels of the validity test for linear hexahedra (gfx950).
//
//   k_top_f64      first pass, one element per lane: gather the 8 corners,
//                  20 triple products (Section 5), Table 3, certified
//                  decisions of Section 6 steps 2 and 4; ambiguous elements
//                  go to the subdivision list through a per-wave LDS buffer,
//                  uncertain ones to the exact list (ballot + one atomic per
//                  wave).  k_filter_f32: the same in FP32 with a forward
//                  bound, the rest to the FP64 recheck list.
//   k_minj_*       certified bounds of min J: first pass, levels, fold.
//   k_corner_*     Test 1 (corner values only) and corner quality.
//   k_quad_*       linear quadrangles (Section 2.1).
//   k_exact_device the exact tier in 256-bit integers.
//   k_roots        root sub-boxes (level 0) of the subdivided elements.
//   k_level        one level of the subdivision: eight lanes per stored
//                  sub-box, one lane per child (de Casteljau at 1/2);
//                  children that stay ambiguous are appended as the next
//                  level until the depth cap.
//   k_fold         folds the per-element flags of subdivided elements into
//                  verdicts (INVALID > exact > overflow > UNDECIDED > VALID).
//   small kernels  counter reset, batched tile table, deferred-element
//                  collection, exact-tier gather/scatter, coefficients.
#include <hip/hip_runtime.h>

#include "hexval_exact_dev.hpp"
#include "hexval_internal.hpp"
#include "hexval_kernels.hpp"
#include "hexval_math.hpp"

namespace hexval {

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// The same address as a global-memory pointer.  Mesh records read from the
// batch table reach the kernels as plain pointers; without the address space
// their loads and stores compile to flat instructions, which also count
// against the LDS and scalar-load counter and so stall every LDS wait behind
// them.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* global(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// A 64-bit value that every lane of the wave holds, as a scalar.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Mesh record mi of a batch table (written before the launch, read only),
// with scalar loads: mi is the same in every lane of the wave.
__device__ __forceinline__ MeshDev uniform_mesh_record(const MeshDev* meshes, int mi)
{
    typedef __attribute__((address_space(4))) const uint64_t* const_u64;
    static_assert(sizeof(MeshDev) == 64, "mesh record of 8 words");
    const const_u64 w = (const_u64)(meshes + mi);
    uint64_t words[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) words[i] = w[i];
    MeshDev r;
    __builtin_memcpy(&r, words, sizeof r);
    return r;
}

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ unsigned long long wave_bcast(unsigned long long v, int src)
{
    return __shfl(v, src, 64);
}

// Reserves `count` consecutive slots of counter `c` for the lanes of `mask`;
// returns this lane's slot (valid only for lanes in mask).
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long* c, uint64_t mask)
{
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(c, (unsigned long long)__popcll(mask));
    base = wave_bcast(base, leader);
    return base + (unsigned long long)lane_rank(mask);
}

// Adds the number of lanes with `pred` to *c with one atomic per wave (every
// lane of the wave must call this).
__device__ __forceinline__ void wave_count(unsigned long long* c, bool pred)
{
    const uint64_t mask = ballot(pred);
    if (mask && (threadIdx.x & 63) == __ffsll((unsigned long long)mask) - 1)
        atomicAdd(c, (unsigned long long)__popcll(mask));
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_relaxed(unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- gather

// Gather modes: which layouts a kernel instantiation handles.
enum Gather : int {
    kGatherAny = 0,       // decided per mesh at run time
    kGatherPoints = 1,    // [n,8,3] points
    kGatherConn = 2,      // connectivity, trusted indices
    kGatherChecked = 3    // connectivity, indices validated
};

template <int G>
__device__ __forceinline__ void load_points_t(const MeshDev& m, int64_t e, V3 p[8], bool& bad_index)
{
    const bool conn = G == kGatherAny ? m.conn != nullptr : G != kGatherPoints;
    const bool validate = G == kGatherAny ? m.validate != 0 : G == kGatherChecked;
    if (conn) {
        const auto* row = global(m.conn) + 8 * e;
        int idx[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) idx[k] = row[k];
        if (validate) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                bad_index |= (idx[k] < 0) || ((int64_t)idx[k] >= m.n_points);
            if (bad_index) return;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const auto* v = global(m.points) + 3 * (int64_t)idx[k];
            p[k] = {v[0], v[1], v[2]};
        }
    } else {
        const auto* v = global(m.points) + 24 * e;
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = {v[3 * k], v[3 * k + 1], v[3 * k + 2]};
    }
}

__device__ __forceinline__ void load_points(const MeshDev& m, int64_t e, V3 p[8], bool& bad_index)
{
    load_points_t<kGatherAny>(m, e, p, bad_index);
}

// Writes a top-level node for a subdivided element.
__device__ void write_root(Node* nd, const ElementValues& r, int64_t slot)
{
    // the node's first 240 bytes as 15 aligned 16-byte stores
    double w[30];
#pragma unroll
    for (int a = 0; a < 27; ++a) w[fig3_to_tensor(a)] = coefficient(r, a);
    w[27] = r.scale;
    w[28] = __longlong_as_double(slot);
    w[29] = __longlong_as_double(0);   // level 0, orientation 0
    double2* out = reinterpret_cast<double2*>(nd);
#pragma unroll
    for (int k = 0; k < 15; ++k) out[k] = make_double2(w[2 * k], w[2 * k + 1]);
}

// Orders this wave's LDS writes before its later LDS reads by other lanes
// (a compiler barrier: one wave's LDS accesses complete in issue order).
__device__ __forceinline__ void lds_order() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// Elements a first pass sends on (to subdivision, or from the FP32 filter to
// the FP64 recheck) are held per wave in LDS and appended to their list up to
// kPushBuf at a time, with one atomic: on invalid-heavy meshes most waves send
// some element, and one atomic per wave and tile on the single list counter
// serialises the pass.  Their verdict (pending, or deferred when the list is
// full) is written when they are appended.  Every lane of the wave calls
// push_flush; each kernel that fills a buffer flushes it after its last tile.
constexpr int kPushBuf = 256;

struct PushBuf {
    __attribute__((address_space(3))) int64_t* elem;   // this wave's kPushBuf entries
    __attribute__((address_space(3))) int32_t* mesh;
    int n;                                              // entries held (wave-uniform)
};

// The buffers of the (at most 4) waves of a block, and this wave's.
#define HX_PUSH_STORAGE                                              \
    __shared__ int64_t push_elem_[4 * kPushBuf];                     \
    __shared__ int32_t push_mesh_[4 * kPushBuf];                     \
    PushBuf pb{(__attribute__((address_space(3))) int64_t*)(push_elem_ + (threadIdx.x >> 6) * kPushBuf), \
               (__attribute__((address_space(3))) int32_t*)(push_mesh_ + (threadIdx.x >> 6) * kPushBuf), 0}

// A second set for kernels that append to two lists (the FP32 filter: its
// recheck list, and the subdivision list for what filter_subdivides sends).
#define HX_SUB_PUSH_STORAGE                                          \
    __shared__ int64_t sub_elem_[4 * kPushBuf];                      \
    __shared__ int32_t sub_mesh_[4 * kPushBuf];                      \
    PushBuf sb{(__attribute__((address_space(3))) int64_t*)(sub_elem_ + (threadIdx.x >> 6) * kPushBuf), \
               (__attribute__((address_space(3))) int32_t*)(sub_mesh_ + (threadIdx.x >> 6) * kPushBuf), 0}

// A list that buffered entries are appended to: the subdivision list, or
// the FP32 filter's FP64 recheck list.
struct ListRef {
    unsigned long long* count;
    int64_t* elem;
    int32_t* mesh;
    uint64_t cap;
};

__device__ __forceinline__ ListRef sub_list(const QueueDev& q)
{
    return {&q.cnt->n_sub, q.sub_elem, q.sub_mesh, q.root_cap};
}
__device__ __forceinline__ ListRef recheck_list(const QueueDev& q)
{
    return {&q.cnt->n_list, q.list_elem, q.list_mesh, q.list_cap};
}

// meshes: the batch table, or nullptr when every entry belongs to `single`.
__device__ void push_flush(PushBuf& pb, const ListRef& l, const QueueDev& q, const MeshDev& single,
                           const MeshDev* meshes)
{
    if (pb.n == 0) return;
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(l.count, (unsigned long long)pb.n);
    base = wave_bcast(base, 0);
    lds_order();                       // the entries other lanes wrote are visible
    unsigned long long deferred = 0;
    for (int i = lane; i < pb.n; i += 64) {
        const int64_t e = pb.elem[i];
        const int mi = pb.mesh[i];
        uint8_t* verdict = meshes ? meshes[mi].verdict : single.verdict;
        const unsigned long long slot = base + (unsigned long long)i;
        if (slot < l.cap) {
            l.elem[slot] = e;
            l.mesh[slot] = mi;
            *global(verdict + e) = kPending;
        } else {
            *global(verdict + e) = kDeferred;
            ++deferred;
        }
    }
    if (deferred) atomicAdd(&q.cnt->n_deferred, deferred);
    lds_order();                       // reads done before the buffer is refilled
    pb.n = 0;
}

// Adds this wave's lanes with `want` to the buffer, flushing it to list l
// first when it could overflow.  Every lane of the wave calls this.
__device__ __forceinline__ void push_entry(PushBuf& pb, const ListRef& l, const QueueDev& q, const MeshDev& single,
                                           const MeshDev* meshes, bool want, int64_t e, int mesh_idx)
{
    const uint64_t mask = ballot(want);
    if (!mask) return;
    if (want) {
        const int k = pb.n + lane_rank(mask);
        pb.elem[k] = e;
        pb.mesh[k] = mesh_idx;
    }
    pb.n += __popcll(mask);
}

// One element: decides, writes outputs, takes part in the compaction of
// subdivided and exact-tier elements into their lists (every thread of the
// block must call this: the subdivision list is reserved per block).  Subdivided elements only get their id listed here;
// k_roots recomputes their 27 coefficients, which keeps this kernel's
// register footprint small.
template <bool EDGES>
__device__ void finish_element(const MeshDev& m, int mesh_idx, int64_t e, bool active, const V3 p[8],
                               bool bad, const QueueDev& q, int max_depth, PushBuf& pb, const MeshDev* meshes)
{
    int st = -1;
    double mn = 0.0;
    if (active) {
        if (!bad) {
            const LeanResult r = element_lean(p, EDGES);
            st = lean_state(r, max_depth);
            mn = r.min27;
        }
    }
    uint8_t v = 0;
    if (active) {
        if (bad) v = 3;
        else if (st <= kTopUndecided) v = (uint8_t)st;
    }
    bool deferred = false;
    const bool push = active && st == kTopSubdivide;
    push_entry(pb, sub_list(q), q, m, meshes, push, e, mesh_idx);   // room for 64: flushed below once fuller
    const bool exact = active && st == kTopExact;
    const uint64_t xmask = ballot(exact);
    if (xmask) {
        const unsigned long long slot = wave_reserve(&q.cnt->n_exact, xmask);
        if (exact) {
            if (slot < q.exact_cap) {
                q.exact_elem[slot] = e;
                q.exact_mesh[slot] = mesh_idx;
                v = kExact;
            } else {
                v = kDeferred;
                deferred = true;
            }
        }
    }
    if (xmask) wave_count(&q.cnt->n_deferred, deferred);
    if (active) {
        if (!push) *global(m.verdict + e) = v;   // listed elements: at push_flush
        if (m.min_coeff) *global(m.min_coeff + e) = bad ? __builtin_nan("") : mn;
    }
    if (pb.n > kPushBuf - 64) push_flush(pb, sub_list(q), q, m, meshes);
}

template <bool EDGES, int G>
__device__ void process_element(const MeshDev& m, int mesh_idx, int64_t e, bool active,
                                const QueueDev& q, int max_depth, PushBuf& pb, const MeshDev* meshes)
{
    V3 p[8];
    bool bad = false;
    if (active) load_points_t<G>(m, e, p, bad);
    finish_element<EDGES>(m, mesh_idx, e, active, p, bad, q, max_depth, pb, meshes);
}

// Root nodes of the subdivided elements listed by the first pass: the full
// set of 27 coefficients is recomputed (same arithmetic as the first pass)
// and written to queue slot s = list index.
__global__ __launch_bounds__(256) void k_roots(RootArgs a)
{
    const QueueDev& q = a.q;
    const unsigned long long ns = q.cnt->n_sub;
    const int64_t n = (int64_t)(ns < q.root_cap ? ns : q.root_cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) q.cnt->lvl[0] = (unsigned long long)n;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int mi = q.sub_mesh[s];
        const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
        V3 p[8];
        bool bad = false;
        load_points(m, q.sub_elem[s], p, bad);
        ElementValues r;
        element_values(p, r);
        Node* nd = q.nodes + s;
        write_root(nd, r, s);
        q.sub_flags[s] = 0u;
    }
}

// XCD (accelerator complex die) the calling wave runs on: bits 3:0 of the
// XCC_ID hardware register (0..7 on MI355X).
__device__ __forceinline__ int xcd_id() { return (int)(__builtin_amdgcn_s_getreg(20 | (3 << 11)) & 15); }

// Tile scheduler of the first passes.  The tiles are cut into `xcds`
// contiguous chunks; chunk x is served first to the blocks that run on XCD x
// (read from the hardware, which also holds when other kernels share the
// device and the dispatcher's placement no longer follows the block index),
// so neighbouring tiles, which share vertices, meet in the same L2.  Work is
// handed out in runs: with w blocks per chunk, run r of a chunk is the tiles
// g*R*w + o + j*w (j < R, g = r / w, o = r % w, R up to 16), so the w blocks
// working on a chunk sweep a window of about w consecutive tiles together
// while one atomic serves R tiles.  A block whose chunk is used up takes
// runs from the other chunks, so a chunk that costs more (private vertices,
// say) does not hold up the launch.
struct TileSched {
    int64_t n_tiles;
    int xcds, home;
    int64_t run;                // tiles per run (R)
    int64_t width;              // blocks per chunk (w): stride of a run's tiles
    unsigned long long* next;   // Counters::tile_next: runs taken per chunk
    int64_t base = 0, j = 0, jend = 0;   // the block's current run (block-uniform)
    __device__ TileSched(int64_t n, int x, Counters* c)
        : n_tiles(n), xcds(x), home(xcd_id() % x), next(c->tile_next)
    {
        const int64_t per_block = n / ((int64_t)gridDim.x * 4);
        run = per_block < 1 ? 1 : per_block > 16 ? 16 : per_block;
        width = ((int64_t)gridDim.x + x - 1) / x;
    }
    // First tile of run r of a chunk of `size` tiles (>= size: no such run).
    __device__ int64_t first_of(int64_t r) const { return (r / width) * run * width + r % width; }
    __device__ void grab(int64_t& first, int64_t& count)   // one thread of the block
    {
        for (int k = 0; k < xcds; ++k) {
            const int c = (home + k) % xcds;
            const int64_t cs = n_tiles * c / xcds, size = n_tiles * (c + 1) / xcds - cs;
            unsigned long long* ctr = next + 32 * c;
            if (first_of((int64_t)load_relaxed(ctr)) >= size) continue;   // used up: skip the atomic
            const int64_t f = first_of((int64_t)atomicAdd(ctr, 1ull));
            if (f < size) {
                const int64_t m = (size - f + width - 1) / width;
                first = cs + f;
                count = m < run ? m : run;
                return;
            }
        }
        first = count = 0;
    }
    // The block's next tile, or -1 when none is left (every thread calls it).
    __device__ int64_t next_tile()
    {
        if (j < jend) return base + (j++) * width;
        __shared__ int64_t range[2];
        __syncthreads();                 // everyone has read the previous run
        if (threadIdx.x == 0) grab(range[0], range[1]);
        __syncthreads();
        base = range[0];
        jend = range[1];
        j = 0;
        return j < jend ? base + (j++) * width : -1;
    }
};

// EDGES: include the edge-midpoint values in the step-2 test (needed only
// when the depth cap is 0, see element_lean).
template <bool BATCHED, bool EDGES, int G>
__global__ __launch_bounds__(256) void k_top_f64_range(TopArgs a)
{
    HX_PUSH_STORAGE;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        MeshDev m;
        int mi;
        int64_t e;
        if (BATCHED) {
            mi = a.tile_mesh[t];
            m = a.meshes[mi];
            e = (t - m.tile_begin) * (int64_t)blockDim.x + threadIdx.x;
        } else {
            mi = 0;
            m = a.mesh;
            e = t * (int64_t)blockDim.x + threadIdx.x;
        }
        process_element<EDGES, G>(m, mi, e, e < m.n, a.q, a.max_depth, pb, BATCHED ? a.meshes : nullptr);
    }
    push_flush(pb, sub_list(a.q), a.q, a.mesh, BATCHED ? a.meshes : nullptr);
}

// LDS address space pointer, as the direct global-to-LDS loads take it.
typedef __attribute__((address_space(3))) void* lds_ptr;

// Waits until this wave's LDS reads have returned (s_waitcnt lgkmcnt(0)).
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Waits until every earlier vector memory operation of the wave has completed
// (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Wave priority in the prefetching loops and the corner test: a wave raises
// its priority while it issues an iteration's loads, so that they go out
// before the other waves' arithmetic resumes, and drops back to the default
// before it waits for them (A/B on the 400^3 lattice: first pass 2-3% faster,
// identical outputs).  The quadrangle kernel, at 50 registers and high
// occupancy, measured no change and keeps its plain loop.
__device__ __forceinline__ void issue_priority() { __builtin_amdgcn_s_setprio(2); }

// Back to the default priority, then wait_vmem().
__device__ __forceinline__ void wait_loads()
{
    __builtin_amdgcn_s_setprio(0);
    wait_vmem();
}

// First-pass loop over a single mesh with trusted connectivity (K corners per
// element, 4 or 8): the connectivity row of a lane's next element is loaded
// straight into LDS (global_load_lds_dwordx4: lane i of a wave lands at the
// wave's base + 16 i, no registers) before the current element's vertex
// loads, so both are in flight together and an iteration waits for one
// round of memory latency instead of two dependent ones.  body(e, active,
// idx) issues the vertex loads of idx (every lane holds a valid row: lanes
// past the end hold row n-1), calls wait_loads(), which also covers the
// prefetch and ends the raised priority the loop set before it, and
// computes.  stage: [K/4][256] int4 in LDS.
template <int K, typename Body>
__device__ __forceinline__ void conn_prefetch_loop(const int32_t* conn, int64_t n, TileSched& ts, int4* stage,
                                                   Body body)
{
    const int wave_base = threadIdx.x & ~63;
    auto prefetch = [&](int64_t t) {
        int64_t e = t * (int64_t)blockDim.x + threadIdx.x;
        e = e < n ? e : n - 1;        // past the end: a valid row, ignored
        const int* src = conn + (int64_t)K * e;
#pragma unroll
        for (int h = 0; h < K / 4; ++h)
            __builtin_amdgcn_global_load_lds(src + 4 * h, (lds_ptr)&stage[h * 256 + wave_base], 16, 0, 0);
    };
    int64_t t = ts.next_tile();
    if (t >= 0) prefetch(t);
    wait_vmem();
    while (t >= 0) {
        const int64_t e = t * (int64_t)blockDim.x + threadIdx.x;
        // this iteration's rows are in LDS: the wait after the previous
        // iteration's loads covered the prefetch issued before them
        int idx[K];
#pragma unroll
        for (int h = 0; h < K / 4; ++h) {
            const int4 c = stage[h * 256 + threadIdx.x];
            idx[4 * h] = c.x;
            idx[4 * h + 1] = c.y;
            idx[4 * h + 2] = c.z;
            idx[4 * h + 3] = c.w;
        }
        // the next rows go out before this element's vertex loads (the last
        // iteration reloads its own rows)
        const int64_t tn = ts.next_tile();
        wait_lds();                    // the slots are free: every lane has read its row
        issue_priority();
        prefetch(tn >= 0 ? tn : t);
        body(e, e < n, idx);
        t = tn;
    }
}


__device__ __forceinline__ void gather8(const double* points, const int idx[8], V3 p[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const auto* v = global(points) + 3 * (int64_t)idx[k];
        p[k] = {v[0], v[1], v[2]};
    }
}

// conn_prefetch_loop for a batch whose meshes all have trusted connectivity.
// The mesh of a tile comes from the tile -> mesh table; the next tile's mesh
// is looked up (scalar loads, which often miss) while the current tile's
// vertex loads are in flight, and its rows are prefetched right after.
// finish(m, mi, e, active, p) runs once the vertices p of element e of mesh
// m (index mi) have landed.
template <typename Finish>
__device__ __forceinline__ void batch_prefetch_loop(const MeshDev* meshes, const int32_t* tile_mesh, TileSched& ts,
                                                    int4* stage, Finish finish)
{
    const int wave_base = threadIdx.x & ~63;
    // scalar loads: both tables are written before the launch and only read here
    typedef __attribute__((address_space(4))) const int32_t* const_i32;
    auto mesh_of = [&](int64_t t, int& mi) {
        mi = ((const_i32)tile_mesh)[(int64_t)uniform_u64((uint64_t)t)];
        return uniform_mesh_record(meshes, mi);
    };
    auto prefetch = [&](int64_t t, const MeshDev& m) {
        int64_t e = (t - m.tile_begin) * (int64_t)blockDim.x + threadIdx.x;
        e = e < m.n ? e : m.n - 1;    // past the end: a valid row of the same mesh, ignored
        const int* src = m.conn + 8 * e;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            __builtin_amdgcn_global_load_lds(src + 4 * h, (lds_ptr)&stage[h * 256 + wave_base], 16, 0, 0);
    };
    int mi = 0;
    MeshDev m{};
    int64_t t = ts.next_tile();
    if (t >= 0) {
        m = mesh_of(t, mi);
        prefetch(t, m);
    }
    wait_vmem();
    while (t >= 0) {
        const int64_t e = (t - m.tile_begin) * (int64_t)blockDim.x + threadIdx.x;
        int idx[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int4 c = stage[h * 256 + threadIdx.x];
            idx[4 * h] = c.x;
            idx[4 * h + 1] = c.y;
            idx[4 * h + 2] = c.z;
            idx[4 * h + 3] = c.w;
        }
        const int64_t tn = ts.next_tile();
        V3 p[8];
        issue_priority();
        gather8(m.points, idx, p);     // every lane holds a valid row
        int mi_n = mi;
        MeshDev mn = m;
        // the tables only when the next tile leaves this mesh (a tile's
        // successor is usually a later tile of the same mesh): the next rows
        // then go out without waiting for scalar loads
        const int64_t rel = tn - m.tile_begin;
        if (tn >= 0 && !(rel >= 0 && rel * (int64_t)blockDim.x < m.n)) mn = mesh_of(tn, mi_n);
        wait_lds();                    // the slots are free: every lane has read its row
        prefetch(tn >= 0 ? tn : t, mn);
        wait_loads();                  // vertices and the next rows have landed
        finish(m, mi, e, e < m.n, p);
        t = tn;
        m = mn;
        mi = mi_n;
    }
}

// k_top_f64_range for a single mesh with trusted connectivity, through
// conn_prefetch_loop.
template <bool EDGES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_top_f64_conn(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    HX_PUSH_STORAGE;
    const MeshDev& m = a.mesh;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    conn_prefetch_loop<8>(m.conn, m.n, ts, stage, [&](int64_t e, bool active, const int* idx) {
        V3 p[8];
        gather8(m.points, idx, p);
        wait_loads();                  // vertices and the next rows have landed
        finish_element<EDGES>(m, 0, e, active, p, false, a.q, a.max_depth, pb, nullptr);
    });
    push_flush(pb, sub_list(a.q), a.q, m, nullptr);
}

// ------------------------------------------------------------ column walk
//
// In a structured mesh stacked layer by layer, element e + s (s elements per
// layer) has as its bottom face (corners 0..3) the top face (corners 4..7) of
// element e.  The walking first passes give each lane a column of elements
// e, e + s, e + 2s, ...: a lane loads the 4 new corners of each element and
// takes the other 4 from LDS, where it left the previous element's top face,
// which halves the vertex loads and the distinct cache lines per element and
// keeps a vertex plane on chip between the two layers that share it.  The
// carried face is a cache keyed by vertex index: a lane compares the
// element's bottom corner ids with the ids it holds and loads all 8 corners
// when they differ, so any connectivity gives the same result, and only the
// speed depends on the stride found.


// Finds the smallest e in [1, limit) whose corners 0..3 are corners 4..7 of
// element 0, and records it as limit - e in c->walk_code (atomicMax, so the
// smallest e wins; 0 = none).  Threads stop once a smaller e is recorded.
__global__ __launch_bounds__(256) void k_walk_detect(const int32_t* conn, int64_t limit, Counters* c)
{
    const int t0 = conn[4], t1 = conn[5], t2 = conn[6], t3 = conn[7];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < limit; e += stride) {
        if ((int64_t)load_relaxed(&c->walk_code) > limit - e) return;
        const int32_t* b = conn + 8 * e;
        if (b[0] == t0 && b[1] == t1 && b[2] == t2 && b[3] == t3)
            atomicMax(&c->walk_code, (unsigned long long)(limit - e));
    }
}

constexpr unsigned long long kWalkBreakBase = 1ull << 62;

// With the stride s found, the first layer l >= 1 whose element l s does not
// sit on element (l - 1) s (its corners 0..3 are not the other's 4..7), as
// 2^62 - l in c->walk_break (atomicMax: the first such layer wins; 0 =
// none).  The walk covers the layers before it; a mesh whose stacked part is
// followed by unrelated elements checks those with plain tiles.
__global__ __launch_bounds__(256) void k_walk_extent(const int32_t* conn, int64_t n, int64_t limit, Counters* c)
{
    const unsigned long long code = c->walk_code;
    const int64_t s = code ? limit - (int64_t)code : 0;
    if (s < kWalkMinStride || s >= n) return;
    const int64_t nl = (n + s - 1) / s;
    for (int64_t l = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < nl; l += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* lo = conn + 8 * ((l - 1) * s);
        const int32_t* up = conn + 8 * (l * s);
        if (up[0] != lo[4] || up[1] != lo[5] || up[2] != lo[6] || up[3] != lo[7])
            atomicMax(&c->walk_break, kWalkBreakBase - (unsigned long long)l);
    }
}

// Tiles of a walking pass: blockDim.x consecutive columns of a layer times
// `layers` consecutive layers; walk tile t covers column block t % ncb of
// the layer block t / ncb, over the layers before the first break.  The
// elements after them are the tail, in plain tiles of blockDim.x elements
// numbered after the walk tiles.  Without a usable stride the whole mesh is
// the tail.
struct WalkShape {
    int64_t s;        // elements per layer
    int32_t ncb;      // column blocks per layer
    int32_t nl;       // layers walked
    int32_t layers;   // layers per tile
    int64_t n_walk;   // walk tiles
    int64_t tail;     // first element of the tail
    int64_t n_tiles;
    WalkShape() = default;
    // A single mesh: the stride and break found by k_walk_detect / k_walk_extent.
    __device__ WalkShape(int64_t n, const Counters* c, int64_t limit, int walk_layers)
    {
        const unsigned long long code = c->walk_code, brk = c->walk_break;
        const int64_t st = code ? limit - (int64_t)code : 0;
        int64_t l = 0;
        if (st >= kWalkMinStride && st < n) l = brk ? (int64_t)(kWalkBreakBase - brk) : (n + st - 1) / st;
        init(n, st, l, walk_layers, blockDim.x);
    }
    // Stride st with walked layers l (st = 0 or l = 0: plain tiles only), in
    // tiles of `block` columns.
    __host__ __device__ void init(int64_t n, int64_t st, int64_t l, int walk_layers, int64_t block)
    {
        s = st;
        layers = walk_layers;
        if (s < kWalkMinStride || s >= n || layers < 1 || l < 1) {
            s = n;
            nl = 0;
            layers = 1;
        } else {
            nl = (int32_t)l;
        }
        ncb = (int32_t)((s + block - 1) / block);
        n_walk = (int64_t)ncb * ((nl + layers - 1) / layers);
        tail = (int64_t)nl * s < n ? (int64_t)nl * s : n;
        n_tiles = n_walk + (n - tail + block - 1) / block;
    }
};

// The block's position in a walking pass (block-uniform): the element of
// its column 0 in the current layer, the columns of its block that exist,
// and the layers left in the current tile.  Lane l checks element base + l.
struct WalkPos {
    int64_t base;
    int64_t cols;
    int32_t left;
    // First layer of tile t.
    __device__ void start(const WalkShape& ws, int64_t t)
    {
        if (t >= ws.n_walk) {         // a plain tile of the tail
            base = ws.tail + (t - ws.n_walk) * blockDim.x;
            cols = blockDim.x;
            left = 1;
            return;
        }
        const int32_t lb = (int32_t)(t / ws.ncb);
        const int64_t c0 = (t - (int64_t)lb * ws.ncb) * blockDim.x;
        const int32_t l0 = lb * ws.layers;
        cols = ws.s - c0;
        base = (int64_t)l0 * ws.s + c0;
        left = ws.nl - l0 < ws.layers ? ws.nl - l0 : ws.layers;
    }
};

// conn_prefetch_loop over the steps (tile, layer) of a walking pass: the
// connectivity rows of a lane's next element go to LDS before the current
// element's vertex loads.  body(e, active, idx) as in conn_prefetch_loop.
template <typename Body>
__device__ __forceinline__ void walk_prefetch_loop(const int32_t* conn, int64_t n, const WalkShape& ws,
                                                   TileSched& ts, int4* stage, Body body)
{
    const int wave_base = threadIdx.x & ~63;
    auto prefetch = [&](int64_t e) {
        e = e < n ? e : n - 1;        // past the end: a valid row, ignored
        const int* src = conn + 8 * e;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            __builtin_amdgcn_global_load_lds(src + 4 * h, (lds_ptr)&stage[h * 256 + wave_base], 16, 0, 0);
    };
    WalkPos pos;
    int64_t t = ts.next_tile();
    if (t >= 0) {
        pos.start(ws, t);
        prefetch(pos.base + threadIdx.x);
    }
    wait_vmem();
    while (t >= 0) {
        int idx[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int4 c = stage[h * 256 + threadIdx.x];
            idx[4 * h] = c.x;
            idx[4 * h + 1] = c.y;
            idx[4 * h + 2] = c.z;
            idx[4 * h + 3] = c.w;
        }
        const int64_t e = pos.base + threadIdx.x;
        const bool active = (int64_t)threadIdx.x < pos.cols && e < n;
        // the next step: the layer above in the same tile, else the next tile
        if (pos.left > 1) {
            pos.base += ws.s;
            --pos.left;
        } else {
            t = ts.next_tile();
            if (t >= 0) pos.start(ws, t);
        }
        wait_lds();                    // the slots are free: every lane has read its row
        issue_priority();
        prefetch(t >= 0 ? pos.base + threadIdx.x : e);
        body(e, active, idx);
    }
}

// This lane's carried face in LDS: the ids of the 4 vertices it holds and
// their coordinates, coordinate-major per lane so that a wave's accesses are
// conflict-free.
struct CarrySlots {
    int id[4 * 256];
    double xyz[12 * 256];
};

// Vertex loads of one element with the carried face: corners 4..7 always,
// corners 0..3 only when this lane's slots do not hold them.  Returns
// whether they do.  The 4 ids are compared as two 64-bit pairs, after the
// loads have gone out: as a chain of short-circuit branches each slot read
// waited for the one before, and the vertex loads went out only after the
// last.
__device__ __forceinline__ bool carry_issue(const double* points, const int idx[8], const CarrySlots& cs, V3 p[8])
{
    const int l = threadIdx.x;
#pragma unroll
    for (int k = 4; k < 8; ++k) {
        const auto* v = global(points) + 3 * (int64_t)idx[k];
        p[k] = {v[0], v[1], v[2]};
    }
    auto pair = [](int lo, int hi) { return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32); };
    const bool hit = (pair(idx[0], idx[1]) == pair(cs.id[l], cs.id[256 + l])) &
                     (pair(idx[2], idx[3]) == pair(cs.id[512 + l], cs.id[768 + l]));
    if (!hit) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const auto* v = global(points) + 3 * (int64_t)idx[k];
            p[k] = {v[0], v[1], v[2]};
        }
    }
    return hit;
}

// After the loads have landed: corners 0..3 from the slots on a hit, and
// corners 4..7 left there for the element above.
__device__ __forceinline__ void carry_finish(const int idx[8], bool hit, CarrySlots& cs, V3 p[8])
{
    const int l = threadIdx.x;
    if (hit) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            p[k] = {cs.xyz[(3 * k) * 256 + l], cs.xyz[(3 * k + 1) * 256 + l], cs.xyz[(3 * k + 2) * 256 + l]};
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cs.xyz[(3 * k) * 256 + l] = p[k + 4].x;
        cs.xyz[(3 * k + 1) * 256 + l] = p[k + 4].y;
        cs.xyz[(3 * k + 2) * 256 + l] = p[k + 4].z;
        cs.id[k * 256 + l] = idx[k + 4];
    }
}

// No vertex held yet (before the first element; indices are >= 0).
__device__ __forceinline__ void carry_clear(CarrySlots& cs)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) cs.id[k * 256 + threadIdx.x] = -1;
}

// k_top_f64_conn with the column walk.
template <bool EDGES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_top_f64_walk(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    __shared__ CarrySlots cs;
    HX_PUSH_STORAGE;
    const MeshDev& m = a.mesh;
    const WalkShape ws(m.n, a.q.cnt, a.walk_limit, a.walk_layers);
    TileSched ts(ws.n_tiles, a.xcds, a.q.cnt);
    carry_clear(cs);
    walk_prefetch_loop(m.conn, m.n, ws, ts, stage, [&](int64_t e, bool active, const int* idx) {
        V3 p[8];
        const bool hit = carry_issue(m.points, idx, cs, p);
        wait_loads();                  // vertices and the next rows have landed
        carry_finish(idx, hit, cs, p);
        finish_element<EDGES>(m, 0, e, active, p, false, a.q, a.max_depth, pb, nullptr);
    });
    push_flush(pb, sub_list(a.q), a.q, m, nullptr);
}

// Walk record mi of the batch (set on the device by an earlier launch, read
// only here), with scalar loads.
__device__ __forceinline__ WalkMesh uniform_walk_record(const WalkMesh* wm, int mi)
{
    typedef __attribute__((address_space(4))) const int64_t* const_i64;
    const const_i64 w = (const_i64)(wm + mi);
    return {w[0], w[1], w[2], w[3]};
}

// Forgets this lane's carried face (the next element loads all 8 corners).
__device__ __forceinline__ void carry_forget(CarrySlots& cs)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) cs.id[k * 256 + threadIdx.x] = -1;
}

// walk_prefetch_loop over a batch: tile t of the walking numbering belongs to
// mesh tile_mesh[t] and is tile t - tile_begin of that mesh's WalkShape.
// Vertex ids only mean something within one mesh, so each lane forgets its
// carried face when a new tile starts.  body(m, mi, e, active, idx).
template <typename Body>
__device__ __forceinline__ void batch_walk_loop(const TopArgs& a, TileSched& ts, int4* stage, CarrySlots& cs,
                                                Body body)
{
    const int wave_base = threadIdx.x & ~63;
    typedef __attribute__((address_space(4))) const int32_t* const_i32;
    auto prefetch = [&](const MeshDev& m, int64_t e) {
        e = e < m.n ? e : m.n - 1;    // past the end: a valid row of the same mesh, ignored
        const int* src = m.conn + 8 * e;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            __builtin_amdgcn_global_load_lds(src + 4 * h, (lds_ptr)&stage[h * 256 + wave_base], 16, 0, 0);
    };
    WalkShape ws;
    WalkPos pos;
    auto enter = [&](int64_t t, MeshDev& m, int& mi) {
        mi = ((const_i32)a.tile_mesh)[(int64_t)uniform_u64((uint64_t)t)];
        m = uniform_mesh_record(a.meshes, mi);
        const WalkMesh w = uniform_walk_record(a.walk_meshes, mi);
        ws.init(m.n, w.s, w.nl, a.walk_layers, blockDim.x);
        pos.start(ws, t - w.tile_begin);
    };
    int mi = 0;
    MeshDev m{};
    int64_t t = ts.next_tile();
    if (t >= 0) {
        enter(t, m, mi);
        prefetch(m, pos.base + threadIdx.x);
    }
    carry_forget(cs);
    wait_vmem();
    while (t >= 0) {
        int idx[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int4 c = stage[h * 256 + threadIdx.x];
            idx[4 * h] = c.x;
            idx[4 * h + 1] = c.y;
            idx[4 * h + 2] = c.z;
            idx[4 * h + 3] = c.w;
        }
        const int64_t e = pos.base + threadIdx.x;
        const bool active = (int64_t)threadIdx.x < pos.cols && e < m.n;
        // the next step: the layer above in the same tile, else the next tile
        int mi_n = mi;
        MeshDev mn = m;
        bool fresh = false;
        if (pos.left > 1) {
            pos.base += ws.s;
            --pos.left;
        } else {
            t = ts.next_tile();
            if (t >= 0) {
                enter(t, mn, mi_n);
                fresh = true;
            }
        }
        wait_lds();                    // the slots are free: every lane has read its row
        issue_priority();
        if (t >= 0) prefetch(mn, pos.base + threadIdx.x);
        else prefetch(m, e);
        body(m, mi, e, active, idx);
        if (fresh) carry_forget(cs);
        m = mn;
        mi = mi_n;
    }
}

// k_top_f64_batch_conn with the column walk of each stacked mesh.  (A batched
// FP32 filter does not walk: its plain pass runs 4 waves per SIMD, which the
// carried face's LDS would cut to 3, and rechecking in FP64 inside the pass
// costs whole waves when the elements FP32 cannot decide are scattered, as
// in meshes whose every vertex is jittered.)
template <bool EDGES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_top_f64_batch_walk(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    __shared__ CarrySlots cs;
    HX_PUSH_STORAGE;
    TileSched ts((int64_t)a.q.cnt->walk_tiles, a.xcds, a.q.cnt);
    batch_walk_loop(a, ts, stage, cs, [&](const MeshDev& m, int mi, int64_t e, bool active, const int* idx) {
        V3 p[8];
        const bool hit = carry_issue(m.points, idx, cs, p);
        wait_loads();
        carry_finish(idx, hit, cs, p);
        finish_element<EDGES>(m, mi, e, active, p, false, a.q, a.max_depth, pb, a.meshes);
    });
    push_flush(pb, sub_list(a.q), a.q, a.mesh, a.meshes);
}

// k_top_f64_range for a batch whose meshes all have trusted connectivity,
// through batch_prefetch_loop.
template <bool EDGES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_top_f64_batch_conn(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    HX_PUSH_STORAGE;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    batch_prefetch_loop(a.meshes, a.tile_mesh, ts, stage,
                        [&](const MeshDev& m, int mi, int64_t e, bool active, const V3* p) {
        finish_element<EDGES>(m, mi, e, active, p, false, a.q, a.max_depth, pb, a.meshes);
    });
    push_flush(pb, sub_list(a.q), a.q, a.mesh, a.meshes);
}

template <bool BATCHED, bool EDGES>
__global__ __launch_bounds__(256) void k_top_f64_list(TopArgs a)
{
    HX_PUSH_STORAGE;
    const unsigned long long cnt = *a.list_count;
    const int64_t n = (int64_t)(cnt < a.q.list_cap ? cnt : a.q.list_cap);
    const int64_t n_tiles = (n + blockDim.x - 1) / blockDim.x;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t i = t * blockDim.x + threadIdx.x;
        const bool active = i < n;
        int mi = 0;
        int64_t e = 0;
        if (active) {
            e = a.q.list_elem[i];
            mi = a.q.list_mesh[i];
        }
        const MeshDev m = BATCHED && active ? a.meshes[mi] : a.mesh;
        process_element<EDGES, kGatherAny>(m, mi, e, active, a.q, a.max_depth, pb, BATCHED ? a.meshes : nullptr);
    }
    push_flush(pb, sub_list(a.q), a.q, a.mesh, BATCHED ? a.meshes : nullptr);
}

// FP32 filter, one element per lane: certain INVALID / VALID elements are
// final here (min_coeff is the FP32 minimum, widened); every other element
// is listed for the FP64 pass (k_top_f64_list), which decides it exactly as
// the plain FP64 path would.

// FP32 decisions for one element per lane.  Elements that need the FP64 pass
// go to the recheck list through the wave's buffer (as finish_element sends
// elements to subdivision), without a block barrier per tile.
// Elements filter_subdivides clears (with a depth cap above 0) skip the
// recheck: they go to the subdivision list through a second buffer, sb, with
// their FP32 minimum as min_coeff, as the FP32-decided elements.
__device__ void filter_finish(const MeshDev& m, int mesh_idx, int64_t e, bool active, const V3 p[8], bool bad,
                              const QueueDev& q, int max_depth, PushBuf& pb, PushBuf& sb, const MeshDev* meshes)
{
    int st = -1;
    bool sub = false;
    float mn = 0.0f;
    if (active) {
        if (!bad) {
            const LeanT<float> r = element_lean_t<float>(p, false);
            st = filter_state(r);
            sub = st < 0 && max_depth > 0 && filter_subdivides(r);
            mn = r.min27;
        }
    }
    const bool recheck = active && !bad && st < 0 && !sub;
    const uint8_t v = bad ? 3 : (uint8_t)st;
    push_entry(pb, recheck_list(q), q, m, meshes, recheck, e, mesh_idx);
    push_entry(sb, sub_list(q), q, m, meshes, sub, e, mesh_idx);
    if (active && !recheck) {
        if (!sub) *global(m.verdict + e) = v;   // listed elements: at push_flush
        if (m.min_coeff) *global(m.min_coeff + e) = bad ? __builtin_nan("") : (double)mn;
    }
    if (pb.n > kPushBuf - 64) push_flush(pb, recheck_list(q), q, m, meshes);
    if (sb.n > kPushBuf - 64) push_flush(sb, sub_list(q), q, m, meshes);
}

template <int G>
__device__ void filter_element(const MeshDev& m, int mesh_idx, int64_t e, bool active, const QueueDev& q,
                               int max_depth, PushBuf& pb, PushBuf& sb, const MeshDev* meshes)
{
    V3 p[8];
    bool bad = false;
    if (active) load_points_t<G>(m, e, p, bad);
    filter_finish(m, mesh_idx, e, active, p, bad, q, max_depth, pb, sb, meshes);
}

template <bool BATCHED, int G>
__global__ __launch_bounds__(256) void k_filter_f32_range(TopArgs a)
{
    HX_PUSH_STORAGE;
    HX_SUB_PUSH_STORAGE;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        MeshDev m;
        int mi;
        int64_t e;
        if (BATCHED) {
            mi = a.tile_mesh[t];
            m = a.meshes[mi];
            e = (t - m.tile_begin) * (int64_t)blockDim.x + threadIdx.x;
        } else {
            mi = 0;
            m = a.mesh;
            e = t * (int64_t)blockDim.x + threadIdx.x;
        }
        filter_element<G>(m, mi, e, e < m.n, a.q, a.max_depth, pb, sb, BATCHED ? a.meshes : nullptr);
    }
    push_flush(pb, recheck_list(a.q), a.q, a.mesh, BATCHED ? a.meshes : nullptr);
    push_flush(sb, sub_list(a.q), a.q, a.mesh, BATCHED ? a.meshes : nullptr);
}

// k_filter_f32_range for a single mesh with trusted connectivity, through
// conn_prefetch_loop.
__global__ __launch_bounds__(256) void k_filter_f32_conn(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    HX_PUSH_STORAGE;
    HX_SUB_PUSH_STORAGE;
    const MeshDev& m = a.mesh;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    conn_prefetch_loop<8>(m.conn, m.n, ts, stage, [&](int64_t e, bool active, const int* idx) {
        V3 p[8];
        gather8(m.points, idx, p);
        wait_loads();
        filter_finish(m, 0, e, active, p, false, a.q, a.max_depth, pb, sb, nullptr);
    });
    push_flush(pb, recheck_list(a.q), a.q, m, nullptr);
    push_flush(sb, sub_list(a.q), a.q, m, nullptr);
}

// k_filter_f32_conn with the column walk, and the FP64 recheck in the same
// pass: the carried face's LDS already limits the block count to what 168
// registers allow, so the elements the FP32 pass cannot decide are redone in
// FP64 here (as finish_element decides them, subdivision list included)
// instead of being listed for a second kernel.  A wave where most lanes need
// it (a run of near-degenerate elements) redoes them at once from the corners
// in its registers; scattered ones are kept in a per-wave LDS buffer and
// redone 64 at a time, each lane gathering its element again, so that a few
// uncertain lanes do not cost their wave a whole FP64 evaluation.  The count
// goes out with one atomic per wave at the end.
constexpr int kRecheckBuf = 128;
constexpr int kRecheckInPlace = 48;   // uncertain lanes from which a wave redoes them at once

template <bool EDGES>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_filter_f32_walk(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    __shared__ CarrySlots cs;
    __shared__ int64_t recheck_buf_[4 * kRecheckBuf];
    HX_PUSH_STORAGE;
    const MeshDev& m = a.mesh;
    const WalkShape ws(m.n, a.q.cnt, a.walk_limit, a.walk_layers);
    TileSched ts(ws.n_tiles, a.xcds, a.q.cnt);
    const int lane = threadIdx.x & 63;
    __attribute__((address_space(3))) int64_t* rbuf =
        (__attribute__((address_space(3))) int64_t*)(recheck_buf_ + (threadIdx.x >> 6) * kRecheckBuf);
    int rn = 0;                          // buffered elements (wave-uniform)
    unsigned long long rechecked = 0;    // elements this wave redid in FP64 (wave-uniform)
    // FP64 decisions of the first `count` buffered elements, one per lane
    auto recheck_buffered = [&](int count) {
        lds_order();                     // the entries other lanes wrote are visible
        const bool on = lane < count;
        int64_t eb = 0;
        V3 q[8];
        bool bad = false;
        if (on) {
            eb = rbuf[lane];
            load_points_t<kGatherConn>(m, eb, q, bad);
        }
        finish_element<EDGES>(m, 0, eb, on, q, false, a.q, a.max_depth, pb, nullptr);
        rechecked += (unsigned long long)count;
    };
    carry_clear(cs);
    walk_prefetch_loop(m.conn, m.n, ws, ts, stage, [&](int64_t e, bool active, const int* idx) {
        if (rn >= 64) {
            // a full batch of buffered elements, before this element's corners
            // are loaded; the rest (fewer than kRecheckInPlace) to the front:
            // reads from [64, rn), writes to [0, rn - 64), disjoint
            recheck_buffered(64);
            int64_t rest = 0;
            if (lane < rn - 64) rest = rbuf[64 + lane];
            if (lane < rn - 64) rbuf[lane] = rest;
            rn -= 64;
        }
        V3 p[8];
        const bool hit = carry_issue(m.points, idx, cs, p);
        wait_loads();
        carry_finish(idx, hit, cs, p);
        int st = -1;
        bool sub = false;
        float mn = 0.0f;
        if (active) {
            const LeanT<float> r = element_lean_t<float>(p, false);
            st = filter_state(r);
            sub = st < 0 && a.max_depth > 0 && filter_subdivides(r);
            mn = r.min27;
        }
        // what filter_subdivides clears goes to subdivision without the recheck
        push_entry(pb, sub_list(a.q), a.q, m, nullptr, sub, e, 0);
        const bool recheck = active && st < 0 && !sub;
        if (active && !recheck) {
            if (!sub) *global(m.verdict + e) = (uint8_t)st;   // listed elements: at push_flush
            if (m.min_coeff) *global(m.min_coeff + e) = (double)mn;
        }
        if (pb.n > kPushBuf - 64) push_flush(pb, sub_list(a.q), a.q, m, nullptr);
        const uint64_t rm = ballot(recheck);
        const int nr = __popcll(rm);
        if (nr >= kRecheckInPlace) {
            // most lanes: at once, from the corners in registers
            rechecked += (unsigned long long)nr;
            finish_element<EDGES>(m, 0, e, recheck, p, false, a.q, a.max_depth, pb, nullptr);
        } else if (nr) {
            // scattered: buffered, redone 64 at a time
            if (recheck) rbuf[rn + lane_rank(rm)] = e;
            rn += nr;
        }
    });
    // what the last steps left (up to 63 + kRecheckInPlace - 1 entries)
    while (rn > 0) {
        const int k = rn < 64 ? rn : 64;
        recheck_buffered(k);
        int64_t rest = 0;
        if (lane < rn - k) rest = rbuf[k + lane];
        if (lane < rn - k) rbuf[lane] = rest;
        rn -= k;
    }
    if (lane == 0 && rechecked) atomicAdd(&a.q.cnt->n_rechecked, rechecked);
    push_flush(pb, sub_list(a.q), a.q, m, nullptr);
}

// k_filter_f32_range for a batch whose meshes all have trusted
// connectivity, through batch_prefetch_loop.
__global__ __launch_bounds__(256) void k_filter_f32_batch_conn(TopArgs a)
{
    __shared__ int4 stage[2 * 256];
    HX_PUSH_STORAGE;
    HX_SUB_PUSH_STORAGE;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    batch_prefetch_loop(a.meshes, a.tile_mesh, ts, stage,
                        [&](const MeshDev& m, int mi, int64_t e, bool active, const V3* p) {
        filter_finish(m, mi, e, active, p, false, a.q, a.max_depth, pb, sb, a.meshes);
    });
    push_flush(pb, recheck_list(a.q), a.q, a.mesh, a.meshes);
    push_flush(sb, sub_list(a.q), a.q, a.mesh, a.meshes);
}

// ------------------------------------------------------------ subdivision

__device__ __forceinline__ int mirrored(int t, int pattern)
{
    const int i = t % 3, j = (t / 3) % 3, k = t / 9;
    const int mi = (pattern & 1) ? 2 - i : i;
    const int mj = (pattern & 2) ? 2 - j : j;
    const int mk = (pattern & 4) ? 2 - k : k;
    return mi + 3 * mj + 9 * mk;
}

// Range of the stored sub-boxes of level L (see Counters::lvl).  Every
// count it reads is final: it was produced by an earlier launch.
struct LevelRange {
    uint64_t base, count, next_base;
};

__device__ LevelRange level_range(const Counters* cnt, int L, uint64_t cap)
{
    uint64_t base = 0, count = 0;
    for (int l = 0; l <= L; ++l) {
        base += count;
        const uint64_t c = cnt->lvl[l];
        count = c < cap - base ? c : cap - base;
    }
    return {base, count, base + count};
}


constexpr int kNodeWords = 30;   // words of a Node that carry data

// One level of the adaptive subdivision (Section 6, step 5).  Each stored
// sub-box of level L gets eight lanes of a wave, one per child octant: the
// group copies the node into LDS (one 256-byte span), every lane takes its
// octant's coefficients by de Casteljau at 1/2 (on the mirrored tensor
// order) and applies the certified decisions.  Children that stay ambiguous
// below the depth cap are appended as level L+1.  A block takes G groups of
// 32 sub-boxes per step (G up to 8, fewer when the level is too small to
// give every block G groups): it first decides every child of the G groups,
// then reserves room for all children to append with one atomic, then
// recomputes the appended children (from the node, still in L2) and writes
// them.  Same-address atomics serialise at about 13 ns, so one per 32
// sub-boxes had dominated the large levels of invalid-heavy batches.  With
// one group per step (small levels) the children stay in registers across
// the reservation instead.
constexpr int kLevelGroups = 8;

__device__ __forceinline__ void level_stage_node(const double* nodes, uint64_t node, int child, double* dst)
{
    // 8 lanes x 32 bytes: the whole node (words 30, 31 are padding)
    const double2* src = reinterpret_cast<const double2*>(nodes + node * 32 + 4 * child);
    const double2 w0 = src[0], w1 = src[1];
    dst += 4 * child;
    dst[0] = w0.x;
    dst[1] = w0.y;
    if (child < 7) {
        dst[2] = w1.x;
        dst[3] = w1.y;
    }
}

// The lane's child octant of the staged node: its 27 coefficients in t, and
// the node's scale, element slot and orientation pattern.
__device__ __forceinline__ void level_child(const double* nd, int child, double t[27], double& scale,
                                            int64_t& sslot)
{
    const uint64_t lo = __double_as_longlong(nd[29]);
    const int pat = (int)(lo >> 32) ^ child;
    sslot = (int64_t)__double_as_longlong(nd[28]);
    scale = nd[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) t[k] = nd[mirrored(k, pat)];
    lower_octant(t);
}

// The certified decisions of Section 6 for one child sub-box of the given
// level (tau: the rounding-error bound at that level).
enum LevelDecision : int { kChildDone = 0, kChildPush, kChildInvalid, kChildUndecided, kChildInexact };

__device__ __forceinline__ int level_decide(const double t[27], double scale, int level, int max_depth)
{
    const double tau = level_threshold(scale, level);
    const double m8 = fmin(fmin(fmin(t[0], t[2]), fmin(t[6], t[8])),
                           fmin(fmin(t[18], t[20]), fmin(t[24], t[26])));
    double m19 = t[1];
#pragma unroll
    for (int k = 3; k < 26; ++k)
        if (k != 6 && k != 8 && k != 18 && k != 20 && k != 24) m19 = fmin(m19, t[k]);
    if (m8 <= -tau) return kChildInvalid;
    if (!(m8 > tau)) return kChildInexact;
    if (m19 > tau) return kChildDone;          // positive on this sub-box
    if (level < max_depth) return kChildPush;
    if (m19 <= -tau) return kChildUndecided;
    return kChildInexact;
}

__device__ __forceinline__ uint32_t level_flags(int d)
{
    return d == kChildInvalid ? kFlagInvalid : d == kChildUndecided ? kFlagUndecided
                                             : d == kChildInexact ? kFlagExact : 0u;
}

// Stores an appended child at slot ns; false when the store is full.
__device__ __forceinline__ bool level_write(const QueueDev& q, uint64_t ns, const double t[27], double scale,
                                            int64_t sslot, int level, int child)
{
    if (ns >= q.node_cap) return false;
    double* out = reinterpret_cast<double*>(q.nodes + ns);
#pragma unroll
    for (int k = 0; k < 27; ++k) out[k] = t[k];
    out[27] = scale;
    out[28] = __longlong_as_double(sslot);
    out[29] = __longlong_as_double((long long)((uint64_t)(uint32_t)level | ((uint64_t)(uint32_t)child << 32)));
    return true;
}

__global__ __launch_bounds__(256) void k_level(LevelArgs a)
{
    __shared__ double stage_mem[4][8][kNodeWords];
    __shared__ unsigned int wave_push[kLevelGroups][4];
    __shared__ unsigned long long block_base;
    const int wid = threadIdx.x >> 6;
    double (*stage)[kNodeWords] = stage_mem[wid];
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 3;
    const int child = lane & 7;
    const QueueDev& q = a.q;
    Counters* cnt = q.cnt;
    const uint64_t cap = q.node_cap;
    const LevelRange r = level_range(cnt, a.level, cap);
    const int level = a.level + 1;   // level of the children evaluated here
    const double* nodes = reinterpret_cast<const double*>(q.nodes);
    // groups per step: as many as keep every block busy, at most kLevelGroups
    const uint64_t groups = (r.count + 31) / 32;
    const uint64_t per_block = groups / gridDim.x;
    const int G = per_block >= (uint64_t)kLevelGroups ? kLevelGroups : per_block < 1 ? 1 : (int)per_block;
    const uint64_t span = 32ull * (uint64_t)G;
    if (G == 1) {
        for (uint64_t b0 = (uint64_t)blockIdx.x * 32; b0 < r.count; b0 += (uint64_t)gridDim.x * 32) {
            // one group per step (small levels): decide, reserve and write
            // with the children still in registers
            const uint64_t i = b0 + (uint64_t)(wid * 8 + grp);
            const bool act = i < r.count;
            if (act) level_stage_node(nodes, r.base + i, child, stage[grp]);
            lds_order();
            int d = kChildDone;
            int64_t sslot = 0;
            double scale = 0.0;
            double t[27];
            if (act) {
                level_child(stage[grp], child, t, scale, sslot);
                const bool dead = (__hip_atomic_load(q.sub_flags + sslot, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) & kFlagInvalid) != 0u;
                if (!dead) d = level_decide(t, scale, level, a.max_depth);
            }
            const bool push = d == kChildPush;
            uint32_t fl = level_flags(d);
            const uint64_t pmask = ballot(push);
            if (lane == 0) wave_push[0][wid] = (unsigned int)__popcll(pmask);
            __syncthreads();
            if (threadIdx.x == 0) {
                const unsigned long long total = wave_push[0][0] + wave_push[0][1] + wave_push[0][2] + wave_push[0][3];
                block_base = total ? atomicAdd(&cnt->lvl[level], total) : 0ull;
            }
            __syncthreads();
            if (push) {
                unsigned long long o = block_base + (unsigned long long)lane_rank(pmask);
                for (int w = 0; w < wid; ++w) o += wave_push[0][w];
                if (!level_write(q, r.next_base + o, t, scale, sslot, level, child)) fl |= kFlagOverflow;
            }
            if (fl) atomicOr(q.sub_flags + sslot, fl);
            __syncthreads();   // wave_push and block_base are rewritten next step
        }
        return;
    }
    for (uint64_t b0 = (uint64_t)blockIdx.x * span; b0 < r.count; b0 += (uint64_t)gridDim.x * span) {
        // decide every child of the G groups
        uint32_t pushed = 0;   // bit g: this lane's child of group g is appended
        for (int g = 0; g < G; ++g) {
            const uint64_t i = b0 + (uint64_t)(32 * g + wid * 8 + grp);
            const bool act = i < r.count;
            if (act) level_stage_node(nodes, r.base + i, child, stage[grp]);
            lds_order();
            int d = kChildDone;
            int64_t sslot = 0;
            if (act) {
                double t[27];
                double scale;
                level_child(stage[grp], child, t, scale, sslot);
                const bool dead = (__hip_atomic_load(q.sub_flags + sslot, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) & kFlagInvalid) != 0u;
                if (!dead) d = level_decide(t, scale, level, a.max_depth);
            }
            const bool push = d == kChildPush;
            const uint32_t fl = level_flags(d);
            if (fl) atomicOr(q.sub_flags + sslot, fl);
            const uint64_t pmask = ballot(push);
            if (lane == 0) wave_push[g][wid] = (unsigned int)__popcll(pmask);
            if (push) pushed |= 1u << g;
            lds_order();               // the node is read before the next one is staged
        }
        // room for every appended child of the step: one atomic per block
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long total = 0;
            for (int g = 0; g < G; ++g)
                total += wave_push[g][0] + wave_push[g][1] + wave_push[g][2] + wave_push[g][3];
            block_base = total ? atomicAdd(&cnt->lvl[level], total) : 0ull;
        }
        __syncthreads();
        // write the appended children, in order of groups, waves and lanes
        unsigned long long off = block_base;
        for (int g = 0; g < G; ++g) {
            const bool push = (pushed >> g) & 1u;
            const uint64_t pmask = ballot(push);
            if (pmask) {
                const uint64_t i = b0 + (uint64_t)(32 * g + wid * 8 + grp);
                if (i < r.count) level_stage_node(nodes, r.base + i, child, stage[grp]);
                lds_order();
                if (push) {
                    double t[27];
                    double scale;
                    int64_t sslot;
                    level_child(stage[grp], child, t, scale, sslot);
                    unsigned long long o = off + (unsigned long long)lane_rank(pmask);
                    for (int w = 0; w < wid; ++w) o += wave_push[g][w];
                    if (!level_write(q, r.next_base + o, t, scale, sslot, level, child))
                        atomicOr(q.sub_flags + sslot, kFlagOverflow);
                }
                lds_order();
            }
            off += wave_push[g][0] + wave_push[g][1] + wave_push[g][2] + wave_push[g][3];
        }
        __syncthreads();   // wave_push and block_base are rewritten next step
    }
}

// ------------------------------------------------ depth-first subdivision
//
// The level-by-level subdivision keeps a whole level of every listed
// element's tree in the store.  An element whose ambiguous region is a
// surface (min J = 0 along a curve, say) needs about 4^L sub-boxes at level L,
// more than any store holds at deep caps.  Such elements, when a round with a
// single listed element still overflows, are decided here instead, as the
// recursion of Section 6 does: depth first, one lane per element, keeping
// only the path from the root (one node per level) and the next child to
// visit at each level.  The decisions are those of the level kernel
// (level_decide), and the verdict folds the same flags (INVALID > exact >
// UNDECIDED > VALID), so it is the level-by-level verdict.

// Child cursor of a stack node (word 28).
__device__ __forceinline__ int dfs_cursor(const double* nd) { return (int)__double_as_longlong(nd[28]); }
__device__ __forceinline__ void dfs_set_cursor(double* nd, int c) { nd[28] = __longlong_as_double((long long)c); }

// Depth-first walk of the tree below the root in st[0..26] (tensor order);
// st holds max_depth + 1 nodes of 32 words.  Returns the element's flags.
__device__ uint32_t dfs_subdivide(double* st, double scale, int max_depth)
{
    uint32_t flags = 0;
    dfs_set_cursor(st, 0);
    int L = 0;
    while (L >= 0) {
        double* nd = st + 32 * L;
        const int c = dfs_cursor(nd);
        if (c == 8) {
            --L;
            continue;
        }
        dfs_set_cursor(nd, c + 1);
        double t[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) t[k] = nd[mirrored(k, c)];
        lower_octant(t);
        const int d = level_decide(t, scale, L + 1, max_depth);
        if (d == kChildInvalid) return flags | kFlagInvalid;
        if (d == kChildInexact) {
            flags |= kFlagExact;
        } else if (d == kChildUndecided) {
            flags |= kFlagUndecided;
        } else if (d == kChildPush) {
            double* ch = nd + 32;
#pragma unroll
            for (int k = 0; k < 27; ++k) ch[mirrored(k, c)] = t[k];   // the child in its own orientation
            dfs_set_cursor(ch, 0);
            ++L;
        }
    }
    return flags;
}

__global__ __launch_bounds__(64) void k_dfs(DfsArgs a)
{
    const QueueDev& q = a.q;
    const unsigned long long cnt = *(&q.cnt->n_list);
    const int64_t n = (int64_t)(cnt < q.list_cap ? cnt : q.list_cap);
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double* st = reinterpret_cast<double*>(q.nodes) + 32 * (a.max_depth + 1) * lane;
    // lane l (below a.lanes, the stacks the store holds) takes the elements
    // l, l + lanes, ...; whole waves iterate together (wave-level list
    // appends) until none of their lanes has an element left
    for (int64_t i = lane;; i += a.lanes) {
        const bool active = lane < a.lanes && i < n;
        if (!ballot(active)) break;
        int64_t e = 0;
        int mi = 0;
        uint8_t v = 0;
        bool exact = false;
        if (active) {
            e = q.list_elem[i];
            mi = q.list_mesh[i];
            const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
            V3 p[8];
            bool bad = false;
            load_points(m, e, p, bad);
            if (bad) {
                v = 3;
            } else {
                ElementValues r;
                element_values(p, r);
                const int ts = top_state(r, summarize(r), a.max_depth);
                if (ts == kTopSubdivide) {
#pragma unroll
                    for (int k = 0; k < 27; ++k) st[fig3_to_tensor(k)] = coefficient(r, k);
                    const uint32_t f = dfs_subdivide(st, r.scale, a.max_depth);
                    v = (f & kFlagInvalid) ? 0 : (f & kFlagExact) ? kExact : (f & kFlagUndecided) ? 2 : 1;
                } else {
                    v = ts == kTopExact ? kExact : (uint8_t)ts;
                }
                exact = v == kExact;
            }
        }
        bool deferred = false;
        const uint64_t xmask = ballot(exact);
        if (xmask) {
            const unsigned long long x = wave_reserve(&q.cnt->n_exact, xmask);
            if (exact && x < q.exact_cap) {
                q.exact_elem[x] = e;
                q.exact_mesh[x] = mi;
            } else if (exact) {
                v = kDeferred;
                deferred = true;
            }
        }
        wave_count(&q.cnt->n_deferred, deferred);
        if (active) {
            const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
            m.verdict[e] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_fold(FoldArgs a)
{
    const QueueDev& q = a.q;
    const unsigned long long ns = *(&q.cnt->n_sub);
    const int64_t n = (int64_t)(ns < q.root_cap ? ns : q.root_cap);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // whole waves iterate together (wave-level list appends and counters)
    for (int64_t s0 = blockIdx.x * (int64_t)blockDim.x; s0 < n; s0 += stride) {
        const int64_t s = s0 + threadIdx.x;
        const bool active = s < n;
        uint32_t f = 0;
        int64_t e = -1;
        int mi = 0;
        if (active) {
            e = q.sub_elem[s];
            f = q.sub_flags[s];
            mi = q.sub_mesh[s];
        }
        const bool live = active && e >= 0;
        const bool to_exact = live && !(f & kFlagInvalid) && (f & kFlagExact);
        bool deferred = live && !(f & kFlagInvalid) && !(f & kFlagExact) && (f & kFlagOverflow);
        uint8_t v = (f & kFlagInvalid) ? 0 : (f & kFlagUndecided) ? 2 : 1;
        if (deferred) v = kDeferred;
        const uint64_t xmask = ballot(to_exact);
        if (xmask) {
            const unsigned long long x = wave_reserve(&q.cnt->n_exact, xmask);
            if (to_exact) {
                if (x < q.exact_cap) {
                    q.exact_elem[x] = e;
                    q.exact_mesh[x] = mi;
                    v = kExact;
                } else {
                    v = kDeferred;
                    deferred = true;
                }
            }
        }
        wave_count(&q.cnt->n_deferred, deferred);
        if (live) {
            const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
            m.verdict[e] = v;
        }
    }
}

// ======================================================= minimum of J
//
// Certified bounds lo <= min J <= hi over [0,1]^3 (hexval_min_jacobian).  The
// bounds of Section 3.1: on a box, the smallest of its 27 coefficients bounds
// J from below (convex hull property) and each corner coefficient is a value
// of J, so the smallest corner value met bounds min J from above.  They are
// sharpened level by level: a box of level L is retired when its lower bound
// is within tol = rtol * M^/6 of U_L, the smallest corner value over the boxes
// of levels 0..L, or when L is the depth cap; otherwise its 8 children are
// stored as level L+1.  Decisions at level L read U_L only, so the result does
// not depend on the order in which boxes are processed.
//
// Per subdivided element (slot) three arrays u[0..2] rotate by level: the
// launch for level L reads U_L from u[L%3], lowers u[(L+1)%3] to
// min(U_L, corner values of level L+1) for every box it splits, and resets
// u[(L+2)%3], which the next launch writes.

// Range of the stored boxes of level L.  Children are reserved 8 at a time
// from a multiple of 8 past the level's base and a box is stored only when
// all 8 fit, so at levels >= 1 the stored span is the reserved count cut to
// whole groups of 8 below the capacity (slots past it were never written).
__device__ LevelRange minj_level_range(const Counters* cnt, int L, uint64_t cap)
{
    uint64_t base = 0, count = 0;
    for (int l = 0; l <= L; ++l) {
        base += count;
        const uint64_t c = cnt->lvl[l];
        const uint64_t room = l == 0 ? cap - base : (cap - base) & ~7ull;
        count = c < room ? c : room;
    }
    return {base, count, base + count};
}

// Order-preserving map of doubles (never NaN here) to unsigned integers.
__device__ __forceinline__ unsigned long long ord_of(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double of_ord(unsigned long long o)
{
    return __longlong_as_double((long long)((o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o));
}

// Widening of a computed bound: the coefficient error bound at the depth cap
// (it covers corner values and coefficients of every level), then one ulp
// outwards for the rounding of the addition.
__device__ __forceinline__ double minj_margin(double scale, int max_depth)
{
    return (kTauCoeff + kTauLevel * max_depth) * kU64 * scale;
}

__device__ __forceinline__ void minj_write(const MinjArgs& a, int64_t e, double lo, double hi, double scale,
                                           int st)
{
    if (st <= 2) {
        const double mg = minj_margin(scale, a.max_depth);
        lo = next_down(lo - mg);
        hi = next_up(hi + mg);
    } else {
        lo = hi = __builtin_nan("");
    }
    a.mj.lo[e] = lo;
    a.mj.hi[e] = hi;
    if (a.mj.status) a.mj.status[e] = (uint8_t)st;
}

// Status codes (match HEXVAL_MINJ_* of the C ABI).
constexpr int kMjConverged = 0, kMjCapped = 1, kMjQueueFull = 2, kMjBadInput = 3, kMjOutOfRange = 4;

// Level 0, one element per lane: the bounds of the whole element from the
// first-pass arithmetic; elements whose bounds are not yet within tol are
// listed for subdivision, up to root_cap of them, the rest deferred to the
// next round.  Later rounds take their elements from in_list.
__device__ void minj_element(const MinjArgs& a, int64_t e, bool active, const V3 p[8], bool bad)
{
    const QueueDev& q = a.q;
    int st = -1;
    double lo = 0.0, hi = 0.0, scale = 0.0;
    if (active) {
        if (bad) {
            st = kMjBadInput;
        } else {
            // before the arithmetic, so that the corners need not stay live
            // through it
            bool finite = true;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                finite = finite && isfinite(p[k].x) && isfinite(p[k].y) && isfinite(p[k].z);
            const LeanResult r = element_lean(p, false);
            if (!r.certified_range) {
                st = finite ? kMjOutOfRange : kMjBadInput;
            } else {
                lo = r.min27;
                hi = r.m20;
                scale = r.scale;
                const double tol = a.mj.rtol * (1.0 / 6.0) * scale;
                if (lo >= hi - tol) st = kMjConverged;
                else if (a.max_depth == 0) st = kMjCapped;
            }
        }
    }
    const bool push = active && st < 0;
    const uint64_t pmask = ballot(push);
    bool defer = false;
    if (pmask) {
        const unsigned long long slot = wave_reserve(&q.cnt->n_sub, pmask);
        if (push) {
            if (slot < a.root_cap) {
                q.sub_elem[slot] = e;
                q.sub_mesh[slot] = 0;
            } else {
                defer = true;
            }
        }
    }
    const uint64_t dmask = ballot(defer);
    if (dmask) {
        const unsigned long long d = wave_reserve(&q.cnt->n_deferred, dmask);
        if (defer) a.out_list[d] = e;
    }
    if (active && st >= 0) minj_write(a, e, lo, hi, scale, st);
}

__global__ __launch_bounds__(256) void k_minj_top(MinjArgs a)
{
    const MeshDev& m = a.mesh;
    const int64_t count = a.in_list ? a.in_count : m.n;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        const int64_t i = t * (int64_t)blockDim.x + threadIdx.x;
        const bool active = i < count;
        const int64_t e = !active ? 0 : a.in_list ? a.in_list[i] : i;
        V3 p[8];
        bool bad = false;
        if (active) load_points(m, e, p, bad);
        minj_element(a, e, active, p, bad);
    }
}

// k_minj_top over a whole single mesh with trusted connectivity (the first
// round), through conn_prefetch_loop.
__global__ __launch_bounds__(256) void k_minj_top_conn(MinjArgs a)
{
    __shared__ int4 stage[2 * 256];
    const MeshDev& m = a.mesh;
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    conn_prefetch_loop<8>(m.conn, m.n, ts, stage, [&](int64_t e, bool active, const int* idx) {
        V3 p[8];
        gather8(m.points, idx, p);
        wait_loads();
        minj_element(a, e, active, p, false);
    });
}

// k_minj_top_conn with the column walk.
__global__ __launch_bounds__(256) void k_minj_top_walk(MinjArgs a)
{
    __shared__ int4 stage[2 * 256];
    __shared__ CarrySlots cs;
    const MeshDev& m = a.mesh;
    const WalkShape ws(m.n, a.q.cnt, a.walk_limit, a.walk_layers);
    TileSched ts(ws.n_tiles, a.xcds, a.q.cnt);
    carry_clear(cs);
    walk_prefetch_loop(m.conn, m.n, ws, ts, stage, [&](int64_t e, bool active, const int* idx) {
        V3 p[8];
        const bool hit = carry_issue(m.points, idx, cs, p);
        wait_loads();
        carry_finish(idx, hit, cs, p);
        minj_element(a, e, active, p, false);
    });
}

// Root boxes of the listed elements: full coefficients, their minimum (word
// 30 of the node) and the per-element arrays.
__global__ __launch_bounds__(256) void k_minj_roots(MinjArgs a)
{
    const QueueDev& q = a.q;
    const unsigned long long ns = q.cnt->n_sub;
    const int64_t n = (int64_t)(ns < a.root_cap ? ns : a.root_cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) q.cnt->lvl[0] = (unsigned long long)n;
    const unsigned long long inf = ord_of(HUGE_VAL);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        V3 p[8];
        bool bad = false;
        load_points(a.mesh, q.sub_elem[s], p, bad);
        ElementValues r;
        element_values(p, r);
        Node* nd = q.nodes + s;
        write_root(nd, r, s);
        double m27 = coefficient(r, 0), mc = r.c[0];
#pragma unroll
        for (int k = 1; k < 27; ++k) m27 = fmin(m27, coefficient(r, k));
#pragma unroll
        for (int k = 1; k < 8; ++k) mc = fmin(mc, r.c[k]);
        reinterpret_cast<double*>(nd)[30] = m27;
        q.sub_flags[s] = 0u;
        a.mj.u[0][s] = ord_of(mc);
        a.mj.u[1][s] = inf;
        a.mj.u[2][s] = inf;
        a.mj.ufinal[s] = ord_of(mc);
        a.mj.lb[s] = inf;
    }
}

// One level: eight lanes per stored box (one per child octant).  The box is
// retired or split by the rule above; a split box gets 8 consecutive slots of
// level L+1 (one atomic per block of 32 boxes) and every lane writes its
// child, with the child's minimum coefficient in word 30.  A box whose
// children do not fit is retired and its element flagged.
__device__ __forceinline__ void minj_stage_node(const double* nodes, uint64_t node, int child, double* dst)
{
    const double2* src = reinterpret_cast<const double2*>(nodes + node * 32 + 4 * child);
    const double2 w0 = src[0], w1 = src[1];
    dst += 4 * child;
    dst[0] = w0.x;
    dst[1] = w0.y;
    dst[2] = w1.x;
    dst[3] = w1.y;
}

// One level of the min J refinement: eight lanes per stored box.  A box whose
// bounds are not yet within the tolerance is split into its 8 octants (all
// stored, 8 slots).  As in k_level, a block decides G groups of 32 boxes,
// reserves the slots of all their split boxes with one atomic, then writes
// the octants.
__global__ __launch_bounds__(256) void k_minj_level(MinjArgs a)
{
    __shared__ double stage_mem[4][8][32];
    __shared__ unsigned int wave_split[kLevelGroups][4];
    __shared__ unsigned long long block_base;
    const int wid = threadIdx.x >> 6;
    double (*stage)[32] = stage_mem[wid];
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 3;
    const int child = lane & 7;
    const QueueDev& q = a.q;
    Counters* cnt = q.cnt;
    const uint64_t cap = q.node_cap;
    const int L = a.level;
    const uint64_t* R = a.mj.u[L % 3];
    uint64_t* W = a.mj.u[(L + 1) % 3];
    uint64_t* Z = a.mj.u[(L + 2) % 3];
    {
        const unsigned long long ns = cnt->n_sub;
        const uint64_t n_slots = ns < a.root_cap ? ns : a.root_cap;
        const unsigned long long inf = ord_of(HUGE_VAL);
        for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < n_slots;
             s += (uint64_t)gridDim.x * blockDim.x)
            Z[s] = inf;
    }
    const LevelRange r = minj_level_range(cnt, L, cap);
    const double* nodes = reinterpret_cast<const double*>(q.nodes);
    const uint64_t groups = (r.count + 31) / 32;
    const uint64_t per_block = groups / gridDim.x;
    const int G = per_block >= (uint64_t)kLevelGroups ? kLevelGroups : per_block < 1 ? 1 : (int)per_block;
    const uint64_t span = 32ull * (uint64_t)G;
    // the box of the lane's group: bounds and the decision
    struct Box {
        double lo, scale, U;
        int64_t sslot;
        int orient;
        bool split, capped;
    };
    auto decide = [&](const double* nd) {
        Box x;
        x.lo = nd[30];
        x.scale = nd[27];
        x.sslot = (int64_t)__double_as_longlong(nd[28]);
        x.orient = (int)((uint64_t)__double_as_longlong(nd[29]) >> 32);
        x.U = of_ord(R[x.sslot]);
        const bool close = x.lo >= x.U - a.mj.rtol * (1.0 / 6.0) * x.scale;
        x.split = L == 0 || (!close && L < a.max_depth);
        x.capped = !x.split && !close;
        return x;
    };
    for (uint64_t b0 = (uint64_t)blockIdx.x * span; b0 < r.count; b0 += (uint64_t)gridDim.x * span) {
        // decide the boxes of the G groups; boxes not split are final here
        uint32_t splits = 0;   // bit g: the lane's box of group g is split
        for (int g = 0; g < G; ++g) {
            const uint64_t i = b0 + (uint64_t)(32 * g + wid * 8 + grp);
            const bool act = i < r.count;
            if (act) minj_stage_node(nodes, r.base + i, child, stage[grp]);
            lds_order();
            bool split = false;
            if (act) {
                const Box x = decide(stage[grp]);
                split = x.split;
                if (!split && child == 0) {
                    atomicMin(&a.mj.lb[x.sslot], ord_of(x.lo));
                    if (x.capped) atomicOr(q.sub_flags + x.sslot, kFlagUndecided);
                }
            }
            const uint64_t smask = ballot(split && child == 0);
            if (lane == 0) wave_split[g][wid] = (unsigned int)__popcll(smask);
            if (split) splits |= 1u << g;
            lds_order();               // the box is read before the next one is staged
        }
        // 8 slots per split box, for the whole step at once
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long total = 0;
            for (int g = 0; g < G; ++g)
                total += wave_split[g][0] + wave_split[g][1] + wave_split[g][2] + wave_split[g][3];
            block_base = total ? atomicAdd(&cnt->lvl[L + 1], 8ull * total) : 0ull;
        }
        __syncthreads();
        unsigned long long before = 0;   // split boxes of the step's earlier groups
        for (int g = 0; g < G; ++g) {
            const bool split = (splits >> g) & 1u;
            const uint64_t smask = ballot(split && child == 0);
            if (smask) {
                const uint64_t i = b0 + (uint64_t)(32 * g + wid * 8 + grp);
                if (i < r.count) minj_stage_node(nodes, r.base + i, child, stage[grp]);
                lds_order();
                double cmin = HUGE_VAL;
                bool stored = false;
                Box x{};
                if (split) {
                    x = decide(stage[grp]);
                    unsigned long long rank = before + (unsigned long long)__popcll(smask & ((1ull << (grp * 8)) - 1ull));
                    for (int w = 0; w < wid; ++w) rank += wave_split[g][w];
                    const uint64_t first = r.next_base + block_base + 8ull * rank;
                    stored = first + 8 <= cap;
                    if (stored) {
                        double t[27];
                        const double* nd = stage[grp];
                        const int pat = x.orient ^ child;
#pragma unroll
                        for (int k = 0; k < 27; ++k) t[k] = nd[mirrored(k, pat)];
                        lower_octant(t);
                        cmin = fmin(fmin(fmin(t[0], t[2]), fmin(t[6], t[8])),
                                    fmin(fmin(t[18], t[20]), fmin(t[24], t[26])));
                        double m27 = t[0];
#pragma unroll
                        for (int k = 1; k < 27; ++k) m27 = fmin(m27, t[k]);
                        double* out = reinterpret_cast<double*>(q.nodes + first + child);
#pragma unroll
                        for (int k = 0; k < 27; ++k) out[k] = t[k];
                        out[27] = x.scale;
                        out[28] = __longlong_as_double(x.sslot);
                        out[29] = __longlong_as_double((long long)((uint64_t)(uint32_t)(L + 1) |
                                                                   ((uint64_t)(uint32_t)child << 32)));
                        out[30] = m27;
                    }
                }
#pragma unroll
                for (int d = 1; d < 8; d <<= 1) cmin = fmin(cmin, __shfl_xor(cmin, d, 64));
                if (split && child == 0) {
                    if (stored) {
                        atomicMin(&W[x.sslot], ord_of(fmin(x.U, cmin)));
                        atomicMin(&a.mj.ufinal[x.sslot], ord_of(cmin));
                    } else {
                        atomicMin(&a.mj.lb[x.sslot], ord_of(x.lo));
                        atomicOr(q.sub_flags + x.sslot, kFlagOverflow);
                    }
                }
                lds_order();
            }
            before += wave_split[g][0] + wave_split[g][1] + wave_split[g][2] + wave_split[g][3];
        }
        __syncthreads();   // wave_split and block_base are rewritten next step
    }
}

// Outputs of the subdivided elements; an element that ran out of room is
// deferred to the next round (redone from scratch), or reports QUEUE_FULL
// with its bounds so far in the final round.  Whole waves iterate together
// (wave-level list appends).
__global__ __launch_bounds__(256) void k_minj_fold(MinjArgs a)
{
    const QueueDev& q = a.q;
    const unsigned long long ns = q.cnt->n_sub;
    const int64_t n = (int64_t)(ns < a.root_cap ? ns : a.root_cap);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s0 = blockIdx.x * (int64_t)blockDim.x; s0 < n; s0 += stride) {
        const int64_t s = s0 + threadIdx.x;
        const bool active = s < n;
        const uint32_t f = active ? q.sub_flags[s] : 0u;
        const bool over = active && (f & kFlagOverflow);
        const bool defer = over && !a.final_round;
        const uint64_t dmask = ballot(defer);
        if (dmask) {
            const unsigned long long d = wave_reserve(&q.cnt->n_deferred, dmask);
            if (defer) a.out_list[d] = q.sub_elem[s];
        }
        if (active && !defer) {
            const int st = over ? kMjQueueFull : (f & kFlagUndecided) ? kMjCapped : kMjConverged;
            minj_write(a, q.sub_elem[s], of_ord(a.mj.lb[s]), of_ord(a.mj.ufinal[s]), q.nodes[s].scale, st);
        }
    }
}

// ================================================= corner-only test
//
// Test 1 of the comparison in Section 7: the element passes when its 8
// corner values of J (the corner coefficients b_1..b_8, 6 x the volumes of
// the corner tetrahedra) are all positive.  It is a necessary condition of
// validity.  Signs are certified with the value bound (kTauValue u M^);
// elements whose signs are not certified, or whose scales leave the guard
// range, go to the exact tier.  Corner quality: the minimum over the corners
// of J_c / (|e_xi| |e_eta| |e_zeta|), the three edge vectors leaving the
// corner (a corner with a zero-length edge counts as 0); NaN for bad input
// and outside the guard range.

__device__ __forceinline__ double norm3(const W3<double>& v)
{
    return sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
}

// 3 waves per SIMD (168 VGPRs) instead of the 2 that 175 allowed: 16M
// independent hexes 0.696 -> 0.665 ms (with the quality output 0.774 -> 0.742)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_corner_test(CornerArgs a)
{
    const MeshDev& m = a.mesh;
    const QueueDev& q = a.q;
    TileSched ts(a.n_tiles, a.xcds, q.cnt);
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        const int64_t e = t * (int64_t)blockDim.x + threadIdx.x;
        const bool active = e < m.n;
        uint8_t v = 0;
        double qual = __builtin_nan("");
        bool exact = false;
        V3 p[8];
        bool bad = false;
        issue_priority();   // (A/B on 16M independent hexes: 4% faster)
        if (active) load_points(m, e, p, bad);
        wait_loads();
        if (active) {
            if (bad) {
                v = 3;
            } else {
                typedef W3<double> E;
                const E a00 = edge_t<double>(p[1], p[0]), a10 = edge_t<double>(p[2], p[3]);
                const E a01 = edge_t<double>(p[5], p[4]), a11 = edge_t<double>(p[6], p[7]);
                const E b00 = edge_t<double>(p[3], p[0]), b10 = edge_t<double>(p[2], p[1]);
                const E b01 = edge_t<double>(p[7], p[4]), b11 = edge_t<double>(p[6], p[5]);
                const E c00 = edge_t<double>(p[4], p[0]), c10 = edge_t<double>(p[5], p[1]);
                const E c01 = edge_t<double>(p[7], p[3]), c11 = edge_t<double>(p[6], p[2]);
                const double sx = fmax(fmax(amax_t(fabs(a00.x), a10), amax_t(fabs(a00.y), a01)), amax_t(fabs(a00.z), a11));
                const double sy = fmax(fmax(amax_t(fabs(b00.x), b10), amax_t(fabs(b00.y), b01)), amax_t(fabs(b00.z), b11));
                const double sz = fmax(fmax(amax_t(fabs(c00.x), c10), amax_t(fabs(c00.y), c01)), amax_t(fabs(c00.z), c11));
                // corner (i,j,k): xi-edge a_jk, eta-edge b_ik, zeta-edge c_ij
                const double J[8] = {triple_t(a00, b00, c00), triple_t(a00, b10, c10), triple_t(a10, b10, c11),
                                     triple_t(a10, b00, c01), triple_t(a01, b01, c00), triple_t(a01, b11, c10),
                                     triple_t(a11, b11, c11), triple_t(a11, b01, c01)};
                bool finite = true;
#pragma unroll
                for (int k = 0; k < 8; ++k) finite = finite && isfinite(J[k]);
                const bool in_range = sx >= Guard<double>::lo && sx <= Guard<double>::hi && sy >= Guard<double>::lo &&
                                      sy <= Guard<double>::hi && sz >= Guard<double>::lo && sz <= Guard<double>::hi;
                if (!finite) {
                    bool coords = true;
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        coords = coords && isfinite(p[k].x) && isfinite(p[k].y) && isfinite(p[k].z);
                    if (coords) exact = true;   // overflow of a finite input: outside the guard
                    else v = 3;
                } else if (!in_range) {
                    exact = true;
                } else {
                    const double tau = kTauValue * kU64 * ((6.0 * sx) * sy * sz);
                    bool neg = false, pos = true;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        neg = neg || J[k] <= -tau;
                        pos = pos && J[k] > tau;
                    }
                    if (neg) v = 0;
                    else if (pos) v = 1;
                    else exact = true;
                    const double na[4] = {norm3(a00), norm3(a10), norm3(a01), norm3(a11)};
                    const double nb[4] = {norm3(b00), norm3(b10), norm3(b01), norm3(b11)};
                    const double nc[4] = {norm3(c00), norm3(c10), norm3(c01), norm3(c11)};
                    qual = HUGE_VAL;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int i = k == 1 || k == 2 || k == 5 || k == 6;
                        const int j = k == 2 || k == 3 || k == 6 || k == 7;
                        const int l = k >= 4;
                        const double den = na[j + 2 * l] * nb[i + 2 * l] * nc[i + 2 * j];
                        qual = fmin(qual, den > 0.0 ? J[k] / den : 0.0);
                    }
                }
            }
        }
        const uint64_t xmask = ballot(exact);
        if (xmask) {
            const unsigned long long slot = wave_reserve(&q.cnt->n_exact, xmask);
            if (exact && slot < q.exact_cap) {
                q.exact_elem[slot] = e;
                q.exact_mesh[slot] = 0;
            }
        }
        if (exact) v = kExact;   // pending: settled by the exact tier
        if (active) {
            m.verdict[e] = v;
            if (a.quality) a.quality[e] = qual;
        }
    }
}

// Lists pending elements into the exact list (up to its capacity), for the
// rounds after the first when more were pending than it holds.  Whole waves
// iterate together.
__global__ __launch_bounds__(256) void k_corner_collect(CornerArgs a)
{
    const MeshDev& m = a.mesh;
    const QueueDev& q = a.q;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = blockIdx.x * (int64_t)blockDim.x; e0 < m.n; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        const bool pend = e < m.n && m.verdict[e] == kExact;
        const uint64_t mask = ballot(pend);
        if (mask) {
            const unsigned long long slot = wave_reserve(&q.cnt->n_exact, mask);
            if (pend && slot < q.exact_cap) {
                q.exact_elem[slot] = e;
                q.exact_mesh[slot] = 0;
            }
        }
    }
}

// ================================================ linear quadrangles
//
// Section 2.1: the bilinear map of [0,1]^2 (corners at (0,0) (1,0) (1,1)
// (0,1)) has a bilinear J, whose minimum is one of the four corner values
// J = det[x_xi x_eta] at the corner.  Signs are certified with 9 u S^2 (S the
// largest |component| of the four edge vectors, in [2^-450, 2^450]); other
// elements go to the exact tier.  min_j: the smallest corner value.

__device__ __forceinline__ void load_quad(const MeshDev& m, int64_t e, double2 p[4], bool& bad)
{
    if (m.conn) {
        const int4 c = *reinterpret_cast<const int4*>(m.conn + 4 * e);
        const int idx[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (m.validate && (idx[k] < 0 || (int64_t)idx[k] >= m.n_points)) bad = true;
        }
        if (bad) return;
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = *reinterpret_cast<const double2*>(m.points + 2 * (int64_t)idx[k]);
    } else {
        const double2* v = reinterpret_cast<const double2*>(m.points + 8 * e);
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = v[k];
    }
}

__device__ __forceinline__ double cross2(double ax, double ay, double bx, double by)
{
    return fma(ax, by, -(ay * bx));
}

__device__ __forceinline__ void quad_element(const CornerArgs& a, int64_t e, bool active, const double2 p[4], bool bad)
{
    const MeshDev& m = a.mesh;
    const QueueDev& q = a.q;
    uint8_t v = 0;
    double mn = __builtin_nan("");
    bool exact = false;
    if (active) {
        bool finite = !bad;
#pragma unroll
        for (int k = 0; k < 4; ++k) finite = finite && isfinite(p[k].x) && isfinite(p[k].y);
        if (!finite) {
            v = 3;
        } else {
            // x_xi on eta = 0 and 1, x_eta on xi = 0 and 1
            const double ax0 = p[1].x - p[0].x, ay0 = p[1].y - p[0].y;
            const double ax1 = p[2].x - p[3].x, ay1 = p[2].y - p[3].y;
            const double bx0 = p[3].x - p[0].x, by0 = p[3].y - p[0].y;
            const double bx1 = p[2].x - p[1].x, by1 = p[2].y - p[1].y;
            const double S = fmax(fmax(fmax(fabs(ax0), fabs(ay0)), fmax(fabs(ax1), fabs(ay1))),
                                  fmax(fmax(fabs(bx0), fabs(by0)), fmax(fabs(bx1), fabs(by1))));
            const double J0 = cross2(ax0, ay0, bx0, by0);   // (0,0)
            const double J1 = cross2(ax0, ay0, bx1, by1);   // (1,0)
            const double J2 = cross2(ax1, ay1, bx1, by1);   // (1,1)
            const double J3 = cross2(ax1, ay1, bx0, by0);   // (0,1)
            mn = fmin(fmin(J0, J1), fmin(J2, J3));
            const double tau = 9.0 * kU64 * S * S;
            const bool in_range = S >= 0x1p-450 && S <= 0x1p+450;
            if (!in_range) exact = true;
            else if (mn <= -tau) v = 0;
            else if (mn > tau) v = 1;
            else exact = true;
        }
    }
    const uint64_t xmask = ballot(exact);
    if (xmask) {
        const unsigned long long slot = wave_reserve(&q.cnt->n_exact, xmask);
        if (exact && slot < q.exact_cap) {
            q.exact_elem[slot] = e;
            q.exact_mesh[slot] = 0;
        }
    }
    if (exact) v = kExact;
    if (active) {
        m.verdict[e] = v;
        if (a.quality) a.quality[e] = mn;
    }
}

__global__ __launch_bounds__(256) void k_quad_check(CornerArgs a)
{
    TileSched ts(a.n_tiles, a.xcds, a.q.cnt);
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        const int64_t e = t * (int64_t)blockDim.x + threadIdx.x;
        const bool active = e < a.mesh.n;
        double2 p[4];
        bool bad = false;
        if (active) load_quad(a.mesh, e, p, bad);
        quad_element(a, e, active, p, bad);
    }
}

// Quadrangles stacked in rows (quad e + r has as corners 0, 1 the corners
// 3, 2 of quad e, r found by k_quad_walk_detect): each lane walks up its
// column of quads, in the tiles of WalkShape, and keeps the shared edge's two
// vertices in registers, so it loads 2 vertices per quad instead of 4.  The
// ids decide whether the kept edge is the quad's first one, so any
// connectivity gives the results of k_quad_check.
__global__ __launch_bounds__(256) void k_quad_walk(CornerArgs a)
{
    const MeshDev& m = a.mesh;
    const WalkShape ws(m.n, a.q.cnt, a.walk_limit, a.walk_layers);
    TileSched ts(ws.n_tiles, a.xcds, a.q.cnt);
    const int l = threadIdx.x;
    int k0 = -1, k1 = -1;         // ids of the kept edge
    double2 v0 = make_double2(0.0, 0.0), v1 = v0;
    for (int64_t t = ts.next_tile(); t >= 0; t = ts.next_tile()) {
        WalkPos pos;
        pos.start(ws, t);
        for (int r = 0; r < pos.left; ++r) {
            const int64_t e = pos.base + (int64_t)r * ws.s + l;
            const bool active = (int64_t)l < pos.cols && e < m.n;
            double2 p[4];
            if (active) {
                const int4 c = *reinterpret_cast<const int4*>(m.conn + 4 * e);
                const bool hit = c.x == k0 && c.y == k1;
                p[2] = *reinterpret_cast<const double2*>(m.points + 2 * (int64_t)c.z);
                p[3] = *reinterpret_cast<const double2*>(m.points + 2 * (int64_t)c.w);
                if (hit) {
                    p[0] = v0;
                    p[1] = v1;
                } else {
                    p[0] = *reinterpret_cast<const double2*>(m.points + 2 * (int64_t)c.x);
                    p[1] = *reinterpret_cast<const double2*>(m.points + 2 * (int64_t)c.y);
                }
                k0 = c.w;
                k1 = c.z;
                v0 = p[3];
                v1 = p[2];
            }
            quad_element(a, e, active, p, false);
        }
    }
}

__global__ __launch_bounds__(256) void k_quad_walk_detect(const int32_t* conn, int64_t limit, Counters* c)
{
    const int t0 = conn[3], t1 = conn[2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < limit; e += stride) {
        if ((int64_t)load_relaxed(&c->walk_code) > limit - e) return;
        const int32_t* b = conn + 4 * e;
        if (b[0] == t0 && b[1] == t1) atomicMax(&c->walk_code, (unsigned long long)(limit - e));
    }
}

__global__ __launch_bounds__(256) void k_quad_walk_extent(const int32_t* conn, int64_t n, int64_t limit, Counters* c)
{
    const unsigned long long code = c->walk_code;
    const int64_t s = code ? limit - (int64_t)code : 0;
    if (s < kWalkMinStride || s >= n) return;
    const int64_t nl = (n + s - 1) / s;
    for (int64_t l = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < nl; l += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* lo = conn + 4 * ((l - 1) * s);
        const int32_t* up = conn + 4 * (l * s);
        if (up[0] != lo[3] || up[1] != lo[2]) atomicMax(&c->walk_break, kWalkBreakBase - (unsigned long long)l);
    }
}

// The 4 points (8 doubles) of each listed element, for the exact tier.
__global__ void k_quad_gather(CornerArgs a, int64_t n, double* out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 p[4];
        bool bad = false;
        load_quad(a.mesh, a.q.exact_elem[i], p, bad);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            out[8 * i + 2 * k] = p[k].x;
            out[8 * i + 2 * k + 1] = p[k].y;
        }
    }
}

// mode 0: verdict (points: 24 doubles per entry), 1: corner-only test (24),
// 2: quadrangle (8).
__global__ __launch_bounds__(64) void k_exact_device(const double* pts, uint8_t* out, int64_t n, int mode,
                                                     int max_depth)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = mode == 2 ? exact_device_quad(pts + 8 * i) : exact_device_hex(pts + 24 * i, max_depth, mode == 1);
}

// Exact subdivision of the elements the device tier marked kExactSubdivide:
// lane l takes the elements l, l + lanes, ... with its path in `stack`
// ((max_depth + 1) * kExactDfsWords words per lane).
__global__ __launch_bounds__(64) void k_exact_dfs(const double* pts, uint8_t* out, int64_t n, int max_depth,
                                                  IW* stack, int64_t lanes)
{
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (lane >= lanes) return;
    IW* st = stack + lane * (int64_t)(max_depth + 1) * kExactDfsWords;
    for (int64_t i = lane; i < n; i += lanes)
        if (out[i] == kExactSubdivide) out[i] = exact_device_verdict(pts + 24 * i, max_depth, st);
}

// ------------------------------------------------------------ small kernels

__global__ void k_reset(Counters* c)
{
    unsigned long long* w = reinterpret_cast<unsigned long long*>(c);
    const int nw = (int)(sizeof(Counters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;
}

__global__ void k_tile_table(const MeshDev* meshes, int n_meshes, int tile, int32_t* tile_mesh)
{
    for (int mi = blockIdx.x; mi < n_meshes; mi += gridDim.x) {
        const MeshDev m = meshes[mi];
        const int64_t nt = (m.n + tile - 1) / tile;
        for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) tile_mesh[m.tile_begin + t] = mi;
    }
}

// Per mesh of a batch (one block each): the stack stride among the first
// n / 8 elements (so that at least 8 layers are walked), 1024 rows a step,
// and the first layer whose column 0 does not sit on the one below, as
// k_walk_detect and k_walk_extent find them for a single mesh.
__global__ __launch_bounds__(256) void k_batch_walk_detect(const MeshDev* meshes, int n_meshes, WalkMesh* wm)
{
    __shared__ unsigned long long found, brk;
    for (int mi = blockIdx.x; mi < n_meshes; mi += gridDim.x) {
        const MeshDev m = meshes[mi];
        int64_t s = 0, nl = 0;
        if (m.conn && m.n >= 8 * kWalkMinStride) {           // the same in every thread of the block
            const int32_t* conn = m.conn;
            const int t0 = conn[4], t1 = conn[5], t2 = conn[6], t3 = conn[7];
            const int64_t limit = m.n / 8 + 1 < kWalkSearch ? m.n / 8 + 1 : kWalkSearch;
            if (threadIdx.x == 0) found = (unsigned long long)limit;
            __syncthreads();
            for (int64_t e0 = 1; e0 < limit; e0 += 4 * blockDim.x) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t e = e0 + k * (int64_t)blockDim.x + threadIdx.x;
                    if (e < limit) {
                        const int32_t* b = conn + 8 * e;
                        if (b[0] == t0 && b[1] == t1 && b[2] == t2 && b[3] == t3)
                            atomicMin(&found, (unsigned long long)e);
                    }
                }
                __syncthreads();
                const bool done = found < (unsigned long long)limit;
                __syncthreads();
                if (done) break;
            }
            s = (int64_t)found;
            if (s >= kWalkMinStride && s < limit) {
                const int64_t all = (m.n + s - 1) / s;
                if (threadIdx.x == 0) brk = (unsigned long long)all;
                __syncthreads();
                for (int64_t l0 = 1; l0 < all; l0 += blockDim.x) {
                    const int64_t l = l0 + threadIdx.x;
                    if (l < all) {
                        const int32_t* lo = conn + 8 * ((l - 1) * s);
                        const int32_t* up = conn + 8 * (l * s);
                        if (up[0] != lo[4] || up[1] != lo[5] || up[2] != lo[6] || up[3] != lo[7])
                            atomicMin(&brk, (unsigned long long)l);
                    }
                    __syncthreads();
                    const bool done = brk < (unsigned long long)all;
                    __syncthreads();
                    if (done) break;
                }
                nl = (int64_t)brk;
            } else {
                s = 0;
            }
        }
        if (threadIdx.x == 0) {
            wm[mi].s = s;
            wm[mi].nl = nl;
        }
        __syncthreads();   // found and brk are set again for the next mesh
    }
}

// One block of 1024 threads: each mesh's tile count in the walking pass
// (plain tiles where walking would take more tiles than plain ones), their
// exclusive prefix sums as the meshes' first tiles, and the total.
__global__ __launch_bounds__(1024) void k_batch_walk_tiles(const MeshDev* meshes, int n_meshes, int block,
                                                           int layers, WalkMesh* wm, Counters* c)
{
    __shared__ int64_t part[1024];
    const int per = (n_meshes + (int)blockDim.x - 1) / (int)blockDim.x;
    const int m0 = (int)threadIdx.x * per;
    const int m1 = m0 + per < n_meshes ? m0 + per : n_meshes;
    int64_t sum = 0;
    for (int mi = m0; mi < m1; ++mi) {
        const int64_t n = meshes[mi].n;
        WalkShape ws;
        ws.init(n, wm[mi].s, wm[mi].nl, layers, block);
        const int64_t plain = (n + block - 1) / block;
        int64_t nt = ws.n_tiles;
        if (ws.nl == 0 || nt > plain) {
            wm[mi].s = 0;
            wm[mi].nl = 0;
            nt = plain;
        }
        wm[mi].n_tiles = nt;
        sum += nt;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {   // inclusive scan
        const int64_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t begin = part[threadIdx.x] - sum;
    for (int mi = m0; mi < m1; ++mi) {
        wm[mi].tile_begin = begin;
        begin += wm[mi].n_tiles;
    }
    if (threadIdx.x == blockDim.x - 1) c->walk_tiles = (unsigned long long)part[threadIdx.x];
}

__global__ void k_batch_walk_table(int n_meshes, const WalkMesh* wm, int32_t* tile_mesh)
{
    for (int mi = blockIdx.x; mi < n_meshes; mi += gridDim.x) {
        const int64_t b = wm[mi].tile_begin, nt = wm[mi].n_tiles;
        for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) tile_mesh[b + t] = mi;
    }
}

__global__ __launch_bounds__(256) void k_collect_deferred(CollectArgs a)
{
    for (int mi = 0; mi < a.n_meshes; ++mi) {
        const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m.n;
             e += (int64_t)gridDim.x * blockDim.x) {
            const bool d = m.verdict[e] == kDeferred;
            const uint64_t mask = ballot(d);
            if (mask) {
                const unsigned long long s = wave_reserve(&a.q.cnt->n_list, mask);
                if (d && s < a.q.list_cap) {
                    a.q.list_elem[s] = e;
                    a.q.list_mesh[s] = mi;
                }
            }
        }
    }
}

__global__ void k_gather_exact(GatherArgs a)
{
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int mi = a.q.exact_mesh[i];
        const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
        V3 p[8];
        bool bad = false;
        load_points(m, a.q.exact_elem[i], p, bad);
        double* o = a.out + 24 * i;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            o[3 * k] = p[k].x;
            o[3 * k + 1] = p[k].y;
            o[3 * k + 2] = p[k].z;
        }
    }
}

__global__ void k_scatter_exact(ScatterArgs a)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int mi = a.q.exact_mesh[i];
        const MeshDev m = a.meshes ? a.meshes[mi] : a.mesh;
        const int64_t e = a.q.exact_elem[i];
        const uint8_t v = a.verdicts[i];
        m.verdict[e] = v;
        if (v == 3 && m.min_coeff) m.min_coeff[e] = __builtin_nan("");
    }
}

__global__ __launch_bounds__(256) void k_coefficients(MeshDev m, double* out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m.n;
         e += (int64_t)gridDim.x * blockDim.x) {
        V3 p[8];
        bool bad = false;
        load_points(m, e, p, bad);
        ElementValues r;
        element_values(p, r);
#pragma unroll
        for (int a = 0; a < 27; ++a) out[27 * e + a] = coefficient(r, a);
    }
}

// ------------------------------------------------------------ launchers

#define HX_LAUNCH(kernel, grid, block, stream, ...) \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__)

void launch_top_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s)
{
    const bool edges = a.max_depth == 0;
    if (batched) {
        if (a.batch_conn && a.walk_layers && edges) HX_LAUNCH((k_top_f64_batch_walk<true>), grid, block, s, a);
        else if (a.batch_conn && a.walk_layers) HX_LAUNCH((k_top_f64_batch_walk<false>), grid, block, s, a);
        else if (a.batch_conn && edges) HX_LAUNCH((k_top_f64_batch_conn<true>), grid, block, s, a);
        else if (a.batch_conn) HX_LAUNCH((k_top_f64_batch_conn<false>), grid, block, s, a);
        else if (edges) HX_LAUNCH((k_top_f64_range<true, true, kGatherAny>), grid, block, s, a);
        else HX_LAUNCH((k_top_f64_range<true, false, kGatherAny>), grid, block, s, a);
        return;
    }
    const int g = !a.mesh.conn ? kGatherPoints : a.mesh.validate ? kGatherChecked : kGatherConn;
#define HX_TOP(E, G) HX_LAUNCH((k_top_f64_range<false, E, G>), grid, block, s, a)
    if (edges) {
        if (g == kGatherPoints) HX_TOP(true, kGatherPoints);
        else if (g == kGatherConn && a.walk_layers) HX_LAUNCH((k_top_f64_walk<true>), grid, block, s, a);
        else if (g == kGatherConn) HX_LAUNCH((k_top_f64_conn<true>), grid, block, s, a);
        else HX_TOP(true, kGatherChecked);
    } else {
        if (g == kGatherPoints) HX_TOP(false, kGatherPoints);
        else if (g == kGatherConn && a.walk_layers) HX_LAUNCH((k_top_f64_walk<false>), grid, block, s, a);
        else if (g == kGatherConn) HX_LAUNCH((k_top_f64_conn<false>), grid, block, s, a);
        else HX_TOP(false, kGatherChecked);
    }
#undef HX_TOP
}

void launch_filter_range(const TopArgs& a, bool batched, int grid, int block, hipStream_t s)
{
    if (batched) {
        if (a.batch_conn) HX_LAUNCH(k_filter_f32_batch_conn, grid, block, s, a);
        else HX_LAUNCH((k_filter_f32_range<true, kGatherAny>), grid, block, s, a);
        return;
    }
    if (!a.mesh.conn) HX_LAUNCH((k_filter_f32_range<false, kGatherPoints>), grid, block, s, a);
    else if (a.mesh.validate) HX_LAUNCH((k_filter_f32_range<false, kGatherChecked>), grid, block, s, a);
    else if (a.walk_layers && a.max_depth == 0) HX_LAUNCH(k_filter_f32_walk<true>, grid, block, s, a);
    else if (a.walk_layers) HX_LAUNCH(k_filter_f32_walk<false>, grid, block, s, a);
    else HX_LAUNCH(k_filter_f32_conn, grid, block, s, a);
}

void launch_top_list(const TopArgs& a, bool batched, int grid, int block, hipStream_t s)
{
    const bool edges = a.max_depth == 0;
    if (batched && edges) HX_LAUNCH((k_top_f64_list<true, true>), grid, block, s, a);
    else if (batched) HX_LAUNCH((k_top_f64_list<true, false>), grid, block, s, a);
    else if (edges) HX_LAUNCH((k_top_f64_list<false, true>), grid, block, s, a);
    else HX_LAUNCH((k_top_f64_list<false, false>), grid, block, s, a);
}

void launch_level(const LevelArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_level, grid, 256, s, a); }
void launch_roots(const RootArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_roots, grid, 256, s, a); }
void launch_fold(const FoldArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_fold, grid, 256, s, a); }
void launch_reset(Counters* c, hipStream_t s) { HX_LAUNCH(k_reset, 1, 64, s, c); }
void launch_walk_detect(const int32_t* conn, int64_t n, int64_t limit, Counters* c, hipStream_t s)
{
    const int64_t g = (limit + 255) / 256;
    HX_LAUNCH(k_walk_detect, g < 1024 ? g : 1024, 256, s, conn, limit, c);
    HX_LAUNCH(k_walk_extent, 64, 256, s, conn, n, limit, c);
}
void launch_batch_walk(const MeshDev* meshes, int n_meshes, int block, int layers, WalkMesh* wm,
                       int32_t* tile_mesh, Counters* c, hipStream_t s)
{
    const int g = n_meshes < 4096 ? n_meshes : 4096;
    HX_LAUNCH(k_batch_walk_detect, g, 256, s, meshes, n_meshes, wm);
    HX_LAUNCH(k_batch_walk_tiles, 1, 1024, s, meshes, n_meshes, block, layers, wm, c);
    HX_LAUNCH(k_batch_walk_table, g, 256, s, n_meshes, wm, tile_mesh);
}
void launch_tile_table(const MeshDev* meshes, int n_meshes, int tile, int32_t* tile_mesh, hipStream_t s)
{
    HX_LAUNCH(k_tile_table, n_meshes < 4096 ? n_meshes : 4096, 256, s, meshes, n_meshes, tile, tile_mesh);
}
void launch_collect_deferred(const CollectArgs& a, int grid, hipStream_t s)
{
    HX_LAUNCH(k_collect_deferred, grid, 256, s, a);
}
void launch_exact_dfs(const double* pts, uint8_t* out, int64_t n, int max_depth, void* stack, int64_t lanes,
                      hipStream_t s)
{
    const int64_t g = (lanes + 63) / 64;
    HX_LAUNCH(k_exact_dfs, g < 1024 ? g : 1024, 64, s, pts, out, n, max_depth, (IW*)stack,
              lanes < 1024 * 64 ? lanes : 1024 * 64);
}
void launch_dfs(const DfsArgs& a, hipStream_t s)
{
    const int64_t g = (a.lanes + 63) / 64;
    HX_LAUNCH(k_dfs, g < 4096 ? g : 4096, 64, s, a);
}
void launch_gather_exact(const GatherArgs& a, hipStream_t s)
{
    const int64_t g = (a.n + 255) / 256;
    HX_LAUNCH(k_gather_exact, g < 1024 ? g : 1024, 256, s, a);
}
void launch_scatter_exact(const ScatterArgs& a, hipStream_t s)
{
    const int64_t g = (a.n + 255) / 256;
    HX_LAUNCH(k_scatter_exact, g < 1024 ? g : 1024, 256, s, a);
}
void launch_corner_test(const CornerArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_corner_test, grid, 256, s, a); }
void launch_corner_collect(const CornerArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_corner_collect, grid, 256, s, a); }
// (The quadrangle kernel needs about 50 registers, so occupancy already
// hides its gather latency; the prefetching loop measured slower for it.)
void launch_quad_check(const CornerArgs& a, int grid, hipStream_t s)
{
    if (a.walk_layers) HX_LAUNCH(k_quad_walk, grid, 256, s, a);
    else HX_LAUNCH(k_quad_check, grid, 256, s, a);
}
void launch_quad_walk_detect(const int32_t* conn, int64_t n, int64_t limit, Counters* c, hipStream_t s)
{
    const int64_t g = (limit + 255) / 256;
    HX_LAUNCH(k_quad_walk_detect, g < 1024 ? g : 1024, 256, s, conn, limit, c);
    HX_LAUNCH(k_quad_walk_extent, 64, 256, s, conn, n, limit, c);
}
void launch_quad_gather(const CornerArgs& a, int64_t n, double* out, hipStream_t s)
{
    const int64_t g = (n + 255) / 256;
    HX_LAUNCH(k_quad_gather, g < 4096 ? g : 4096, 256, s, a, n, out);
}
void launch_minj_top(const MinjArgs& a, int grid, hipStream_t s)
{
    if (!a.in_list && a.mesh.conn && !a.mesh.validate && a.walk_layers) HX_LAUNCH(k_minj_top_walk, grid, 256, s, a);
    else if (!a.in_list && a.mesh.conn && !a.mesh.validate) HX_LAUNCH(k_minj_top_conn, grid, 256, s, a);
    else HX_LAUNCH(k_minj_top, grid, 256, s, a);
}
void launch_minj_roots(const MinjArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_minj_roots, grid, 256, s, a); }
void launch_minj_level(const MinjArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_minj_level, grid, 256, s, a); }
void launch_minj_fold(const MinjArgs& a, int grid, hipStream_t s) { HX_LAUNCH(k_minj_fold, grid, 256, s, a); }

void launch_exact_device(const double* pts, uint8_t* out, int64_t n, int mode, int max_depth, hipStream_t s)
{
    const int64_t g = (n + 63) / 64;
    HX_LAUNCH(k_exact_device, g < 1024 ? g : 1024, 64, s, pts, out, n, mode, max_depth);
}

void launch_coefficients(const MeshDev& m, double* out, hipStream_t s)
{
    const int64_t g = (m.n + 255) / 256;
    HX_LAUNCH(k_coefficients, g < 65536 ? g : 65536, 256, s, m, out);
}

}  // namespace hexval
