/*
 * hexval.h: C ABI of libhexval, a validity test for linear hexahedra on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: A. Johnen, J.-C. Weill, J.-F. Remacle, "Robust and efficient
 * validation of the linear hexahedral element", IMR 2017.  For each element
 * the 8 corner points (Appendix A order: (0,0,0) (1,0,0) (1,1,0) (0,1,0)
 * (0,0,1) (1,0,1) (1,1,1) (0,1,1) of the reference cube [0,1]^3) give the 20
 * values of the Jacobian determinant at the corners and edge midpoints as
 * triple products (Section 5); the fixed 27x20 matrix of Table 3 maps them to
 * the 27 Bezier coefficients of the triquadratic determinant (Sections 3-4);
 * the algorithm of Section 6 then decides: a non-positive value -> INVALID,
 * all coefficients b_9..b_27 positive -> VALID, otherwise the element is
 * subdivided adaptively.
 *
 * Semantics fixed by this library (where the paper is silent):
 *   - validity is strict positivity of J on [0,1]^3: a value <= 0 is invalid,
 *     only values > 0 certify;
 *   - subdivision stops at a depth cap (default 6): an element with an
 *     ambiguous sub-box at the cap and no non-positive value found is
 *     UNDECIDED;
 *   - verdicts are those of the algorithm in EXACT arithmetic: every FP64
 *     (or FP32) sign decision is checked against a rigorous error bound and
 *     the few elements whose decisions cannot be certified are recomputed in
 *     integer arithmetic, subdivision included, on the device (on host
 *     threads for coordinates spanning more than 78 bits);
 *   - min_coeff is the minimum of the 27 top-level coefficients (a lower
 *     bound of min J by the convex-hull property of Section 3.1), NaN for
 *     BAD_INPUT.  Computed in FP64 it is within 256 u M^ of the exact
 *     minimum (u = 2^-53, M^ = 6 S_xi S_eta S_zeta, S_d the largest |component|
 *     of the element's four edge vectors along direction d); under
 *     HEXVAL_FP32_FILTER an element the FP32 pass decides, or sends to
 *     subdivision itself (every corner value above twice its FP32 bound and
 *     some coefficient certainly negative), returns the FP32 minimum widened
 *     to double, within 256 u32 M^ (u32 = 2^-24), and an element rechecked
 *     in FP64 returns the FP64 value.
 *
 * Conventions for every entry point:
 *   - array pointers named "device" are device pointers (hipMalloc'd memory or
 *     ROCm torch tensors) on the current HIP device; the caller owns all
 *     buffers it passes and the library never frees them;
 *   - status codes are returned, nothing is thrown across the ABI; the message
 *     of the last non-OK status of the calling thread is hexval_last_error();
 *   - n == 0 is a no-op returning HEXVAL_OK; a NULL required pointer with
 *     n > 0, n < 0 or an option out of range returns HEXVAL_E_ARG without
 *     touching the GPU;
 *   - per-element input problems never fail a call: the element gets verdict
 *     HEXVAL_BAD_INPUT;
 *   - entry points may be called from several host threads at once: each
 *     call takes its own workspace from a pool, and calls on one stream run
 *     in order.
 */
#ifndef HEXVAL_H
#define HEXVAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-element verdicts (uint8). */
enum {
    HEXVAL_INVALID = 0,   /* J <= 0 somewhere on [0,1]^3 (a value <= 0 was found) */
    HEXVAL_VALID = 1,     /* J > 0 on [0,1]^3 (all coefficients of a cover positive) */
    HEXVAL_UNDECIDED = 2, /* depth cap reached with no non-positive value found */
    HEXVAL_BAD_INPUT = 3  /* non-finite coordinate, or index out of range when validated */
};

/* Status codes. */
enum {
    HEXVAL_OK = 0,
    HEXVAL_E_ARG = 1,   /* invalid argument (see conventions) */
    HEXVAL_E_HIP = 2,   /* HIP runtime error, no usable gfx950 device, or kernel failure */
    HEXVAL_E_NOMEM = 3, /* device or host allocation failed */
    HEXVAL_E_QUEUE = 4, /* the subdivision queue cannot hold one element's tree */
    HEXVAL_E_BUSY = 5   /* server: one request's uploads alone exceed what the budget leaves */
};

/* Precision of the first pass. */
enum {
    HEXVAL_FP64 = 0,        /* every element in FP64 */
    HEXVAL_FP32_FILTER = 1  /* FP32 pass with a forward error bound per value and
                               coefficient; elements it cannot certify, and every
                               subdivision, are recomputed in FP64.  Verdicts are
                               those of HEXVAL_FP64; min_coeff of an element the
                               FP32 pass decides or sends to subdivision is
                               FP32-accurate (within 256 u32 M^, see min_coeff
                               above) */
};

/* A mesh.  points: device, [n_points,3] float64 when connectivity != NULL,
 * else [n,8,3] float64 (8 points per element, Appendix A order).
 * connectivity: device, [n,8] int32 vertex ids (Appendix A order) or NULL.
 * n_points: number of vertices; used only to validate indices. */
typedef struct {
    const double* points;
    int64_t n_points;
    const int32_t* connectivity;
    int64_t n;
} hexval_mesh_t;

/* Counters and device timings of one call (filled when opts->stats != NULL). */
typedef struct {
    int64_t n_elements;    /* elements checked */
    int64_t n_subdivided;  /* elements sent to subdivision */
    int64_t n_nodes;       /* sub-boxes evaluated by the subdivision kernel */
    int64_t n_exact;       /* elements settled by the exact tier (device, else host) */
    int64_t n_recheck;     /* FP32_FILTER: elements recomputed in FP64 */
    int64_t n_rounds;      /* passes (more than 1 only after queue overflow) */
    int32_t max_level;     /* deepest sub-box level evaluated */
    int32_t timing;        /* IN: nonzero -> record the device times below */
    float ms_first_pass;   /* device time of the first-pass kernel (FP64 or FP32) */
    float ms_recheck;      /* device time of the FP64 recheck kernel (FP32_FILTER) */
    float ms_subdivision;  /* device time of subdivision drain + verdict fold */
    float ms_total;        /* device time from first launch to last kernel */
    int32_t block_threads; /* first-pass block size used (tuned or given) */
    int32_t n_exact_host;  /* of n_exact: elements the device exact tier left to
                              the host (a coordinate span over 78 bits, or a
                              subdivision store too small for one path) */
    int64_t grid_blocks;   /* first-pass grid used */
    int32_t walk_layers;   /* layers per column tile of the first pass (0: plain
                              tiles) */
    int32_t reserved;
    int64_t walk_stride;   /* single mesh: stack stride found for the column
                              walk (0: none; batches report 0) */
} hexval_stats_t;

/* Options.  Use hexval_opts_default() and change fields. */
typedef struct {
    int32_t precision;        /* HEXVAL_FP64 (default) or HEXVAL_FP32_FILTER */
    int32_t max_depth;        /* subdivision depth cap, 0..20, default 6 */
    int32_t validate_indices; /* nonzero: connectivity entries outside [0,n_points)
                                 give BAD_INPUT (default 0: indices are trusted) */
    int32_t block_threads;    /* first-pass block size: 0 = tuned, else 64..256,
                                 a multiple of 64 */
    int64_t queue_capacity;   /* subdivision queue nodes, 0 = automatic.  Elements
                                 that do not fit are checked in later rounds,
                                 fewer at a time when a round completes none */
    int64_t grid_blocks;      /* first-pass grid: 0 = tuned, else blocks (rounded up
                                 to a multiple of 8) */
    void* stream;             /* hipStream_t to run on; NULL = the null stream */
    hexval_stats_t* stats;    /* optional output */
    int32_t walk_layers;      /* trusted connectivity (a single mesh, or an
                                 FP64 batch whose meshes all have it): the first
                                 pass checks columns of elements stacked with
                                 the stride it finds per mesh (element e + s
                                 has as corners 0..3 the corners 4..7 of
                                 element e), loading each shared face once;
                                 this many layers per column tile.  Meshes
                                 under 32768 elements, or with a stride under
                                 4096 or fewer than 8 layers of it in a batch,
                                 take plain tiles.  0 = tuned (default), -1 =
                                 plain tiles, 1..64 = this many.  The same for
                                 the rows of a quadrangle mesh with trusted
                                 connectivity (quad e + s has as corners 0, 1
                                 the corners 3, 2 of quad e; 0 = 16 rows).
                                 Results never depend on it */
    int32_t reserved;         /* must be 0 */
} hexval_opts_t;

/* Fills *opts with the defaults above. */
void hexval_opts_default(hexval_opts_t* opts);

/*
 * hexval_check: the Section 6 algorithm for n elements, FP64, default options,
 * on the null stream; returns when the outputs are final.
 * points: device [n,8,3] float64 when connectivity is NULL, else the vertex
 *   array [*,3] float64 indexed by connectivity (device [n,8] int32; indices
 *   are trusted).
 * verdicts: device [n] uint8 (HEXVAL_INVALID .. HEXVAL_BAD_INPUT).
 * min_coeffs: device [n] float64, or NULL.
 */
int hexval_check(const double* points, const int32_t* connectivity, int64_t n,
                 uint8_t* verdicts, double* min_coeffs);

/*
 * hexval_check_ex: as hexval_check with options (precision, depth cap, index
 * validation, stream, tuning, statistics).  Work is enqueued on opts->stream
 * (NULL opts = defaults); the call returns when the outputs are final.
 */
int hexval_check_ex(const hexval_mesh_t* mesh, const hexval_opts_t* opts,
                    uint8_t* verdicts, double* min_coeffs);

/*
 * hexval_check_batched: n_meshes independent meshes of different sizes in one
 * persistent launch (elements of all meshes share the grid and one
 * subdivision queue).  meshes: host array [n_meshes]; verdicts and min_coeffs:
 * host arrays [n_meshes] of device pointers (min_coeffs may be NULL, or hold
 * NULL entries).  Results equal those of hexval_check_ex on each mesh alone.
 */
int hexval_check_batched(const hexval_mesh_t* meshes, int32_t n_meshes,
                         const hexval_opts_t* opts, uint8_t* const* verdicts,
                         double* const* min_coeffs);

/*
 * hexval_coefficients: the 27 top-level Bezier coefficients of every element
 * (Table 3 applied to the 20 triple-product values, FP64), Fig. 3 order.
 * coeffs: device [n,27] float64.  stream: hipStream_t or NULL.  Returns after
 * the kernel has completed.
 */
int hexval_coefficients(const hexval_mesh_t* mesh, void* stream, double* coeffs);

/*
 * hexval_check_noalloc: hexval_check_ex for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It allocates no device or pinned host memory: its
 * subdivision store, check lists, counters and exact-tier staging live in a
 * fixed array of the library (about 38 MiB of device memory per GPU it runs
 * on, held until the process ends) and in fixed host arrays.  The caller
 * passes inputs and outputs as for hexval_check_ex; the results are the same.
 * Limits: max_depth <= 8 and queue_capacity <= 2^17 (else HEXVAL_E_ARG);
 * devices 0..15; timing statistics are not recorded (stats->ms_* stay 0).
 * Elements beyond the fixed capacities are checked in later rounds.  The
 * host exact tier, reached only for elements whose exact decision the device
 * tier cannot settle, uses ordinary host memory.  Every call on one GPU uses
 * that GPU's single copy of the array and leaves its contents behind: calls
 * that overlap on one GPU (from several host threads or on several streams)
 * race and must be serialised by the caller.
 */
int hexval_check_noalloc(const hexval_mesh_t* mesh, const hexval_opts_t* opts,
                         uint8_t* verdicts, double* min_coeffs);

/* ---- corner-only test and corner quality ------------------------------------
 * hexval_corner_test: Test 1 of the comparison in Section 7 (the volumes of
 * the 8 corner tetrahedra, i.e. the 8 corner values of J = the corner
 * coefficients b_1..b_8, must all be positive) and the corner quality quoted
 * for Fig. 7 (minimum over the corners of the scaled Jacobian
 * J_c / (|e_xi| |e_eta| |e_zeta|), e_* the three edge vectors leaving corner
 * c; a corner with a zero-length edge counts as 0).  The test is a necessary
 * condition of validity: it can pass invalid elements ("false valid"), never
 * fail valid ones; comparing it with hexval_check counts what the Bezier test
 * adds.  Signs are exact (certified FP64, else integer arithmetic).
 * mesh: as for hexval_check_ex.  opts: validate_indices, stream, stats (NULL =
 *   defaults; precision and depth are not used).
 * test1: device [n] uint8: HEXVAL_VALID (all 8 corner values > 0),
 *   HEXVAL_INVALID, HEXVAL_BAD_INPUT.
 * quality: device [n] float64 or NULL; NaN for BAD_INPUT and for elements
 *   whose per-direction edge scales leave [2^-300, 2^300].
 * Returns when the outputs are final.
 */
int hexval_corner_test(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* test1,
                       double* quality);

/* ---- linear quadrangles -------------------------------------------------------
 * hexval_quad_check: validity of linear quadrangles (Section 2.1).  The map of
 * [0,1]^2 is bilinear, so is J, and its minimum over the element is one of
 * the four corner values; the element is VALID when all four are > 0 and
 * INVALID otherwise (same strict reading as for hexahedra).  Signs are exact
 * (certified FP64, else integer arithmetic).
 * mesh: points device float64, [n,4,2] when connectivity is NULL, else
 *   [n_points,2] with connectivity device [n,4] int32; corners in the order
 *   (0,0) (1,0) (1,1) (0,1) of the reference square (counter-clockwise for a
 *   valid element in a right-handed plane); rows 16-byte aligned.
 * opts: validate_indices, walk_layers, stream, stats (NULL = defaults).
 * verdicts: device [n] uint8 (HEXVAL_INVALID, HEXVAL_VALID, HEXVAL_BAD_INPUT).
 * min_j: device [n] float64 or NULL: min J = the smallest corner value
 *   (FP64; NaN for BAD_INPUT).
 * Returns when the outputs are final.
 */
int hexval_quad_check(const hexval_mesh_t* mesh, const hexval_opts_t* opts, uint8_t* verdicts,
                      double* min_j);

/* ---- minimum of the Jacobian determinant to a tolerance --------------------
 * The bounds of Section 3.1, sharpened by subdivision (the method the
 * introduction recalls, which computes min J to any prescribed tolerance): on
 * a box, the smallest of its 27 Bezier coefficients is a lower bound of J
 * (convex hull property) and each corner coefficient is a value of J.  Boxes
 * are refined level by level: a box of level L is kept as final when its
 * lower bound is within tol of the smallest corner value found on levels
 * 0..L, else split in 8 until the depth cap.  tol = rtol * S_xi S_eta S_zeta,
 * S_d the largest |component| of the element's edge vectors along direction
 * d (for an undistorted cube of edge h, tol = rtol h^3 = rtol J).  The result
 * does not depend on the order in which boxes are processed. */

/* Per-element status of hexval_min_jacobian (uint8). */
enum {
    HEXVAL_MINJ_CONVERGED = 0,    /* hi - lo <= tol (+ the error margins) */
    HEXVAL_MINJ_DEPTH_CAP = 1,    /* opts->max_depth reached first: lo <= min J <= hi still holds */
    HEXVAL_MINJ_QUEUE_FULL = 2,   /* box storage ran out: lo <= min J <= hi still holds */
    HEXVAL_MINJ_BAD_INPUT = 3,    /* non-finite coordinate or (validated) index out of range: lo = hi = NaN */
    HEXVAL_MINJ_OUT_OF_RANGE = 4  /* an S_d outside [2^-300, 2^300]: lo = hi = NaN */
};

/*
 * hexval_min_jacobian: certified bounds lo[e] <= min over [0,1]^3 of J <= hi[e]
 * for every element (FP64; both are widened by a rigorous rounding-error bound
 * and rounded outwards).
 * mesh: as for hexval_check_ex.  opts: max_depth (default 6), validate_indices,
 *   queue_capacity (stored boxes; 0 = max(n, 2^19) rounded up to a power of 2,
 *   at most 2^26), stream, stats; precision must be HEXVAL_FP64.  NULL = defaults.
 * rtol: relative tolerance, finite and > 0 (see tol above).
 * lo, hi: device [n] float64.  status: device [n] uint8 (HEXVAL_MINJ_*) or NULL.
 * Returns when the outputs are final.  With a full box store the elements
 * concerned report HEXVAL_MINJ_QUEUE_FULL and which ones they are may vary
 * from run to run; otherwise the outputs are deterministic.
 */
int hexval_min_jacobian(const hexval_mesh_t* mesh, const hexval_opts_t* opts, double rtol,
                        double* lo, double* hi, uint8_t* status);

/* ---- request queue with continuous batching --------------------------------
 * A server runs max_slots worker threads, each with its own HIP stream.  A
 * free worker admits the oldest submitted request if its device footprint
 * fits the HBM budget; when that request is device-resident, the
 * device-resident requests queued right behind it (up to 64 requests and
 * 2^24 elements in all) join it in one batched call.  Admitted work runs
 * concurrently on the workers' streams.  Outputs never depend on how
 * requests were grouped.  A request whose mesh pointers are device pointers
 * references that memory (the caller keeps it alive until the request is
 * done); with host_points/host_conn set the worker copies the mesh to the
 * device itself, on its stream, into an upload buffer that it keeps between
 * requests (the host copies, too, stay alive until the request is done).  That buffer counts against the budget while the worker holds
 * it; a free worker gives its buffer back when the oldest waiting request
 * does not fit. */
typedef struct hexval_server hexval_server_t;

typedef struct {
    hexval_mesh_t mesh;        /* device mesh, or sizes only when host_* are set */
    const double* host_points; /* optional host copy of mesh.points */
    const int32_t* host_conn;  /* optional host copy of mesh.connectivity */
    uint8_t* verdicts;         /* device [n] */
    double* min_coeffs;        /* device [n] or NULL */
} hexval_request_t;

/* opts: precision, max_depth, validate_indices apply to every request (stream and
 * stats are ignored).  hbm_budget_bytes: device memory the server may hold
 * (the workers' workspaces, allocated at creation, plus their upload
 * buffers), > 0; HEXVAL_E_ARG when the workspaces alone exceed it.
 * max_slots: 1..64. */
int hexval_server_create(const hexval_opts_t* opts, int64_t hbm_budget_bytes, int32_t max_slots,
                         hexval_server_t** server);
/* Never blocks on the GPU.  *ticket identifies the request.  Returns
 * HEXVAL_E_BUSY only if one request alone can never fit the budget. */
int hexval_server_submit(hexval_server_t* server, const hexval_request_t* request,
                         uint64_t* ticket);
/* *done = 1 once the outputs of ticket are final; latency_ms (optional) =
 * submit-to-completion wall time.  The status of the finished request is the
 * return value once done.  A ticket is forgotten once poll has reported it
 * done or wait has returned it (and no other thread still waits on it):
 * later calls with it return HEXVAL_E_ARG. */
int hexval_server_poll(hexval_server_t* server, uint64_t ticket, int* done, double* latency_ms);
/* Blocks until ticket is done; returns its status. */
int hexval_server_wait(hexval_server_t* server, uint64_t ticket, double* latency_ms);
/* Waits for all requests, stops the scheduler, frees the server's memory.
 * No other call on this server may run during or after it. */
int hexval_server_destroy(hexval_server_t* server);

/* Message of the last non-OK status returned to the calling thread. */
const char* hexval_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HEXVAL_H */
