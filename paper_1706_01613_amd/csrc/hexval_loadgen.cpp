// Open-loop request generator for the hexval server (benchmark and test
// driver; uses only the public C ABI of libhexval).
//
// Requests are submitted at prescribed arrival times (a Poisson stream drawn
// by the caller), whatever the state of the server, and their completions are
// polled; the latency of a request is the server's submit-to-completion wall
// time.  Each request owns its outputs, carved sequentially from a caller
// provided device arena (verdicts, then min coefficients 8-byte aligned).
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <thread>
#include <vector>

#include "hexval.h"

extern "C" {

/* sv: server.  n requests; arrival_s[i] (non-decreasing, seconds after the
 * call starts) and mesh_idx[i] into pool[n_pool] (request templates: mesh and
 * optional host copies; their output fields are ignored).  arena: device
 * memory of arena_bytes for the outputs; want_min: also return min
 * coefficients.  Outputs per request: latency_ms[i], status[i],
 * out_offset[i] (byte offset of its verdicts in the arena; min coefficients
 * follow at the next multiple of 8).  *wall_s: first submit to last
 * completion.  Returns HEXVAL_OK, or HEXVAL_E_NOMEM when the arena is too
 * small (nothing is submitted then). */
int hexval_loadgen_run(hexval_server_t* sv, int64_t n, const double* arrival_s, const int32_t* mesh_idx,
                       const hexval_request_t* pool, int32_t n_pool, uint8_t* arena, int64_t arena_bytes,
                       int32_t want_min, double* latency_ms, int32_t* status, int64_t* out_offset,
                       double* wall_s)
{
    if (!sv || n < 0 || !pool || n_pool <= 0) return HEXVAL_E_ARG;
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (mesh_idx[i] < 0 || mesh_idx[i] >= n_pool) return HEXVAL_E_ARG;
        const int64_t m = pool[mesh_idx[i]].mesh.n;
        out_offset[i] = off;
        off += (m + 7) / 8 * 8;
        if (want_min) off += 8 * m;
        off = (off + 255) / 256 * 256;
    }
    if (off > arena_bytes) return HEXVAL_E_NOMEM;
    using Clock = std::chrono::steady_clock;
    const Clock::time_point t0 = Clock::now();
    std::vector<uint64_t> ticket(n);
    std::vector<int64_t> open;
    open.reserve(n);
    int64_t next = 0, done = 0;
    double last_done = 0.0;
    while (done < n) {
        const double now = std::chrono::duration<double>(Clock::now() - t0).count();
        while (next < n && arrival_s[next] <= now) {
            hexval_request_t r = pool[mesh_idx[next]];
            r.verdicts = arena + out_offset[next];
            r.min_coeffs = want_min ? reinterpret_cast<double*>(
                                          arena + out_offset[next] + (r.mesh.n + 7) / 8 * 8)
                                    : nullptr;
            const int st = hexval_server_submit(sv, &r, &ticket[next]);
            if (st != HEXVAL_OK) {
                status[next] = st;
                latency_ms[next] = 0.0;
                ++done;
            } else {
                open.push_back(next);
            }
            ++next;
        }
        bool progressed = false;
        for (size_t k = 0; k < open.size();) {
            const int64_t i = open[k];
            int fin = 0;
            double lat = 0.0;
            const int st = hexval_server_poll(sv, ticket[i], &fin, &lat);
            if (fin) {
                status[i] = st;
                latency_ms[i] = lat;
                ++done;
                progressed = true;
                last_done = std::chrono::duration<double>(Clock::now() - t0).count();
                open[k] = open.back();
                open.pop_back();
            } else {
                ++k;
            }
        }
        if (!progressed && (next >= n || arrival_s[next] > now + 20e-6))
            std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
    if (wall_s) *wall_s = last_done - (n ? arrival_s[0] : 0.0);
    return HEXVAL_OK;
}
}
