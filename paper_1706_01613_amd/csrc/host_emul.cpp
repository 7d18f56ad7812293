// CPU replay of the kernels' per-element arithmetic, for tests only (built
// as libhexval_emul.so, never loaded by the library or its binding).
//
// It runs the same operations as the HIP kernels (hexval_math.hpp: identical
// IEEE roundings, explicit fma) in a sequential version of the pipeline:
// first pass, subdivision queue drained in FIFO order with the kernel's
// mirrored-octant arithmetic, flag fold, and the library's exact tier.  Tests
// use it to check the error bounds and the decision logic of the kernels
// against the oracle on the CPU, before and beside the GPU parity tests.
#include <stdint.h>
#include <string.h>

#include <deque>
#include <vector>

#include "hexval_exact.hpp"
#include "hexval_exact_dev.hpp"
#include "hexval_math.hpp"

using namespace hexval;

namespace {

struct EmulNode {
    double b[27];
    double scale;
    int64_t slot;
    int level;
    int orient;
};

int mirrored(int t, int pattern)
{
    const int i = t % 3, j = (t / 3) % 3, k = t / 9;
    const int mi = (pattern & 1) ? 2 - i : i;
    const int mj = (pattern & 2) ? 2 - j : j;
    const int mk = (pattern & 4) ? 2 - k : k;
    return mi + 3 * mj + 9 * mk;
}

void gather(const double* pts, const int32_t* conn, int64_t e, V3 p[8], double raw[24])
{
    for (int k = 0; k < 8; ++k) {
        const double* v = conn ? pts + 3 * (int64_t)conn[8 * e + k] : pts + 24 * e + 3 * k;
        p[k] = {v[0], v[1], v[2]};
        raw[3 * k] = v[0];
        raw[3 * k + 1] = v[1];
        raw[3 * k + 2] = v[2];
    }
}

}  // namespace

extern "C" {

// Per element: the 27 coefficients (Fig. 3 order), the bound scale M^, the
// first-pass state (0 INVALID, 1 VALID, 2 UNDECIDED, 3 SUBDIVIDE, 4 EXACT) and
// min27.  Any output may be NULL.
void hexval_emul_values(const double* pts, const int32_t* conn, int64_t n, int max_depth,
                        double* coeffs, double* scale, int32_t* state, double* min27)
{
    for (int64_t e = 0; e < n; ++e) {
        V3 p[8];
        double raw[24];
        gather(pts, conn, e, p, raw);
        ElementValues r;
        element_values(p, r);
        const Summary s = summarize(r);
        if (coeffs)
            for (int a = 0; a < 27; ++a) coeffs[27 * e + a] = coefficient(r, a);
        if (scale) scale[e] = r.scale;
        if (state) state[e] = top_state(r, s, max_depth);
        if (min27) min27[e] = s.min27;
    }
}

// Sequential replay of the whole GPU pipeline.  verdicts [n], min27 [n] (may
// be NULL), stats (may be NULL): [0] subdivided elements, [1] sub-boxes,
// [2] exact-tier elements, [3] deepest level.
void hexval_emul_check(const double* pts, const int32_t* conn, int64_t n, int max_depth,
                       uint8_t* verdicts, double* min27, int64_t* stats)
{
    std::vector<int64_t> sub_elem;
    std::vector<uint32_t> flags;
    std::deque<EmulNode> queue;
    std::vector<int64_t> exact;
    int64_t nodes = 0, deepest = 0;
    for (int64_t e = 0; e < n; ++e) {
        V3 p[8];
        double raw[24];
        gather(pts, conn, e, p, raw);
        ElementValues r;
        element_values(p, r);
        const Summary s = summarize(r);
        const int st = top_state(r, s, max_depth);
        if (min27) min27[e] = s.min27;
        if (st <= kTopUndecided) {
            verdicts[e] = (uint8_t)st;
        } else if (st == kTopExact) {
            exact.push_back(e);
        } else {
            EmulNode nd;
            for (int a = 0; a < 27; ++a) nd.b[fig3_to_tensor(a)] = coefficient(r, a);
            nd.scale = r.scale;
            nd.slot = (int64_t)sub_elem.size();
            nd.level = 0;
            nd.orient = 0;
            sub_elem.push_back(e);
            flags.push_back(0u);
            queue.push_back(nd);
        }
    }
    while (!queue.empty()) {
        const EmulNode nd = queue.front();
        queue.pop_front();
        for (int child = 0; child < 8; ++child) {
            if (flags[nd.slot] & 1u) break;
            double t[27];
            const int pat = nd.orient ^ child;
            for (int k = 0; k < 27; ++k) t[k] = nd.b[mirrored(k, pat)];
            lower_octant(t);
            const int level = nd.level + 1;
            nodes++;
            if (level > deepest) deepest = level;
            const double tau = level_threshold(nd.scale, level);
            double m8 = t[0], m19 = t[1];
            for (int k = 0; k < 27; ++k) {
                const int i = k % 3, j = (k / 3) % 3, kk = k / 9;
                if (i != 1 && j != 1 && kk != 1) m8 = fmin(m8, t[k]);
                else m19 = fmin(m19, t[k]);
            }
            if (m8 <= -tau) flags[nd.slot] |= 1u;
            else if (!(m8 > tau)) flags[nd.slot] |= 4u;
            else if (m19 > tau) continue;
            else if (level < max_depth) {
                EmulNode c;
                memcpy(c.b, t, sizeof t);
                c.scale = nd.scale;
                c.slot = nd.slot;
                c.level = level;
                c.orient = child;
                queue.push_back(c);
            } else if (m19 <= -tau) flags[nd.slot] |= 2u;
            else flags[nd.slot] |= 4u;
        }
    }
    for (size_t s = 0; s < sub_elem.size(); ++s) {
        const uint32_t f = flags[s];
        const int64_t e = sub_elem[s];
        if (f & 1u) verdicts[e] = 0;
        else if (f & 4u) exact.push_back(e);
        else if (f & 2u) verdicts[e] = 2;
        else verdicts[e] = 1;
    }
    for (int64_t e : exact) {
        V3 p[8];
        double raw[24];
        gather(pts, conn, e, p, raw);
        verdicts[e] = exact_verdict(raw, max_depth);
        if (verdicts[e] == 3 && min27) min27[e] = __builtin_nan("");
    }
    if (stats) {
        stats[0] = (int64_t)sub_elem.size();
        stats[1] = nodes;
        stats[2] = (int64_t)exact.size();
        stats[3] = deepest;
    }
}

// The library's exact tier on n elements [n,8,3].
// The device exact tier on the host: mode 0 verdict (24 doubles per
// element), 1 corner-only test (24), 2 quadrangle (8); 0xFE = left to the
// host tier.
void hexval_emul_exact_device(const double* pts, int64_t n, int mode, int max_depth, uint8_t* out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = mode == 2 ? exact_device_quad(pts + 8 * i) : exact_device_hex(pts + 24 * i, max_depth, mode == 1);
    // exact subdivision where the device tier asks for it, as k_exact_dfs
    std::vector<IW> st((size_t)(max_depth + 1) * kExactDfsWords);
    for (int64_t i = 0; i < n; ++i)
        if (mode == 0 && out[i] == kExactSubdivide) out[i] = exact_device_verdict(pts + 24 * i, max_depth, st.data());
}

// The host exact tier: mode 0 verdict, 1 corner-only test, 2 quadrangle.
void hexval_emul_exact_host(const double* pts, int64_t n, int mode, int max_depth, uint8_t* out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = mode == 2 ? exact_quad(pts + 8 * i) : mode == 1 ? exact_corner_test(pts + 24 * i)
                                                                 : exact_verdict(pts + 24 * i, max_depth);
}

void hexval_emul_exact(const double* pts, int64_t n, int max_depth, uint8_t* verdicts)
{
    for (int64_t e = 0; e < n; ++e) verdicts[e] = exact_verdict(pts + 24 * e, max_depth);
}

// First-pass quantities of the lean kernels (precision 0: FP64, 1: FP32
// filter): m20 (min of the values tested at step 2), mb (min b_9..b_27),
// min27, scale M^, certified-range flag, and the state the kernel takes
// (FP64: 0..4 as hexval_emul_values; FP32: 0 INVALID, 1 VALID, -1 recheck).
void hexval_emul_lean(const double* pts, const int32_t* conn, int64_t n, int precision, int check_edges,
                      double* m20, double* mb, double* min27, double* scale, int32_t* state)
{
    for (int64_t e = 0; e < n; ++e) {
        V3 p[8];
        double raw[24];
        gather(pts, conn, e, p, raw);
        if (precision == 0) {
            const LeanResult r = element_lean(p, check_edges != 0);
            m20[e] = r.m20; mb[e] = r.mb; min27[e] = r.min27; scale[e] = r.scale;
            state[e] = lean_state(r, check_edges ? 0 : 6);
        } else {
            const LeanT<float> r = element_lean_t<float>(p, check_edges != 0);
            m20[e] = r.m20; mb[e] = r.mb; min27[e] = r.min27; scale[e] = r.scale;
            state[e] = filter_state(r);
        }
    }
}

// Per element: 1 where the FP32 filter sends the element to subdivision
// itself (filter_subdivides), else 0; and the FP64 pass's state at depth
// cap 6 (0..4 as hexval_emul_values).
void hexval_emul_filter_subdivides(const double* pts, const int32_t* conn, int64_t n, int32_t* sub,
                                   int32_t* state64)
{
    for (int64_t e = 0; e < n; ++e) {
        V3 p[8];
        double raw[24];
        gather(pts, conn, e, p, raw);
        sub[e] = filter_subdivides(element_lean_t<float>(p, false)) ? 1 : 0;
        state64[e] = lean_state(element_lean(p, false), 6);
    }
}

// Bound constants of the kernels: {tau_value, tau_coeff, tau_level, u64, u32}.
// The kernels' outward rounding of min-J bounds, element-wise.
void hexval_emul_next(const double* x, int64_t n, double* down, double* up)
{
    for (int64_t i = 0; i < n; ++i) {
        down[i] = next_down(x[i]);
        up[i] = next_up(x[i]);
    }
}

void hexval_emul_constants(double* out)
{
    out[0] = kTauValue;
    out[1] = kTauCoeff;
    out[2] = kTauLevel;
    out[3] = kU64;
    out[4] = kU32;
}
}
