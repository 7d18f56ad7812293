#!/usr/bin/env python3
"""Throughput of the hexahedron validity test on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one full call of the library (first pass, subdivision, fold,
exact tier) on the 64M-hex structured mesh: 400^3 cells of a float64 vertex
lattice warped by a sinusoidal map (amplitude 0.2 cell, wavelength 16
cells), 1% of the vertices jittered by U(-0.8, 0.8)^3 cell, int32
connectivity [N,8] and shared vertices [M,3] resident in HBM, plain FP64.
Prints one JSON line (see the keys below).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "hexes validated/s: plain FP64 vs FP32-filter+FP64; p50/p99 request ms"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n_hex, n_vert, with_min=True):
    """Bytes the first pass must move at least once: connectivity (32 B/hex),
    each vertex once (24 B), verdict (1 B/hex) and min coefficient (8 B/hex)."""
    return 32 * n_hex + 24 * n_vert + n_hex * (9 if with_min else 1)


# FP64 VALU issue rate of MI355X: 256 CUs x 64 lanes x 2.4 GHz (one FP64
# add, multiply, FMA or min per lane per clock).
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# FP64 arithmetic operations per hex of the first pass (add, sub, mul, FMA,
# min, max each counted once): 36 edge differences, 35 for the scale bound,
# 8 corner cross products (6 each) and their dot products (3 each), 8 xi/eta
# 2 b_e as six-product dot chains (6 each), 56 for the zeta-edges (pair sums,
# 4 triple products, corner sums, subtractions), 38 for the face and centre
# sums of Table 3, 29 for the minima and the final scalings.
VALU_OPS_PER_HEX = 36 + 35 + 8 * 6 + 8 * 3 + 8 * 6 + 56 + 38 + 29
KERNEL_SOURCES = ["hexval_kernels.hip", "hexval_kernels.hpp", "hexval_math.hpp", "hexval_internal.hpp"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "first_pass_fp64_lattice400_traffic.md")


def kernel_source_digest():
    """sha256 over the sources the first-pass kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1706_01613_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per first-pass launch from the committed counter profile, or
    None when the kernel sources have changed since it was taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        key, _, val = line.strip().partition(": ")
        if key in ("traffic_bytes_per_launch", "source_sha256"):
            vals[key] = val.strip()
    if vals.get("source_sha256") != kernel_source_digest() or "traffic_bytes_per_launch" not in vals:
        return None
    return int(vals["traffic_bytes_per_launch"])


def run_steps(hx, torch, pts, conn, steps, precision, stream):
    """Runs `steps` calls; returns (wall seconds, per-call stats list)."""
    n = conn.shape[0]
    verdicts = torch.empty(n, dtype=torch.uint8, device="cuda")
    mins = torch.empty(n, dtype=torch.float64, device="cuda")
    mesh = hx.make_mesh(pts, conn, n)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = hx.hexval_stats_t()
        st.timing = 1
        opts = hx.make_opts(precision=precision, stream=stream, stats=st)
        hx.hexval_check_ex(mesh, opts, verdicts, mins)
        stats.append(st.as_dict())
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats, verdicts, mins


def machine_ceilings(torch):
    """Achievable rates of this GPU from kernels of known work
    (libhexval_calib.so): a read-only stream over 8 GiB, a 2 GiB copy, and
    FP64 FMA chains on every lane (with the shader clock during them)."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1706_01613_amd", "libhexval_calib.so"))
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.hexval_calib_read.argtypes = [P, I64, I, P]
    L.hexval_calib_copy.argtypes = [P, P, I64, I, P]
    L.hexval_calib_fp64.argtypes = [I64, I, P, P, P]
    ms = ctypes.c_float()
    out = {}
    nb = 8 << 30
    buf = torch.ones(nb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    assert L.hexval_calib_read(buf.data_ptr(), nb, 10, ctypes.byref(ms)) == 0
    out["hbm_read_GBps"] = nb / (ms.value * 1e-3) / 1e9
    del buf
    nb = 2 << 30
    src = torch.ones(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    assert L.hexval_calib_copy(dst.data_ptr(), src.data_ptr(), nb, 10, ctypes.byref(ms)) == 0
    out["hbm_copy_GBps"] = 2 * nb / (ms.value * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    flops, mhz = ctypes.c_double(), ctypes.c_double()
    assert L.hexval_calib_fp64(1 << 14, 5, ctypes.byref(ms), ctypes.byref(flops), ctypes.byref(mhz)) == 0
    out["fp64_fma_TFLOPs"] = flops.value / (ms.value * 1e-3) / 1e12
    out["shader_clock_MHz_during_fp64"] = mhz.value
    out["what"] = ("read-only 16-byte stream over 8 GiB; copy of 2 GiB (read + write bytes); 8 independent "
                   "FP64 FMA chains per lane on 8 blocks of 256 per CU")
    return out


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timed_oracle_check(oracle, V, C, threads):
    t0 = time.perf_counter()
    ref = oracle.check(V, C, threads=threads)
    return ref, time.perf_counter() - t0


def cpu_baseline(V, C, gpu_verdicts, work, target_s=12.0):
    """The oracle (plain FP64 C, OpenMP over elements, untuned) timed on the
    host's cores: a bounded leading sample of the main mesh with all threads
    and with one thread, the whole precision-stress mesh, a stated sample of
    the batched workload's meshes, and the min-J oracle on a leading sample.
    Every timed sample also checks the GPU results of the same elements."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    probe = min(C.shape[0], 1 << 20)
    _, dt = timed_oracle_check(oracle, V, C[:probe], threads)
    rate = probe / max(dt, 1e-6)
    n = int(min(C.shape[0], max(probe, rate * target_s)))
    ref, dt = timed_oracle_check(oracle, V, C[:n], threads)
    mism = int((ref["verdict"] != gpu_verdicts[:n]).sum())
    # one thread, on a sample of about 3 s of its work
    n1 = int(min(C.shape[0], max(1 << 16, 3.0 * rate / threads)))
    ref1, dt1 = timed_oracle_check(oracle, V, C[:n1], 1)
    out = {"value": n / dt, "unit": "hex/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} hexes of the same mesh ({dt:.1f} s)",
           "per_core": n / dt / threads, "one_thread": n1 / dt1,
           "one_thread_sample": f"first {n1} hexes of the same mesh ({dt1:.1f} s)",
           "paper_one_core_context": "about 6e6 hex/s on one core of a 2016 laptop (context only)",
           "cpu_model": host_cpu_model(), "nproc": os.cpu_count(),
           "verdict_mismatches_vs_gpu": mism + int((ref1["verdict"] != gpu_verdicts[:n1]).sum())}
    if "precision_stress" in work:
        Vs, Cs, vs = work["precision_stress"]
        ref, dt = timed_oracle_check(oracle, Vs, Cs, threads)
        out["precision_stress"] = {"value": Cs.shape[0] / dt, "unit": "hex/s", "hexes": int(Cs.shape[0]),
                                   "seconds": dt, "n_fragile_exact": int(ref["fragile"].size),
                                   "verdict_mismatches_vs_gpu": int((ref["verdict"] != vs).sum())}
    if "batched_sample" in work:
        sample, label = work["batched_sample"]
        nb, dt, mism_b = 0, 0.0, 0
        for Vb, Cb, vb in sample:
            ref, d = timed_oracle_check(oracle, Vb, Cb, threads)
            nb += Cb.shape[0]
            dt += d
            mism_b += int((ref["verdict"] != vb).sum())
        out["batched_sample"] = {"value": nb / dt, "unit": "hex/s", "hexes": nb, "seconds": dt,
                                 "sample": label, "verdict_mismatches_vs_gpu": mism_b}
    if "min_jacobian" in work:
        m, rtol, lo, hi = work["min_jacobian"]
        t0 = time.perf_counter()
        ref = oracle.min_jacobian(V, C[:m], rtol=rtol, max_depth=6, threads=threads)
        dt = time.perf_counter() - t0
        disjoint = int(np.count_nonzero((lo > ref["hi"]) | (ref["lo"] > hi)))
        out["min_jacobian"] = {"value": m / dt, "unit": "hex/s", "sample": f"first {m} hexes",
                               "disjoint_intervals_vs_gpu": disjoint}
    return out


def fp32_leg(hx, torch, synth, steps, stream, work):
    """Precision stress workload: the same lattice plus 5% near-degenerate,
    rescaled independent hexes; plain FP64 against the FP32 filter + FP64
    recheck on the same device-resident mesh."""
    V, C = synth.precision_stress(seed=0, seed_extra=1)
    pts = torch.from_numpy(V).to("cuda")
    conn = torch.from_numpy(C).to("cuda")
    n = conn.shape[0]
    out = {"workload": "400^3 warped lattice + 5% near-degenerate hexes (one corner within 1e-7 "
                       "relative of flat, coordinates scaled by 10^U(-3,3))", "hexes": n}
    res = {}
    for name, prec in (("fp64", hx.FP64), ("fp32_filter", hx.FP32_FILTER)):
        run_steps(hx, torch, pts, conn, 2, prec, stream)
        wall, stats, v, m = run_steps(hx, torch, pts, conn, steps, prec, stream)
        res[name] = (v.clone(), m.clone())
        out[name] = {"value": n * steps / wall, "unit": "hex/s", "ms_per_step": 1e3 * wall / steps,
                     "ms_first_pass": float(np.mean([s["ms_first_pass"] for s in stats])),
                     "ms_recheck": float(np.mean([s["ms_recheck"] for s in stats])),
                     "n_recheck": stats[-1]["n_recheck"], "n_exact": stats[-1]["n_exact"]}
    out["speedup_fp32_filter"] = out["fp32_filter"]["value"] / out["fp64"]["value"]
    out["verdicts_identical"] = bool(torch.equal(res["fp64"][0], res["fp32_filter"][0]))
    work["precision_stress"] = (V, C, res["fp64"][0].cpu().numpy())
    # FP32 error of min_coeff against FP64, relative to each element's largest
    # FP64 coefficient (elements rechecked in FP64 have error 0)
    coeffs = hx.coefficients(pts, conn)
    bmax = coeffs.abs().amax(dim=1)
    del coeffs
    err = (res["fp32_filter"][1] - res["fp64"][1]).abs() / bmax
    err = err[torch.isfinite(err)]
    out["fp32_min_coeff_error_vs_fp64"] = {"max": float(err.max()), "p99": float(torch.quantile(
        err[torch.randperm(err.numel(), device=err.device)[:1 << 22]], 0.99))}
    return out


def serving_leg(hx, torch, synth, capacity_hex_s, n_req=2000, n_pool=32, seed=5):
    """Poisson request streams against the server (device-resident request
    meshes, sizes log-uniform in [1e3, 1e7] hexes, generated as in the
    precision-stress workload), rate swept geometrically from 0.05x to 2x the
    estimated capacity; p50/p99 latency and hexes/s per rate, FP64 and FP32
    filter servers, plus the host-upload mode at three rates."""
    from paper_1706_01613_amd import loadgen
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(3.0, 7.0, size=n_pool)).astype(int)
    pool = [synth.near_degenerate_mesh_torch(int(s), seed=seed * 1000 + k) for k, s in enumerate(sizes)]
    n_hex = np.array([C.shape[0] for _, C in pool])
    mean = float(n_hex.mean())
    cap_req = capacity_hex_s / mean
    fracs = [0.05, 0.15, 0.4, 0.8, 1.2, 2.0]
    out = {"workload": f"Poisson arrivals, {n_req} requests per rate, pool of {n_pool} device-resident "
                       f"meshes (mean {mean:.3g} hexes, log-uniform sizes 1e3..1e7, 5% near-degenerate)",
           "estimated_capacity_req_s": cap_req, "slots": 8}
    idx_all = rng.integers(0, n_pool, size=n_req)
    arena = torch.empty(loadgen.arena_bytes(n_hex[idx_all]), dtype=torch.uint8, device="cuda")

    def one(server, frac, templates, n):
        rate = frac * cap_req
        arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
        arrival -= arrival[0]
        lat, st, _, wall = loadgen.run(server, arrival, idx_all[:n], templates, arena)
        assert (st == hx.OK).all()
        hexes = float(n_hex[idx_all[:n]].sum())
        return {"rate_x_capacity": frac, "offered_req_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "hex_s": hexes / wall, "requests": n}

    dev_t = []
    for V, C in pool:
        r = hx.hexval_request_t()
        r.mesh = hx.make_mesh(V, C)
        dev_t.append(r)
    for name, prec in (("fp64", hx.FP64), ("fp32_filter", hx.FP32_FILTER)):
        sv = hx.hexval_server_create(hx.make_opts(precision=prec), 64 << 30, 8)
        try:
            one(sv, 0.5, dev_t, 200)   # warm-up (autotuning, allocations)
            out[name] = [one(sv, f, dev_t, n_req) for f in fracs]
        finally:
            hx.hexval_server_destroy(sv)
        log(f"serving {name}: " + ", ".join(f"{r['rate_x_capacity']}x p50 {r['p50_ms']:.3f} "
                                            f"p99 {r['p99_ms']:.3f} ms" for r in out[name]))
    # host-upload mode: meshes in pinned host memory, copied by the server
    host = [(V.cpu().pin_memory(), C.cpu().pin_memory()) for V, C in pool]
    host_t = []
    for V, C in host:
        r = hx.hexval_request_t()
        r.mesh = hx.hexval_mesh_t(None, V.shape[0], None, C.shape[0])
        r.host_points = V.data_ptr()
        r.host_conn = C.data_ptr()
        host_t.append(r)
    sv = hx.hexval_server_create(hx.make_opts(), 64 << 30, 8)
    try:
        one(sv, 0.05, host_t, 100)
        out["fp64_host_upload"] = [one(sv, f, host_t, n_req // 4) for f in (0.02, 0.05, 0.1)]
    finally:
        hx.hexval_server_destroy(sv)
    return out


def batched_leg(hx, torch, synth, steps, work):
    """Batched workload: 10,000 meshes, hex counts log-uniform in [1e2, 1e6],
    every vertex jittered by U(-a_m, a_m)^3 with a_m ~ U(0, 0.6), FP32 filter +
    FP64, depth cap 6: one persistent launch per step, against one
    hexval_check_ex call per mesh.  The FP32-filter verdicts are compared with
    the FP64 batch's and with the per-mesh calls' on every element; every
    100th mesh and the largest are kept for the oracle in the CPU leg."""
    meshes = list(synth.batched_meshes_torch(10000, seed=4))
    sizes = [C.shape[0] for _, C in meshes]
    total = int(sum(sizes))
    verts = int(sum(V.shape[0] for V, _ in meshes))
    vs = [torch.empty(C.shape[0], dtype=torch.uint8, device="cuda") for _, C in meshes]
    ms = [torch.empty(C.shape[0], dtype=torch.float64, device="cuda") for _, C in meshes]
    descs = [hx.make_mesh(V, C) for V, C in meshes]
    stream = torch.cuda.current_stream()
    alg = algorithmic_bytes(total, verts)
    res = {"workload": "10,000 warped lattices, 1e2..1e6 hexes (log-uniform), all vertices jittered "
                       "U(0,0.6) cell, FP32 filter + FP64, cap 6", "hexes": total, "meshes": len(meshes),
           "vertices": verts}
    verdicts = {}
    for name, prec in (("fp32_filter", hx.FP32_FILTER), ("fp64", hx.FP64)):
        st = hx.hexval_stats_t()
        st.timing = 1
        opts = hx.make_opts(precision=prec, stream=stream, stats=st)
        args = hx.BatchArgs(descs, vs, ms)                 # C arrays built once
        hx.hexval_check_batched(args, opts)               # warm-up + tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        first = []
        for _ in range(steps):
            hx.hexval_check_batched(args, opts)
            first.append(st.ms_first_pass)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        verdicts[name] = torch.cat(vs)
        gbps = alg / (float(np.mean(first)) * 1e-3) / 1e9
        res[name] = {"value": total / wall, "unit": "hex/s", "ms_per_step": 1e3 * wall,
                     "first_pass": {"ms": float(np.mean(first)), "algorithmic_bytes": alg,
                                    "achieved_GBps": gbps, "frac_of_8TBps": gbps / 8000.0},
                     "stats": st.as_dict()}
    # the same meshes one call at a time (FP32 filter)
    opts = hx.make_opts(precision=hx.FP32_FILTER, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, v, m in zip(descs, vs, ms):
        hx.hexval_check_ex(d, opts, v, m)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_mesh = torch.cat(vs)
    res["fp32_filter_one_call_per_mesh"] = {"value": total / wall, "unit": "hex/s", "ms_per_pass": 1e3 * wall}
    res["speedup_batched_vs_per_mesh"] = res["fp32_filter"]["value"] / res["fp32_filter_one_call_per_mesh"]["value"]
    res["verdict_mismatches_fp32_filter_vs_fp64"] = int((verdicts["fp32_filter"] != verdicts["fp64"]).sum())
    res["verdict_mismatches_batched_vs_per_mesh"] = int((verdicts["fp32_filter"] != per_mesh).sum())
    res["verdicts_identical"] = (res["verdict_mismatches_fp32_filter_vs_fp64"] == 0
                                 and res["verdict_mismatches_batched_vs_per_mesh"] == 0)
    pick = sorted(set(range(0, len(meshes), 100)) | {int(np.argmax(sizes))})
    offsets = np.cumsum([0] + sizes)
    v_host = verdicts["fp32_filter"].cpu().numpy()
    work["batched_sample"] = ([(meshes[k][0].cpu().numpy(), meshes[k][1].cpu().numpy(),
                                v_host[offsets[k]:offsets[k + 1]]) for k in pick],
                              f"every 100th of the 10,000 meshes and the largest ({len(pick)} meshes)")
    del meshes, vs, ms, descs, verdicts, per_mesh
    return res


def min_jacobian_leg(hx, torch, V, C, pts, conn, steps, stream, work, rtol=1e-3):
    """Certified bounds of min J (hexval_min_jacobian, rtol 1e-3, cap 6) on the
    main mesh, inputs resident; a leading sample is kept for the oracle in the
    CPU leg."""
    n = conn.shape[0]
    lo = torch.empty(n, dtype=torch.float64, device="cuda")
    hi = torch.empty_like(lo)
    status = torch.empty(n, dtype=torch.uint8, device="cuda")
    mesh = hx.make_mesh(pts, conn, n)
    st = hx.hexval_stats_t()
    st.timing = 1
    opts = hx.make_opts(stream=stream, stats=st)
    hx.hexval_min_jacobian(mesh, opts, rtol, lo, hi, status)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hx.hexval_min_jacobian(mesh, opts, rtol, lo, hi, status)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    hist = np.bincount(status.cpu().numpy(), minlength=5)[:5].tolist()
    m = 1 << 22
    work["min_jacobian"] = (m, rtol, lo[:m].cpu().numpy(), hi[:m].cpu().numpy())
    # first pass: connectivity, each vertex once, lo + hi + status (17 B/hex)
    alg = 32 * n + 24 * pts.shape[0] + 17 * n
    gbps = alg / (st.ms_first_pass * 1e-3) / 1e9
    return {"workload": "min J to rtol 1e-3 (certified bounds), same 400^3 lattice, cap 6",
            "value": n / wall, "unit": "hex/s", "ms_per_step": 1e3 * wall, "status_counts": hist,
            "first_pass": {"kernel": "k_minj_top_walk" if st.walk_layers else "k_minj_top_conn",
                           "ms": st.ms_first_pass,
                           "algorithmic_bytes": alg, "achieved_GBps": gbps, "frac_of_8TBps": gbps / 8000.0},
            "stats": st.as_dict()}


def corner_test_leg(hx, torch, synth, steps, n_pool=16_000_000):
    """The false-valid accounting of Section 7 (Table 4's methodology) on
    synthetic data: a pool of independent tangled hexes (unit cube corners +
    U(-0.6, 0.6)^3, seed 6) split, as the paper's datasets are, by a minimal
    corner quality q in {0.5, 0, -1}; for each subset, the number of invalid
    elements (full method), the corner-only test's false valid and false
    invalid counts, and the device time of both."""
    P = torch.from_numpy(synth.independent_hexes(n_pool, noise=0.6, seed=6)).to("cuda")
    _, q, _ = hx.corner_test(P)
    rows = []
    for qmin in (0.5, 0.0, -1.0):
        sub = P[q >= qmin].contiguous()
        n = sub.shape[0]
        mesh = hx.make_mesh(sub, None, n)
        v = torch.empty(n, dtype=torch.uint8, device="cuda")
        t1 = torch.empty_like(v)
        opts = hx.make_opts(stream=torch.cuda.current_stream())
        times = {}
        for name, call in (("full", lambda: hx.hexval_check_ex(mesh, opts, v, None)),
                           ("test1", lambda: hx.hexval_corner_test(mesh, opts, t1, None))):
            call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) / steps
        inv = v == hx.INVALID
        # Test 1 reads the 8 corners (192 B) and writes one byte per hex
        t1_gbps = 193 * n / times["test1"] / 1e9
        rows.append({"q_min": qmin, "hexes": n, "invalid": int(inv.sum()),
                     "undecided": int((v == hx.UNDECIDED).sum()),
                     "test1_false_valid": int((inv & (t1 == hx.VALID)).sum()),
                     "test1_false_invalid": int(((v == hx.VALID) & (t1 == hx.INVALID)).sum()),
                     "ms_full": 1e3 * times["full"], "ms_test1": 1e3 * times["test1"],
                     "test1_algorithmic_GBps": t1_gbps, "test1_frac_of_8TBps": t1_gbps / 8000.0})
        del sub, v, t1
    return {"workload": f"{n_pool} independent hexes, unit cube + U(-0.6,0.6)^3, split by min corner "
                        "quality as Table 4's datasets", "rows": rows}


def quad_leg(hx, torch, synth, steps, n=8000):
    """Linear quadrangles (Section 2.1): n^2-cell warped lattice, 1% of the
    vertices jittered 0.8 cell, int32 connectivity + f64 shared vertices
    resident in HBM; verdicts and min J."""
    V, C = synth.quad_lattice(n, n, seed=0)
    pts, conn = torch.from_numpy(V).to("cuda"), torch.from_numpy(C).to("cuda")
    nq = C.shape[0]
    v = torch.empty(nq, dtype=torch.uint8, device="cuda")
    m = torch.empty(nq, dtype=torch.float64, device="cuda")
    st = hx.hexval_stats_t()
    st.timing = 1
    mesh = hx.hexval_mesh_t(pts.data_ptr(), V.shape[0], conn.data_ptr(), nq)
    opts = hx.make_opts(stream=torch.cuda.current_stream(), stats=st)
    hx.hexval_quad_check(mesh, opts, v, m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = []
    for _ in range(steps):
        hx.hexval_quad_check(mesh, opts, v, m)
        ms.append(st.ms_first_pass)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    alg = 16 * nq + 16 * V.shape[0] + 9 * nq
    k = float(np.mean(ms))
    return {"workload": f"{n}^2 warped quad lattice, 1% of vertices jittered 0.8 cell", "quads": nq,
            "value": nq / wall, "unit": "quad/s", "ms_per_step": 1e3 * wall, "ms_kernel": k,
            "algorithmic_GBps": alg / (k * 1e-3) / 1e9, "frac_of_8TBps": alg / (k * 1e-3) / 8e12,
            "invalid": int((v == hx.INVALID).sum()), "stats": st.as_dict()}


def exact_tier_leg(hx, torch, synth, n=1_000_000):
    """The exact tier: n integer hexes (2 x unit cube + U{-1,0,1}^3 per
    coordinate, seed 12, every fourth with two coincident corners), most of
    whose values and coefficients are exactly 0 or too close to 0 for the
    FP64 bounds.  Once as they are (integers: the device tier settles what
    needs no subdivision) and once with one coordinate per element moved to
    2^-60 (a span beyond the device tier's integers: everything uncertain
    goes to the host)."""
    rng = np.random.default_rng(12)
    P = (synth.CUBE[None] * 2 + rng.integers(-1, 2, size=(n, 8, 3))).astype(np.float64)
    P[::4, 1] = P[::4, 0]
    W = P.copy()
    W[:, 0, 2] = np.where(W[:, 0, 2] == 0.0, 2.0 ** -60, W[:, 0, 2])
    out = {"workload": f"{n} integer hexes with exact zeros (device tier) / with a 2^-60 coordinate "
                       "(host tier)"}
    for name, X in (("device", P), ("host", W)):
        Xd = torch.from_numpy(X).to("cuda")
        hx.check(Xd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st = hx.check(Xd, stats=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"ms": 1e3 * wall, "n_exact": st["n_exact"], "n_exact_host": st["n_exact_host"],
                     "exact_elements_per_s": st["n_exact"] / wall}
    return out


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size, for scaling the profiler's
    FETCH_SIZE / WRITE_SIZE counters."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x {nbytes} bytes copied")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=400, help="lattice cells per axis")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32-filter and serving legs")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 1 GiB copy (profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (elements are independent, so several GPUs "
              "would each check their own share of the elements). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1706_01613_amd import hexval as hx
    from paper_1706_01613_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nc = args.cells
    log(f"generating the {nc}^3 warped lattice")
    V, C = synth.warped_lattice(nc, nc, nc, seed=0)
    n_hex, n_vert = C.shape[0], V.shape[0]
    pts = torch.from_numpy(V).to("cuda")
    conn = torch.from_numpy(C).to("cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    log(f"warmup {args.warmup}")
    run_steps(hx, torch, pts, conn, args.warmup, hx.FP64, stream)
    log(f"timing {args.steps} steps")
    wall, stats, verdicts, mins = run_steps(hx, torch, pts, conn, args.steps, hx.FP64, stream)
    ms_step = 1e3 * wall / args.steps
    value = n_hex * args.steps / wall
    first = np.array([s["ms_first_pass"] for s in stats])
    alg = algorithmic_bytes(n_hex, n_vert)
    achieved = alg / (first.mean() * 1e-3) / 1e9
    valu_ops = VALU_OPS_PER_HEX * n_hex / (first.mean() * 1e-3)
    v_host = verdicts.cpu().numpy()
    hist = np.bincount(v_host, minlength=4)[:4].tolist()
    log(f"{value:.4g} hex/s, {ms_step:.3f} ms/step, first pass {first.mean():.3f} ms "
        f"({achieved:.0f} GB/s algorithmic), verdicts {hist}, stats {stats[-1]}")
    if args.copy_calib:
        copy_calibration(torch)
    log("machine ceilings")
    ceilings = machine_ceilings(torch)
    log(f"machine ceilings {ceilings}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "hex/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"warped {nc}^3-cell hex lattice, 1% of vertices jittered 0.8 cell, "
                               f"int32 connectivity + f64 shared vertices, plain FP64",
                   "hexes": n_hex, "vertices": n_vert, "max_depth": 6, "precision": "fp64",
                   "inputs": "resident in HBM"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": ("k_top_f64_walk" if stats[-1]["walk_layers"] else "k_top_f64_conn")
                               + " (first pass)",
                     "algorithmic_bytes_per_launch": alg,
                     "avg_launch_ms": float(first.mean()),
                     "valu": {"achieved": valu_ops, "peak": VALU_PEAK_OPS, "unit": "FP64 lane-ops/s",
                              "frac": valu_ops / VALU_PEAK_OPS, "ops_per_hex": VALU_OPS_PER_HEX},
                     "frac_of_measured_read_ceiling": achieved / ceilings["hbm_read_GBps"],
                     # the whole call (first pass, stride search, subdivision, fold, counters
                     # read back) against the same bytes: what the step's wall time reaches
                     "frac_per_call": alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "machine_ceilings": ceilings,
        "verdicts": {"invalid": hist[0], "valid": hist[1], "undecided": hist[2],
                     "bad_input": hist[3]},
        "call_stats": stats[-1],
        "paper_context": "about 6e6 hex/s on one core of a 2016 laptop (the paper's serial C++), context only",
    }
    work = {}   # host copies of GPU results for the oracle comparisons of the CPU leg
    if not args.no_extras:
        log("min J leg")
        out["min_jacobian"] = min_jacobian_leg(hx, torch, V, C, pts, conn, max(3, args.steps // 4), stream,
                                               work)
        log(f"min J leg {out['min_jacobian']}")
        log("fp32 filter leg (precision stress workload)")
        del pts, conn
        torch.cuda.empty_cache()
        out["fp32_filter_vs_fp64"] = fp32_leg(hx, torch, synth, max(5, args.steps // 2), stream, work)
        log(f"fp32 leg {out['fp32_filter_vs_fp64']}")
        torch.cuda.empty_cache()
        log("quad leg")
        out["quads"] = quad_leg(hx, torch, synth, 10)
        log(f"quad leg {out['quads']}")
        torch.cuda.empty_cache()
        log("corner-only test leg")
        out["corner_test_vs_full"] = corner_test_leg(hx, torch, synth, 5)
        log(f"corner leg {out['corner_test_vs_full']}")
        torch.cuda.empty_cache()
        log("exact tier leg")
        out["exact_tier"] = exact_tier_leg(hx, torch, synth)
        log(f"exact tier leg {out['exact_tier']}")
        log("batched leg")
        out["batched"] = batched_leg(hx, torch, synth, 3, work)
        log(f"batched leg {out['batched']}")
        torch.cuda.empty_cache()
        log("serving leg")
        out["serving"] = serving_leg(hx, torch, synth, value)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(V, C, v_host, work)
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
