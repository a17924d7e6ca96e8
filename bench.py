"""Benchmark: weighted-quadrature assembly of Poisson mass + stiffness on one MI355X.

Workload (default): 256 x 256 control faces on [0,1]^2, ~1% of interior vertices
replaced by EPs of valence 3/5/6 (seeded), smooth seeded displacement (amplitude 0.05),
bicubic EP-enriched splines, TSVD cutoff 1e-12 relative, FP64.

One step = the whole path on the resident mesh: build_points (classification, points,
pattern, point sets, basis/geometry), solve_weights (Gauss right-hand sides + TSVD
weights of the mass, x and y families) and the fused mass + stiffness assembly with
variable coefficients c = 1 + sin(2 pi x) sin(2 pi y) / 2, k = 1 + cos(pi x) cos(pi y) / 2.
The metric is assembled CSR nonzeros (M and K) per second of step time. The assembly
alone (the repeated operation when the domain is fixed) is reported beside it.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector


def aggregate(recs, steps):
    """Per kernel: total ms, launches, summed algorithmic work (library timing records)."""
    out = {}
    for name, ms, work in recs:
        e = out.setdefault(name, {"ms": 0.0, "launches": 0, "work": 0})
        e["ms"] += ms
        e["launches"] += 1
        e["work"] += work
    for e in out.values():
        e["ms_per_step"] = e["ms"] / steps
    return out


def traffic_of(kernel):
    """HBM bytes per launch from the committed counter summary of `kernel`, if it was
    taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 4 and parts[0] == kernel:
            rec = {"src": parts[1], "sha": parts[2], "bytes": float(parts[3])}
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2605_29334_amd", "csrc", rec["src"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != rec["sha"]:
        return None
    return rec["bytes"]


def roofline_of(name, e):
    """Roofline entry of one kernel from its timing aggregate: algorithmic work per launch
    over the average launch duration."""
    avg_ms = e["ms"] / e["launches"]
    per_launch = e["work"] / e["launches"]
    if name.startswith(("k_tsvd", "k_wsolve")):
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        return {"kernel": name, "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_of(name), "avg_launch_ms": avg_ms,
                "launches": e["launches"], "algorithmic_per_launch": per_launch}
    if name.startswith("k_assemble"):
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_of(name), "avg_launch_ms": avg_ms,
                "launches": e["launches"], "algorithmic_per_launch": per_launch}
    return {"kernel": name, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": avg_ms, "launches": e["launches"]}


def small_pool(seed=3000):
    """Seeded small meshes for the batched and served measurements: grids and EP meshes
    of 16..64 control faces per side (displacement 0.05)."""
    import fixtures as fx
    pool = []
    for j, N in enumerate((16, 24, 32, 40, 48, 64)):
        pool.append(fx.fixture_grid(N, displace=0.05, seed=seed + j))
    for j, N in enumerate((32, 48, 64)):
        pool.append(fx.fixture_eps(N, 0.02, (3, 5, 6), displace=0.05, seed=seed + 10 + j))
    return pool


def measure_batched(W, torch, pool, copies):
    """The same meshes one by one (points, weights, mass + stiffness each) against one
    batch of all of them (one set of launches), and the batch's assembly replayed as a
    HIP graph against eager per-mesh assemblies."""
    meshes = [pool[i % len(pool)] for i in range(copies * len(pool))]
    mask = W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    nnz = 0
    for F in meshes:
        m = W.Mesh(F)
        p = W.Points(m)
        w = W.Weights(m, p, mask)
        W.assemble_mass_stiffness(p, w)
        per.append((m, p, w))
        nnz += 2 * p.nnz
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = W.Batch(meshes).build(mask)
    Mb, Kb = W.assemble_mass_stiffness(B.points, B.weights)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    s = torch.cuda.Stream()
    reps = 20

    def graph_ms():
        B.graph_assemble(None, None, Mb, Kb, stream=s)  # (captured again after a retune)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.graph_assemble(None, None, Mb, Kb, stream=s)
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    g0_ms = graph_ms()
    cap, chunk, _ = W.autotune_tiles(B.points, B.weights)  # tile work cap and XCD run length
    g_ms = graph_ms()
    outs = [(W.assemble_mass_stiffness(p, w)) for (_, p, w) in per]  # outputs allocated once
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for (_, p, w), (M, K) in zip(per, outs):
            W.assemble_mass_stiffness(p, w, None, None, M, K)
    e1.record()
    e1.synchronize()
    s_ms = e0.elapsed_time(e1) / reps
    return {"meshes": len(meshes), "rows": int(B.points.n_rows), "nnz_M_plus_K": int(nnz),
            "setup_to_matrices_s": {"one_by_one": t_single, "batched": t_batch},
            "nnz_per_s_setup_to_matrices": {"one_by_one": nnz / t_single, "batched": nnz / t_batch},
            "assembly_ms": {"eager_per_mesh": s_ms, "batched_graph": g_ms, "batched_graph_default_tiles": g0_ms},
            "autotuned": {"tile_step_cap": cap, "xcd_chunk": chunk},
            "nnz_per_s_assembly": {"eager_per_mesh": nnz / (s_ms * 1e-3), "batched_graph": nnz / (g_ms * 1e-3)}}


def served_pool(n_meshes=6, seed=5):
    """Distinct seeded meshes for the served workload: N ~ U{32..256} control faces per
    side (multiples of 4), 1 % extraordinary points (valence 3/5/6), displacement 0.05."""
    import fixtures as fx
    rng = np.random.default_rng(seed)
    sizes = sorted(4 * int(v) for v in rng.integers(8, 65, n_meshes))  # the EP templates need N divisible by 4
    return [fx.fixture_eps(N, 0.01, (3, 5, 6), displace=0.05, seed=5000 + j) for j, N in enumerate(sizes)], sizes


def measure_served(W, pool, n_requests, rate, slots, seed=5, n_steps=1, tangent=0, reuse=False, join=1,
                   join_rows=1 << 15, workload=""):
    """Nonlinear heat requests (k = 1 + u^2, manufactured source, n_steps of dt 0.1 from
    T = 0) on meshes drawn from the pool, arriving as a Poisson stream of `rate` per
    second, served with continuous admission on `slots` concurrent streams; latency =
    completion - arrival. reuse = False: every request sets its domain up from scratch.
    join > 1: requests queued together run as one union of up to `join` meshes and
    `join_rows` rows."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    picks = rng.integers(0, len(pool), n_requests)
    S = W.Server(64 << 30, slots)
    if join > 1:
        S.set_join(join, join_rows)
    t0 = time.perf_counter()
    tickets = []
    for a, j in zip(arrivals, picks):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        F = pool[j]
        tickets.append(S.submit(F, F["dir1"], 0.1, n_steps, k=(W.K_QUADRATIC, 1.0, 1.0), tangent=tangent,
                                reuse_setup=reuse))
    res = [S.poll(t)[1] for t in tickets]
    wall = time.perf_counter() - t0
    S.close()
    lat = np.array([r["finished"] - r["submitted"] for r in res]) * 1e3
    svc = np.array([r["finished"] - r["started"] for r in res]) * 1e3
    ok = sum(r["status"] == 0 for r in res)
    failed = [{"status": r["status"], "rows": r["n_rows"], "newton_iters": r["newton_iters"],
               "krylov_iters": r["cg_iters"], "residual": r["residual"]} for r in res if r["status"] != 0]
    return {"requests": n_requests, "arrival_rate_per_s": rate, "slots": slots, "completed_ok": int(ok),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "service_ms_mean": float(svc.mean()), "solves_per_s": ok / wall,
            "newton_iters_mean": float(np.mean([r["newton_iters"] for r in res]) / max(n_steps, 1)),
            "krylov_iters_mean": float(np.mean([r["cg_iters"] for r in res]) / max(n_steps, 1)),
            "rows_mean": float(np.mean([r["n_rows"] for r in res])),
            "setups_reused": int(sum(r["setup_reused"] for r in res)),
            "joined_mean": float(np.mean([r["joined"] for r in res])), "failed": failed, "workload": workload}


def make_fixture(N, density, seed):
    import fixtures as fx
    return fx.fixture_eps(N, density, (3, 5, 6), displace=0.05, seed=seed)


def cpu_baseline(F, budget_s, all_cores_s):
    """The FP64 oracle on this host: the whole-mesh classification and point allocation
    once, then the per-row path (points/basis of the row's cells, Gauss right-hand
    sides, TSVD weights, mass + stiffness row) on seeded sampled rows until the time
    budget is spent; extrapolated to all rows. BLAS is held to one thread. Then the same
    per-row path on all host cores (one process per core, row blocks) for all_cores_s.
    Returns (baseline entry, the sampled oracle rows)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        one, rows, glob = _cpu_baseline(F, budget_s)
    if all_cores_s > 0:
        one["all_cores"] = _cpu_all_cores(F, glob, all_cores_s)
    one["host_cores"] = os.cpu_count()
    return one, rows


COEF = {"mass": lambda x: 1 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1]),
        "stiffness": lambda x: 1 + 0.5 * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])}


def _cpu_baseline(F, budget_s):
    import oracle as O
    t0 = time.perf_counter()
    cls = O.classify(F)
    s = O.points_per_element(F, cls)
    glob = {"cls": cls, "s": s, "cells": O.cells(F, s)}
    t_glob = time.perf_counter() - t0
    rng = np.random.default_rng(7)
    order = rng.permutation(F["n_fn"])
    done, nnz, t_rows = 0, 0, 0.0
    rows = {}
    while t_rows < budget_s and done < len(order):
        batch = [int(i) for i in order[done:done + 20]]
        t1 = time.perf_counter()
        res, glob = O.sample_rows(F, batch, ("mass", "x", "y"), 1e-12, COEF, glob)
        t_rows += time.perf_counter() - t1
        done += len(batch)
        nnz += sum(2 * len(r["S"]) for r in res.values())
        rows.update({i: {"M": r["M"], "K": r["K"], "A": (r["A_mass"], r["A_x"], r["A_y"]), "x": r["x"]}
                     for i, r in res.items()})
    per_row = t_rows / done
    total_s = t_glob + per_row * F["n_fn"]
    total_nnz = nnz / done * F["n_fn"]
    return ({"value": total_nnz / total_s, "unit": "nnz/s", "cores": 1, "kind": "oracle",
             "sample": f"whole-mesh classification + point allocation ({t_glob:.1f} s) and {done} seeded "
                       f"rows of the per-row path ({t_rows:.1f} s), extrapolated to {F['n_fn']} rows; "
                       f"one Python thread, BLAS limited to one thread"}, rows, glob)


_WORKER = {}


def _rows_init(F, glob):
    _WORKER["F"], _WORKER["glob"] = F, glob


def _rows_worker(rows):
    import oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        res, _ = O.sample_rows(_WORKER["F"], rows, ("mass", "x", "y"), 1e-12, COEF, _WORKER["glob"])
    return sum(2 * len(r["S"]) for r in res.values())


def _cpu_all_cores(F, glob, budget_s):
    """The per-row path on every host core: row blocks of 20 handed to a process pool
    until budget_s of wall time has passed; nnz/s extrapolated to all rows as above."""
    import multiprocessing as mp
    cores = os.cpu_count() or 1
    rng = np.random.default_rng(11)
    order = [int(i) for i in rng.permutation(F["n_fn"])]
    blocks = [order[k:k + 20] for k in range(0, len(order), 20)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    nnz, rows_done = 0, 0
    with ctx.Pool(cores, initializer=_rows_init, initargs=(F, glob)) as pool:
        pending = [pool.apply_async(_rows_worker, (b,)) for b in blocks[:4 * cores]]
        nxt = 4 * cores
        while pending:
            r = pending.pop(0)
            nnz += r.get()
            rows_done += 20
            if time.perf_counter() - t0 < budget_s and nxt < len(blocks):
                pending.append(pool.apply_async(_rows_worker, (blocks[nxt],)))
                nxt += 1
        wall = time.perf_counter() - t0
        pool.terminate()
    rate_rows = rows_done / wall
    return {"value": nnz / rows_done * rate_rows, "unit": "nnz/s", "cores": cores,
            "sample": f"{rows_done} seeded rows of the per-row path in {wall:.1f} s on {cores} processes "
                      f"(BLAS one thread each); whole-mesh setup not included"}


def oracle_row_errors(rows, row_ptr, qptr, gpu_weights, outs):
    """Errors of the GPU matrices over the oracle's sampled rows, max |GPU - ref| / max |ref|
    per matrix, against two references: the oracle's rows end to end (its own weights: for
    stiffness this is dominated by the TSVD weights' conditioning, the same in every
    precision), and the oracle's contraction of Eqs. (9) and (11) with the GPU's FP64
    weights (the error of the contraction's arithmetic alone)."""
    ref_own, ref_gpu = {}, {}
    for i, r in rows.items():
        q0, q1 = qptr[i], qptr[i + 1]
        w0, wx, wy = (gpu_weights[f][q0:q1] for f in ("mass", "x", "y"))
        A0, Ax, Ay = r["A"]
        cm, ck = COEF["mass"](r["x"]), COEF["stiffness"](r["x"])
        ref_own[i] = (r["M"], r["K"])
        ref_gpu[i] = (A0 @ (cm * w0), Ax @ (ck * wx) + Ay @ (ck * wy))
    res = {}
    for name, (M, K) in outs.items():
        Mh, Kh = M.double().cpu().numpy(), K.double().cpu().numpy()
        e = {}
        for tag, ref in (("oracle", ref_own), ("oracle_with_gpu_weights", ref_gpu)):
            dm = dk = sm = sk = 0.0
            for i, (mo, ko) in ref.items():
                a, b = row_ptr[i], row_ptr[i + 1]
                dm, dk = max(dm, np.abs(Mh[a:b] - mo).max()), max(dk, np.abs(Kh[a:b] - ko).max())
                sm, sk = max(sm, np.abs(mo).max()), max(sk, np.abs(ko).max())
            e[tag] = {"M": dm / sm, "K": dk / sk}
        res[name] = e
    return res


def c1_context(budget_rows=None):
    """Config 1 (the half strip with one valence-5 and one valence-3 EP): the oracle's 4x4
    Gauss assembly in CPU seconds (basis evaluation included), and Gauss against WQ
    formation + assembly of the stiffness matrix with the basis (and WQ weights) computed
    ahead, both unfactored: the paper's comparison (Section 6.1) on the oracle."""
    import fixtures as fx
    import oracle as O
    from threadpoolctl import threadpool_limits
    F = fx.fixture_half_strip()
    with threadpool_limits(limits=1):
        R = O.setup(F, families=("mass", "x", "y"))
        cl = R["cells"]
        t0 = time.perf_counter()
        O.gq_matrices(F, cl)
        t_gq_full = time.perf_counter() - t0
        gd = O.gauss_data(F, cl)
        k = COEF["stiffness"]
        xq = O.point_values(R["data"], "x")
        t0 = time.perf_counter()
        O.gq_assemble(F, gd, "stiffness", k)
        t_gq = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.wq_assemble(F, R["pat"], R["data"], R["W"], "stiffness", k(xq))
        t_wq = time.perf_counter() - t0
    return {"mesh": f"half strip, {F['n_fn']} functions, valence-5 and valence-3 EP",
            "oracle_gq_assembly_s": t_gq_full, "stiffness_formation_s": {"gauss": t_gq, "wq": t_wq},
            "gauss_over_wq": t_gq / t_wq, "paper_gauss_over_wq": 9.0,
            "note": "one Python thread; both unfactored, basis and weights computed ahead"}


def measure_c3(W, torch, args, N=512, budget_s=20.0):
    """Config 3: biharmonic matrix B (Eq. 12, coefficient 1) on a 512 x 512 mesh with 0.5 %
    EPs of valence 3 and 5 (clamped problem: the outer two function layers are the
    prescribed ones; the matrix is formed on all rows). FP64 TSVD weights; the row
    contraction in FP64 and in the three low-precision forms, each timed (flushed caches)
    and compared with the FP64 oracle on seeded sampled rows."""
    import fixtures as fx
    import oracle as O
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    F = fx.fixture_eps(N, 0.005, (3, 5), displace=0.05, seed=3000)
    t_fix = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    mesh = W.Mesh(F)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pts = W.Points(mesh, want_laplacian=True, stream=stream)
    wts = W.Weights(mesh, pts, W.WQ_FAM_MASS | W.WQ_FAM_LAP, tau=1e-12, stream=stream)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    row_ptr = pts.get(W.ARR_ROW_PTR).cpu().numpy()
    flush = torch.empty(512 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    res, outs = {}, {}
    for pname, prec in (("fp64", W.WQ_FP64), ("fp16x2", W.WQ_SPLIT_FP16), ("bf16x3", W.WQ_SPLIT_BF16),
                        ("sliced_fp16", W.WQ_SLICED_FP16)):
        B = W.assemble_biharmonic(pts, wts, None, prec=prec, stream=stream)
        torch.cuda.synchronize()
        W.timing_enable(True)
        W.timings()
        for _ in range(10):
            flush.fill_(1.0)
            W.assemble_biharmonic(pts, wts, None, B, prec=prec, stream=stream)
        torch.cuda.synchronize()
        recs = [r for r in W.timings() if r[0].startswith("k_assemble")]
        W.timing_enable(False)
        ms = float(np.median([r[1] for r in recs]))
        e = {"kernel": recs[0][0], "ms": ms, "launches": 1, "work": float(recs[0][2])}
        res[pname] = {"median_ms": ms, "nnz_per_s": pts.nnz / (ms * 1e-3), "roofline": roofline_of(e["kernel"], e)}
        outs[pname] = B
    rows = {}
    with threadpool_limits(limits=1):
        cls = O.classify(F)
        s = O.points_per_element(F, cls)
        glob = {"cls": cls, "s": s, "cells": O.cells(F, s)}
        rng = np.random.default_rng(13)
        order = rng.permutation(F["n_fn"])
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < budget_s:
            batch = [int(i) for i in order[done:done + 10]]
            out, glob = O.sample_rows(F, batch, ("mass", "lap"), 1e-12, None, glob)
            rows.update({i: r["B"] for i, r in out.items()})
            done += len(batch)
    sc = max(np.abs(v).max() for v in rows.values())
    for pname, B in outs.items():
        Bh = B.double().cpu().numpy()
        d = max(np.abs(Bh[row_ptr[i]:row_ptr[i + 1]] - v).max() for i, v in rows.items())
        res[pname]["rel_err_vs_oracle_rows"] = d / sc
    return {"workload": f"biharmonic B (coefficient 1), {N}x{N} faces, 0.5% EPs of valence 3/5, clamped problem, "
                        "TSVD cutoff 1e-12", "n_rows": int(pts.n_rows), "nnz": int(pts.nnz),
            "n_points": int(pts.n_points), "fixture_s": t_fix, "setup_s": t_setup,
            "oracle_rows_compared": len(rows), "precisions": res, "solve_report": wts.report}


def measure_c4(W, torch, n_distinct=24, n_meshes=200, seed=4000):
    """Config 4: many independent meshes with N ~ U{16..128} faces per side and EP
    density ~ U(0.5 %, 2 %), mass + stiffness, through one batch (one set of setup launches,
    assembly replayed as one HIP graph). The meshes are drawn from a pool of n_distinct
    seeded meshes (generating each mesh in Python on the host is the limit here)."""
    import fixtures as fx
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    pool = []
    for j in range(n_distinct):
        N = 4 * int(rng.integers(4, 33))  # 16..128, divisible by 4 (EP templates)
        dens = float(rng.uniform(0.005, 0.02))
        pool.append(fx.fixture_eps(N, dens, (3, 5, 6), displace=0.05, seed=seed + j) if N >= 24
                    else fx.fixture_grid(N, displace=0.05, seed=seed + j))
    t_fix = time.perf_counter() - t0
    picks = rng.integers(0, n_distinct, n_meshes)
    meshes = [pool[int(i)] for i in picks]
    mask = W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = W.Batch(meshes).build(mask)
    Mb, Kb = W.assemble_mass_stiffness(B.points, B.weights)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    s = torch.cuda.Stream()
    B.graph_assemble(None, None, Mb, Kb, stream=s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(10):
        B.graph_assemble(None, None, Mb, Kb, stream=s)
    e1.record(s)
    e1.synchronize()
    g_ms = e0.elapsed_time(e1) / 10
    nnz = 2 * int(B.points.nnz)
    return {"workload": f"{n_meshes} meshes drawn from {n_distinct} distinct seeded meshes, N ~ U{{16..128}}, "
                        "EP density ~ U(0.5%, 2%), mass + stiffness, FP64",
            "sizes_distinct": sorted(int(F["n_fn"]) for F in pool), "fixture_s": t_fix, "rows": int(B.points.n_rows),
            "nnz_M_plus_K": nnz, "setup_to_matrices_s": t_setup, "nnz_per_s_setup_to_matrices": nnz / t_setup,
            "assembly_graph_ms": g_ms, "nnz_per_s_assembly": nnz / (g_ms * 1e-3), "solve_report": B.report}


def measure_gauss(W, torch, mesh, pts, wts, c, k, M, K, stream, flush, reps):
    """Element-wise 4 x 4 Gauss assembly (the comparison system) against row-wise WQ on the
    same mesh, pattern and coefficients (evaluated at each rule's own points), the basis at
    the quadrature points computed ahead for both (Section 6.1 times formation with basis
    evaluation excluded). Kernel times by the library's HIP events, caches flushed between
    repetitions; the paper's figure is the stiffness ratio, GQ / WQ (about 9 on its CPU)."""
    G = W.Gauss(mesh, pts, stream=stream)
    xg = G.x(stream).reshape(-1, 2)
    cg = (1 + 0.5 * torch.sin(2 * np.pi * xg[:, 0]) * torch.sin(2 * np.pi * xg[:, 1])).contiguous()
    kg = (1 + 0.5 * torch.cos(np.pi * xg[:, 0]) * torch.cos(np.pi * xg[:, 1])).contiguous()
    Mg = G.assemble(W.GQ_MASS, cg, stream=stream)
    Kg = G.assemble(W.GQ_STIFFNESS, kg, stream=stream)
    Kw = W.assemble_stiffness(pts, wts, k, stream=stream)
    torch.cuda.synchronize()

    def med(run, prefix):
        W.timing_enable(True)
        W.timings()
        for _ in range(reps):
            flush.fill_(1.0)
            run()
        torch.cuda.synchronize()
        recs = [r for r in W.timings() if r[0] == prefix]
        W.timing_enable(False)
        return float(np.median([r[1] for r in recs]))

    gm = med(lambda: G.assemble(W.GQ_MASS, cg, Mg, stream), "k_gq_assemble_mass")
    gk = med(lambda: G.assemble(W.GQ_STIFFNESS, kg, Kg, stream), "k_gq_assemble_stiffness")
    wk = med(lambda: W.assemble_stiffness(pts, wts, k, Kw, stream=stream), "k_assemble_stiffness")
    wmk = med(lambda: W.assemble_mass_stiffness(pts, wts, c, k, M, K, stream=stream), "k_assemble_mass_stiffness")
    out = {"gq_points": int(G.size), "wq_points": int(pts.n_points),
           "gq_ms": {"mass": gm, "stiffness": gk}, "wq_ms": {"stiffness": wk, "mass_stiffness": wmk},
           "ratio_gq_over_wq": {"stiffness": gk / wk, "mass_plus_stiffness": (gm + gk) / wmk},
           "rel_diff_wq_vs_gq": {"M": float((M - Mg).abs().max() / Mg.abs().max()),
                                 "K": float((K - Kg).abs().max() / Kg.abs().max())},
           "note": "GQ: one wave per Bezier cell, 16 x 16 local tiles on FP64 MFMA, FP64 atomics into CSR"}
    G.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--density", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=2000)
    ap.add_argument("--assembly-reps", type=int, default=30)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-all-cores", type=float, default=12.0, help="seconds of the all-cores oracle run (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--side-streams", type=int, default=4,
                    help="streams for the independent launches within one call in the timed steps (1: none)")
    ap.add_argument("--no-extra-forms", action="store_true", help="skip the batched and served measurements")
    ap.add_argument("--extra", default="", help="comma-separated extra workloads: c1, c3, c4")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the assembly shards by rows without communication; see the design notes)", flush=True)
        sys.exit(2)

    import torch
    import paper_2605_29334_amd.wq as W
    W.set_side_streams(args.side_streams)

    torch.cuda.set_device(0)
    print(f"[bench] generating fixture N={args.N}", file=sys.stderr, flush=True)
    F = make_fixture(args.N, args.density, args.seed)
    mesh = W.Mesh(F)
    stream = torch.cuda.current_stream()
    mask = W.WQ_FAM_MASS | W.WQ_FAM_DX | W.WQ_FAM_DY

    def step(coefs):
        pts = W.Points(mesh, stream=stream)
        wts = W.Weights(mesh, pts, mask, tau=1e-12, stream=stream)
        c, k = coefs if coefs is not None else (None, None)
        M, K = W.assemble_mass_stiffness(pts, wts, c, k, stream=stream)
        return pts, wts, M, K

    # coefficients (PDE data) at the points, resident in HBM before timing
    pts0 = W.Points(mesh, stream=stream)
    x = pts0.get(W.ARR_X).reshape(-1, 2)
    c = (1 + 0.5 * torch.sin(2 * np.pi * x[:, 0]) * torch.sin(2 * np.pi * x[:, 1])).contiguous()
    k = (1 + 0.5 * torch.cos(np.pi * x[:, 0]) * torch.cos(np.pi * x[:, 1])).contiguous()
    row_ptr = pts0.get(W.ARR_ROW_PTR).cpu().numpy()
    qptr = pts0.get(W.ARR_QPTR).cpu().numpy()
    n_i, r_i = np.diff(row_ptr), np.diff(qptr)
    nnz = int(row_ptr[-1])
    n_points = pts0.n_points
    sum_r = int(qptr[-1])
    pts0.close()
    del pts0

    live = None
    for _ in range(args.warmup):
        live = step((c, k))
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    live = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        live = None  # release the previous step's handles (device memory) inside the step
        live = step((c, k))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s ({args.side_streams} side streams)",
          file=sys.stderr, flush=True)
    # per-kernel records (HIP events on each launch's stream): the same steps again with
    # every launch on the step's stream, so that a record is the kernel's own time and not
    # shared with kernels of other size buckets running beside it
    W.set_side_streams(1)
    W.timing_enable(True)
    W.timings()
    for _ in range(args.steps):
        live = None
        live = step((c, k))
    torch.cuda.synchronize()
    recs = W.timings()
    W.timing_enable(False)
    W.set_side_streams(args.side_streams)

    per_kernel = aggregate(recs, args.steps)
    dom_name, dom = max(per_kernel.items(), key=lambda kv: kv[1]["ms"])
    roofline = roofline_of(dom_name, dom)
    roofline["launch_timing"] = ("a second pass of the timed steps with one launch at a time (side streams 1), "
                                 "so that each kernel's duration is its own")

    # assembly only (weights and basis resident; caches flushed between repetitions),
    # timed by the library's HIP events on the launch stream; FP64 and the low-precision
    # contractions, with the normwise error of each matrix against the FP64 result
    pts, wts, M, K = live
    flush = torch.empty(512 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    precisions = {"fp64": W.WQ_FP64, "fp16x2": W.WQ_SPLIT_FP16, "bf16x3": W.WQ_SPLIT_BF16,
                  "sliced_fp16": W.WQ_SLICED_FP16}
    by_prec = {}
    outs = {}
    for pname, prec in precisions.items():
        Mp, Kp = W.assemble_mass_stiffness(pts, wts, c, k, prec=prec, stream=stream)  # converts basis data once
        torch.cuda.synchronize()
        W.timing_enable(True)
        W.timings()
        for _ in range(args.assembly_reps):
            flush.fill_(1.0)
            W.assemble_mass_stiffness(pts, wts, c, k, Mp, Kp, prec=prec, stream=stream)
        torch.cuda.synchronize()
        arecs = [r for r in W.timings() if r[0].startswith("k_assemble_mass_stiffness")]
        W.timing_enable(False)
        a_ms = float(np.median([r[1] for r in arecs]))
        e = {"kernel": arecs[0][0], "ms": a_ms, "launches": 1, "work": float(arecs[0][2])}
        entry = {"median_ms": a_ms, "nnz_per_s": 2 * nnz / (a_ms * 1e-3), "roofline": roofline_of(e["kernel"], e)}
        if prec != W.WQ_FP64:
            entry["rel_err_vs_fp64"] = {
                "M": float((Mp.double() - M).abs().max() / M.abs().max()),
                "K": float((Kp.double() - K).abs().max() / K.abs().max())}
        outs[pname] = (Mp, Kp)
        by_prec[pname] = entry
    assembly = dict(by_prec["fp64"])
    assembly["precisions"] = by_prec
    gauss = measure_gauss(W, torch, mesh, pts, wts, c, k, M, K, stream, flush, args.assembly_reps)

    value = args.steps * 2 * nnz / elapsed
    out = {
        "metric": "assembled CSR nonzeros/sec, WQ plain vs mixed-prec at rel err ≤1e-6; p50/p99 latency",
        "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Poisson mass+stiffness, FP64 plain WQ, {args.N}x{args.N} faces, "
                               f"EP density {args.density} (valence 3/5/6), TSVD cutoff 1e-12",
                   "n_rows": int(len(n_i)), "nnz_per_matrix": nnz, "n_points": int(n_points),
                   "sum_r": sum_r, "weight_systems": int(3 * len(n_i)), "seed": args.seed},
        "roofline": roofline,
        "assembly_only": assembly,
        "gauss_comparison": gauss,
        "kernels_ms_per_step": {kname: round(e["ms_per_step"], 4) for kname, e in per_kernel.items()},
        "solve_report": wts.report,
        "structure": pts.info(),
    }
    if not args.no_extra_forms:
        print("[bench] batched form", file=sys.stderr, flush=True)
        pool = small_pool()
        out["batched"] = measure_batched(W, torch, pool, copies=4)
        print("[bench] served form (distinct meshes of 32..256 faces per side, no setup reuse)", file=sys.stderr,
              flush=True)
        spool, sizes = served_pool()
        desc = (f"pool of {len(spool)} distinct seeded meshes, N = {sizes} faces per side, 1% EPs; k = 1 + u^2, "
                "manufactured source, 1 step of dt 0.1 from T = 0, theta = 1, exact Newton tangent, ||R|| <= 1e-10; "
                "every request sets its domain up from scratch")
        out["served"] = measure_served(W, spool, n_requests=60, rate=200.0, slots=4, tangent=W.TANGENT_EXACT,
                                       reuse=False, workload=desc)
        cap = out["served"]["solves_per_s"]
        out["served_below_capacity"] = measure_served(
            W, spool, n_requests=40, rate=0.7 * cap, slots=4, seed=6, tangent=W.TANGENT_EXACT, reuse=False,
            workload="as 'served', arrivals at 0.7 x its measured throughput")
        out["served_joined"] = measure_served(
            W, spool, n_requests=60, rate=200.0, slots=4, tangent=W.TANGENT_EXACT, reuse=False, join=16,
            workload="as 'served', with joining: requests queued together run as one union of up to 16 meshes "
                     "and 32768 rows (shared launches for the setup and every Newton and Krylov step)")
        small = ("pool of 9 meshes (16..64 faces per side, grids and 2% EPs), k = 1 + u^2, manufactured source, "
                 "1 step of dt 0.1, exact tangent; every request sets its domain up from scratch")
        out["served_small"] = measure_served(W, pool, n_requests=64, rate=400.0, slots=4, tangent=W.TANGENT_EXACT,
                                             reuse=False, workload=small)
        out["served_small_joined"] = measure_served(
            W, pool, n_requests=64, rate=400.0, slots=4, tangent=W.TANGENT_EXACT, reuse=False, join=16,
            workload=small + "; joining: requests queued together run as one union of up to 16 meshes and 32768 rows")
        out["served_reuse"] = measure_served(
            W, pool, n_requests=40, rate=200.0, slots=4, n_steps=2, tangent=W.TANGENT_EXACT, reuse=True,
            workload="pool of 9 meshes (16..64 faces per side, grids and 2% EPs), 2 steps of dt 0.1, exact tangent; "
                     "a held setup of an identical domain is taken over")
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"], orows = cpu_baseline(F, args.cpu_budget, args.cpu_all_cores)
        gw = {f: wts.weights(b).cpu().numpy() for f, b in (("mass", W.WQ_FAM_MASS), ("x", W.WQ_FAM_DX),
                                                             ("y", W.WQ_FAM_DY))}
        errs = oracle_row_errors(orows, row_ptr, qptr, gw, outs)
        for pname, e in errs.items():
            out["assembly_only"]["precisions"][pname]["rel_err_vs_oracle_rows"] = e
        out["assembly_only"]["oracle_rows_compared"] = len(orows)
    extra = [e for e in args.extra.split(",") if e]
    if "c1" in extra:
        print("[bench] config 1 context", file=sys.stderr, flush=True)
        out["c1"] = c1_context()
    if "c3" in extra:
        print("[bench] config 3 (512^2 biharmonic)", file=sys.stderr, flush=True)
        out["c3"] = measure_c3(W, torch, args)
    if "c4" in extra:
        print("[bench] config 4 (batched meshes)", file=sys.stderr, flush=True)
        out["c4"] = measure_c4(W, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
