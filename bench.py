"""Benchmark of the tangent-point hot path on one MI355X.

One step on the 40,000-face noisy torus (R = 1, r = 0.3, 200 x 100 grid, vertex noise
0.002 r, seed 0), with inputs resident in HBM:
  1. E and dE (all pairs, FP32 pair terms, FP64 accumulation),
  2. L^sigma u for u ~ N(0,1) in R^{V x 3} (all pairs),
  3. A~^{-1} dE = C^-1 L^sigma C^-1 dE: two FP64 CG Poisson solves (1e-10) around one more
     all-pairs fractional apply on 3 columns.
value = ordered face-pair interactions per second over the whole step (3 F (F - 1) per step).

Prints ONE JSON line (rank 0).  `--gpus N` with N > 1 exits: the path runs on one GPU.

`--copy-probe` instead runs a plain device-to-device copy of known size; its FETCH_SIZE
and WRITE_SIZE counter readings calibrate those counters for the traffic figure.
`--pairs-only` runs only the all-pairs launches of the step (E + dE and L^sigma u) and
prints their timings: a short program for hardware-counter passes (`--pairs-workload`
picks another workload for it, e.g. bumpy327k).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per ordered face pair (FMA = 2 FLOP, other arithmetic and
# transcendental = 1), counted from the formulas evaluated once per pair:
#   energy + differential: 57, fractional apply with k columns: 12 + 3 k.
FLOP_PER_PAIR_GRAD = 57.0
FLOP_PER_PAIR_ENERGY = 21.0
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the E + dE kernel on this workload, from one FETCH_SIZE and one
# WRITE_SIZE counter pass (`--pairs-only`), each scaled by what the same counter reads for
# a plain copy of known size (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00).  Reported only while
# the kernel's sources are the ones the passes measured.
GRAD_TRAFFIC = {
    "sources": ["paper_2107_01664_amd/csrc/tp_pairs.hip", "paper_2107_01664_amd/csrc/tp_tiles.h",
                "paper_2107_01664_amd/csrc/tp_internal.h", "paper_2107_01664_amd/csrc/tp_sym.h"],
    "sha256": "5c05e40fbf4863bb757f34705e256546ea9ba153b9480c4d6d93b914f5e60f9b",
    "fetch_bytes": int(58749.90625 * 1024) * 2,
    "write_bytes": 172543 * 1024,
}


def grad_traffic():
    import hashlib
    h = hashlib.sha256()
    try:
        for f in GRAD_TRAFFIC["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != GRAD_TRAFFIC["sha256"]:
        return None
    return GRAD_TRAFFIC["fetch_bytes"] + GRAD_TRAFFIC["write_bytes"]


def frac_flop_per_pair(k: float) -> float:
    return 12.0 + 3.0 * k


def sobolev_flop_per_pair(k: float) -> float:
    # d 3, |d|^2 5, r2^-s a_T 4, the low-order weight w (q_S^2 + q_T^2) / r2^2 17 (two dot
    # products, a reciprocal and five products / sums); per column 4 differences + 4 FMA
    return 29.0 + 12.0 * k


def sobolev_report(tp, P, u, launches: int = 10) -> dict:
    """A u = (B + B0) u (the inner product's operator) with the three columns of u, timed
    outside the step: the pair kernel by HIP events on its stream, the whole call by the
    host clock around synchronized calls."""
    import torch

    Au = torch.empty_like(u)
    for _ in range(2):
        P.sobolev_apply(u, out=Au)
    torch.cuda.synchronize()
    tp.profile_reset()
    tp.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(launches):
        P.sobolev_apply(u, out=Au)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tp.profile_enable(False)
    st = tp.profile_get(tp.KIND_SOBOLEV)
    n = max(1, st["launches"])
    ms = st["ms_total"] / n
    k = st["cols_total"] / max(1.0, st["pairs_total"])
    pairs = st["pairs_total"] / n
    tflops = sobolev_flop_per_pair(k) * pairs / (ms * 1e-3) / 1e12
    return {"avg_launch_ms": ms, "call_ms": 1e3 * wall / launches, "columns": k,
            "flop_per_pair": sobolev_flop_per_pair(k), "achieved_tflops": tflops,
            "frac": tflops / PEAK_FP32_VALU_TFLOPS, "pairs_per_s": pairs / (ms * 1e-3),
            "launches": int(st["launches"])}


def gmres_report(P, dE) -> dict:
    """x = A^+ P dE (the descent direction with the true operator A = B + B0) by GMRES to a
    relative residual of 1e-6, timed outside the step: once with the weighted diagonal
    term beside the paper's preconditioner, once with the paper's preconditioner alone
    (capped at 60 iterations)."""
    out = {}
    for name, pc, maxit in (("with_diagonal", 1, 300), ("paper_preconditioner", 0, 60)):
        _, rep = P.sobolev_solve(dE, rtol=1e-6, restart=50, maxiter=maxit, precond=pc, check=False)
        out[name] = {"iters": rep["iters"], "relres": rep["relres"], "ms": rep["t_ms"],
                     "converged": rep["status"] == 0, "precond_cg_iters": rep["precond_cg_iters"],
                     "omega": rep["omega"]}
    return out


def accuracy_report(tp, V, F, u, E, dE, Lu) -> dict:
    """Each result of the step's FP32 path against the FP64 path of the same library on the
    same inputs (FP64 pair terms; the GPU tests hold that path to the FP64 oracle)."""
    import numpy as np

    with tp.Problem(V, F, tp.default_params(precision=2)) as P64:
        E64, g64 = P64.gradient()
        L64 = P64.fractional_apply(u)
    g64, L64 = g64.cpu().numpy(), L64.cpu().numpy()
    dE, Lu = dE.cpu().numpy(), Lu.cpu().numpy()
    return {"reference": "fp64 pair terms on the GPU (held to the FP64 oracle by the GPU tests)",
            "E_rel": abs(E - E64) / abs(E64),
            "dE_rel": float(np.linalg.norm(dE - g64) / np.linalg.norm(g64)),
            "Lu_rel": float(np.linalg.norm(Lu - L64) / np.linalg.norm(L64))}


def descent_step_report(tp, V, F, steps: int = 4) -> dict:
    """The full descent step (tp_precond_step: E + dE, A~^{-1} on the 9 columns of
    [dE, J_A, J_V], Schur system, Armijo, corrective projection) on the bench mesh, with the
    Poisson solves started from zero and warm-started from the previous step."""
    import numpy as np

    out = {}
    for name, warm in (("cold", 0), ("warm_start", 1)):
        with tp.Problem(V, F) as P:
            reps = [P.step(tp.step_opts(warm_start=warm)) for _ in range(steps + 1)]
        later = reps[1:]
        out[name] = {"ms": float(np.mean([r.t_ms[6] for r in later])),
                     "precond_ms": float(np.mean([r.t_ms[2] for r in later])),
                     "cg_iters": [list(r.cg_iters) for r in later],
                     "warm_started": [int(r.warm_started) for r in later]}
    out["steps_timed"] = steps
    out["note"] = "device ms per step (the step's own events), steps 2..%d of a fresh problem" % (steps + 1)
    return out


def cpu_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


def cpu_one_core_rate(seconds: float = 3.0) -> float:
    """Ordered E + dE pair terms per second of the oracle on one core (a child process with
    OMP_NUM_THREADS=1, a band of rows of the bench mesh)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import oracle as O\n"
            "from paper_2107_01664_amd import meshgen as mg\n"
            "m = mg.workload('torus40k'); O.lib(); O.gradient_rows(m.V, m.F, 0, 4)\n"
            "t = time.perf_counter(); O.gradient_rows(m.V, m.F, 0, 16); dt = time.perf_counter() - t\n"
            "n = max(16, int(16 * %f / max(dt, 1e-6)))\n"
            "t = time.perf_counter(); O.gradient_rows(m.V, m.F, 0, n); dt = time.perf_counter() - t\n"
            "print(n * (m.nF - 1) / dt)\n") % (ROOT, seconds)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    return float(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 and r.stdout.strip() else float("nan")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", type=int, default=3,
                    help="0 fp32 hi/lo, 1 fp32, 2 fp64, 3 fp32 hi/lo + fp64 near field (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving comparison (0 skips it)")
    ap.add_argument("--serve-fmax", type=float, default=200000.0)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--serve-capacity-requests", type=int, default=96,
                    help="requests of the saturated serial pass that measures the serial capacity")
    ap.add_argument("--serve-lane-order", choices=["alternate", "oldest"], default="oldest",
                    help="batched path: lanes take turns, or the lane with the oldest request goes first")
    ap.add_argument("--serve-saturated", action="store_true",
                    help="also serve the whole mix batched with every request present at t = 0")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving comparison and print its JSON line")
    ap.add_argument("--sweep", action="store_true",
                    help="precision and Barnes-Hut sweep (bumpy sphere, linked tori) instead of the step")
    ap.add_argument("--pairs-only", action="store_true",
                    help="time only the all-pairs launches (E + dE, L^sigma u, and E alone; for counter passes)")
    ap.add_argument("--pairs-workload", default="torus40k",
                    help="workload of --pairs-only (a name known to meshgen.workload)")
    ap.add_argument("--large-solve", action="store_true",
                    help="time the preconditioned Poisson solve (9 columns) on a 163,842-vertex sphere, "
                         "the multi-launch path, against plain CG")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 256 MiB device copy 5 times (counter calibration)")
    return ap.parse_args()


def large_solve():
    """The Poisson solve of the preconditioner on a mesh of more blocks than one
    co-resident workgroup each: icosphere level 7 (163,842 vertices) with vertex noise 5e-4
    (seed 1), 9 random columns (seed 2), solved twice (the second timed) with the
    preconditioned and with plain CG."""
    import torch
    from paper_2107_01664_amd import meshgen as mg
    from paper_2107_01664_amd import tpsurf as tp
    m = mg.add_noise(mg.icosphere(7), 0.0005, 1)
    V = torch.from_numpy(m.V).cuda()
    F = torch.from_numpy(m.F).cuda()
    b = torch.from_numpy(mg.random_columns(m.nV, 9, 2)).cuda()
    out = {"large_solve": {"vertices": m.nV, "columns": 9}}
    for pc in (1, 0):
        with tp.Problem(V, F, tp.default_params(cg_precond=pc)) as P:
            for _ in range(2):
                _, r = P.poisson_solve(b)
        out["large_solve"]["preconditioned" if pc else "plain"] = {
            "iterations": int(r.cg_iters[0]), "relres": float(r.cg_relres[0]), "ms": float(r.t_ms[0])}
    print(json.dumps(out), flush=True)


def copy_probe():
    """A copy of known size: 256 MiB read and 256 MiB written per launch."""
    import torch

    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


def cpu_baseline(mesh, u, target_s: float):
    """The FP64 oracle timed on a bounded band of rows of the same step, scaled to the
    whole step: t_step = F (t_grad / n_g + 2 t_frac / n_f) + 2 t_poisson."""
    import numpy as np
    import oracle as O

    O.lib()
    nF = mesh.nF
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on bands wide enough to keep every thread busy (after one warm-up call),
    # then size the timed bands to about 80 % of target_s (the Poisson solve adds the rest)
    O.gradient_rows(mesh.V, mesh.F, 0, 64)
    t0 = time.perf_counter()
    O.gradient_rows(mesh.V, mesh.F, 0, 512)
    per_row_g = (time.perf_counter() - t0) / 512
    t0 = time.perf_counter()
    O.fractional_rows(mesh.V, mesh.F, u, 0, 512, 1.0 / 3.0)
    per_row_f = (time.perf_counter() - t0) / 512
    budget = max(1.0, 0.8 * target_s)
    n_g = int(min(nF, max(64, budget * 0.7 / per_row_g)))
    n_f = int(min(nF, max(64, budget * 0.3 / per_row_f)))
    t0 = time.perf_counter()
    O.gradient_rows(mesh.V, mesh.F, 0, n_g)
    t_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.fractional_rows(mesh.V, mesh.F, u, 0, n_f, 1.0 / 3.0)
    t_f = time.perf_counter() - t0
    C = O.cotan_laplacian(mesh.V, mesh.F)
    _, labels = O.components(mesh.F, mesh.nV)
    t0 = time.perf_counter()
    y = O.poisson_solve(C, u, labels)
    t_p = time.perf_counter() - t0
    t_step = nF * (t_g / n_g + 2.0 * t_f / n_f) + 2.0 * t_p
    pairs = 3.0 * nF * (nF - 1)
    return {
        "value": pairs / t_step,
        "unit": "tri-pair interactions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle E+dE rows [0,{n_g}) of {nF} ({t_g:.2f} s), L^sigma rows [0,{n_f}) k=3 "
                   f"({t_f:.2f} s), one sparse direct Poisson solve k=3 ({t_p:.2f} s); step time "
                   f"extrapolated over all {nF} rows, 2 fractional applies, 2 solves = {t_step:.1f} s"),
        "est_step_s": t_step,
    }


def pcg_report(n: int, k: int, cg_ms, iters) -> dict:
    """The preconditioned CG launches, the largest share of the step: time per iteration and
    the algorithmic HBM bytes of one iteration (the block solves written and read once,
    8 n k each; block sums and partial dot products, 64 nb k), against the HBM peak."""
    nb = -(-n // 128)
    it = max(1, sum(iters))
    us = 1e3 * sum(cg_ms) / it
    bytes_it = 16.0 * n * k + 64.0 * nb * k
    gbs = bytes_it / (us * 1e-6) / 1e9
    return {"bound": "grid-barrier latency (two grid-wide exchanges per iteration)",
            "us_per_iteration": us, "hbm_bytes_per_iteration": bytes_it, "achieved_GBs": gbs,
            "peak_GBs": PEAK_HBM_GBS, "frac_hbm": gbs / PEAK_HBM_GBS}


def _timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return out, best * 1e3


def sweep():
    """E and dE of the 327,680-face bumpy sphere (icosphere level 7, harmonic bumps l <= 8,
    amplitude 0.05) in every variant against the FP64 direct sums on the GPU (which the GPU
    tests hold to the oracle at sampled vertices of the same mesh), and direct vs
    Barnes-Hut on the linked tori (51,200 faces).  Times are wall time of one synchronous
    E + dE call and of one E call (best of 3 each)."""
    import numpy as np
    import torch
    from paper_2107_01664_amd import meshgen as mg
    from paper_2107_01664_amd import tpsurf as tp

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    report = {}
    for wname in ("bumpy327k", "linked_tori"):
        m = mg.workload(wname)
        V = torch.from_numpy(m.V).cuda()
        F = torch.from_numpy(m.F).cuda()
        rows = {}
        ref = None
        variants = [("fp64 direct", dict(precision=2)),
                    ("fp32 direct, fp32 accumulation (naive)", dict(precision=4)),
                    ("fp32 direct, kahan fp32 accumulation", dict(precision=5)),
                    ("fp32 direct, fp64 accumulation", dict(precision=1)),
                    ("fp32 hi/lo direct, fp64 accumulation", dict(precision=0)),
                    ("fp32 hi/lo direct + fp64 near field (default)", dict(precision=3)),
                    ("barnes-hut theta=0.5 fp32", dict(precision=0, theta=0.5)),
                    ("barnes-hut theta=0.25 fp32", dict(precision=0, theta=0.25)),
                    ("barnes-hut theta=0.5 fp64", dict(precision=2, theta=0.5))]
        for name, kw in variants:
            with tp.Problem(V, F, tp.default_params(**kw)) as P:
                (E, g), ms = _timed(lambda: P.gradient())
                g = g.cpu().numpy()
                terms = P.bh_stats() if kw.get("theta") else None
                _, ms_e = _timed(lambda: P.energy())
            if ref is None:
                ref = (E, g)
                rows[name] = {"E": E, "ms": ms, "energy_only_ms": ms_e}
                print(f"[sweep] {wname} {name}: {ms:.1f} ms", file=sys.stderr, flush=True)
                continue
            r = {"E": E, "ms": ms, "energy_only_ms": ms_e, "E_rel_err": abs(E - ref[0]) / ref[0],
                 "dE_rel_err": rel(g, ref[1])}
            if terms:
                r["terms_far_near"] = list(terms)
            rows[name] = r
            print(f"[sweep] {wname} {name}: {ms:.1f} ms (E alone {ms_e:.1f} ms), E {r['E_rel_err']:.2e}, "
                  f"dE {r['dE_rel_err']:.2e}",
                  file=sys.stderr, flush=True)
        report[wname] = {"faces": m.nF, "pairs": float(m.nF) * (m.nF - 1), "variants": rows}
        # the fractional operator L^sigma u (3 random columns): direct sums, Barnes-Hut on the
        # kernel matrix and the block cluster tree's hierarchical product, against the FP64
        # direct sums; times of one synchronous call (best of 3)
        u = torch.from_numpy(mg.random_columns(m.nV, 3, 1)).cuda()
        frows, fref = {}, None
        fvariants = [("fp64 direct", dict(precision=2)), ("fp32 hi/lo direct", dict(precision=3)),
                     ("barnes-hut theta=0.5 fp32", dict(precision=0, theta=0.5)),
                     ("block cluster tree chi=0.5 fp32", dict(precision=0, chi=0.5)),
                     ("block cluster tree chi=0.25 fp32", dict(precision=0, chi=0.25))]
        for name, kw in fvariants:
            with tp.Problem(V, F, tp.default_params(**kw)) as P:
                L, ms = _timed(lambda: P.fractional_apply(u))
                L = L.cpu().numpy()
                blocks = P.bct_stats() if kw.get("chi") else None
            if fref is None:
                fref = L
                frows[name] = {"ms": ms}
            else:
                frows[name] = {"ms": ms, "Lu_rel_err": rel(L, fref)}
                if blocks:
                    frows[name]["blocks_admissible_inadmissible"] = list(blocks)
            print(f"[sweep] {wname} L^sigma u {name}: {ms:.1f} ms", file=sys.stderr, flush=True)
        report[wname]["fractional_apply"] = frows
    return report


def _build(spec):
    from paper_2107_01664_amd import meshgen as mg
    m = mg.build_request_mesh(spec)
    return m.V, m.F


def serving_meshes(n_req: int, fmax: float, steps: int, seed: int = 0, workers: int = 1):
    """Request specs and meshes; with workers > 1 the meshes are built in forked worker
    processes, which must happen before this process touches the GPU."""
    from paper_2107_01664_amd import meshgen as mg
    specs = mg.serving_requests(n_req, seed, 2000.0, fmax, steps)
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            built = pool.map(_build, specs)
    else:
        built = [_build(sp) for sp in specs]
    return specs, built


def serving_bench(specs, built, steps: int, fmax: float, seed: int = 0, load: float = 0.8,
                  max_active: int = 16, small_faces: int = 32768, max_large: int = 2,
                  verbose: bool = False, capacity_requests: int = 0, saturated: bool = True,
                  lane_order: str = "oldest"):
    """Continuous batching against the serial one-mesh-at-a-time path on the same requests:
    noisy icospheres / tori with F log-uniform in [2,000, fmax], `steps` descent steps
    each.  The serial path first runs with every request present at t = 0 -- the whole mix,
    or its first `capacity_requests` requests -- which gives its capacity (requests/s); with
    `saturated` the batched path is run the same way on the whole mix.  Both paths then
    serve the whole mix with Poisson arrivals at `load` x that capacity."""
    import numpy as np
    from paper_2107_01664_amd import meshgen as mg
    from paper_2107_01664_amd import serve

    n_req = len(specs)

    def requests(arrivals):
        return [serve.Request(sp["id"], float(t), V, F.astype(np.int32), steps)
                for sp, (V, F), t in zip(specs, built, arrivals)]

    def progress(tag):
        def f(r):
            print(f"[serve] {tag} request {r.rid} nF={r.nF} steps={len(r.step_done)} "
                  f"done at {r.finished:.2f} s", file=sys.stderr, flush=True)
        return f if verbose else None

    ex = serve.GpuExecutor()
    serve.run_serial(requests(np.zeros(1))[:1], ex)                  # warm-up
    zero = np.zeros(n_req)
    n_cap = n_req if capacity_requests <= 0 else min(n_req, capacity_requests)
    sat_ser = serve.run_serial(requests(zero)[:n_cap], ex, on_done=progress("saturated serial"))
    lanes = dict(small_faces=small_faces, max_large=max_large, lane_order=lane_order)
    sat_bat = (serve.run(requests(zero), ex, budget_bytes=200 << 30, max_active=max_active,
                         on_done=progress("saturated batched"), **lanes) if saturated else None)
    # the batched path saturated on the same sample as the serial capacity pass
    sample_bat = (serve.run(requests(zero)[:n_cap], ex, budget_bytes=200 << 30, max_active=max_active,
                            on_done=progress("saturated batched sample"), **lanes)
                  if not saturated and n_cap < n_req else None)
    cap = n_cap / max(serve.summary(sat_ser)["makespan_s"], 1e-9)      # requests/s
    rate = load * cap
    arr = mg.poisson_arrivals(n_req, rate, seed + 1)
    bat = serve.run(requests(arr), ex, budget_bytes=200 << 30, max_active=max_active,
                    keep_vertices=True, on_done=progress("poisson batched"), **lanes)
    ser = serve.run_serial(requests(arr), ex, keep_vertices=True, on_done=progress("poisson serial"))
    same = all(np.array_equal(a.vertices, b.vertices) for a, b in zip(bat, ser))
    nf = np.array([sp["nF"] for sp in specs], dtype=float)
    sb, ss = serve.summary(bat), serve.summary(ser)
    out = {
        "workload": (f"{n_req} requests, noisy icosphere/torus, F log-uniform in [2000, {int(fmax)}] "
                     f"(mean {nf.mean():.0f}), {steps} preconditioned steps each (FP32 pair terms, FP64 CG, "
                     f"area + volume constraints, Armijo), Poisson arrivals at {load} x serial capacity "
                     f"({rate:.2f} requests/s); batched path: meshes of up to {small_faces} faces share "
                     f"steps ({max_active} at most), larger ones ({max_large} admitted at most) step "
                     f"oldest first, one at a time; " +
                     ("lanes take turns" if lane_order == "alternate" else
                      "each round goes to the lane whose oldest request arrived first")),
        "serial_capacity_req_per_s": cap,
        "serial_capacity_sample": (f"saturated serial pass over requests 0..{n_cap - 1} "
                                   f"({serve.summary(sat_ser)['makespan_s']:.1f} s)"),
        "batched": sb,
        "serial": ss,
        "steps_per_s": {"batched": sb["steps_per_s"], "serial": ss["steps_per_s"]},
        "request_latency_p99_ms": {"batched": sb["request_latency_ms"]["p99"],
                                   "serial": ss["request_latency_ms"]["p99"]},
        "all_requests_identical_to_serial": bool(same),
    }
    if sat_bat is not None:
        out["saturated"] = {"batched": serve.summary(sat_bat),
                            "serial": serve.summary(sat_ser), "note": "serial: the capacity sample"}
    if sample_bat is not None:
        out["saturated_sample"] = {"requests": n_cap, "batched": serve.summary(sample_bat),
                                   "serial": serve.summary(sat_ser),
                                   "steps_per_s": {"batched": serve.summary(sample_bat)["steps_per_s"],
                                                   "serial": serve.summary(sat_ser)["steps_per_s"]}}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the path runs on one GPU; --gpus {a.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    serve_mesh = None
    if a.serve_requests > 0 and not (a.sweep or a.pairs_only or a.copy_probe or a.large_solve):
        # build the request meshes in worker processes before any GPU use
        serve_mesh = serving_meshes(a.serve_requests, a.serve_fmax, a.serve_steps,
                                    workers=min(16, os.cpu_count() or 1))

    import numpy as np
    import torch
    from paper_2107_01664_amd import meshgen as mg
    from paper_2107_01664_amd import tpsurf as tp

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.copy_probe:
        copy_probe()
        return
    if a.large_solve:
        large_solve()
        return
    if a.sweep:
        print(json.dumps(sweep()), flush=True)
        return
    tp.lib()
    if a.serve_only:
        print(json.dumps(serving_bench(*serve_mesh, a.serve_steps, a.serve_fmax, verbose=True,
                                       capacity_requests=a.serve_capacity_requests,
                                       saturated=a.serve_saturated, lane_order=a.serve_lane_order)), flush=True)
        return
    dev = torch.device("cuda", 0)
    mesh = mg.workload(a.pairs_workload if a.pairs_only else "torus40k")
    u_np = mg.random_columns(mesh.nV, 3, 1)
    V = torch.from_numpy(mesh.V).to(dev)
    F = torch.from_numpy(mesh.F).to(dev)
    u = torch.from_numpy(u_np).to(dev)
    nF = mesh.nF
    params = tp.default_params(precision=a.precision)
    P = tp.Problem(V, F, params)
    dE = torch.empty((mesh.nV, 3), dtype=torch.float64, device=dev)
    Lu = torch.empty_like(u)
    x = torch.empty_like(dE)

    def step():
        # a descent step sees new vertex positions: the face data, the cotan Laplacian's
        # values, the preconditioner's block and coarse inverses and the near-field grid
        # are all formed again from them
        P.set_vertices(V)
        E, _ = P.gradient(out=dE)
        P.fractional_apply(u, out=Lu)
        _, rep = P.precond_apply(dE, out=x)
        return E, rep

    if a.pairs_only:
        for _ in range(a.warmup):
            P.gradient(out=dE)
            P.fractional_apply(u, out=Lu)
            P.energy()
        torch.cuda.synchronize()
        tp.profile_reset()
        tp.profile_enable(True)
        for _ in range(a.steps):
            P.gradient(out=dE)
            P.fractional_apply(u, out=Lu)
            P.energy()
        torch.cuda.synchronize()
        tp.profile_enable(False)
        g, f = tp.profile_get(tp.KIND_GRAD), tp.profile_get(tp.KIND_FRAC)
        e = tp.profile_get(tp.KIND_ENERGY)
        print(json.dumps({"pairs_only": True, "faces": nF, "grad_launches": g["launches"],
                          "grad_avg_ms": g["ms_total"] / max(1, g["launches"]),
                          "frac_launches": f["launches"], "frac_avg_ms": f["ms_total"] / max(1, f["launches"]),
                          "energy_launches": e["launches"], "energy_avg_ms": e["ms_total"] / max(1, e["launches"])}),
              flush=True)
        P.close()
        return

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    tp.profile_reset()
    tp.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(a.steps):
        E, rep = step()
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tp.profile_enable(False)
    ms_per_step = 1e3 * wall / a.steps
    pairs_per_step = 3.0 * nF * (nF - 1)
    value = pairs_per_step * a.steps / wall

    g = tp.profile_get(tp.KIND_GRAD)
    f = tp.profile_get(tp.KIND_FRAC)
    grad_ms = g["ms_total"] / max(1, g["launches"])
    grad_tflops = FLOP_PER_PAIR_GRAD * (g["pairs_total"] / max(1, g["launches"])) / (grad_ms * 1e-3) / 1e12
    kfrac = f["cols_total"] / max(1.0, f["pairs_total"])
    frac_ms = f["ms_total"] / max(1, f["launches"])
    frac_tflops = frac_flop_per_pair(kfrac) * (f["pairs_total"] / max(1, f["launches"])) / (frac_ms * 1e-3) / 1e12
    cg_ms = [float(np.mean([r.t_ms[0] for r in reps])), float(np.mean([r.t_ms[2] for r in reps]))]
    sob = sobolev_report(tp, P, u)
    gm = gmres_report(P, dE)
    P.gradient(out=dE)
    P.fractional_apply(u, out=Lu)
    acc = accuracy_report(tp, V, F, u, E, dE, Lu)
    dstep = descent_step_report(tp, V, F)

    out = {
        "metric": "tri-pair interactions/s (E+dE, H-apply) vs FP32 roofline; served steps/s + p99",
        "value": value,
        "unit": "tri-pair interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "fp32", 1: "fp32", 2: "f64", 3: "fp32"}[a.precision],
        "data": "synthetic",
        "config": {
            "workload": ("torus40k: torus R=1 r=0.3 on a 200x100 grid (40,000 faces), vertex noise "
                         "0.002 r seed 0; per step: vertex positions set (face data, cotan "
                         "Laplacian values, preconditioner set-up and near-field grid formed "
                         "again), E+dE, L^sigma u (u~N(0,1), k=3), and C^-1 L^sigma C^-1 dE with "
                         "two FP64 CG solves to 1e-10"),
            "faces": nF,
            "vertices": mesh.nV,
            "alpha": 6, "beta": 12, "sigma": 1.0 / 3.0,
            "precision": {0: "fp32 pair terms, hi/lo barycenters, fp64 accumulation",
                          1: "fp32 pair terms, fp64 accumulation",
                          2: "fp64 pair terms",
                          3: "fp32 pair terms, hi/lo barycenters, fp64 accumulation; pairs closer "
                             "than 2 mean edge lengths in fp64"}[a.precision],
            "pairs_per_step": pairs_per_step,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "all-pairs energy + differential (k_grad32_sym: each unordered pair once, for both rows)",
            "achieved": grad_tflops,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": grad_tflops / PEAK_FP32_VALU_TFLOPS,
            "traffic": grad_traffic(),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "flop_per_pair": FLOP_PER_PAIR_GRAD,
            "avg_launch_ms": grad_ms,
            "launches": g["launches"],
            "pairs_per_s": (g["pairs_total"] / max(1, g["launches"])) / (grad_ms * 1e-3),
        },
        "kernels": {
            "fractional_apply": {
                "avg_launch_ms": frac_ms, "columns": kfrac, "flop_per_pair": frac_flop_per_pair(kfrac),
                "achieved_tflops": frac_tflops, "frac": frac_tflops / PEAK_FP32_VALU_TFLOPS,
                "pairs_per_s": (f["pairs_total"] / max(1, f["launches"])) / (frac_ms * 1e-3),
            },
            "sobolev_apply": sob,
            "sobolev_solve": gm,
            "cg_ms": {"solve1": cg_ms[0], "solve2": cg_ms[1]},
            "cg_iters": [int(reps[-1].cg_iters[0]), int(reps[-1].cg_iters[1])],
            "pcg": pcg_report(mesh.nV, 3, cg_ms, [int(reps[-1].cg_iters[0]), int(reps[-1].cg_iters[1])]),
        },
        "energy": E,
        "accuracy_vs_fp64": acc,
        "descent_step": dstep,
    }
    P.close()
    if serve_mesh is not None:
        out["serving"] = serving_bench(*serve_mesh, a.serve_steps, a.serve_fmax, verbose=True,
                                       capacity_requests=a.serve_capacity_requests,
                                       saturated=a.serve_saturated, lane_order=a.serve_lane_order)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, u_np, a.cpu_seconds)
        out["cpu_baseline"].update(cpu_info())
        one = cpu_one_core_rate()
        out["cpu_baseline"]["one_core_pairs_per_s"] = one
        out["cpu_baseline"]["one_core_note"] = ("ordered E + dE pair terms per second of the oracle on one "
                                                "core (OMP_NUM_THREADS=1), a band of rows of the same mesh")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
