"""Continuous batching of descent steps over many meshes on one GPU.

A request asks for a number of preconditioned descent steps on its mesh.  The loop admits
arrived requests in arrival order while a slot and device memory are free (memory is
reserved by the library's own upper bound for the request, `tp_estimate_device_bytes`),
keeps each admitted mesh resident as a `tp_problem` (geometry, incidence, cotan matrix,
preconditioner and work arrays stay on the device between steps), and advances all
admitted meshes together, one step per round, with `tp_batch_step`: the same phase of
every mesh's step runs in shared launches.  A request leaves when its steps are done (or
one fails) and its memory and slot go to the next arrivals, so requests join and leave
between rounds while others are mid-flight.

Latencies: a step's latency is the time from the previous step's completion (for the
first step, from admission) to its completion; a request's latency is arrival to
completion of its last step.

`run_serial` is the reference: one request at a time in arrival order, steps taken with
the same library call on that mesh alone.

The loop is written against a small executor interface (estimate / create / step /
vertices / destroy) so that its scheduling can be tested without a GPU.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the run
    V: np.ndarray               # (nV, 3) float64
    F: np.ndarray               # (nF, 3) int32
    steps: int = 10


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    nF: int
    admitted: float = float("nan")
    finished: float = float("nan")
    step_done: List[float] = dataclasses.field(default_factory=list)
    energies: List[float] = dataclasses.field(default_factory=list)
    status: int = 0
    reserved_bytes: int = 0
    batch_sizes: List[int] = dataclasses.field(default_factory=list)
    vertices: Optional[np.ndarray] = None

    def step_latencies(self) -> List[float]:
        prev = self.admitted
        out = []
        for t in self.step_done:
            out.append(t - prev)
            prev = t
        return out


def count_components(F: np.ndarray, nV: int) -> int:
    """Connected components of the mesh's vertex graph (edges of the faces); vertices used
    by no face count as components of their own."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    F = np.asarray(F)
    r = np.concatenate([F[:, 0], F[:, 1]])
    c = np.concatenate([F[:, 1], F[:, 2]])
    G = sp.coo_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(nV, nV))
    return int(connected_components(G, directed=False)[0])


class GpuExecutor:
    """Executor over libtpsurf: one resident tp_problem per admitted request."""

    def __init__(self, params=None, opts=None, device="cuda"):
        import torch
        from . import tpsurf as tp

        self.torch, self.tp = torch, tp
        self.params = params if params is not None else tp.default_params()
        self.opts = opts if opts is not None else tp.step_opts()
        self.device = torch.device(device)
        tp.lib()

    def estimate(self, req: Request) -> int:
        deg = np.bincount(req.F.reshape(-1), minlength=req.V.shape[0]).max()
        ncon = int(bool(self.opts.constrain_area)) + int(bool(self.opts.constrain_volume))
        return self.tp.estimate_device_bytes(req.V.shape[0], req.F.shape[0], int(deg),
                                             count_components(req.F, req.V.shape[0]), self.params, ncon)

    def create(self, req: Request):
        V = self.torch.from_numpy(np.ascontiguousarray(req.V, dtype=np.float64)).to(self.device)
        F = self.torch.from_numpy(np.ascontiguousarray(req.F, dtype=np.int32)).to(self.device)
        return self.tp.Problem(V, F, self.params)

    def step(self, handles: Sequence) -> tuple:
        sts, reps = self.tp.batch_step(list(handles), self.opts)
        return sts, [r.E_new for r in reps]

    def vertices(self, h) -> np.ndarray:
        return h.vertices().cpu().numpy()

    def destroy(self, h):
        h.close()


def run(requests: Sequence[Request], executor, budget_bytes: int, max_active: int = 16,
        clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
        keep_vertices: bool = False, on_done: Optional[Callable[[Result], None]] = None,
        small_faces: Optional[int] = None, max_large: int = 2, lane_order: str = "alternate") -> List[Result]:
    """Continuous batching: admit by arrival, slot and memory; shared steps in rounds.

    With small_faces None every admitted mesh takes part in every shared step.  With
    small_faces set, meshes with more faces form a second lane whose round is one step of
    its oldest admitted mesh (first come, first served within the lane, so a large request
    is not slowed down by the large requests admitted after it); a small-lane round is one
    shared step of all admitted small meshes.  lane_order "alternate": the lanes take turns,
    so a small mesh's step never waits for more than one large step; "oldest": each round
    goes to the lane whose oldest admitted request arrived first, so requests are served in
    arrival order as on the serial path while the small ones that are due together share
    their steps.  Each lane admits in arrival order (small meshes may overtake large ones);
    memory is shared.
    """
    if lane_order not in ("alternate", "oldest"):
        raise ValueError("lane_order must be 'alternate' or 'oldest'")
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    results = {r.rid: Result(r.rid, r.arrival, int(r.F.shape[0])) for r in reqs}
    if small_faces is None:
        lanes = [{"pending": reqs, "limit": max_active, "one": False}]
    else:
        lanes = [{"pending": [r for r in reqs if r.F.shape[0] <= small_faces], "limit": max_active, "one": False},
                 {"pending": [r for r in reqs if r.F.shape[0] > small_faces], "limit": max_large, "one": True}]
    for ln in lanes:
        ln.update(qi=0, active=[], rr=0)
    used = 0
    turn = 0
    t0 = clock()

    def busy():
        return any(ln["qi"] < len(ln["pending"]) or ln["active"] for ln in lanes)

    while busy():
        now = clock() - t0
        # admission: each lane in arrival order; a request that does not fit waits
        for ln in lanes:
            pend, act = ln["pending"], ln["active"]
            while ln["qi"] < len(pend) and pend[ln["qi"]].arrival <= now and len(act) < ln["limit"]:
                req = pend[ln["qi"]]
                need = int(executor.estimate(req))
                res = results[req.rid]
                if need > budget_bytes:
                    res.status = -1            # larger than the whole budget: rejected
                    res.finished = now
                    ln["qi"] += 1
                    continue
                if used + need > budget_bytes:
                    break
                h = executor.create(req)
                used += need
                res.reserved_bytes = need
                res.admitted = clock() - t0
                act.append([req, h, 0])
                ln["qi"] += 1
        ready = [q for q, ln in enumerate(lanes) if ln["active"]]
        if not ready:
            nxt = [ln["pending"][ln["qi"]].arrival for ln in lanes if ln["qi"] < len(ln["pending"])]
            if nxt:
                sleep(max(0.0, min(nxt) - (clock() - t0)))
            continue
        if lane_order == "oldest":
            q = min(ready, key=lambda i: (lanes[i]["active"][0][0].arrival, lanes[i]["active"][0][0].rid))
        else:
            q = turn % len(lanes)
            if q not in ready:
                q = ready[0]
        turn = q + 1
        ln = lanes[q]
        if ln["one"]:
            batch = [ln["active"][0]]          # the oldest admitted large mesh
        else:
            batch = list(ln["active"])
        sts, energies = executor.step([a[1] for a in batch])
        t = clock() - t0
        gone = set()
        for a, st, e in zip(batch, sts, energies):
            req, h, _ = a
            res = results[req.rid]
            a[2] += 1
            res.step_done.append(t)
            res.energies.append(e)
            res.batch_sizes.append(len(batch))
            if st != 0 and st != 5:        # 5: CG not converged, step still taken
                res.status = st
            if a[2] >= req.steps or res.status != 0:
                res.finished = t
                if keep_vertices:
                    res.vertices = executor.vertices(h)
                executor.destroy(h)
                used -= res.reserved_bytes
                gone.add(id(a))
                if on_done:
                    on_done(res)
        if gone:
            ln["active"] = [a for a in ln["active"] if id(a) not in gone]
    return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def run_serial(requests: Sequence[Request], executor, clock: Callable[[], float] = time.perf_counter,
               sleep: Callable[[float], None] = time.sleep, keep_vertices: bool = False,
               on_done: Optional[Callable[[Result], None]] = None) -> List[Result]:
    """One request at a time in arrival order, each step on that mesh alone."""
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    results = {}
    t0 = clock()
    for req in pending:
        now = clock() - t0
        if req.arrival > now:
            sleep(req.arrival - now)
        res = Result(req.rid, req.arrival, int(req.F.shape[0]))
        h = executor.create(req)
        res.admitted = clock() - t0
        for _ in range(req.steps):
            sts, energies = executor.step([h])
            res.step_done.append(clock() - t0)
            res.energies.append(energies[0])
            res.batch_sizes.append(1)
            if sts[0] != 0 and sts[0] != 5:
                res.status = sts[0]
                break
        res.finished = res.step_done[-1] if res.step_done else clock() - t0
        if keep_vertices:
            res.vertices = executor.vertices(h)
        executor.destroy(h)
        results[req.rid] = res
        if on_done:
            on_done(res)
    return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summary(results: Sequence[Result]) -> dict:
    """Steps/s over the makespan, p50/p99 of step and request latency (ms)."""
    ok = [r for r in results if r.status == 0 and r.step_done]
    steps = sum(len(r.step_done) for r in ok)
    if not ok:
        return {"requests": 0, "steps": 0}
    start = min(r.arrival for r in ok)
    end = max(r.finished for r in ok)
    lat = np.array([x for r in ok for x in r.step_latencies()]) * 1e3
    req = np.array([r.finished - r.arrival for r in ok]) * 1e3
    bs = np.array([b for r in ok for b in r.batch_sizes], dtype=float)
    return {
        "requests": len(ok),
        "failed": sum(1 for r in results if r.status != 0),
        "steps": steps,
        "makespan_s": end - start,
        "steps_per_s": steps / max(end - start, 1e-12),
        "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                            "mean": float(lat.mean())},
        "request_latency_ms": {"p50": float(np.percentile(req, 50)), "p99": float(np.percentile(req, 99))},
        "mean_batch": float(bs.mean()),
    }
