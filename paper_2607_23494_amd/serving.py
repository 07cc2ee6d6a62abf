"""Serving loop for the field-window estimator: continuous batching of
statistics requests on one GPU.

A request carries a catalogue (positions, optional weights), a box size, a
grid size and a set of statistics (2PCF, 2PCF multipoles, 3PCF multipoles,
counts-in-cells moments) with a contraction precision.  The loop

  * admits a waiting request as soon as a worker slot is free and the
    request's device-memory model fits the HBM budget that is left, in
    arrival order with backfilling: a later request that fits may pass a head
    that does not, until the head has waited longer than an age bound, after
    which nothing passes it (a request larger than the whole budget is
    rejected);
  * runs it on the slot's own HIP stream: assignment and FFT once, then every
    requested statistic on the resident contrast spectrum, so requests on
    different slots overlap on the device;
  * keeps reconstructed fields resident in a byte-bounded LRU cache keyed by
    catalogue, so a later request on the same catalogue skips assignment and
    FFT;
  * frees the request's memory on completion and admits the next request at
    once, recording arrival, admission and completion times.

The admission controller and the memory model are plain host code and can
run without a GPU (the workspace sizes are injected).
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Callable

import numpy as np

STAT_KINDS = ("xi", "xi_ell", "zeta", "cic")


@dataclasses.dataclass
class Request:
    rid: int
    pos: np.ndarray                       # float32 [n, 3] host positions
    box_L: float
    n_grid: int
    stats: dict                           # kind -> parameters (see run_stat)
    precision: str = "bf16x3"
    weight: np.ndarray | None = None
    arrival: float = 0.0                  # seconds after the start of the run
    catalogue_id: str | None = None       # enables the resident-field cache


@dataclasses.dataclass
class Result:
    rid: int
    status: str                           # "ok" | "rejected" | "error"
    message: str = ""
    arrival: float = 0.0
    admit: float = float("nan")
    finish: float = float("nan")
    nbytes: int = 0
    cached_field: bool = False
    outputs: dict = dataclasses.field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


# ----------------------------------------------------------------------------
# memory model and admission (host only)
# ----------------------------------------------------------------------------

def field_bytes(n_grid: int) -> int:
    """Resident field of one catalogue: float32 contrast + complex64 half spectrum."""
    return n_grid ** 3 * 4 + n_grid * n_grid * (n_grid // 2 + 1) * 8


def request_bytes(req: Request, ws_fn: Callable[[str, int, dict], int]) -> int:
    """Device bytes a request holds while it runs: its catalogue, the
    assignment grid, the resident field, the largest workspace (assignment
    and statistics run one after another on the request's stream) and
    outputs.  ws_fn(kind, n_grid, params) returns the workspace bytes of the
    assignment (kind "assign", params {"n_pts"}) or of a statistic."""
    n = req.n_grid
    cat = req.pos.shape[0] * 12 + (req.pos.shape[0] * 4 if req.weight is not None else 0)
    # the assignment's workspace and the statistics' are used one after another
    work = max([ws_fn(k, n, p) for k, p in req.stats.items()] + [ws_fn("assign", n, {"n_pts": req.pos.shape[0]})])
    outputs = 0
    for k, p in req.stats.items():
        if k == "cic":
            outputs += len(p["windows"]) * 24
            continue
        nb = len(p["edges"]) - 1
        if k == "zeta":
            outputs += (p["l_max"] + 1) * nb * nb * 8
        else:
            outputs += len(p.get("ells", (0,))) * nb * 8
    return cat + n ** 3 * 4 + field_bytes(n) + work + outputs


def pick_next(waiting_sizes: list[int], head_wait: float, adm: "Admission", bypass_age: float):
    """Index of the next waiting request to admit, or None.  The queue is in
    arrival order; the head goes first if it fits, otherwise the first later
    request that fits passes it, unless the head has already waited longer
    than bypass_age (then the queue waits for the head)."""
    if not waiting_sizes:
        return None
    if adm.fits(waiting_sizes[0]):
        return 0
    if head_wait > bypass_age:
        return None
    for i in range(1, len(waiting_sizes)):
        if adm.fits(waiting_sizes[i]):
            return i
    return None


class Admission:
    """Slot and HBM-budget bookkeeping."""

    def __init__(self, budget_bytes: int, slots: int):
        if budget_bytes <= 0 or slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.used = 0
        self.active = 0

    def oversized(self, nbytes: int) -> bool:
        return nbytes > self.budget

    def fits(self, nbytes: int) -> bool:
        return self.active < self.slots and self.used + nbytes <= self.budget

    def admit(self, nbytes: int) -> None:
        if not self.fits(nbytes):
            raise RuntimeError("admission beyond the slot or memory budget")
        self.used += nbytes
        self.active += 1

    def release(self, nbytes: int) -> None:
        self.used -= nbytes
        self.active -= 1
        if self.used < 0 or self.active < 0:
            raise RuntimeError("release without admission")


def schedule(arrivals: list[tuple[float, int]], service: dict[int, float], sizes: dict[int, int],
             adm: Admission, bypass_age: float = 0.0) -> dict[int, tuple[float, float]]:
    """Discrete-event simulation of the admission policy with given service
    times (host only; used to test the policy).  bypass_age = 0 is strict
    first come, first served.  Returns rid -> (admit, finish) for admitted
    requests; oversized ones are absent."""
    waiting = []
    running = []          # (finish, rid)
    out = {}
    arrived = {}
    events = sorted(arrivals)
    i = 0
    now = 0.0
    while i < len(events) or waiting or running:
        while True:
            head_wait = now - arrived[waiting[0]] if waiting else 0.0
            j = pick_next([sizes[r] for r in waiting], head_wait, adm, bypass_age)
            if j is None:
                break
            rid = waiting.pop(j)
            adm.admit(sizes[rid])
            running.append((now + service[rid], rid))
            out[rid] = (now, now + service[rid])
        t_arr = events[i][0] if i < len(events) else float("inf")
        t_fin = min(running)[0] if running else float("inf")
        if t_arr == float("inf") and t_fin == float("inf"):
            break   # waiting requests that can never fit (cannot happen after the oversize check)
        if t_arr <= t_fin:
            now = t_arr
            rid = events[i][1]
            i += 1
            if not adm.oversized(sizes[rid]):
                waiting.append(rid)
                arrived[rid] = now
        else:
            now = t_fin
            running.sort()
            _, rid = running.pop(0)
            adm.release(sizes[rid])
    return out


# ----------------------------------------------------------------------------
# GPU execution
# ----------------------------------------------------------------------------

def _workspace_fn(device: int):
    from . import hermes
    import torch

    def ws(kind, n, p):
        if kind == "assign":
            return hermes.workspace_size(hermes.OP_ASSIGN, n, torch.float32, int(p["n_pts"]), 1, device)
        if kind in ("xi", "xi_ell"):
            nb = len(p["edges"]) - 1
            return hermes.workspace_size(hermes.OP_XI, n, torch.float32, nb, len(p.get("ells", (0,))), device)
        if kind == "zeta":
            return hermes.workspace_size(hermes.OP_ZETA, n, torch.float32, len(p["edges"]) - 1, 1, device)
        if kind == "cic":
            return hermes.workspace_size(hermes.OP_FILTER, n, torch.float32, len(p["windows"]), 1, device)
        raise ValueError(f"unknown statistic {kind}")
    return ws


def run_stat(kind: str, p: dict, req: Request, dk, delta, stream):
    """One statistic on a resident field; returns a device tensor."""
    from . import hermes
    if kind in ("xi", "xi_ell"):
        return hermes.xi(dk, req.box_L, p["edges"], ells=p.get("ells", (0,)), los_axis=p.get("los", 2),
                         stream=stream)
    if kind == "zeta":
        return hermes.zeta_l(delta, dk, req.box_L, p["edges"], p["l_max"], precision=req.precision, stream=stream)
    if kind == "cic":
        return hermes.filter_bins(dk, req.box_L, p["windows"], store_fields=False, moments=True, stream=stream)[1]
    raise ValueError(f"unknown statistic {kind}")


class FieldCache:
    """Resident fields (delta, delta^) keyed by catalogue, LRU within a byte budget."""

    def __init__(self, max_bytes: int):
        self.max_bytes = int(max_bytes)
        self.used = 0
        self.lock = threading.Lock()
        self.entries: collections.OrderedDict = collections.OrderedDict()

    def get(self, key):
        with self.lock:
            e = self.entries.get(key)
            if e is not None:
                self.entries.move_to_end(key)
            return e

    def put(self, key, value, nbytes: int) -> None:
        if nbytes > self.max_bytes:
            return
        with self.lock:
            if key in self.entries:
                return
            while self.used + nbytes > self.max_bytes and self.entries:
                _, (_, old) = self.entries.popitem(last=False)
                self.used -= old
            self.entries[key] = (value, nbytes)
            self.used += nbytes


class Server:
    """Continuous-batching request loop on one device.

    budget_bytes bounds the memory of admitted requests; cache_bytes (taken
    from the same device, outside that budget) holds resident fields; every
    slot owns one HIP stream at the default priority."""

    def __init__(self, device: int = 0, budget_bytes: int = 200 << 30, slots: int = 4,
                 cache_bytes: int = 0, bypass_age: float = 1.0):
        import torch
        self.device = device
        self.bypass_age = float(bypass_age)
        self.adm = Admission(budget_bytes, slots)
        self.ws_fn = _workspace_fn(device)
        self.cache = FieldCache(cache_bytes)
        torch.cuda.set_device(device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]

    def _execute(self, req: Request, stream):
        import torch
        from . import hermes
        key = (req.catalogue_id, req.n_grid, req.box_L, req.weight is not None)
        hit = self.cache.get(key) if req.catalogue_id is not None else None
        with torch.cuda.stream(stream):
            if hit is not None:
                (delta, dk), _ = hit
            else:
                pos = torch.from_numpy(np.ascontiguousarray(req.pos, dtype=np.float32)).pin_memory()
                pos = pos.to(f"cuda:{self.device}", non_blocking=True)
                w = None
                if req.weight is not None:
                    w = torch.from_numpy(np.ascontiguousarray(req.weight, dtype=np.float32)).pin_memory()
                    w = w.to(f"cuda:{self.device}", non_blocking=True)
                eps, sw = hermes.assign(pos, w, req.box_L, req.n_grid, stream=stream)
                dk, delta = hermes.fft(eps, sw, stream=stream)
                del eps, pos, w
            outs = {k: run_stat(k, p, req, dk, delta, stream) for k, p in req.stats.items()}
            stream.synchronize()
            host = {k: v.cpu().numpy() for k, v in outs.items()}
        if hit is None and req.catalogue_id is not None:
            self.cache.put(key, (delta, dk), field_bytes(req.n_grid))
        return host, hit is not None

    def _worker(self, slot: int, work_q: queue.Queue, done_q: queue.Queue, t0: float):
        import torch
        torch.cuda.set_device(self.device)
        stream = self.streams[slot]
        while True:
            item = work_q.get()
            if item is None:
                return
            req, res = item
            try:
                res.outputs, res.cached_field = self._execute(req, stream)
                res.status = "ok"
            except Exception as exc:  # reported per request; the loop keeps serving
                res.status, res.message = "error", f"{type(exc).__name__}: {exc}"
            res.finish = time.perf_counter() - t0
            done_q.put(res)

    def run(self, requests: list[Request], on_event: Callable[[str], None] | None = None) -> list[Result]:
        """Serve requests arriving at their arrival times; returns results in rid order."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: collections.deque = collections.deque()
        results: dict[int, Result] = {}
        work_q: queue.Queue = queue.Queue()
        done_q: queue.Queue = queue.Queue()
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(i, work_q, done_q, t0), daemon=True)
                   for i in range(self.adm.slots)]
        for w in workers:
            w.start()
        i = 0
        outstanding = 0
        try:
            while i < len(pending) or waiting or outstanding:
                now = time.perf_counter() - t0
                while i < len(pending) and pending[i].arrival <= now:
                    req = pending[i]
                    i += 1
                    res = Result(req.rid, "waiting", arrival=req.arrival)
                    try:
                        res.nbytes = request_bytes(req, self.ws_fn)
                    except Exception as exc:
                        res.status, res.message, res.finish = "error", f"{type(exc).__name__}: {exc}", now
                        results[req.rid] = res
                        continue
                    if self.adm.oversized(res.nbytes):
                        res.status, res.message, res.finish = "rejected", "exceeds the HBM budget", now
                        results[req.rid] = res
                        continue
                    waiting.append((req, res))
                while True:
                    now = time.perf_counter() - t0
                    head_wait = now - waiting[0][0].arrival if waiting else 0.0
                    j = pick_next([x[1].nbytes for x in waiting], head_wait, self.adm, self.bypass_age)
                    if j is None:
                        break
                    req, res = waiting[j]
                    del waiting[j]
                    self.adm.admit(res.nbytes)
                    res.admit = time.perf_counter() - t0
                    outstanding += 1
                    work_q.put((req, res))
                    if on_event:
                        on_event(f"admit {req.rid} at {res.admit:.3f}s")
                next_arrival = pending[i].arrival - (time.perf_counter() - t0) if i < len(pending) else None
                timeout = None if next_arrival is None else max(0.0, next_arrival)
                if outstanding == 0 and timeout is None and waiting:
                    raise RuntimeError("waiting requests cannot be admitted")
                try:
                    res = done_q.get(timeout=timeout) if (outstanding or timeout is not None) else None
                except queue.Empty:
                    res = None
                if res is not None:
                    outstanding -= 1
                    self.adm.release(res.nbytes)
                    results[res.rid] = res
                    if on_event:
                        on_event(f"done {res.rid} {res.status} at {res.finish:.3f}s")
        finally:
            for _ in workers:
                work_q.put(None)
            for w in workers:
                w.join()
        return [results[k] for k in sorted(results)]


# ----------------------------------------------------------------------------
# the serving workload
# ----------------------------------------------------------------------------

def make_workload(n_requests: int = 64, seed: int = 2607_0005, grids=(128, 256, 512),
                  n_pts_range=(1e5, 1e7), precision: str = "bf16x3") -> list[Request]:
    """Requests of the serving form: Neyman-Scott catalogues (100 children per
    parent, sigma = 3, L = 1000) with log-uniform sizes, a grid from `grids`
    and a random non-empty subset of {2PCF 40 bins, xi_l l <= 4 over 30 bins,
    3PCF l <= 6 over 12 bins in [10, 150]}.  Arrival times are set later."""
    from . import synth
    rng = np.random.default_rng(seed)
    reqs = []
    choices = {
        "xi": {"edges": np.linspace(2.0, 200.0, 41), "ells": (0,)},
        "xi_ell": {"edges": np.linspace(2.0, 200.0, 31), "ells": (0, 2, 4)},
        "zeta": {"edges": np.linspace(10.0, 150.0, 13), "l_max": 6},
    }
    names = list(choices)
    for r in range(n_requests):
        n_pts = int(np.exp(rng.uniform(np.log(n_pts_range[0]), np.log(n_pts_range[1]))))
        n_par = max(1, n_pts // 100)
        pos = synth.neyman_scott(n_par, 100, 3.0, 1000.0, seed=seed + 1000 + r)
        mask = 0
        while mask == 0:
            mask = int(rng.integers(1, 8))
        stats = {names[b]: choices[names[b]] for b in range(3) if mask & (1 << b)}
        reqs.append(Request(rid=r, pos=pos, box_L=1000.0, n_grid=int(rng.choice(grids)), stats=stats,
                            precision=precision))
    return reqs


def poisson_arrivals(reqs: list[Request], rate: float, seed: int) -> None:
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in reqs:
        t += rng.exponential(1.0 / rate)
        r.arrival = t


def latency_summary(results: list[Result]) -> dict:
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok])
    span = max(r.finish for r in ok) - min(r.arrival for r in ok) if ok else float("nan")
    return {
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in results),
        "errors": sum(r.status == "error" for r in results),
        "p50_s": float(np.percentile(lat, 50)) if ok else None,
        "p99_s": float(np.percentile(lat, 99)) if ok else None,
        "throughput_req_per_s": len(ok) / span if ok else None,
    }
