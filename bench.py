#!/usr/bin/env python3
"""Benchmark of the field-window estimator's hot path on one MI355X.

One step is the whole path over one synthetic catalogue already resident in
HBM: B3 assignment of 10^7 marked Neyman-Scott points onto a 512^3 grid,
contrast and r2c FFT, the 40-bin 2PCF over [2, 200] Mpc/h by Parseval, and
the 3PCF multipoles l = 0..10 over 20 radial bins in [10, 150] Mpc/h.
Prints one JSON line on stdout (everything else goes to stderr).

  python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3|fp16x3]
                  [--compare] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
WORKLOAD = "ns512_3pcf"
L_MAX = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2607_23494_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(name: str, n: int, nb: int):
    """Bytes a pass must move per launch (read + write), by kernel class."""
    spec = n * n * (n // 2 + 1) * 8      # complex64 half spectrum
    field = n ** 3 * 4                   # float32 real field
    table = {
        "fwd_z": field + spec + field,   # read eps; write delta^ and delta
        "fwd_y": 2 * spec,
        "fwd_x": 2 * spec,
        "inv_x_window": spec + nb * spec,   # read delta^ once; write nb spectra
        "inv_x_window2": spec + 2 * nb * spec,   # two m of one l: write 2 nb spectra
        "inv_y": 2 * nb * spec,
        "inv_z_contract": nb * spec + field,  # read nb spectra and delta
    }
    return table.get(name)


def measured_traffic(kernel: str):
    """Per-launch HBM bytes from the committed counter summary, if it was
    taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def cpu_baseline(n: int, box_L: float, nb_xi: int, nb_zeta: int, l_max: int) -> dict:
    """Time the FP64 oracle on a bounded sample of the same 512^3 workload and
    extrapolate to one step."""
    import numpy as np
    import oracle as O
    from oracle import hermes_oracle as OH

    rng = np.random.default_rng(1)
    t = {}
    delta = rng.standard_normal((n, n, n))
    t0 = time.perf_counter()
    dh = O.dft3(delta)
    t["dft"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.xi_multipoles(dh, box_L, [100.0, 105.0], ells=(0,))
    t["xi_bin"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ylm = O.sh_window(n, box_L, 2, 1)
    t["ylm"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    a, _ = O.multipole_field(dh, box_L, 2, 1, 80.0, 87.0, ylm)
    t["field"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    da = delta * a
    t["da"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    float(np.sum(da * a))
    t["prod"] = time.perf_counter() - t0
    n_lm = (l_max + 1) ** 2
    step = (t["dft"] + nb_xi * t["xi_bin"] + n_lm * t["ylm"] + n_lm * nb_zeta * t["field"]
            + n_lm * nb_zeta * (t["da"] + nb_zeta * t["prod"]))
    sampled = sum(t.values())
    log(f"cpu baseline sample {sampled:.1f}s: " + ", ".join(f"{k}={v:.2f}s" for k, v in t.items()))
    return {
        "value": step,
        "unit": "s",
        "cores": OH._WORKERS,
        "kind": "oracle",
        "sample": (f"timed at {n}^3: one forward DFT, one 2PCF bin, one real-SH window, one multipole field "
                   f"and one delta*a*a product ({sampled:.1f} s of CPU); extrapolated to 1 DFT + {nb_xi} bins + "
                   f"{n_lm} windows + {n_lm * nb_zeta} fields + {n_lm * nb_zeta * nb_zeta} products. "
                   f"Assignment not included. FFT threads = cores; elementwise work single-threaded."),
    }


def serving_benchmark(precisions, n_requests: int = 64) -> dict:
    """The serving workload: requests with Poisson arrivals at 0.7 of the
    solo service capacity, continuous admission under an HBM budget."""
    import copy

    import numpy as np

    from paper_2607_23494_amd import serving as S

    t0 = time.perf_counter()
    base = S.make_workload(n_requests)
    log(f"serving workload: {n_requests} requests generated in {time.perf_counter() - t0:.1f}s")
    out = {"workload": f"{n_requests} Neyman-Scott catalogues, 1e5-1e7 points (log-uniform), grids "
                       "128/256/512, random subsets of {2PCF 40 bins, xi_l l<=4 30 bins, 3PCF l<=6 12 bins}; "
                       "4 slots, 200 GB budget, Poisson arrivals at 0.7 / mean solo service time"}
    warm = S.Server(slots=1)
    for prec in precisions:
        reqs = copy.copy(base)
        reqs = [dataclasses_replace(r, precision=prec, arrival=0.0) for r in reqs]
        warm.run([dataclasses_replace(reqs[0], rid=-1)])
        solo = S.Server(slots=1).run(reqs)
        service = np.array([r.finish - r.admit for r in solo if r.status == "ok"])
        mean = float(service.mean())
        rate = 0.7 / mean
        S.poisson_arrivals(reqs, rate, seed=2607_0005)
        res = S.Server(slots=4, budget_bytes=200 << 30).run(reqs)
        summ = S.latency_summary(res)
        summ.update({"mean_solo_service_s": round(mean, 4), "arrival_rate_per_s": round(rate, 3)})
        for k in ("p50_s", "p99_s", "throughput_req_per_s"):
            if summ[k] is not None:
                summ[k] = round(summ[k], 4)
        out[prec] = summ
        log(f"serving {prec}: " + json.dumps(summ))
    return out


def dataclasses_replace(obj, **kw):
    import dataclasses
    return dataclasses.replace(obj, **kw)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--compare", action="store_true",
                    help="also time one step with the fp32 contraction for the mixed-vs-fp32 ratio")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise kernel that reads and writes 1 GiB, as the reference "
                         "for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU only: the path is built for a single MI355X and has no multi-GPU mode.")
        return 2

    import numpy as np
    import torch

    from paper_2607_23494_amd import hermes, synth

    dev = 0
    torch.cuda.set_device(dev)
    wl = synth.WORKLOADS[WORKLOAD]
    n, L = wl.n_grid, wl.box_L
    edges_xi = synth.EDGES["ns512_2pcf"]
    edges_z = synth.EDGES["ns512_3pcf"]
    nb_xi, nb_z = edges_xi.size - 1, edges_z.size - 1

    t0 = time.perf_counter()
    pos_np, w_np = wl.catalogue()
    log(f"catalogue: {pos_np.shape[0]} points in {time.perf_counter() - t0:.1f}s")
    pos = torch.from_numpy(pos_np).cuda()
    w = torch.from_numpy(w_np).cuda()
    eps = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    sw = torch.empty(1, dtype=torch.float64, device="cuda")
    dk = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    delta = torch.empty_like(eps)
    xi_out = torch.empty((1, nb_xi), dtype=torch.float64, device="cuda")
    zeta_out = torch.empty((L_MAX + 1, nb_z, nb_z), dtype=torch.float64, device="cuda")
    xi_work = torch.empty(hermes.workspace_size(hermes.OP_XI, n, torch.float32, nb_xi, 1), dtype=torch.uint8,
                          device="cuda")
    z_work = torch.empty(hermes.workspace_size(hermes.OP_ZETA, n, torch.float32, nb_z, 1), dtype=torch.uint8,
                         device="cuda")

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.neg(a)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 1 GiB read + 1 GiB write done")

    def step(precision):
        hermes.assign(pos, w, L, n, eps=eps, sum_w=sw)
        hermes.fft(eps, sw, delta_k=dk, delta=delta)
        hermes.xi(dk, L, edges_xi, ells=(0,), out=xi_out, work=xi_work)
        hermes.zeta_l(delta, dk, L, edges_z, L_MAX, precision=precision, out=zeta_out, work=z_work)

    for i in range(args.warmup):
        step(args.precision)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    hermes.profile_enable(True)
    hermes.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.precision)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = hermes.profile_read()
    hermes.profile_enable(False)
    s_per_step = elapsed / args.steps
    log(f"timed {args.steps} steps: {s_per_step * 1e3:.1f} ms/step")

    stages = {k: round(v[1] / args.steps, 3) for k, v in sorted(prof.items())}
    log("per-step kernel ms: " + json.dumps(stages))
    # dominant kernel among the bandwidth-bound passes
    cands = [(v[1], k) for k, v in prof.items() if algorithmic_bytes(k, n, nb_z) is not None]
    _, dom = max(cands)
    launches, total_ms = prof[dom]
    avg_s = total_ms / launches / 1e3
    abytes = algorithmic_bytes(dom, n, nb_z)
    achieved = abytes / avg_s / 1e9
    traffic = measured_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_ms": round(avg_s * 1e3, 4), "algorithmic_bytes": abytes, "launches": launches}
    # the same figures for every pass that has an algorithmic byte count
    passes = {}
    for _, k in sorted(cands, reverse=True):
        nl, tms = prof[k]
        a_s = tms / nl / 1e3
        ab = algorithmic_bytes(k, n, nb_z)
        passes[k] = {"avg_launch_ms": round(a_s * 1e3, 4), "launches": nl, "algorithmic_bytes": ab,
                     "achieved_GBps": round(ab / a_s / 1e9, 1), "frac": round(ab / a_s / 1e9 / HBM_PEAK_GBS, 4)}

    extra = {}
    if args.compare:
        other = "fp32" if args.precision != "fp32" else None
        if other:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            step(other)
            torch.cuda.synchronize()
            extra["fp32_s_per_step"] = round(time.perf_counter() - t1, 4)

    n_lm = (L_MAX + 1) ** 2
    cells = n ** 3
    cells_bins = cells * nb_xi + cells * nb_z * n_lm
    result = {
        "metric": "2PCF+3PCF wall-time per catalogue at 512^3",
        "value": round(s_per_step, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s_per_step * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"f32+{args.precision}",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_points": int(pos_np.shape[0]), "grid": n, "box_L": L,
                   "marks": "lognormal", "xi_bins": nb_xi, "zeta_bins": nb_z, "l_max": L_MAX,
                   "precision": args.precision},
        "cells_bins_per_s": round(cells_bins / s_per_step, 1),
        "stage_ms": stages,
        "roofline": roofline,
        "passes": passes,
    }
    result.update(extra)
    if not args.no_serving:
        del pos, w, eps, delta, dk, z_work, xi_work
        torch.cuda.empty_cache()
        precs = [args.precision] + (["fp32"] if args.precision != "fp32" else [])
        result["serving"] = serving_benchmark(precs)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(n, L, nb_xi, nb_z, L_MAX)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
