#!/usr/bin/env python3
"""Benchmark of the field-window estimator's hot path on one MI355X.

One step is the whole path over one synthetic catalogue already resident in
HBM: B3 assignment of 10^7 marked Neyman-Scott points onto a 512^3 grid,
contrast and r2c FFT, the 40-bin 2PCF over [2, 200] Mpc/h by Parseval, and
the 3PCF multipoles l = 0..10 over 20 radial bins in [10, 150] Mpc/h.
The same step is then timed with the float32 (vector-unit) contraction, the
other workloads (64^3 float64, 256^3 redshift space, 10^8 marked points on
1024^3) and the serving mix are measured, and the FP64 oracle is timed on a
bounded sample.  Prints one JSON line on stdout (everything else goes to
stderr).

  python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3|fp16x3]
                  [--no-compare] [--no-configs] [--no-serving] [--no-cpu-baseline]
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
MFMA_PEAK_TFLOPS = {"bf16x3": 2500.0, "fp16x3": 2500.0}   # dense bf16 / fp16 matrix cores
WORKLOAD = "ns512_3pcf"
L_MAX = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that hold no kernel the 512^3 benchmark step launches (the other
# workloads' kernels, and the host-side entry points and tables); the
# counters recorded in profiles/ stay valid while the rest of csrc/ is
# unchanged.
_NOT_IN_STEP = {"aniso.hip", "api.hip", "basis.hip", "gamma.hip", "readout.hip", "triplet.hip"}


def kernel_source_hash() -> str:
    """Hash of the sources the benchmark step's kernels are built from."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2607_23494_amd", "csrc", "*"))):
        if os.path.basename(p) in _NOT_IN_STEP:
            continue
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
    extrapolate to one step.  The oracle's DFTs run on scipy's thread pool
    (one worker per core); everything else is single-threaded numpy."""
    import numpy as np
    import oracle as O
    from oracle import hermes_oracle as OH
    from paper_2607_23494_amd import synth

    rng = np.random.default_rng(1)
    t = {}
    wl = synth.WORKLOADS[WORKLOAD]
    sub = 1_000_000
    pos = synth.neyman_scott(sub // wl.n_children, wl.n_children, wl.sigma, box_L, seed=wl.seed)
    marks = synth.lognormal_marks(pos.shape[0], wl.seed)
    t0 = time.perf_counter()
    O.assign(pos, marks, box_L, n)
    t["assign_1e6"] = time.perf_counter() - t0
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
    n_pts = wl.n_pts
    step = (t["assign_1e6"] * n_pts / sub + t["dft"] + nb_xi * t["xi_bin"] + n_lm * t["ylm"]
            + n_lm * nb_zeta * t["field"] + n_lm * nb_zeta * (t["da"] + nb_zeta * t["prod"]))
    sampled = sum(t.values())
    log(f"cpu baseline sample {sampled:.1f}s: " + ", ".join(f"{k}={v:.2f}s" for k, v in t.items()))
    return {
        "value": round(step, 1),
        "unit": "s",
        "cores": OH._WORKERS,
        "threads": {"dft": OH._WORKERS, "assignment, windows, products": 1},
        "kind": "oracle",
        "sample_s": {k: round(v, 3) for k, v in t.items()},
        "sample": (f"timed at {n}^3 ({sampled:.1f} s): the assignment of 1e6 of the 1e7 marked points, one "
                   f"forward DFT, one 2PCF bin, one real-SH window, one multipole field and one delta*a*a "
                   f"product; extrapolated (not run) to 1e7 points + 1 DFT + {nb_xi} bins + {n_lm} windows + "
                   f"{n_lm * nb_zeta} fields + {n_lm * nb_zeta * nb_zeta} products. The DFTs (inside each "
                   f"multipole field too) use {OH._WORKERS} threads; the elementwise work is single-threaded."),
    }


def _normwise_dev(a, b) -> float:
    import numpy as np
    scale = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b)) / scale) if scale > 0 else float(np.max(np.abs(a - b)))


def _result_deviation(mix, solo) -> float:
    """Largest normwise deviation of one request's outputs in the mix from its
    solo outputs: per xi row, per zeta_l matrix, per moment column."""
    dev = 0.0
    for k, v in solo.outputs.items():
        m = mix.outputs[k]
        if k == "zeta":
            rows = [(m[l], v[l]) for l in range(v.shape[0])]
        elif k == "cic":
            rows = [(m[:, p], v[:, p]) for p in range(v.shape[1])]
        else:
            rows = [(m[i], v[i]) for i in range(v.shape[0])]
        for a, b in rows:
            dev = max(dev, _normwise_dev(a, b))
    return dev


def serving_benchmark(precisions, n_requests: int = 64) -> dict:
    """The serving workload: one Poisson arrival trace at 0.7 of the solo
    service capacity of the first precision, served at every precision with
    continuous admission under an HBM budget; each request's result in the mix
    is compared with its result served alone."""
    import numpy as np

    from paper_2607_23494_amd import serving as S

    t0 = time.perf_counter()
    base = S.make_workload(n_requests)
    log(f"serving workload: {n_requests} requests generated in {time.perf_counter() - t0:.1f}s")
    out = {"workload": f"{n_requests} Neyman-Scott catalogues, 1e5-1e7 points (log-uniform), grids "
                       "128/256/512, random subsets of {2PCF 40 bins, xi_l l<=4 30 bins, 3PCF l<=6 12 bins}; "
                       "4 slots, 200 GB budget, one Poisson arrival trace at 0.7 / mean solo service time of "
                       f"{precisions[0]}, the same trace for every precision"}
    warm = S.Server(slots=1)
    rate = None
    for prec in precisions:
        reqs = [dataclasses_replace(r, precision=prec, arrival=0.0) for r in base]
        warm.run([dataclasses_replace(reqs[0], rid=-1)])
        solo = {r.rid: r for r in S.Server(slots=1).run(reqs)}
        service = np.array([r.finish - r.admit for r in solo.values() if r.status == "ok"])
        mean = float(service.mean())
        if rate is None:
            rate = 0.7 / mean
            S.poisson_arrivals(base, rate, seed=2607_0005)
        reqs = [dataclasses_replace(r, precision=prec) for r in base]
        res = S.Server(slots=4, budget_bytes=200 << 30).run(reqs)
        summ = S.latency_summary(res)
        dev = max(_result_deviation(r, solo[r.rid]) for r in res if r.status == "ok" and solo[r.rid].status == "ok")
        # the tail of the service times alone: a request's latency in the mix
        # is at least its own service time
        summ.update({"mean_solo_service_s": round(mean, 4),
                     "p50_solo_service_s": round(float(np.percentile(service, 50)), 4),
                     "p99_solo_service_s": round(float(np.percentile(service, 99)), 4),
                     "arrival_rate_per_s": round(rate, 3),
                     "max_dev_vs_solo": float(f"{dev:.3g}"),
                     "dev_tolerance": 1e-3 if prec != "fp32" else 1e-5})
        for k in ("p50_s", "p99_s", "throughput_req_per_s"):
            if summ[k] is not None:
                summ[k] = round(summ[k], 4)
        out[prec] = summ
        log(f"serving {prec}: " + json.dumps(summ))
    return out


def dataclasses_replace(obj, **kw):
    import dataclasses
    return dataclasses.replace(obj, **kw)


def time_steps(step, warmup: int, steps: int, hermes, label: str):
    """W untimed steps, then K timed steps with per-kernel HIP-event timing."""
    import torch
    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"{label}: warmup step {i + 1}/{warmup} done")
    hermes.profile_enable(True)
    hermes.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = hermes.profile_read()
    hermes.profile_enable(False)
    log(f"{label}: {steps} timed steps, {elapsed / steps * 1e3:.1f} ms/step")
    return elapsed / steps, prof


def other_configs(warmup: int, steps: int) -> dict:
    """The 64^3 float64, 256^3 redshift-space and 1024^3 marked workloads,
    each timed as one step of its statistics on a resident catalogue."""
    import numpy as np
    import torch

    from paper_2607_23494_amd import hermes, synth

    out = {}

    def record(name, step, count, desc, per="cells_bins", n_steps=None):
        k = steps if n_steps is None else n_steps
        s, prof = time_steps(step, warmup, k, hermes, name)
        out[name] = {"workload": desc, "ms_per_step": round(s * 1e3, 3), "steps": k, "warmup": warmup,
                     f"{per}_per_s": round(count / s, 1),
                     "stage_ms": {kk: round(v[1] / k, 3) for kk, v in sorted(prof.items())}}

    # 64^3, float64: 2e4 points, 20-bin 2PCF over [5, 50]
    wl = synth.WORKLOADS["ns64_fp64"]
    pos = torch.from_numpy(wl.catalogue()[0]).cuda()
    e = synth.EDGES["ns64_fp64"]
    n = wl.n_grid

    def step64():
        eps, sw = hermes.assign(pos, None, wl.box_L, n, dtype=torch.float64)
        dk, _ = hermes.fft(eps, sw, want_delta=False)
        hermes.xi(dk, wl.box_L, e)
    record("ns64_fp64", step64, n ** 3 * (e.size - 1),
           "2e4 Neyman-Scott points, 64^3, float64: assign, FFT, 20-bin 2PCF")

    # 256^3: 2e6 points with z displacements, 40-bin 2PCF and xi_0,2,4 over 30 bins
    wl = synth.WORKLOADS["ns256_rsd"]
    pos = torch.from_numpy(wl.catalogue()[0]).cuda()
    e40, e30 = synth.EDGES["ns256_rsd"], synth.EDGES["ns256_rsd_ell"]
    n = wl.n_grid

    def step256():
        eps, sw = hermes.assign(pos, None, wl.box_L, n)
        dk, _ = hermes.fft(eps, sw, want_delta=False)
        hermes.xi(dk, wl.box_L, e40)
        hermes.xi(dk, wl.box_L, e30, ells=(0, 2, 4))
    record("ns256_rsd", step256, n ** 3 * ((e40.size - 1) + 3 * (e30.size - 1)),
           "2e6 Neyman-Scott points with z displacements, 256^3, float32: assign, FFT, 40-bin 2PCF, "
           "xi_0,2,4 over 30 bins")

    # the same catalogue: DD(s, mu) with thin ring windows, 46 s x 51 mu
    rings = synth.smu_rings()
    xawork = torch.empty(hermes.workspace_size(hermes.OP_XI_ANISO, n, torch.float32, len(rings), 0),
                         dtype=torch.uint8, device="cuda")

    def step_smu():
        eps, sw = hermes.assign(pos, None, wl.box_L, n)
        dk, _ = hermes.fft(eps, sw, want_delta=False)
        hermes.xi_aniso(dk, wl.box_L, rings, work=xawork)
    record("ns256_smu", step_smu, n ** 3 * len(rings),
           "2e6 Neyman-Scott points with z displacements, 256^3, float32: assign, FFT, DD(s, mu) with thin ring "
           "windows at 46 x 51 (s, mu) bin centres (s in [2, 186], mu in [0, 1])")
    out["ns256_smu"]["ms_per_window"] = round(out["ns256_smu"]["ms_per_step"] / len(rings), 6)
    del xawork

    # DDD(theta; r12 = 20, r13 = 40) by Monte-Carlo triangles, 20 opening
    # angles, the secondary vertices on the sphere-smoothed (R = 5) contrast:
    # dual sphere (406,728 catalogue points as primary vertices, 1000
    # rotations each) and triplet sphere (8e6 box points, 200 rotations)
    eps, sw = hermes.assign(pos, None, wl.box_L, n)
    dk, _ = hermes.fft(eps, sw, want_delta=False)
    fld = hermes.filter_bins(dk, wl.box_L, [("sphere", 0.0, 5.0)], store_fields=True, moments=False)[0][0]
    del eps, dk
    cen = pos[:406_728].contiguous()
    twork = torch.empty(hermes.workspace_size(hermes.OP_TRIPLET, n, torch.float32, 20, 8_000_000),
                        dtype=torch.uint8, device="cuda")
    tout = torch.empty((20, 4), dtype=torch.float64, device="cuda")
    for name, n_c, n_rot, kw, desc in [
            ("ns256_ddd_particle", cen.shape[0], 1000, {"centres": cen},
             "DDD(theta; 20, 40), 20 angles: 406,728 catalogue points of the 256^3 workload as primary vertices "
             "x 1000 rotations, sphere-smoothed (R = 5) contrast at the other vertices"),
            ("ns256_ddd_box", 8_000_000, 200, {"n_box": 8_000_000, "f1": fld},
             "DDD(theta; 20, 40), 20 angles: 8e6 uniform box points x 200 rotations, sphere-smoothed (R = 5) "
             "contrast at all three vertices")]:
        def step_ddd(kw=kw, n_rot=n_rot):
            hermes.triplet_mc(fld, fld, wl.box_L, 20.0, 40.0, 20, n_rot, 2607, out=tout, work=twork, **kw)
        combos = n_c * n_rot * 20
        record(name, step_ddd, combos, desc, per="combinations", n_steps=1)
        out[name]["ns_per_combination"] = round(out[name]["ms_per_step"] * 1e6 / combos, 4)
    del fld, cen, twork, tout

    # 3PCF monopole through triple connection coefficients: the contrast and
    # 20 thick-shell filtered fields over [10, 150] (the 3PCF bins), every bin
    # pair, at 256^3
    e20 = synth.EDGES["ns512_3pcf"]
    shells = [("shell", float(e20[i]), float(e20[i + 1])) for i in range(e20.size - 1)]
    gfields = torch.empty((len(shells), n, n, n), dtype=torch.float32, device="cuda")

    def step_gamma():
        eps, sw = hermes.assign(pos, None, wl.box_L, n)
        dk, delta = hermes.fft(eps, sw)
        hermes.filter_bins(dk, wl.box_L, shells, store_fields=True, moments=False, out=gfields)
        hermes.ddd_gamma(delta, gfields)
    npairs = len(shells) * (len(shells) + 1) // 2
    record("ns256_gamma", step_gamma, n ** 3 * npairs,
           "2e6 Neyman-Scott points, 256^3, float32: assign, FFT, 20 thick-shell fields over [10, 150], the "
           "connection-coefficient 3PCF monopole of all 210 bin pairs (exact triple integral of the B3 "
           "expansions)", per="cells_pairs")
    # the same with the orthonormal Daubechies D4 basis (the paper's exact
    # stencil route: projection, window kernel and connection coefficients
    # of D4)
    with hermes.basis("db2"):
        record("ns256_gamma_db2", step_gamma, n ** 3 * npairs,
               "2e6 Neyman-Scott points, 256^3, float32, Daubechies D4 basis: assign, FFT, 20 thick-shell fields "
               "over [10, 150], the connection-coefficient 3PCF monopole of all 210 bin pairs (D4 triple "
               "connection coefficients, offsets in [-2, 2]^3)", per="cells_pairs")
    del gfields
    del pos
    torch.cuda.empty_cache()

    # counts in cells by random spheres (Sec. 3.1): the 512^3 field of the
    # 1e7-point catalogue smoothed with spheres of R = 10, 15, 20, each read
    # at 1e8 uniform random positions (values and their moments)
    wl = synth.WORKLOADS["ns512_3pcf"]
    pos_np, w_np = wl.catalogue()
    n, L = wl.n_grid, wl.box_L
    cpos = torch.from_numpy(pos_np).cuda()
    cw = torch.from_numpy(w_np).cuda()
    del pos_np, w_np
    eps, sw = hermes.assign(cpos, None, L, n)
    dk, _ = hermes.fft(eps, sw, want_delta=False)
    del eps, cpos, cw
    spheres = [("sphere", 0.0, R) for R in (10.0, 15.0, 20.0)]
    cfields, _ = hermes.filter_bins(dk, L, spheres, store_fields=True, moments=False)
    del dk
    g = torch.Generator(device="cuda").manual_seed(2607)
    rpos = (torch.rand((100_000_000, 3), device="cuda", generator=g) * L).contiguous()
    vals = torch.empty((3, 100_000_000), dtype=torch.float32, device="cuda")
    moms = torch.empty((3, 3), dtype=torch.float64, device="cuda")
    rwork = torch.empty(hermes.workspace_size(hermes.OP_READOUT, n, torch.float32, 100_000_000),
                        dtype=torch.uint8, device="cuda")

    def step_cic_random():
        hermes.readout_fields(cfields, L, rpos, out=vals, moments_out=moms, work=rwork)
    record("ns512_cic_random", step_cic_random, 3 * 100_000_000,
           "counts in cells by random spheres: the 512^3 contrast of the 1e7-point catalogue smoothed with "
           "spheres of R = 10, 15, 20, all read at the same 1e8 uniform random positions (values and moments "
           "p = 2, 3, 4 of each)",
           per="readouts")
    del cfields, rpos, vals, moms, rwork
    torch.cuda.empty_cache()

    # 1024^3: 1e8 marked points, marked 2PCF (40 bins) and the unmarked 2PCF on
    # the mark-weighted and number fields, counts-in-cells moments of the
    # number field for the sphere and Gaussian at 8 radii
    wl = synth.WORKLOADS["ns1024_cic"]
    t0 = time.perf_counter()
    pos_np, w_np = wl.catalogue()
    log(f"ns1024 catalogue: {pos_np.shape[0]} points in {time.perf_counter() - t0:.1f}s")
    pos = torch.from_numpy(pos_np).cuda()
    w = torch.from_numpy(w_np).cuda()
    del pos_np, w_np
    n, L = wl.n_grid, wl.box_L
    e = synth.EDGES["ns1024_cic"]
    wins = [("sphere", 0.0, R) for R in synth.CIC_RADII] + [("gauss", 0.0, R) for R in synth.CIC_RADII]
    eps = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    sw = torch.empty(1, dtype=torch.float64, device="cuda")
    dk = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    fwork = torch.empty(hermes.workspace_size(hermes.OP_FILTER, n, torch.float32, len(wins)), dtype=torch.uint8,
                        device="cuda")
    xwork = torch.empty(hermes.workspace_size(hermes.OP_XI, n, torch.float32, e.size - 1, 1), dtype=torch.uint8,
                        device="cuda")
    awork = torch.empty(hermes.workspace_size(hermes.OP_ASSIGN, n, torch.float32, int(pos.shape[0]), 1),
                        dtype=torch.uint8, device="cuda")

    xi_m = torch.empty((1, e.size - 1), dtype=torch.float64, device="cuda")
    xi_n = torch.empty_like(xi_m)
    mr = torch.empty_like(xi_m)

    def step1024():
        hermes.assign(pos, w, L, n, eps=eps, sum_w=sw, work=awork)
        hermes.fft(eps, sw, want_delta=False, delta_k=dk)
        hermes.xi(dk, L, e, out=xi_m, work=xwork)
        hermes.assign(pos, None, L, n, eps=eps, sum_w=sw, work=awork)
        hermes.fft(eps, sw, want_delta=False, delta_k=dk)
        hermes.xi(dk, L, e, out=xi_n, work=xwork)
        hermes.mark_ratio(xi_m, xi_n, out=mr)
        hermes.filter_bins(dk, L, wins, store_fields=False, moments=True, work=fwork)
    record("ns1024_cic", step1024, n ** 3 * (2 * (e.size - 1) + len(wins)),
           "1e8 marked Neyman-Scott points, 1024^3, float32: assign and FFT of the mark-weighted and number "
           "fields, 40-bin 2PCF of each and their ratio M(r) = (1 + xi_m) / (1 + xi), counts-in-cells moments "
           "(p = 2, 3, 4) of the number field for the sphere and Gaussian at 8 radii (16 windows)")
    del pos, w, eps, dk, fwork, xwork, awork
    torch.cuda.empty_cache()
    return out


def mfma_rate(prof: dict, n: int, nb: int, precision: str):
    """Matrix-core rate of the fused z pass: each row group of C cells issues,
    per wavefront quarter, 2 MFMA 32x32x16 per 16 cells (the hi.hi and lo.hi
    products), i.e. 2 * 2 * 32 * 32 * 16 / 16 flops per cell; the useful part
    is the nb x nb block of the 32 x 32 tile."""
    if precision not in MFMA_PEAK_TFLOPS or "inv_z_contract" not in prof:
        return None
    launches, total_ms = prof["inv_z_contract"]
    avg_s = total_ms / launches / 1e3
    issued = n ** 3 * 2 * (2 * 32 * 32 * 16) / 16
    useful = issued * (nb * nb) / (32 * 32)
    return {"kernel": "inv_z_contract", "avg_launch_ms": round(avg_s * 1e3, 4),
            "issued_flops": issued, "useful_flops": useful,
            "issued_tflops": round(issued / avg_s / 1e12, 2), "useful_tflops": round(useful / avg_s / 1e12, 2),
            "peak": MFMA_PEAK_TFLOPS[precision], "unit": "TFLOP/s",
            "frac": round(issued / avg_s / 1e12 / MFMA_PEAK_TFLOPS[precision], 4)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the step with the float32 contraction (mixed-vs-FP32 ratio)")
    ap.add_argument("--no-configs", action="store_true", help="skip the 64^3, 256^3 and 1024^3 workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--configs-only", action="store_true",
                    help="run only the other workloads, 64^3 to 1024^3 (for hardware counters of their "
                         "kernels); prints their timings, not the benchmark line")
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
    a_work = torch.empty(hermes.workspace_size(hermes.OP_ASSIGN, n, torch.float32, int(pos_np.shape[0]), 1),
                         dtype=torch.uint8, device="cuda")

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.neg(a)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 1 GiB read + 1 GiB write done")

    if args.configs_only:
        del pos, w, eps, sw, dk, delta, xi_out, zeta_out, xi_work, z_work, a_work
        torch.cuda.empty_cache()
        print(json.dumps({"configs": other_configs(1, max(1, min(args.steps, 5)))}), flush=True)
        return 0

    def step_at(precision):
        def step():
            hermes.assign(pos, w, L, n, eps=eps, sum_w=sw, work=a_work)
            hermes.fft(eps, sw, delta_k=dk, delta=delta)
            hermes.xi(dk, L, edges_xi, ells=(0,), out=xi_out, work=xi_work)
            hermes.zeta_l(delta, dk, L, edges_z, L_MAX, precision=precision, out=zeta_out, work=z_work)
        return step

    s_per_step, prof = time_steps(step_at(args.precision), args.warmup, args.steps, hermes, args.precision)

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
                     "achieved_GBps": round(ab / a_s / 1e9, 1), "frac": round(ab / a_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(k)}
    # the 3PCF stage as a whole against the method's bytes: one spectrum read
    # and one real field written per filtered field
    zeta_ms = sum(v[1] for k, v in prof.items() if k.startswith("inv_") or k in ("radial_table", "reduce"))
    fields = nb_z * (L_MAX + 1) ** 2 * args.steps
    stage_bytes = fields * (n * n * (n // 2 + 1) * 8 + n ** 3 * 4)
    stage = {"ms_per_step": round(zeta_ms / args.steps, 2), "fields_per_step": fields // args.steps,
             "method_bytes_per_step": stage_bytes // args.steps,
             "achieved_GBps": round(stage_bytes / (zeta_ms / 1e3) / 1e9, 1),
             "frac": round(stage_bytes / (zeta_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

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
        "zeta_stage": stage,
        "mfma": mfma_rate(prof, n, nb_z, args.precision),
    }
    if not args.no_compare and args.precision != "fp32":
        s32, prof32 = time_steps(step_at("fp32"), args.warmup, args.steps, hermes, "fp32")
        z_mixed = prof["inv_z_contract"][1] / prof["inv_z_contract"][0]
        z_fp32 = prof32["inv_z_contract"][1] / prof32["inv_z_contract"][0]
        result["fp32_compare"] = {
            "ms_per_step": round(s32 * 1e3, 2), "steps": args.steps, "warmup": args.warmup,
            "speedup_end_to_end": round(s32 / s_per_step, 3),
            "z_pass_ms_fp32": round(z_fp32, 4), "z_pass_ms_mixed": round(z_mixed, 4),
            "speedup_z_pass": round(z_fp32 / z_mixed, 3),
            "stage_ms": {k: round(v[1] / args.steps, 3) for k, v in sorted(prof32.items())}}
    del pos, w, eps, delta, dk, z_work, xi_work, a_work
    torch.cuda.empty_cache()
    if not args.no_configs:
        result["configs"] = other_configs(1, max(1, min(args.steps, 5)))
    if not args.no_serving:
        precs = [args.precision] + (["fp32"] if args.precision != "fp32" else [])
        result["serving"] = serving_benchmark(precs)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(n, L, nb_xi, nb_z, L_MAX)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
