"""Write the oracle's spot values for the full-size parity tests.

Calls only the FP64 oracle and the seeded input generators; the GPU path is
never involved.  Each target writes one JSON file beside this script:

  ns512   ns512_spots.json: the 10^7-point marked catalogue on 512^3 (L = 1000):
          3PCF multipoles zeta_l[b1][b2] for l in {0, 1, 2, 5, 10} and bins
          {0, 9, 19} of 20 linear bins over [10, 150], and the 2PCF in bins
          {0, 13, 26, 39} of 40 linear bins over [2, 200].
  ns1024  ns1024_subset_spots.json: the first 10^6 points (10^4 parents with
          their children) of the 10^8-point marked catalogue on 1024^3
          (L = 2000): the marked 2PCF (mark-weighted field) in bins
          {0, 13, 26, 39} of 40 bins over [2, 200], and counts-in-cells
          moments <delta_W^p>, p = 2, 3, 4 of the number field for the sphere
          and Gaussian windows at R = 4 and 32 (the ends of the geometric set).

Usage: python tests/golden/make_fullsize_spots.py ns512|ns1024 [out_dir]
The 1024^3 target holds about 60 GB of host memory at its peak; it writes its
file after every window and, when run again, computes only what is missing.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2607_23494_amd import synth  # noqa: E402

NS512_ELLS = (0, 1, 2, 5, 10)
NS512_ZBINS = (0, 9, 19)
XI_BINS = (0, 13, 26, 39)
NS1024_SUBSET = 1_000_000
NS1024_RADII_IDX = (0, 7)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def ns512(out_dir):
    wl = synth.WORKLOADS["ns512_3pcf"]
    pos, w = wl.catalogue()
    log(f"catalogue {pos.shape[0]} points")
    eps, sw = O.assign(pos, w, wl.box_L, wl.n_grid)
    delta = O.contrast(eps, sw)
    del eps
    dh = O.dft3(delta)
    log("field and spectrum done")
    e2 = synth.EDGES["ns512_2pcf"]
    xi = [float(O.xi_multipoles(dh, wl.box_L, [e2[b], e2[b + 1]])[0, 0]) for b in XI_BINS]
    log("2PCF spot bins done")
    ez = synth.EDGES["ns512_3pcf"]
    zeta = {}
    for ell in NS512_ELLS:
        z = O.zeta_multipoles(delta, dh, wl.box_L, ez, ells=(ell,), bins=list(NS512_ZBINS))[0]
        zeta[str(ell)] = z.tolist()
        log(f"zeta_{ell} done")
    out = {
        "workload": "ns512_3pcf: 1e7 marked Neyman-Scott points, 512^3, L = 1000",
        "source": "oracle/hermes_oracle.py (assign, contrast, dft3, xi_multipoles, zeta_multipoles)",
        "xi_edges": e2.tolist(), "xi_bins": list(XI_BINS), "xi": xi,
        "zeta_edges": ez.tolist(), "zeta_bins": list(NS512_ZBINS), "zeta": zeta,
    }
    with open(os.path.join(out_dir, "ns512_spots.json"), "w") as f:
        json.dump(out, f, indent=1)


def ns1024(out_dir):
    wl = synth.WORKLOADS["ns1024_cic"]
    path = os.path.join(out_dir, "ns1024_subset_spots.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)

    def save():
        with open(path, "w") as f:
            json.dump(out, f, indent=1)

    pos, w = wl.catalogue()
    pos, w = pos[:NS1024_SUBSET].copy(), w[:NS1024_SUBSET].copy()
    log(f"subset {pos.shape[0]} points")
    n, L = wl.n_grid, wl.box_L
    e2 = synth.EDGES["ns1024_cic"]
    out.update({
        "workload": "ns1024_cic subset: first 1e6 points of the 1e8-point marked catalogue, 1024^3, L = 2000",
        "source": "oracle/hermes_oracle.py (assign, contrast, dft3, xi_multipoles, filtered_field, cic_window, field_moments)",
        "n_points": int(pos.shape[0]), "xi_edges": e2.tolist(), "xi_bins": list(XI_BINS),
    })
    if "xi_marked" not in out:
        # marked 2PCF on the mark-weighted field
        eps, sw = O.assign(pos, w, L, n)
        delta = O.contrast(eps, sw)
        del eps
        dh = O.dft3(delta)
        del delta
        log("marked spectrum done")
        out["xi_marked"] = [float(O.xi_multipoles(dh, L, [e2[b], e2[b + 1]])[0, 0]) for b in XI_BINS]
        del dh
        save()
        log("marked 2PCF spot bins done")
    radii = [float(synth.CIC_RADII[i]) for i in NS1024_RADII_IDX]
    wins = [["sphere", R] for R in radii] + [["gauss", R] for R in radii]
    done = {(k, R): m for (k, R), m in zip(out.get("cic_windows", []), out.get("cic_moments", []))}
    todo = [x for x in wins if (x[0], x[1]) not in done]
    if todo:
        # counts in cells on the number field
        eps, sw = O.assign(pos, None, L, n)
        delta = O.contrast(eps, sw)
        del eps
        dh = O.dft3(delta)
        del delta
        log("number spectrum done")
        for kind, R in todo:
            dw = O.filtered_field(dh, L, O.cic_window(kind, R))
            log(f"cic {kind} {R} field done")
            done[(kind, R)] = O.field_moments(dw).tolist()
            del dw
            out["cic_windows"] = [list(k) for k in done]
            out["cic_moments"] = list(done.values())
            save()
            log(f"cic {kind} {R} done")
    save()


if __name__ == "__main__":
    target = sys.argv[1]
    out_dir = sys.argv[2] if len(sys.argv) > 2 else HERE
    os.makedirs(out_dir, exist_ok=True)
    {"ns512": ns512, "ns1024": ns1024}[target](out_dir)
    log("written")
