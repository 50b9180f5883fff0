"""Write tests/golden/setpoint_zc.json: the tip-sample separation of every workload's truth.

AFM amplitude feedback holds the oscillation amplitude at a set-point (paper Sec. 1), so each
workload fixes the separation z_c at which the oracle's steady amplitude at the truth
parameters equals setpoint * A0 (approach curve from A0 + 2 nm in 0.25 nm steps, then
bisection to 1e-9 A0).  For the 3-mode workload the modal frequency ratios and base-drive gains of
a uniform Euler-Bernoulli cantilever (paper Sec. 3.2, Eq. 6-7, 501-point Simpson as in
Appendix A) are stored too, and those of the paper's eight-mode beam ("eb8").

Calls the oracle only.  Run from the repository root: python tests/golden/make_setpoints.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def beam(n, out):
    """Frequency ratios and base-drive gains of the first n modes of a uniform Euler-Bernoulli
    cantilever (Eq. 6-7 with the corrected denominator, 501-point Simpson), stored as "eb<n>"."""
    eb = O.eb_modes(n, 501)
    out[f"eb{n}"] = {"ratio": [float(r) for r in eb["ratio"]],
                     "gain": [float(g) for g in eb["gain"]]}


def main(names=("c1", "c2", "c3", "c4", "c5", "eb8")):
    out = {}
    if os.path.exists(W.ZC_FILE):
        with open(W.ZC_FILE) as f:
            out = json.load(f)
    for name in names:
        if name.startswith("eb"):
            beam(int(name[2:]), out)
            with open(W.ZC_FILE, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)
            print(f"{name}: stored", flush=True)
            continue
        t0 = time.time()
        cfg = W.config(name)
        rec = {}
        if cfg["model"]["n_modes"] > 1:
            eb = O.eb_modes(cfg["model"]["n_modes"], 501)
            rec["gain"] = [float(g) for g in eb["gain"]]
            rec["eb_ratio"] = [float(r) for r in eb["ratio"]]
            cfg["model"]["gain"] = rec["gain"]
        p = W.full_params(cfg, zc=0.0)
        zc = O.zc_from_setpoint(cfg["model"], p, cfg["setpoint"])
        rec["zc"] = zc
        rec["setpoint"] = cfg["setpoint"]
        rec["steps_per_cycle"] = cfg["model"]["steps_per_cycle"]
        out[name] = rec
        print(f"{name}: zc = {zc:.6e} m ({time.time() - t0:.1f} s)", flush=True)
        with open(W.ZC_FILE, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("c1", "c2", "c3", "c4", "c5", "eb8"))
