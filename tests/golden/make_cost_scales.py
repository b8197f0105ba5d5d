"""Writes tests/golden/cost_scales.json: max_ij ||x_i - y_j||^2 of the full-size synthetic
workloads (the cost normalisation s = 1/max, so that ||C||_inf = 1), computed with the
oracle's exact FP64 C routine.  Calls nothing but oracle/ and the input generators.

    python tests/golden/make_cost_scales.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cmax  # noqa: E402
from paper_2511_11359_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_scales.json")


def main():
    res = {}
    for name, fn in W.WORKLOADS.items():
        wl = fn()
        t0 = time.time()
        md = cmax.max_sqdist(wl.x, wl.y)
        res[name] = {"n": wl.n, "m": wl.m, "d": wl.d, "max_sqdist": md, "cost_scale": 1.0 / md}
        print(name, md, f"{time.time() - t0:.1f}s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
