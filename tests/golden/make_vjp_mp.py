"""Write vjp_mp_small.json and vjp_mp_aet.json: high-precision gradients for the two-channel gapped test data and
for the small-beta templates of the three-channel test data.

Calls only the oracle (oracle.o2_mp at 60 digits) and the seeded input generators.  Run from the
repository root:  python tests/golden/make_vjp_mp.py
The GPU VJP test compares the kernel's FP64 gradients with these values.
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

TEMPLATES = [0, 4, 6, 93, 94, 95]
G_STAT = 0.5
G_SEG_SEED = 5


def _one(i):
    from gpu_common import small_data
    from oracle import o2_mp
    from oracle import track as otrk
    d = small_data()
    lay = otrk.Layout(d["bank"], d["grid"])
    g_seg = np.random.default_rng(G_SEG_SEED).normal(size=int(lay.seg_offset[-1]))
    o = lay.seg_offset[i]
    gs = g_seg[o:o + lay.nseg[i]] + G_STAT
    val, grad = o2_mp.gradient(d["pix"], d["u"], d["wm"], d["bank"], d["grid"], i, g_seg=gs)
    val64, grad64 = o2_mp.gradient(d["pix"], d["u"], d["wm"], d["bank"], d["grid"], i, g_seg=gs,
                                   float64_phase=True)
    return i, val, grad.tolist(), val64, grad64.tolist()


AET_TEMPLATES = [0, 3, 38]  # the three-channel test's templates with beta = fdot0 dT^2 below 1e-3


def _one_aet(i):
    from test_gpu_t_channel import _data
    from oracle import o2_mp
    d = _data()
    val64, grad64 = o2_mp.gradient(d["pix"], d["u"], d["wm"], d["bank"], d["grid"], i, float64_phase=True)
    return i, val64, grad64.tolist()


def main():
    with Pool(min(len(AET_TEMPLATES), 8)) as pool:
        rows = pool.map(_one_aet, AET_TEMPLATES)
    out = {
        "about": "Upsilon and its gradient w.r.t. (ln Mc, f0, cos theta, phi, psi) for the small-beta templates of "
                 "the three-channel (A, E, T) test data of tests/test_gpu_t_channel.py; oracle.o2_mp at 60 digits, "
                 "central differences with step 1e-15, exact except for the float64 rounding of the tranche "
                 "phases, which every float64 track shares",
        "command": "python tests/golden/make_vjp_mp.py",
        "templates": {str(i): {"value_f64phase": v64, "grad_f64phase": g64} for i, v64, g64 in rows},
    }
    with open(os.path.join(HERE, "vjp_mp_aet.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", len(rows), "three-channel templates")
    with Pool(min(len(TEMPLATES), 8)) as pool:
        rows = pool.map(_one, TEMPLATES)
    out = {
        "about": "sum_n g_n Upsilon_n and its gradient w.r.t. (ln Mc, f0, cos theta, phi, psi) for templates of the "
                 "two-channel gapped test bank (small_data), g_n = g_seg[n] + g_stat with g_seg ~ N(0, 1) from "
                 "numpy default_rng(seed); oracle.o2_mp at 60 digits, central differences with step 1e-15. "
                 "'value'/'grad': exact arithmetic; 'value_f64phase'/'grad_f64phase': exact except for the "
                 "float64 rounding of the tranche phases, which every float64 track shares",
        "command": "python tests/golden/make_vjp_mp.py",
        "g_stat": G_STAT,
        "g_seg_seed": G_SEG_SEED,
        "templates": {str(i): {"value": v, "grad": g, "value_f64phase": v64, "grad_f64phase": g64}
                      for i, v, g, v64, g64 in rows},
    }
    with open(os.path.join(HERE, "vjp_mp_small.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", len(rows), "templates")


if __name__ == "__main__":
    main()
