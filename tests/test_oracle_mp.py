"""The float64 oracle against the same formulas in 60-digit arithmetic (oracle.o2_mp), CPU only.

tests/golden/vjp_mp_small.json holds high-precision gradients written by tests/golden/make_vjp_mp.py
(oracle only).  Two effects set how close float64 can get:
* the tranche phase Phi reaches 1e9 rad, so every float64 track rounds it by ~1e-7 rad; this moves
  Upsilon by up to ~1e-8 relative for light, slowly chirping templates;
* the literal Fresnel form carries phases pi (f - f_k)^2 / fdot of 1e6 rad and more when
  beta = fdot dT^2 is small; their derivatives cancel between terms, so float64 autograd of it
  loses digits (a few 1e-6 relative at beta ~ 2e-5).
"""
import json
import os

import numpy as np
import pytest

from oracle import cpu as ocpu
from oracle import o2, o2_mp
from oracle import track as otrk

from gpu_common import small_data

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "vjp_mp_small.json")) as fh:
        return json.load(fh)


def test_mp_statistic_reproduces_float64_oracle():
    d = small_data()
    for i, tol_exact in ((0, 1e-9), (94, 1e-6)):
        ref = ocpu.statistic(d["pix"], d["u"], d["wm"], d["bank"].subset([i]), d["grid"]).stat[0]
        v64 = o2_mp.statistic(d["pix"], d["u"], d["wm"], d["bank"], d["grid"], i, float64_phase=True)
        assert abs(v64 - ref) / ref < 1e-8, i
        vex = o2_mp.statistic(d["pix"], d["u"], d["wm"], d["bank"], d["grid"], i)
        assert abs(vex - ref) / ref < tol_exact, i


def test_float64_autograd_against_high_precision(golden):
    d = small_data()
    b, g = d["bank"], d["grid"]
    lay = otrk.Layout(b, g)
    g_seg = np.random.default_rng(golden["g_seg_seed"]).normal(size=int(lay.seg_offset[-1]))
    dT = g.tranche_dur
    for key, row in golden["templates"].items():
        i = int(key)
        o = lay.seg_offset[i]
        gs = g_seg[o:o + lay.nseg[i]] + golden["g_stat"]
        grad, val = o2.gradient(d["pix"], d["u"], d["wm"], b, g, i, g_seg=gs, layout=lay)
        ref = np.array(row["grad_f64phase"])
        assert abs(val - row["value_f64phase"]) / abs(row["value_f64phase"]) < 1e-8
        rel = np.abs(grad - ref) / np.abs(ref)
        beta = lay.fdot0[i] * dT * dT
        # digits lost by the literal Fresnel form at small beta (see module docstring)
        bound = 1e-7 if beta > 1e-3 else 1e-5
        assert rel.max() < bound, (i, beta, rel)
