"""Segment ladder: candidates refined while the number of segments is reduced to the coherent N_seg = 1.

Paper Sec. "Methods" (the detection statistic): for a given N_seg the statistic maximises over a phase
and an amplitude per segment; as the search progresses N_seg is reduced stage by stage, and the last
stage, N_seg = 1, is fully coherent, Upsilon_1 = max over the phase of rho^2.  Sec. "Search" uses a
particle-swarm optimiser per parameter tile at each stage; here each stage is the gradient-ascent
follow-up (``follow_up``: statistic, VJP and Adam step in HIP, step sizes set from the statistic's
resolution 0.1 / T_seg, so they shrink as the segments lengthen), started from the previous stage's
best parameters.  Every segment of a stage has the same length (N_seg fixed for all candidates).

Nothing here computes any part of the statistic: the work is done by libtfsc.so.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import BankTensors, GridSpec, PixelStore, bank_statistic, follow_up, segment_layout

DEFAULT_LADDER = (16, 8, 4, 2, 1)


@dataclass
class LadderResult:
    """Outcome of ``segment_ladder`` for n candidates."""
    nseg: tuple                              # the stages' N_seg, largest first
    start: list = field(default_factory=list)  # per stage: Upsilon_{N_seg} at the stage's starting point [n]
    best: list = field(default_factory=list)   # per stage: best Upsilon_{N_seg} reached [n]
    params: torch.Tensor | None = None       # [n][5] final (mc, f0, cos theta, phi, psi)
    upsilon1: torch.Tensor | None = None     # Upsilon_1 (coherent) at the final parameters [n]
    bank: BankTensors | None = None          # the candidates at the final parameters


def _with_params(bank: BankTensors, p: torch.Tensor) -> BankTensors:
    return BankTensors(p[:, 0].contiguous(), bank.eta, p[:, 1].contiguous(), p[:, 2].contiguous(),
                       p[:, 3].contiguous(), p[:, 4].contiguous(), bank.cos_iota)


def segment_ladder(grid: GridSpec, pixels: PixelStore, bank: BankTensors, ladder=DEFAULT_LADDER, steps: int = 30,
                   lr_scale: float = 0.5, precision: str = "f32") -> LadderResult:
    """Run the stages of ``ladder`` (N_seg values, strictly decreasing, ending at 1) on the candidates.

    Each stage takes ``steps`` ascent steps on Upsilon_{N_seg} from the previous stage's best point and
    keeps the best point it visits, so a stage never ends below where it started.  ``bank`` is not
    modified.  Returns the per-stage statistics, the final parameters and Upsilon_1 there.
    """
    ladder = tuple(int(v) for v in ladder)
    if not ladder or ladder[-1] != 1 or any(b >= a for a, b in zip(ladder, ladder[1:])) or ladder[-1] < 1:
        raise ValueError("ladder must be strictly decreasing positive N_seg values ending at 1")
    out = LadderResult(ladder)
    cur = bank
    for ns in ladder:
        first, best, params = follow_up(grid, pixels, cur, steps=steps, lr_scale=lr_scale, nseg_fixed=ns,
                                        precision=precision)
        out.start.append(first)
        out.best.append(best)
        cur = _with_params(cur, params)
    out.params = torch.stack([cur.mc, cur.f0, cur.cos_theta, cur.phi, cur.psi], dim=1)
    out.bank = cur
    out.upsilon1 = bank_statistic(grid, pixels, cur, segment_layout(grid, cur, 1), precision=precision).stat
    return out
