"""Batching around the statistic: launch-shape autotuning and HIP-graph replay over noise realisations.

Paper Sec. "Hardware acceleration and computational cost": the method evaluates large batches of
parameter sets per launch.  Here that is one persistent launch over the whole bank, with

* ``autotune``: the WAVE schedule's launch shape (waves per block, resident blocks per compute unit)
  chosen by the library's tuner (tfsc_tune_statistic: candidates timed with HIP events on a tuning
  bank), cached in a JSON file keyed by the device and the workload's shape;
* ``RealisationGraph``: the sequence transform(r) -> bank_statistic(r) for R noise realisations of
  the same grid, captured once into a HIP graph (torch.cuda.CUDAGraph) and replayed.  Every kernel
  in it is a launch (work counters are cleared by a fill kernel, never by a memset node).

Nothing here computes any part of the statistic: the work is done by libtfsc.so.
"""
from __future__ import annotations

import json
import os

import torch

import ctypes

from . import (BankTensors, GridSpec, PixelStore, SegmentLayout, StatResult, TfscError, _lib, bank_statistic,
               bank_statistic_interleaved, bank_statistic_multi, interleave_store, interleaved_store, lib,
               realisation_stores, transform, tune_statistic)


def _cache_path(path: str | None) -> str:
    if path:
        return path
    env = os.environ.get("TFSC_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "tfsc", "launch_shapes.json")


def _key(grid: GridSpec, pixels: PixelStore, precision: str) -> str:
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{name}|C{grid.n_channels}|M{grid.tranche_len}|Nt{grid.n_tranches}|{pixels.dtype}|{precision}"


def autotune(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout, precision: str = "f32",
             order: torch.Tensor | None = None, cache: str | None = None, refresh: bool = False) -> tuple[int, int]:
    """(block_waves, groups_per_cu) with the shortest WAVE statistic launch on ``bank`` (a tuning bank).

    The timing is the library's own tuner (tfsc_tune_statistic, eight launch shapes); the result is also cached
    on disk under the device name and workload shape, and ``refresh`` re-times it.
    """
    path = _cache_path(cache)
    key = _key(grid, pixels, precision)
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
    if key in table and not refresh:
        bw, gpc = table[key]["shape"]
        return int(bw), int(gpc)
    best = tune_statistic(grid, pixels, bank, seg, key, precision=precision, order=order)
    table[key] = {"shape": list(best), "tuning_templates": bank.n}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(table, fh, indent=1)
    except OSError:
        pass  # a read-only home only loses the cache
    return int(best[0]), int(best[1])


class RealisationGraph:
    """transform(r) -> bank_statistic(r) for R realisations, captured into one HIP graph.

    xs: [R][C][N] device time series (f32 or f64).  The pixel stores (``layout``: "layer_ci" or
    "layer", the two the WAVE schedule reads), results and workspace are
    allocated once (eager warm-up) and reused by every replay; ``results[r]`` holds realisation r's
    output after ``replay()``.  multi=True keeps the stores in one block and evaluates every
    realisation in one pass over the bank (bank_statistic_multi) instead of one launch each.
    interleave=NR (2 or 4; f32 or i16 channel-interleaved stores) transforms each realisation into one staging
    store, copies it into its slot of an interleaved store of NR realisations, and evaluates each group of
    NR realisations in one pass over the bank (bank_statistic_interleaved); R must be a multiple of NR.
    """

    def __init__(self, grid: GridSpec, xs: torch.Tensor, psd0: torch.Tensor, mu: torch.Tensor, keep: torch.Tensor,
                 bank: BankTensors, seg: SegmentLayout, store: str = "f32", precision: str = "f32",
                 order: torch.Tensor | None = None, block_waves: int = 0, groups_per_cu: int = 0,
                 layout: str = "layer_ci", multi: bool = False, group: int = 0, interleave: int = 0):
        self.grid, self.xs, self.psd0, self.mu, self.keep = grid, xs, psd0, mu, keep
        self.bank, self.seg, self.store, self.precision, self.order = bank, seg, store, precision, order
        self.shape = dict(block_waves=block_waves, groups_per_cu=groups_per_cu)
        self.multi, self.group, self.interleave = multi, group, interleave
        R = xs.shape[0]
        dev = bank.device
        L = lib()
        g = grid.c()
        nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, None, _lib.WS_STATISTIC)
        self.ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        if interleave:
            if store not in ("f32", "i16") or layout != "layer_ci" or precision != "f32" or R % interleave:
                raise TfscError("interleaved realisations take f32 or i16 channel-interleaved stores, R a "
                                "multiple of NR")
            self.staging = transform(grid, xs[0], psd0, mu, keep, dtype=store, layout="layer_ci")
            self.groups = []
            for q in range(R // interleave):
                ri = interleaved_store(grid, interleave, self.staging)
                for j in range(interleave):
                    transform(grid, xs[q * interleave + j], psd0, mu, keep, dtype=store, layout="layer_ci",
                              out=self.staging)
                    interleave_store(grid, self.staging, interleave, j, ri)
                res = bank_statistic_interleaved(grid, ri, interleave, bank, seg, order=order, ws=self.ws,
                                                 **self.shape)
                self.groups.append((ri, res))
            self.stores = [grp[0] for grp in self.groups]
            self.results = [grp[1].realisation(r) for grp in self.groups for r in range(interleave)]
            torch.cuda.synchronize()
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._enqueue()
            return
        if multi:
            self.stores = realisation_stores(grid, R, dtype=store, layout=layout, device=dev)
            for r in range(R):
                transform(grid, xs[r], psd0, mu, keep, dtype=store, out=self.stores[r])
        else:
            self.stores = [transform(grid, xs[r], psd0, mu, keep, dtype=store, layout=layout) for r in range(R)]
        if multi:
            self.multi_result = bank_statistic_multi(grid, self.stores, bank, seg, precision=precision, order=order,
                                                     ws=self.ws, group=group, **self.shape)
            self.results = [self.multi_result.realisation(r) for r in range(R)]
        else:
            self.results = [bank_statistic(grid, self.stores[r], bank, seg, precision=precision, schedule="wave",
                                           order=order, ws=self.ws, **self.shape) for r in range(R)]
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()

    def _enqueue(self):
        if self.interleave:
            NR = self.interleave
            for q, (ri, res) in enumerate(self.groups):
                for j in range(NR):
                    transform(self.grid, self.xs[q * NR + j], self.psd0, self.mu, self.keep, dtype=self.store,
                              layout="layer_ci", out=self.staging)
                    interleave_store(self.grid, self.staging, NR, j, ri)
                bank_statistic_interleaved(self.grid, ri, NR, self.bank, self.seg, order=self.order, out=res,
                                           ws=self.ws, **self.shape)
            return
        for r in range(self.xs.shape[0]):
            transform(self.grid, self.xs[r], self.psd0, self.mu, self.keep, dtype=self.store, out=self.stores[r])
            if not self.multi:
                bank_statistic(self.grid, self.stores[r], self.bank, self.seg, precision=self.precision,
                               schedule="wave", order=self.order, out=self.results[r], ws=self.ws, **self.shape)
        if self.multi:
            bank_statistic_multi(self.grid, self.stores, self.bank, self.seg, precision=self.precision,
                                 order=self.order, out=self.multi_result, ws=self.ws, group=self.group, **self.shape)

    def replay(self) -> list[StatResult]:
        self.graph.replay()
        return self.results

    def eager(self) -> list[StatResult]:
        """The same work launched directly (for comparison with the graph)."""
        self._enqueue()
        return self.results
