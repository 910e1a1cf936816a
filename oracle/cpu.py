"""Build and call the plain-C O2 oracle (``o2_cpu.c``).  Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "o2_cpu.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libo2cpu.so")

_lib = None


def build(force: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.o2_cpu_layout.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                    P, P, P, P, P, ctypes.c_int, P, P, P, ctypes.c_int]
        L.o2_cpu_statistic.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       P, P, P, ctypes.c_int64, P, P, P, P, P, P, P,
                                       P, P, P, P, P, P, P, ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class CpuResult:
    pass


def statistic(pix, u, wm, bank, grid, nseg_fixed: int | None = None, threads: int = 0,
              want_zn: bool = False) -> CpuResult:
    """O2 statistic for every template of ``bank`` (same outputs as oracle.o2.statistic)."""
    L = lib()
    n = len(bank.mc)
    cols = [np.ascontiguousarray(getattr(bank, k), dtype=np.float64) for k in
            ("mc", "eta", "f0", "cos_theta", "phi", "psi", "cos_iota")]
    mc, eta, f0, ct, ph, ps, ci = cols
    fixed = grid.nseg_fixed if nseg_fixed is None else nseg_fixed
    nseg = np.zeros(n, np.int64)
    m_end = np.zeros(n, np.int64)
    flags = np.zeros(n, np.int64)
    L.o2_cpu_layout(grid.tranche_len, grid.n_tranches, grid.dt, n, _p(mc), _p(eta), _p(f0), _p(ct), _p(ci),
                    int(fixed or 0), _p(nseg), _p(m_end), _p(flags), threads)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(nseg)
    pixc = np.ascontiguousarray(np.asarray(pix, dtype=np.complex128))
    u = np.ascontiguousarray(u, dtype=np.float64)
    wm = np.ascontiguousarray(wm, dtype=np.float64)
    seg = np.zeros(int(off[-1]))
    stat = np.zeros(n)
    zn = np.zeros((int(off[-1]), 3)) if want_zn else None
    C = pixc.shape[0]
    L.o2_cpu_statistic(C, grid.tranche_len, grid.n_tranches, grid.dt, _p(pixc), _p(u), _p(wm), n,
                       _p(mc), _p(eta), _p(f0), _p(ct), _p(ph), _p(ps), _p(ci), _p(nseg), _p(off), _p(m_end),
                       _p(flags), _p(seg), _p(stat), _p(zn) if zn is not None else None, threads)
    r = CpuResult()
    r.stat, r.seg_terms, r.seg_offset, r.nseg, r.m_end, r.flags, r.seg_zn = stat, seg, off, nseg, m_end, flags, zn
    return r
