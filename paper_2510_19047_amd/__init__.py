"""tfsc: the semi-coherent time-frequency detection statistic of arXiv 2510.19047 on MI355X.

Every step runs in the HIP kernels of ``libtfsc.so`` (C ABI in include/tfsc.h).
This module only marshals torch device tensors and the current HIP stream into
those calls; it never computes any part of the statistic itself, and it raises
if the library is missing or if a tensor is not on the GPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import TfscError

__all__ = ["GridSpec", "PixelStore", "BankTensors", "SegmentLayout", "StatResult", "transform", "transform_tf", "segment_layout",
           "bank_statistic", "bank_statistic_multi", "bank_statistic_harmonics", "realisation_stores", "MultiResult",
           "statistic_vjp", "track", "tile_max", "orbit_positions", "link_lengths", "tune_statistic", "TFSCStatistic", "lib",
           "TfscError", "interleaved_store", "interleave_store", "interleave_stores", "bank_statistic_interleaved"]

_DTYPE = {"f64": _lib.F64, "f32": _lib.F32, "bf16": _lib.BF16, "f16": _lib.F16, "i16": _lib.I16}
_TORCH_STORE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
                "i16": torch.int16}
_STORE16 = ("bf16", "f16", "i16")
_LAYOUT = {"layer": _lib.LAYER_MAJOR, "tranche": _lib.TRANCHE_MAJOR, "layer_ci": _lib.LAYER_MAJOR_CI}
_SCHED = {"thread": _lib.SCHED_THREAD, "wave": _lib.SCHED_WAVE}
_PREC = {"f64": _lib.F64, "f32": _lib.F32}
_FRESNEL = {"paper": _lib.FRESNEL_PAPER, "accurate": _lib.FRESNEL_ACCURATE}


def lib():
    return _lib.load()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise TfscError("tfsc calls take device tensors only")
    if not t.is_contiguous():
        raise TfscError("tfsc calls take contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class GridSpec:
    """Sampling grid: C channels, Nt tranches of M samples at cadence dt."""
    n_channels: int
    tranche_len: int
    n_tranches: int
    dt: float = 5.0
    tukey_alpha: float = 0.1

    @property
    def n_bins(self) -> int:
        return self.tranche_len // 2 + 1

    def c(self) -> _lib.Grid:
        return _lib.Grid(self.n_channels, self.tranche_len, self.n_tranches, 21, float(self.dt), float(self.tukey_alpha))


@dataclass
class PixelStore:
    """Whitened TF pixels plus template weights (see tfsc_pixels)."""
    pix: torch.Tensor                 # [C][K][Nt][2] (layer), [C][Nt][K][2] (tranche) or [K][Nt][C][2] (layer_ci)
    inv_asd: torch.Tensor             # [K] f64
    tranche_w: torch.Tensor           # [Nt] f64
    dtype: str = "f32"
    layout: str = "layer"
    layer_scale: torch.Tensor | None = None  # [C][K] f32 for 16-bit stores (bf16, f16, i16)
    rho: torch.Tensor | None = None   # [K][Nt] f32 per-pixel weight factor of a general per-tranche PSD
    orbit: torch.Tensor | None = None  # [3][3][Nt] f64 spacecraft positions (light-seconds), None = analytic orbit
    links: torch.Tensor | None = None  # [6][Nt] f64 link light times (seconds), None = equal arms
    tdi_generation: int = 1            # 2: second-generation TDI (with links)

    def c(self) -> _lib.Pixels:
        return _lib.Pixels(_DTYPE[self.dtype], _LAYOUT[self.layout], _ptr(self.pix), _ptr(self.layer_scale),
                           _ptr(self.inv_asd), _ptr(self.tranche_w), _ptr(self.rho), _ptr(self.orbit),
                           _ptr(self.links), int(self.tdi_generation))

    @staticmethod
    def from_complex(pix: torch.Tensor, inv_asd: torch.Tensor, tranche_w: torch.Tensor, dtype: str = "f64",
                     layout: str = "layer") -> "PixelStore":
        """Wrap complex [C][K][Nt] pixels (already whitened) as a store of FP64 or FP32 values."""
        if dtype not in ("f64", "f32"):
            raise TfscError("from_complex stores f64 or f32; 16-bit stores come from transform()")
        if layout not in _LAYOUT:
            raise TfscError(f"unknown pixel layout {layout!r}")
        p = {"layer": pix, "tranche": pix.transpose(1, 2), "layer_ci": pix.permute(1, 2, 0)}[layout]
        real = torch.view_as_real(p.contiguous().to(torch.complex128 if dtype == "f64" else torch.complex64))
        return PixelStore(real.contiguous(), inv_asd.to(torch.float64).contiguous(),
                          tranche_w.to(torch.float64).contiguous(), dtype, layout)


@dataclass
class BankTensors:
    """Template parameters as FP64 device tensors (see tfsc_bank).  The chirp mass is given either as ``mc`` or
    as ``ln_mc`` (then ``mc`` is None and the library forms exp(ln_mc) on the device)."""
    mc: torch.Tensor | None
    eta: torch.Tensor
    f0: torch.Tensor
    cos_theta: torch.Tensor
    phi: torch.Tensor
    psi: torch.Tensor
    cos_iota: torch.Tensor
    ln_mc: torch.Tensor | None = None

    FIELDS = ("mc", "eta", "f0", "cos_theta", "phi", "psi", "cos_iota")

    @property
    def n(self) -> int:
        return int((self.mc if self.mc is not None else self.ln_mc).numel())

    @property
    def device(self):
        return (self.mc if self.mc is not None else self.ln_mc).device

    @staticmethod
    def from_host(bank, device="cuda") -> "BankTensors":
        import numpy as np
        return BankTensors(*(torch.as_tensor(np.ascontiguousarray(getattr(bank, k), dtype=np.float64), device=device)
                             for k in BankTensors.FIELDS))

    def c(self) -> _lib.Bank:
        return _lib.Bank(self.n, *(_ptr(getattr(self, k)) for k in self.FIELDS), _ptr(self.ln_mc))


@dataclass
class SegmentLayout:
    nseg: torch.Tensor        # [n] int32
    seg_offset: torch.Tensor  # [n+1] int64
    nseg_fixed: int = 0
    total: int = 0            # seg_offset[n], read once on the host

    def c(self) -> _lib.Segments:
        return _lib.Segments(int(self.nseg_fixed), _ptr(self.nseg), _ptr(self.seg_offset))


@dataclass
class StatResult:
    stat: torch.Tensor        # [n] f64
    seg_terms: torch.Tensor   # [total] f64
    flags: torch.Tensor       # [n] int32
    seg_zn: torch.Tensor | None = None  # [total][3] f64
    n_active: torch.Tensor | None = None  # [n] int32


def _options(precision="f32", schedule="wave", block_waves=0, groups_per_cu=0, order=None, fresnel="paper",
             tune_key: str | None = None) -> _lib.Options:
    return _lib.Options(_PREC[precision], _SCHED[schedule], int(block_waves), int(groups_per_cu), _ptr(order),
                        _FRESNEL[fresnel], None if tune_key is None else tune_key.encode())


def transform(grid: GridSpec, x: torch.Tensor, psd0: torch.Tensor, mu: torch.Tensor, keep: torch.Tensor,
              dtype: str = "f32", layout: str = "layer", out: PixelStore | None = None) -> PixelStore:
    """tfsc_transform: time series [C][N] (f64 or f32) -> whitened pixel store."""
    L = lib()
    dev = x.device
    K, Nt, C = grid.n_bins, grid.n_tranches, grid.n_channels
    if out is None:
        if layout not in _LAYOUT:
            raise TfscError(f"unknown pixel layout {layout!r}")
        shape = {"layer": (C, K, Nt, 2), "tranche": (C, Nt, K, 2), "layer_ci": (K, Nt, C, 2)}[layout]
        out = PixelStore(torch.empty(shape, dtype=_TORCH_STORE[dtype], device=dev),
                         torch.empty(K, dtype=torch.float64, device=dev), torch.empty(Nt, dtype=torch.float64, device=dev),
                         dtype, layout,
                         torch.empty((C, K), dtype=torch.float32, device=dev) if dtype in _STORE16 else None)
    g = grid.c()
    xd = _lib.F64 if x.dtype == torch.float64 else _lib.F32
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), 0, None, _lib.WS_TRANSFORM)
    ws = _ws(nb, dev) if dtype in _STORE16 else None
    pc = out.c()
    st = L.tfsc_transform(ctypes.byref(g), _ptr(x), xd, _ptr(psd0), _ptr(mu), _ptr(keep), ctypes.byref(pc),
                          _ptr(ws), nb if ws is not None else 0, _stream())
    _lib.check(st, "tfsc_transform")
    return out


def transform_tf(grid: GridSpec, x: torch.Tensor, psd_tf: torch.Tensor, keep: torch.Tensor, dtype: str = "f32",
                 layout: str = "layer", out: PixelStore | None = None) -> PixelStore:
    """tfsc_transform_tf: time series [C][N] -> pixel store whitened by a PSD given per (bin, tranche),
    psd_tf[K][Nt] = S_m(f_k) (f64, device); the store carries the per-pixel weight factor ``rho``."""
    L = lib()
    dev = x.device
    K, Nt, C = grid.n_bins, grid.n_tranches, grid.n_channels
    if tuple(psd_tf.shape) != (K, Nt) or psd_tf.dtype != torch.float64 or not psd_tf.is_contiguous():
        raise TfscError(f"psd_tf must be a contiguous float64 [{K}, {Nt}] tensor")
    if out is None:
        if layout not in _LAYOUT:
            raise TfscError(f"unknown pixel layout {layout!r}")
        shape = {"layer": (C, K, Nt, 2), "tranche": (C, Nt, K, 2), "layer_ci": (K, Nt, C, 2)}[layout]
        out = PixelStore(torch.empty(shape, dtype=_TORCH_STORE[dtype], device=dev),
                         torch.empty(K, dtype=torch.float64, device=dev), torch.empty(Nt, dtype=torch.float64, device=dev),
                         dtype, layout,
                         torch.empty((C, K), dtype=torch.float32, device=dev) if dtype in _STORE16 else None,
                         torch.empty((K, Nt), dtype=torch.float32, device=dev))
    elif out.rho is None:
        raise TfscError("transform_tf needs a store with a rho tensor")
    g = grid.c()
    xd = _lib.F64 if x.dtype == torch.float64 else _lib.F32
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), 0, None, _lib.WS_TRANSFORM)
    ws = _ws(nb, dev) if dtype in _STORE16 else None
    pc = out.c()
    st = L.tfsc_transform_tf(ctypes.byref(g), _ptr(x), xd, _ptr(psd_tf), _ptr(keep), ctypes.byref(pc), _ptr(ws),
                             nb if ws is not None else 0, _stream())
    _lib.check(st, "tfsc_transform_tf")
    return out


def segment_layout(grid: GridSpec, bank: BankTensors, nseg_fixed: int = 0, out: SegmentLayout | None = None,
                   read_total: bool = True) -> SegmentLayout:
    """tfsc_segment_layout: N_seg per template and CSR offsets (reads the total back unless told not to)."""
    L = lib()
    dev = bank.device
    seg = out if out is not None else SegmentLayout(torch.empty(bank.n, dtype=torch.int32, device=dev),
                                                    torch.empty(bank.n + 1, dtype=torch.int64, device=dev), nseg_fixed)
    g = grid.c()
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, None, _lib.WS_LAYOUT)
    ws = _ws(nb, dev)
    sc = seg.c()
    bc = bank.c()
    st = L.tfsc_segment_layout(ctypes.byref(g), ctypes.byref(bc), ctypes.byref(sc), _ptr(ws), nb, _stream())
    _lib.check(st, "tfsc_segment_layout")
    if read_total:
        seg.total = int(seg.seg_offset[-1].item())
    return seg


def bank_statistic(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout,
                   precision: str = "f32", schedule: str = "wave", want_zn: bool = False, block_waves: int = 0,
                   groups_per_cu: int = 0, order: torch.Tensor | None = None, out: StatResult | None = None,
                   ws: torch.Tensor | None = None, want_active: bool = False, fresnel: str = "paper",
                   tune_key: str | None = None) -> StatResult:
    """tfsc_bank_statistic: Upsilon, per-segment terms and flags for every template (``fresnel``: "paper" for the
    paper's Fresnel forms, "accurate" for the Fresnel integrals)."""
    L = lib()
    dev = bank.device
    if out is None:
        out = StatResult(torch.empty(bank.n, dtype=torch.float64, device=dev),
                         torch.empty(max(seg.total, 1), dtype=torch.float64, device=dev),
                         torch.empty(bank.n, dtype=torch.int32, device=dev),
                         torch.empty((max(seg.total, 1), 3), dtype=torch.float64, device=dev) if want_zn else None,
                         torch.empty(bank.n, dtype=torch.int32, device=dev) if want_active else None)
    g = grid.c()
    opt = _options(precision, schedule, block_waves, groups_per_cu, order, fresnel, tune_key)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_STATISTIC)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    pc, bc, sc = pixels.c(), bank.c(), seg.c()
    st = L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(sc),
                               ctypes.byref(opt), _ptr(out.seg_terms), _ptr(out.stat), _ptr(out.seg_zn),
                               _ptr(out.flags), _ptr(out.n_active), _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "tfsc_bank_statistic")
    return out


def bank_statistic_noalloc(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout,
                           precision: str = "f32", schedule: str = "wave", want_zn: bool = False,
                           block_waves: int = 0, groups_per_cu: int = 0, order: torch.Tensor | None = None,
                           out: StatResult | None = None, want_active: bool = False) -> StatResult:
    """tfsc_bank_statistic_noalloc: bank_statistic with the library's static device scratch as workspace (the
    call allocates no device memory; outputs are allocated here only when ``out`` is not given)."""
    L = lib()
    dev = bank.device
    if out is None:
        out = StatResult(torch.empty(bank.n, dtype=torch.float64, device=dev),
                         torch.empty(max(seg.total, 1), dtype=torch.float64, device=dev),
                         torch.empty(bank.n, dtype=torch.int32, device=dev),
                         torch.empty((max(seg.total, 1), 3), dtype=torch.float64, device=dev) if want_zn else None,
                         torch.empty(bank.n, dtype=torch.int32, device=dev) if want_active else None)
    g = grid.c()
    opt = _options(precision, schedule, block_waves, groups_per_cu, order)
    pc, bc, sc = pixels.c(), bank.c(), seg.c()
    st = L.tfsc_bank_statistic_noalloc(ctypes.byref(g), ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(sc),
                                       ctypes.byref(opt), _ptr(out.seg_terms), _ptr(out.stat), _ptr(out.seg_zn),
                                       _ptr(out.flags), _ptr(out.n_active), _stream())
    _lib.check(st, "tfsc_bank_statistic_noalloc")
    return out


def bank_statistic_harmonics(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout,
                             harmonics, amp: torch.Tensor, precision: str = "f32", want_zn: bool = False,
                             block_waves: int = 0, groups_per_cu: int = 0, order: torch.Tensor | None = None,
                             out: StatResult | None = None, want_active: bool = False) -> StatResult:
    """tfsc_bank_statistic_harmonics: the statistic of templates made of harmonics h (of the orbital phase) with
    complex factors amp [n][H] (complex128, or float64 [n][H][2]) per template and harmonic."""
    L = lib()
    dev = bank.device
    hs = [int(h) for h in harmonics]
    H = len(hs)
    if amp.dtype == torch.complex128:
        amp = torch.view_as_real(amp.contiguous())
    if tuple(amp.shape) != (bank.n, H, 2) or amp.dtype != torch.float64:
        raise TfscError(f"amp must be complex128 [{bank.n}, {H}] or float64 [{bank.n}, {H}, 2]")
    amp = amp.contiguous()
    if out is None:
        out = StatResult(torch.empty(bank.n, dtype=torch.float64, device=dev),
                         torch.empty(max(seg.total, 1), dtype=torch.float64, device=dev),
                         torch.empty(bank.n, dtype=torch.int32, device=dev),
                         torch.empty((max(seg.total, 1), 3), dtype=torch.float64, device=dev) if want_zn else None,
                         torch.empty(bank.n, dtype=torch.int32, device=dev) if want_active else None)
    g = grid.c()
    opt = _options(precision, "wave", block_waves, groups_per_cu, order)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_STATISTIC)
    ws = _ws(nb, dev)
    harr = (ctypes.c_int32 * max(H, 1))(*hs)
    pc, bc, sc = pixels.c(), bank.c(), seg.c()
    st = L.tfsc_bank_statistic_harmonics(ctypes.byref(g), ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(sc),
                                         ctypes.byref(opt), H, harr, _ptr(amp), _ptr(out.seg_terms), _ptr(out.stat),
                                         _ptr(out.seg_zn), _ptr(out.flags), _ptr(out.n_active), _ptr(ws), ws.numel(),
                                         _stream())
    _lib.check(st, "tfsc_bank_statistic_harmonics")
    return out


def orbit_positions(grid: GridSpec, device="cuda") -> torch.Tensor:
    """tfsc_orbit_positions: the analytic orbit's spacecraft positions [3][3][Nt] (light-seconds, FP64)."""
    L = lib()
    out = torch.empty((3, 3, grid.n_tranches), dtype=torch.float64, device=device)
    g = grid.c()
    _lib.check(L.tfsc_orbit_positions(ctypes.byref(g), _ptr(out), _stream()), "tfsc_orbit_positions")
    return out


def link_lengths(grid: GridSpec, orbit: torch.Tensor | None = None, device="cuda") -> torch.Tensor:
    """tfsc_link_lengths: |p_r - p_s| of the six links [6][Nt] (seconds, FP64) of ``orbit`` [3][3][Nt] or of the
    analytic orbit (None)."""
    L = lib()
    out = torch.empty((6, grid.n_tranches), dtype=torch.float64, device=device)
    g = grid.c()
    _lib.check(L.tfsc_link_lengths(ctypes.byref(g), _ptr(orbit), _ptr(out), _stream()), "tfsc_link_lengths")
    return out


def tune_statistic(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout, tune_key: str,
                   precision: str = "f32", order: torch.Tensor | None = None) -> tuple[int, int]:
    """tfsc_tune_statistic: the library's launch-shape autotuner on a tuning bank; returns (block_waves,
    groups_per_cu), also kept by the library under ``tune_key`` for bank_statistic(..., tune_key=...)."""
    L = lib()
    dev = bank.device
    res = StatResult(torch.empty(bank.n, dtype=torch.float64, device=dev),
                     torch.empty(max(seg.total, 1), dtype=torch.float64, device=dev),
                     torch.empty(bank.n, dtype=torch.int32, device=dev))
    g = grid.c()
    opt = _options(precision, "wave", 0, 0, order)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_STATISTIC)
    ws = _ws(nb, dev)
    pc, bc, sc = pixels.c(), bank.c(), seg.c()
    bw, gpc = ctypes.c_int32(0), ctypes.c_int32(0)
    st = L.tfsc_tune_statistic(ctypes.byref(g), ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(sc),
                               ctypes.byref(opt), tune_key.encode(), _ptr(res.seg_terms), _ptr(res.stat),
                               _ptr(res.flags), _ptr(ws), ws.numel(), _stream(), ctypes.byref(bw), ctypes.byref(gpc))
    _lib.check(st, "tfsc_tune_statistic")
    return int(bw.value), int(gpc.value)


def realisation_stores(grid: GridSpec, n_real: int, dtype: str = "f32", layout: str = "layer_ci",
                       device="cuda") -> list:
    """n_real pixel stores in one contiguous block (the input of bank_statistic_multi), sharing inv_asd and
    tranche_w; fill them with ``transform(..., out=stores[r])``."""
    if dtype not in ("f32", "f64") or layout not in ("layer", "layer_ci"):
        raise TfscError("several realisations take f32 or f64 stores in a layer-major layout")
    K, Nt, C = grid.n_bins, grid.n_tranches, grid.n_channels
    shape = (C, K, Nt, 2) if layout == "layer" else (K, Nt, C, 2)
    block = torch.empty((n_real, *shape), dtype=_TORCH_STORE[dtype], device=device)
    inv_asd = torch.empty(K, dtype=torch.float64, device=device)
    tranche_w = torch.empty(Nt, dtype=torch.float64, device=device)
    return [PixelStore(block[r], inv_asd, tranche_w, dtype, layout) for r in range(n_real)]


@dataclass
class MultiResult:
    """bank_statistic_multi outputs: stat [R][n], seg_terms [R][total], flags and n_active [n] (shared)."""
    stat: torch.Tensor
    seg_terms: torch.Tensor
    flags: torch.Tensor
    n_active: torch.Tensor | None = None

    def realisation(self, r: int) -> "StatResult":
        return StatResult(self.stat[r], self.seg_terms[r], self.flags, None, self.n_active)


def bank_statistic_multi(grid: GridSpec, stores: list, bank: BankTensors, seg: SegmentLayout, precision: str = "f32",
                         block_waves: int = 0, groups_per_cu: int = 0, order: torch.Tensor | None = None,
                         out: MultiResult | None = None, ws: torch.Tensor | None = None,
                         want_active: bool = False, group: int = 0) -> MultiResult:
    """tfsc_bank_statistic_multi: the statistic of every realisation in ``stores`` (from realisation_stores,
    or any stores laid out at one stride in one block), ``group`` realisations (1, 2, 4, 8; 0 = 8) per pass
    over the bank."""
    L = lib()
    dev = bank.device
    R = len(stores)
    if R == 0:
        raise TfscError("no realisations")
    p0 = stores[0].pix
    stride = (stores[1].pix.data_ptr() - p0.data_ptr()) if R > 1 else p0.numel() * p0.element_size()
    for r in range(1, R):
        if stores[r].pix.data_ptr() - p0.data_ptr() != r * stride:
            raise TfscError("realisation stores must lie at one stride in one block")
    total = max(seg.total, 1)
    if out is None:
        out = MultiResult(torch.empty((R, bank.n), dtype=torch.float64, device=dev),
                          torch.empty((R, total), dtype=torch.float64, device=dev),
                          torch.empty(bank.n, dtype=torch.int32, device=dev),
                          torch.empty(bank.n, dtype=torch.int32, device=dev) if want_active else None)
    g = grid.c()
    opt = _options(precision, "wave", block_waves, groups_per_cu, order)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_STATISTIC)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    pc, bc, sc = stores[0].c(), bank.c(), seg.c()
    st = L.tfsc_bank_statistic_multi(ctypes.byref(g), ctypes.byref(pc), R, stride, int(group), ctypes.byref(bc),
                                     ctypes.byref(sc),
                                     ctypes.byref(opt), out.seg_terms.shape[1], _ptr(out.seg_terms), _ptr(out.stat),
                                     _ptr(out.flags), _ptr(out.n_active), _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "tfsc_bank_statistic_multi")
    return out


def interleaved_store(grid: GridSpec, n_real: int, like: PixelStore) -> PixelStore:
    """An (uninitialised) store [K][Nt][n_real][C] for n_real interleaved realisations of like's dtype (f32, or
    i16 with layer scales [n_real C][K]) and weights."""
    K, Nt, C = grid.n_bins, grid.n_tranches, grid.n_channels
    if like.dtype not in ("f32", "i16"):
        raise TfscError("interleaved stores hold f32 or i16 pixels")
    dev = like.pix.device
    return PixelStore(torch.empty((K, Nt, n_real * C, 2), dtype=_TORCH_STORE[like.dtype], device=dev),
                      like.inv_asd, like.tranche_w, like.dtype, "layer_ci",
                      torch.empty((n_real * C, K), dtype=torch.float32, device=dev) if like.dtype == "i16" else None,
                      None, like.orbit, like.links, like.tdi_generation)


def interleave_store(grid: GridSpec, src: PixelStore, n_real: int, r: int, out: PixelStore) -> PixelStore:
    """tfsc_interleave_store: realisation r (an f32 or i16 channel-interleaved store) into slot r of ``out``."""
    L = lib()
    g, pc, oc = grid.c(), src.c(), out.c()
    _lib.check(L.tfsc_interleave_store(ctypes.byref(g), ctypes.byref(pc), int(n_real), int(r), ctypes.byref(oc),
                                       _stream()), "tfsc_interleave_store")
    return out


def interleave_stores(grid: GridSpec, stores: list, out: PixelStore | None = None) -> PixelStore:
    """One FP32 store [K][Nt][R][C] holding the R stores' pixels cell by cell (weights of the first store)."""
    R = len(stores)
    if out is None:
        out = interleaved_store(grid, R, stores[0])
    for r, s in enumerate(stores):
        interleave_store(grid, s, R, r, out)
    return out


def bank_statistic_interleaved(grid: GridSpec, store: PixelStore, n_real: int, bank: BankTensors, seg: SegmentLayout,
                               block_waves: int = 0, groups_per_cu: int = 0, order: torch.Tensor | None = None,
                               out: MultiResult | None = None, ws: torch.Tensor | None = None,
                               want_active: bool = False) -> MultiResult:
    """tfsc_bank_statistic_multi with real_stride 0: the statistic of the n_real realisations interleaved in
    ``store`` (from interleave_stores), all of them in one pass over the bank."""
    L = lib()
    dev = bank.device
    total = max(seg.total, 1)
    if out is None:
        out = MultiResult(torch.empty((n_real, bank.n), dtype=torch.float64, device=dev),
                          torch.empty((n_real, total), dtype=torch.float64, device=dev),
                          torch.empty(bank.n, dtype=torch.int32, device=dev),
                          torch.empty(bank.n, dtype=torch.int32, device=dev) if want_active else None)
    g = grid.c()
    opt = _options("f32", "wave", block_waves, groups_per_cu, order)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_STATISTIC)
    if ws is None or ws.numel() < nb:
        ws = _ws(nb, dev)
    pc, bc, sc = store.c(), bank.c(), seg.c()
    st = L.tfsc_bank_statistic_multi(ctypes.byref(g), ctypes.byref(pc), int(n_real), 0, 0, ctypes.byref(bc),
                                     ctypes.byref(sc), ctypes.byref(opt), out.seg_terms.shape[1],
                                     _ptr(out.seg_terms), _ptr(out.stat), _ptr(out.flags), _ptr(out.n_active),
                                     _ptr(ws), ws.numel(), _stream())
    _lib.check(st, "tfsc_bank_statistic_multi")
    return out


def statistic_vjp(grid: GridSpec, pixels: PixelStore, bank: BankTensors, seg: SegmentLayout, seg_zn: torch.Tensor,
                  g_stat: torch.Tensor | None = None, g_seg: torch.Tensor | None = None, precision: str = "f64",
                  block_waves: int = 0, groups_per_cu: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """tfsc_statistic_vjp: [n][5] gradient w.r.t. (ln Mc, f0, cos theta, phi, psi).

    ``precision`` "f64" computes every tangent in FP64; "f32" computes spectra, response and tangents in FP32
    (the track, phases and integer decisions stay FP64), for any pixel type.
    """
    L = lib()
    dev = bank.device
    if out is None:
        out = torch.empty((bank.n, 5), dtype=torch.float64, device=dev)
    g = grid.c()
    opt = _options(precision, "wave", block_waves, groups_per_cu, None)
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, ctypes.byref(opt), _lib.WS_VJP)
    ws = _ws(nb, dev)
    pc, bc, sc = pixels.c(), bank.c(), seg.c()
    st = L.tfsc_statistic_vjp(ctypes.byref(g), ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(sc),
                              ctypes.byref(opt), _ptr(seg_zn), _ptr(g_stat), _ptr(g_seg), _ptr(out), _ptr(ws),
                              ws.numel(), _stream())
    _lib.check(st, "tfsc_statistic_vjp")
    return out


def processing_order(grid: GridSpec, bank: BankTensors, out: torch.Tensor | None = None) -> torch.Tensor:
    """tfsc_processing_order: an int32 permutation grouping templates by the frequency bin of f0, then by ln Mc."""
    L = lib()
    dev = bank.device
    if out is None:
        out = torch.empty(max(bank.n, 1), dtype=torch.int32, device=dev)
    g, bc = grid.c(), bank.c()
    nb = L.tfsc_workspace_bytes(ctypes.byref(g), bank.n, None, _lib.WS_ORDER)
    ws = _ws(nb, dev)
    _lib.check(L.tfsc_processing_order(ctypes.byref(g), ctypes.byref(bc), _ptr(out), _ptr(ws), nb, _stream()),
               "tfsc_processing_order")
    return out[: bank.n]


def follow_up_step(grid: GridSpec, bank: BankTensors, seg: SegmentLayout, stat: torch.Tensor,
                   g_params: torch.Tensor, state: torch.Tensor, lr_scale: float, step: int) -> None:
    """tfsc_follow_up_step: one Adam ascent step on bank (in place); state is [n][16] float64."""
    L = lib()
    g, bc, sc = grid.c(), bank.c(), seg.c()
    st = L.tfsc_follow_up_step(ctypes.byref(g), ctypes.byref(bc), ctypes.byref(sc), _ptr(stat), _ptr(g_params),
                               _ptr(state), float(lr_scale), int(step), _stream())
    _lib.check(st, "tfsc_follow_up_step")


def follow_up(grid: GridSpec, pixels: PixelStore, bank: BankTensors, steps: int = 50, lr_scale: float = 0.5,
              nseg_fixed: int = 0, precision: str = "f32", vjp_precision: str = "f64", sort: bool = True):
    """Gradient-ascent follow-up of a candidate set: ``steps`` rounds of statistic, VJP and Adam step.

    ``precision`` is the statistic's arithmetic and ``vjp_precision`` the VJP's.  The segment layout is fixed
    at the candidates' initial parameters.  Returns (initial Upsilon, best Upsilon, best parameters [n][5] =
    (mc, f0, cos theta, phi, psi)), in the order of ``bank``, which is not modified.  ``sort`` works on a copy
    of the candidates in the processing order (f0 bin, then ln Mc), so that the statistic and VJP waves that
    run together read neighbouring pixel rows; every template's arithmetic is its own, so the results are the
    same either way.
    """
    dev = bank.device
    perm = processing_order(grid, bank).long() if sort and bank.n > 1 else None

    def take(t):
        if t is None:
            return None
        return (t[perm] if perm is not None else t).clone()

    work = BankTensors(*(take(getattr(bank, k)) for k in BankTensors.FIELDS), ln_mc=take(bank.ln_mc))
    seg = segment_layout(grid, work, nseg_fixed)
    state = torch.empty((work.n, 16), dtype=torch.float64, device=dev)
    ones = torch.ones(work.n, dtype=torch.float64, device=dev)
    gp = torch.empty((work.n, 5), dtype=torch.float64, device=dev)
    res = None
    first = None
    for step in range(1, steps + 2):
        res = bank_statistic(grid, pixels, work, seg, precision=precision, want_zn=True, out=res)
        if first is None:
            first = res.stat.clone()
        if step == steps + 1:
            follow_up_step(grid, work, seg, res.stat, gp, state, 0.0, step)  # record the last point only
            break
        statistic_vjp(grid, pixels, work, seg, res.seg_zn, g_stat=ones, precision=vjp_precision, out=gp)
        follow_up_step(grid, work, seg, res.stat, gp, state, lr_scale, step)
    best, params = state[:, 10].clone(), state[:, 11:16].clone()
    if perm is not None:
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(perm.numel(), device=dev)
        first, best, params = first[inv], best[inv], params[inv]
    return first, best, params


def tile_max(stat: torch.Tensor, tile: torch.Tensor, n_tiles: int, out: tuple | None = None):
    """tfsc_tile_max: (largest stat per tile [n_tiles] f64, smallest index attaining it [n_tiles] int64, -1 if
    the tile is empty).  ``tile`` is int32 per template (negative = left out)."""
    L = lib()
    if stat.dtype != torch.float64 or tile.dtype != torch.int32 or stat.numel() != tile.numel():
        raise TfscError("tile_max takes float64 stat and int32 tile ids of the same length")
    dev = stat.device
    if out is None:
        out = (torch.empty(n_tiles, dtype=torch.float64, device=dev), torch.empty(n_tiles, dtype=torch.int64, device=dev))
    stat, tile = stat.contiguous(), tile.contiguous()
    _lib.check(L.tfsc_tile_max(_ptr(stat), _ptr(tile), stat.numel(), int(n_tiles), _ptr(out[0]), _ptr(out[1]),
                               _stream()), "tfsc_tile_max")
    return out


def track(grid: GridSpec, bank: BankTensors) -> torch.Tensor:
    """tfsc_track: [n][Nt][4] = (Phi, f, fdot, end code) at every tranche start (FP64)."""
    L = lib()
    out = torch.empty((bank.n, grid.n_tranches, 4), dtype=torch.float64, device=bank.device)
    g, bc = grid.c(), bank.c()
    _lib.check(L.tfsc_track(ctypes.byref(g), ctypes.byref(bc), _ptr(out), _stream()), "tfsc_track")
    return out


class TFSCStatistic(torch.autograd.Function):
    """Upsilon as a differentiable function of (ln Mc, f0, cos theta, phi, psi); the backward is the HIP VJP.

    forward(ctx, ln_mc, f0, cos_theta, phi, psi, fixed) with ``fixed`` a dict holding grid, pixels, eta,
    cos_iota, nseg_fixed, precision (the forward's) and vjp_precision (the backward's, "f64" by default).
    The segment layout is recomputed for the given parameters.
    """

    @staticmethod
    def forward(ctx, ln_mc, f0, cos_theta, phi, psi, fixed):
        grid, pixels = fixed["grid"], fixed["pixels"]
        bank = BankTensors(None, fixed["eta"], f0.contiguous(), cos_theta.contiguous(), phi.contiguous(),
                           psi.contiguous(), fixed["cos_iota"], ln_mc=ln_mc.contiguous())
        seg = segment_layout(grid, bank, fixed.get("nseg_fixed", 0))
        res = bank_statistic(grid, pixels, bank, seg, precision=fixed.get("precision", "f32"), want_zn=True)
        ctx.fixed = fixed
        ctx.bank, ctx.seg, ctx.zn = bank, seg, res.seg_zn
        return res.stat

    @staticmethod
    def backward(ctx, g):
        fixed = ctx.fixed
        gp = statistic_vjp(fixed["grid"], fixed["pixels"], ctx.bank, ctx.seg, ctx.zn,
                           g_stat=g.contiguous().to(torch.float64), precision=fixed.get("vjp_precision", "f64"))
        return gp[:, 0], gp[:, 1], gp[:, 2], gp[:, 3], gp[:, 4], None
