"""Serving storage of a trained surfel set (CityGaussianV2 Sec. 3.3 and the appendix's vector-tree
quantization): SH of degree 2, the least important surfels' SH replaced by the nearest row of a k-means
codebook (8192 rows, ratio 0.4), everything else but the positions in float16.  Every step runs in
libcgv2r's kernels; ``Engine.project`` (and so ``Engine.forward`` and the ``Server``) accepts a
``CompactParams`` wherever it takes ``Params``.

    c_avg = ...  # Eq. 4 average contribution per surfel (Engine.contribution over the training views)
    cp, info = compress(params, c_avg, ratio=0.4, codebook_size=8192, iters=10)
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, ptr
from .raster import Params, _stream, trim_mask


class CompactParams:
    """Device arrays of cgv2_surfels_compact: mean float32 [3][n]; log_scale [2][n], quat [4][n],
    opacity_logit [n] float16; sh float16 [n_full][K][3]; code int16-stored u16 [n - n_full]; codebook
    float16 [cb][K][3].  Slot order: kept surfels, then quantized ones (``order`` maps slot -> source)."""

    is_compact = True

    def __init__(self, mean, log_scale, quat, opacity_logit, sh, code, codebook, n_full: int, sh_degree: int,
                 order=None):
        self.mean, self.log_scale, self.quat, self.opacity_logit = mean, log_scale, quat, opacity_logit
        self.sh, self.code, self.codebook = sh, code, codebook
        self.n_full, self.sh_degree, self.order = int(n_full), int(sh_degree), order

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.mean, self.log_scale, self.quat, self.opacity_logit,
                                                           self.sh, self.code, self.codebook))

    def struct(self) -> _lib.SurfelsCompact:
        s = _lib.SurfelsCompact()
        s.n, s.n_full, s.sh_degree = self.n, self.n_full, self.sh_degree
        s.codebook_size = int(self.codebook.shape[0])
        s.mean, s.log_scale, s.quat = ptr(self.mean), ptr(self.log_scale), ptr(self.quat)
        s.opacity_logit, s.sh, s.code, s.codebook = ptr(self.opacity_logit), ptr(self.sh), ptr(self.code), \
            ptr(self.codebook)
        return s


def compact_order(quantize):
    """(order [n] int32-stored u32, n_full device int64 [1]) of the stable partition by quantize [n]."""
    L = _lib.lib()
    n = quantize.numel()
    order = torch.empty(max(n, 1), dtype=torch.int32, device=quantize.device)
    n_full = torch.empty(1, dtype=torch.int64, device=quantize.device)
    ws = torch.empty(max(L.cgv2_compact_order_workspace(n), 256), dtype=torch.uint8, device=quantize.device)
    check(L.cgv2_compact_order(ptr(quantize), n, ptr(order), ptr(n_full), ptr(ws), ws.numel(), _stream()),
          "cgv2_compact_order")
    return order[:n], n_full


def vq_init(x, D: int, rows, K: int):
    L = _lib.lib()
    cb = torch.empty((K, D), dtype=torch.float32, device=x.device)
    check(L.cgv2_vq_init(ptr(x), D, ptr(rows), rows.numel(), K, ptr(cb), _stream()), "cgv2_vq_init")
    return cb


def vq_assign(x, D: int, rows, codebook, half_codebook: bool = False, code=None):
    """Nearest-codeword index (int16-stored u16) of each selected D-vector."""
    L = _lib.lib()
    m = rows.numel()
    K = codebook.shape[0]
    if code is None:
        code = torch.empty(max(m, 1), dtype=torch.int16, device=x.device)[:m]
    ws = torch.empty(max(L.cgv2_vq_assign_workspace(K), 256), dtype=torch.uint8, device=x.device)
    check(L.cgv2_vq_assign(ptr(x), D, ptr(rows), m, ptr(codebook), K, 1 if half_codebook else 0, ptr(code), ptr(ws),
                           ws.numel(), _stream()), "cgv2_vq_assign")
    return code


def vq_update(x, D: int, rows, code, codebook, counts=None, ws=None):
    """Lloyd update of codebook [K][D] in place; returns the member counts."""
    L = _lib.lib()
    K = codebook.shape[0]
    if counts is None:
        counts = torch.empty(K, dtype=torch.int32, device=x.device)
    need = max(L.cgv2_vq_update_workspace(K, D), 256)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    check(L.cgv2_vq_update(ptr(x), D, ptr(rows), rows.numel(), ptr(code), K, ptr(codebook), ptr(counts), ptr(ws),
                           ws.numel(), _stream()), "cgv2_vq_update")
    return counts


def compact_write(params: Params, order, n_full, codebook: Optional[torch.Tensor], n_full_host: int, code):
    """CompactParams of params in the partition order; code are the quantized slots' codebook rows."""
    L = _lib.lib()
    n, dev = params.n, params.mean.device
    Kc = (params.sh_degree + 1) ** 2
    K = 0 if codebook is None else int(codebook.shape[0])
    h = lambda *shape: torch.empty(shape, dtype=torch.float16, device=dev)
    mean = torch.empty((3, n), dtype=torch.float32, device=dev)
    ls, qt, op, sh = h(2, n), h(4, n), h(n), h(max(n, 1), Kc, 3)
    cbh = h(max(K, 1), Kc, 3)
    o = _lib.CompactOut()
    o.n, o.sh_degree = n, params.sh_degree
    o.mean, o.log_scale, o.quat, o.opacity_logit, o.sh = ptr(mean), ptr(ls), ptr(qt), ptr(op), ptr(sh)
    o.codebook = ptr(cbh) if K else None
    s = params.struct()
    check(L.cgv2_compact_write(ctypes.byref(s), ptr(order), ptr(n_full), ptr(codebook) if K else None, K,
                               ctypes.byref(o), _stream()), "cgv2_compact_write")
    if K == 0:
        cbh = h(1, Kc, 3).zero_()
    return CompactParams(mean, ls, qt, op, sh[:n_full_host], code, cbh[:max(K, 1)], n_full_host, params.sh_degree,
                         order)


def compress(params: Params, contribution, ratio: float = 0.4, codebook_size: int = 8192, iters: int = 10):
    """The serving storage of params: surfels at or below the ratio-percentile contribution get a codeword
    (k-means, ``iters`` Lloyd iterations from rows floor(j m / K); the final assignment is against the
    stored float16 codewords).  Returns (CompactParams, info)."""
    n = params.n
    D = 3 * (params.sh_degree + 1) ** 2
    _, qmask, _ = trim_mask(contribution, ratio)
    order, n_full_d = compact_order(qmask)
    n_full = int(n_full_d.item())
    rows = order[n_full:]
    m = rows.numel()
    x = params.sh.reshape(n, D) if n else params.sh
    if m == 0:
        cp = compact_write(params, order, n_full_d, None, n_full, torch.zeros(1, dtype=torch.int16, device=x.device)[:0])
        return cp, dict(quantized=0, codebook_size=0)
    K = min(codebook_size, m)
    cb = vq_init(x, D, rows, K)
    code = torch.empty(m, dtype=torch.int16, device=x.device)
    counts = None
    ws = None
    for _ in range(iters):
        vq_assign(x, D, rows, cb, code=code)
        counts = vq_update(x, D, rows, code, cb, counts=counts, ws=ws)
    vq_assign(x, D, rows, cb, half_codebook=True, code=code)
    cp = compact_write(params, order, n_full_d, cb, n_full, code)
    return cp, dict(quantized=m, codebook_size=K, iters=iters, codebook=cb)
