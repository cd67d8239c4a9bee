"""FP64 reference of the serving storage format -- TEST INFRASTRUCTURE ONLY.

Sec. 3.3 trains with SH degree 2 from the start; after the merge, the appendix's vector-tree quantization
evaluates every surfel's contribution, replaces the SH of the least important ones (quantization ratio
0.4) by the nearest row of a learned codebook (8192 rows), and stores the remaining SH and the other
attributes of shape, rotation and opacity in float16.

Readings (parity unpinned beyond the mathematics):
  * the least important surfels are those at or below the floor(ratio (n - 1))-th smallest contribution
    (the rule of the trimming bound, ties included);
  * the codebook is learned by Lloyd's k-means on their SH vectors (squared Euclidean distance), started
    from the rows floor(j m / K) of the m quantized surfels in id order; a codeword left without members
    keeps its value; the nearest codeword is the one of smallest index among equals;
  * the positions stay float32; the codebook is stored in float16 and the final assignment is made
    against the stored (float16) codewords;
  * storage order: the kept surfels in id order, then the quantized ones in id order.

Plain numpy in float64 (float16 conversion by numpy's IEEE round-to-nearest-even).
"""
from __future__ import annotations

import numpy as np

# relative gap between the nearest and the second-nearest codeword below which an FP32 evaluation of
# the distances may choose the other one
FRAGILE = 1e-5


def order_partition(quantize):
    """(order [n] slot -> source id, n_full): the surfels with quantize == 0 in id order, then the rest."""
    q = np.asarray(quantize).astype(bool)
    keep = np.flatnonzero(~q)
    return np.concatenate([keep, np.flatnonzero(q)]).astype(np.int64), int(keep.size)


def vq_init(X, K):
    """Initial codebook [K][D]: rows floor(j m / K) of X [m][D]."""
    X = np.asarray(X, np.float64)
    m = X.shape[0]
    return X[(np.arange(K) * m) // K].copy()


def vq_assign(X, C):
    """Nearest codeword of each row of X [m][D] in C [K][D] by squared Euclidean distance (smallest index
    among equals): (codes [m], best distance, relative gap to the second best)."""
    X = np.asarray(X, np.float64)
    C = np.asarray(C, np.float64)
    m = X.shape[0]
    codes = np.empty(m, np.int64)
    best = np.empty(m)
    gap = np.empty(m)
    for a in range(0, m, 4096):
        x = X[a:a + 4096]
        d = ((x[:, None, :] - C[None, :, :]) ** 2).sum(-1)
        k = np.argmin(d, axis=1)  # first index of the minimum
        codes[a:a + 4096] = k
        b = d[np.arange(x.shape[0]), k]
        best[a:a + 4096] = b
        d[np.arange(x.shape[0]), k] = np.inf
        second = d.min(axis=1) if C.shape[0] > 1 else np.full(x.shape[0], np.inf)
        scale = (x * x).sum(1) + (C * C).sum(1).max() + 1e-30
        gap[a:a + 4096] = (second - b) / scale
    return codes, best, gap


def vq_update(X, codes, C_prev):
    """Lloyd update: each codeword becomes the mean of its members; one without members keeps its value.
    Returns (codebook, counts)."""
    X = np.asarray(X, np.float64)
    K, D = np.asarray(C_prev).shape
    sums = np.zeros((K, D))
    np.add.at(sums, codes, X)
    cnt = np.bincount(codes, minlength=K)
    C = np.asarray(C_prev, np.float64).copy()
    nz = cnt > 0
    C[nz] = sums[nz] / cnt[nz, None]
    return C, cnt


def quantization_error(X, C, codes):
    X = np.asarray(X, np.float64)
    return float(((X - np.asarray(C, np.float64)[codes]) ** 2).sum())


def kmeans(X, K, iters):
    """Lloyd's iterations from vq_init; returns (codebook, codes, errors per iteration)."""
    C = vq_init(X, K)
    errs = []
    for _ in range(iters):
        codes, _, _ = vq_assign(X, C)
        errs.append(quantization_error(X, C, codes))
        C, _ = vq_update(X, codes, C)
    codes, _, _ = vq_assign(X, C)
    errs.append(quantization_error(X, C, codes))
    return C, codes, errs


def pack(P, order, n_full, codes, codebook):
    """The stored arrays of a set P (planar; sh [K][3][n]) in the order `order`; codes [n - n_full] are
    the codebook rows of slots n_full.. ; codebook [cb][3K] float64 -> float16.  Returns a dict with
    mean float32 [3][n], log_scale / quat / opacity_logit float16, sh float16 [n_full][K][3], code,
    codebook float16 [cb][K][3]."""
    o = np.asarray(order)
    Kc = np.asarray(P["sh"]).shape[0]
    sh = np.asarray(P["sh"], np.float32)[:, :, o[:n_full]].transpose(2, 0, 1)
    return dict(mean=np.asarray(P["mean"], np.float32)[:, o],
                log_scale=np.asarray(P["log_scale"], np.float32)[:, o].astype(np.float16),
                quat=np.asarray(P["quat"], np.float32)[:, o].astype(np.float16),
                opacity_logit=np.asarray(P["opacity_logit"], np.float32)[o].astype(np.float16),
                sh=np.ascontiguousarray(sh).astype(np.float16), code=np.asarray(codes, np.int64),
                codebook=np.asarray(codebook, np.float64).astype(np.float32).astype(np.float16).reshape(-1, Kc, 3),
                n_full=int(n_full), sh_degree=int(round(np.sqrt(Kc))) - 1)


def decode(c):
    """Float32 planar parameters (sh [K][3][n]) of a packed set: what the projection sees."""
    n = c["mean"].shape[1]
    Kc = c["codebook"].shape[1] if c["codebook"].size else c["sh"].shape[1]
    sh = np.empty((n, Kc, 3), np.float32)
    sh[:c["n_full"]] = c["sh"].astype(np.float32)
    if n > c["n_full"]:
        sh[c["n_full"]:] = c["codebook"][c["code"]].astype(np.float32)
    return dict(mean=c["mean"].astype(np.float32), log_scale=c["log_scale"].astype(np.float32),
                quat=c["quat"].astype(np.float32), opacity_logit=c["opacity_logit"].astype(np.float32),
                sh=np.ascontiguousarray(sh.transpose(1, 2, 0)), sh_degree=c["sh_degree"])
