"""Contribution-based trimming (Sec. 3.3, Eq. 3/4 and the percentile bound) against the oracle.

Per-surfel contributions: where the oracle finds no fragile pixel among those a surfel is evaluated at
(a pixel whose decisions fall inside the FP32 error bound), pixel counts |P| exactly and C within the
oracle's first-order FP32 error bound of the terms alpha^gamma T^(1-gamma) plus 1e-5 relative and the
rounding bound of their FP32 sum (one wave reduction and one atomic add per tile or quadrant block, in
arbitrary order); with fp such pixels, the count
within fp and the sum within fp terms (each term is at most 1).  Whatever the bound, no surfel's C may be
off by more than 1e-3 relative.  The trimming bound and mask are
checked bit for bit against the oracle on the oracle's averages over views (rounded to FP32), and the
bound of the whole GPU chain against the oracle's within the averages' tolerance."""
import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes
from tests.helpers import FRAGILE, gpu_forward

pytestmark = pytest.mark.gpu

# each term alpha^gamma T^(1-gamma) carries the FP32 error of alpha and of the accumulated T: the oracle
# bounds it per surfel (ref["err"], the error model behind the fragility margins); 1e-5 relative on top
C_REL = 1e-5
C_CAP = 1e-3  # largest relative error allowed for any surfel's C, whatever its error bound
U32 = 2.0 ** -24


def _sum_tol(po, ref):
    """Absolute bound of the GPU's FP32 sum of a surfel's terms: the terms' own error (ref["err"]) plus
    the rounding of their summation (one wave reduction per tile or quadrant block, one atomic add of
    each partial: at most min(|P|, 4 x rect tiles) of them) and C_REL."""
    r = po["tile_rect"].astype(np.int64)
    tiles = np.maximum(r[:, 2] - r[:, 0], 0) * np.maximum(r[:, 3] - r[:, 1], 0)
    return ref["err"] + (C_REL + U32 * (np.minimum(ref["cnt"], 4 * tiles) + 8)) * ref["sum"]


def _gpu_contrib(eng, cs, gamma):
    import torch
    V, n = eng.V, eng.n
    cv = torch.empty((V, n), device="cuda")
    px = torch.empty((V, n), dtype=torch.int32, device="cuda")
    cs_sum = torch.zeros(n, device="cuda")
    eng.contribution(cs, gamma, c_view=cv, c_sum=cs_sum, pixels=px)
    torch.cuda.synchronize()
    return cv.cpu().numpy().astype(np.float64), px.cpu().numpy().view(np.uint32).astype(np.int64), cs_sum


def _check_view(sc, cam, c_gpu, px_gpu, flags_gpu, gamma, min_exact):
    po, off, ids, _ = oracle.forward_view(sc, cam)
    ref = oracle.contribution(po, cam, off, ids, gamma, FRAGILE)
    both = ((po["flags"] & 1) > 0) & ((flags_gpu & 1) > 0)
    fp = ref["fragile"].astype(np.int64)
    ok = both & (fp == 0)
    assert ok.sum() >= min_exact * max(both.sum(), 1), (ok.sum(), both.sum())
    # surfels evaluated at fragile pixels: count within fp, sum within fp terms
    fr = both & (fp > 0)
    assert np.all(np.abs(px_gpu[fr] - ref["cnt"][fr]) <= fp[fr])
    tol = _sum_tol(po, ref)
    s_gpu = c_gpu[fr] * px_gpu[fr]
    assert np.all(np.abs(s_gpu - ref["sum"][fr]) <= fp[fr] + tol[fr])
    assert np.array_equal(px_gpu[ok], ref["cnt"][ok])
    err = np.abs(c_gpu[ok] - ref["C"][ok])
    # C = sum / |P|; the GPU's division and float32 result add two roundings
    bound = tol[ok] / np.maximum(ref["cnt"][ok], 1) + 2 * U32 * ref["C"][ok] + 1e-12
    # the error model's bound, capped at C_CAP relative: a surfel whose FP32 error exceeded the cap fails
    # here even where the model (ill-conditioned fragments) would allow more
    rel_bound = bound / np.maximum(ref["C"][ok], 1e-30)
    seen = ref["C"][ok] > 0
    print(f"[trim] bound / C: max {float(rel_bound[seen].max(initial=0)):.2e}, "
          f"{int((rel_bound[seen] > C_CAP).sum())} of {int(seen.sum())} surfels above the {C_CAP:g} cap", flush=True)
    bound = np.minimum(bound, C_CAP * ref["C"][ok] + 1e-12)
    bad = err > bound
    if bad.any():
        k = np.flatnonzero(ok)[bad]
        print("[trim] outside the bound:", [(int(i), float(ref["C"][i]), float(c_gpu[i]), int(ref["cnt"][i]),
                                             float(ref["err"][i])) for i in k[:8]], flush=True)
    assert not bad.any(), float((err / bound).max())
    print(f"[trim] C: {int(ok.sum())} surfels, worst error / bound {float((err / bound).max()):.3f}, "
          f"median bound / C {float(np.median(bound[ref['C'][ok] > 0] / ref['C'][ok][ref['C'][ok] > 0])):.2e}", flush=True)
    # surfels the oracle never blends have C = 0 on both sides
    unseen = ok & (ref["cnt"] == 0)
    assert np.all(c_gpu[unseen] == 0)
    return ref


@pytest.mark.parametrize("gamma", [0.5, 0.25])
def test_contribution_tiny(cuda, gamma):
    w = scenes.workload(0)
    sc, cam = w["scene"], w["cameras"][0]
    eng, params, cs = gpu_forward(sc, [cam], capacity=1 << 16)
    cv, px, _ = _gpu_contrib(eng, cs, gamma)
    flags = eng.flags.view(1, sc.n)[0].cpu().numpy().astype(np.int32)
    ref = _check_view(sc, cam, cv[0], px[0], flags, gamma, 0.8)
    assert ref["cnt"].sum() > 10000


def test_contribution_aerial_views_average_and_trim(cuda):
    import torch
    from paper_2411_00771_amd import raster
    w = scenes.workload(1)
    sc = w["scene"]
    cams = [w["cameras"][k] for k in (0, 3, 7, 11)]
    eng, params, cs = gpu_forward(sc, cams, capacity=12_000_000)
    assert eng.status.item() == 0
    cv, px, c_sum = _gpu_contrib(eng, cs, 0.5)
    flags = eng.flags.view(len(cams), sc.n).cpu().numpy().astype(np.int32)
    per_view = []
    for k, cam in enumerate(cams):
        ref = _check_view(sc, cam, cv[k], px[k], flags[k], 0.5, 0.0)
        per_view.append(ref["C"])
    # Eq. 4 over the four views: the GPU's running sum / 4 against the oracle's mean
    avg_ref = oracle.average_contribution(per_view)
    avg = c_sum.cpu().numpy().astype(np.float64) / len(cams)
    rel = np.abs(avg - avg_ref) / np.maximum(avg_ref, 1e-6)
    assert np.mean(rel > 1e-4) < 1e-3
    # trimming at the paper's ratio on the oracle's averages rounded to FP32, given to both sides: bit-exact
    a32 = avg_ref.astype(np.float32)
    bound, mask, removed = raster.trim_mask(torch.from_numpy(a32).cuda(), 0.025)
    torch.cuda.synchronize()
    b_ref, m_ref = oracle.trim_threshold(a32, 0.025)
    assert np.float32(bound.item()) == np.float32(b_ref)
    assert np.array_equal(mask.cpu().numpy().astype(bool), m_ref)
    assert removed.item() == int(m_ref.sum())
    # the whole GPU chain (contributions, average, bound) against the oracle's bound up to the comparison
    # tolerance of the averages
    c_avg = (c_sum / len(cams)).contiguous()
    b_gpu, _, _ = raster.trim_mask(c_avg, 0.025)
    assert abs(b_gpu.item() - b_ref) <= 1e-4 * max(b_ref, 1e-6)


@pytest.mark.parametrize("case", ["ties", "zeros", "one", "ratio0", "ratio1", "random"])
def test_trim_edge_cases(cuda, case):
    import torch
    from paper_2411_00771_amd import raster
    rng = np.random.default_rng(5)
    arrays = {
        "ties": (np.array([0.3, 0.0, 0.1, 0.0, 0.5, 0.2, 0.4, 0.1, 0.6, 0.05], np.float32), 0.4),
        "zeros": (np.zeros(1000, np.float32), 0.025),
        "one": (np.array([0.7], np.float32), 0.5),
        "ratio0": (rng.uniform(0, 1, 5000).astype(np.float32), 0.0),
        "ratio1": (rng.uniform(0, 1, 5000).astype(np.float32), 1.0),
        "random": (np.where(rng.uniform(size=300_001) < 0.3, 0, rng.lognormal(-3, 2, 300_001)).astype(np.float32), 0.1),
    }
    c, ratio = arrays[case]
    bound, mask, removed = raster.trim_mask(torch.from_numpy(c).cuda(), ratio)
    torch.cuda.synchronize()
    b_ref, m_ref = oracle.trim_threshold(c, ratio)
    assert np.float32(bound.item()) == np.float32(b_ref)
    assert np.array_equal(mask.cpu().numpy().astype(bool), m_ref)
    assert removed.item() == int(m_ref.sum())
