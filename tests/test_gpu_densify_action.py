"""Densification action (Sec. 3.2 candidates, Sec. 3.3 removal, the clone / split rule of the 3DGS / 2DGS
family) on the GPU against the oracle.

Actions, slots, counts and the slot -> source map are integer work: bit-exact.  Survivors and clone
copies, and every copied field of a child (rotation, opacity, SH), are bit-exact copies.  A child's mean
and log-scales are evaluated in FP64 on both sides and rounded once to float32 on the GPU: within one
float32 ulp of the oracle's FP64 value rounded to float32."""
import math

import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes

pytestmark = pytest.mark.gpu

SHRINK = float(np.float32(1.6))


def _scene(n, seed, deg=3, low_opacity=0.01):
    sc = scenes.tiny_scene(seed, n, sh_degree=deg)
    rng = np.random.default_rng(seed + 7)
    # a share of surfels below the minimum opacity, so the opacity removal is exercised
    low = rng.random(n) < low_opacity
    sc.opacity_logit[low] = np.float32(-7.0)
    return sc


def _oracle_params(sc):
    return dict(mean=sc.mean.astype(np.float64), log_scale=sc.log_scale.astype(np.float64),
                quat=sc.quat.astype(np.float64), opacity_logit=sc.opacity_logit.astype(np.float64),
                sh=sc.sh.astype(np.float64), sh_degree=sc.sh_degree)


def _run(sc, mask, remove, z, dense_scale, min_opacity, n_out=None):
    import torch
    from paper_2411_00771_amd import raster
    params = raster.Params.from_scene(sc)
    m = torch.from_numpy(mask).cuda()
    r = None if remove is None else torch.from_numpy(remove).cuda()
    plan = raster.densify_plan(params, m, r, dense_scale=dense_scale, min_opacity=min_opacity)
    zt = torch.from_numpy(np.ascontiguousarray(z, np.float32)).cuda()
    out, src = raster.densify_apply(params, plan, zt, split_shrink=SHRINK, n_out=n_out)
    torch.cuda.synchronize()
    return params, plan, out, src


def _within_ulp(gpu, ref64):
    ref32 = ref64.astype(np.float32)
    return np.all(np.abs(gpu.astype(np.float64) - ref32.astype(np.float64)) <=
                  np.spacing(np.abs(ref32)).astype(np.float64))


def _check(sc, mask, remove, z, dense_scale, min_opacity):
    n = sc.mean.shape[1]
    print(f"[densify_action] n={n} deg={sc.sh_degree} dense={dense_scale} min_op={min_opacity}", flush=True)
    params, plan, out, src = _run(sc, mask, remove, z, dense_scale, min_opacity)
    from paper_2411_00771_amd import raster
    act_ref = oracle.densify_actions((mask & 4) > 0, None if remove is None else remove > 0, sc.log_scale,
                                     sc.opacity_logit, float(np.float32(dense_scale)),
                                     float(np.float32(min_opacity)))
    act = plan.actions.cpu().numpy().astype(np.int32)
    assert np.array_equal(act, act_ref)
    dst_ref, src_ref, kind_ref = oracle.densify_slots(act_ref)
    dst = plan.dst.cpu().numpy().view(np.uint32).astype(np.int64)
    dst[dst == 0xffffffff] = -1
    assert np.array_equal(dst, dst_ref)
    counts = plan.counts.cpu().numpy()
    assert list(counts[:4]) == [int((act_ref == k).sum()) for k in range(4)]
    assert counts[4] == len(src_ref)
    s = src.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(s >> 2, src_ref) and np.array_equal(s & 3, kind_ref)

    ref = oracle.densify_apply(_oracle_params(sc), act_ref, z.astype(np.float64), shrink=SHRINK)
    got = dict(mean=out.mean.cpu().numpy(), log_scale=out.log_scale.cpu().numpy(), quat=out.quat.cpu().numpy(),
               opacity_logit=out.opacity_logit.cpu().numpy(), sh=raster.Params.sh_planar(out.sh))
    for k in ("quat", "opacity_logit", "sh"):
        assert np.array_equal(got[k].astype(np.float64), ref[k]), k
    child = kind_ref >= 2
    for k in ("mean", "log_scale"):
        assert np.array_equal(got[k][:, ~child].astype(np.float64), ref[k][:, ~child]), k
        assert _within_ulp(got[k][:, child], ref[k][:, child]), k
    return act_ref, counts, out, src, plan, params


def _dense_scale(sc, q=0.5):
    return float(np.float32(np.quantile(np.exp(sc.log_scale.astype(np.float64)).max(0), q)))


def test_action_tiny_all_kinds(cuda):
    sc = _scene(4096, 0)
    mask, remove, z = scenes.densify_inputs(11, 4096, cand_frac=0.4, remove_frac=0.05)
    act, counts, *_ = _check(sc, mask, remove, z, _dense_scale(sc), 0.005)
    assert all(counts[k] > 0 for k in range(4))
    # removal wins over a candidate
    assert np.all(act[(remove > 0) & ((mask & 4) > 0)] == 3)


@pytest.mark.parametrize("n", [1, 7, 2047, 2048, 2049, 6151])
def test_action_ragged_sizes(cuda, n):
    sc = _scene(n, n, low_opacity=0.05)
    mask, remove, z = scenes.densify_inputs(100 + n, n, cand_frac=0.5, remove_frac=0.1)
    _check(sc, mask, remove, z, _dense_scale(sc), 0.005)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_action_sh_degrees(cuda, deg):
    sc = _scene(3000, 3 + deg, deg=deg)
    mask, remove, z = scenes.densify_inputs(200 + deg, 3000, cand_frac=0.3)
    _check(sc, mask, remove, z, _dense_scale(sc), 0.005)


def test_action_degenerate_cases(cuda):
    n = 5000
    sc = _scene(n, 9, low_opacity=0.0)
    mask, remove, z = scenes.densify_inputs(9, n)
    # nothing to do: all keep, the output equals the input
    act, counts, out, *_ = _check(sc, np.zeros(n, np.uint8), None, z, 0.01, 0.0)
    assert counts[4] == n and np.array_equal(out.mean.cpu().numpy(), sc.mean)
    # every surfel removed: an empty output
    act, counts, out, *_ = _check(sc, mask, np.ones(n, np.uint8), z, 0.01, 0.0)
    assert counts[4] == 0 and out.mean.shape[1] == 0
    # every surfel a candidate: all clones (dense scale above every scale), then all splits (below)
    _, counts, *_ = _check(sc, np.full(n, 4, np.uint8), None, z, 1e3, 0.0)
    assert counts[1] == n and counts[4] == 2 * n
    _, counts, *_ = _check(sc, np.full(n, 4, np.uint8), None, z, 0.0, 0.0)
    assert counts[2] == n and counts[4] == 2 * n


def test_gather_fields_and_fresh_moments(cuda):
    import torch
    from paper_2411_00771_amd import raster
    n = 4099
    sc = _scene(n, 21)
    mask, remove, z = scenes.densify_inputs(21, n, cand_frac=0.3)
    act, counts, out, src, plan, params = _check(sc, mask, remove, z, _dense_scale(sc), 0.005)
    _, src_ref, kind_ref = oracle.densify_slots(act)
    n_out = len(src_ref)
    rng = np.random.default_rng(5)
    planar = rng.standard_normal((3, n)).astype(np.float32)
    blocked = rng.standard_normal((n, 16, 3)).astype(np.float32)
    for f, blk in ((planar, False), (blocked, True), (planar[0].copy(), False)):
        ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
        for zero_new in (False, True):
            g = raster.densify_gather(ft, src, plan, n_out, blocked=blk, zero_new=zero_new).cpu().numpy()
            want = f[src_ref] if blk else f[..., src_ref]
            if zero_new:
                if blk:
                    want = want * (kind_ref == 0)[:, None, None]
                else:
                    want = want * (kind_ref == 0)
            assert np.array_equal(g, want.astype(np.float32)), (blk, zero_new)


def test_apply_with_short_output_stays_in_bounds(cuda):
    """An output smaller than the plan's count receives its first slots and nothing beyond."""
    n = 3000
    sc = _scene(n, 31)
    mask, remove, z = scenes.densify_inputs(31, n, cand_frac=0.5)
    ds = _dense_scale(sc)
    _, plan, full, _ = _run(sc, mask, remove, z, ds, 0.005)
    short = plan.n_out() - 777
    _, _, part, src = _run(sc, mask, remove, z, ds, 0.005, n_out=short)
    assert np.array_equal(part.mean.cpu().numpy(), full.mean.cpu().numpy()[:, :short])
    assert np.array_equal(part.sh.cpu().numpy(), full.sh.cpu().numpy()[:short])


def test_action_aerial_full_size(cuda):
    """The aerial 1 M-surfel set with the trimming share of removals and a few % candidates."""
    w = scenes.workload(1)
    sc = w["scene"]
    n = sc.mean.shape[1]
    mask, remove, z = scenes.densify_inputs(1001, n, cand_frac=0.05, remove_frac=0.025)
    act, counts, *_ = _check(sc, mask, remove, z, _dense_scale(sc, 0.5), 0.005)
    assert counts[4] > n * 1.0 and math.isclose(counts[1] + counts[2], ((mask & 4) > 0).sum() -
                                                ((act == 3) & ((mask & 4) > 0)).sum())
