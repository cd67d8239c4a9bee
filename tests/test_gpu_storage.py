"""Serving storage (Sec. 3.3 SH degree 2, the appendix's vector-tree quantization and float16 storage) on
the GPU against the oracle.

Integer work (the partition, codes, counts) is bit-exact; a code may differ only where the oracle's
nearest and second-nearest codewords are within its FP32 tie margin (relative gap below 1e-5), and
then the GPU's pick must be within that margin of the best.  float16 arrays are bit-exact (both sides
round to nearest, ties to even).  Lloyd means are FP64 sums rounded once: within one float32 ulp.  A
compact set projects to exactly the records of its decoded float32 copy."""
import numpy as np
import pytest

from oracle import compact as oc
from paper_2411_00771_amd import scenes

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 2049, 100003])
def test_partition(cuda, n):
    from paper_2411_00771_amd import storage
    q = (np.random.default_rng(n).random(n) < 0.4).astype(np.uint8)
    order, nf = storage.compact_order(_t(q))
    ref, rnf = oc.order_partition(q)
    assert int(nf.item()) == rnf
    assert np.array_equal(order.cpu().numpy().view(np.uint32).astype(np.int64), ref)


def _check_codes(code_gpu, X, C, label):
    codes, best, gap = oc.vq_assign(X, C)
    g = code_gpu.cpu().numpy().view(np.uint16).astype(np.int64)
    ok = gap >= oc.FRAGILE
    print(f"[storage] {label}: m={len(g)} K={len(C)} fragile={int((~ok).sum())}", flush=True)
    assert np.array_equal(g[ok], codes[ok])
    # near-ties: the GPU's pick is within the margin of the best
    if (~ok).any():
        Xf, Cf = X[~ok].astype(np.float64), C[g[~ok]].astype(np.float64)
        d = ((Xf - Cf) ** 2).sum(1)
        scale = (Xf * Xf).sum(1) + (C.astype(np.float64) ** 2).sum(1).max()
        assert np.all(d - best[~ok] <= oc.FRAGILE * scale)
    return codes


@pytest.mark.parametrize("D,K", [(27, 8192), (27, 1), (48, 300), (12, 129), (3, 64)])
def test_vq_assign_and_init(cuda, D, K):
    from paper_2411_00771_amd import storage
    rng = np.random.default_rng(D * 1000 + K)
    N = 6000
    x = rng.normal(0, 0.3, (N, D)).astype(np.float32)
    rows = np.sort(rng.choice(N, 4097, replace=False)).astype(np.uint32)
    xt, rt = _t(x), _t(rows.view(np.int32))
    K = min(K, len(rows))
    cb = storage.vq_init(xt, D, rt, K)
    C0 = oc.vq_init(x[rows], K)
    assert np.array_equal(cb.cpu().numpy().astype(np.float64), C0)
    # the assignment on the oracle's codebook, given to both sides
    cbo = _t(C0.astype(np.float32))
    code = storage.vq_assign(xt, D, rt, cbo)
    _check_codes(code, x[rows].astype(np.float64), C0, f"D={D}")
    # against the float16 rounding of the codewords
    code = storage.vq_assign(xt, D, rt, cbo, half_codebook=True)
    ch = C0.astype(np.float32).astype(np.float16).astype(np.float64)
    _check_codes(code, x[rows].astype(np.float64), ch, f"D={D} half")


def test_vq_update(cuda):
    from paper_2411_00771_amd import storage
    rng = np.random.default_rng(3)
    D, K, N = 27, 500, 20000
    x = rng.normal(0, 1, (N, D)).astype(np.float32)
    rows = np.arange(0, N, 2).astype(np.uint32)
    code = rng.integers(0, K - 7, rows.size).astype(np.uint16)  # the last 7 codewords stay empty
    C0 = rng.normal(0, 1, (K, D)).astype(np.float32)
    cb = _t(C0)
    counts = storage.vq_update(_t(x), D, _t(rows.view(np.int32)), _t(code.view(np.int16)), cb)
    C1, cnt = oc.vq_update(x[rows], code.astype(np.int64), C0)
    assert np.array_equal(counts.cpu().numpy().astype(np.int64), cnt)
    got = cb.cpu().numpy()
    ref32 = C1.astype(np.float32)
    assert np.all(np.abs(got.astype(np.float64) - ref32) <= np.spacing(np.abs(ref32)).astype(np.float64))
    assert np.array_equal(got[-7:], C0[-7:])


def _scene2(n, seed):
    return scenes.tiny_scene(seed, n, sh_degree=2)


def test_compact_write_and_projection(cuda):
    import torch
    from paper_2411_00771_amd import raster, storage
    sc = _scene2(5000, 21)
    cam = scenes.tiny_camera()
    params = raster.Params.from_scene(sc)
    q = (np.arange(5000) % 5 < 2).astype(np.uint8)
    order, nfd = storage.compact_order(_t(q))
    nf = int(nfd.item())
    # a synthetic codebook and codes (within it), given to both sides
    rng = np.random.default_rng(21)
    C = rng.normal(0, 0.5, (256, 27)).astype(np.float32)
    codes = rng.integers(0, 256, 5000 - nf).astype(np.uint16)
    cp = storage.compact_write(params, order, nfd, _t(C), nf, _t(codes.view(np.int16)))
    torch.cuda.synchronize()
    # stored arrays against the oracle's packing
    P = dict(mean=sc.mean, log_scale=sc.log_scale, quat=sc.quat, opacity_logit=sc.opacity_logit, sh=sc.sh,
             sh_degree=2)
    o, rnf = oc.order_partition(q)
    assert rnf == nf
    ref = oc.pack(P, o, nf, codes.astype(np.int64), C.astype(np.float64))
    h = lambda t: t.cpu().numpy().view(np.uint16)
    assert np.array_equal(cp.mean.cpu().numpy(), ref["mean"])
    for k in ("log_scale", "quat", "opacity_logit", "sh", "codebook"):
        assert np.array_equal(h(getattr(cp, k)), ref[k].view(np.uint16)), k
    # the compact set projects exactly like its decoded float32 copy
    dec = oc.decode(ref)
    full = raster.Params(*(_t(a.astype(np.float32)) for a in (dec["mean"], dec["log_scale"], dec["quat"],
                                                               dec["opacity_logit"])),
                         _t(np.ascontiguousarray(dec["sh"].transpose(2, 0, 1)).astype(np.float32)), 2)
    e1 = raster.Engine(5000, cam.width, cam.height, 1, capacity=1 << 17)
    e2 = raster.Engine(5000, cam.width, cam.height, 1, capacity=1 << 17)
    c1, c2 = e1.cams([cam]), e2.cams([cam])
    e1.forward(cp, c1)
    e2.forward(full, c2)
    torch.cuda.synchronize()
    assert np.array_equal(e1.flags.cpu().numpy(), e2.flags.cpu().numpy())
    vis = (e1.flags.cpu().numpy() & 1) > 0
    r1 = e1.rec.cpu().numpy().reshape(-1, 24)[vis.reshape(-1)]
    r2 = e2.rec.cpu().numpy().reshape(-1, 24)[vis.reshape(-1)]
    assert vis.sum() > 1000 and np.array_equal(r1.view(np.uint32), r2.view(np.uint32))
    assert np.array_equal(e1.rgb.cpu().numpy(), e2.rgb.cpu().numpy())


def test_invalid_code_is_culled(cuda):
    import torch
    from paper_2411_00771_amd import raster, storage
    sc = _scene2(300, 5)
    cam = scenes.tiny_camera()
    params = raster.Params.from_scene(sc)
    q = np.zeros(300, np.uint8)
    q[150:] = 1
    order, nfd = storage.compact_order(_t(q))
    cb = torch.zeros((4, 27), device="cuda")
    code = torch.full((150,), 9, dtype=torch.int16, device="cuda")  # rows beyond the 4-row codebook
    cp = storage.compact_write(params, order, nfd, cb, 150, code)
    e = raster.Engine(300, cam.width, cam.height, 1, capacity=1 << 15)
    e.project(cp, e.cams([cam]))
    torch.cuda.synchronize()
    fl = e.flags.cpu().numpy().reshape(-1)
    assert np.all(fl[150:] == 16) and not np.any(fl[:150] & 16)


def test_compress_pipeline_on_clustered_sh(cuda):
    """The whole pipeline (partition, init, Lloyd iterations, final float16 assignment, packing) against
    the oracle's, on SH vectors drawn around well-separated centres so that no assignment is near a tie."""
    import torch
    from paper_2411_00771_amd import raster, storage
    rng = np.random.default_rng(8)
    n, K = 20000, 64
    sc = _scene2(n, 8)
    centres = rng.uniform(-1, 1, (K, 27))
    # the quantized surfels are the ids i % 5 < 2 (their contributions are the 40 % smallest); in their
    # storage order p, cluster = p K / m in contiguous runs, so the codebook start (rows floor(j m / K))
    # takes one row of every cluster and no assignment comes near a tie
    qid = np.flatnonzero(np.arange(n) % 5 < 2)
    lab = rng.integers(0, K, n)
    lab[qid] = (np.arange(qid.size) * K) // qid.size
    sh = (centres[lab] + rng.normal(0, 0.01, (n, 27))).astype(np.float32)
    sc.sh = np.ascontiguousarray(sh.reshape(n, 9, 3).transpose(1, 2, 0))
    params = raster.Params.from_scene(sc)
    contrib = (rng.random(n) * 0.5 + np.where(np.arange(n) % 5 < 2, 0.0, 0.5)).astype(np.float32)
    cp, info = storage.compress(params, _t(contrib), ratio=0.4, codebook_size=K, iters=4)
    torch.cuda.synchronize()
    bound = np.sort(contrib.astype(np.float64))[int(np.floor(0.4 * (n - 1)))]
    q = (contrib <= bound).astype(np.uint8)
    o, nf = oc.order_partition(q)
    assert cp.n_full == nf
    X = sh[o[nf:]].astype(np.float64)
    C = oc.vq_init(X, K)
    for _ in range(4):
        codes, _, _ = oc.vq_assign(X, C)
        C, _ = oc.vq_update(X, codes, C)
    codes, _, gap = oc.vq_assign(X, C.astype(np.float32).astype(np.float16).astype(np.float64))
    assert gap.min() > 1e-3
    assert np.array_equal(cp.code.cpu().numpy().view(np.uint16).astype(np.int64), codes)
    ref = C.astype(np.float32).astype(np.float16)
    got = cp.codebook.cpu().numpy().reshape(K, 27)
    # FP64 means in another summation order: the float16 codewords agree to one float16 step
    assert np.all(np.abs(got.astype(np.float64) - ref.astype(np.float64)) <=
                  np.spacing(np.abs(ref)).astype(np.float64))
    assert cp.nbytes() < 0.5 * sum(t.numel() * 4 for t in (params.mean, params.log_scale, params.quat,
                                                            params.opacity_logit, params.sh))
