"""GPU tests of the batched GEMM (per-GEMM launches, one persistent launch,
hipGraph replay), the FP64 error reduction, the cost-model kernels against
the oracle's double-precision MLP, and a real (measured) tuning run.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import batched_inputs, batched_shapes, matmul_inputs

from gpu_util import dev, from_bf16_codes, host, normwise, say

pytestmark = pytest.mark.gpu


def _batch(shapes, seed=1, dist="normal"):
    ins = batched_inputs(shapes, seed=seed, dist=dist)
    probs, codes = [], []
    for (A, B), (M, N, K) in zip(ins, shapes):
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        codes.append((qa, qb))
        probs.append((from_bf16_codes(qa), from_bf16_codes(qb), torch.zeros(M, N, device="cuda")))
    return probs, codes


def _outs(probs):
    torch.cuda.synchronize()
    return [p[2].cpu().numpy().copy() for p in probs]


def _zero(probs):
    for p in probs:
        p[2].zero_()


def test_batched_256_persistent_equals_per_gemm_and_oracle():
    shapes = batched_shapes(256, seed=0)
    probs, codes = _batch(shapes)
    cfg = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0)
    mlk.batched_matmul(probs, cfg=cfg)                     # one launch per GEMM
    base = _outs(probs)
    _zero(probs)
    mlk.batched_matmul(probs, cfg=cfg, persistent=True)    # one persistent launch
    pers = _outs(probs)
    for i, (a, b) in enumerate(zip(base, pers)):
        assert np.array_equal(a, b), i
    # oracle on a sample of the GEMMs (all sizes of the draw are covered by the bit equality)
    for i in list(range(0, 256, 37)) + [int(np.argmin([m * n * k for m, n, k in shapes]))]:
        qa, qb = codes[i]
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), threads=oracle.default_threads())
        assert normwise(pers[i], ref) <= 1e-5, (i, shapes[i])


@pytest.mark.parametrize("tile", [(128, 128, 64, 2, 2), (256, 128, 64, 2, 2)])
def test_batched_persistent_register_loaded_tiles(tile):
    """The persistent launch of the register-loaded direct-layout kernel (any
    alignment, K not a multiple of the stage depth) against per-GEMM launches
    of the same configuration, bit for bit, and against the oracle."""
    shapes = batched_shapes(64, seed=5)
    probs, codes = _batch(shapes, seed=4)
    cfg = mlk.TileConfig(*tile, 1, 1, 0, 1, 0)
    mlk.batched_matmul(probs, cfg=cfg)
    base = _outs(probs)
    _zero(probs)
    mlk.batched_matmul(probs, cfg=cfg, persistent=True, graph=True)
    pers = _outs(probs)
    for i, (a, b) in enumerate(zip(base, pers)):
        assert np.array_equal(a, b), i
    for i in range(0, 64, 9):
        qa, qb = codes[i]
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), threads=oracle.default_threads())
        assert normwise(pers[i], ref) <= 1e-5, (i, shapes[i])


@pytest.mark.parametrize("tile", [(256, 256, 64, 2, 4, 2), (128, 128, 64, 2, 2, 4), (256, 128, 64, 2, 2, 3)])
def test_batched_persistent_direct_tiles_with_packing(tile):
    """Direct-to-LDS tiles on a batch with odd K and N: the operands are packed
    into zero-padded copies inside the launch (and its graph); the result must
    equal per-GEMM launches of the register-loaded kernel bit for bit (same
    MFMA sequence over the same 32-deep k chunks) on every graph replay."""
    shapes = batched_shapes(48, seed=6) + [(64, 128, 128), (1, 1, 1), (300, 8, 64)]
    probs, codes = _batch(shapes, seed=7)
    ref_cfg = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 0)
    mlk.batched_matmul(probs, cfg=ref_cfg)
    base = _outs(probs)
    cfg = mlk.TileConfig(*tile[:5], 1, 1, 0, tile[5], 0)
    _zero(probs)
    mlk.batched_matmul(probs, cfg=cfg)                      # per-GEMM launches, each packing its own
    for i, (a, b) in enumerate(zip(base, _outs(probs))):
        assert np.array_equal(a, b), ("per-GEMM", i, shapes[i])
    for rep in range(3):
        _zero(probs)
        junk = torch.randn(1000, device="cuda").sum()       # eager work between replays
        mlk.batched_matmul(probs, cfg=cfg, persistent=True, graph=rep > 0)
        got = _outs(probs)
        for i, (a, b) in enumerate(zip(base, got)):
            assert np.array_equal(a, b), (rep, i, shapes[i])
        del junk
    for i in (0, 17, 48, 49, 50):
        qa, qb = codes[i]
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), threads=oracle.default_threads())
        assert normwise(got[i], ref) <= 1e-5, (i, shapes[i])


def test_batched_graph_replays_match_eager():
    shapes = batched_shapes(40, seed=3)
    probs, _ = _batch(shapes, seed=2, dist="small_int")
    cfg = mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0)
    mlk.batched_matmul(probs, cfg=cfg, accumulate=False, persistent=True)
    want = _outs(probs)
    for persistent in (True, False):
        for rep in range(3):
            _zero(probs)
            # eager work between replays
            junk = torch.randn(1000, device="cuda").sum()
            mlk.batched_matmul(probs, cfg=cfg, accumulate=False, persistent=persistent, graph=True)
            got = _outs(probs)
            for i, (a, b) in enumerate(zip(want, got)):
                assert np.array_equal(a, b), (persistent, rep, i)
            del junk


def test_batched_call_replays_accumulate():
    """A BatchedCall bound once: every call is one graph replay and adds A B
    into C again (C = 3 A B after three calls on small integers, exact)."""
    shapes = batched_shapes(32, seed=8) + [(1, 1, 1), (70, 9, 33)]
    probs, _ = _batch(shapes, seed=9, dist="small_int")
    cfg = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 2, 0)
    mlk.batched_matmul(probs, cfg=cfg, accumulate=False, persistent=True)
    once = _outs(probs)
    _zero(probs)
    call = mlk.BatchedCall(probs, cfg=cfg, persistent=True, graph=True)
    for rep in range(3):
        junk = torch.randn(1000, device="cuda").sum()       # eager work between replays
        call()
        got = _outs(probs)
        for i, (a, b) in enumerate(zip(once, got)):
            assert np.array_equal(a * (rep + 1), b), (rep, i, shapes[i])
        del junk
    with pytest.raises(mlk.MlkError):
        mlk.BatchedCall([])


def test_batched_f32_and_default_config():
    shapes = [(33, 65, 17), (128, 128, 128), (1, 300, 7), (200, 1, 64)]
    ins = batched_inputs(shapes, seed=5, dist="small_int")
    probs = [(dev(A), dev(B), torch.zeros(M, N, device="cuda")) for (A, B), (M, N, K) in zip(ins, shapes)]
    mlk.batched_matmul(probs, persistent=True)
    for (A, B), p in zip(ins, probs):
        assert np.array_equal(host(p[2]).astype(np.float64), oracle.matmul_f64(A, B))


def test_err_stats_matches_oracle():
    rng = np.random.default_rng(0)
    n = 300001
    r = rng.standard_normal(n)
    c = (r + rng.standard_normal(n) * 1e-3).astype(np.float32)
    bound = np.abs(rng.standard_normal(n)) * 1e-2
    bound[::7] = 0.0
    got = host(mlk.err_stats(dev(c), dev(r), dev(bound)))
    want = oracle.err_stats(c, r, bound)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    ci = rng.integers(-1000, 1000, n).astype(np.int32)
    got = host(mlk.err_stats(dev(ci), dev(r)))
    want = oracle.err_stats(ci, r)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # reproducible
    assert np.array_equal(host(mlk.err_stats(dev(c), dev(r), dev(bound))),
                          host(mlk.err_stats(dev(c), dev(r), dev(bound))))


D0, H1, H2 = 26, 32, 24


def test_mlp_forward_and_gradient_vs_oracle():
    rng = np.random.default_rng(1)
    P = oracle.mlp_param_count(D0, H1, H2)
    p = (rng.standard_normal(P) * 0.3).astype(np.float32)
    X = rng.standard_normal((300, D0)).astype(np.float32)
    t = rng.standard_normal(300).astype(np.float32)
    y = host(mlk.mlp_forward(dev(p), dev(X), H1, H2))
    yr = oracle.mlp_forward(p, X, H1, H2)
    np.testing.assert_allclose(y, yr, rtol=1e-4, atol=1e-5)
    loss, g = mlk.mlp_loss_grad(dev(p), dev(X), dev(t), H1, H2)
    lr_, gr = oracle.mlp_loss_grad(p, X, t, H1, H2)
    assert abs(host(loss)[0] - lr_) <= 1e-4 * abs(lr_)
    assert np.linalg.norm(host(g) - gr) <= 1e-4 * np.linalg.norm(gr)


def test_adam_vs_oracle():
    rng = np.random.default_rng(2)
    n = 5000
    p = rng.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    pd, md, vd = dev(p.astype(np.float32)), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for step in range(1, 6):
        g = rng.standard_normal(n)
        oracle.adam_step(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, step)
        mlk.adam_step(pd, dev(g.astype(np.float32)), md, vd, 1e-2, 0.9, 0.999, 1e-8, step)
    np.testing.assert_allclose(host(pd), p, rtol=1e-5, atol=1e-6)


def test_model_trains_and_predicts():
    rng = np.random.default_rng(3)
    model = mlk.CostModel(hidden=32, seed=1)
    p = mlk.matmul_problem(1024, 1024, 1024, L.MLK_BF16, L.MLK_F32)
    cfgs = mlk.configs(p)
    # synthetic target: a smooth function of the tile
    for c in cfgs:
        model.add_sample(p, c, 10.0 + c.bm / 16 + 3 * c.split_k + rng.uniform(0, 0.1))
    loss = model.train(epochs=300, batch=64, lr=3e-3)
    say("model loss", loss)
    assert loss < 0.1
    pred = np.array(model.predict(p, cfgs))
    truth = np.array([10.0 + c.bm / 16 + 3 * c.split_k for c in cfgs])
    assert np.corrcoef(pred, truth)[0, 1] > 0.9


def test_tune_measured_small_problem(tmp_path):
    p = mlk.matmul_problem(512, 384, 256, L.MLK_BF16, L.MLK_F32)
    best, rep, times = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, reps=5, warmup=1, want_times=True,
                                db_path=str(tmp_path / "db.jsonl"))
    say("tuned", best, rep.best_us, rep.n_legal)
    assert rep.n_measured == rep.n_legal and all(t > 0 for t in times)
    assert rep.best_us <= 1.01 * min(times)
    # the tuned config is now the default for this problem: a launch without cfg uses it
    A, B = matmul_inputs(512, 384, 256, seed=0, dist="small_int")
    C = torch.zeros(512, 384, device="cuda")
    mlk.matmul(dev(A, torch.bfloat16), dev(B, torch.bfloat16), C)
    assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))


def test_batched_per_gemm_configs():
    """One configuration per GEMM: per-GEMM launches honour each (split K
    included); the persistent launch groups the GEMMs by kernel (here a
    register-staged tile, the register-loaded direct-layout tile and a
    direct-to-LDS tile with packing) and equals per-GEMM launches of the same
    configurations (split 1) bit for bit on every graph replay; a zeroed entry
    leaves that GEMM to choose."""
    shapes = batched_shapes(36, seed=11) + [(64, 128, 128), (1, 1, 1), (300, 8, 64)]
    probs, codes = _batch(shapes, seed=12)
    fam = [mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 0, 0), mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 0),
           mlk.TileConfig(256, 128, 64, 2, 2, 1, 1, 0, 3, 0)]
    cfgs = [fam[i % 3] for i in range(len(shapes))]
    split = [mlk.TileConfig(*(list(c.as_tuple())[:5] + [2 if s[2] >= 512 and c.stages == 0 else 1] +
                              list(c.as_tuple())[6:])) for c, s in zip(cfgs, shapes)]
    # per-GEMM launches with split K where the depth allows it: oracle
    _zero(probs)
    mlk.batched_matmul(probs, cfg=split)
    got = _outs(probs)
    for i in range(0, len(shapes), 5):
        qa, qb = codes[i]
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), threads=oracle.default_threads())
        assert normwise(got[i], ref) <= 1e-5, (i, shapes[i], split[i])
    # split 1 per-GEMM launches, the reference for the persistent groups
    _zero(probs)
    mlk.batched_matmul(probs, cfg=cfgs)
    base = _outs(probs)
    call = mlk.BatchedCall(probs, cfg=cfgs, persistent=True, graph=True)
    for rep in range(3):
        _zero(probs)
        junk = torch.randn(1000, device="cuda").sum()
        call()
        for i, (a, b) in enumerate(zip(base, _outs(probs))):
            assert np.array_equal(a, b), (rep, i, shapes[i], cfgs[i])
        del junk
    # zeroed entries: those GEMMs choose (persistent: the batch's choice)
    mixed = [None if i % 4 == 0 else c for i, c in enumerate(cfgs)]
    _zero(probs)
    mlk.batched_matmul(probs, cfg=mixed, persistent=True)
    got = _outs(probs)
    for i in (0, 4, 8, len(shapes) - 1):
        qa, qb = codes[i]
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), threads=oracle.default_threads())
        assert normwise(got[i], ref) <= 1e-5, (i, shapes[i])
    mlk.release()
