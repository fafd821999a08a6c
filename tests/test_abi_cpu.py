"""CPU checks of the C ABI: the library loads, exports every function that
include/mlk.h declares, rejects bad arguments before touching a GPU, and its
configuration space and search logic behave (with the analytic fake timer,
no GPU).  No compute kernel is launched here.
"""
import ctypes
import json
import os
import re

import pytest

import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlk.h")

NULL = None


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlk_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)


def test_status_strings_and_version():
    lib = L.lib()
    for i, name in enumerate(L.STATUS_NAMES):
        assert lib.mlk_status_str(i).decode() == name
    assert b"gfx950" in lib.mlk_version()


def _mm(**kw):
    args = dict(inp=L.MLK_F32, out=L.MLK_F32, M=4, N=4, K=4, A=0x1000, lda=4, B=0x2000, ldb=4,
                C=0x3000, ldc=4, sa=NULL, sb=NULL, acc=1, cfg=NULL)
    args.update(kw)
    st = L.lib().mlk_matmul(args["inp"], args["out"], args["M"], args["N"], args["K"], args["A"],
                            args["lda"], args["B"], args["ldb"], args["C"], args["ldc"], args["sa"],
                            args["sb"], args["acc"], args["cfg"], NULL)
    return st, L.lib().mlk_last_error().decode()


def test_matmul_validation():
    assert _mm(M=-1)[0] == 2
    assert _mm(A=NULL)[0] == 1
    assert _mm(C=NULL)[0] == 1
    assert _mm(lda=3)[0] == 3
    assert _mm(ldb=3)[0] == 3
    assert _mm(ldc=2)[0] == 3
    assert _mm(inp=L.MLK_BF16, out=L.MLK_I32)[0] == 4
    assert _mm(inp=L.MLK_I8, out=L.MLK_F32)[0] == 4
    assert _mm(inp=7)[0] == 4
    # C overlapping A
    st, msg = _mm(C=0x1008)
    assert st == 3 and "overlap" in msg
    # scales only for e4m3
    assert _mm(sa=0x5000)[0] == 9
    # illegal explicit configuration
    bad = L.TileConfig(48, 64, 32, 2, 2, 1, 1, 0)
    st, msg = _mm(cfg=ctypes.byref(bad))
    assert st == 5 and "no compiled kernel" in msg
    bad = L.TileConfig(64, 64, 16, 2, 2, 9, 1, 0)  # split larger than the K stages
    assert _mm(K=32, lda=32, cfg=ctypes.byref(bad))[0] == 5


def _mmb(**kw):
    args = dict(inp=L.MLK_F32, out=L.MLK_F32, M=4, N=4, K=4, A=0x1000, lda=4, B=0x2000, ldb=4,
                bias=0x4000, C=0x3000, ldc=4, sa=NULL, sb=NULL, acc=0, cfg=NULL)
    args.update(kw)
    st = L.lib().mlk_matmul_bias(args["inp"], args["out"], args["M"], args["N"], args["K"], args["A"],
                                 args["lda"], args["B"], args["ldb"], args["bias"], args["C"], args["ldc"],
                                 args["sa"], args["sb"], args["acc"], args["cfg"], NULL)
    return st, L.lib().mlk_last_error().decode()


def test_matmul_bias_validation():
    assert _mmb(bias=NULL)[0] == 1
    assert _mmb(M=-1)[0] == 2
    assert _mmb(ldc=2)[0] == 3
    assert _mmb(inp=L.MLK_I8, out=L.MLK_I32)[0] == 4   # integer outputs take no bias
    st, msg = _mmb(bias=0x3008)                         # bias inside C
    assert st == 3 and "bias" in msg
    assert _mmb(sa=0x5000)[0] == 9
    # M == 0 (nothing to write) accepts a NULL bias, as mlk_matmul accepts NULL operands
    assert _mmb(M=0, bias=NULL)[0] == 0


def test_bf16_output_pairs_and_split_rule():
    # bf16 C from bf16 or e4m3 inputs (matmul only); a bf16 result is not split over K
    assert _mm(inp=L.MLK_BF16, out=L.MLK_BF16, acc=0, A=0x10000, B=0x20000, C=0x30000)[0] != 4
    for inp in (L.MLK_BF16, L.MLK_F8E4M3):
        p = mlk.matmul_problem(256, 256, 4096, inp, L.MLK_BF16)
        cfgs = mlk.configs(p)
        assert cfgs and all(c.split_k == 1 and c.stages != 1 for c in cfgs)
        c = cfgs[0]
        split = mlk.TileConfig(c.bm, c.bn, c.bk, c.wm, c.wn, 2, 1, 0, c.stages, c.layout)
        assert not mlk.config_legal(p, split)
        assert mlk.config_legal(mlk.matmul_problem(256, 256, 4096, inp, L.MLK_F32), split)
    assert _mm(inp=L.MLK_F32, out=L.MLK_BF16)[0] == 4
    assert _mm(inp=L.MLK_I8, out=L.MLK_BF16)[0] == 4
    # C overlap is measured in bf16 elements: 4 x 4 bf16 C at 0x3000 ends at 0x3020
    assert _mm(inp=L.MLK_BF16, out=L.MLK_BF16, A=0x3020, B=0x6000)[0] != 3
    assert _mm(inp=L.MLK_BF16, out=L.MLK_BF16, A=0x301E, B=0x6000)[0] == 3


def test_binding_refuses_host_tensors():
    """The binding passes device pointers only: torch tensors in host memory are
    refused before the library is called (a host address must never reach a kernel)."""
    import torch
    A, B, C = torch.zeros(4, 4), torch.zeros(4, 4), torch.zeros(4, 4)
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.matmul(A, B, C)
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.matmul_bias(A, B, torch.zeros(4), C)
    x, w, y = torch.zeros(1, 1, 5, 5), torch.zeros(2, 1, 3, 3), torch.zeros(1, 2, 3, 3)
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.conv2d_nchw_fchw(x, w, y)
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.quantize(torch.zeros(8), "bf16", q=torch.zeros(8, dtype=torch.bfloat16))
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.BatchedCall([(A, B, C)])


def test_binding_checks_shapes_and_dtypes():
    """The C ABI sees pointers only, so the binding checks what it can of each
    tensor (shape, dtype, element count) before any pointer is taken: a short
    output or a wider operand type would otherwise be read or written past its
    allocation."""
    import torch
    A, B, C = torch.zeros(4, 8), torch.zeros(8, 4), torch.zeros(4, 4)
    with pytest.raises(mlk.MlkError, match="one dtype"):
        mlk.matmul(A.to(torch.bfloat16), B, C)
    with pytest.raises(mlk.MlkError, match="scale_a"):
        mlk.matmul(A, B, C, scale_a=torch.zeros(1, dtype=torch.float16))
    with pytest.raises(mlk.MlkError, match="one dtype"):
        mlk.matmul_bias(A, B.to(torch.bfloat16), torch.zeros(4), C)
    x, w = torch.zeros(1, 2, 5, 5), torch.zeros(3, 2, 3, 3)
    with pytest.raises(mlk.MlkError, match="y must be"):
        mlk.conv2d_nchw_fchw(x, w, torch.zeros(1, 3, 2, 3))
    with pytest.raises(mlk.MlkError, match="one dtype"):
        mlk.conv2d_nchw_fchw(x, w.to(torch.bfloat16), torch.zeros(1, 3, 3, 3))
    with pytest.raises(mlk.MlkError, match="y must be"):
        mlk.ConvCall(x, w, torch.zeros(1, 3, 2, 3))
    with pytest.raises(mlk.MlkError, match="GPU memory"):
        mlk.ConvCall(x, w, torch.zeros(1, 3, 3, 3))
    with pytest.raises(mlk.MlkError, match="q must be"):
        mlk.quantize(torch.zeros(8), "bf16", q=torch.zeros(4, dtype=torch.bfloat16))
    with pytest.raises(mlk.MlkError, match="q must be"):
        mlk.quantize(torch.zeros(8), "e4m3", q=torch.zeros(8, dtype=torch.bfloat16))
    with pytest.raises(mlk.MlkError, match="batched"):
        mlk.BatchedCall([(A, B, torch.zeros(4, 5))])
    with pytest.raises(mlk.MlkError, match="batched"):
        mlk.BatchedCall([(A, B, C), (A.to(torch.bfloat16), B.to(torch.bfloat16), C)])
    with pytest.raises(mlk.MlkError, match="params"):
        mlk.mlp_forward(torch.zeros(10), torch.zeros(2, 3), 4, 4)
    assert mlk.mlp_param_count(3, 4, 4) == 3 * 4 + 4 + 4 * 4 + 4 + 4 + 1
    with pytest.raises(mlk.MlkError, match="element count"):
        mlk.err_stats(torch.zeros(4), torch.zeros(5, dtype=torch.float64))


def test_conv_quant_err_validation():
    lib = L.lib()
    conv = lambda **k: lib.mlk_conv2d_nchw_fchw(
        k.get("inp", 0), k.get("out", 0), k.get("N", 1), k.get("C", 2), k.get("H", 5), k.get("W", 5),
        k.get("F", 2), k.get("KH", 3), k.get("KW", 3), k.get("sh", 1), k.get("sw", 1), k.get("ph", 0),
        k.get("pw", 0), k.get("x", 0x1000), k.get("w", 0x9000), k.get("y", 0x20000), 1, NULL, NULL)
    assert conv(sh=0) == 2
    assert conv(ph=-1) == 2
    assert conv(KH=9) == 2            # filter larger than the padded image
    assert conv(x=NULL) == 1
    assert conv(inp=L.MLK_I8, out=L.MLK_I32) == 4
    assert conv(inp=L.MLK_BF16, out=L.MLK_BF16) == 4   # bf16 outputs: matmul only
    assert conv(y=0x1004) == 3        # y overlapping x
    assert lib.mlk_quantize(L.MLK_F32, 4, 0x1000, 0x2000, 0x3000, NULL) == 4
    assert lib.mlk_quantize(L.MLK_F8E4M3, 4, 0x1000, 0x2000, NULL, NULL) == 1
    assert lib.mlk_quantize(L.MLK_BF16, -1, 0x1000, 0x2000, NULL, NULL) == 2
    assert lib.mlk_quantize(L.MLK_BF16, 16, 0x1000, 0x1010, NULL, NULL) == 3
    assert lib.mlk_err_stats(L.MLK_BF16, 4, 0x1000, 0x2000, NULL, 0x3000, NULL) == 4
    assert lib.mlk_err_stats(L.MLK_F32, 4, 0x1000, NULL, NULL, 0x3000, NULL) == 1
    assert lib.mlk_adam_step(4, 0x1000, 0x2000, 0x3000, 0x4000, 0.1, 0.9, 1.5, 1e-8, 1, NULL) == 9
    assert lib.mlk_adam_step(4, 0x1000, 0x2000, 0x3000, 0x4000, 0.1, 0.9, 0.99, 1e-8, 0, NULL) == 9
    assert lib.mlk_mlp_forward(4, 0, 8, 8, 0x1, 0x2, 0x3, NULL) == 2


def test_batched_validation():
    lib = L.lib()
    d = (L.GemmDesc * 2)()
    d[0] = L.GemmDesc(4, 4, 4, 0x1000, 4, 0x2000, 4, 0x3000, 4)
    d[1] = L.GemmDesc(4, 4, 4, 0x4000, 4, 0x5000, 3, 0x6000, 4)
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, NULL, 0, 1, 0, NULL) == 3
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 0, d, NULL, 0, 1, 0, NULL) == 2
    assert lib.mlk_batched_matmul(L.MLK_I8, L.MLK_I32, 2, d, NULL, 0, 1, 0, NULL) == 4
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, NULL, 0, 1, 0x8, NULL) == 9
    d[1] = L.GemmDesc(4, 4, 4, 0x4000, 4, NULL, 4, 0x6000, 4)
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, NULL, 0, 1, 0, NULL) == 1


def test_config_space():
    p = mlk.matmul_problem(4096, 4096, 4096, L.MLK_BF16, L.MLK_F32)
    cfgs = mlk.configs(p)
    assert 50 <= len(cfgs) <= 600
    assert len({c.as_tuple() for c in cfgs}) == len(cfgs)
    for c in cfgs:
        assert mlk.config_legal(p, c)
    # small problems prune tiles that are twice the problem or more
    small = mlk.configs(mlk.matmul_problem(40, 40, 40, L.MLK_BF16, L.MLK_F32))
    assert all(c.bm <= 64 and c.bn <= 64 for c in small)
    # conv and batched spaces
    cp = mlk.conv_problem(32, 64, 56, 56, 64, 3, 3, 1, 1)
    assert mlk.config_count(cp) > 20
    assert {c.layout for c in mlk.configs(cp)} == {0, 1, 3}
    # layout 3 (NCHW channel gather): the register-loaded channels-last tiles only
    assert all(c.stages == 1 for c in mlk.configs(cp) if c.layout == 3)
    assert {c.layout for c in mlk.configs(mlk.conv_problem(2, 64, 16, 16, 64, 3, 3, 1, 1, L.MLK_F32))} == {0, 1}
    # channels-last and channel gather need C a multiple of the 16-byte vector
    # (8 bf16); with F <= 16 the direct (stencil) conv adds its layout-2 tiles
    c3 = mlk.conv_problem(1, 3, 32, 32, 16, 3, 3, 1, 1)
    assert {c.layout for c in mlk.configs(c3)} == {0, 2}
    assert not mlk.config_legal(c3, mlk.TileConfig(32, 32, 32, 1, 1, 1, 1, 0, 0, 1))
    assert not mlk.config_legal(c3, mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 1, 3))
    direct = [c for c in mlk.configs(c3) if c.layout == 2]
    assert direct and all(c.wm == 0 and c.wn == 0 and c.split_k == 1 and c.bk == 1 for c in direct)
    d0 = direct[0]
    assert not mlk.config_legal(c3, mlk.TileConfig(*list(d0.as_tuple())[:9], 0))      # only as layout 2
    assert not mlk.config_legal(c3, mlk.TileConfig(d0.bm, d0.bn, 1, 0, 0, 2, 1, 0, 0, 2))  # no split K
    # beyond its limits: 17 filters, stride 3, a 9x9 filter
    for q in (mlk.conv_problem(1, 3, 32, 32, 17, 3, 3, 1, 1), mlk.conv_problem(1, 3, 32, 32, 8, 3, 3, 3, 1),
              mlk.conv_problem(1, 3, 32, 32, 8, 9, 9, 1, 4)):
        assert not any(c.layout == 2 for c in mlk.configs(q))
        assert not mlk.config_legal(q, d0)
    # and layout is meaningless for matmul
    assert not mlk.config_legal(mlk.matmul_problem(64, 64, 64, L.MLK_BF16, L.MLK_F32),
                                mlk.TileConfig(64, 64, 32, 2, 2, 1, 1, 0, 0, 1))
    # the direct-layout conv form (stages 1) exists channels-last and as the
    # NCHW channel gather, never as the plain NCHW form (layout 0)
    fast_conv = [c for c in mlk.configs(cp) if c.stages == 1]
    assert fast_conv and {c.layout for c in fast_conv} == {1, 3}
    f0 = fast_conv[0]
    assert not mlk.config_legal(cp, mlk.TileConfig(*list(f0.as_tuple())[:9], 0))
    assert not any(c.stages == 1 for c in mlk.configs(c3))
    # direct-to-LDS tiles take any matmul shape (operands are packed as needed)
    odd = mlk.matmul_problem(1000, 1001, 999, L.MLK_BF16, L.MLK_F32)
    assert any(c.stages >= 2 for c in mlk.configs(odd))
    assert mlk.config_legal(odd, mlk.TileConfig(256, 256, 64, 2, 4, 1, 8, 0, 2, 0))
    # int8 has its own direct-layout tiles (int32 output stage only); fp32 has none
    assert not any(c.stages for c in mlk.configs(mlk.matmul_problem(999, 999, 999, L.MLK_F32, L.MLK_F32)))
    i8 = mlk.matmul_problem(999, 999, 999, L.MLK_I8, L.MLK_I32)
    assert {c.stages for c in mlk.configs(i8)} >= {0, 1, 2, 3, 4}
    assert all(c.bk == 128 for c in mlk.configs(i8) if c.stages)
    assert mlk.config_legal(i8, mlk.TileConfig(64, 64, 128, 2, 2, 4, 1, 0, 3, 0))
    bp = mlk.batched_problem([(100, 200, 300), (64, 64, 64)])
    bc = mlk.configs(bp)
    assert bc and all(c.split_k == 1 for c in bc)
    # batches take every persistent tile family, direct-to-LDS ones included
    assert {c.stages for c in bc} >= {0, 1, 2}
    # invalid problems count as -1
    bad = mlk.matmul_problem(4, 4, 4, L.MLK_I8, L.MLK_F32)
    assert L.lib().mlk_config_count(ctypes.byref(bad)) == -1


def test_features_shape():
    p = mlk.matmul_problem(1024, 512, 256, L.MLK_BF16, L.MLK_F32)
    f = mlk.features(p, mlk.configs(p)[0])
    assert len(f) == L.lib().mlk_model_feature_count()
    assert f[0] == 10.0 and f[1] == 9.0 and f[2] == 8.0


def test_tune_exhaustive_fake_timer_returns_argmin():
    p = mlk.matmul_problem(2048, 1024, 512, L.MLK_BF16, L.MLK_F32)
    best, rep, times = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True, want_times=True, seed=3)
    assert rep.n_measured == rep.n_legal == len(times)
    assert all(t > 0 for t in times)
    tmin = min(times)
    tied = [i for i, t in enumerate(times) if t <= 1.01 * tmin]
    assert rep.best_index in tied
    assert best.as_tuple() == mlk.configs(p)[rep.best_index].as_tuple()


def test_tune_random_budget_and_determinism():
    p = mlk.matmul_problem(1000, 3000, 700, L.MLK_F32, L.MLK_F32)
    S = mlk.config_count(p)
    b1, r1, t1 = mlk.tune(p, mlk.MLK_TUNE_RANDOM, budget_frac=0.2, seed=11, fake_timer=True,
                          want_times=True)
    b2, r2, t2 = mlk.tune(p, mlk.MLK_TUNE_RANDOM, budget_frac=0.2, seed=11, fake_timer=True,
                          want_times=True)
    measured = [i for i, t in enumerate(t1) if t > 0]
    assert r1.n_measured == len(measured) == -(-S * 2 // 10)
    assert b1.as_tuple() == b2.as_tuple() and t1 == t2
    _, _, t3 = mlk.tune(p, mlk.MLK_TUNE_RANDOM, budget_frac=0.2, seed=12, fake_timer=True,
                        want_times=True)
    assert [i for i, t in enumerate(t3) if t > 0] != measured


def _table(p, seed=3):
    _, _, times = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True, want_times=True, seed=seed)
    return times


def test_tune_es_budget_determinism_and_neighbourhood():
    """ES measures exactly its budget of distinct configurations, reads its
    times from the replayed table, and is a function of its seed."""
    p = mlk.conv_problem(32, 64, 56, 56, 64, 3, 3, 1, 1, L.MLK_BF16, L.MLK_F32)
    S = mlk.config_count(p)
    tab = _table(p)
    b1, r1, t1 = mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=0.2, seed=5, table=tab, want_times=True)
    b2, r2, t2 = mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=0.2, seed=5, table=tab, want_times=True)
    measured = [i for i, t in enumerate(t1) if t > 0]
    assert r1.n_measured == len(measured) == -(-S * 2 // 10)
    assert b1.as_tuple() == b2.as_tuple() and t1 == t2
    assert all(t1[i] == tab[i] for i in measured)               # the table, not a measurement
    assert rep_best_is_measured_min(r1, t1)
    _, _, t3 = mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=0.2, seed=6, table=tab, want_times=True)
    assert [i for i, t in enumerate(t3) if t > 0] != measured


def rep_best_is_measured_min(rep, times):
    tmin = min(t for t in times if t > 0)
    return times[rep.best_index] <= 1.01 * tmin


def test_tune_es_full_budget_and_failed_configurations():
    """With the whole budget ES visits every configuration (restarts included)
    and returns the table's fastest; configurations whose time is <= 0 count
    as failed launches and are never returned."""
    p = mlk.matmul_problem(1000, 300, 2000, L.MLK_F32, L.MLK_F32)
    S = mlk.config_count(p)
    tab = _table(p, seed=1)
    fastest = min(range(S), key=lambda i: tab[i])
    _, rep, _ = mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=1.0, seed=2, table=tab)
    assert rep.n_measured == S and rep_best_is_measured_min(rep, tab)
    failed = list(tab)
    failed[fastest] = -1.0                                      # the fastest cannot launch
    best, rep, times = mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=1.0, seed=2, table=failed, want_times=True)
    assert rep.best_index != fastest and times[rep.best_index] > 0
    with pytest.raises(mlk.MlkError):
        mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=0.5, table=tab[:-1])


def test_tune_es_beats_random_on_replayed_tables():
    """On the analytic timer's tables ES's mean regret over 40 seeds is no
    worse than random sampling's at the same 20% budget on each problem, and
    the sum of the medians is lower.  (Per problem the medians can invert: on a
    plateau of near-equal configurations more than half of ES's runs may settle
    one step above the best while random sampling's spread is wider.)"""
    import numpy as np
    probs = [mlk.conv_problem(1, 256, 14, 14, 512, 3, 3, 2, 1, L.MLK_BF16, L.MLK_F32),
             mlk.conv_problem(32, 128, 28, 28, 256, 3, 3, 2, 1, L.MLK_BF16, L.MLK_F32),
             mlk.matmul_problem(4096, 4096, 4096, L.MLK_BF16, L.MLK_F32)]
    es_tot = rnd_tot = 0.0
    for p in probs:
        tab = _table(p, seed=0)
        best = min(tab)
        es = [mlk.tune(p, mlk.MLK_TUNE_ES, budget_frac=0.2, seed=s, table=tab)[1].best_us / best - 1
              for s in range(40)]
        rnd = [mlk.tune(p, mlk.MLK_TUNE_RANDOM, budget_frac=0.2, seed=s, table=tab)[1].best_us / best - 1
               for s in range(40)]
        assert np.mean(es) <= np.mean(rnd) + 1e-12
        es_tot += float(np.median(es))
        rnd_tot += float(np.median(rnd))
    assert es_tot < rnd_tot


def test_tune_database_append_and_resume(tmp_path):
    db = str(tmp_path / "tune.jsonl")
    p = mlk.matmul_problem(512, 512, 512, L.MLK_BF16, L.MLK_F32)
    best, rep, _ = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True, db_path=db)
    assert rep.from_db == 0
    lines = [json.loads(l) for l in open(db)]
    assert len(lines) == 1 and lines[0]["cfg"] == list(best.as_tuple())
    best2, rep2, _ = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True, db_path=db, use_db=True)
    assert rep2.from_db == 1 and rep2.n_measured == 0
    assert best2.as_tuple() == best.as_tuple()
    # a corrupt line is skipped, a different problem is tuned afresh
    with open(db, "a") as f:
        f.write("{not json\n")
    q = mlk.matmul_problem(256, 512, 512, L.MLK_BF16, L.MLK_F32)
    _, rep3, _ = mlk.tune(q, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True, db_path=db, use_db=True)
    assert rep3.from_db == 0 and rep3.n_measured == rep3.n_legal
    assert len(open(db).read().splitlines()) == 3


def test_tune_bad_arguments(tmp_path):
    p = mlk.matmul_problem(64, 64, 64, L.MLK_BF16, L.MLK_F32)
    with pytest.raises(mlk.MlkError, match="budget_frac"):
        mlk.tune(p, mlk.MLK_TUNE_RANDOM, budget_frac=0.0, fake_timer=True)
    with pytest.raises(mlk.MlkError, match="model"):
        mlk.tune(p, mlk.MLK_TUNE_MODEL, budget_frac=0.2, fake_timer=True)
    with pytest.raises(mlk.MlkError, match="MLK_ERR_DB"):
        mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, fake_timer=True,
                 db_path=str(tmp_path / "no_such_dir" / "db.jsonl"))


def test_direct_layout_tiles_refuse_overflowing_output_offsets():
    """The direct-layout tiles address their output tile with 32-bit offsets: an
    ldc that would overflow them is refused before anything is enqueued, and
    such tiles are not offered for a problem whose N alone would overflow."""
    fast = L.TileConfig(256, 256, 64, 2, 4, 1, 1, 0, 2, 0)
    big_ldc = (1 << 31) // 255 + 1
    st = L.lib().mlk_matmul(L.MLK_BF16, L.MLK_F32, 256, 256, 64, 0x10000000, 64, 0x20000000, 256,
                            0x100000000, big_ldc, NULL, NULL, 1, ctypes.byref(fast), NULL)
    assert st == 5 and "32-bit" in L.lib().mlk_last_error().decode()
    p = mlk.matmul_problem(256, (1 << 31) // 255 + 1, 64, L.MLK_BF16, L.MLK_F32)
    assert not mlk.config_legal(p, fast)
    N = p.N
    assert all(c.stages == 0 or (c.bm - 1) * N + c.bn < (1 << 31) for c in mlk.configs(p))
    assert any(c.stages >= 1 for c in mlk.configs(p))   # the smaller direct-layout tiles stay


def test_matmul_noalloc_validation():
    """mlk_matmul_noalloc checks its arguments like mlk_matmul and refuses a
    shape whose packed operand copies exceed its fixed workspace, all before
    any HIP call (no GPU here)."""
    lib = L.lib()

    def call(M, N, K, A, lda, B, ldb, C, ldc, cfg):
        return lib.mlk_matmul_noalloc(L.MLK_BF16, L.MLK_F32, M, N, K, A, lda, B, ldb, C, ldc, NULL, NULL, 1,
                                      cfg, NULL)

    packed = L.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 4, 0)
    assert call(-1, 4, 4, 0x1000, 4, 0x2000, 4, 0x3000, 4, NULL) == 2
    assert call(4, 4, 4, NULL, 4, 0x2000, 4, 0x3000, 4, NULL) == 1
    assert call(4, 4, 4, 0x1000, 3, 0x2000, 4, 0x3000, 4, NULL) == 3
    # 4096 x 8193 bf16 A packed to 4096 x 8256: more than the 64 MiB workspace
    st = call(4096, 64, 8193, 0x10000000, 8193, 0x20000000, 64, 0x30000000, 64, ctypes.byref(packed))
    msg = lib.mlk_last_error().decode()
    assert st == 2 and "no-alloc workspace" in msg, msg


def test_batched_config_count_validation():
    """ncfgs must be 0, 1 or count; a per-GEMM configuration is checked against
    its own GEMM; all before any HIP call."""
    lib = L.lib()
    d = (L.GemmDesc * 2)(L.GemmDesc(4, 4, 4, 0x1000, 4, 0x2000, 4, 0x3000, 4),
                         L.GemmDesc(8, 8, 8, 0x4000, 8, 0x5000, 8, 0x6000, 8))
    good = L.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 0, 0)
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, ctypes.byref(good), 3, 1, 0, NULL) == 9
    assert lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, NULL, 1, 1, 0, NULL) == 1
    bad = (L.TileConfig * 2)(good, L.TileConfig(48, 64, 32, 2, 2, 1, 1, 0, 0, 0))
    st = lib.mlk_batched_matmul(L.MLK_BF16, L.MLK_F32, 2, d, bad, 2, 1, 0, NULL)
    assert st == 5 and "desc 1" in lib.mlk_last_error().decode()


def test_conv_batch_validation():
    """mlk_conv2d_batch_create refuses bad dtypes, counts, shapes, channels not
    a multiple of 8, NULL or overlapping buffers and configurations that are
    not a register-loaded conv tile -- all before any HIP call."""
    lib = L.lib()
    h = ctypes.c_void_p()

    def desc(x, w, y, C=8, F=16, H=8, W=8):
        return L.ConvDesc(1, C, H, W, F, 3, 3, 1, 1, 1, 1, x, w, y)

    one = (L.ConvDesc * 1)(desc(0x100000, 0x200000, 0x300000))
    create = lambda d, n, cfg=NULL, dt=L.MLK_BF16: lib.mlk_conv2d_batch_create(dt, L.MLK_F32, n, d, 1, cfg, NULL,
                                                                                ctypes.byref(h))
    assert create(one, 1, dt=L.MLK_F32) == 4
    assert create(one, 0) == 9
    assert create(NULL, 1) == 1
    assert lib.mlk_conv2d_batch_create(L.MLK_BF16, L.MLK_F32, 1, one, 1, NULL, NULL, NULL) == 1
    assert create((L.ConvDesc * 1)(desc(0x100000, 0x200000, 0x300000, C=12)), 1) == 2
    bad_shape = (L.ConvDesc * 1)(L.ConvDesc(1, 8, 2, 2, 16, 5, 5, 1, 0, 1, 0, 0x100000, 0x200000, 0x300000))
    assert create(bad_shape, 1) == 2
    assert create((L.ConvDesc * 1)(desc(0x100000, 0, 0x300000)), 1) == 1
    # y of one convolution over another's input, or two outputs sharing memory
    two = (L.ConvDesc * 2)(desc(0x100000, 0x200000, 0x300000), desc(0x300100, 0x400000, 0x500000))
    st = create(two, 2)
    assert st == 3 and "descriptor 0" in lib.mlk_last_error().decode()
    two = (L.ConvDesc * 2)(desc(0x100000, 0x200000, 0x300000), desc(0x600000, 0x400000, 0x300800))
    assert create(two, 2) == 3
    # configurations: a register-loaded conv tile (stages 1) with a split cap in [1, 32]
    assert create(one, 1, ctypes.byref(L.TileConfig(64, 64, 64, 2, 2, 0, 1, 0, 1, 3))) == 5
    assert create(one, 1, ctypes.byref(L.TileConfig(64, 64, 64, 2, 2, 33, 1, 0, 1, 3))) == 5
    assert create(one, 1, ctypes.byref(L.TileConfig(64, 64, 64, 2, 2, 4, 1, 0, 2, 1))) == 5
    assert create(one, 1, ctypes.byref(L.TileConfig(48, 64, 64, 2, 2, 4, 1, 0, 1, 3))) == 5
    # run / info / destroy of a NULL batch
    assert lib.mlk_conv2d_batch_run(NULL, NULL) == 1
    assert lib.mlk_conv2d_batch_info(NULL, NULL, NULL, NULL) == 1
    assert lib.mlk_conv2d_batch_update_filters(NULL, NULL) == 1
    lib.mlk_conv2d_batch_destroy(NULL)


def test_mfma_rate_validation():
    """mlk_mfma_rate refuses other dtypes, iteration counts outside [1, 16384],
    NULL pointers and an output buffer shorter than the launch writes, before
    launching anything."""
    lib = L.lib()
    fl = ctypes.c_int64()
    buf = 0x100000
    assert lib.mlk_mfma_rate(L.MLK_F32, 16, buf, 1 << 20, ctypes.byref(fl), NULL) == 4
    assert lib.mlk_mfma_rate(L.MLK_BF16, 0, buf, 1 << 20, ctypes.byref(fl), NULL) == 9
    assert lib.mlk_mfma_rate(L.MLK_BF16, 16385, buf, 1 << 20, ctypes.byref(fl), NULL) == 9
    assert lib.mlk_mfma_rate(L.MLK_BF16, 16, NULL, 1 << 20, ctypes.byref(fl), NULL) == 1
    assert lib.mlk_mfma_rate(L.MLK_F8E4M3, 16, buf, 1 << 20, NULL, NULL) == 1
    assert lib.mlk_mfma_rate(L.MLK_BF16, 16, buf, 0, ctypes.byref(fl), NULL) == 2
    assert lib.mlk_mfma_rate(L.MLK_BF16, 16, buf, 8, ctypes.byref(fl), NULL) == 2   # fewer than one per wave
