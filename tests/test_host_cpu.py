"""The OpenMP host kernels (libmlkhost.so) against the CPU oracle, on the CPU:
fp32 matmul and conv2d over every configuration of their search space on
ragged shapes (normwise <= 1e-5 against the double-precision result; exact on
small integers, where every fp32 partial sum is exact), accumulate and
overwrite, and the search itself.  The library exports every function its
header declares."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2307_16080_amd import host
from workloads import conv_inputs, matmul_inputs, random_c

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _normwise(c, r):
    r = np.asarray(r, np.float64)
    return float(np.linalg.norm(np.asarray(c, np.float64) - r) / max(np.linalg.norm(r), 1e-300))


def test_exports_every_declared_symbol():
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "mlk_host.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(mlkh_[a-z0-9_]+)\s*\(", text)))
    assert len(names) >= 6
    lib = host.lib()
    assert all(hasattr(lib, n) for n in names), names
    assert set(names) <= set(host.SIGNATURES)


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 13, 31), (33, 65, 17), (128, 128, 128), (129, 257, 100)])
def test_matmul_every_config(shape):
    M, N, K = shape
    A, B = matmul_inputs(M, N, K, seed=M + N + K, dist="uniform")
    C0 = random_c(M, N, seed=K)
    ref = C0.astype(np.float64) + oracle.matmul_f64(A, B)
    Si, Sj = matmul_inputs(M, N, K, seed=3, dist="small_int")
    exact = oracle.matmul_f64(Si, Sj)
    cfgs = host.configs("matmul", (M, N, K))
    assert cfgs
    for c in cfgs:
        C = C0.copy()
        host.matmul_f32(A, B, C, cfg=c)
        assert _normwise(C, ref) <= 1e-5, c
        C = np.full((M, N), 7.0, np.float32)
        host.matmul_f32(Si, Sj, C, accumulate=False, cfg=c)
        assert np.array_equal(C.astype(np.float64), exact), c


@pytest.mark.parametrize("case", [(1, 64, 56, 56, 64, 3, 3, 1, 1), (2, 3, 15, 17, 5, 3, 3, 2, 1),
                                  (1, 1, 40, 40, 3, 3, 3, 1, 0), (1, 8, 9, 9, 16, 1, 1, 2, 0)])
def test_conv_every_config(case):
    N, C, H, W, F, KH, KW, s, p = case
    x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=N + C + F)
    ref = oracle.conv2d_f64(x, w, (s, s), (p, p))
    xi, wi = conv_inputs(N, C, H, W, F, KH, KW, seed=7, dist="small_int")
    exact = oracle.conv2d_f64(xi, wi, (s, s), (p, p))
    dims = (N, C, H, W, F, KH, KW, s, s, p, p)
    for c in host.configs("conv", dims):
        y = np.zeros(ref.shape, np.float32)
        host.conv2d_f32(x, w, y, (s, s), (p, p), cfg=c)
        host.conv2d_f32(x, w, y, (s, s), (p, p), cfg=c)          # accumulate: twice
        assert _normwise(y, 2.0 * ref) <= 1e-5, c
        y = np.full(ref.shape, 3.0, np.float32)
        host.conv2d_f32(xi, wi, y, (s, s), (p, p), accumulate=False, cfg=c)
        assert np.array_equal(y.astype(np.float64), exact), c


def test_search_picks_a_measured_best():
    best, us, times = host.tune("matmul", (64, 64, 64), strategy=0, reps=3, want_times=True)
    ok = [t for t in times if t > 0]
    assert len(ok) == len(times) and us == min(ok)
    assert best.as_tuple() == host.configs("matmul", (64, 64, 64))[times.index(us)].as_tuple()
    S = len(times)
    _, _, t2 = host.tune("conv", (1, 8, 16, 16, 8, 3, 3, 1, 1, 1, 1), strategy=1, budget_frac=0.5, reps=2,
                         want_times=True)
    assert 1 <= sum(1 for t in t2 if t > 0) <= int(np.ceil(0.5 * len(t2)))
    assert S > 1


def test_bad_arguments():
    A = np.zeros((4, 4), np.float32)
    with pytest.raises(RuntimeError):
        host.matmul_f32(A, A, A.copy(), cfg=host.HostConfig(16, 64, 64, 3, 0))   # unroll 3
    with pytest.raises(TypeError):
        host.matmul_f32(A.astype(np.float64), A, A.copy())
