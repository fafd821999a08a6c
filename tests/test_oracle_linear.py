"""Pins of the oracle's Linear layer (matmul nest into a zeroed buffer, then
the bias nest of the paper's lowered torch.nn.Linear, Sec. 2.1 listing
"listing1"): a hand-computed example, the zero-bias and zero-input special
cases, and the per-column broadcast of the bias."""
import numpy as np

import oracle


def test_linear_worked_example():
    # [[1, 2], [3, 4]] @ [[5, 6], [7, 8]] = [[19, 22], [43, 50]]; bias (0.5, -1) on the columns
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[5.0, 6.0], [7.0, 8.0]])
    got = oracle.linear_f64(A, B, np.array([0.5, -1.0]))
    assert np.array_equal(got, np.array([[19.5, 21.0], [43.5, 49.0]]))


def test_linear_special_cases_and_broadcast():
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 9, (7, 5)).astype(np.float64)
    B = rng.integers(-8, 9, (5, 11)).astype(np.float64)
    bias = rng.integers(-8, 9, 11).astype(np.float64)
    # zero bias: the plain product
    assert np.array_equal(oracle.linear_f64(A, B, np.zeros(11)), oracle.matmul_f64(A, B))
    # zero input: every row is the bias
    assert np.array_equal(oracle.linear_f64(np.zeros((7, 5)), B, bias), np.tile(bias, (7, 1)))
    # the bias runs along columns (j), the same for every row (exact on integers)
    d = oracle.linear_f64(A, B, bias) - oracle.matmul_f64(A, B)
    assert np.array_equal(d, np.broadcast_to(bias, (7, 11)))
    # accumulate mode: C + (A B + bias)
    C0 = rng.integers(-8, 9, (7, 11)).astype(np.float64)
    assert np.array_equal(oracle.linear_f64(A, B, bias, C=C0), C0 + oracle.linear_f64(A, B, bias))
