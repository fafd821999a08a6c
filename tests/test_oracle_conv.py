"""Pins for the oracle's conv2d (paper Sec. 4.1, listing "2dnchwconv"), generalised
to stride and symmetric zero padding.

Independent routes: im2col followed by numpy's product, scipy's 2-D
correlation for single-channel slices, closed forms (all-ones, delta filter),
the 1x1 case as a plain matrix product, and the output-size formula.
"""
import numpy as np
import pytest
from scipy import signal

from workloads import conv_inputs

CASES = [
    # N, C, H, W, F, KH, KW, stride, pad
    (1, 1, 5, 5, 1, 3, 3, 1, 0),
    (1, 3, 7, 6, 2, 3, 3, 1, 1),
    (2, 3, 9, 9, 4, 3, 3, 2, 1),
    (1, 4, 8, 8, 3, 1, 1, 2, 0),
    (2, 2, 6, 7, 3, 2, 3, 1, 0),
    (1, 5, 11, 11, 2, 5, 5, 3, 2),
    (3, 2, 4, 4, 2, 3, 3, 1, 2),
]


def _conv_via_im2col(orc, x, w, s, p):
    N, C, H, W = x.shape
    F, _, KH, KW = w.shape
    col = orc.im2col_f64(x, KH, KW, (s, s), (p, p))
    HO = (H + 2 * p - KH) // s + 1
    WO = (W + 2 * p - KW) // s + 1
    y = w.reshape(F, -1).astype(np.float64) @ col        # F x (N*HO*WO)
    return y.reshape(F, N, HO, WO).transpose(1, 0, 2, 3)


@pytest.mark.parametrize("case", CASES)
def test_conv_equals_im2col_matmul(orc, case):
    N, C, H, W, F, KH, KW, s, p = case
    x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case))
    got = orc.conv2d_f64(x, w, (s, s), (p, p))
    np.testing.assert_allclose(got, _conv_via_im2col(orc, x, w, s, p), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_conv_matches_scipy_correlate(orc, case):
    # scipy.signal.correlate2d on the zero-padded image, summed over channels,
    # then subsampled by the stride.
    N, C, H, W, F, KH, KW, s, p = case
    x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case) + 1)
    got = orc.conv2d_f64(x, w, (s, s), (p, p))
    for n in range(N):
        for f in range(F):
            acc = 0.0
            for c in range(C):
                xp = np.pad(x[n, c].astype(np.float64), p)
                acc = acc + signal.correlate2d(xp, w[f, c].astype(np.float64), mode="valid")
            np.testing.assert_allclose(got[n, f], acc[::s, ::s], rtol=1e-12, atol=1e-12)


def test_paper_listing_unpadded_indexing(orc):
    # The listing's own indexing: output[n,co,ho,wo] += input[n,ci,ho+ki,wo+kj] * kernel[co,ci,ki,kj]
    x, w = conv_inputs(1, 2, 6, 5, 3, 3, 3, seed=42)
    got = orc.conv2d_f64(x, w)
    HO, WO = 4, 3
    want = np.zeros((1, 3, HO, WO))
    for co in range(3):
        for ho in range(HO):
            for wo in range(WO):
                for ci in range(2):
                    for ki in range(3):
                        for kj in range(3):
                            want[0, co, ho, wo] += float(x[0, ci, ho + ki, wo + kj]) * float(w[co, ci, ki, kj])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_one_by_one_is_matmul(orc):
    x, w = conv_inputs(2, 6, 5, 4, 3, 1, 1, seed=8)
    got = orc.conv2d_f64(x, w)
    for n in range(2):
        want = w[:, :, 0, 0].astype(np.float64) @ x[n].reshape(6, -1).astype(np.float64)
        np.testing.assert_allclose(got[n].reshape(3, -1), want, rtol=1e-13, atol=1e-13)


def test_delta_filter_copies(orc):
    x, _ = conv_inputs(1, 3, 6, 6, 3, 3, 3, seed=1)
    w = np.zeros((3, 3, 3, 3), np.float32)
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    assert np.array_equal(orc.conv2d_f64(x, w, (1, 1), (1, 1)), x.astype(np.float64))


def test_all_ones_closed_form(orc):
    # 3x3, pad 1, stride 1: interior 9C, edge 6C, corner 4C
    C = 5
    x, w = conv_inputs(1, C, 6, 7, 2, 3, 3, dist="ones")
    y = orc.conv2d_f64(x, w, (1, 1), (1, 1))[0, 0]
    assert y[2, 3] == 9 * C
    assert y[0, 3] == 6 * C and y[5, 3] == 6 * C and y[2, 0] == 6 * C and y[2, 6] == 6 * C
    assert y[0, 0] == 4 * C and y[5, 6] == 4 * C and y[0, 6] == 4 * C and y[5, 0] == 4 * C


@pytest.mark.parametrize("h,k,s,p,ho", [(56, 3, 2, 1, 28), (28, 3, 2, 1, 14), (14, 3, 2, 1, 7),
                                         (56, 1, 2, 0, 28), (1280, 3, 1, 0, 1278), (56, 3, 1, 1, 56),
                                         (2, 3, 1, 0, 0)])
def test_output_size(orc, h, k, s, p, ho):
    assert orc.conv_out_size(h, k, s, p) == ho


def test_accumulates_into_output(orc):
    x, w = conv_inputs(1, 2, 5, 5, 2, 3, 3, seed=3, dist="small_int")
    y0 = np.full((1, 2, 5, 5), 100.0)
    assert np.array_equal(orc.conv2d_f64(x, w, (1, 1), (1, 1), y=y0) - 100.0,
                          orc.conv2d_f64(x, w, (1, 1), (1, 1)))


def test_conv_threads_and_f32(orc):
    x, w = conv_inputs(2, 4, 9, 9, 3, 3, 3, seed=5, dist="small_int")
    r1 = orc.conv2d_f64(x, w, (2, 2), (1, 1), threads=1)
    r3 = orc.conv2d_f64(x, w, (2, 2), (1, 1), threads=3)
    assert np.array_equal(r1, r3)
    # small integers: every float partial sum is exact
    assert np.array_equal(orc.conv2d_f32(x, w, (2, 2), (1, 1)).astype(np.float64), r1)
