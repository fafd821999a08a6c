"""Pins for the oracle's matmul (paper Sec. 1 listing "nelli_for_to_affine_for",
Sec. 2.1 listing "linalg-matmul": C[M,N] += A[M,K] B[K,N]).

Each check is fixed by something other than the oracle itself: numpy's float64
/ int64 products (a library routine), closed forms, or exact integer
arithmetic.  A dropped term, a transposed operand, a wrong index or an
overwrite instead of an accumulate fails at least one of them.
"""
import numpy as np
import pytest

from workloads import matmul_inputs, random_c

SHAPES = [
    (1, 1, 1),
    (4, 8, 16),    # the affine listing's 4 x 16 x 8 matmul, in C[M,N] += A[M,K] B[K,N] naming
    (32, 32, 32),  # the Linear(32, 32) nest of listing "listing1"
    (7, 13, 31),
    (31, 7, 13),
    (33, 65, 17),
    (5, 1, 9),
    (1, 9, 5),
]


@pytest.mark.parametrize("M,N,K", SHAPES)
def test_f64_matches_numpy(orc, M, N, K):
    A, B = matmul_inputs(M, N, K, seed=M * 100 + N * 10 + K)
    C0 = random_c(M, N, seed=K)
    got = orc.matmul_f64(A, B, C0)
    want = C0.astype(np.float64) + A.astype(np.float64) @ B.astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_f64_threads_do_not_change_result(orc):
    A, B = matmul_inputs(37, 29, 53, seed=3, dist="normal")
    r1 = orc.matmul_f64(A, B, threads=1)
    r4 = orc.matmul_f64(A, B, threads=4)
    assert np.array_equal(r1, r4)


def test_f64_is_not_transposed(orc):
    # A non-square, non-symmetric case where A^T-style index slips change the answer.
    A = np.arange(6, dtype=np.float32).reshape(2, 3)
    B = np.arange(12, dtype=np.float32).reshape(3, 4)
    want = np.array([[20, 23, 26, 29], [56, 68, 80, 92]], np.float64)
    assert np.array_equal(orc.matmul_f64(A, B), want)


@pytest.mark.parametrize("K", [1, 7, 128, 1000])
def test_all_ones_gives_K(orc, K):
    A, B = matmul_inputs(5, 6, K, dist="ones")
    assert np.all(orc.matmul_f64(A, B) == K)
    assert np.all(orc.matmul_f32(A, B) == K)


def test_identity(orc):
    A, _ = matmul_inputs(9, 9, 9, seed=5)
    eye = np.eye(9, dtype=np.float32)
    assert np.array_equal(orc.matmul_f64(A, eye), A.astype(np.float64))
    assert np.array_equal(orc.matmul_f64(eye, A), A.astype(np.float64))


def test_rank1_ramp(orc):
    # A[i,k] = i, B[k,j] = j  =>  C[i,j] = K * i * j exactly
    M, N, K = 11, 13, 17
    A = np.repeat(np.arange(M, dtype=np.float32)[:, None], K, axis=1)
    B = np.repeat(np.arange(N, dtype=np.float32)[None, :], K, axis=0)
    i, j = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    assert np.array_equal(orc.matmul_f64(A, B), (K * i * j).astype(np.float64))


def test_accumulates_into_c(orc):
    A, B = matmul_inputs(6, 5, 4, seed=11, dist="small_int")
    C0 = np.full((6, 5), 1000.0, np.float32)
    assert np.array_equal(orc.matmul_f64(A, B, C0) - orc.matmul_f64(A, B), np.full((6, 5), 1000.0))
    assert np.array_equal(orc.matmul_f32(A, B, C0) - 1000.0, orc.matmul_f32(A, B))


def test_f32_faithful_is_sequential_rounding(orc):
    # The float mode rounds the product and then the sum, k ascending.  Brute
    # force the same recurrence with numpy float32 scalars on a tiny case.
    A, B = matmul_inputs(3, 4, 9, seed=2, dist="normal")
    got = orc.matmul_f32(A, B)
    for i in range(3):
        for j in range(4):
            c = np.float32(0.0)
            for k in range(9):
                c = np.float32(c + np.float32(A[i, k] * B[k, j]))
            assert got[i, j] == c


def test_f32_within_standard_bound(orc):
    # |fl(C) - C| <= gamma_K * sum_k |a_ik||b_kj|, gamma_K = K u / (1 - K u)
    M, N, K = 16, 16, 512
    A, B = matmul_inputs(M, N, K, seed=9, dist="normal")
    ref = orc.matmul_f64(A, B)
    got = orc.matmul_f32(A, B).astype(np.float64)
    u = 2.0 ** -24
    gamma = K * u / (1 - K * u)
    bound = gamma * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)))
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (4, 8, 16), (7, 13, 31), (64, 33, 129)])
def test_i8_matches_numpy_int64(orc, M, N, K):
    A, B = matmul_inputs(M, N, K, seed=K, dist="int8")
    C0 = random_c(M, N, seed=M, dtype=np.int32)
    got = orc.matmul_i8(A, B, C0)
    want = (C0.astype(np.int64) + A.astype(np.int64) @ B.astype(np.int64))
    assert got.dtype == np.int32
    assert np.array_equal(got.astype(np.int64), want)


def test_i8_extremes_and_wraparound(orc):
    # (-128)(-128) K times: K * 16384, exact for K = 1024 (2^24, no overflow).
    K = 1024
    A = np.full((2, K), -128, np.int8)
    B = np.full((K, 3), -128, np.int8)
    assert np.all(orc.matmul_i8(A, B) == K * 16384)
    # Starting near INT32_MAX the sum must wrap exactly like two's complement.
    C0 = np.full((2, 3), 2**31 - 1, np.int32)
    got = orc.matmul_i8(A[:, :1], B[:1, :], C0)
    want = ((2**31 - 1 + 16384 + 2**31) % 2**32) - 2**31
    assert np.all(got == want)
    # sign extension: -1 * 127 = -127
    a = np.array([[-1]], np.int8)
    b = np.array([[127]], np.int8)
    assert orc.matmul_i8(a, b)[0, 0] == -127


def test_i8_threads(orc):
    A, B = matmul_inputs(33, 17, 64, seed=4, dist="int8")
    assert np.array_equal(orc.matmul_i8(A, B, threads=1), orc.matmul_i8(A, B, threads=3))
