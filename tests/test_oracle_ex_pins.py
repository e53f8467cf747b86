"""Pins of the oracle's extended interface, Y <- alpha * K(op(A), op(B)[,
op(C)]) X + beta * Y (Section 3's batched interface, op in {N, T}), against
brute force that forms the Kronecker matrix of the explicitly transposed
factors with numpy: every op combination, alpha and beta applied as the
update they define, and beta = 0 leaving a NaN-filled Y unread."""
import itertools

import numpy as np
import pytest

import oracle


def _mat(flat, n):
    """Column-major flat n x n -> numpy matrix M[i, j] = flat[i + n*j]."""
    return np.asarray(flat, np.float64).reshape(n, n).T


def _op(M, op):
    return M.T if op == "T" else M


def _brute2d(n, opA, opB, A, B, X, batch):
    K = np.kron(_op(_mat(A, n), opA), _op(_mat(B, n), opB))
    return (X.reshape(batch, n * n) @ K.T).reshape(-1)


def _brute3d(n, opA, opB, opC, A, B, C, X, batch):
    K = np.kron(_op(_mat(A, n), opA), np.kron(_op(_mat(B, n), opB), _op(_mat(C, n), opC)))
    return (X.reshape(batch, n ** 3) @ K.T).reshape(-1)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=2)))
def test_ex2d_matches_brute_force(n, ops):
    rng = np.random.default_rng(100 + n)
    batch = 7
    A, B = rng.uniform(-1, 1, n * n), rng.uniform(-1, 1, n * n)
    X = rng.standard_normal(batch * n * n)
    Y0 = rng.standard_normal(batch * n * n)
    for alpha, beta in ((1.0, 0.0), (-0.75, 0.0), (0.5, 2.0), (0.0, -1.5)):
        got = oracle.kron2d_ex(n, ops[0], ops[1], alpha, A, B, X, beta, Y0, batch)
        want = alpha * _brute2d(n, ops[0], ops[1], A, B, X, batch) + beta * Y0
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=3)))
def test_ex3d_matches_brute_force(n, ops):
    rng = np.random.default_rng(200 + n)
    batch = 5
    A, B, C = (rng.uniform(-1, 1, n * n) for _ in range(3))
    X = rng.standard_normal(batch * n ** 3)
    Y0 = rng.standard_normal(batch * n ** 3)
    for alpha, beta in ((1.0, 0.0), (2.5, 0.0), (-1.0, 0.25)):
        got = oracle.kron3d_ex(n, *ops, alpha, A, B, C, X, beta, Y0, batch)
        want = alpha * _brute3d(n, *ops, A, B, C, X, batch) + beta * Y0
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 4])
@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=2)))
def test_ex2d_op_x_matches_brute_force(n, ops):
    """op(X_p) = X_p^T in 2-D (Section 2.2): brute force on explicitly
    transposed operands; op(X) = N is the plain extended call."""
    rng = np.random.default_rng(300 + n)
    batch = 6
    A, B = rng.uniform(-1, 1, n * n), rng.uniform(-1, 1, n * n)
    X = rng.standard_normal(batch * n * n)
    Y0 = rng.standard_normal(batch * n * n)
    Xt = X.reshape(batch, n, n).transpose(0, 2, 1).reshape(-1)
    for alpha, beta in ((1.0, 0.0), (-2.0, 0.5)):
        got = oracle.kron2d_ex(n, ops[0], ops[1], alpha, A, B, X, beta, Y0, batch, opX="T")
        want = alpha * _brute2d(n, ops[0], ops[1], A, B, Xt, batch) + beta * Y0
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)
        plain = oracle.kron2d_ex(n, ops[0], ops[1], alpha, A, B, X, beta, Y0, batch, opX="N")
        np.testing.assert_allclose(plain, oracle.kron2d_ex(n, ops[0], ops[1], alpha, A, B, X, beta, Y0, batch),
                                   rtol=0, atol=0)
    if n > 1:
        # the transposed operand differs from the plain one
        assert not np.allclose(oracle.kron2d_ex(n, "N", "N", 1.0, A, B, X, 0.0, Y0, batch, opX="T"),
                               oracle.kron2d_ex(n, "N", "N", 1.0, A, B, X, 0.0, Y0, batch))


def test_ex_beta_zero_does_not_read_y():
    rng = np.random.default_rng(7)
    n, batch = 4, 3
    A, B, C = (rng.uniform(-1, 1, n * n) for _ in range(3))
    X = rng.standard_normal(batch * n ** 3)
    nan = np.full(batch * n ** 3, np.nan)
    got = oracle.kron3d_ex(n, "T", "N", "T", 1.5, A, B, C, X, 0.0, nan, batch)
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, 1.5 * _brute3d(n, "T", "N", "T", A, B, C, X, batch), rtol=1e-13, atol=1e-13)


def test_ex_all_n_with_identity_ops_equal_plain_action():
    """op = N, alpha = 1, beta = 0 is the plain action (both sides computed
    here from the brute force, so this also pins the plain oracle)."""
    rng = np.random.default_rng(9)
    for n in (4, 6):
        A, B = rng.uniform(-1, 1, n * n), rng.uniform(-1, 1, n * n)
        X = rng.standard_normal(3 * n * n)
        got = oracle.kron2d_ex(n, "N", "N", 1.0, A, B, X, 0.0, np.zeros(3 * n * n), 3)
        np.testing.assert_allclose(got, _brute2d(n, "N", "N", A, B, X, 3), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(oracle.kron2d(n, A, B, X, 3), got, rtol=1e-13, atol=1e-13)
