"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes an oracle object (``oracle.Oracle``) and raises
AssertionError when the oracle disagrees with a value that does not come from
the oracle's own arithmetic: a hand-derived worked example, an explicitly
formed Kronecker matrix (numpy.kron), an algebraic identity, a closed form, a
reduction to a numpy library routine, the triple summation of Section 2.1 as one
numpy einsum, or central finite differences.  The same functions are run against
deliberately altered builds of the oracle to show that they catch mistakes.

Conventions (shared with the oracle): matrices are column-major flat arrays;
2-D operands are column-major n x n blocks with Y_p = B X_p A^T; 3-D operands
hold element (a, b, c) at a*n^2 + b*n + c and vec(Y) = (A kron B kron C) vec(X).
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---- small helpers (no Kronecker arithmetic here) ---------------------------

def cm(M):
    """Math matrix -> column-major flat array."""
    return np.asarray(M).reshape(-1, order="F")


def mat(flat, n):
    """Column-major flat array -> math matrix."""
    return np.asarray(flat).reshape(n, n, order="F")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = np.array([float(v) for v in rest])
    return vals


def rand_mats(rng, n, k):
    return [rng.uniform(-1, 1, n * n) for _ in range(k)]


# ---- P0: hand-derived worked examples (golden fixtures) --------------------

def pin_worked_examples(orc):
    g = read_golden("worked_2d_n2.txt")
    n = int(g["n"][0])
    for prec in ("f64", "f32"):
        y = orc.kron2d(n, g["A"], g["B"], g["X"], 1, prec)
        assert np.array_equal(y.astype(np.float64), g["Y"]), ("worked 2-D", prec, y)
    g = read_golden("worked_3d_n2.txt")
    n = int(g["n"][0])
    for prec in ("f64", "f32"):
        y = orc.kron3d(n, g["A"], g["B"], g["C"], g["X"], 1, prec)
        assert np.array_equal(y.astype(np.float64), g["Y"]), ("worked 3-D", prec, y)


# ---- P1: brute force with the explicitly formed Kronecker matrix ------------

def pin_brute_force(orc, seed=1):
    rng = np.random.default_rng(seed)
    for n in range(1, 9):
        A, B = rand_mats(rng, n, 2)
        batch = 3
        X = rng.standard_normal(batch * n * n)
        K = np.kron(mat(A, n), mat(B, n))
        want = (X.reshape(batch, n * n) @ K.T).reshape(-1)
        got = orc.kron2d(n, A, B, X, batch, "f64")
        assert rel(got, want) < 1e-14, ("2-D brute force", n, rel(got, want))
        got32 = orc.kron2d(n, A, B, X, batch, "f32")
        assert rel(got32, want) < 2e-6, ("2-D brute force f32", n, rel(got32, want))
    for n in range(1, 6):
        A, B, C = rand_mats(rng, n, 3)
        batch = 2
        X = rng.standard_normal(batch * n ** 3)
        K = np.kron(mat(A, n), np.kron(mat(B, n), mat(C, n)))
        want = (X.reshape(batch, n ** 3) @ K.T).reshape(-1)
        got = orc.kron3d(n, A, B, C, X, batch, "f64")
        assert rel(got, want) < 1e-14, ("3-D brute force", n, rel(got, want))
        got32 = orc.kron3d(n, A, B, C, X, batch, "f32")
        assert rel(got32, want) < 3e-6, ("3-D brute force f32", n, rel(got32, want))


# ---- P2: identity factors reproduce X bit for bit ----------------------------

def pin_identity(orc, seed=2):
    rng = np.random.default_rng(seed)
    for n in (1, 3, 7, 16):
        I = cm(np.eye(n))
        X = rng.standard_normal(5 * n * n)
        for prec in ("f64", "f32"):
            y = orc.kron2d(n, I, I, X, 5, prec)
            assert np.array_equal(y, X.astype(y.dtype)), ("identity 2-D", n, prec)
        X3 = rng.standard_normal(2 * n ** 3)
        for prec in ("f64", "f32"):
            y = orc.kron3d(n, I, I, I, X3, 2, prec)
            assert np.array_equal(y, X3.astype(y.dtype)), ("identity 3-D", n, prec)


# ---- P3: permutation factors move entries exactly ----------------------------

def perm_cm(n, perm):
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    return cm(P)


def pin_permutation(orc, seed=3):
    """With P[i, perm[i]] = 1 the action is a pure gather, computed here with
    numpy indexing: 2-D Y[p, i, j] = X[p, pa[i], pb[j]] in the (slow, fast)
    memory view; 3-D Y[p, i, j, k] = X[p, pa[i], pb[j], pc[k]]."""
    rng = np.random.default_rng(seed)
    for n in (2, 5, 8, 13, 16):
        pa, pb, pc = (rng.permutation(n) for _ in range(3))
        batch = 3
        X = np.arange(batch * n * n, dtype=np.float64) + 1.0
        want = X.reshape(batch, n, n)[:, pa][:, :, pb].reshape(-1)
        for prec in ("f64", "f32"):
            y = orc.kron2d(n, perm_cm(n, pa), perm_cm(n, pb), X, batch, prec)
            assert np.array_equal(y.astype(np.float64), want), ("perm 2-D", n, prec)
        X3 = np.arange(batch * n ** 3, dtype=np.float64) + 1.0
        want3 = X3.reshape(batch, n, n, n)[:, pa][:, :, pb][:, :, :, pc].reshape(-1)
        for prec in ("f64", "f32"):
            y = orc.kron3d(n, perm_cm(n, pa), perm_cm(n, pb), perm_cm(n, pc), X3, batch, prec)
            assert np.array_equal(y.astype(np.float64), want3), ("perm 3-D", n, prec)


# ---- P4: small integers, where every partial sum is exact -------------------

def pin_small_integers(orc, seed=4):
    """Entries of A, B, C in {-2..2} and of X in {-8..8}: every partial sum is an
    integer below 2^24, so float and double results must both equal the exact
    integer result of the explicitly formed (integer) Kronecker matrix."""
    rng = np.random.default_rng(seed)
    for n in (3, 8, 16):
        A, B, C = (rng.integers(-2, 3, n * n) for _ in range(3))
        batch = 2
        X = rng.integers(-8, 9, batch * n * n)
        K = np.kron(mat(A, n), mat(B, n)).astype(np.int64)
        want = (X.reshape(batch, -1).astype(np.int64) @ K.T).reshape(-1)
        for prec in ("f64", "f32"):
            y = orc.kron2d(n, A, B, X, batch, prec)
            assert np.array_equal(y.astype(np.int64), want) and np.all(y == want), ("ints 2-D", n, prec)
        if n <= 8:
            X3 = rng.integers(-8, 9, batch * n ** 3)
            K3 = np.kron(mat(A, n), np.kron(mat(B, n), mat(C, n))).astype(np.int64)
            want3 = (X3.reshape(batch, -1).astype(np.int64) @ K3.T).reshape(-1)
            for prec in ("f64", "f32"):
                y = orc.kron3d(n, A, B, C, X3, batch, prec)
                assert np.all(y == want3), ("ints 3-D", n, prec)


# ---- P5: mixed-product rule -------------------------------------------------

def pin_mixed_product(orc, seed=5):
    """(A1 kron B1)(A2 kron B2) = (A1 A2) kron (B1 B2): applying two actions in
    a row equals one action with the products of the factors."""
    rng = np.random.default_rng(seed)
    for n in (4, 11, 16):
        A1, B1, C1, A2, B2, C2 = rand_mats(rng, n, 6)
        M = lambda P, Q: cm(mat(P, n) @ mat(Q, n))
        X = rng.standard_normal(4 * n * n)
        two = orc.kron2d(n, A1, B1, orc.kron2d(n, A2, B2, X, 4), 4)
        one = orc.kron2d(n, M(A1, A2), M(B1, B2), X, 4)
        assert rel(two, one) < 1e-13, ("mixed product 2-D", n)
        X3 = rng.standard_normal(2 * n ** 3)
        two = orc.kron3d(n, A1, B1, C1, orc.kron3d(n, A2, B2, C2, X3, 2), 2)
        one = orc.kron3d(n, M(A1, A2), M(B1, B2), M(C1, C2), X3, 2)
        assert rel(two, one) < 1e-13, ("mixed product 3-D", n)


# ---- P6: adjoint identity --------------------------------------------------

def pin_adjoint(orc, seed=6):
    """<K(A,B) X, Z> = <X, K(A^T, B^T) Z>, since (A kron B)^T = A^T kron B^T."""
    rng = np.random.default_rng(seed)
    T = lambda P, n: cm(mat(P, n).T)
    for n in (3, 10, 16):
        A, B, C = rand_mats(rng, n, 3)
        X, Z = rng.standard_normal(3 * n * n), rng.standard_normal(3 * n * n)
        lhs = np.dot(orc.kron2d(n, A, B, X, 3), Z)
        rhs = np.dot(X, orc.kron2d(n, T(A, n), T(B, n), Z, 3))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1), ("adjoint 2-D", n)
        X, Z = rng.standard_normal(2 * n ** 3), rng.standard_normal(2 * n ** 3)
        lhs = np.dot(orc.kron3d(n, A, B, C, X, 2), Z)
        rhs = np.dot(X, orc.kron3d(n, T(A, n), T(B, n), T(C, n), Z, 2))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1), ("adjoint 3-D", n)


# ---- P7: one non-identity factor reduces to a plain matrix product ----------

def pin_single_factor(orc, seed=7):
    rng = np.random.default_rng(seed)
    for n in (2, 9, 16):
        I = cm(np.eye(n))
        M = rng.uniform(-1, 1, n * n)
        Mm = mat(M, n)
        batch = 4
        X = rng.standard_normal(batch * n * n)
        Xm = X.reshape(batch, n, n).transpose(0, 2, 1)   # column-major operands
        # K(I, B) X = B X  and  K(A, I) X = X A^T
        got = orc.kron2d(n, I, M, X, batch).reshape(batch, n, n).transpose(0, 2, 1)
        assert rel(got, np.matmul(Mm, Xm)) < 1e-14, ("B only", n)
        got = orc.kron2d(n, M, I, X, batch).reshape(batch, n, n).transpose(0, 2, 1)
        assert rel(got, np.matmul(Xm, Mm.T)) < 1e-14, ("A only", n)
        X3 = rng.standard_normal(2 * n ** 3).reshape(2, n, n, n)
        # each factor alone acts along its own memory axis (A slowest, C fastest)
        got = orc.kron3d(n, M, I, I, X3, 2).reshape(2, n, n, n)
        assert rel(got, np.einsum("ia,pabc->pibc", Mm, X3)) < 1e-14, ("A only 3-D", n)
        got = orc.kron3d(n, I, M, I, X3, 2).reshape(2, n, n, n)
        assert rel(got, np.einsum("jb,pabc->pajc", Mm, X3)) < 1e-14, ("B only 3-D", n)
        got = orc.kron3d(n, I, I, M, X3, 2).reshape(2, n, n, n)
        assert rel(got, np.matmul(X3, Mm.T)) < 1e-14, ("C only 3-D", n)


# ---- P8: rank-one operands have a closed form ------------------------------

def pin_rank_one(orc, seed=8):
    """X = u kron v (kron w) in memory order maps to (A u) kron (B v) (kron (C w))."""
    rng = np.random.default_rng(seed)
    for n in (1, 6, 16):
        A, B, C = rand_mats(rng, n, 3)
        u, v, w = (rng.standard_normal(n) for _ in range(3))
        X = np.kron(u, v)
        want = np.kron(mat(A, n) @ u, mat(B, n) @ v)
        assert rel(orc.kron2d(n, A, B, X, 1), want) < 1e-14, ("rank-1 2-D", n)
        X3 = np.kron(u, np.kron(v, w))
        want3 = np.kron(mat(A, n) @ u, np.kron(mat(B, n) @ v, mat(C, n) @ w))
        assert rel(orc.kron3d(n, A, B, C, X3, 1), want3) < 1e-14, ("rank-1 3-D", n)


# ---- P9: the triple summation of Section 2.1 as one contraction -------------

def triple_sum(P, Q, R, X):
    """Section 2.1's triple summation Y_ijk = sum_{l,m,n} P_il Q_jm R_kn X_lmn on
    one array X indexed (l, m, n), written as a single einsum: no mode order,
    no intermediate array."""
    return np.einsum("il,jm,kn,lmn->ijk", P, Q, R, X)


def pin_triple_sum(orc, seed=9):
    rng = np.random.default_rng(seed)
    for n in (2, 5, 10, 16):
        A, B, C = rand_mats(rng, n, 3)
        Xflat = rng.standard_normal(n ** 3)
        # memory index a*n^2 + b*n + c: the library's A acts on a, C on c
        Xt = Xflat.reshape(n, n, n)
        want = triple_sum(mat(A, n), mat(B, n), mat(C, n), Xt).reshape(-1)
        got = orc.kron3d(n, A, B, C, Xflat, 1)
        assert rel(got, want) < 1e-14, ("triple summation", n, rel(got, want))


# ---- P10: linearity ---------------------------------------------------------

def pin_linearity(orc, seed=10):
    rng = np.random.default_rng(seed)
    n = 7
    A, B, C, A2 = rand_mats(rng, n, 4)
    X1, X2 = rng.standard_normal(2 * n ** 3), rng.standard_normal(2 * n ** 3)
    a, b = 0.75, -2.5
    lhs = orc.kron3d(n, A, B, C, a * X1 + b * X2, 2)
    rhs = a * orc.kron3d(n, A, B, C, X1, 2) + b * orc.kron3d(n, A, B, C, X2, 2)
    assert rel(lhs, rhs) < 1e-14, "linearity in X"
    lhs = orc.kron3d(n, A + A2, B, C, X1, 2)
    rhs = orc.kron3d(n, A, B, C, X1, 2) + orc.kron3d(n, A2, B, C, X1, 2)
    assert rel(lhs, rhs) < 1e-14, "linearity in A"
    lhs = orc.kron2d(n, A, 3.0 * B, X1[: 2 * n * n], 2)
    rhs = 3.0 * orc.kron2d(n, A, B, X1[: 2 * n * n], 2)
    assert rel(lhs, rhs) < 1e-14, "scaling in B"


# ---- P11: batch independence ------------------------------------------------

def pin_batch_independence(orc, seed=11):
    rng = np.random.default_rng(seed)
    for n in (4, 16):
        A, B, C = rand_mats(rng, n, 3)
        batch, q = 6, 3
        X = rng.standard_normal(batch * n * n)
        X[q * n * n + 5] = np.nan
        Y = orc.kron2d(n, A, B, X, batch).reshape(batch, -1)
        for p in range(batch):
            assert np.all(np.isnan(Y[p])) if p == q else np.all(np.isfinite(Y[p])), ("NaN 2-D", n, p)
        # each operand alone gives the same result as in the batch
        single = orc.kron2d(n, A, B, X[: n * n], 1)
        assert np.array_equal(single, Y[0]), ("batch 2-D", n)
        X3 = rng.standard_normal(batch * n ** 3)
        X3[q * n ** 3 + 7] = np.nan
        Y3 = orc.kron3d(n, A, B, C, X3, batch).reshape(batch, -1)
        for p in range(batch):
            assert np.any(np.isnan(Y3[p])) if p == q else np.all(np.isfinite(Y3[p])), ("NaN 3-D", n, p)
        single = orc.kron3d(n, A, B, C, X3[(batch - 1) * n ** 3:], 1)
        assert np.array_equal(single, Y3[batch - 1]), ("batch 3-D", n)


# ---- P12: gradients against central differences and the explicit matrix ----

def _fd(f, x, h):
    g = np.empty(x.size)
    for i in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


def pin_gradients(orc, seed=12):
    """L = sum_p <dY_p, Y_p> is linear in X and in each factor, so a central
    difference with h = 1e-3 has no truncation error; dX is also checked
    against the transposed explicit Kronecker matrix."""
    rng = np.random.default_rng(seed)
    h = 1e-3
    for n in (1, 3, 5):
        batch = 3
        A, B = rand_mats(rng, n, 2)
        X, dY = rng.standard_normal(batch * n * n), rng.standard_normal(batch * n * n)
        dX, dA, dB = orc.kron2d_grad(n, A, B, X, dY, batch)
        K = np.kron(mat(A, n), mat(B, n))
        assert rel(dX, (dY.reshape(batch, -1) @ K).reshape(-1)) < 1e-13, ("dX 2-D", n)
        L = lambda A_, B_, X_: float(np.dot(dY, orc.kron2d(n, A_, B_, X_, batch)))
        assert rel(dA, _fd(lambda a: L(a, B, X), A, h)) < 1e-8, ("dA 2-D", n)
        assert rel(dB, _fd(lambda b: L(A, b, X), B, h)) < 1e-8, ("dB 2-D", n)
    for n in (1, 2, 4):
        batch = 2
        A, B, C = rand_mats(rng, n, 3)
        X, dY = rng.standard_normal(batch * n ** 3), rng.standard_normal(batch * n ** 3)
        dX, dA, dB, dC = orc.kron3d_grad(n, A, B, C, X, dY, batch)
        K = np.kron(mat(A, n), np.kron(mat(B, n), mat(C, n)))
        assert rel(dX, (dY.reshape(batch, -1) @ K).reshape(-1)) < 1e-13, ("dX 3-D", n)
        L = lambda A_, B_, C_: float(np.dot(dY, orc.kron3d(n, A_, B_, C_, X, batch)))
        assert rel(dA, _fd(lambda a: L(a, B, C), A, h)) < 1e-8, ("dA 3-D", n)
        assert rel(dB, _fd(lambda b: L(A, b, C), B, h)) < 1e-8, ("dB 3-D", n)
        assert rel(dC, _fd(lambda c: L(A, B, c), C, h)) < 1e-8, ("dC 3-D", n)


# ---- FP32 variant tracks FP64 at float accuracy ----------------------------

def pin_float_accuracy(orc, seed=13):
    rng = np.random.default_rng(seed)
    for n in (10, 16):
        A, B, C = rand_mats(rng, n, 3)
        X = rng.standard_normal(8 * n * n)
        e = rel(orc.kron2d(n, A, B, X, 8, "f32"), orc.kron2d(n, A, B, X, 8, "f64"))
        assert 0 < e < 1e-6, ("f32 2-D accuracy", n, e)
        X3 = rng.standard_normal(2 * n ** 3)
        e = rel(orc.kron3d(n, A, B, C, X3, 2, "f32"), orc.kron3d(n, A, B, C, X3, 2, "f64"))
        assert 0 < e < 1e-6, ("f32 3-D accuracy", n, e)


def pin_extended_interface(orc, seed=14):
    """Y <- alpha * K(op(A), op(B)[, op(C)]) X + beta * Y against brute force
    with the explicitly transposed factors (Section 3's interface), for every
    op combination, and in 2-D with op on the operands as well; beta = 0 must
    not read a NaN-filled Y."""
    import itertools
    rng = np.random.default_rng(seed)
    for n, batch in ((3, 4), (2, 3)):
        A, B, C = rand_mats(rng, n, 3)
        opm = lambda M, o: mat(M, n).T if o == "T" else mat(M, n)
        X2 = rng.standard_normal(batch * n * n)
        Y2 = rng.standard_normal(batch * n * n)
        for ops in itertools.product("NT", repeat=2):
            K = np.kron(opm(A, ops[0]), opm(B, ops[1]))
            base = (X2.reshape(batch, n * n) @ K.T).reshape(-1)
            for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
                got = orc.kron2d_ex(n, ops[0], ops[1], alpha, A, B, X2, beta, Y2, batch)
                assert rel(got, alpha * base + beta * Y2) < 1e-13, ("2d", ops, alpha, beta)
        X3 = rng.standard_normal(batch * n ** 3)
        Y3 = rng.standard_normal(batch * n ** 3)
        for ops in itertools.product("NT", repeat=3):
            K = np.kron(opm(A, ops[0]), np.kron(opm(B, ops[1]), opm(C, ops[2])))
            base = (X3.reshape(batch, n ** 3) @ K.T).reshape(-1)
            for alpha, beta in ((1.0, 0.0), (1.5, -0.25)):
                got = orc.kron3d_ex(n, *ops, alpha, A, B, C, X3, beta, Y3, batch)
                assert rel(got, alpha * base + beta * Y3) < 1e-13, ("3d", ops, alpha, beta)
        got = orc.kron3d_ex(n, "T", "N", "T", 2.0, A, B, C, X3, 0.0, np.full(batch * n ** 3, np.nan), batch)
        assert np.all(np.isfinite(got)), "beta = 0 read Y"
        # 2-D op on the operands: each X_p transposed explicitly (numpy index
        # [p, m, l] holds X_p(l, m) of the column-major operand)
        X2t = X2.reshape(batch, n, n).transpose(0, 2, 1).reshape(-1)
        for ops in itertools.product("NT", repeat=2):
            K = np.kron(opm(A, ops[0]), opm(B, ops[1]))
            base = (X2t.reshape(batch, n * n) @ K.T).reshape(-1)
            got = orc.kron2d_ex(n, ops[0], ops[1], 0.75, A, B, X2, -1.0, Y2, batch, opX="T")
            assert rel(got, 0.75 * base - Y2) < 1e-13, ("2d opX", ops)


def pin_tkron1(orc, seed=15):
    """1-D (Section 3's TKRON1): y_p = alpha op(A) x_p + beta y_p against a
    numpy matrix product on the explicitly transposed matrix, with padded
    strides (the gaps keep their values); and, with op = N, alpha = 1,
    beta = 0, against the 2-D action with an identity first factor on
    operands made of n consecutive vectors (Y_q = A X_q I^T)."""
    rng = np.random.default_rng(seed)
    for n, batch in ((1, 5), (3, 7), (4, 8)):
        A = rng.uniform(-1, 1, n * n)
        for op in "NT":
            Aop = mat(A, n).T if op == "T" else mat(A, n)
            ldxp, ldyp = n + 2, n + 1
            X = rng.standard_normal(ldxp * batch)
            Y = rng.standard_normal(ldyp * batch)
            got = orc.kron1d_ex(n, op, -1.5, A, X, 0.5, Y, batch, ldxp, ldyp)
            want = Y.copy()
            for p in range(batch):
                want[p * ldyp:p * ldyp + n] = -1.5 * Aop @ X[p * ldxp:p * ldxp + n] + 0.5 * Y[p * ldyp:p * ldyp + n]
            assert rel(got, want) < 1e-13, ("tkron1", n, op)
        # n vectors at a time form one 2-D operand whose columns they are
        Xd = rng.standard_normal(n * n * batch)
        got = orc.kron1d_ex(n, "N", 1.0, A, Xd, 0.0, np.full(Xd.size, np.nan), n * batch)
        ident = np.eye(n).reshape(-1)
        assert rel(got, orc.kron2d(n, ident, A, Xd, batch)) < 1e-13, ("tkron1 vs 2-D", n)


ALL_PINS = [
    pin_worked_examples, pin_brute_force, pin_identity, pin_permutation,
    pin_small_integers, pin_mixed_product, pin_adjoint, pin_single_factor,
    pin_rank_one, pin_triple_sum, pin_linearity, pin_batch_independence,
    pin_gradients, pin_float_accuracy, pin_extended_interface, pin_tkron1,
]


# ---- the general action: d dimensions, rectangular, complex, per operand ----

def _read_nd_golden():
    vals = {}
    with open(os.path.join(GOLDEN, "worked_nd.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            if key.endswith("_ops"):
                vals[key] = rest[0]
            elif key.endswith(("_m", "_n")):
                vals[key] = [int(v) for v in rest]
            else:
                vals[key] = np.array([complex(*map(float, v.split(","))) if "," in v else float(v) for v in rest])
    return vals


def pin_nd_worked_examples(orc):
    g = _read_nd_golden()
    for tag in ("c", "r"):
        m, n, ops = g[tag + "_m"], g[tag + "_n"], g[tag + "_ops"]
        fs = [g[f"{tag}_F{k}"] for k in range(len(m))]
        ldf = [m[k] if ops[k] == "N" else n[k] for k in range(len(m))]
        Y = orc.kron_nd(m, n, ops, 1.0, fs, g[tag + "_X"], 0.0, np.zeros(int(np.prod(m))), 1, ldf=ldf)
        assert np.allclose(Y, g[tag + "_Y"], rtol=0, atol=1e-14), (tag, Y)


def _opm(S, op):
    """op(S) of a math matrix: 'N' S, 'T' S^T, 'C' S^* (conjugate transpose)."""
    return S if op == "N" else (S.T if op == "T" else S.conj().T)


def _nd_random_case(rng, d, cplx, varying, batch):
    m = [int(v) for v in rng.integers(1, 5, d)]
    n = [int(v) for v in rng.integers(1, 5, d)]
    ops = "".join(rng.choice(list("NTC" if cplx else "NT"), d))
    ldf, ldfp, fs, mats = [], [], [], []
    for k in range(d):
        rows, cols = (m[k], n[k]) if ops[k] == "N" else (n[k], m[k])
        ld = rows + int(rng.integers(0, 3))
        stride = ld * cols + int(rng.integers(0, 4)) if varying else 0
        count = batch if varying else 1
        size = (count - 1) * stride + ld * cols
        flat = rng.uniform(-1, 1, size) + (1j * rng.uniform(-1, 1, size) if cplx else 0)
        per = []
        for p in range(count):
            blk = flat[p * stride:p * stride + ld * cols].reshape(cols, ld).T[:rows]   # column-major, ld rows
            per.append(_opm(blk, ops[k]))
        ldf.append(ld)
        ldfp.append(stride)
        fs.append(flat)
        mats.append(per)
    X = rng.standard_normal(batch * int(np.prod(n))) + (1j * rng.standard_normal(batch * int(np.prod(n))) if cplx else 0)
    return m, n, ops, fs, ldf, ldfp, mats, X


def pin_nd_brute_force(orc, seed=16):
    """Explicit Kronecker matrices (numpy.kron of op(F_k), per operand when the
    factors vary) on memory-order vectors, with alpha, beta and padded
    leading dimensions: d = 1..4, rectangular, real and complex."""
    rng = np.random.default_rng(seed)
    for trial in range(24):
        d = 1 + trial % 4
        cplx = bool(trial % 2)
        varying = trial % 3 == 0
        batch = 3
        m, n, ops, fs, ldf, ldfp, mats, X = _nd_random_case(rng, d, cplx, varying, batch)
        ny = int(np.prod(m))
        alpha = 1.5 - 0.5j if cplx else -0.75
        beta = (0.25 + 1j if cplx else 2.0) if trial % 4 == 1 else 0.0
        Y0 = rng.standard_normal(batch * ny) + (1j * rng.standard_normal(batch * ny) if cplx else 0)
        got = orc.kron_nd(m, n, ops, alpha, fs, X, beta, Y0, batch, ldf=ldf, ldfp=ldfp)
        nx = int(np.prod(n))
        for p in range(batch):
            K = np.ones((1, 1))
            for k in range(d):
                K = np.kron(K, mats[k][p if varying else 0])
            want = alpha * (K @ X[p * nx:(p + 1) * nx]) + beta * Y0[p * ny:(p + 1) * ny]
            assert np.allclose(got[p * ny:(p + 1) * ny], want, rtol=1e-13, atol=1e-13), (trial, p)


def pin_nd_adjoint(orc, seed=17):
    """<K(op(F)) X, Z> = <X, K(op'(F)) Z> with op' the conjugate transpose of op
    ('N' <-> 'C' on the same stored matrices; complex inner product)."""
    rng = np.random.default_rng(seed)
    flip = {"N": "C", "C": "N"}
    for d in (1, 2, 3):
        m = [int(v) for v in rng.integers(1, 5, d)]
        n = [int(v) for v in rng.integers(1, 5, d)]
        ops = "".join(rng.choice(["N", "C"], d))
        fs, ldf = [], []
        for k in range(d):
            rows, cols = (m[k], n[k]) if ops[k] == "N" else (n[k], m[k])
            fs.append(rng.standard_normal(rows * cols) + 1j * rng.standard_normal(rows * cols))
            ldf.append(rows)
        X = rng.standard_normal(int(np.prod(n))) + 1j * rng.standard_normal(int(np.prod(n)))
        Z = rng.standard_normal(int(np.prod(m))) + 1j * rng.standard_normal(int(np.prod(m)))
        KX = orc.kron_nd(m, n, ops, 1.0, fs, X, 0.0, np.zeros(Z.size, complex), 1, ldf=ldf)
        KhZ = orc.kron_nd(n, m, "".join(flip[o] for o in ops), 1.0, fs, Z, 0.0, np.zeros(X.size, complex), 1,
                          ldf=ldf)
        lhs, rhs = np.vdot(Z, KX), np.vdot(KhZ, X)
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs)), (d, lhs, rhs)


def pin_nd_special_cases(orc, seed=18):
    """d = 1 is a batched matrix-vector product (numpy.matmul); identity
    factors copy; with square real shared factors, d = 2 and 3 equal the
    pinned 2-D / 3-D actions; a NaN-filled Y with beta = 0 is not read."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (5, 3))
    X = rng.standard_normal(4 * 3)
    got = orc.kron_nd([5], [3], "N", 1.0, [cm(A)], X, 0.0, np.full(4 * 5, np.nan), 4)
    assert np.allclose(got.reshape(4, 5), np.matmul(A, X.reshape(4, 3).T).T, rtol=1e-14, atol=1e-14)
    dims = [2, 3, 4]
    I = [cm(np.eye(k)) for k in dims]
    Xc = rng.standard_normal(2 * 24) + 1j * rng.standard_normal(2 * 24)
    assert np.array_equal(orc.kron_nd(dims, dims, "NTC", 1.0, I, Xc, 0.0, np.zeros(48, complex), 2), Xc)
    n = 4
    mats = rand_mats(rng, n, 3)
    X3 = rng.standard_normal(3 * n ** 3)
    want = orc.kron3d_ex(n, "T", "N", "T", 1.25, *mats, X3, 0.0, np.zeros(X3.size), 3)
    got = orc.kron_nd([n] * 3, [n] * 3, "TNT", 1.25, mats, X3, 0.0, np.zeros(X3.size), 3)
    assert rel(got, want) <= 1e-14
    X2 = rng.standard_normal(3 * n * n)
    want = orc.kron2d_ex(n, "N", "T", -2.0, mats[0], mats[1], X2, 0.5, X2[::-1].copy(), 3)
    got = orc.kron_nd([n] * 2, [n] * 2, "NT", -2.0, mats[:2], X2, 0.5, X2[::-1].copy(), 3)
    assert rel(got, want) <= 1e-14


ALL_PINS += [pin_nd_worked_examples, pin_nd_brute_force, pin_nd_adjoint, pin_nd_special_cases]
