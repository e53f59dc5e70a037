"""Pins of the oracle against facts fixed by the mathematics, not by itself.

Each test below checks the oracle (``oracle.solve`` and ``oracle.reduce``)
against something independent of its own code: closed forms (diagonal and
modal systems), brute-force exact rational arithmetic (Cramer's rule),
LAPACK's ``zgesv`` and ``dgehrd``, the Neumann series of a nilpotent matrix,
and invariance of the transfer function under orthogonal similarity
(Section 2: the controller-Hessenberg reduction is a change of coordinates
that leaves ``C (A - sigma I)^{-1} B`` unchanged).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads

RNG = np.random.default_rng(12345)


def _rand_orth(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


# --------------------------------------------------------------------------
# P1: diagonal A -- x_i = b_i / (a_i - sigma), G = sum_i c_i b_i^T / (a_i - sigma)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,p", [(1, 1, 1), (7, 2, 3), (40, 3, 2)])
def test_diagonal_closed_form(n, m, p):
    a = RNG.standard_normal(n) - 1.0
    A = np.diag(a)
    B = RNG.standard_normal((n, m))
    C = RNG.standard_normal((p, n))
    shifts = np.array([0.3j, -2.0 + 1.5j, 5.0, 1e-3j])
    X, G, st = oracle.solve(A, B, C, shifts)
    assert (st == 0).all()
    for j, sg in enumerate(shifts):
        Xc = B / (a - sg)[:, None]
        Gc = (C * (1.0 / (a - sg))[None, :]) @ B
        Xj = X[:, j * m:(j + 1) * m]
        Gj = G[:, j * m:(j + 1) * m]
        assert np.abs(Xj - Xc).max() <= 1e-14 * np.abs(Xc).max()
        assert np.abs(Gj - Gc).max() <= 1e-13 * max(1.0, np.abs(Gc).max())
        assert oracle.backward_error(A, B, Xj, sg) <= 1e-15


# --------------------------------------------------------------------------
# P2: modal closed form, A = U D U^T with real 1x1 and 2x2 rotation blocks
# --------------------------------------------------------------------------
def _modal_system(n, m, p, rng):
    U = _rand_orth(n, rng)
    D = np.zeros((n, n))
    blocks = []
    i = 0
    while i < n:
        if i + 1 < n and rng.random() < 0.5:
            al, be = -1.5 + rng.uniform(-1, 1), rng.uniform(0.2, 1.0)
            D[i:i + 2, i:i + 2] = [[al, be], [-be, al]]
            blocks.append((i, 2, al, be))
            i += 2
        else:
            d = -1.5 + rng.uniform(-1, 1)
            D[i, i] = d
            blocks.append((i, 1, d, 0.0))
            i += 1
    A = U @ D @ U.T
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    return A, B, C, U, blocks


def _modal_resolvent(blocks, n, sigma):
    """(D - sigma I)^{-1} block by block, in closed form."""
    Rv = np.zeros((n, n), dtype=np.complex128)
    for (i, k, al, be) in blocks:
        if k == 1:
            Rv[i, i] = 1.0 / (al - sigma)
        else:
            a = al - sigma
            det = a * a + be * be
            Rv[i:i + 2, i:i + 2] = np.array([[a, -be], [be, a]]) / det
    return Rv


@pytest.mark.parametrize("n,m,p", [(12, 1, 1), (33, 4, 3)])
def test_modal_closed_form(n, m, p):
    rng = np.random.default_rng(7 + n)
    A, B, C, U, blocks = _modal_system(n, m, p, rng)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 9)
    X, G, st = oracle.solve(A, B, C, shifts)
    assert (st == 0).all()
    for j, sg in enumerate(shifts):
        Rv = _modal_resolvent(blocks, n, sg)
        Xc = U @ (Rv @ (U.T @ B))
        Gc = (C @ U) @ Rv @ (U.T @ B)
        assert oracle.forward_error(X[:, j * m:(j + 1) * m], Xc) <= 1e-12
        assert oracle.forward_error(G[:, j * m:(j + 1) * m], Gc) <= 1e-12
        assert oracle.backward_error(A, B, X[:, j * m:(j + 1) * m], sg) <= 1e-14


# --------------------------------------------------------------------------
# P4: brute force, exact rational arithmetic (Cramer's rule) for n <= 4
# --------------------------------------------------------------------------
class _Q:
    """Exact complex rational a + b i."""

    def __init__(self, a, b=0):
        self.a, self.b = Fraction(a), Fraction(b)

    def __add__(self, o):
        return _Q(self.a + o.a, self.b + o.b)

    def __sub__(self, o):
        return _Q(self.a - o.a, self.b - o.b)

    def __mul__(self, o):
        return _Q(self.a * o.a - self.b * o.b, self.a * o.b + self.b * o.a)

    def __truediv__(self, o):
        d = o.a * o.a + o.b * o.b
        return _Q((self.a * o.a + self.b * o.b) / d, (self.b * o.a - self.a * o.b) / d)

    def c(self):
        return complex(float(self.a), float(self.b))


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def _det(M):
    n = len(M)
    tot = _Q(0)
    for perm in itertools.permutations(range(n)):
        t = _Q(_perm_sign(perm))
        for i in range(n):
            t = t * M[i][perm[i]]
        tot = tot + t
    return tot


@pytest.mark.parametrize("n,m,p", [(1, 1, 1), (2, 1, 2), (3, 2, 1), (4, 3, 2), (4, 1, 1)])
def test_bruteforce_exact(n, m, p):
    rng = np.random.default_rng(100 + 10 * n + m)
    A = rng.integers(-5, 6, size=(n, n)).astype(float)
    B = rng.integers(-5, 6, size=(n, m)).astype(float)
    C = rng.integers(-5, 6, size=(p, n)).astype(float)
    shifts = [complex(1, 2) / 3, complex(-7, 1) / 4, complex(0, 5) / 2]
    X, G, st = oracle.solve(A, B, C, np.array(shifts))
    for j, sg in enumerate(shifts):
        sq = _Q(Fraction(sg.real).limit_denominator(100), Fraction(sg.imag).limit_denominator(100))
        M = [[_Q(A[i, k]) - (sq if i == k else _Q(0)) for k in range(n)] for i in range(n)]
        d = _det(M)
        assert st[j] == 0
        Xe = np.zeros((n, m), dtype=complex)
        for c in range(m):
            for i in range(n):
                Mi = [row[:] for row in M]
                for r in range(n):
                    Mi[r][i] = _Q(B[r, c])
                Xe[i, c] = (_det(Mi) / d).c()
        Ge = C @ Xe
        assert oracle.forward_error(X[:, j * m:(j + 1) * m], Xe) <= 1e-14
        assert oracle.forward_error(G[:, j * m:(j + 1) * m], Ge) <= 1e-13


# --------------------------------------------------------------------------
# P5: LAPACK zgesv on (A - sigma I, B)
# --------------------------------------------------------------------------
def test_agrees_with_lapack():
    A, B, C = workloads.system(150, 3, 2, 99)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 6)
    X, G, st = oracle.solve(A, B, C, shifts)
    for j, sg in enumerate(shifts):
        Xl = np.linalg.solve(A - sg * np.eye(150), B.astype(complex))
        assert oracle.forward_error(X[:, j * 3:(j + 1) * 3], Xl) <= 1e-12
        assert oracle.forward_error(G[:, j * 3:(j + 1) * 3], C @ Xl) <= 1e-12
        assert oracle.backward_error(A, B, X[:, j * 3:(j + 1) * 3], sg) <= 1e-14


def test_pivoting_against_lapack():
    # zero diagonal: every elimination step must swap rows
    rng = np.random.default_rng(9)
    n = 24
    A = np.fliplr(np.diag(rng.uniform(1.0, 2.0, n))) + 0.01 * rng.standard_normal((n, n))
    np.fill_diagonal(A, 0.0)
    B = rng.standard_normal((n, 3))
    C = rng.standard_normal((2, n))
    shifts = np.array([0.01j, 1e-6 + 0j, 0.5 - 0.5j])
    X, G, st = oracle.solve(A, B, C, shifts)
    for j, sg in enumerate(shifts):
        Xl = np.linalg.solve(A - sg * np.eye(n), B.astype(complex))
        assert oracle.forward_error(X[:, 3 * j:3 * j + 3], Xl) <= 1e-12
        assert oracle.backward_error(A, B, X[:, 3 * j:3 * j + 3], sg) <= 1e-15


# --------------------------------------------------------------------------
# P7: nilpotent N: (N - sigma I)^{-1} = -sum_k N^k / sigma^{k+1}
# --------------------------------------------------------------------------
def test_nilpotent_neumann_series():
    n = 9
    rng = np.random.default_rng(5)
    N = np.triu(rng.standard_normal((n, n)), 1)
    B = rng.standard_normal((n, 2))
    C = rng.standard_normal((1, n))
    for sg in [2.0 + 1.0j, -0.7j, 3.0]:
        X, G, st = oracle.solve(N, B, C, np.array([sg]))
        S = np.zeros((n, n), dtype=complex)
        Nk = np.eye(n)
        for k in range(n):
            S -= Nk / sg ** (k + 1)
            Nk = Nk @ N
        assert oracle.forward_error(X, S @ B) <= 1e-13


def test_singular_shift_is_flagged_and_isolated():
    n = 6
    rng = np.random.default_rng(8)
    A = np.triu(rng.standard_normal((n, n)))
    A[2, 2] = 0.5
    B = rng.standard_normal((n, 1))
    C = rng.standard_normal((1, n))
    shifts = np.array([1j, 0.5, -1.0 + 2j])
    X, G, st = oracle.solve(A, B, C, shifts)
    assert list(st) == [0, 1, 0]
    assert np.isnan(X[:, 1]).all() and np.isnan(G[:, 1]).all()
    for j in (0, 2):
        Xl = np.linalg.solve(A - shifts[j] * np.eye(n), B.astype(complex))
        assert oracle.forward_error(X[:, j], Xl[:, 0]) <= 1e-13


def test_backward_error_metric_closed_form():
    # A = I, sigma = 0, B = ones, X = (1 + e) B  ->  eta = e / (2 + e)
    n = 5
    A = np.eye(n)
    B = np.ones((n, 1))
    for e in [1e-3, 1e-9]:
        X = (1 + e) * B
        assert abs(oracle.backward_error(A, B, X, 0.0) - e / (2 + e)) <= 1e-15
    # exact solution -> 0
    assert oracle.backward_error(A, B, B.astype(complex), 0.0) == 0.0


def _eta_diagonal_closed_form(a, B, sigma, e):
    """eta of X = (1 + e) (A - sigma I)^{-1} B for A = diag(a), in closed form:
    the residual is -e B, ||A - sigma I||_inf = max_i |a_i - sigma| and
    ||x_c||_inf = (1 + e) max_i |b_ic / (a_i - sigma)|."""
    d = np.abs(a - sigma)
    out = 0.0
    for c in range(B.shape[1]):
        b = np.abs(B[:, c])
        out = max(out, e * b.max() / (d.max() * (1 + e) * (b / d).max() + b.max()))
    return out


def backward_error_pins_hold(fn) -> bool:
    """The closed forms the backward-error metric must reproduce, at shifts
    away from zero and on a non-diagonal matrix; True if ``fn`` passes all."""
    # 1. diagonal A, perturbed exact solution, complex shifts off the axis:
    #    the shift enters the residual, the norm of A - sigma I and x
    a = np.array([-1.0, -2.0, -0.5, -3.0, 0.25])
    B = np.array([[1.0, -2.0], [0.5, 1.0], [-1.0, 0.25], [2.0, 1.0], [0.1, -0.3]])
    for sigma in (3.0 + 4.0j, -0.5j, 2.5 - 1.0j):
        # the residual B - (A - sigma I) X carries a rounding error of about
        # u ||B||, i.e. a relative error of about u / e in eta
        for e in (1e-3, 1e-5):
            X = (1 + e) * B / (a - sigma)[:, None]
            want = _eta_diagonal_closed_form(a, B, sigma, e)
            got = fn(np.diag(a), B, X, sigma)
            if not abs(got - want) <= 1e-8 * want:
                return False
    # 2. a worked 2 x 2 example with off-diagonal entries (values by hand):
    #    A = [[1, 2], [0, 3]], sigma = i, b = [1, 1], x = [1, 0]:
    #    (A - sigma I) x = [1 - i, 0], r = [i, 1], ||r||_inf = 1,
    #    ||A - sigma I||_inf = max(|1 - i| + 2, |3 - i|) = 2 + sqrt(2),
    #    ||x||_inf = ||b||_inf = 1, so eta = 1 / (3 + sqrt(2)).
    A2 = np.array([[1.0, 2.0], [0.0, 3.0]])
    got = fn(A2, np.array([[1.0], [1.0]]), np.array([[1.0], [0.0]], dtype=complex), 1j)
    if not abs(got - 1.0 / (3.0 + np.sqrt(2.0))) <= 1e-15:
        return False
    return True


def test_backward_error_pins_at_nonzero_shifts():
    assert backward_error_pins_hold(oracle.backward_error)


def test_backward_error_transposed_is_the_transpose():
    # op = transpose: the same metric on A^T (worked example transposed:
    # A^T = [[1, 0], [2, 3]], x = [1, 0] -> (A^T - i I) x = [1 - i, 2],
    # r = [i, -1], ||A^T - i I||_inf = max(|1 - i|, 2 + |3 - i|) = 2 + sqrt(10))
    A2 = np.array([[1.0, 2.0], [0.0, 3.0]])
    got = oracle.backward_error(A2, np.array([[1.0], [1.0]]), np.array([[1.0], [0.0]], dtype=complex), 1j,
                                trans=True)
    assert abs(got - 1.0 / (3.0 + np.sqrt(10.0))) <= 1e-15


BACKWARD_ERROR_MUTANTS = {
    "shift_sign_in_residual": ("r = B - (A @ X - sigma * X)", "r = B - (A @ X + sigma * X)"),
    "shift_sign_in_norm": ("Ms[np.diag_indices(A.shape[0])] -= sigma", "Ms[np.diag_indices(A.shape[0])] += sigma"),
    "norm_of_A_not_shifted": ("Ms[np.diag_indices(A.shape[0])] -= sigma", "pass"),
    "dropped_rhs_norm": ("den = anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)",
                         "den = anorm * np.abs(X).max(axis=0)"),
    "max_entry_not_row_sum": ("anorm = np.abs(Ms).sum(axis=1).max()", "anorm = np.abs(Ms).max(axis=1).max()"),
    "column_sum_norm": ("anorm = np.abs(Ms).sum(axis=1).max()", "anorm = np.abs(Ms).sum(axis=0).max()"),
}


@pytest.mark.parametrize("name", sorted(BACKWARD_ERROR_MUTANTS))
def test_backward_error_mutant_is_caught(name):
    """Plausible slips planted in a copy of the metric fail the pins."""
    import inspect
    import textwrap
    old, new = BACKWARD_ERROR_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.backward_error))
    assert src.count(old) == 1, name
    ns = {"np": np}
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    assert not backward_error_pins_hold(ns["backward_error"]), f"mutant {name} slipped past the pins"


def test_spectral_distance_modal_closed_form():
    # the eigenvalues of U D U^T are those of the blocks of D: d, or
    # al +- i be for a rotation block
    rng = np.random.default_rng(77)
    A, B, C, U, blocks = _modal_system(24, 1, 1, rng)
    lam = []
    for (i, k, al, be) in blocks:
        lam += [complex(al, 0.0)] if k == 1 else [complex(al, be), complex(al, -be)]
    lam = np.array(lam)
    shifts = np.array([0.3j, -1.5 + 0.1j, 2.0 - 1.0j, -3.0 + 0.0j])
    want = np.abs(shifts[:, None] - lam[None, :]).min(axis=1)
    got = oracle.spectral_distance(A, shifts)
    assert np.abs(got - want).max() <= 1e-12


def test_structured_pseudospectrum_closed_forms():
    # m = p = 1: |g|; a diagonal G_j: the largest modulus on the diagonal;
    # a rank-one G_j = u v^T: ||u||_2 ||v||_2
    g = np.array([[3.0 - 4.0j, 0.5j]])
    assert np.allclose(oracle.structured_pseudospectrum(g, 1), [5.0, 0.5], rtol=0, atol=1e-15)
    G = np.zeros((3, 6), dtype=complex)
    G[:, :3] = np.diag([1.0, -2.0j, 0.5])
    u = np.array([1.0, 2.0j, -2.0])
    v = np.array([3.0, 0.0, 4.0j])
    G[:, 3:] = np.outer(u, v)
    got = oracle.structured_pseudospectrum(G, 3)
    assert abs(got[0] - 2.0) <= 1e-15 and abs(got[1] - 15.0) <= 1e-13


# --------------------------------------------------------------------------
# P3: invariance under orthogonal similarity (Section 2)
# --------------------------------------------------------------------------
def test_similarity_invariance_of_G():
    A, B, C = workloads.system(60, 2, 3, 3)
    U = _rand_orth(60, np.random.default_rng(4))
    shifts = workloads.imag_axis_shifts(1e-1, 1e1, 5)
    X1, G1, _ = oracle.solve(A, B, C, shifts)
    X2, G2, _ = oracle.solve(U.T @ A @ U, U.T @ B, C @ U, shifts)
    assert oracle.forward_error(G2, G1) <= 1e-12
    assert oracle.forward_error(U @ X2, X1) <= 1e-12


# --------------------------------------------------------------------------
# Reduction (Algorithm 1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,p", [(10, 1, 1), (31, 3, 2), (64, 8, 8), (20, 19, 2), (17, 16, 3)])
def test_reduction_invariants(n, m, p):
    A, B, C = workloads.system(n, m, p, 11 + n)
    H, R, Ct, Q = oracle.reduce(A, B, C)
    u = np.finfo(float).eps
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 50 * n * u
    assert np.linalg.norm(Q.T @ A @ Q - H) <= 50 * n * u * np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ B - R) <= 50 * n * u * np.linalg.norm(B)
    assert np.linalg.norm(C @ Q - Ct) <= 50 * n * u * np.linalg.norm(C)
    i, j = np.indices((n, n))
    assert (H[i > j + m] == 0).all()
    assert (R[np.indices(R.shape)[0] > np.indices(R.shape)[1]] == 0).all()
    assert (np.diag(R) >= 0).all()
    assert all(H[k + m, k] >= 0 for k in range(n - m))
    # transfer function unchanged
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 4)
    _, G1, _ = oracle.solve(A, B, C, shifts)
    _, G2, _ = oracle.solve(H, R, Ct, shifts)
    assert oracle.forward_error(G2, G1) <= 1e-11


def test_reduction_of_reduced_input_is_identity():
    n, m = 25, 3
    rng = np.random.default_rng(21)
    H0 = np.triu(rng.standard_normal((n, n)), -m)
    for k in range(n - m):
        H0[k + m, k] = abs(H0[k + m, k]) + 0.1
    R0 = np.zeros((n, m))
    R0[:m, :] = np.triu(rng.standard_normal((m, m)))
    R0[np.arange(m), np.arange(m)] = np.abs(np.diag(R0)) + 0.1
    C0 = rng.standard_normal((2, n))
    H, R, Ct, Q = oracle.reduce(H0, R0, C0)
    assert np.abs(Q - np.eye(n)).max() <= 1e-15
    assert np.abs(H - H0).max() <= 1e-15 and np.abs(R - R0).max() <= 1e-15


def test_reduction_m1_matches_lapack_hessenberg():
    # with B = e_1 the controller-Hessenberg form is the ordinary Hessenberg
    # form with Q e_1 = e_1 (LAPACK dgehrd), up to the sign normalisation
    n = 40
    A, _, C = workloads.system(n, 1, 1, 31)
    B = np.zeros((n, 1))
    B[0, 0] = 1.0
    H, R, Ct, Q = oracle.reduce(A, B, C)
    Hl, Ql = scipy.linalg.hessenberg(A, calc_q=True)
    s = np.ones(n)
    for k in range(n - 1):
        s[k + 1] = -1.0 if Hl[k + 1, k] * s[k] < 0 else 1.0
    Hl = Hl * s[:, None] * s[None, :]
    Ql = Ql * s[None, :]
    assert np.abs(H - Hl).max() <= 1e-12
    assert np.abs(Q - Ql).max() <= 1e-12


def test_reduction_unique_under_similarity():
    # the sign-normalised controller-Hessenberg form depends only on the
    # orbit (U^T A U, U^T B, C U): Q' = U^T Q, same H, R, Ct
    n, m, p = 30, 2, 2
    A, B, C = workloads.system(n, m, p, 41)
    U = _rand_orth(n, np.random.default_rng(42))
    H1, R1, C1, Q1 = oracle.reduce(A, B, C)
    H2, R2, C2, Q2 = oracle.reduce(U.T @ A @ U, U.T @ B, C @ U)
    assert np.abs(H1 - H2).max() <= 1e-10
    assert np.abs(R1 - R2).max() <= 1e-10
    assert np.abs(C1 - C2).max() <= 1e-10
    assert np.abs(U @ Q2 - Q1).max() <= 1e-10


# --------------------------------------------------------------------------
# Per-shift right-hand sides and transposed systems (Section 3.3)
# --------------------------------------------------------------------------
def test_rhs_leg_diagonal_closed_form():
    # diag(a) is its own transpose: x_i = f_i / (a_i - sigma) either way
    rng = np.random.default_rng(61)
    n, r = 9, 2
    a = rng.standard_normal(n) - 1.0
    shifts = np.array([0.2j, -1.0 + 1.0j, 4.0 + 0.0j])
    F = rng.standard_normal((n, 3 * r)) + 1j * rng.standard_normal((n, 3 * r))
    for trans in (False, True):
        X, st = oracle.solve_rhs(np.diag(a), F, shifts, r, trans=trans)
        assert (st == 0).all()
        for j, sg in enumerate(shifts):
            Xc = F[:, j * r:(j + 1) * r] / (a - sg)[:, None]
            assert oracle.forward_error(X[:, j * r:(j + 1) * r], Xc) <= 1e-15


@pytest.mark.parametrize("trans", [False, True])
def test_rhs_leg_agrees_with_lapack(trans):
    A, _, _ = workloads.system(80, 1, 1, 62)
    rng = np.random.default_rng(63)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 5)
    F = rng.standard_normal((80, 5)) + 1j * rng.standard_normal((80, 5))
    X, st = oracle.solve_rhs(A, F, shifts, 1, trans=trans)
    op = A.T if trans else A
    for j, sg in enumerate(shifts):
        xl = np.linalg.solve(op - sg * np.eye(80), F[:, j])
        assert oracle.forward_error(X[:, j], xl) <= 1e-12
        assert oracle.backward_error(A, F[:, j:j + 1], X[:, j:j + 1], sg, trans=trans) <= 1e-15


@pytest.mark.parametrize("n", [2, 3, 4])
def test_transposed_bruteforce_exact(n):
    # Cramer's rule on (A - sigma I)^T in exact rationals
    rng = np.random.default_rng(200 + n)
    A = rng.integers(-5, 6, size=(n, n)).astype(float)
    f = rng.integers(-5, 6, size=n).astype(float) + 1j * rng.integers(-3, 4, size=n)
    sg = complex(1, 2) / 3
    X, st = oracle.solve_rhs(A, f[:, None], np.array([sg]), 1, trans=True)
    sq = _Q(Fraction(1, 3), Fraction(2, 3))
    M = [[_Q(A[k, i]) - (sq if i == k else _Q(0)) for k in range(n)] for i in range(n)]   # transposed
    d = _det(M)
    xe = np.zeros(n, dtype=complex)
    for i in range(n):
        Mi = [row[:] for row in M]
        for rr in range(n):
            Mi[rr][i] = _Q(Fraction(f[rr].real), Fraction(f[rr].imag))
        xe[i] = (_det(Mi) / d).c()
    assert oracle.forward_error(X[:, 0], xe) <= 1e-14


def test_transposed_duality():
    # c^T (A - sigma I)^{-1} b = ((A - sigma I)^{-T} c)^T b: the transposed leg
    # reproduces every entry of G through the other leg's transposes
    A, B, C = workloads.system(60, 3, 2, 64)
    shifts = workloads.imag_axis_shifts(1e-1, 1e1, 4)
    _, G, _ = oracle.solve(A, B, C, shifts)
    F = np.concatenate([C.T.astype(complex)] * len(shifts), axis=1)
    Xt, st = oracle.solve_rhs(A, F, shifts, 2, trans=True)
    for j in range(len(shifts)):
        Gd = Xt[:, 2 * j:2 * j + 2].T @ B
        assert oracle.forward_error(Gd, G[:, 3 * j:3 * j + 3]) <= 1e-12


def test_per_shift_direction_is_a_combination_of_columns():
    # (A - sigma I)^{-1} (B b_hat) = X b_hat, checked against LAPACK
    A, B, C = workloads.system(50, 4, 1, 65)
    rng = np.random.default_rng(66)
    shifts = workloads.imag_axis_shifts(1e-1, 1e1, 3)
    bh = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    F = B @ bh
    X, st = oracle.solve_rhs(A, F, shifts, 1)
    for j, sg in enumerate(shifts):
        Xl = np.linalg.solve(A - sg * np.eye(50), B.astype(complex))
        assert oracle.forward_error(X[:, j], Xl @ bh[:, j]) <= 1e-12


# --------------------------------------------------------------------------
# P2 at any size: the modal closed form used at full size on the GPU
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,p", [(30, 2, 3), (61, 8, 8)])
def test_modal_transfer_closed_form(n, m, p):
    # the closed form against the LU oracle and LAPACK on the dense A
    ms = workloads.modal_system(n, m, p, 300 + n)
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, 7)
    Gc = oracle.modal_transfer(ms.V, ms.blocks, ms.B, ms.C, shifts)
    _, G, st = oracle.solve(ms.A, ms.B, ms.C, shifts)
    assert (st == 0).all()
    for j, sg in enumerate(shifts):
        cols = slice(j * m, (j + 1) * m)
        assert oracle.forward_error(Gc[:, cols], G[:, cols]) <= 1e-12
        Gl = ms.C @ np.linalg.solve(ms.A - sg * np.eye(n), ms.B.astype(complex))
        assert oracle.forward_error(Gc[:, cols], Gl) <= 1e-12
    # the spectrum is the blocks' eigenvalues
    lam = np.sort_complex(oracle.modal_eigenvalues(ms.blocks))
    assert np.abs(np.sort_complex(np.linalg.eigvals(ms.A)) - lam).max() <= 1e-12
