"""Oracle for the shifted-system solver: plain, slow, obviously correct.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_1708_06290_amd``) never imports, links or calls it, and the
two share no code; both take their inputs from ``workloads``.

Contents, each citing the passage it follows:

* :func:`solve` -- ``X_j = (A - sigma_j I)^{-1} B`` and ``G_j = C X_j`` by
  Gaussian elimination with partial pivoting in plain C (``lu_oracle.c``),
  one shift at a time (Section 1: the transfer function and the shifted
  systems; Section 2: the same quantity in controller-Hessenberg
  coordinates).  ``G_j`` is minus the paper's transfer function
  ``C (sigma I - A)^{-1} B``.
* :func:`solve_rhs` -- ``op(A - sigma_j I) X_j = F_j`` with a right-hand side
  of its own per shift, op the identity or the transpose: the two system
  families of Section 3.3 (per-shift directions, and the transposed systems
  with unstructured right-hand sides), by the same elimination.
* :func:`reduce` -- the controller-Hessenberg form of Algorithm 1 (QR of B,
  the similarity with Q_B, the m-Hessenberg reduction by Householder
  reflectors of Section 2.1, the update of C), unblocked, in NumPy float64,
  with a final sign normalisation that makes the result essentially unique.
* :func:`backward_error`, :func:`forward_error`, :func:`spectral_distance` --
  the acceptance metrics (normwise backward error, relative forward error,
  distance of a shift from the spectrum).
* :func:`structured_pseudospectrum` -- ``||G(z)||_2`` over a set of points
  (Section 1, the structured pseudospectrum of the transfer function), from
  the oracle's ``G`` by a library SVD.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lu_oracle.c")
_LIB = os.path.join(_HERE, "liblu_oracle.so")
_lib = None

STATUS_OK = 0
STATUS_SINGULAR = 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over shifts)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Open a compiled oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.oracle_solve.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, i64, dp,
                                 dp, i64, dp, i64, ip, ctypes.c_int]
    lib.oracle_solve.restype = ctypes.c_int
    lib.oracle_solve_rhs.argtypes = [i64, dp, i64, ctypes.c_int, i64, dp, i64, dp, i64, dp, i64, ip,
                                     ctypes.c_int]
    lib.oracle_solve_rhs.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def solve(A, B, C, shifts, nthreads: int = 0, lib=None):
    """Solve ``(A - sigma_j I) X_j = B`` for every shift; return (X, G, status).

    ``X`` is ``n x (s*m)`` complex with ``X[:, j*m:(j+1)*m] = X_j``, ``G`` is
    ``p x (s*m)`` with ``G_j = C X_j``; ``status`` is 0 (ok) or 1 (exactly
    singular pivot, NaN outputs for that shift).
    """
    A = np.asfortranarray(A, dtype=np.float64)
    B = np.asfortranarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    C = np.asfortranarray(C, dtype=np.float64)
    if C.ndim == 1:
        C = C[None, :]
    n, m = B.shape
    p = C.shape[0]
    assert A.shape == (n, n) and C.shape[1] == n
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.complex128).reshape(-1))
    s = sh.size
    X = np.zeros((n, s * m), dtype=np.complex128, order="F")
    G = np.zeros((p, s * m), dtype=np.complex128, order="F")
    status = np.zeros(s, dtype=np.int32)
    lib = _load() if lib is None else lib
    rc = lib.oracle_solve(n, m, p, _dptr(A), n, _dptr(B), n, _dptr(C), max(p, 1),
                          s, _dptr(sh),
                          _dptr(X), n, _dptr(G), max(p, 1),
                          status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_solve: out of memory")
    return X, G, status


def solve_rhs(A, F, shifts, r: int, trans: bool = False, nthreads: int = 0, lib=None):
    """Solve ``op(A - sigma_j I) X_j = F_j`` with per-shift right-hand sides.

    ``F`` is ``n x (s*r)`` (complex or real) with ``F[:, j*r:(j+1)*r] = F_j``;
    op is the transpose when ``trans`` (Section 3.3, the transposed systems
    of the interpolation method), else the identity (its per-shift
    directions).  Returns (X, status) with X laid out like F.
    """
    A = np.asfortranarray(A, dtype=np.float64)
    n = A.shape[0]
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.complex128).reshape(-1))
    s = sh.size
    F = np.asfortranarray(np.asarray(F, dtype=np.complex128).reshape(n, s * r))
    X = np.zeros((n, s * r), dtype=np.complex128, order="F")
    status = np.zeros(s, dtype=np.int32)
    lib = _load() if lib is None else lib
    rc = lib.oracle_solve_rhs(n, _dptr(A), n, 1 if trans else 0, s, _dptr(sh), r, _dptr(F), n,
                              _dptr(X), n, status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_solve_rhs: out of memory")
    return X, status


# ---------------------------------------------------------------------------
# Controller-Hessenberg reduction (Algorithm 1), unblocked
# ---------------------------------------------------------------------------

def _householder(x: np.ndarray):
    """Real Householder reflector: (I - tau v v^T) x = beta e_1 with v[0] = 1.

    beta = -sign(x_0) ||x||; an x whose tail is already zero gives tau = 0.
    """
    alpha = float(x[0])
    sig = float(np.linalg.norm(x[1:])) if x.size > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    if sig == 0.0:
        return v, 0.0, alpha
    nu = float(np.hypot(alpha, sig))
    beta = -nu if alpha >= 0.0 else nu
    v[1:] = x[1:] / (alpha - beta)
    tau = (beta - alpha) / beta
    return v, tau, beta


def reduce(A, B, C):
    """Controller-Hessenberg form of (A, B, C) following Algorithm 1.

    Returns ``(H, R, Ct, Q)`` with ``H = Q^T A Q`` m-Hessenberg (entries with
    ``i > j + m`` exactly zero), ``R = Q^T B`` upper triangular (rows ``>= m``
    exactly zero), ``Ct = C Q`` and ``Q`` orthogonal, ``Q = Q_B Q_A`` with
    ``Q_A = diag(I_m, *)`` (Section 2).  Steps: QR of B by Householder
    reflectors; ``A <- Q_B^T A Q_B`` and ``C <- C Q_B``; one reflector per
    column j annihilating ``A(j+m+1:, j)`` applied from both sides and to C
    (Section 2.1 describes the same reflector sequence in blocked form).
    Finally a diagonal sign matrix S makes ``R(i, i) >= 0`` and
    ``H(j+m, j) >= 0``; with those entries nonzero the form is then unique.
    """
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    B = np.array(B, dtype=np.float64, order="F", copy=True)
    C = np.array(C, dtype=np.float64, order="F", copy=True)
    if B.ndim == 1:
        B = B[:, None]
    if C.ndim == 1:
        C = C[None, :]
    n, m = B.shape
    Q = np.eye(n)
    # 1. QR factorisation of B (reflectors j = 0..m-1 on rows j..n-1)
    for j in range(min(m, n)):
        v, tau, _ = _householder(B[j:, j].copy())
        if tau == 0.0:
            continue
        B[j:, :] -= tau * np.outer(v, v @ B[j:, :])
        # 2. similarity with the same reflector, and C <- C P
        A[j:, :] -= tau * np.outer(v, v @ A[j:, :])
        A[:, j:] -= tau * np.outer(A[:, j:] @ v, v)
        C[:, j:] -= tau * np.outer(C[:, j:] @ v, v)
        Q[:, j:] -= tau * np.outer(Q[:, j:] @ v, v)
    for j in range(min(m, n)):
        B[j + 1:, j] = 0.0
    # 3./4. m-Hessenberg reduction of A; reflector on rows j+m..n-1
    for j in range(0, n - m - 1):
        v, tau, _ = _householder(A[j + m:, j].copy())
        if tau != 0.0:
            A[j + m:, :] -= tau * np.outer(v, v @ A[j + m:, :])
            A[:, j + m:] -= tau * np.outer(A[:, j + m:] @ v, v)
            C[:, j + m:] -= tau * np.outer(C[:, j + m:] @ v, v)
            Q[:, j + m:] -= tau * np.outer(Q[:, j + m:] @ v, v)
        A[j + m + 1:, j] = 0.0
    # sign normalisation
    sgn = np.ones(n)
    for i in range(min(m, n)):
        if B[i, i] < 0.0:
            sgn[i] = -1.0
    for j in range(0, n - m):
        h = A[j + m, j] * sgn[j]
        sgn[j + m] = -1.0 if h < 0.0 else 1.0
    H = A * sgn[:, None] * sgn[None, :]
    R = B * sgn[:, None]
    Ct = C * sgn[None, :]
    Q = Q * sgn[None, :]
    return H, R, Ct, Q


# ---------------------------------------------------------------------------
# Acceptance metrics
# ---------------------------------------------------------------------------

def backward_error(A, B, X, sigma, trans: bool = False) -> float:
    """Normwise backward error of one shift.

    ``max_c ||r_c||_inf / (||M||_inf ||x_c||_inf + ||b_c||_inf)`` with
    ``M = op(A) - sigma I`` and ``r = B - M X`` in float64 (the usual normwise
    backward error of a linear system, taken column by column); op is the
    transpose when ``trans``.
    """
    A = np.asarray(A, dtype=np.float64)
    if trans:
        A = A.T
    B = np.asarray(B)
    if B.ndim == 1:
        B = B[:, None]
    X = np.asarray(X, dtype=np.complex128).reshape(B.shape[0], -1)
    r = B - (A @ X - sigma * X)
    Ms = A.astype(np.complex128)
    Ms[np.diag_indices(A.shape[0])] -= sigma
    anorm = np.abs(Ms).sum(axis=1).max()
    num = np.abs(r).max(axis=0)
    den = anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(den > 0, num / den, np.where(num > 0, np.inf, 0.0))
    return float(e.max())


def forward_error(Xhat, X) -> float:
    """Relative forward error ``||Xhat - X||_F / ||X||_F``."""
    X = np.asarray(X)
    d = np.linalg.norm(np.asarray(Xhat) - X)
    nx = np.linalg.norm(X)
    return float(d / nx) if nx > 0 else float(d)


def spectral_distance(A, shifts, eigvals=None) -> np.ndarray:
    """Distance of each shift from the spectrum of A (LAPACK eigenvalues)."""
    lam = np.linalg.eigvals(np.asarray(A)) if eigvals is None else np.asarray(eigvals)
    sh = np.asarray(shifts).reshape(-1)
    return np.abs(sh[:, None] - lam[None, :]).min(axis=1)


def structured_pseudospectrum(G, m: int) -> np.ndarray:
    """``||G_j||_2`` for every point: the largest singular value of each
    ``p x m`` block ``G_j = G[:, j*m:(j+1)*m]`` (Section 1: the structured
    pseudospectrum of (A, B, C) at a point z is read off ``||G(z)||_2``).
    """
    G = np.asarray(G, dtype=np.complex128)
    s = G.shape[1] // m
    if G.shape[0] == 0:
        return np.zeros(s)
    blocks = G.reshape(G.shape[0], s, m).transpose(1, 0, 2)
    return np.linalg.svd(blocks, compute_uv=False)[:, 0]


def modal_transfer(V, blocks, B, C, shifts) -> np.ndarray:
    """G(sigma) = C (A - sigma I)^{-1} B in closed form for a modal system
    A = U D U^T (``workloads.modal_system``): U = P_k ... P_1 with
    P_i = I - 2 v_i v_i^T, so with B' = U^T B and C' = C U,
    G(sigma) = C' (D - sigma I)^{-1} B' and the resolvent of D is taken block
    by block: 1/(d - sigma) for a 1 x 1 block, and for a rotation block
    [[a, be], [-be, a]] (a = al - sigma) the inverse [[a, -be], [be, a]] /
    (a^2 + be^2).  O(n m p) per shift.  Returns p x (s m), laid out as
    :func:`solve`'s G."""
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    k = V.shape[1]
    Bp, Cp = B.copy(), C.copy()
    for q in reversed(range(k)):          # U^T B = P_1 ... P_k B: P_k first
        v = V[:, q]
        Bp -= 2.0 * np.outer(v, v @ Bp)
    for q in reversed(range(k)):          # C U = C P_k ... P_1: P_k first
        v = V[:, q]
        Cp -= 2.0 * np.outer(Cp @ v, v)
    n, m = Bp.shape
    p = Cp.shape[0]
    sh = np.asarray(shifts, dtype=np.complex128).reshape(-1)
    i1 = np.array([b[0] for b in blocks if b[1] == 1], dtype=np.int64)
    d1 = np.array([b[2] for b in blocks if b[1] == 1])
    i2 = np.array([b[0] for b in blocks if b[1] == 2], dtype=np.int64)
    al = np.array([b[2] for b in blocks if b[1] == 2])
    be = np.array([b[3] for b in blocks if b[1] == 2])
    G = np.zeros((p, sh.size * m), dtype=np.complex128)
    for j, sg in enumerate(sh):
        Y = np.zeros((n, m), dtype=np.complex128)     # (D - sigma I)^{-1} B'
        Y[i1] = Bp[i1] / (d1 - sg)[:, None]
        a = al - sg
        det = a * a + be * be
        x0, x1 = Bp[i2], Bp[i2 + 1]
        Y[i2] = (a[:, None] * x0 - be[:, None] * x1) / det[:, None]
        Y[i2 + 1] = (be[:, None] * x0 + a[:, None] * x1) / det[:, None]
        G[:, j * m:(j + 1) * m] = Cp @ Y
    return G


def modal_eigenvalues(blocks) -> np.ndarray:
    """The eigenvalues of a modal system: d, or al +- i be per block."""
    lam = []
    for (i, k, al, be) in blocks:
        lam += [complex(al, 0.0)] if k == 1 else [complex(al, be), complex(al, -be)]
    return np.array(lam)
