"""Planted mistakes in a copy of the C oracle must be caught by the pins.

Each mutant below is a plausible slip (a wrong sign, a dropped term, a
transposed operand, a missing row swap) applied textually to a temporary copy
of ``oracle/lu_oracle.c``, compiled on the CPU and run against the closed
forms the pins use.  The real oracle passes the same checks.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads

SRC = os.path.join(os.path.dirname(oracle.__file__), "lu_oracle.c")

MUTANTS = {
    "shift_sign": ("M[j + j * n] -= sigma;", "M[j + j * n] += sigma;"),
    "dropped_rhs_update": ("F[i + c * n] -= M[i + k * n] * fk;", "(void)fk;"),
    "transposed_backsub": ("f[i] -= M[i + k * n] * xk;", "f[i] -= M[k + i * n] * xk;"),
    "multiplier_times": ("M[i + k * n] /= piv;", "M[i + k * n] *= piv;"),
    "no_rhs_swap": ("zc t = F[k + c * n]; F[k + c * n] = F[r + c * n]; F[r + c * n] = t;", ";"),
    "conj_in_G": ("acc += C[i + k * ldc] * Xj[k + c * ldx];", "acc += C[i + k * ldc] * conj(Xj[k + c * ldx]);"),
    "transpose_ignored": ("trans ? A[j + i * lda] : A[i + j * lda]", "A[i + j * lda]"),
    "rhs_leg_reads_B": ("F0 ? F0[i + c * ldf] : B[i + c * ldb]", "F0 ? F0[i + c * ldf] * 0.5 : B[i + c * ldb]"),
    "backsub_no_divide": ("zc xk = f[k] / M[k + k * n];", "zc xk = f[k];"),
    "trailing_off_by_one": ("for (int64_t i = k + 1; i <= last; ++i) M[i + j * n]",
                            "for (int64_t i = k + 1; i < last; ++i) M[i + j * n]"),
}


def _pins_pass(lib) -> bool:
    """The checks the pins make, in compact form; True if all hold."""
    rng = np.random.default_rng(3)
    # diagonal closed form
    n, m, p = 12, 2, 2
    a = rng.standard_normal(n) - 1.0
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    shifts = np.array([0.4j, -1.0 + 2.0j])
    X, G, _ = oracle.solve(np.diag(a), B, C, shifts, lib=lib)
    for j, sg in enumerate(shifts):
        Xc = B / (a - sg)[:, None]
        if oracle.forward_error(X[:, j * m:(j + 1) * m], Xc) > 1e-13:
            return False
        if oracle.forward_error(G[:, j * m:(j + 1) * m], C @ Xc) > 1e-13:
            return False
    # dense system against LAPACK (library routine)
    A, B, C = workloads.system(30, 2, 2, 17)
    X, G, _ = oracle.solve(A, B, C, shifts, lib=lib)
    for j, sg in enumerate(shifts):
        Xl = np.linalg.solve(A - sg * np.eye(30), B.astype(complex))
        if not np.isfinite(X).all() or oracle.forward_error(X[:, j * m:(j + 1) * m], Xl) > 1e-12:
            return False
        if oracle.forward_error(G[:, j * m:(j + 1) * m], C @ Xl) > 1e-12:
            return False
    # a matrix whose diagonal is zero, so every column needs a row swap
    rng = np.random.default_rng(9)
    n = 16
    A = np.fliplr(np.diag(rng.uniform(1.0, 2.0, n))) + 0.01 * rng.standard_normal((n, n))
    np.fill_diagonal(A, 0.0)
    B = rng.standard_normal((n, 2))
    C = rng.standard_normal((1, n))
    X, _, _ = oracle.solve(A, B, C, np.array([0.01j]), lib=lib)
    Xl = np.linalg.solve(A - 0.01j * np.eye(n), B.astype(complex))
    if not np.isfinite(X).all() or oracle.forward_error(X, Xl) > 1e-12:
        return False
    # per-shift right-hand sides, plain and transposed, against LAPACK
    A, _, _ = workloads.system(30, 1, 1, 18)
    F = rng.standard_normal((30, 2)) + 1j * rng.standard_normal((30, 2))
    for trans in (False, True):
        X, _ = oracle.solve_rhs(A, F, shifts, 1, trans=trans, lib=lib)
        op = A.T if trans else A
        for j, sg in enumerate(shifts):
            xl = np.linalg.solve(op - sg * np.eye(30), F[:, j])
            if not np.isfinite(X).all() or oracle.forward_error(X[:, j], xl) > 1e-12:
                return False
    return True


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path_c = tmp_path / f"{name}.c"
    path_c.write_text(src.replace(old, new))
    path_so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           str(path_c), "-o", str(path_so), "-lm"])
    return oracle.load_library(str(path_so))


def test_unmutated_oracle_passes():
    assert _pins_pass(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_variant(tmp_path, name, old, new)
    assert not _pins_pass(lib), f"mutant {name} slipped past the pins"
