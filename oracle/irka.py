"""Oracle for the interpolation method: plain iterative rational Krylov steps.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product's IRKA
driver never imports this module, and the two share no code.

Section 1 (equations for V_k and W_k) describes the iteration: at step k,
with r interpolation points sigma_i and tangential directions b_i (m) and
c_i (p),

    V(:, i) = (A - sigma_i I)^{-1} B b_i,      W(:, i) = (A - sigma_i I)^{-T} C^T c_i,

then a Petrov-Galerkin projection of (A, B, C) onto those spaces, whose
poles, mirrored, are the next points.  Section 2 notes that the iteration
may run on the controller-Hessenberg form instead; this oracle runs it on
the original (A, B, C), with the oracle's Gaussian elimination for the
shifted systems (``solve_rhs``) and LAPACK (through NumPy/SciPy) for the
r x r problems, as the paper's own implementation does on the CPU
(Section 4.5).

One step, in the order the method states it:

1. solve the 2r shifted systems above (the points are closed under
   conjugation; a conjugate pair has conjugate directions, so its two
   columns are conjugate);
2. real bases spanning the same spaces: for a pair, the real and imaginary
   parts of the first column; for a real point, the real part;
3. orthonormal bases (the paper: orthogonalising the columns of V_k and
   W_k); QR of each basis;
4. Ar = W^T A V, Er = W^T V, Br = W^T B, Cr = C V;
5. eigenvalues lambda_i and left/right eigenvectors y_i, x_i of the pencil
   Ar - lambda Er, scaled so that y_i^* Er x_i = 1: the reduced transfer
   function is sum_i (Cr x_i)(y_i^* Br) / (s - lambda_i);
6. next points sigma_i = -lambda_i (mirror images of the reduced poles) with
   directions b_i = (y_i^* Br)^T and c_i = Cr x_i.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import solve_rhs


def order_points(sig, bdir, cdir, tol: float = 0.0):
    """Put real points first (ascending), then conjugate pairs (upper half
    plane member first, ascending by real part then imaginary part), with the
    lower member's point and directions set to the exact conjugates of the
    upper one's.  A point with |Im| <= tol |sigma| counts as real (its
    directions then lose their imaginary parts)."""
    sig = np.asarray(sig, dtype=np.complex128)
    bdir = np.asarray(bdir, dtype=np.complex128)
    cdir = np.asarray(cdir, dtype=np.complex128)
    isreal = np.abs(sig.imag) <= tol * np.abs(sig)
    real_idx = [i for i in np.argsort(sig.real) if isreal[i]]
    upper = [i for i in range(sig.size) if not isreal[i] and sig[i].imag > 0]
    lower = [i for i in range(sig.size) if not isreal[i] and sig[i].imag < 0]
    if len(upper) != len(lower):
        raise ValueError("points are not closed under conjugation")
    upper.sort(key=lambda i: (sig[i].real, sig[i].imag))
    out_s, out_b, out_c = [], [], []
    for i in real_idx:
        out_s.append(complex(sig[i].real, 0.0))
        out_b.append(bdir[:, i].real.astype(np.complex128))
        out_c.append(cdir[:, i].real.astype(np.complex128))
    for i in upper:
        out_s += [sig[i], np.conj(sig[i])]
        out_b += [bdir[:, i], np.conj(bdir[:, i])]
        out_c += [cdir[:, i], np.conj(cdir[:, i])]
    return np.array(out_s), np.stack(out_b, axis=1), np.stack(out_c, axis=1)


def real_basis(Z, sig):
    """Columns spanning the same real space as the complex columns Z of the
    ordered points sig: Re for a real point, (Re, Im) of the first member of
    a pair."""
    cols = []
    i = 0
    while i < sig.size:
        if sig[i].imag == 0.0:
            cols.append(Z[:, i].real)
            i += 1
        else:
            cols += [Z[:, i].real, Z[:, i].imag]
            i += 2
    return np.stack(cols, axis=1)


def projection(A, B, C, sig, bdir, cdir):
    """Steps 1-4 for ordered points: returns (Ar, Er, Br, Cr, V, W) with V, W
    the orthonormal real bases."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    Vc, st1 = solve_rhs(A, B @ bdir, sig, 1)
    Wc, st2 = solve_rhs(A, C.T @ cdir, sig, 1, trans=True)
    if st1.any() or st2.any():
        raise ZeroDivisionError("a point is an eigenvalue of A")
    V, _ = np.linalg.qr(real_basis(Vc, sig))
    W, _ = np.linalg.qr(real_basis(Wc, sig))
    return W.T @ A @ V, W.T @ V, W.T @ B, C @ V, V, W


def pole_residue(Ar, Er, Br, Cr):
    """Step 5: poles lambda, right residue directions (y_i^* Br)^T (columns of
    an m x r array) and left ones Cr x_i (p x r)."""
    lam, Yl, Xr = scipy.linalg.eig(Ar, Er, left=True, right=True)
    scale = np.einsum("ij,ik,kj->j", Yl.conj(), Er, Xr)   # y_i^* Er x_i
    Xr = Xr / scale[None, :]
    return lam, (Yl.conj().T @ Br).T, Cr @ Xr


def reduced_transfer(Ar, Er, Br, Cr, s):
    """Cr (s Er - Ar)^{-1} Br, the reduced model's transfer function."""
    return Cr @ np.linalg.solve(s * Er - Ar, Br.astype(np.complex128))


def irka(A, B, C, sig0, bdir0, cdir0, iters: int):
    """``iters`` steps from the points sig0 with directions bdir0 (m x r) and
    cdir0 (p x r).  Returns the list of ordered point sets, one per step
    (the first is the ordered start), and the last projection."""
    sig, bd, cd = order_points(sig0, bdir0, cdir0)
    history = [sig]
    proj = None
    for _ in range(iters):
        proj = projection(A, B, C, sig, bd, cd)
        Ar, Er, Br, Cr = proj[:4]
        lam, bn, cn = pole_residue(Ar, Er, Br, Cr)
        sig, bd, cd = order_points(-lam, bn, cn, tol=1e-14)
        history.append(sig)
    return history, proj
