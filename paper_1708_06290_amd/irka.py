"""Iterative rational Krylov on a resident system (the interpolation method of
Section 1, in the controller-Hessenberg coordinates of Section 2).

Every n-sized step runs in the library's kernels: the 2r shifted systems per
iteration (``shs_solve_vec`` and ``shs_solve_transposed_vec``, Section 3.3),
the real bases, their orthonormalisation and the projections
(``shs_project``).  The r x r pencil's eigenvalues and eigenvectors are taken
on the host with LAPACK (through SciPy), the split the paper uses for its own
implementation (Section 4.5: the parts of the method that deal with small
matrices stay on the CPU).

One iteration, for points sigma_i closed under conjugation and directions
b_i, c_i:

    V(:, i) = (H - sigma_i I)^{-1} R b_i,     W(:, i) = (H - sigma_i I)^{-T} Ct^T c_i
    real orthonormal bases of span V, span W;  Ar = W^T H V, Er = W^T V, Br = W^T R, Cr = Ct V
    pencil Ar - lambda Er:  right eigenvectors x_i, left y_i with y_i^* Er x_i = 1
    next points -lambda_i, directions b_i = (y_i^* Br)^T, c_i = Cr x_i

The paper fixes the number of iterations (30) for its measurements; so does
:func:`irka` (no stopping test), and it records the points of every
iteration so that a caller can judge convergence.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.linalg

from ._lib import SHS_OUT_ETA, SHS_OUT_X, shs_project


@dataclasses.dataclass
class IrkaResult:
    points: list            # ordered points of every iteration (the start first)
    directions: list        # (b, c) directions that went with each entry of points (m x r, p x r)
    Ar: np.ndarray          # last projection: r x r, r x r, r x m, p x r
    Er: np.ndarray
    Br: np.ndarray
    Cr: np.ndarray
    max_eta: float          # largest backward error over all shifted solves
    solve_s: float          # wall time of the shifted solves (device)
    project_s: float        # wall time of the projections (device)
    host_s: float           # wall time of the r x r eigenproblems (host)


def _arrange(points, bdir, cdir, real_tol):
    """Real points first, then each conjugate pair as (upper, lower) with the
    lower member exactly the conjugate of the upper one; returns the points,
    directions and the real-basis selector of shs_project."""
    pts = np.asarray(points, dtype=np.complex128)
    bd = np.asarray(bdir, dtype=np.complex128)
    cd = np.asarray(cdir, dtype=np.complex128)
    mag = np.maximum(np.abs(pts), np.finfo(float).tiny)
    real = np.abs(pts.imag) <= real_tol * mag
    up = np.flatnonzero(~real & (pts.imag > 0))
    if 2 * up.size != np.count_nonzero(~real):
        raise ValueError("interpolation points must be closed under conjugation")
    rl = np.flatnonzero(real)
    rl = rl[np.argsort(pts[rl].real, kind="stable")]
    up = up[np.lexsort((pts[up].imag, pts[up].real))]
    P, Bd, Cd, sel = [], [], [], []
    for i in rl:
        sel.append(2 * len(P))
        P.append(complex(pts[i].real, 0.0))
        Bd.append(bd[:, i].real + 0j)
        Cd.append(cd[:, i].real + 0j)
    for i in up:
        k = len(P)
        sel += [2 * k, 2 * k + 1]          # real and imaginary part of the upper column
        P += [pts[i], np.conj(pts[i])]
        Bd += [bd[:, i], np.conj(bd[:, i])]
        Cd += [cd[:, i], np.conj(cd[:, i])]
    return np.array(P), np.stack(Bd, axis=1), np.stack(Cd, axis=1), np.array(sel, dtype=np.int32)


def _next_points(Ar, Er, Br, Cr):
    lam, yl, xr = scipy.linalg.eig(Ar, Er, left=True, right=True)
    norm = np.array([yl[:, i].conj() @ Er @ xr[:, i] for i in range(lam.size)])
    xr = xr / norm[None, :]
    bnew = (yl.conj().T @ Br).T           # m x r
    cnew = Cr @ xr                        # p x r
    return -lam, bnew, cnew


def irka(system, points, bdir, cdir, iters: int = 30, stream=None) -> IrkaResult:
    """Run ``iters`` iterations from ``points`` (r values closed under
    conjugation) with directions ``bdir`` (m x r) and ``cdir`` (p x r)."""
    import torch
    dev = system.device
    n, m, p = system.n, system.m, system.p
    P, Bd, Cd, sel = _arrange(points, bdir, cdir, 0.0)
    r = P.size
    history = [P]
    dirs = [(Bd, Cd)]
    out = None
    max_eta = 0.0
    t_solve = t_proj = t_host = 0.0
    Ar = torch.empty((r, r), dtype=torch.float64, device=dev)
    Er = torch.empty((r, r), dtype=torch.float64, device=dev)
    Br = torch.empty((m, r), dtype=torch.float64, device=dev)
    Cr = torch.empty((r, max(1, p)), dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    # the two families of solves are independent: the transposed ones go on
    # a second stream (default priority), so that the latency-bound tile
    # kernels of one family overlap the other's update GEMMs
    main = stream if stream is not None else torch.cuda.current_stream(dev)
    side = torch.cuda.Stream(device=dev)
    for _ in range(iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(main):
            bd = torch.from_numpy(Bd).to(dev)
            cd = torch.from_numpy(Cd).to(dev) if p > 0 else None
            side.wait_stream(main)
            sv = system.solve_vec(P, bd, outputs=SHS_OUT_X | SHS_OUT_ETA, stream=main)
        with torch.cuda.stream(side):
            sw = system.solve_transposed_vec(P, cd, outputs=SHS_OUT_X | SHS_OUT_ETA, stream=side)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stv = torch.cat([sv.status, sw.status]).cpu().numpy()
        if stv.any():
            raise ArithmeticError(f"shifted solve failed (status {stv.max()})")
        max_eta = max(max_eta, float(torch.cat([sv.eta, sw.eta]).max().cpu()))
        shs_project(system.handle, sv.X.t(), sw.X.t(), torch.from_numpy(sel).to(dev), Ar, Er, Br, Cr, flag,
                    stream=main)
        out = (Ar.t().cpu().numpy(), Er.t().cpu().numpy(), Br.t().cpu().numpy(), Cr.t()[:p].cpu().numpy())
        if int(flag.cpu()[0]):
            raise ArithmeticError("the interpolation bases lost rank")
        t2 = time.perf_counter()
        pts, bn, cn = _next_points(*out)
        if p == 0:
            cn = np.zeros((0, r), dtype=np.complex128)
        P, Bd, Cd, sel = _arrange(pts, bn, cn, 1e-14)
        history.append(P)
        dirs.append((Bd, Cd))
        t3 = time.perf_counter()
        t_solve += t1 - t0
        t_proj += t2 - t1
        t_host += t3 - t2
    if out is None:
        out = (np.zeros((r, r)), np.zeros((r, r)), np.zeros((r, m)), np.zeros((p, r)))
    return IrkaResult(history, dirs, *out, max_eta, t_solve, t_proj, t_host)
