"""Pins of the oracle's interpolation-method steps (oracle/irka.py) against
what the mathematics fixes, independent of the oracle's own code:

* the projection interpolates: for the points sigma_i and directions b_i,
  c_i it was built from, G(sigma_i) b_i = G_r(sigma_i) b_i,
  c_i^T G(sigma_i) = c_i^T G_r(sigma_i) and c_i^T G'(sigma_i) b_i =
  c_i^T G_r'(sigma_i) b_i (the Hermite tangential interpolation Section 1
  attributes to the method), with G from LAPACK on the dense A;
* at full order (r = n) the projection is a similarity: G_r = G everywhere;
* the pole-residue form the next directions are read from reproduces G_r;
* a first-order system is its own optimal approximation: one step from any
  point lands on the mirror image of its pole (a sign slip in the mirroring
  fails here).
"""
import numpy as np
import pytest

import workloads
from oracle import irka as ok


def _G(A, B, C, s):
    n = A.shape[0]
    return C @ np.linalg.solve(s * np.eye(n) - A, B.astype(complex))


def _dG(A, B, C, s):
    n = A.shape[0]
    R = np.linalg.inv(s * np.eye(n) - A)
    return -C @ R @ R @ B


def _start(rng, m, p, pairs, reals=0):
    pts = list(rng.uniform(0.5, 2.0, reals) + 0j)
    for _ in range(pairs):
        z = complex(rng.uniform(0.2, 2.0), rng.uniform(0.1, 3.0))
        pts += [z, np.conj(z)]
    r = len(pts)
    bd = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    cd = rng.standard_normal((p, r)) + 1j * rng.standard_normal((p, r))
    return ok.order_points(np.array(pts), bd, cd)


@pytest.mark.parametrize("n,m,p,pairs,reals", [(40, 2, 2, 3, 0), (35, 1, 3, 2, 2), (50, 3, 1, 4, 1)])
def test_projection_interpolates(n, m, p, pairs, reals):
    A, B, C = workloads.system(n, m, p, 700 + n)
    rng = np.random.default_rng(n)
    sig, bd, cd = _start(rng, m, p, pairs, reals)
    Ar, Er, Br, Cr, V, W = ok.projection(A, B, C, sig, bd, cd)
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() <= 1e-12
    for i, s in enumerate(sig):
        Gs, Grs = _G(A, B, C, s), ok.reduced_transfer(Ar, Er, Br, Cr, s)
        scale = np.linalg.norm(Gs)
        assert np.linalg.norm(Gs @ bd[:, i] - Grs @ bd[:, i]) <= 1e-9 * scale * np.linalg.norm(bd[:, i])
        assert np.linalg.norm(cd[:, i] @ Gs - cd[:, i] @ Grs) <= 1e-9 * scale * np.linalg.norm(cd[:, i])
        # derivative of the reduced transfer function: -Cr (s Er - Ar)^{-1} Er (s Er - Ar)^{-1} Br
        K = np.linalg.inv(s * Er - Ar)
        dGr = -Cr @ K @ Er @ K @ Br
        d, dr = cd[:, i] @ _dG(A, B, C, s) @ bd[:, i], cd[:, i] @ dGr @ bd[:, i]
        assert abs(d - dr) <= 1e-8 * max(abs(d), 1e-300)


def test_full_order_projection_is_exact():
    n, m, p = 6, 1, 2
    A, B, C = workloads.system(n, m, p, 711)
    rng = np.random.default_rng(711)
    sig, bd, cd = _start(rng, m, p, 3)
    Ar, Er, Br, Cr, _, _ = ok.projection(A, B, C, sig, bd, cd)
    for s in (0.3j, 1.0 + 2.0j, -0.4 - 0.7j, 5.0):
        assert np.abs(ok.reduced_transfer(Ar, Er, Br, Cr, s) - _G(A, B, C, s)).max() <= 1e-10


def test_pole_residue_form():
    A, B, C = workloads.system(30, 2, 2, 712)
    rng = np.random.default_rng(712)
    sig, bd, cd = _start(rng, 2, 2, 3)
    Ar, Er, Br, Cr, _, _ = ok.projection(A, B, C, sig, bd, cd)
    lam, bres, cres = ok.pole_residue(Ar, Er, Br, Cr)
    for s in (0.7j, 2.0 + 0.5j):
        want = ok.reduced_transfer(Ar, Er, Br, Cr, s)
        got = sum(np.outer(cres[:, i], bres[:, i]) / (s - lam[i]) for i in range(lam.size))
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_first_order_system_is_a_fixed_point():
    a = -1.7
    A = np.array([[a]])
    B = np.array([[2.0]])
    C = np.array([[0.5]])
    for s0 in (0.3, 4.0, 1.1):
        hist, _ = ok.irka(A, B, C, np.array([s0 + 0j]), np.ones((1, 1)), np.ones((1, 1)), 2)
        assert abs(hist[1][0] - (-a)) <= 1e-14 and abs(hist[2][0] - (-a)) <= 1e-14


def test_points_stay_closed_under_conjugation():
    A, B, C = workloads.system(45, 2, 2, 713)
    rng = np.random.default_rng(713)
    sig, bd, cd = _start(rng, 2, 2, 3, 1)
    hist, _ = ok.irka(A, B, C, sig, bd, cd, 3)
    for pts in hist:
        assert np.allclose(np.sort_complex(pts), np.sort_complex(np.conj(pts)), rtol=0, atol=1e-12)
