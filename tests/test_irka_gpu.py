"""The interpolation method (IRKA) on the GPU driver against the oracle's
(Section 1; Section 2 for the reduced coordinates; Section 3.3 for the
shifted systems it needs):

* the point sets of every iteration agree with the oracle's (which runs on
  the original A with Gaussian elimination) to a relative 1e-8;
* the GPU projection interpolates the oracle's transfer function at the
  points it was built from: G(sigma_i) b_i = G_r(sigma_i) b_i and
  c_i^T G(sigma_i) = c_i^T G_r(sigma_i) (relative 1e-9);
* the reduced transfer functions of the two drivers agree at test points;
* every shifted solve is certified (backward error <= 1e-13).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import irka as ok

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_06290_amd  # noqa: F401


def _start(rng, m, p, pairs):
    pts = []
    for _ in range(pairs):
        z = complex(rng.uniform(0.3, 2.0), rng.uniform(0.1, 2.0))
        pts += [z, np.conj(z)]
    r = len(pts)
    bd = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    cd = rng.standard_normal((p, r)) + 1j * rng.standard_normal((p, r))
    for k in range(0, r, 2):          # conjugate directions for each pair
        bd[:, k + 1] = np.conj(bd[:, k])
        cd[:, k + 1] = np.conj(cd[:, k])
    return np.array(pts), bd, cd


@pytest.mark.parametrize("n,m,p,pairs,iters", [(300, 2, 2, 4, 4), (500, 1, 1, 3, 3), (260, 4, 3, 5, 3)])
def test_irka_matches_oracle(n, m, p, pairs, iters):
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd.irka import irka
    print(f"irka n={n} m={m} p={p} r={2 * pairs} iters={iters}", flush=True)
    A, B, C = workloads.system(n, m, p, 800 + n)
    rng = np.random.default_rng(800 + n)
    pts, bd, cd = _start(rng, m, p, pairs)
    sysm = ss.System(A, B, C)
    res = irka(sysm, pts, bd, cd, iters=iters)
    hist_o, proj_o = ok.irka(A, B, C, pts, bd, cd, iters)
    assert res.max_eta <= 1e-13
    assert len(res.points) == len(hist_o)
    for k, (pg, po) in enumerate(zip(res.points, hist_o)):
        a, b = np.sort_complex(pg), np.sort_complex(po)
        assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max(), (k, a, b)
    # the last GPU projection interpolates G at the points it was built from
    Ar, Er, Br, Cr = res.Ar, res.Er, res.Br, res.Cr
    # the directions the GPU used at that iteration are the oracle's up to
    # scaling, so interpolation along the oracle's directions must hold
    sig_o, bd_o, cd_o = _last_dirs(A, B, C, hist_o, pts, bd, cd, iters)
    _, Gp, _ = oracle.solve(A, B, C, sig_o)        # C (A - sigma I)^{-1} B = -G(sigma)
    for i, s in enumerate(sig_o):
        Gs = -Gp[:, i * m:(i + 1) * m]
        Grs = ok.reduced_transfer(Ar, Er, Br, Cr, s)
        sc = np.linalg.norm(Gs)
        assert np.linalg.norm((Gs - Grs) @ bd_o[:, i]) <= 1e-9 * sc * np.linalg.norm(bd_o[:, i])
        assert np.linalg.norm(cd_o[:, i] @ (Gs - Grs)) <= 1e-9 * sc * np.linalg.norm(cd_o[:, i])
    Aro, Ero, Bro, Cro = proj_o[:4]
    for s in (0.5j, 1.0 + 1.0j, -0.3 + 2.0j):
        g1 = ok.reduced_transfer(Ar, Er, Br, Cr, s)
        g2 = ok.reduced_transfer(Aro, Ero, Bro, Cro, s)
        assert np.abs(g1 - g2).max() <= 1e-8 * np.abs(g2).max()
    sysm.close()


def _last_dirs(A, B, C, hist_o, pts, bd, cd, iters):
    """Points and directions the oracle used in its last projection."""
    sig, b, c = ok.order_points(pts, bd, cd)
    for _ in range(iters - 1):
        Ar, Er, Br, Cr = ok.projection(A, B, C, sig, b, c)[:4]
        lam, bn, cn = ok.pole_residue(Ar, Er, Br, Cr)
        sig, b, c = ok.order_points(-lam, bn, cn, tol=1e-14)
    return sig, b, c
