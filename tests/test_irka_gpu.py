"""The interpolation method (IRKA) with the GPU driver against the oracle's
(Section 1; Section 2 for the reduced coordinates; Section 3.3 for the
shifted systems it needs).

* One step from the same start: the GPU's next points agree with the
  oracle's (which works on the original A with Gaussian elimination) within
  the accuracy the problem allows.  The projected pencil is known to the
  accuracy of the computed subspaces, about max(1e-10, u kappa(V), u kappa(W))
  relative (1e-10: the forward-error bar of the shifted solves; kappa of the
  column-scaled real bases, which for nearby points can reach 1e7), and an
  eigenvalue moves by that times its condition number kappa_i; both
  condition numbers are taken from the oracle's own step.  The reduced
  transfer functions after that step agree to the same level.
* Several steps: every projection the GPU driver built interpolates the
  transfer function G of the original system (from the oracle) at its own
  points along its own directions, G(sigma_i) b_i = G_r(sigma_i) b_i and
  c_i^T G(sigma_i) = c_i^T G_r(sigma_i); the point sets stay closed under
  conjugation; every shifted solve is certified (backward error <= 1e-13).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from oracle import irka as ok

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = np.finfo(float).eps


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


def _step_accuracy(A, B, C, sig, bd, cd):
    """Relative accuracy of one oracle step's points: subspace accuracy times
    each eigenvalue's condition number (both from the oracle's step)."""
    Vc, _ = oracle.solve_rhs(A, B @ bd, sig, 1)
    Wc, _ = oracle.solve_rhs(A, C.T @ cd, sig, 1, trans=True)
    kv = []
    for Z in (ok.real_basis(Vc, sig), ok.real_basis(Wc, sig)):
        kv.append(np.linalg.cond(Z / np.linalg.norm(Z, axis=0)))
    sub = max(1e-10, U * max(kv))
    Ar, Er = ok.projection(A, B, C, sig, bd, cd)[:2]
    lam, yl, xr = scipy.linalg.eig(Ar, Er, left=True, right=True)
    na, ne = np.linalg.norm(Ar, 2), np.linalg.norm(Er, 2)
    kap = [np.linalg.norm(xr[:, i]) * np.linalg.norm(yl[:, i]) * (na + abs(lam[i]) * ne)
           / abs(yl[:, i].conj() @ Er @ xr[:, i]) for i in range(lam.size)]
    return sub, np.array(kap), -lam


CASES = [(300, 2, 2, 4, 4), (500, 1, 1, 3, 3), (260, 4, 3, 5, 3)]


@pytest.mark.parametrize("n,m,p,pairs,iters", CASES)
def test_one_step_matches_oracle(n, m, p, pairs, iters):
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd.irka import irka
    print(f"irka one step n={n} m={m} p={p} r={2 * pairs}", flush=True)
    A, B, C = workloads.system(n, m, p, 800 + n)
    pts, bd, cd = _start(np.random.default_rng(800 + n), m, p, pairs)
    sysm = ss.System(A, B, C)
    res = irka(sysm, pts, bd, cd, iters=1)
    assert res.max_eta <= 1e-13
    sig, b, c = ok.order_points(pts, bd, cd)
    hist_o, proj_o = ok.irka(A, B, C, pts, bd, cd, 1)
    sub, kap, nxt = _step_accuracy(A, B, C, sig, b, c)
    got = res.points[1]
    for i, z in enumerate(nxt):      # each oracle point has a GPU point within its bound
        d = np.abs(got - z).min()
        assert d <= 10 * sub * kap[i] + 1e-12 * abs(z), (i, z, d, sub, kap[i])
    Aro, Ero, Bro, Cro = proj_o[:4]
    for s in (0.5j, 1.0 + 1.0j, -0.3 + 2.0j):
        g1 = ok.reduced_transfer(res.Ar, res.Er, res.Br, res.Cr, s)
        g2 = ok.reduced_transfer(Aro, Ero, Bro, Cro, s)
        assert np.abs(g1 - g2).max() <= 10 * sub * kap.max() * np.abs(g2).max()
    sysm.close()


@pytest.mark.parametrize("n,m,p,pairs,iters", CASES)
def test_iterations_interpolate(n, m, p, pairs, iters):
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd.irka import irka
    print(f"irka n={n} m={m} p={p} r={2 * pairs} iters={iters}", flush=True)
    A, B, C = workloads.system(n, m, p, 800 + n)
    pts, bd, cd = _start(np.random.default_rng(800 + n), m, p, pairs)
    sysm = ss.System(A, B, C)
    res = irka(sysm, pts, bd, cd, iters=iters)
    assert res.max_eta <= 1e-13
    assert len(res.points) == iters + 1
    for P in res.points:
        assert np.array_equal(np.sort_complex(P), np.sort_complex(np.conj(P)))
    # the last projection was built from the second-to-last points and directions
    sig = res.points[-2]
    b, c = res.directions[-2]
    _, Gp, _ = oracle.solve(A, B, C, sig)           # C (A - sigma I)^{-1} B = -G(sigma)
    Vc, _ = oracle.solve_rhs(A, B @ b, sig, 1)
    kv = np.linalg.cond(ok.real_basis(Vc, sig) / np.linalg.norm(ok.real_basis(Vc, sig), axis=0))
    tol = max(1e-9, 100 * U * kv)
    for i, s in enumerate(sig):
        Gs = -Gp[:, i * m:(i + 1) * m]
        Grs = ok.reduced_transfer(res.Ar, res.Er, res.Br, res.Cr, s)
        sc = np.linalg.norm(Gs)
        assert np.linalg.norm((Gs - Grs) @ b[:, i]) <= tol * sc * np.linalg.norm(b[:, i]), i
        assert np.linalg.norm(c[:, i] @ (Gs - Grs)) <= tol * sc * np.linalg.norm(c[:, i]), i
    sysm.close()


def _orthonormal(Z):
    """Orthonormal basis of Z's columns with a positive diagonal in its
    triangular factor (what Gram-Schmidt produces), from LAPACK's QR."""
    Q, Rq = np.linalg.qr(Z)
    return Q * np.sign(np.diag(Rq))[None, :]


@pytest.mark.parametrize("n,m,p,ncol", [(700, 3, 2, 5), (2100, 8, 8, 50), (130, 1, 1, 7)])
def test_projection_against_householder_qr(n, m, p, ncol):
    """shs_project alone: real bases from selected Re / Im parts of random
    complex columns, orthonormalised on the GPU (Gram-Schmidt over the whole
    chip), then W^T H V, W^T V, W^T R, Ct V, against the same products of
    the bases LAPACK's Householder QR gives (sign-fixed to a positive
    triangular diagonal), relative Frobenius error <= 1e-11."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd._lib import shs_project
    rng = np.random.default_rng(300 + n)
    A, B, C = workloads.system(n, m, p, 301 + n)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    r = 2 * ncol
    dev = torch.device("cuda", 0)
    V = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    W = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    sel = np.arange(r, dtype=np.int32)            # Re and Im of columns 0 .. ncol-1
    Ar = torch.empty((r, r), dtype=torch.float64, device=dev)
    Er = torch.empty((r, r), dtype=torch.float64, device=dev)
    Br = torch.empty((m, r), dtype=torch.float64, device=dev)
    Cr = torch.empty((r, max(1, p)), dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    shs_project(sysm.handle, torch.from_numpy(V.T.copy()).to(dev), torch.from_numpy(W.T.copy()).to(dev),
                torch.from_numpy(sel).to(dev), Ar, Er, Br, Cr, flag)
    torch.cuda.synchronize()
    assert int(flag.cpu()[0]) == 0
    pick = lambda Z: np.stack([Z[:, k >> 1].imag if k & 1 else Z[:, k >> 1].real for k in sel], axis=1)
    Vq, Wq = _orthonormal(pick(V)), _orthonormal(pick(W))
    want = {"Ar": Wq.T @ H @ Vq, "Er": Wq.T @ Vq, "Br": Wq.T @ R, "Cr": Ct @ Vq}
    got = {"Ar": Ar.t().cpu().numpy(), "Er": Er.t().cpu().numpy(), "Br": Br.t().cpu().numpy(),
           "Cr": Cr.t()[:p].cpu().numpy()}
    for k in want:
        err = np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k])
        print(f"{k}: relative error {err:.2e}", flush=True)
        assert err <= 1e-11, (k, err)
    sysm.close()


def test_projection_flags_a_dependent_column():
    """A basis column that is a copy of an earlier one vanishes under
    Gram-Schmidt: shs_project flags the bases as rank deficient."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd._lib import shs_project
    n, m, p, ncol = 900, 2, 2, 6
    rng = np.random.default_rng(310)
    A, B, C = workloads.system(n, m, p, 311)
    sysm = ss.System(A, B, C)
    r = 2 * ncol
    dev = torch.device("cuda", 0)
    V = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    W = V.copy()
    W[:, 4] = W[:, 1]                                 # Re / Im of column 4 repeat those of column 1
    sel = np.arange(r, dtype=np.int32)
    outs = [torch.empty(s, dtype=torch.float64, device=dev) for s in ((r, r), (r, r), (m, r), (r, p))]
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    shs_project(sysm.handle, torch.from_numpy(V.T.copy()).to(dev), torch.from_numpy(W.T.copy()).to(dev),
                torch.from_numpy(sel).to(dev), *outs, flag)
    torch.cuda.synchronize()
    assert int(flag.cpu()[0]) == 1
    sysm.close()
