"""Systems with a direction of their own per shift (Section 3.3): on the GPU,
through the C ABI, against the oracle's per-shift right-hand-side leg.

    (H - sigma_j I) x_j = R b_j          (shs_solve_vec)
    (H - sigma_j I)^T w_j = Ct^T c_j     (shs_solve_transposed_vec)

Bar: relative Frobenius error <= 1e-10 per shift against the oracle, and a
normwise backward error <= 1e-13 from the library and recomputed
independently on the CPU.  In A's coordinates, Q x_j and Q w_j solve the
original systems (A - sigma I) x = B b and (A - sigma I)^T w = C^T c.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_TOL = 1e-10
ETA_TOL = 1e-13


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_06290_amd  # noqa: F401


def _dirs(rng, k, s):
    return rng.standard_normal((k, s)) + 1j * rng.standard_normal((k, s))


CASES = [(200, 1, 1, 7, 301), (300, 2, 3, 5, 302), (257, 4, 4, 6, 303), (520, 8, 8, 4, 304), (300, 10, 10, 3, 305),
         (260, 13, 5, 3, 306), (300, 16, 16, 3, 307), (17, 16, 2, 2, 308), (600, 5, 0, 3, 309)]


@pytest.mark.parametrize("n,m,p,s,seed", CASES)
def test_vec_matches_oracle(n, m, p, s, seed):
    _need_gpu()
    import paper_1708_06290_amd as ss
    print(f"vec n={n} m={m} p={p} s={s}", flush=True)
    A, B, C = workloads.system(n, m, p, seed)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    rng = np.random.default_rng(seed)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, s)
    bh = _dirs(rng, m, s)
    res = sysm.solve_vec(shifts, torch.from_numpy(bh).cuda())
    torch.cuda.synchronize()
    assert (res.status.cpu().numpy() == 0).all()
    x = res.X.cpu().numpy()
    eta = res.eta.cpu().numpy()
    assert (eta <= ETA_TOL).all(), eta
    F = R @ bh                                            # n x s: R b_j
    xo, sto = oracle.solve_rhs(H, F, shifts, 1)
    assert (sto == 0).all()
    for j, sg in enumerate(shifts):
        assert oracle.forward_error(x[:, j], xo[:, j]) <= FWD_TOL, j
        assert oracle.backward_error(H, F[:, j], x[:, j], sg) <= ETA_TOL
    # the same column as the full solve's X_j b_j
    full = sysm.solve(shifts, outputs=ss.SHS_OUT_X)
    Xf = full.X.cpu().numpy()
    for j in range(s):
        comb = Xf[:, j * m:(j + 1) * m] @ bh[:, j]
        assert oracle.forward_error(x[:, j], comb) <= FWD_TOL
    # A's coordinates: Q x_j solves (A - sigma_j I) x = B b_j
    xa = sysm.apply_q(res.X).cpu().numpy()
    xa_o, _ = oracle.solve_rhs(A, B @ bh, shifts, 1)
    for j in range(s):
        assert oracle.forward_error(xa[:, j], xa_o[:, j]) <= FWD_TOL
    if p > 0:
        ch = _dirs(rng, p, s)
        rt = sysm.solve_transposed_vec(shifts, torch.from_numpy(ch).cuda())
        torch.cuda.synchronize()
        assert (rt.status.cpu().numpy() == 0).all()
        w = rt.X.cpu().numpy()
        assert (rt.eta.cpu().numpy() <= ETA_TOL).all()
        D = Ct.T @ ch                                     # n x s: Ct^T c_j
        wo, _ = oracle.solve_rhs(H, D, shifts, 1, trans=True)
        for j, sg in enumerate(shifts):
            assert oracle.forward_error(w[:, j], wo[:, j]) <= FWD_TOL, j
            assert oracle.backward_error(H, D[:, j], w[:, j], sg, trans=True) <= ETA_TOL
        wa = sysm.apply_q(rt.X).cpu().numpy()
        wa_o, _ = oracle.solve_rhs(A, C.T @ ch, shifts, 1, trans=True)
        for j in range(s):
            assert oracle.forward_error(wa[:, j], wa_o[:, j]) <= FWD_TOL
    sysm.close()


def test_vec_batch_invariance():
    """A shift's solution does not depend on the shifts solved with it: the
    same shift alone and inside a batch gives bitwise the same column."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, m, p = 700, 3, 2
    A, B, C = workloads.system(n, m, p, 310)
    sysm = ss.System(A, B, C)
    rng = np.random.default_rng(310)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 9)
    bh = _dirs(rng, m, 9)
    res = sysm.solve_vec(shifts, torch.from_numpy(bh).cuda())
    one = sysm.solve_vec(shifts[4:5], torch.from_numpy(bh[:, 4:5]).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(res.X.cpu().numpy()[:, 4], one.X.cpu().numpy()[:, 0])
    sysm.close()
