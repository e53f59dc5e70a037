"""Transposed systems (H - sigma I)^T Y = D with unstructured right-hand sides
(Section 3.3, Algorithm 11) on the GPU, through the C ABI, against the
oracle's transposed leg (plain elimination on the explicitly formed
transpose): relative Frobenius error <= 1e-10 per shift, the transposed
system's normwise backward error <= 1e-13 from the library and recomputed
independently, and the duality Y_j^T R = C~ (H - sigma_j I)^{-1} R = G_j,
which ties the transposed solve to the transfer function of the original
(A, B, C)."""
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


# (n, m, r, s, seed): every m; r = 1 (one direction per shift, the
# interpolation method's case), r = m, and r > m (two groups of m)
CASES = [(300, 1, 1, 5, 91), (257, 2, 2, 4, 92), (330, 3, 1, 3, 93), (400, 4, 7, 3, 94), (350, 5, 5, 3, 95),
         (310, 6, 2, 2, 96), (290, 7, 9, 2, 97), (520, 8, 1, 4, 98), (480, 8, 8, 3, 99), (300, 9, 4, 2, 100),
         (300, 10, 13, 2, 101), (280, 11, 1, 2, 102), (270, 12, 12, 2, 103), (290, 13, 1, 2, 104),
         (250, 14, 3, 2, 105), (260, 15, 15, 2, 106), (260, 16, 16, 2, 107), (65, 16, 3, 2, 108), (17, 16, 2, 2, 109)]


@pytest.mark.parametrize("n,m,r,s,seed", CASES)
def test_transposed_matches_oracle(n, m, r, s, seed):
    _need_gpu()
    import paper_1708_06290_amd as ss
    print(f"transposed n={n} m={m} r={r} s={s}", flush=True)
    A, B, C = workloads.system(n, m, 2, seed)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    rng = np.random.default_rng(seed)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, s)
    D = rng.standard_normal((n, s * r)) + 1j * rng.standard_normal((n, s * r))
    res = sysm.solve_transposed(shifts, torch.from_numpy(D).cuda(), r)
    torch.cuda.synchronize()
    st = res.status.cpu().numpy()
    assert (st == 0).all(), st
    Y = res.X.cpu().numpy()
    eta = res.eta.cpu().numpy()
    assert (eta <= ETA_TOL).all(), eta
    Yo, sto = oracle.solve_rhs(H, D, shifts, r, trans=True)
    assert (sto == 0).all()
    for j, sg in enumerate(shifts):
        cols = slice(j * r, (j + 1) * r)
        err = oracle.forward_error(Y[:, cols], Yo[:, cols])
        assert err <= FWD_TOL, (j, err)
        assert oracle.backward_error(H, D[:, cols], Y[:, cols], sg, trans=True) <= ETA_TOL
    sysm.close()


@pytest.mark.parametrize("n,m,p", [(1500, 4, 3), (900, 8, 8), (700, 10, 12)])
def test_transposed_duality_with_transfer_function(n, m, p):
    """D_j = C~^T for every shift: Y_j^T R = G_j = C (A - sigma_j I)^{-1} B."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    A, B, C = workloads.system(n, m, p, 110 + m)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, 6)
    D = np.concatenate([Ct.T.astype(complex)] * len(shifts), axis=1)
    res = sysm.solve_transposed(shifts, torch.from_numpy(D).cuda(), p)
    torch.cuda.synchronize()
    assert (res.status.cpu().numpy() == 0).all()
    assert (res.eta.cpu().numpy() <= ETA_TOL).all()
    Y = res.X.cpu().numpy()
    _, Go, _ = oracle.solve(H, R, Ct, shifts)
    for j in range(len(shifts)):
        Gd = Y[:, j * p:(j + 1) * p].T @ R
        assert oracle.forward_error(Gd, Go[:, j * m:(j + 1) * m]) <= FWD_TOL
    sysm.close()


def test_transposed_full_size_n10000():
    """The n = 10^4, m = 8 system with 100 shifts and one direction each (the
    interpolation method's shape, r = 100 shifts per iteration): every shift
    certified on the transposed system; sampled shifts through the duality
    with the FP64 solve of the oracle in reduced coordinates."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    wl = workloads.C3
    A, B, C = workloads.system(wl.n, wl.m, wl.p, wl.seed)
    dev = torch.device("cuda", 0)
    sysm = ss.System(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), torch.from_numpy(C).to(dev))
    del A
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    s = 100
    rng = np.random.default_rng(111)
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, s)
    chat = rng.standard_normal((wl.p, s)) + 1j * rng.standard_normal((wl.p, s))
    D = Ct.T @ chat                      # D_j = C~^T c_hat_j
    res = sysm.solve_transposed(shifts, torch.from_numpy(D).to(dev), 1)
    torch.cuda.synchronize()
    assert (res.status.cpu().numpy() == 0).all()
    eta = res.eta.cpu().numpy()
    print(f"transposed n=10^4: max eta {eta.max():.2e}", flush=True)
    assert (eta <= ETA_TOL).all()
    Y = res.X.cpu().numpy()
    idx = workloads.subset_indices(s, 3)
    _, Go, _ = oracle.solve(H, R, Ct, shifts[idx])
    m = wl.m
    for q, j in enumerate(idx):
        # y_j^T R = c_hat_j^T G_j
        lhs = Y[:, j] @ R
        rhs = chat[:, j] @ Go[:, q * m:(q + 1) * m]
        assert oracle.forward_error(lhs, rhs) <= FWD_TOL, j
    sysm.close()


@pytest.mark.parametrize("m", [6, 10])
def test_transposed_many_shifts_96_column_tiles(m):
    """m = r = 6 and 10 (24 and 48 real columns per shift in the blocked
    sweep, update tiles of 96 columns) with 1024 shifts: the update launches
    hold many more workgroups than the chip runs at once, which is where a
    tile reading another tile's columns while that one overwrites them in
    place would show.  Every shift's backward error from the library, and
    sampled shifts against the oracle with the backward error recomputed
    here."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, r, s = 2048, m, 1024
    print(f"transposed n={n} m={m} r={r} s={s}", flush=True)
    A, B, C = workloads.system(n, m, 2, 112 + m)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    rng = np.random.default_rng(112 + m)
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, s)
    D = rng.standard_normal((n, s * r)) + 1j * rng.standard_normal((n, s * r))
    res = sysm.solve_transposed(shifts, torch.from_numpy(D).cuda(), r)
    torch.cuda.synchronize()
    assert (res.status.cpu().numpy() == 0).all()
    eta = res.eta.cpu().numpy()
    print(f"max eta {eta.max():.2e}", flush=True)
    assert (eta <= ETA_TOL).all(), (np.flatnonzero(eta > ETA_TOL)[:10], eta.max())
    idx = workloads.subset_indices(s, 4)
    cols = np.concatenate([np.arange(j * r, (j + 1) * r) for j in idx])
    Y = res.X[:, torch.as_tensor(cols, device=res.X.device)].cpu().numpy()
    Ds = D[:, cols]
    Yo, sto = oracle.solve_rhs(H, Ds, shifts[idx], r, trans=True)
    assert (sto == 0).all()
    for q, j in enumerate(idx):
        c = slice(q * r, (q + 1) * r)
        assert oracle.forward_error(Y[:, c], Yo[:, c]) <= FWD_TOL, j
        assert oracle.backward_error(H, Ds[:, c], Y[:, c], shifts[j], trans=True) <= ETA_TOL, j
    sysm.close()
