"""Full-size workloads on the GPU, in the configuration bench.py times.

Every shift's backward error is certified (eta <= 1e-13, from the library's
FP64 residual and, for sampled shifts, recomputed here), and sampled shifts
are compared one by one with the oracle in reduced coordinates, where it is
O(n^2 m) per shift.  The mixed form is checked against the FP64 form on all
shifts of the n = 10^4 workload.  Shifts of the complex-plane grid pass
through the spectrum, so that workload is judged by backward error, and the
forward error only on grid points well outside the spectrum's disc.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ETA_TOL = 1e-13
FWD_TOL = 1e-10


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_06290_amd  # noqa: F401


def _system(wl):
    import paper_1708_06290_amd as ss
    A, B, C = workloads.system(wl.n, wl.m, wl.p, wl.seed)
    dev = torch.device("cuda", 0)
    sysm = ss.System(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), torch.from_numpy(C).to(dev))
    del A, B, C
    return sysm


def _shifts(wl):
    if wl.shifts_kind == "imag":
        return workloads.imag_axis_shifts(wl.lo, wl.hi, wl.s)
    return workloads.plane_grid_shifts()[:wl.s]


def _check_samples(sysm, res, shifts, idx, m):
    """Sampled shifts against the oracle on (H, R, Ct), and eta recomputed."""
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    cols = np.concatenate([np.arange(j * m, (j + 1) * m) for j in idx])
    X = res.X[:, torch.as_tensor(cols, device=res.X.device)].cpu().numpy()
    G = res.G[:, torch.as_tensor(cols, device=res.G.device)].cpu().numpy()
    Xo, Go, st_o = oracle.solve(H, R, Ct, shifts[idx])
    for q, j in enumerate(idx):
        xo, xg = Xo[:, q * m:(q + 1) * m], X[:, q * m:(q + 1) * m]
        err = oracle.forward_error(xg, xo)
        assert err <= FWD_TOL, f"shift {j}: X relative error {err:.3e}"
        go, gg = Go[:, q * m:(q + 1) * m], G[:, q * m:(q + 1) * m]
        assert oracle.forward_error(gg, go) <= FWD_TOL, f"shift {j}: G"
        assert oracle.backward_error(H, R, xg, shifts[j]) <= ETA_TOL, f"shift {j}: eta"


def _end_to_end(sysm, wl, res, shifts, idx):
    """Sampled shifts checked against the original (A, B): Q X_j must solve
    (A - sigma_j I) X = B with eta <= 1e-13 (this checks the full-size
    reduction as well as the sweep)."""
    A, B, _ = workloads.system(wl.n, wl.m, wl.p, wl.seed)
    m = wl.m
    for j in idx:
        Xa = sysm.apply_q(res.X[:, j * m:(j + 1) * m].contiguous()).cpu().numpy()
        e = oracle.backward_error(A, B, Xa, shifts[j])
        print(f"shift {j}: backward error of Q X on A {e:.2e}", flush=True)
        assert e <= ETA_TOL, (j, e)


def _certified(res, allow_fallback=False):
    import paper_1708_06290_amd as ss
    st = res.status.cpu().numpy()
    ok = [0, ss.SHS_STATUS_FALLBACK] if allow_fallback else [0]
    assert np.isin(st, ok).all(), np.unique(st, return_counts=True)
    eta = res.eta.cpu().numpy()
    assert (eta <= ETA_TOL).all(), eta.max()


def test_c2_fp64_full():
    _need_gpu()
    wl = workloads.C2
    print(f"workload {wl.name}", flush=True)
    sysm = _system(wl)
    shifts = _shifts(wl)
    res = sysm.solve(shifts)
    torch.cuda.synchronize()
    _certified(res)
    idx = workloads.subset_indices(wl.s, 8)
    _check_samples(sysm, res, shifts, idx, wl.m)
    _end_to_end(sysm, wl, res, shifts, idx[:3])
    sysm.close()


def test_c3_fp64_and_mixed_full():
    _need_gpu()
    import paper_1708_06290_amd as ss
    wl = workloads.C3
    print(f"workload {wl.name}", flush=True)
    sysm = _system(wl)
    shifts = _shifts(wl)
    r64 = sysm.solve(shifts, mode=ss.SHS_MODE_FP64)
    torch.cuda.synchronize()
    _certified(r64)
    idx = workloads.subset_indices(wl.s, 4)
    _check_samples(sysm, r64, shifts, idx, wl.m)
    _end_to_end(sysm, wl, r64, shifts, idx[:2])
    rmx = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE)
    torch.cuda.synchronize()
    _certified(rmx)          # imaginary-axis shifts: no FP64 fallback
    # mixed against FP64, every shift, relative Frobenius error per shift
    m = wl.m
    # X is a view of (s m, n) storage: row j m + c holds column c of shift j
    d = (rmx.X - r64.X).t().abs().square().reshape(wl.s, m, wl.n).sum(dim=(1, 2)).sqrt()
    ref = r64.X.t().abs().square().reshape(wl.s, m, wl.n).sum(dim=(1, 2)).sqrt()
    rel = (d / ref).cpu().numpy()
    print(f"mixed vs FP64: max relative difference {rel.max():.3e}", flush=True)
    assert (rel <= FWD_TOL).all(), rel.max()
    sysm.close()


def test_c5_mixed_full():
    _need_gpu()
    import paper_1708_06290_amd as ss
    wl = workloads.C5
    print(f"workload {wl.name}", flush=True)
    sysm = _system(wl)
    shifts = _shifts(wl)
    res = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE)
    torch.cuda.synchronize()
    _certified(res, allow_fallback=True)
    # grid points far outside the spectrum's disc (centre -1.5, radius ~1)
    far = np.flatnonzero(np.abs(shifts + 1.5) > 2.2)
    idx = far[np.linspace(0, len(far) - 1, 2).round().astype(int)]
    _check_samples(sysm, res, shifts, idx, wl.m)
    sysm.close()


def test_modal_system_n10000_all_shifts():
    """A = U D U^T of order 10^4 with m = p = 8 (known spectrum): G on all
    2000 imaginary-axis shifts of the n = 10^4 workload against the closed
    form C U (D - sigma I)^{-1} U^T B, relative Frobenius error <= 1e-10 per
    shift, every shift certified.  This runs the full-size reduction and the
    blocked sweep end to end with no LU anywhere."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    wl = workloads.C3
    print("modal system n=10000 m=8", flush=True)
    ms = workloads.modal_system(wl.n, wl.m, wl.p, workloads.SEED_BASE + 7)
    dev = torch.device("cuda", 0)
    sysm = ss.System(torch.from_numpy(ms.A).to(dev), torch.from_numpy(ms.B).to(dev), torch.from_numpy(ms.C).to(dev))
    shifts = _shifts(wl)
    # every shift is far from the spectrum (the filter of the forward-error check)
    lam = oracle.modal_eigenvalues(ms.blocks)
    dist = np.abs(shifts[:, None] - lam[None, :]).min(axis=1)
    # ||A||_2 = ||D||_2: |d| for a 1 x 1 block, sqrt(al^2 + be^2) for a
    # rotation block (a normal 2 x 2 matrix)
    anorm = max(np.hypot(al, be) for (_, _, al, be) in ms.blocks)
    assert (dist >= 1e-2 * anorm).all()
    res = sysm.solve(shifts, outputs=ss.SHS_OUT_G | ss.SHS_OUT_ETA)
    torch.cuda.synchronize()
    _certified(res)
    G = res.G.cpu().numpy()
    Gc = oracle.modal_transfer(ms.V, ms.blocks, ms.B, ms.C, shifts)
    m = wl.m
    err = np.array([oracle.forward_error(G[:, j * m:(j + 1) * m], Gc[:, j * m:(j + 1) * m]) for j in range(wl.s)])
    print(f"modal G: max relative error {err.max():.3e}", flush=True)
    assert (err <= FWD_TOL).all(), (err.argmax(), err.max())
    sysm.close()


@pytest.mark.parametrize("m", [9, 12])
def test_mixed_many_shifts_96_column_tiles(m):
    """m = 9 and 12 (24 real columns per shift in the structured sweeps, 48
    in the dense correction sweeps, update tiles of 96 columns) with 1024
    imaginary-axis shifts, so that each update launch holds many more
    workgroups than the chip runs at once: every shift certified by the FP64
    solve, and by the FP32 sweep and its refinement alone (no FP64
    fallback), and every shift's X against the FP64 solve."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, s = 2048, 1024
    print(f"mixed n={n} m={m} s={s}", flush=True)
    A, B, C = workloads.system(n, m, m, 120 + m)
    sysm = ss.System(A, B, C)
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, s)
    r64 = sysm.solve(shifts, mode=ss.SHS_MODE_FP64)
    rmx = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE)
    torch.cuda.synchronize()
    _certified(r64)
    _certified(rmx)
    d = (rmx.X - r64.X).t().abs().square().reshape(s, m, n).sum(dim=(1, 2)).sqrt()
    ref = r64.X.t().abs().square().reshape(s, m, n).sum(dim=(1, 2)).sqrt()
    rel = (d / ref).cpu().numpy()
    print(f"mixed vs FP64: max relative difference {rel.max():.3e}", flush=True)
    assert (rel <= FWD_TOL).all(), rel.max()
    _check_samples(sysm, rmx, shifts, workloads.subset_indices(s, 2), m)
    sysm.close()
