"""GPU path vs the oracle, element by element, through the C ABI.

Tolerances (the acceptance criteria): relative forward error
||X_gpu - X_oracle||_F / ||X_oracle||_F <= 1e-10 per shift, for X and for G,
on shifts at least 1e-2 ||A||_2 away from the spectrum, and normwise backward
error eta <= 1e-13 on every shift, computed twice: by the library's FP64
residual kernel and independently in NumPy.
"""
import math

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
    import paper_1708_06290_amd  # noqa: F401  (raises if the library is not built)


def _blocks(X, m):
    s = X.shape[1] // m
    return [X[:, j * m:(j + 1) * m] for j in range(s)]


def _check_against(Xg, Xo, m, mask=None, tol=FWD_TOL, what="X"):
    """Relative Frobenius error of every shift's block against the oracle's."""
    for j, (xg, xo) in enumerate(zip(_blocks(Xg, m), _blocks(Xo, m))):
        if mask is not None and not mask[j]:
            continue
        err = oracle.forward_error(xg, xo)
        assert err <= tol, f"{what} shift {j}: relative error {err:.3e} > {tol:g}"


def _run(n, m, p, shifts, seed, mode=None):
    import paper_1708_06290_amd as ss
    A, B, C = workloads.system(n, m, p, seed)
    sysm = ss.System(A, B, C)
    kw = {} if mode is None else {"mode": mode}
    res = sysm.solve(shifts, **kw)
    torch.cuda.synchronize()
    return A, B, C, sysm, res


CASES = [
    # (n, m, p, s, seed)  -- several row tiles and ragged tails for every m
    (512, 1, 1, 64, workloads.C1.seed),   # the CPU-sized workload, all shifts
    (700, 8, 8, 5, 11),
    (300, 4, 2, 6, 12),
    (257, 3, 2, 4, 13),
    (1100, 2, 3, 3, 14),
    (129, 16, 3, 3, 15),
    (400, 5, 1, 3, 16),
    (333, 7, 4, 3, 17),
    (530, 11, 2, 2, 18),
    # several full row tiles, so the all-shift update runs with carried
    # columns for every per-shift column width (2m rounded up to 2, 4, 8, 16,
    # 32; (1100, 2) above covers 4)
    (1300, 1, 1, 3, 19),
    (1200, 4, 2, 3, 20),
    (1100, 6, 3, 2, 21),
    (400, 16, 4, 2, 22),
    # more outputs than one pass of the G kernel takes (8 rows of G at a time)
    (260, 5, 11, 3, 23),
    # every remaining m: each is its own tile-kernel instance (rows per lane,
    # reflector chunk) and, past m = 8, the widest update GEMM (32 real
    # columns per shift); m = 10 is the complex-plane workload's width.
    # Seven or more row tiles with a ragged last one, so grouped updates run.
    (1400, 9, 3, 3, 24),
    (1450, 10, 10, 3, 25),
    (1000, 12, 2, 2, 26),
    (950, 13, 4, 2, 27),
    (1010, 14, 1, 2, 28),
    (990, 15, 3, 2, 29),
]


@pytest.mark.parametrize("n,m,p,s,seed", CASES)
def test_fp64_solve_matches_oracle(n, m, p, s, seed):
    _need_gpu()
    shifts = workloads.C1.shifts() if n == 512 and s == 64 else workloads.imag_axis_shifts(1e-2, 1e2, s)
    print(f"case n={n} m={m} p={p} s={s} seed={seed}", flush=True)
    A, B, C, sysm, res = _run(n, m, p, shifts, seed)
    status = res.status.cpu().numpy()
    assert (status == 0).all(), status
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    X = res.X.cpu().numpy()
    G = res.G.cpu().numpy()
    eta = res.eta.cpu().numpy()
    # spectral-distance filter for the forward-error check
    dist = oracle.spectral_distance(A, shifts)
    keep = dist >= 1e-2 * np.linalg.norm(A, 2)
    assert keep.all()
    # 1. reduced coordinates: the sweep alone against the oracle on (H, R, Ct)
    Xo, Go, st_o = oracle.solve(H, R, Ct, shifts)
    _check_against(X, Xo, m, keep, what="X (reduced)")
    _check_against(G, Go, m, keep, what="G")
    # 2. backward error, from the library and independently from NumPy
    assert (eta <= ETA_TOL).all(), eta.max()
    for j, sg in enumerate(shifts):
        assert oracle.backward_error(H, R, X[:, j * m:(j + 1) * m], sg) <= ETA_TOL
    # 3. end to end: Q X against the oracle on the original (A, B, C)
    Xa = sysm.apply_q(res.X).cpu().numpy()
    Xoa, Goa, _ = oracle.solve(A, B, C, shifts)
    _check_against(Xa, Xoa, m, keep, what="Q X")
    _check_against(G, Goa, m, keep, what="G vs original")


def test_fp64_degenerate_shapes():
    _need_gpu()
    import paper_1708_06290_amd as ss
    for (n, m, p) in [(2, 1, 1), (5, 4, 2), (17, 16, 3), (65, 1, 1), (64, 8, 2), (63, 2, 0)]:
        print(f"shape n={n} m={m} p={p}", flush=True)
        A, B, C = workloads.system(n, m, p, 100 + n)
        shifts = workloads.imag_axis_shifts(1e-1, 1e1, 3)
        sysm = ss.System(A, B, C)
        res = sysm.solve(shifts)
        assert (res.status.cpu().numpy() == 0).all()
        H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
        Xo, Go, _ = oracle.solve(H, R, Ct if p > 0 else np.zeros((0, n)), shifts)
        _check_against(res.X.cpu().numpy(), Xo, m)
        if p > 0:
            _check_against(res.G.cpu().numpy(), Go, m, what="G")
        assert (res.eta.cpu().numpy() <= ETA_TOL).all()


def test_already_reduced_input_and_singular_shift():
    """Upper-triangular A is already m-Hessenberg; sigma = A(k,k) is exactly singular."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, m = 150, 3
    rng = np.random.default_rng(7)
    A = np.triu(rng.standard_normal((n, n)))
    np.fill_diagonal(A, np.linspace(-2.0, -0.5, n))
    B = np.zeros((n, m))
    B[:m, :] = np.triu(rng.standard_normal((m, m))) + 2 * np.eye(m)
    C = rng.standard_normal((2, n))
    kk = 77
    shifts = np.array([0.5j, A[kk, kk] + 0j, -1.0 + 0.25j, 1e6j])
    sysm = ss.System(A, B, C)
    res = sysm.solve(shifts)
    st = res.status.cpu().numpy()
    assert list(st) == [0, ss.SHS_STATUS_SINGULAR, 0, 0], st
    X = res.X.cpu().numpy()
    assert np.isnan(X[:, m:2 * m]).all()
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    good = np.array([0, 2, 3])
    Xo, Go, _ = oracle.solve(H, R, Ct, shifts[good])
    for q, j in enumerate(good):
        xo = Xo[:, q * m:(q + 1) * m]
        assert oracle.forward_error(X[:, j * m:(j + 1) * m], xo) <= FWD_TOL


def test_nonfinite_input_is_flagged():
    _need_gpu()
    import paper_1708_06290_amd as ss
    A, B, C = workloads.system(100, 2, 1, 3)
    A[10, 20] = np.nan
    sysm = ss.System(A, B, C)
    res = sysm.solve(np.array([1j, 2j]))
    st = res.status.cpu().numpy()
    assert (st == ss.SHS_STATUS_NONFINITE).all(), st


# several panels with ragged last panels and mini-blocks; n = 1000 makes the
# trailing products long enough to be split over K
@pytest.mark.parametrize("n,m,p", [(300, 4, 3), (1000, 8, 8), (777, 5, 2), (530, 16, 1), (129, 3, 0), (70, 1, 2)])
def test_reduction_invariants_and_oracle(n, m, p):
    _need_gpu()
    import paper_1708_06290_amd as ss
    print(f"reduction n={n} m={m} p={p}", flush=True)
    A, B, C = workloads.system(n, m, p, 21)
    sysm = ss.System(A, B, C)
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    Q = sysm.apply_q(eye).cpu().numpy().real
    u = np.finfo(float).eps
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 50 * n * u
    assert np.linalg.norm(Q.T @ A @ Q - H) <= 50 * n * u * np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ B - R) <= 50 * n * u * np.linalg.norm(B)
    assert np.linalg.norm(C @ Q - Ct) <= 50 * n * u * np.linalg.norm(C)
    i, j = np.indices((n, n))
    assert (H[i > j + m] == 0).all()
    assert (R[m:] == 0).all() and (np.tril(R[:m], -1) == 0).all()
    assert (np.diag(R[:m]) >= 0).all() and all(H[k + m, k] >= 0 for k in range(n - m))
    Ho, Ro, Cto, Qo = oracle.reduce(A, B, C)
    assert np.abs(H - Ho).max() <= 1e-9 * np.abs(A).max()
    assert np.abs(R - Ro).max() <= 1e-9 * np.abs(B).max()
    assert np.abs(Ct - Cto).max(initial=0.0) <= 1e-9 * np.abs(C).max(initial=0.0)


# every m; m = 13 .. 16 are where the FP32 sweeps keep fewer row slots per
# lane (two for [R; 0], one with a dense right-hand side), so their row
# tiles are shorter than the general budget gives.  The shifts lie on the
# imaginary axis, well away from the spectrum: the FP32 sweep plus
# refinement must certify every one of them without the FP64 fallback
# (status OK), so a broken FP32 sweep or correction cannot hide behind it.
@pytest.mark.parametrize("n,m,p,s,seed", [(600, 4, 2, 12, 31), (350, 13, 3, 4, 32), (300, 16, 2, 4, 33),
                                          (500, 1, 1, 5, 34), (420, 2, 2, 4, 35), (390, 3, 2, 4, 36),
                                          (450, 5, 1, 4, 37), (370, 6, 3, 3, 38), (610, 7, 2, 3, 39),
                                          (520, 8, 8, 3, 40), (333, 9, 2, 3, 41), (480, 10, 10, 3, 42),
                                          (301, 11, 3, 3, 43), (290, 12, 2, 3, 44), (310, 14, 1, 3, 45),
                                          (280, 15, 4, 3, 46)])
def test_fp32_refine_matches_oracle(n, m, p, s, seed):
    _need_gpu()
    import paper_1708_06290_amd as ss
    print(f"mixed n={n} m={m} p={p} s={s}", flush=True)
    shifts = workloads.imag_axis_shifts(1e-3, 1e3, s)
    A, B, C, sysm, res = _run(n, m, p, shifts, seed, mode=ss.SHS_MODE_FP32_REFINE)
    st = res.status.cpu().numpy()
    assert (st == ss.SHS_STATUS_OK).all(), st
    eta = res.eta.cpu().numpy()
    assert (eta <= ETA_TOL).all(), eta
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    X = res.X.cpu().numpy()
    Xo, Go, _ = oracle.solve(H, R, Ct, shifts)
    _check_against(X, Xo, m)
    _check_against(res.G.cpu().numpy(), Go, m, what="G")
    for j, sg in enumerate(shifts):
        assert oracle.backward_error(H, R, X[:, j * m:(j + 1) * m], sg) <= ETA_TOL


# seven or more row tiles, so a full group update (K = 4 n_b over all rows
# above the group's last tile) and the near updates before it run for every
# per-shift column width; checked in reduced coordinates, where the oracle
# is O(n^2 m) per shift
@pytest.mark.parametrize("n,m", [(3300, 1), (3300, 2), (3000, 4), (2100, 6), (1700, 8), (900, 16)])
def test_grouped_update_matches_oracle(n, m):
    _need_gpu()
    print(f"grouped n={n} m={m}", flush=True)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 3)
    A, B, C, sysm, res = _run(n, m, 2, shifts, 60 + m)
    assert (res.status.cpu().numpy() == 0).all()
    assert (res.eta.cpu().numpy() <= ETA_TOL).all()
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    X = res.X.cpu().numpy()
    Xo, Go, _ = oracle.solve(H, R, Ct, shifts)
    _check_against(X, Xo, m, np.ones(len(shifts), bool), what="X (reduced)")
    _check_against(res.G.cpu().numpy(), Go, m, np.ones(len(shifts), bool), what="G")


# single row tile (n = 400, m = 4) and several tiles with narrow shifts that
# share MFMA blocks (m = 2: 4 shifts per 16-column block; m = 4: 2)
@pytest.mark.parametrize("n,m", [(400, 4), (1100, 2), (1200, 4)])
def test_batch_invariance_and_determinism(n, m):
    _need_gpu()
    import paper_1708_06290_amd as ss
    A, B, C = workloads.system(n, m, 2, 41)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 9)
    sysm = ss.System(A, B, C)
    r1 = sysm.solve(shifts)
    r2 = sysm.solve(shifts)
    r3 = sysm.solve(shifts[3:5])
    X1, X2, X3 = (r.X.cpu().numpy() for r in (r1, r2, r3))
    assert np.array_equal(X1, X2)
    assert np.array_equal(X1[:, 3 * m:5 * m], X3)


def test_nonfinite_shift_stays_confined():
    """A NaN shift next to good ones in the same MFMA block (m = 2) is flagged
    and leaves its neighbours' results bitwise unchanged."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, m = 1100, 2
    A, B, C = workloads.system(n, m, 1, 43)
    good = workloads.imag_axis_shifts(1e-1, 1e1, 7)
    mixed = np.concatenate([good[:3], [complex(np.nan, 1.0)], good[3:]])
    sysm = ss.System(A, B, C)
    ra = sysm.solve(good)
    rb = sysm.solve(mixed)
    torch.cuda.synchronize()
    st = rb.status.cpu().numpy()
    assert st[3] == ss.SHS_STATUS_NONFINITE, st
    assert (np.delete(st, 3) == 0).all(), st
    Xa, Xb = ra.X.cpu().numpy(), rb.X.cpu().numpy()
    keep = np.concatenate([np.arange(0, 3 * m), np.arange(4 * m, 8 * m)])
    assert np.array_equal(Xa, Xb[:, keep])


# Enough shifts that the Q* pass packs several shifts into each wavefront
# (m = 2: 8 per wave past 4096 shifts; m = 4: 4 per wave past 2048; the
# mixed form runs the same pass in FP32): a subset solved alone agrees
# bitwise, and sampled shifts agree with the oracle.
@pytest.mark.parametrize("n,m,s,mode", [(300, 2, 4500, "fp64"), (260, 4, 2100, "fp64"), (260, 4, 2100, "mixed")])
def test_many_shifts_per_wave(n, m, s, mode):
    _need_gpu()
    import paper_1708_06290_amd as ss
    md = ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE
    print(f"case n={n} m={m} s={s} {mode}", flush=True)
    A, B, C = workloads.system(n, m, 1, 47)
    rng = np.random.default_rng(47)
    shifts = (rng.uniform(-1.0, 1.0, s) + 1j * rng.uniform(0.5, 20.0, s)) * 10.0
    sysm = ss.System(A, B, C)
    res = sysm.solve(shifts, mode=md)
    torch.cuda.synchronize()
    assert (res.eta.cpu().numpy() <= ETA_TOL).all()
    idx = np.unique(np.linspace(0, s - 1, 24).round().astype(int))
    sub = sysm.solve(shifts[idx], mode=md)
    torch.cuda.synchronize()
    X = res.X.cpu().numpy()
    cols = np.concatenate([np.arange(j * m, (j + 1) * m) for j in idx])
    if mode == "fp64":
        assert np.array_equal(X[:, cols], sub.X.cpu().numpy())
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    Xo, _, _ = oracle.solve(H, R, Ct, shifts[idx])
    _check_against(X[:, cols], Xo, m)


def test_empty_shift_list_and_argument_errors():
    """No shifts: nothing runs and the outputs are empty, in both modes; a
    bad argument is refused with the LAPACK-style code and leaves the
    handle usable."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd import _lib
    n, m, p = 130, 3, 2
    A, B, C = workloads.system(n, m, p, 49)
    sysm = ss.System(A, B, C)
    for mode in (ss.SHS_MODE_FP64, ss.SHS_MODE_FP32_REFINE):
        res = sysm.solve(np.zeros(0, dtype=complex), mode=mode)
        torch.cuda.synchronize()
        assert res.X.shape == (n, 0) and res.G.shape == (p, 0) and res.status.numel() == 0
    with pytest.raises(_lib.ShsError) as err:
        _lib.shs_solve_workspace(sysm.handle, -1, ss.SHS_MODE_FP64, ss.SHS_OUT_X)
    assert err.value.code == -2   # argument 2 (s) is invalid
    shifts = workloads.imag_axis_shifts(1e-1, 1e1, 3)
    res = sysm.solve(shifts)
    torch.cuda.synchronize()
    assert (res.status.cpu().numpy() == 0).all()
    H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
    Xo, _, _ = oracle.solve(H, R, Ct, shifts)
    _check_against(res.X.cpu().numpy(), Xo, m)


def test_mixed_forced_fallback_equals_fp64():
    """max_iter = 0: no correction is allowed, so every shift is recomputed by
    the FP64 sweep (status FALLBACK) and its X is bitwise the FP64 mode's;
    an unreachable tol sends every shift there too, after its corrections,
    with status NOT_CONVERGED (the FP64 result is above tol as well)."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, m, p = 900, 6, 3
    A, B, C = workloads.system(n, m, p, 71)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 9)
    sysm = ss.System(A, B, C)
    r64 = sysm.solve(shifts, mode=ss.SHS_MODE_FP64)
    r0 = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE, max_iter=0)
    rnc = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE, tol=1e-300, max_iter=5)
    torch.cuda.synchronize()
    assert (r0.status.cpu().numpy() == ss.SHS_STATUS_FALLBACK).all(), r0.status
    assert torch.equal(r0.X, r64.X) and torch.equal(r0.G, r64.G)
    assert (r0.eta.cpu().numpy() <= ETA_TOL).all()
    assert (rnc.status.cpu().numpy() == ss.SHS_STATUS_NOT_CONVERGED).all(), rnc.status
    assert torch.equal(rnc.X, r64.X)


def test_mixed_solve_is_asynchronous():
    """shs_solve in mixed mode enqueues everything and returns: queued behind
    a 0.3 s spin on the same stream, the call comes back long before the
    stream is done, and the results are right once it is."""
    _need_gpu()
    import time

    import paper_1708_06290_amd as ss
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep is not available")
    n, m, p = 700, 4, 2
    A, B, C = workloads.system(n, m, p, 72)
    shifts = workloads.imag_axis_shifts(1e-2, 1e2, 16)
    s = len(shifts)
    sysm = ss.System(A, B, C)
    ref = sysm.solve(shifts, mode=ss.SHS_MODE_FP32_REFINE)
    # every input and output in place before the timed call
    dev = sysm.device
    dsh = torch.from_numpy(shifts).to(dev)
    X = torch.empty((s * m, n), dtype=torch.complex128, device=dev)
    G = torch.empty((s * m, p), dtype=torch.complex128, device=dev)
    eta = torch.empty(s, dtype=torch.float64, device=dev)
    status = torch.empty(s, dtype=torch.int32, device=dev)
    outs = ss.SHS_OUT_X | ss.SHS_OUT_G | ss.SHS_OUT_ETA
    work = torch.empty(sysm.workspace_bytes(s, ss.SHS_MODE_FP32_REFINE, outs), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    # calibrate the spin: cycles per second of torch's sleep kernel
    t0 = time.perf_counter()
    torch.cuda._sleep(10_000_000)
    torch.cuda.synchronize()
    rate = 10_000_000 / max(time.perf_counter() - t0, 1e-6)
    stream = torch.cuda.current_stream()
    torch.cuda._sleep(int(0.3 * rate))
    t1 = time.perf_counter()
    ss.shs_solve(sysm.handle, dsh, X, G, eta, status, mode=ss.SHS_MODE_FP32_REFINE, outputs=outs, work=work,
                 stream=stream)
    dt = time.perf_counter() - t1
    busy = not stream.query()
    torch.cuda.synchronize()
    print(f"mixed solve call took {dt * 1e3:.1f} ms; stream busy after the call: {busy}", flush=True)
    assert busy and dt < 0.15
    assert torch.equal(X.t(), ref.X)
    assert (status.cpu().numpy() == 0).all()
