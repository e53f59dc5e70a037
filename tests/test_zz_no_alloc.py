"""shs_solve_noalloc (the solve for callers that cannot allocate) against
shs_solve, through the C ABI: two calls in a row, the second on a smaller
input (a smaller system and fewer shifts), in both precision modes; each
result bitwise equal to shs_solve's on the same inputs (the same kernels run
on a different workspace), and within the parity bar of the oracle.  A
request larger than the static scratch is refused before any work, with its
outputs untouched."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_06290_amd  # noqa: F401


def _outputs(s, n, m, p):
    X = torch.full((s * m, n), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    G = torch.full((s * m, max(1, p)), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    eta = torch.full((s,), -1.0, dtype=torch.float64, device="cuda")
    st = torch.full((s,), -1, dtype=torch.int32, device="cuda")
    return X, G, eta, st


def _solve_both(sysm, shifts, mode):
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd import _lib
    n, m, p = sysm.n, sysm.m, sysm.p
    sh = torch.from_numpy(np.ascontiguousarray(shifts)).cuda()
    outs = ss.SHS_OUT_X | ss.SHS_OUT_G | ss.SHS_OUT_ETA
    ref = _outputs(sh.numel(), n, m, p)
    _lib.shs_solve(sysm.handle, sh, *ref, mode=mode, outputs=outs)
    got = _outputs(sh.numel(), n, m, p)
    rc = _lib.shs_solve_noalloc(sysm.handle, sh, *got, mode=mode, outputs=outs)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got]


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_equals_solve_twice(mode):
    _need_gpu()
    import paper_1708_06290_amd as ss
    for (n, m, p, s, seed) in ((900, 4, 3, 48, 901), (310, 2, 2, 9, 902)):   # second call: smaller input
        print(f"noalloc mode={mode} n={n} m={m} s={s}", flush=True)
        A, B, C = workloads.system(n, m, p, seed)
        sysm = ss.System(A, B, C)
        shifts = workloads.imag_axis_shifts(1e-2, 1e2, s)
        assert sysm.workspace_bytes(s, mode, ss.SHS_OUT_X | ss.SHS_OUT_G | ss.SHS_OUT_ETA) <= \
            ss._lib.SHS_NOALLOC_SCRATCH_BYTES
        ref, got = _solve_both(sysm, shifts, mode)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        X, G, eta, st = got
        assert (st == 0).all() and (eta <= 1e-13).all()
        H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
        Xo, Go, _ = oracle.solve(H, R, Ct, shifts)
        for j in range(s):
            cols = slice(j * m, (j + 1) * m)
            assert oracle.forward_error(X.T[:, cols], Xo[:, cols]) <= 1e-10
            assert oracle.forward_error(G.T[:p, cols], Go[:, cols]) <= 1e-10
        sysm.close()


def test_noalloc_refuses_a_request_beyond_its_scratch():
    _need_gpu()
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd import _lib
    n, m, p = 2000, 8, 2
    A, B, C = workloads.system(n, m, p, 903)
    sysm = ss.System(A, B, C)
    s = 400
    assert sysm.workspace_bytes(s, 0, ss.SHS_OUT_X | ss.SHS_OUT_G) > _lib.SHS_NOALLOC_SCRATCH_BYTES
    sh = torch.from_numpy(workloads.imag_axis_shifts(1e-2, 1e2, s)).cuda()
    X, G, eta, st = _outputs(s, n, m, p)
    rc = _lib.shs_solve_noalloc(sysm.handle, sh, X, G, eta, st, mode=0, outputs=ss.SHS_OUT_X | ss.SHS_OUT_G)
    torch.cuda.synchronize()
    assert rc == _lib.SHS_ERR_SCRATCH
    assert _lib.library().shs_strerror(rc).decode().startswith("the solve needs more")
    assert (st.cpu().numpy() == -1).all() and (X.cpu().numpy() == complex(7.0, 7.0)).all()
    # timing on: refused (phase timing would create events)
    sysm.set_timing(True)
    small = sh[:2].contiguous()
    X2, G2, eta2, st2 = _outputs(2, n, m, p)
    rc = _lib.shs_solve_noalloc(sysm.handle, small, X2, G2, eta2, st2, mode=0, outputs=ss.SHS_OUT_X)
    assert rc == _lib.SHS_ERR_STATE
    sysm.set_timing(False)
    assert ctypes is not None
    sysm.close()
