"""Serving layer on the GPU: uneven (n, m) in one launch, FP64 and mixed
requests interleaved, admission by memory budget, and each request's result
equal alone and in the mix (bitwise for the FP64 work-item kernel; within
the forward-error tolerance in any case)."""
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


SYSTEMS = [(300, 2), (500, 4), (257, 1), (400, 16)]


def _systems(ss):
    out = []
    for i, (n, m) in enumerate(SYSTEMS):
        A, B, C = workloads.system(n, m, m, 500 + i)
        out.append(ss.System(A, B, C))
    return out


def _requests(count, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        sys_id = int(rng.integers(0, len(SYSTEMS)))
        s = int(rng.integers(2, 9))
        shifts = workloads.log_uniform_shifts(rng, 1e-3, 1e3, s)
        mode = "fp64" if r % 3 != 2 else "mixed"
        reqs.append((sys_id, shifts, mode))
    return reqs


def test_mix_equals_alone_and_oracle():
    _need_gpu()
    import paper_1708_06290_amd as ss
    systems = _systems(ss)
    # (400, 16) has 2.1e7 flops per shift: above the threshold it takes the
    # blocked solve, the other three systems share work-item launches
    srv = ss.Server(streams=3, budget_bytes=8 << 30, blocked_flops=1.5e7)
    ids = [srv.register(s) for s in systems]
    reqs = _requests(18)
    handles = []
    for (sys_id, shifts, mode) in reqs:
        md = ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE
        handles.append(srv.submit(ids[sys_id], shifts, mode=md))
    results = [srv.wait(h, timeout_ms=120000) for h in handles]
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_batch_systems"] >= 1
    # the same requests again, one at a time, on an idle server
    solo = ss.Server(streams=3, budget_bytes=8 << 30, blocked_flops=1.5e7)
    solo_ids = [solo.register(s) for s in systems]
    for (sys_id, shifts, mode), res in zip(reqs, results):
        sysm = systems[sys_id]
        m = sysm.m
        md = ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE
        alone = solo.wait(solo.submit(solo_ids[sys_id], shifts, mode=md), timeout_ms=120000)
        batch = sysm.solve(shifts, mode=md)
        torch.cuda.synchronize()
        Xm, Xa, Xb = res.X.cpu().numpy(), alone.X.cpu().numpy(), batch.X.cpu().numpy()
        stm = res.status.cpu().numpy()
        assert np.isin(stm, [0, ss.SHS_STATUS_FALLBACK]).all(), stm
        assert (res.eta.cpu().numpy() <= 1e-13).all()
        if mode == "fp64":
            assert np.array_equal(Xm, Xa), "FP64 result differs between the mix and a solo request"
        # the batch solver (blocked sweep) agrees to rounding
        assert np.abs(Xm - Xb.reshape(Xm.shape)).max() <= 1e-10 * np.abs(Xb).max()
        H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
        Xo, Go, _, _ = oracle.solve(H, R, Ct, shifts)
        for j in range(len(shifts)):
            xo = Xo[:, j * m:(j + 1) * m]
            assert np.abs(Xm[:, j * m:(j + 1) * m] - xo).max() <= 1e-10 * np.linalg.norm(xo)
            go = Go[:, j * m:(j + 1) * m]
            assert np.abs(res.G.cpu().numpy()[:, j * m:(j + 1) * m] - go).max() <= 1e-10 * np.linalg.norm(go)
    solo.close()
    srv.close()


def test_small_budget_queues_instead_of_failing():
    _need_gpu()
    import paper_1708_06290_amd as ss
    systems = _systems(ss)
    # a budget that admits roughly one request at a time
    probe = systems[3].workspace_bytes(8, ss.SHS_MODE_FP32_REFINE)
    srv = ss.Server(streams=4, budget_bytes=int(probe * 2.5))
    ids = [srv.register(s) for s in systems]
    handles = [srv.submit(ids[sys_id], shifts, mode=ss.SHS_MODE_FP64)
               for (sys_id, shifts, _) in _requests(10, seed=9)]
    for h in handles:
        res = srv.wait(h, timeout_ms=120000)
        assert (res.status.cpu().numpy() == 0).all()
    st = srv.stats()
    assert st["completed"] == 10 and st["peak_bytes"] <= int(probe * 2.5)
    # a request larger than the whole budget is refused up front
    with pytest.raises(ss.ShsError):
        srv.submit(ids[3], workloads.imag_axis_shifts(1e-1, 1e1, 4000), mode=ss.SHS_MODE_FP64)
    srv.close()
