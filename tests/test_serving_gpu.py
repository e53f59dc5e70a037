"""Serving layer on the GPU: uneven (n, m) in one launch, FP64 and mixed
requests interleaved, admission by memory budget, cancellation, latency from
the arrival time, and each request's result bitwise equal alone and in the
mix (and within the forward-error tolerance of the oracle)."""
import time

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


# (400, 16) has 2.1e7 flops per shift: above the threshold used below
# (1.5e7) its FP64 requests take the solve route (blocked sweep); the other
# three systems share work-item launches
SYSTEMS = [(300, 2), (500, 4), (257, 1), (400, 16)]
THRESHOLD = 1.5e7


def _systems(ss):
    out = []
    for i, (n, m) in enumerate(SYSTEMS):
        A, B, C = workloads.system(n, m, m, 500 + i)
        out.append(ss.System(A, B, C))
    return out


def _requests(seed=3):
    """FP64 requests on the three work-item systems, FP64 requests on the
    solve-route system, and mixed requests on two systems (two each, so that
    requests of one system and mode can share a solve)."""
    rng = np.random.default_rng(seed)
    plan = [(0, "fp64"), (1, "fp64"), (2, "fp64"), (1, "fp64"), (0, "mixed"), (3, "fp64"), (0, "mixed"),
            (3, "fp64"), (2, "fp64"), (1, "mixed"), (1, "mixed"), (0, "fp64")]
    reqs = []
    for sys_id, mode in plan:
        s = int(rng.integers(2, 9))
        reqs.append((sys_id, workloads.log_uniform_shifts(rng, 1e-3, 1e3, s), mode))
    return reqs


def _mode(ss, mode):
    return ss.SHS_MODE_FP64 if mode == "fp64" else ss.SHS_MODE_FP32_REFINE


def test_mix_equals_alone_and_oracle():
    _need_gpu()
    import paper_1708_06290_amd as ss
    systems = _systems(ss)
    srv = ss.Server(streams=3, budget_bytes=8 << 30, blocked_flops=THRESHOLD)
    ids = [srv.register(s) for s in systems]
    reqs = _requests()
    # hold the workers until every request is queued: the first worker to
    # take a work-item request takes all of them (three systems, uneven n
    # and m, one launch); requests of one system on the solve route share
    # one solve
    srv.pause(True)
    handles = [srv.submit(ids[sys_id], shifts, mode=_mode(ss, mode)) for (sys_id, shifts, mode) in reqs]
    srv.pause(False)
    results = [srv.wait(h, timeout_ms=120000) for h in handles]
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_batch_systems"] >= 2, st
    assert st["max_batch_requests"] >= 3, st
    # the same requests again, one at a time, on an idle server
    solo = ss.Server(streams=3, budget_bytes=8 << 30, blocked_flops=THRESHOLD)
    solo_ids = [solo.register(s) for s in systems]
    for (sys_id, shifts, mode), res in zip(reqs, results):
        sysm = systems[sys_id]
        m = sysm.m
        alone = solo.wait(solo.submit(solo_ids[sys_id], shifts, mode=_mode(ss, mode)), timeout_ms=120000)
        torch.cuda.synchronize()
        stm = res.status.cpu().numpy()
        assert (stm == 0).all(), stm
        assert (res.eta.cpu().numpy() <= ETA_TOL).all()
        assert torch.equal(res.X, alone.X), f"{mode} result on system {sys_id} differs between mix and solo"
        assert torch.equal(res.G, alone.G)
        Xm, Gm = res.X.cpu().numpy(), res.G.cpu().numpy()
        H, R, Ct = (t.cpu().numpy() for t in sysm.reduced())
        Xo, Go, _ = oracle.solve(H, R, Ct, shifts)
        for j in range(len(shifts)):
            cols = slice(j * m, (j + 1) * m)
            assert oracle.forward_error(Xm[:, cols], Xo[:, cols]) <= FWD_TOL
            assert oracle.forward_error(Gm[:, cols], Go[:, cols]) <= FWD_TOL
    assert solo.stats()["max_batch_requests"] == 1
    solo.close()
    srv.close()


def test_cancel_and_arrival_latency():
    _need_gpu()
    import paper_1708_06290_amd as ss
    systems = _systems(ss)
    srv = ss.Server(streams=2, budget_bytes=8 << 30, blocked_flops=THRESHOLD)
    ids = [srv.register(s) for s in systems]
    reqs = _requests(seed=5)[:4]
    srv.pause(True)
    handles = [srv.submit(ids[sys_id], shifts, mode=_mode(ss, mode)) for (sys_id, shifts, mode) in reqs]
    # a queued request is removed at once
    srv.cancel(handles[1])
    assert srv.poll(handles[1]) == ss.SHS_REQ_CANCELLED
    with pytest.raises(ss.ShsError) as err:
        srv.wait(handles[1], timeout_ms=1000)
    assert err.value.code == ss.SHS_ERR_CANCELLED
    # arrival 0.25 s before the submit call: the latency includes it
    sys_id, shifts, mode = reqs[0]
    late = srv.submit(ids[sys_id], shifts, mode=_mode(ss, mode), arrival_s=ss.shs_server_clock() - 0.25)
    srv.pause(False)
    for h in [handles[0], handles[2], handles[3], late]:
        res = srv.wait(h, timeout_ms=120000)
        assert (res.status.cpu().numpy() == 0).all()
    assert srv.latency_ms(late) >= 250.0
    # a finished request can no longer be cancelled
    with pytest.raises(ss.ShsError) as err:
        srv.cancel(handles[0])
    assert err.value.code == ss.SHS_ERR_STATE
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 4, st
    srv.close()


def test_requests_overlap_the_callers_stream():
    """Submitting does not wait for the device: with the caller's stream busy
    for 0.3 s, submit returns at once, and the request's work still runs
    only after what the caller queued (its outputs' allocation)."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep is not available")
    systems = _systems(ss)
    srv = ss.Server(streams=2, budget_bytes=8 << 30, blocked_flops=THRESHOLD)
    ids = [srv.register(s) for s in systems]
    t0 = time.perf_counter()
    torch.cuda._sleep(10_000_000)
    torch.cuda.synchronize()
    rate = 10_000_000 / max(time.perf_counter() - t0, 1e-6)
    sys_id, shifts, mode = _requests(seed=7)[0]
    ref = srv.wait(srv.submit(ids[sys_id], shifts, mode=_mode(ss, mode)), timeout_ms=120000)
    torch.cuda._sleep(int(0.3 * rate))
    t1 = time.perf_counter()
    h = srv.submit(ids[sys_id], shifts, mode=_mode(ss, mode))
    dt = time.perf_counter() - t1
    res = srv.wait(h, timeout_ms=120000)
    print(f"submit took {dt * 1e3:.2f} ms", flush=True)
    assert dt < 0.1
    assert torch.equal(res.X, ref.X)
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
               for (sys_id, shifts, _) in _requests(seed=9)[:10]]
    for h in handles:
        res = srv.wait(h, timeout_ms=120000)
        assert (res.status.cpu().numpy() == 0).all()
    st = srv.stats()
    assert st["completed"] == 10 and st["peak_bytes"] <= int(probe * 2.5)
    # a request larger than the whole budget is refused up front
    with pytest.raises(ss.ShsError):
        srv.submit(ids[3], workloads.imag_axis_shifts(1e-1, 1e1, 4000), mode=ss.SHS_MODE_FP64)
    srv.close()
