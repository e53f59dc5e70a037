"""Structured pseudospectrum (Section 1): ||G(z)||_2 per point on the GPU
(shs_transfer_norm2, through the C ABI) against the oracle's library SVD.

Bar: relative error <= 1e-12 per point.  The Jacobi eigenvalue computation on
the Gram matrix of a block whose largest entry lies in [1, 2) moves the
largest eigenvalue by a few units of rounding of ||G_j||^2 (Weyl's bound on
the rounding of the Gram matrix, k <= 16 terms per entry), so the norm is
within about 16 u of the exact value; 1e-12 leaves a margin of ~50x.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_06290_amd  # noqa: F401


def _gpu_norms(G, m):
    import paper_1708_06290_amd as ss
    from paper_1708_06290_amd import _lib
    s = G.shape[1] // m
    Gs = torch.from_numpy(np.ascontiguousarray(G.T)).cuda()   # (s m, p): column-major p x (s m)
    out = torch.full((s,), -1.0, dtype=torch.float64, device="cuda")
    _lib.shs_transfer_norm2(Gs, m, out)
    torch.cuda.synchronize()
    assert ss is not None
    return out.cpu().numpy()


@pytest.mark.parametrize("p,m,s,seed", [(1, 1, 50, 1), (4, 4, 40, 2), (8, 8, 33, 3), (10, 10, 20, 4),
                                        (16, 16, 17, 5), (3, 16, 9, 6), (16, 3, 9, 7), (40, 5, 8, 8),
                                        (2, 7, 11, 9), (13, 13, 6, 10), (1, 16, 5, 11), (30, 1, 5, 12)])
def test_random_blocks_match_svd(p, m, s, seed):
    _need_gpu()
    print(f"gnorm2 p={p} m={m} s={s}", flush=True)
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((p, s * m)) + 1j * rng.standard_normal((p, s * m))
    # widely different scales per block, including tiny and huge ones
    scales = 10.0 ** rng.uniform(-200, 200, size=s)
    G *= np.repeat(scales, m)[None, :]
    got = _gpu_norms(G, m)
    want = oracle.structured_pseudospectrum(G, m)
    rel = np.abs(got - want) / want
    assert rel.max() <= REL_TOL, (rel.max(), int(rel.argmax()))


def test_structured_blocks():
    """Rank-deficient, diagonal, zero, clustered and ill-conditioned blocks,
    and blocks holding NaN or infinity (NaN out)."""
    _need_gpu()
    rng = np.random.default_rng(21)
    p, m = 6, 5
    blocks = []
    u = rng.standard_normal(p) + 1j * rng.standard_normal(p)
    v = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    blocks.append(np.outer(u, v))                                # rank one: ||u|| ||v||
    d = np.zeros((p, m), dtype=complex)
    d[np.arange(m), np.arange(m)] = [1.0, -3.0j, 2.0, 0.5, 3.0 + 1e-15]
    blocks.append(d)                                             # diagonal, two nearly equal maxima
    blocks.append(np.zeros((p, m), dtype=complex))               # zero block
    U, _ = np.linalg.qr(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    sv = np.array([1.0, 1e-8, 1e-12, 1e-16, 0.0])
    blocks.append(U[:, :m] @ np.diag(sv) @ V.conj().T)           # graded singular values
    blocks.append(np.full((p, m), 1e-310 + 1e-310j))             # subnormal entries
    blocks.append(np.full((p, m), 1e300 - 1e300j))               # near overflow
    G = np.concatenate(blocks, axis=1)
    got = _gpu_norms(G, m)
    want = oracle.structured_pseudospectrum(G, m)
    assert got[2] == 0.0
    assert abs(got[0] - np.linalg.norm(u) * np.linalg.norm(v)) <= 1e-13 * got[0]
    assert abs(got[1] - (3.0 + 1e-15)) <= 1e-15 * 4
    for j in (0, 1, 3, 4, 5):
        assert abs(got[j] - want[j]) <= REL_TOL * want[j], (j, got[j], want[j])
    bad = np.concatenate([blocks[0], blocks[0]], axis=1)
    bad[1, 2] = np.nan
    bad[0, m + 1] = np.inf
    got = _gpu_norms(bad, m)
    assert np.isnan(got).all()


def test_grid_pseudospectrum_matches_oracle():
    """End to end on a complex-plane grid that crosses the spectrum: G from
    the mixed-precision solve (refined to eta <= 1e-13 at every point), then
    ||G(z)||_2; compared with the oracle's G and SVD at the points kept at
    least 1e-2 ||A||_2 from the spectrum (closer to an eigenvalue the forward
    error is governed by the conditioning, which the backward error covers)."""
    _need_gpu()
    import paper_1708_06290_amd as ss
    n, m, p = 400, 4, 3
    A, B, C = workloads.system(n, m, p, workloads.SEED_BASE + 5)
    grid = workloads.plane_grid_shifts(16, 16)
    sysm = ss.System(A, B, C)
    res = sysm.solve(grid, mode=ss.SHS_MODE_FP32_REFINE, outputs=ss.SHS_OUT_G | ss.SHS_OUT_ETA)
    norms = sysm.transfer_norm2(res.G)
    torch.cuda.synchronize()
    st = res.status.cpu().numpy()
    assert np.isin(st, (ss.SHS_STATUS_OK, ss.SHS_STATUS_FALLBACK)).all(), st
    assert (res.eta.cpu().numpy() <= 1e-13).all()
    _, Go, sto = oracle.solve(A, B, C, grid)
    assert (sto == 0).all()
    want = oracle.structured_pseudospectrum(Go, m)
    dist = oracle.spectral_distance(A, grid)
    keep = dist >= 1e-2 * np.linalg.norm(A, 2)
    got = norms.cpu().numpy()
    assert keep.sum() > 150
    rel = np.abs(got - want)[keep] / want[keep]
    assert rel.max() <= 1e-10, rel.max()
    sysm.close()
