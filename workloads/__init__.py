"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays out shift grids; it holds none
of the solver's arithmetic.  Both the oracle (under ``oracle/``) and the GPU
path's tests take their inputs from here, so the two sides see identical data.

Workload recipe (the paper's experiments use random systems, Section 4.2 and
Section 4.5; no public dataset is involved):

* ``A = N(0, 1/n) - 1.5 I`` (a stable spectrum: a disc of radius about 1
  centred at -1.5), ``B`` is ``n x m`` and ``C`` is ``p x n`` with ``N(0, 1)``
  entries.  Draw order from ``numpy.random.default_rng(seed)``: A, then B,
  then C, all float64.  Arrays are returned in Fortran (column-major) order,
  which is the layout the C ABI expects; entry ``(i, j)`` is the same
  mathematical entry in every layout.
* Shifts on the imaginary axis: ``sigma = 1j * logspace(log10(lo), log10(hi), s)``
  (both ends included), the frequency sweep of a Bode plot (Section 1).
* Complex-plane grid: real parts ``linspace(-3, 1, 64)``, imaginary parts
  ``linspace(-2, 2, 64)``, ``sigma[64 b + a] = re[a] + 1j im[b]``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 170806290


def system(n: int, m: int, p: int, seed: int):
    """Return (A, B, C) drawn as described in the module docstring."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / math.sqrt(n)
    A[np.diag_indices(n)] -= 1.5
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    return np.asfortranarray(A), np.asfortranarray(B), np.asfortranarray(C)


def imag_axis_shifts(lo: float, hi: float, s: int) -> np.ndarray:
    """``s`` purely imaginary shifts ``1j*omega`` with omega log-spaced in [lo, hi]."""
    return 1j * np.logspace(math.log10(lo), math.log10(hi), s)


def plane_grid_shifts(nre: int = 64, nim: int = 64, re=(-3.0, 1.0), im=(-2.0, 2.0)) -> np.ndarray:
    """Shifts on an ``nre x nim`` grid of the complex plane, real index fastest."""
    r = np.linspace(re[0], re[1], nre)
    i = np.linspace(im[0], im[1], nim)
    return (r[None, :] + 1j * i[:, None]).reshape(-1).astype(np.complex128)


def subset_indices(s: int, k: int) -> np.ndarray:
    """Deterministic subset of ``k`` indices spread over ``range(s)``."""
    if k >= s:
        return np.arange(s)
    return np.unique(np.round(np.linspace(0, s - 1, k)).astype(np.int64))


def log_uniform_shifts(rng: np.random.Generator, lo: float, hi: float, s: int) -> np.ndarray:
    """``s`` imaginary shifts with omega drawn log-uniformly on [lo, hi]."""
    w = np.exp(rng.uniform(math.log(lo), math.log(hi), size=s))
    return 1j * w


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    m: int
    p: int
    s: int
    seed: int
    shifts_kind: str          # "imag" or "grid"
    lo: float = 0.0
    hi: float = 0.0
    mode: str = "fp64"        # precision form the workload is quoted in

    def inputs(self):
        A, B, C = system(self.n, self.m, self.p, self.seed)
        return A, B, C, self.shifts()

    def shifts(self) -> np.ndarray:
        if self.shifts_kind == "imag":
            return imag_axis_shifts(self.lo, self.hi, self.s)
        return plane_grid_shifts()


# The five workloads: CPU-sized FP64, GPU FP64, the mixed-precision headline
# (n = 10^4, m = 8), and the complex-plane grid.  The serving mix is below.
C1 = Workload("c1_n512_m1_s64", 512, 1, 1, 64, SEED_BASE + 1, "imag", 1e-2, 1e2)
C2 = Workload("c2_n4096_m4_s1000", 4096, 4, 4, 1000, SEED_BASE + 2, "imag", 1e-3, 1e3)
C3 = Workload("c3_n10000_m8_s2000", 10000, 8, 8, 2000, SEED_BASE + 3, "imag", 1e-3, 1e3, "mixed")
C5 = Workload("c5_n16384_m10_s4096", 16384, 10, 10, 4096, SEED_BASE + 5, "grid", mode="mixed")
WORKLOADS = {w.name: w for w in (C1, C2, C3, C5)}

# Serving mix: eight resident systems, p = m.
SERVE_SYSTEMS = [(1024, 1), (1024, 16), (2048, 2), (2048, 4),
                 (4096, 4), (4096, 1), (8192, 16), (8192, 2)]
SERVE_SEED = SEED_BASE + 100
ARRIVAL_SEED = SEED_BASE + 200


def serve_system(i: int, scale: float = 1.0):
    """Resident system ``i`` of the serving mix (optionally with n scaled down)."""
    n, m = SERVE_SYSTEMS[i]
    n = max(m + 1, int(round(n * scale)))
    return system(n, m, m, SERVE_SEED + i)


def request_stream(count: int, rate_hz: float, n_systems: int = 8, seed: int = ARRIVAL_SEED,
                   smin: int = 16, smax: int = 512):
    """Poisson request stream: (arrival_s, system, shifts, mode) tuples.

    Each request holds ``U{smin..smax}`` imaginary shifts with omega
    log-uniform on [1e-3, 1e3]; FP64 and mixed-precision requests alternate
    at random 50:50.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate_hz)
        sys_id = int(rng.integers(0, n_systems))
        s = int(rng.integers(smin, smax + 1))
        shifts = log_uniform_shifts(rng, 1e-3, 1e3, s)
        mode = "fp64" if rng.random() < 0.5 else "mixed"
        out.append((t, sys_id, shifts, mode))
    return out


@dataclasses.dataclass
class ModalSystem:
    """A = U D U^T with D block diagonal (1 x 1 blocks d and 2 x 2 rotation
    blocks [[al, be], [-be, al]]) and U = P_k ... P_1 a product of k
    Householder reflectors P_i = I - 2 v_i v_i^T (unit v_i, column i-1 of V),
    so the spectrum is known exactly and U is cheap to apply."""
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    V: np.ndarray              # n x k, unit columns v_i
    blocks: list               # (first index, size 1 or 2, al, be)


def modal_system(n: int, m: int, p: int, seed: int, k: int = 4) -> ModalSystem:
    """A modal test system of order n with eigenvalues in the left half plane
    (al in [-2.5, -0.5], be in [0.2, 1.0]), B and C with N(0, 1) entries."""
    rng = np.random.default_rng(seed)
    blocks = []
    D = np.zeros((n, n))
    i = 0
    while i < n:
        if i + 1 < n and rng.random() < 0.5:
            al, be = -1.5 + rng.uniform(-1.0, 1.0), rng.uniform(0.2, 1.0)
            D[i, i] = D[i + 1, i + 1] = al
            D[i, i + 1], D[i + 1, i] = be, -be
            blocks.append((i, 2, al, be))
            i += 2
        else:
            d = -1.5 + rng.uniform(-1.0, 1.0)
            D[i, i] = d
            blocks.append((i, 1, d, 0.0))
            i += 1
    V = rng.standard_normal((n, k))
    V /= np.linalg.norm(V, axis=0)[None, :]
    A = D
    for q in range(k):   # A <- P A P with P = I - 2 v v^T: A = P_k ... P_1 D P_1 ... P_k
        v = V[:, q]
        A -= 2.0 * np.outer(v, v @ A)
        A -= 2.0 * np.outer(A @ v, v)
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    return ModalSystem(np.asfortranarray(A), np.asfortranarray(B), np.asfortranarray(C), V, blocks)


# The interpolation method's workload (Section 4.5: random systems, n up to
# 15000, m = p in {1, 10, 32}, reduced order r = 100, 30 iterations; m = 32
# is beyond this library's m <= 16).
IRKA_N, IRKA_M, IRKA_R, IRKA_ITERS = 15000, 10, 100, 30
IRKA_SEED = SEED_BASE + 6


def irka_start(m: int, p: int, r: int, seed: int):
    """Start of the interpolation method: r/2 conjugate pairs on the circle
    of radius 1 about 1.5 (the mirror image of the boundary of the spectral
    disc of A = N(0, 1/n) - 1.5 I), angles (k + 1/2) pi / (r/2) in the upper
    half plane, and N(0, 1) complex directions b (m) and c (p), conjugate
    within each pair.  Returns (points r, b m x r, c p x r)."""
    rng = np.random.default_rng(seed)
    half = r // 2
    th = (np.arange(half) + 0.5) * np.pi / half
    up = 1.5 + np.exp(1j * th)
    pts = np.empty(2 * half, dtype=np.complex128)
    pts[0::2], pts[1::2] = up, np.conj(up)
    bd = rng.standard_normal((m, half)) + 1j * rng.standard_normal((m, half))
    cd = rng.standard_normal((p, half)) + 1j * rng.standard_normal((p, half))
    B = np.empty((m, 2 * half), dtype=np.complex128)
    Cd = np.empty((p, 2 * half), dtype=np.complex128)
    B[:, 0::2], B[:, 1::2] = bd, np.conj(bd)
    Cd[:, 0::2], Cd[:, 1::2] = cd, np.conj(cd)
    return pts, B, Cd
