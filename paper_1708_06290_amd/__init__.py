"""Many shifted linear systems on one MI355X: (A - sigma_j I) X_j = B, G_j = C X_j.

A thin Python layer over ``libshiftsolve.so`` (C ABI in ``include/shiftsolve.h``):
PyTorch provides device memory and streams, the HIP kernels do all the work.

    sys = System(A, B, C)                 # controller-Hessenberg reduction (once)
    res = sys.solve(shifts)               # X (reduced coordinates), G, eta, status
    Xa = sys.apply_q(res.X)               # back to A's coordinates

G_j = C (A - sigma_j I)^{-1} B, which is minus the transfer function
C (sigma I - A)^{-1} B of the paper's notation.
"""
from __future__ import annotations

import dataclasses

from ._lib import (SHS_ERR_CANCELLED, SHS_ERR_STATE, SHS_MAX_M, SHS_MODE_FP32_REFINE, SHS_MODE_FP64, SHS_OUT_ETA,
                   SHS_OUT_G, SHS_OUT_X, SHS_REQ_CANCELLED, SHS_REQ_DONE, SHS_REQ_FAILED, SHS_REQ_QUEUED,
                   SHS_REQ_RUNNING, SHS_STATUS_FALLBACK, SHS_STATUS_NONFINITE, SHS_STATUS_NOT_CONVERGED,
                   SHS_STATUS_OK, SHS_STATUS_SINGULAR, ShsError, library, shs_apply_q, shs_destroy,
                   shs_get_reduced, shs_info, shs_last_timings, shs_reduce, shs_server_cancel, shs_server_clock,
                   shs_server_create, shs_server_destroy, shs_server_latency, shs_server_pause, shs_server_poll,
                   shs_server_register, shs_server_stats, shs_server_submit, shs_server_submit_ex,
                   shs_server_wait, shs_set_timing, shs_solve, shs_solve_transposed,
                   shs_solve_transposed_vec, shs_solve_transposed_vec_workspace, shs_solve_transposed_workspace,
                   shs_solve_vec, shs_solve_vec_workspace, shs_solve_workspace, shs_transfer_norm2)

__all__ = ["System", "SolveResult", "library", "shs_reduce", "shs_solve", "shs_solve_workspace",
           "shs_solve_transposed", "shs_solve_transposed_workspace", "shs_transfer_norm2",
           "shs_solve_vec", "shs_solve_vec_workspace", "shs_solve_transposed_vec",
           "shs_solve_transposed_vec_workspace",
           "shs_apply_q", "shs_get_reduced", "shs_info", "shs_set_timing", "shs_last_timings",
           "shs_destroy", "ShsError", "Server", "Request", "shs_server_create", "shs_server_register",
           "shs_server_submit", "shs_server_submit_ex", "shs_server_poll", "shs_server_wait", "shs_server_latency",
           "shs_server_stats", "shs_server_destroy", "shs_server_cancel", "shs_server_pause", "shs_server_clock",
           "SHS_REQ_QUEUED", "SHS_REQ_RUNNING", "SHS_REQ_DONE", "SHS_REQ_FAILED", "SHS_REQ_CANCELLED",
           "SHS_ERR_CANCELLED", "SHS_ERR_STATE",
           "SHS_MODE_FP64", "SHS_MODE_FP32_REFINE", "SHS_OUT_X", "SHS_OUT_G", "SHS_OUT_ETA",
           "SHS_STATUS_OK", "SHS_STATUS_SINGULAR", "SHS_STATUS_NONFINITE", "SHS_STATUS_FALLBACK",
           "SHS_STATUS_NOT_CONVERGED", "SHS_MAX_M"]


@dataclasses.dataclass
class SolveResult:
    X: object        # (n, s*m) complex128 view (column-major storage), or None
    G: object        # (p, s*m) complex128 view, or None
    eta: object      # (s,) float64, or None
    status: object   # (s,) int32


class System:
    """A reduced system resident on the current GPU."""

    def __init__(self, A, B, C, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        A = torch.as_tensor(A, dtype=torch.float64, device=dev)
        B = torch.as_tensor(B, dtype=torch.float64, device=dev)
        C = torch.as_tensor(C, dtype=torch.float64, device=dev)
        if B.dim() == 1:
            B = B[:, None]
        if C.dim() == 1:
            C = C[None, :]
        self.n, self.m = B.shape
        self.p = C.shape[0]
        self.device = dev
        self.handle = shs_reduce(A, B, C, stream)

    def close(self):
        if self.handle is not None:
            shs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return shs_info(self.handle)

    def set_timing(self, enable=True):
        shs_set_timing(self.handle, enable)

    def last_timings(self):
        return shs_last_timings(self.handle)

    def reduced(self, stream=None):
        """(H, R, Ct) as (n, n), (n, m), (p, n) float64 tensors."""
        import torch
        H = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        R = torch.empty((self.m, self.n), dtype=torch.float64, device=self.device)
        Ct = torch.empty((self.n, max(1, self.p)), dtype=torch.float64, device=self.device)
        shs_get_reduced(self.handle, H, R, Ct, stream)
        return H.t(), R.t(), Ct.t()[: self.p]

    def workspace_bytes(self, s, mode=SHS_MODE_FP64, outputs=SHS_OUT_X | SHS_OUT_G):
        return shs_solve_workspace(self.handle, s, mode, outputs)

    def solve(self, shifts, mode=SHS_MODE_FP64, outputs=SHS_OUT_X | SHS_OUT_G | SHS_OUT_ETA,
              tol=1e-13, max_iter=5, work=None, stream=None, out=None):
        """Solve for every shift; returns a :class:`SolveResult` (tensors on the GPU)."""
        import torch
        shifts = torch.as_tensor(shifts, dtype=torch.complex128, device=self.device).reshape(-1).contiguous()
        s = shifts.numel()
        n, m, p = self.n, self.m, self.p
        if out is not None:
            Xs, Gs, eta, status = out
        else:
            Xs = torch.empty((s * m, n), dtype=torch.complex128, device=self.device) if outputs & SHS_OUT_X else None
            Gs = (torch.empty((s * m, max(1, p)), dtype=torch.complex128, device=self.device)
                  if (outputs & SHS_OUT_G) and p > 0 else None)
            need_eta = (outputs & SHS_OUT_ETA) or mode == SHS_MODE_FP32_REFINE
            eta = torch.empty(s, dtype=torch.float64, device=self.device) if need_eta else None
            status = torch.empty(s, dtype=torch.int32, device=self.device)
        shs_solve(self.handle, shifts, Xs, Gs, eta, status, mode=mode, outputs=outputs, tol=tol,
                  max_iter=max_iter, work=work, stream=stream)
        X = Xs.t() if Xs is not None else None
        G = Gs.t()[:p] if Gs is not None else None
        return SolveResult(X, G, eta, status)

    def solve_transposed(self, shifts, D, r=None, outputs=SHS_OUT_X | SHS_OUT_ETA, stream=None):
        """(H - sigma_j I)^T Y_j = D_j for an (n, s*r) complex tensor D (reduced
        coordinates); returns a :class:`SolveResult` with X = Y and G None."""
        import torch
        shifts = torch.as_tensor(shifts, dtype=torch.complex128, device=self.device).reshape(-1).contiguous()
        s = shifts.numel()
        D = torch.as_tensor(D, dtype=torch.complex128, device=self.device)
        if r is None:
            r = D.shape[1] // max(s, 1)
        Ds = D.t().contiguous()
        Xs = torch.empty_like(Ds) if outputs & SHS_OUT_X else None
        eta = torch.empty(s, dtype=torch.float64, device=self.device) if outputs & SHS_OUT_ETA else None
        status = torch.empty(s, dtype=torch.int32, device=self.device)
        shs_solve_transposed(self.handle, shifts, r, Ds, Xs, eta, status, outputs=outputs, stream=stream)
        return SolveResult(Xs.t() if Xs is not None else None, None, eta, status)

    def solve_vec(self, shifts, bhat, outputs=SHS_OUT_X | SHS_OUT_ETA, stream=None):
        """(H - sigma_j I) x_j = R b_j for an (m, s) complex tensor of directions
        b_j (Section 3.3); returns a :class:`SolveResult` with X (n, s)."""
        import torch
        shifts = torch.as_tensor(shifts, dtype=torch.complex128, device=self.device).reshape(-1).contiguous()
        s = shifts.numel()
        bs = torch.as_tensor(bhat, dtype=torch.complex128, device=self.device).reshape(self.m, s).t().contiguous()
        Xs = torch.empty((s, self.n), dtype=torch.complex128, device=self.device)
        eta = torch.empty(s, dtype=torch.float64, device=self.device) if outputs & SHS_OUT_ETA else None
        status = torch.empty(s, dtype=torch.int32, device=self.device)
        shs_solve_vec(self.handle, shifts, bs, Xs, eta, status, outputs=outputs, stream=stream)
        return SolveResult(Xs.t(), None, eta, status)

    def solve_transposed_vec(self, shifts, chat, outputs=SHS_OUT_X | SHS_OUT_ETA, stream=None):
        """(H - sigma_j I)^T w_j = Ct^T c_j for a (p, s) complex tensor of
        directions c_j (Section 3.3); returns a :class:`SolveResult` with X = W (n, s)."""
        import torch
        shifts = torch.as_tensor(shifts, dtype=torch.complex128, device=self.device).reshape(-1).contiguous()
        s = shifts.numel()
        cs = (torch.as_tensor(chat, dtype=torch.complex128, device=self.device).reshape(self.p, s).t().contiguous()
              if self.p > 0 else None)
        Xs = torch.empty((s, self.n), dtype=torch.complex128, device=self.device) if outputs & SHS_OUT_X else None
        eta = torch.empty(s, dtype=torch.float64, device=self.device) if outputs & SHS_OUT_ETA else None
        status = torch.empty(s, dtype=torch.int32, device=self.device)
        shs_solve_transposed_vec(self.handle, shifts, cs, Xs, eta, status, outputs=outputs, stream=stream)
        return SolveResult(Xs.t() if Xs is not None else None, None, eta, status)

    def transfer_norm2(self, G, stream=None):
        """||G_j||_2 per block of a (p, s*m) complex tensor G (e.g. SolveResult.G):
        the quantity the structured pseudospectrum thresholds (Section 1)."""
        import torch
        m = self.m
        s = G.shape[1] // m
        Gs = G.t().contiguous() if self.p > 0 else torch.zeros((s * m, 1), dtype=torch.complex128,
                                                                device=self.device)
        out = torch.empty(s, dtype=torch.float64, device=self.device)
        shs_transfer_norm2(Gs[:, : self.p] if self.p > 0 else Gs[:, :0], m, out, stream)
        return out

    def pseudospectrum(self, points, mode=SHS_MODE_FP32_REFINE, tol=1e-13, max_iter=5, stream=None):
        """Structured pseudospectrum data on a set of points z: returns
        (||C (zI - A)^{-1} B||_2 per point, the solve's eta, status).  A point
        lies in the structured epsilon-pseudospectrum when its value is at
        least 1/epsilon (Section 1)."""
        res = self.solve(points, mode=mode, outputs=SHS_OUT_G | SHS_OUT_ETA, tol=tol, max_iter=max_iter,
                         stream=stream)
        return self.transfer_norm2(res.G, stream), res.eta, res.status

    def apply_q(self, X, stream=None):
        """Q X for an (n, k) complex128 tensor of reduced-coordinate columns."""
        import torch
        Xs = X.t().contiguous()
        out = torch.empty_like(Xs)
        shs_apply_q(self.handle, Xs, out, stream)
        return out.t()


@dataclasses.dataclass
class Request:
    id: int
    system: "System"
    X: object
    G: object
    eta: object
    status: object

    def result(self):
        s = self.status.numel()
        m, p = self.system.m, self.system.p
        X = self.X.t() if self.X is not None else None
        G = self.G.t()[:p] if self.G is not None else None
        return SolveResult(X, G, self.eta, self.status)


class Server:
    """Continuous-batching server over resident systems (see shs_server_* in shiftsolve.h)."""

    def __init__(self, streams=4, budget_bytes=64 << 30, max_batch=64, blocked_flops=0.0):
        self.handle = shs_server_create(streams, budget_bytes, max_batch, blocked_flops)
        self.systems = []

    def register(self, system: "System") -> int:
        sid = shs_server_register(self.handle, system.handle)
        self.systems.append(system)
        return sid

    def submit(self, sys_id, shifts, mode=SHS_MODE_FP64, outputs=SHS_OUT_X | SHS_OUT_G | SHS_OUT_ETA,
               arrival_s=0.0) -> Request:
        """Queue a request.  Its outputs are allocated on the current stream,
        and the request's work is ordered after that stream (no device-wide
        wait); ``arrival_s`` (on :func:`shs_server_clock`) starts its latency."""
        import numpy as np
        import torch
        sysm = self.systems[sys_id]
        shifts = np.asarray(shifts, dtype=np.complex128).reshape(-1)
        s, n, m, p = shifts.size, sysm.n, sysm.m, sysm.p
        X = torch.empty((s * m, n), dtype=torch.complex128, device=sysm.device) if outputs & SHS_OUT_X else None
        G = (torch.empty((s * m, max(1, p)), dtype=torch.complex128, device=sysm.device)
             if (outputs & SHS_OUT_G) and p > 0 else None)
        eta = (torch.empty(s, dtype=torch.float64, device=sysm.device)
               if (outputs & SHS_OUT_ETA) or mode == SHS_MODE_FP32_REFINE else None)
        status = torch.empty(s, dtype=torch.int32, device=sysm.device)
        rid = shs_server_submit_ex(self.handle, sys_id, shifts, X, G, eta, status, mode=mode, outputs=outputs,
                                   after_stream=torch.cuda.current_stream(), order_after=True, arrival_s=arrival_s)
        return Request(rid, sysm, X, G, eta, status)

    def cancel(self, req: Request):
        shs_server_cancel(self.handle, req.id)

    def pause(self, paused=True):
        shs_server_pause(self.handle, paused)

    def wait(self, req: Request, timeout_ms=-1.0):
        shs_server_wait(self.handle, req.id, timeout_ms)
        return req.result()

    def poll(self, req: Request) -> int:
        return shs_server_poll(self.handle, req.id)

    def latency_ms(self, req: Request) -> float:
        return shs_server_latency(self.handle, req.id)

    def stats(self):
        return shs_server_stats(self.handle)

    def close(self):
        if self.handle is not None:
            shs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
