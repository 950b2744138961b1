"""Plain FP32 PyTorch form of IterNCGP on the GPU -- the comparison baseline
that ``bench.py`` times beside the HIP library.

The same Algorithms 1-3 (IterNCGP outer loop, IterGP with residual actions,
virtual solver run with compression) written with stock PyTorch operations:
products with K formed blockwise as |x|^2 + |x'|^2 - 2 X X'^T -> kernel ->
@ V (tiles of K discarded after use), the residual formed with a fresh
product as Algorithm 2 prints it, FP64 only for scalars and the B x B
eigendecomposition, TF32 disabled.  Problems run one at a time and
prediction requests are served one by one.  This is a baseline, not the
product path.
"""
from __future__ import annotations

import math

import numpy as np
import torch

LOG2E = 1.4426950408889634


class PlainIterNCGP:
    def __init__(self, X: torch.Tensor, y: torch.Tensor, C: int, kind: str, lengthscale: float,
                 outputscale: float, j_max: int = 200, rank_limit: int = 100,
                 tol_abs: float = 1e-5, tol_rel: float = 1e-5, block: int = 4096):
        torch.backends.cuda.matmul.allow_tf32 = False
        self.X = X.float().contiguous()
        self.y = y.long()
        self.N, self.C = X.shape[0], C
        self.kind, self.ell, self.os = kind, lengthscale, outputscale
        self.j_max, self.R = j_max, rank_limit
        self.tol_abs, self.tol_rel = tol_abs, tol_rel
        self.block = block
        self.sq = (self.X * self.X).sum(1)
        n = self.N * C
        dev = X.device
        self.f = torch.zeros(n, device=dev)
        self.S = torch.zeros(n, 0, device=dev)
        self.T = torch.zeros(n, 0, device=dev)
        self.v = torch.zeros(n, device=dev)
        self.Q = torch.zeros(n, 0, device=dev)

    def kfun(self, r2):
        r2 = r2.clamp_min(0) / (self.ell * self.ell)
        if self.kind == "rbf":
            return self.os * torch.exp(-0.5 * r2)
        r = torch.sqrt(r2)
        if self.kind == "matern12":
            return self.os * torch.exp(-r)
        if self.kind == "matern32":
            a = math.sqrt(3.0) * r
            return self.os * (1 + a) * torch.exp(-a)
        a = math.sqrt(5.0) * r
        return self.os * (1 + a + a * a / 3.0) * torch.exp(-a)

    def apply_K(self, V: torch.Tensor, X1: torch.Tensor = None) -> torch.Tensor:
        """(K_X(X1, X) (x) I_C) V for CN-ordered V of shape (N*C,) or (N*C, b)."""
        X1 = self.X if X1 is None else X1
        sq1 = (X1 * X1).sum(1)
        Vm = V.view(self.N, self.C, -1).reshape(self.N, -1)
        out = torch.empty(X1.shape[0], Vm.shape[1], device=V.device)
        for i0 in range(0, X1.shape[0], self.block):
            xb = X1[i0:i0 + self.block]
            r2 = sq1[i0:i0 + self.block, None] + self.sq[None, :] - 2.0 * (xb @ self.X.T)
            out[i0:i0 + self.block] = self.kfun(r2) @ Vm
        return out.reshape(-1) if V.dim() == 1 else out.reshape(X1.shape[0] * self.C, -1)

    def winv(self, pi: torch.Tensor, V: torch.Tensor) -> torch.Tensor:
        """W^+ V per point: P diag(1/pi) P with P = I - 11^T/C."""
        b = V.view(self.N, self.C, -1)
        u = b - b.mean(1, keepdim=True)
        w = u / pi.view(self.N, self.C, 1)
        return (w - w.mean(1, keepdim=True)).reshape(V.shape)

    def newton_step(self, j_max: int = None) -> dict:
        """One Newton step; ``j_max`` overrides the per-step action budget."""
        N, C = self.N, self.C
        jcap = self.j_max if j_max is None else int(j_max)
        F = self.f.view(N, C)
        pi = torch.softmax(F, dim=1)
        onehot = torch.nn.functional.one_hot(self.y, C).float()
        rhs = self.f + self.winv(pi.reshape(-1), (onehot - pi).reshape(-1))
        # Algorithm 3
        if self.S.shape[1] > 0:
            M = (self.S.T @ (self.T + self.winv(pi.reshape(-1), self.S))).double()
            lam, U = torch.linalg.eigh(0.5 * (M + M.T))
            lam, U = lam.flip(0), U.flip(1)
            B = lam.numel()
            keep = lam > lam[0] * B * 2.220446049250313e-16 if lam[0] > 0 else lam < -1
            lam, U = lam[keep], U[:, keep]
            if self.R >= 0:
                lam, U = lam[: self.R], U[:, : self.R]
            Uf = U.float()
            self.S, self.T = self.S @ Uf, self.T @ Uf
            self.Q = self.S / torch.sqrt(lam).float()[None, :]
        else:
            self.Q = self.S.clone()
        v = self.Q @ (self.Q.T @ rhs)
        thresh = max(self.tol_abs, self.tol_rel * float(rhs.double().norm()))
        j = 0
        while j < jcap:
            r = rhs - self.apply_K(v) - self.winv(pi.reshape(-1), v)
            rn = float(r.double().norm())
            if rn < thresh:
                break
            j += 1
            s = r / rn
            alpha = float(s.double() @ r.double())
            t = self.apply_K(s)
            self.S = torch.cat([self.S, s[:, None]], 1)
            self.T = torch.cat([self.T, t[:, None]], 1)
            z = t + self.winv(pi.reshape(-1), s)
            d = s - self.Q @ (self.Q.T @ z)
            eta = float(z.double() @ d.double())
            if eta <= 0:
                self.S, self.T = self.S[:, :-1], self.T[:, :-1]
                j -= 1
                break
            self.Q = torch.cat([self.Q, (d / math.sqrt(eta))[:, None]], 1)
            v = v + (alpha / eta) * d
        self.v = v
        fnew = self.apply_K(v)
        rel = float((fnew - self.f).double().norm() / fnew.double().norm())
        self.f = fnew
        return {"iters": j, "buffer_cols": self.S.shape[1], "rel_change": rel}

    def predict(self, Xs: torch.Tensor):
        mean = self.apply_K(self.v, Xs).view(-1, self.C)
        A = self.apply_K(self.Q, Xs) if self.Q.shape[1] else torch.zeros(Xs.shape[0] * self.C, 0,
                                                                           device=Xs.device)
        var = (self.os - (A * A).sum(1)).view(-1, self.C)
        probs = torch.softmax(mean / torch.sqrt(1 + math.pi / 8 * var.clamp_min(0)), dim=1)
        return mean, var, probs


def dense_k_comparison(X: torch.Tensor, C: int, kind: str, lengthscale: float,
                       outputscale: float, reps: int = 5, block: int = 4096) -> dict:
    """Dense-K-in-HBM FP32 form of the product: K(X, X) formed once (blockwise
    |x|^2 + |x'|^2 - 2 X X^T -> kernel, TF32 off) and kept in HBM as N^2 FP32
    values; each product K V with V of N x C is then one GEMM that streams K.
    Reported beside the fused product where K fits in free device memory."""
    torch.backends.cuda.matmul.allow_tf32 = False
    N = X.shape[0]
    kbytes = N * N * 4
    free, _ = torch.cuda.mem_get_info()
    if kbytes + 4 * block * N * 4 > 0.8 * free:
        return {"skipped": f"K needs {kbytes / 1e9:.1f} GB, {free / 1e9:.1f} GB free"}
    pm = PlainIterNCGP(X.float(), torch.zeros(N, dtype=torch.int32, device=X.device), C, kind,
                       lengthscale, outputscale, block=block)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    K = torch.empty(N, N, device=X.device)
    for i0 in range(0, N, block):
        xb = pm.X[i0:i0 + block]
        r2 = pm.sq[i0:i0 + block, None] + pm.sq[None, :] - 2.0 * (xb @ pm.X.T)
        K[i0:i0 + block] = pm.kfun(r2)
    e1.record()
    torch.cuda.synchronize()
    form_ms = e0.elapsed_time(e1)
    V = torch.randn(N, C, device=X.device)
    out = K @ V
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        out = K @ V
    e1.record()
    torch.cuda.synchronize()
    prod_ms = e0.elapsed_time(e1) / reps
    del K, out
    torch.cuda.empty_cache()
    return {"k_bytes": kbytes, "form_ms": form_ms, "product_ms": prod_ms,
            "k_stream_tb_per_s": kbytes / (prod_ms * 1e-3) / 1e12}


def fifo_replay(served: PlainIterNCGP, requests, fit_config: dict, steps: int,
                realtime: bool = True):
    """Serve a request stream one request at a time in arrival order (no
    batching, no overlap): predictive queries against ``served``, fits as new
    PlainIterNCGP models.  Returns (kind, arrival, done) per request, times in
    seconds from the start of the replay."""
    import time
    dev = served.X.device
    t0 = time.perf_counter()
    out = []
    for r in sorted(requests, key=lambda q: q["t"]):
        ta = r["t"] if realtime else 0.0
        if realtime:
            while time.perf_counter() - t0 < ta:
                time.sleep(2e-5)
        if r["kind"] == "predict":
            Xs = torch.from_numpy(np.ascontiguousarray(r["X"], dtype=np.float32)).to(dev)
            mean, var, probs = served.predict(Xs)
            torch.stack([mean, var, probs]).cpu()
        else:
            X = torch.from_numpy(np.ascontiguousarray(r["X"], dtype=np.float32)).to(dev)
            y = torch.from_numpy(np.ascontiguousarray(r["y"])).to(dev)
            m = PlainIterNCGP(X, y, r["C"], r["kernel"], r["lengthscale"], r["outputscale"],
                              **fit_config)
            for _ in range(steps):
                m.newton_step()
            m.f.cpu()
            del m
        torch.cuda.synchronize()
        out.append((r["kind"], ta, time.perf_counter() - t0))
    return out
