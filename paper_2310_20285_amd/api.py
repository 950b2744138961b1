"""PyTorch-facing binding of the C ABI (include/itergp.h).

Tensors are used only to hold device memory; every call hands raw device
pointers, sizes and the current HIP stream to the library, where all of the
arithmetic runs.  Names follow the C entry points.
"""
from __future__ import annotations

import ctypes as ct
from typing import Optional

import torch

from . import _lib as L

_DTYPE = {L.IGP_FP64: torch.float64, L.IGP_FP32: torch.float32, L.IGP_BF16: torch.float32,
          L.IGP_BF16X3: torch.float32}


def _prec(p) -> int:
    return L.PRECISION_CODE[p] if isinstance(p, str) else int(p)


def _kind(k) -> int:
    return L.KIND_CODE[k] if isinstance(k, str) else int(k)


def _stream() -> ct.c_void_p:
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ct.c_void_p:
    return ct.c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def kernel_params(kind, lengthscale, outputscale, C: int = 1):
    """(array of KernelParams, n_kp): one set shared by all classes, or one per
    class when lengthscale or outputscale is a sequence of C values."""
    per = [isinstance(a, (list, tuple)) or (hasattr(a, "__len__") and not isinstance(a, str))
           for a in (lengthscale, outputscale)]
    if not any(per):
        arr = (L.KernelParams * 1)(L.KernelParams(_kind(kind), 0, float(lengthscale),
                                                  float(outputscale)))
        return arr, 1
    ls = list(lengthscale) if per[0] else [lengthscale] * C
    os_ = list(outputscale) if per[1] else [outputscale] * C
    if len(ls) != C or len(os_) != C:
        raise ValueError(f"per-class hyperparameters need {C} values")
    arr = (L.KernelParams * C)(*[L.KernelParams(_kind(kind), 0, float(a), float(b))
                                 for a, b in zip(ls, os_)])
    return arr, C


def glm_kernel_matmul(X1: torch.Tensor, X2: torch.Tensor, V: torch.Tensor, C: int, kind,
                      lengthscale: float, outputscale: float, precision="fp32",
                      beta: float = 0.0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Out_b = (K_X(X1, X2) (x) I_C) V_b (+ beta Out_b).

    V: (n2*C,) or (nb, n2*C) -- each row one CN-ordered vector.  Returns a
    tensor of the same layout with n1*C entries per vector.
    """
    lib = L.load()
    p = _prec(precision)
    dt = _DTYPE[p]
    for t, nm in ((X1, "X1"), (X2, "X2"), (V, "V")):
        _need(t, dt, nm)
    n1, d = X1.shape
    n2 = X2.shape[0]
    vec = V.dim() == 1
    V2 = V.view(1, -1) if vec else V
    nb = V2.shape[0]
    if V2.shape[1] != n2 * C:
        raise ValueError("V rows must have n2*C entries")
    if out is None:
        out = torch.empty((nb, n1 * C), dtype=dt, device=X1.device)
    O2 = out.view(nb, n1 * C)
    wsb = lib.glm_kernel_matmul_ws_bytes(n1, n2, d, C, nb, p)
    ws = torch.empty(max(int(wsb), 1), dtype=torch.uint8, device=X1.device)
    kp, n_kp = kernel_params(kind, lengthscale, outputscale, C)
    L.check(lib.glm_kernel_matmul(kp, n_kp, _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V2), C, nb,
                                  n2 * C, _ptr(O2), n1 * C, float(beta), p, _ptr(ws), wsb,
                                  _stream()))
    return out.view(-1) if vec else out


def glm_kernel_matmul_noalloc(X1: torch.Tensor, X2: torch.Tensor, V: torch.Tensor, C: int, kind,
                              lengthscale: float, outputscale: float, precision="fp32",
                              beta: float = 0.0, out: Optional[torch.Tensor] = None
                              ) -> torch.Tensor:
    """glm_kernel_matmul through the entry point that allocates no workspace
    (its scratch is the library's static per-GPU array).  `out` may be given so
    that the call allocates nothing at all."""
    lib = L.load()
    p = _prec(precision)
    dt = _DTYPE[p]
    for t, nm in ((X1, "X1"), (X2, "X2"), (V, "V")):
        _need(t, dt, nm)
    n1, d = X1.shape
    n2 = X2.shape[0]
    vec = V.dim() == 1
    V2 = V.view(1, -1) if vec else V
    nb = V2.shape[0]
    if V2.shape[1] != n2 * C:
        raise ValueError("V rows must have n2*C entries")
    if out is None:
        out = torch.empty((nb, n1 * C), dtype=dt, device=X1.device)
    O2 = out.view(nb, n1 * C)
    kp, n_kp = kernel_params(kind, lengthscale, outputscale, C)
    L.check(lib.glm_kernel_matmul_noalloc(kp, n_kp, _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V2), C,
                                          nb, n2 * C, _ptr(O2), n1 * C, float(beta), p,
                                          _stream()))
    return out.view(-1) if vec else out


def glm_softmax_hessian_apply(F: torch.Tensor, V: torch.Tensor, mode="pinv",
                              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Out_n = W_n V_n (mode "w") or W_n^+ V_n (mode "pinv"); F is (N, C)."""
    lib = L.load()
    dt = F.dtype
    p = L.IGP_FP64 if dt == torch.float64 else L.IGP_FP32
    _need(F, dt, "F")
    _need(V, dt, "V")
    N, C = F.shape
    vec = V.dim() == 1
    V2 = V.view(1, -1) if vec else V
    nb = V2.shape[0]
    if out is None:
        out = torch.empty_like(V2)
    m = L.IGP_W_PINV if mode == "pinv" else L.IGP_W
    L.check(lib.glm_softmax_hessian_apply(_ptr(F), N, C, _ptr(V2), nb, N * C, _ptr(out), N * C,
                                          m, p, _stream()))
    return out.view(-1) if vec else out


_LIK = {"softmax": L.IGP_LIK_SOFTMAX, "poisson": L.IGP_LIK_POISSON,
        "gaussian": L.IGP_LIK_GAUSSIAN, "block": L.IGP_LIK_BLOCK}


def solver_config(policy="cg", j_max=100, rank_limit=-1, recycle=True, tol_abs=1e-5,
                  tol_rel=1e-5, precision="fp32", residual_mode="explicit",
                  max_buffer=None, likelihood="softmax", noise_var=1.0) -> L.SolverConfig:
    pol = {"cg": L.IGP_POLICY_CG, "unit": L.IGP_POLICY_UNIT, "user": L.IGP_POLICY_USER}[policy]
    rm = {"explicit": L.IGP_RESIDUAL_EXPLICIT,
          "recurrence": L.IGP_RESIDUAL_RECURRENCE}[residual_mode]
    if max_buffer is None:
        max_buffer = j_max + (rank_limit if rank_limit is not None and rank_limit >= 0 else j_max)
        max_buffer = max(max_buffer, 1)
    return L.SolverConfig(pol, int(j_max), int(-1 if rank_limit is None else rank_limit),
                          1 if recycle else 0, float(tol_abs), float(tol_rel), _prec(precision),
                          rm, int(max_buffer), _LIK[likelihood], float(noise_var))


def state_bytes(N: int, D: int, C: int, **cfg) -> int:
    """itergp_state_bytes: the arena a model of this shape and configuration needs."""
    c = solver_config(**cfg)
    return int(L.load().itergp_state_bytes(int(N), int(D), int(C), ct.byref(c)))


class IterNCGP:
    """A model handle: itergp_init / itergp_newton_step / itergp_predict."""

    def __init__(self, X: torch.Tensor, y: torch.Tensor, C: int, kind, lengthscale: float,
                 outputscale: float, **cfg):
        self.lib = L.load()
        self.cfg = solver_config(**cfg)
        self.precision = self.cfg.precision
        self.dtype = _DTYPE[self.precision]
        _need(X, self.dtype, "X")
        gaussian = self.cfg.likelihood == L.IGP_LIK_GAUSSIAN
        if self.cfg.likelihood != L.IGP_LIK_BLOCK or y is not None:
            _need(y, self.dtype if gaussian else torch.int32, "y")
        self.N, self.D = X.shape
        self.C = int(C)
        self.y = y                       # kept alive: the model reads it every step
        self.kp, self.n_kp = kernel_params(kind, lengthscale, outputscale, self.C)
        nbytes = self.lib.itergp_state_bytes(self.N, self.D, self.C, ct.byref(self.cfg))
        if nbytes == 0:
            raise ValueError("invalid model configuration")
        self.arena = torch.empty(int(nbytes), dtype=torch.uint8, device=X.device)
        self.stream = torch.cuda.current_stream()   # the model runs all its work here
        self.handle = ct.c_void_p()
        L.check(self.lib.itergp_init(ct.byref(self.handle), self.kp, self.n_kp,
                                     ct.byref(self.cfg), _ptr(X),
                                     None if y is None else _ptr(y), self.N, self.D,
                                     self.C, _ptr(self.arena), nbytes, _stream()))
        self._user = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.itergp_destroy(h)
            self.handle = None

    def newton_step(self) -> dict:
        info = L.StepInfo()
        L.check(self.lib.itergp_newton_step(self.handle, ct.byref(info)))
        return info.as_dict()

    def step_begin(self) -> None:
        """itergp_newton_step_begin: the start of a Newton step."""
        L.check(self.lib.itergp_newton_step_begin(self.handle))

    def step_iterate(self, max_iters: int = 1) -> bool:
        """Up to max_iters solver iterations; True once the solver has stopped."""
        done = ct.c_int32()
        L.check(self.lib.itergp_newton_step_iterate(self.handle, int(max_iters), ct.byref(done)))
        return bool(done.value)

    def step_end(self) -> dict:
        """itergp_newton_step_end: f = K v + m and the step record."""
        info = L.StepInfo()
        L.check(self.lib.itergp_newton_step_end(self.handle, ct.byref(info)))
        return info.as_dict()

    def set_block_likelihood(self, grad: torch.Tensor, W: torch.Tensor) -> None:
        """itergp_set_block_likelihood: grad (N*C,) and W (N, C, C) at the current f."""
        _need(grad, self.dtype, "grad")
        _need(W, self.dtype, "W")
        if grad.numel() != self.N * self.C or W.numel() != self.N * self.C * self.C:
            raise ValueError("grad must hold N*C values and W N*C*C")
        L.check(self.lib.itergp_set_block_likelihood(self.handle, _ptr(grad), _ptr(W)))

    def set_profiling(self, enable: bool = True, every: int = 1):
        """Turn product tracing on (timing every ``every``-th product) or off; resets."""
        L.check(self.lib.itergp_set_profiling(self.handle, int(every) if enable else 0))

    def profile(self) -> dict:
        p = L.Profile()
        L.check(self.lib.itergp_get_profile(self.handle, ct.byref(p)))
        return p.as_dict()

    def set_user_actions(self, actions: torch.Tensor):
        """actions: (ncols, N*C), row j is the action of iteration j+1."""
        _need(actions, self.dtype, "actions")
        self._user = actions
        L.check(self.lib.itergp_set_user_actions(self.handle, _ptr(actions), actions.shape[0],
                                                 actions.shape[1]))

    def view(self, which) -> torch.Tensor:
        """A copy of a state buffer: vectors as (N*C,), buffers as (cols, N*C)."""
        ptr, rows, cols, ld = ct.c_void_p(), ct.c_int64(), ct.c_int64(), ct.c_int64()
        L.check(self.lib.itergp_get_view(self.handle, which, ct.byref(ptr), ct.byref(rows),
                                         ct.byref(cols), ct.byref(ld)))
        self.stream.synchronize()
        esz = torch.empty(0, dtype=self.dtype).element_size()
        off = (ptr.value or 0) - self.arena.data_ptr()
        if cols.value == 0:
            return torch.empty((0, rows.value), dtype=self.dtype, device=self.arena.device)
        span = ((cols.value - 1) * ld.value + rows.value) * esz
        raw = self.arena[off:off + span]
        full = raw.view(self.dtype)
        if which in (L.IGP_VIEW_Q, L.IGP_VIEW_S, L.IGP_VIEW_T):
            out = torch.stack([full[b * ld.value: b * ld.value + rows.value]
                               for b in range(cols.value)])
            return out
        if which == L.IGP_VIEW_X:
            return full[: rows.value * cols.value].view(rows.value, cols.value).clone()
        return full[: rows.value].clone()

    def compress(self, rank_limit: int) -> int:
        """itergp_compress: Algorithm 3 over the stored buffer; returns the columns kept."""
        kept = ct.c_int32()
        L.check(self.lib.itergp_compress(self.handle, int(rank_limit), ct.byref(kept)))
        return kept.value

    def predict_ws_bytes(self, Ns: int) -> int:
        return int(self.lib.itergp_predict_ws_bytes(self.handle, int(Ns)))

    def predict(self, Xs: torch.Tensor, var: bool = True, probs: bool = True,
                ws: Optional[torch.Tensor] = None, stream=None):
        """Asynchronous on ``stream`` (default: the current stream).  ``ws``, when
        given, is a uint8 workspace of at least predict_ws_bytes(len(Xs)) bytes."""
        _need(Xs, self.dtype, "Xs")
        Ns = Xs.shape[0]
        mean = torch.empty(Ns * self.C, dtype=self.dtype, device=Xs.device)
        v = torch.empty_like(mean) if var else None
        p = torch.empty_like(mean) if (probs and var) else None
        wsb = self.lib.itergp_predict_ws_bytes(self.handle, Ns)
        if ws is None:
            ws = torch.empty(max(int(wsb), 1), dtype=torch.uint8, device=Xs.device)
        elif ws.numel() < wsb:
            raise ValueError(f"predict workspace of {ws.numel()} bytes, {wsb} needed")
        st = _stream() if stream is None else ct.c_void_p(stream.cuda_stream)
        L.check(self.lib.itergp_predict(self.handle, _ptr(Xs), Ns, _ptr(mean), _ptr(v), _ptr(p),
                                        _ptr(ws), wsb, st))
        shape = (Ns, self.C)
        return (mean.view(shape), None if v is None else v.view(shape),
                None if p is None else p.view(shape))

    def predict_into(self, Xs: torch.Tensor, mean: torch.Tensor, var: Optional[torch.Tensor],
                     probs: Optional[torch.Tensor], ws: torch.Tensor, stream) -> None:
        """itergp_predict into caller-owned buffers (Ns*C elements each, var and
        probs nullable), asynchronous on ``stream``; nothing is allocated."""
        Ns = Xs.shape[0]
        for t in (mean, var, probs):
            if t is not None and (t.numel() < Ns * self.C or not t.is_contiguous()):
                raise ValueError("output buffers must be contiguous with Ns*C elements")
        L.check(self.lib.itergp_predict(self.handle, _ptr(Xs), Ns, _ptr(mean), _ptr(var),
                                        _ptr(probs), _ptr(ws), ws.numel(),
                                        ct.c_void_p(stream.cuda_stream)))


def newton_step_batched(models, ws: Optional[torch.Tensor] = None, device_control: bool = False):
    """itergp_newton_step_batched over a list of IterNCGP models; with
    device_control the solver's control flow runs on the device
    (IGP_BATCH_DEVICE_CONTROL: windows of iterations, one host read each)."""
    lib = L.load()
    n = len(models)
    arr = (ct.c_void_p * n)(*[m.handle.value for m in models])
    wsb = lib.itergp_batched_ws_bytes(arr, n)
    if wsb == 0:
        raise L.IterGPError(L.IGP_EINVAL, lib.igp_last_error().decode() or "incompatible batch")
    if ws is None or ws.numel() < wsb:
        ws = torch.empty(int(wsb), dtype=torch.uint8, device="cuda")
    infos = (L.StepInfo * n)()
    flags = L.IGP_BATCH_DEVICE_CONTROL if device_control else 0
    L.check(lib.itergp_newton_step_batched_ex(arr, n, infos, _ptr(ws), wsb, flags))
    return [i.as_dict() for i in infos], ws


def batched_tuning() -> str:
    lib = L.load()
    buf = ct.create_string_buffer(1 << 16)
    L.check(lib.itergp_batched_tuning(buf, len(buf)))
    return buf.value.decode()


def batched_tuning_load(text: str) -> int:
    """itergp_batched_tuning_load: seed the batched launch-shape table from JSON
    (as batched_tuning() returns it); returns the number of entries added."""
    n = ct.c_int32()
    L.check(L.load().itergp_batched_tuning_load(text.encode(), ct.byref(n)))
    return n.value


def load_batched_tuning_file(path: str) -> int:
    """Seed the table from a JSON file written by save_batched_tuning_file."""
    with open(path) as f:
        return batched_tuning_load(f.read())


def save_batched_tuning_file(path: str) -> None:
    """Write the current launch-shape table as JSON."""
    with open(path, "w") as f:
        f.write(batched_tuning() + "\n")
