"""Serving loop for IterNCGP: continuous batching of predictive queries on a
resident fitted model, with new fits of uneven size admitted by an HBM budget.

Device work:

* Predictive queries (mean, marginal variance and probit probabilities at a
  set of test points, the predictive equations of the IterGP posterior) are
  packed, in arrival order, into prediction batches of at most
  ``max_batch_rows`` test points.  One itergp_predict call serves a batch.
  Up to ``slots`` batches are queued on the prediction stream at a time, each
  with its own preallocated device workspace and pinned host staging, so a
  query that arrives while others are on the device joins the next batch as
  soon as a slot frees up.  A query larger than a batch is served in pieces.
* Fits (Algorithm 1 on new training data) run in worker threads, each on its
  own stream with its own model, and overlap the prediction batches on the
  device.  The library releases the interpreter lock inside its calls.  A fit
  advances a few solver iterations at a time and, between them, waits while
  prediction batches are queued or running (at most ``fit_yield_ms`` per
  slice), so that queries do not queue behind a fit's products.

Admission: the resident model and the prediction slots are charged to the HBM
budget when the server starts.  A fit is charged its model arena plus its
inputs; fits start in arrival order as budget and workers free up, and a fit
that could not fit with nothing else running is refused.

Every prediction launch splits the training rows at fixed boundaries, so a
test point's result does not depend on the other points in its batch: each
result is bitwise the one the same query gets when served alone.
"""
from __future__ import annotations

import dataclasses
import math
import threading
import time
from collections import deque
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np
import torch

from . import _lib as L
from . import api

_ALIGN = 256


def _aligned(n: int) -> int:
    return (int(n) + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclasses.dataclass
class Ticket:
    """One request and, once served, its result and timing (server clock, s)."""

    rid: int
    kind: str                      # "predict" or "fit"
    t_arrive: float
    rows: int                      # test points (predict) or training points (fit)
    payload: dict = dataclasses.field(default_factory=dict, repr=False)
    status: str = "queued"         # queued, running, done, refused, failed
    error: str = ""
    t_start: float = math.nan
    t_done: float = math.nan
    result: Optional[dict] = dataclasses.field(default=None, repr=False)
    bytes: int = 0                 # budget charged (fits)
    served_rows: int = 0           # rows already placed in a batch (predict)
    done_rows: int = 0             # rows whose results are back (predict)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class HBMBudget:
    """Byte accounting for device memory; thread-safe."""

    def __init__(self, total: int):
        self.total = int(total)
        self.used = 0
        self._lock = threading.Lock()

    def try_reserve(self, n: int) -> bool:
        with self._lock:
            if self.used + n > self.total:
                return False
            self.used += n
            return True

    def release(self, n: int) -> None:
        with self._lock:
            self.used -= n
            if self.used < 0:
                raise RuntimeError("budget released more than reserved")

    @property
    def free(self) -> int:
        with self._lock:
            return self.total - self.used


def plan_batch(queue: Deque[Ticket], max_rows: int) -> List[Tuple[Ticket, int, int]]:
    """Take up to ``max_rows`` test points from the head of ``queue`` in
    arrival order: a list of (ticket, first row, row count).  A ticket whose
    rows are all placed leaves the queue; a partly placed one stays at the
    head with ``served_rows`` advanced."""
    out = []
    room = max_rows
    while queue and room > 0:
        t = queue[0]
        k = min(room, t.rows - t.served_rows)
        out.append((t, t.served_rows, k))
        t.served_rows += k
        room -= k
        if t.served_rows == t.rows:
            queue.popleft()
    return out


def admit_fits(queue: Deque[Ticket], budget: HBMBudget, capacity: int,
               free_workers: int) -> Tuple[List[Ticket], List[Ticket]]:
    """Fits that start now and fits refused, in arrival order.  ``capacity``
    is what fits may ever use (the budget less the resident part).  The head
    of the queue blocks later fits while it waits for budget."""
    start, refused = [], []
    while queue:
        t = queue[0]
        if t.bytes > capacity:
            refused.append(queue.popleft())
            continue
        if free_workers <= 0 or not budget.try_reserve(t.bytes):
            break
        start.append(queue.popleft())
        free_workers -= 1
    return start, refused


def fit_bytes(N: int, D: int, C: int, cfg: dict) -> int:
    """Budget charge of a fit: the model arena, X (FP32) and y (int32)."""
    return (_aligned(api.state_bytes(N, D, C, **cfg)) + _aligned(N * D * 4)
            + _aligned(N * 4))


class _Slot:
    """Preallocated buffers of one prediction batch in flight."""

    def __init__(self, model: api.IterNCGP, rows: int, device):
        D, C = model.D, model.C
        self.ws = torch.empty(max(model.predict_ws_bytes(rows), 1), dtype=torch.uint8,
                              device=device)
        self.x_dev = torch.empty((rows, D), dtype=model.dtype, device=device)
        self.out_dev = torch.empty((3, rows * C), dtype=model.dtype, device=device)
        self.x_host = torch.empty((rows, D), dtype=model.dtype).pin_memory()
        self.out_host = torch.empty((3, rows * C), dtype=model.dtype).pin_memory()
        self.event = torch.cuda.Event()
        self.parts: List[Tuple[Ticket, int, int]] = []
        self.rows = 0

    @staticmethod
    def nbytes(model: api.IterNCGP, rows: int) -> int:
        esz = torch.empty(0, dtype=model.dtype).element_size()
        return (_aligned(model.predict_ws_bytes(rows)) + _aligned(rows * model.D * esz)
                + _aligned(3 * rows * model.C * esz))


class Server:
    """Continuous-batching server for one resident fitted model.

    model           fitted api.IterNCGP (compressed for serving if wanted)
    budget_bytes    HBM budget for the resident model, the slots and fits
    max_batch_rows  test points per prediction batch
    slots           prediction batches in flight at a time
    fit_workers     fits running at a time
    fit_config      solver configuration of fits (api.solver_config keywords),
                    plus "steps" (Newton steps per fit)
    fit_slice       solver iterations a fit runs between checks for queries
    fit_yield_ms    longest a fit waits for queries per slice (0: no yielding)
    """

    def __init__(self, model: api.IterNCGP, budget_bytes: int, max_batch_rows: int = 8192,
                 slots: int = 2, fit_workers: int = 2, fit_config: Optional[dict] = None,
                 fit_slice: int = 2, fit_yield_ms: float = 25.0):
        self.model = model
        self.device = model.arena.device
        self.budget = HBMBudget(budget_bytes)
        self.max_rows = int(max_batch_rows)
        self.resident = _aligned(model.arena.numel()) + _aligned(model.N * 4)
        need = self.resident + slots * _Slot.nbytes(model, self.max_rows)
        if not self.budget.try_reserve(need):
            raise ValueError(f"budget of {budget_bytes} bytes below the resident model and "
                             f"prediction slots ({need} bytes)")
        self.fit_capacity = self.budget.total - need
        self.stream = torch.cuda.Stream(device=self.device)
        self.free_slots = [_Slot(model, self.max_rows, self.device) for _ in range(slots)]
        self.inflight: Deque[_Slot] = deque()
        self.pq: Deque[Ticket] = deque()
        self.fq: Deque[Ticket] = deque()
        self.fit_workers = int(fit_workers)
        # one stream per worker, reused, so freed fit memory is reused too
        self.fit_streams = [torch.cuda.Stream(device=self.device) for _ in range(fit_workers)]
        self.fit_config = dict(fit_config or {})
        self.fit_steps = int(self.fit_config.pop("steps", 2))
        self.fit_slice = max(int(fit_slice), 1)
        self.fit_yield_s = max(float(fit_yield_ms), 0.0) / 1e3
        self.tickets: List[Ticket] = []
        self._running = 0
        self._lock = threading.Lock()
        self._threads: List[threading.Thread] = []
        self.t0 = time.perf_counter()
        self.batches = 0
        self.batch_rows: List[int] = []

    # ---- clock and submission -------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit_predict(self, X: np.ndarray, t_arrive: Optional[float] = None) -> Ticket:
        """A predictive query at the rows of X (n x D)."""
        X = np.ascontiguousarray(X, dtype=np.float32 if self.model.dtype == torch.float32
                                 else np.float64)
        if X.ndim != 2 or X.shape[1] != self.model.D:
            raise ValueError(f"query must be n x {self.model.D}")
        t = Ticket(len(self.tickets), "predict", self.now() if t_arrive is None else t_arrive,
                   X.shape[0], {"X": X})
        C = self.model.C
        t.result = {k: np.empty((X.shape[0], C), dtype=X.dtype) for k in ("mean", "var", "probs")}
        self.tickets.append(t)
        if t.rows == 0:
            t.status, t.t_start, t.t_done = "done", t.t_arrive, t.t_arrive
        else:
            self.pq.append(t)
        return t

    def submit_fit(self, X: np.ndarray, y: np.ndarray, C: int, kind, lengthscale: float,
                   outputscale: float, t_arrive: Optional[float] = None) -> Ticket:
        """A new fit: Newton steps of Algorithm 1 on (X, y); the result holds the
        final latent values f (N x C) and the per-step solver records."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.int32)
        t = Ticket(len(self.tickets), "fit", self.now() if t_arrive is None else t_arrive,
                   X.shape[0], {"X": X, "y": y, "C": int(C), "kind": kind,
                                "lengthscale": float(lengthscale),
                                "outputscale": float(outputscale)})
        t.bytes = fit_bytes(X.shape[0], X.shape[1], C, self.fit_config)
        self.tickets.append(t)
        self.fq.append(t)
        return t

    # ---- prediction batches ---------------------------------------------
    def _launch_batch(self) -> None:
        slot = self.free_slots.pop()
        parts = plan_batch(self.pq, self.max_rows)
        rows = 0
        now = self.now()
        for t, a, k in parts:
            if t.status == "queued":
                t.status, t.t_start = "running", now
            slot.x_host[rows:rows + k].numpy()[:] = t.payload["X"][a:a + k]
            rows += k
        slot.parts, slot.rows = parts, rows
        C = self.model.C
        with torch.cuda.stream(self.stream):
            xd = slot.x_dev[:rows]
            xd.copy_(slot.x_host[:rows], non_blocking=True)
            out = slot.out_dev[:, :rows * C]
            self.model.predict_into(xd, slot.out_dev[0, :rows * C], slot.out_dev[1, :rows * C],
                                    slot.out_dev[2, :rows * C], slot.ws, self.stream)
            slot.out_host[:, :rows * C].copy_(out, non_blocking=True)
            slot.event.record(self.stream)
        self.inflight.append(slot)
        self.batches += 1
        self.batch_rows.append(rows)

    def _complete_batches(self) -> bool:
        progressed = False
        while self.inflight and self.inflight[0].event.query():
            slot = self.inflight.popleft()
            now = self.now()
            C = self.model.C
            host = slot.out_host.numpy()
            row = 0
            for t, a, k in slot.parts:
                for i, key in enumerate(("mean", "var", "probs")):
                    t.result[key][a:a + k] = host[i, row * C:(row + k) * C].reshape(k, C)
                row += k
                t.done_rows += k
                if t.done_rows == t.rows:
                    t.status, t.t_done = "done", now
            slot.parts = []
            self.free_slots.append(slot)
            progressed = True
        return progressed

    # ---- fits -----------------------------------------------------------
    def _run_fit(self, t: Ticket, s: torch.cuda.Stream) -> None:
        m = X = y = None
        try:
            with torch.cuda.stream(s):
                p = t.payload
                X = torch.from_numpy(p["X"]).to(self.device)
                y = torch.from_numpy(p["y"]).to(self.device)
                m = api.IterNCGP(X, y, p["C"], p["kind"], p["lengthscale"], p["outputscale"],
                                 **self.fit_config)
                infos = []
                for _ in range(self.fit_steps):
                    m.step_begin()
                    while True:
                        self._yield_to_queries()
                        if m.step_iterate(self.fit_slice):
                            break
                    infos.append(m.step_end())
                f = m.view(L.IGP_VIEW_F).cpu().numpy().reshape(t.rows, p["C"])
            t.result = {"f": f, "steps": infos}
            t.status = "done"
        except Exception as e:   # reported on the ticket; the server keeps going
            t.status, t.error = "failed", f"{type(e).__name__}: {e}"
        finally:
            del m, X, y
            t.t_done = self.now()
            self.budget.release(t.bytes)
            with self._lock:
                self._running -= 1
                self.fit_streams.append(s)

    def _yield_to_queries(self) -> None:
        """Called by fit workers between solver slices: wait while prediction
        batches are queued or on the device, for at most fit_yield_ms."""
        if self.fit_yield_s <= 0.0:
            return
        t_end = time.perf_counter() + self.fit_yield_s
        while (self.pq or self.inflight) and time.perf_counter() < t_end:
            time.sleep(5e-5)

    def _admit_fits(self) -> bool:
        with self._lock:
            free = self.fit_workers - self._running
        start, refused = admit_fits(self.fq, self.budget, self.fit_capacity, free)
        now = self.now()
        for t in refused:
            t.status, t.t_done = "refused", now
            t.error = f"needs {t.bytes} bytes, {self.fit_capacity} available to fits"
        for t in start:
            t.status, t.t_start = "running", now
            with self._lock:
                self._running += 1
                s = self.fit_streams.pop()
            th = threading.Thread(target=self._run_fit, args=(t, s), daemon=True)
            self._threads.append(th)
            th.start()
        return bool(start or refused)

    # ---- loop -------------------------------------------------------------
    def pump(self) -> bool:
        """One pass of the scheduler: collect finished batches, launch new ones
        while slots are free, start admitted fits.  True if anything moved."""
        progressed = self._complete_batches()
        while self.pq and self.free_slots:
            self._launch_batch()
            progressed = True
        progressed |= self._admit_fits()
        return progressed

    def idle(self) -> bool:
        with self._lock:
            running = self._running
        return not (self.pq or self.fq or self.inflight or running)

    def drain(self, poll_s: float = 2e-5) -> None:
        while not self.idle():
            if not self.pump():
                time.sleep(poll_s)
        for th in self._threads:
            th.join()
        self._threads = []

    def replay(self, requests: List[dict], realtime: bool = True,
               poll_s: float = 2e-5) -> List[Ticket]:
        """Serve a request stream.  Each request is a dict with "t" (arrival,
        seconds after the start of the replay), "kind" and its payload:
        "X" for a predict; "X", "y", "C", "kernel", "lengthscale",
        "outputscale" for a fit.  With ``realtime`` the requests are submitted
        at their arrival times, otherwise all at once."""
        reqs = sorted(requests, key=lambda r: r["t"])
        self.t0 = time.perf_counter()
        out, i = [], 0
        while True:
            now = self.now()
            while i < len(reqs) and (not realtime or reqs[i]["t"] <= now):
                r = reqs[i]
                ta = r["t"] if realtime else 0.0
                if r["kind"] == "predict":
                    out.append(self.submit_predict(r["X"], ta))
                else:
                    out.append(self.submit_fit(r["X"], r["y"], r["C"], r["kernel"],
                                               r["lengthscale"], r["outputscale"], ta))
                i += 1
            moved = self.pump()
            if i == len(reqs) and self.idle():
                break
            if not moved:
                wait = poll_s
                if i < len(reqs) and self.idle():
                    wait = max(poll_s, min(reqs[i]["t"] - self.now(), 1e-3))
                time.sleep(wait)
        for th in self._threads:
            th.join()
        self._threads = []
        return out


def latency_stats(tickets: List[Ticket], kind: str) -> Dict[str, float]:
    """p50 / p99 / mean latency (ms) of the served tickets of one kind."""
    lat = np.array([t.latency for t in tickets if t.kind == kind and t.status == "done"])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
