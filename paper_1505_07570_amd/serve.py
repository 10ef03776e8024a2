"""Serving loop for randomized SVD and sketched least-squares requests.

Requests of different sizes arrive over time.  The loop

* admits them in arrival order under a device-memory budget (the native
  first-come-first-served scheduler, ``rmm_sched_*``): a request holds the
  bytes of its matrix, right-hand side, outputs and workspace while it runs;
* generates each admitted request's matrix on the device from its seed;
* groups the admitted LSR requests into one batch whose CountSketch sketches
  run as one grouped launch per stage (``rmm_sketch_batch``), then solves
  each sketched system (``rmm_lsr_solve``) and forms its residual;
* runs rsvd requests with ``rmm_rsvd``;
* spreads successive batches over a pool of streams (one library handle and
  workspace per stream) so that small problems overlap;
* completes a request when the event recorded after its last launch has
  fired, and records its latency from arrival.

``run_plain`` is the comparator: the same library calls, one request at a
time, in arrival order, on one stream, without grouping.
"""

from __future__ import annotations

import math
import time

import torch

from . import Handle, RmmError, Scheduler

LSR_SKETCH = "countsketch"


def lsr_sketch_size(m: int, n: int) -> int:
    return min(m, 4 * n)


def rsvd_params(n: int):
    """(k, p, q) of an rsvd request on an n-column matrix."""
    return max(1, n // 8), 10, 2


def request_bytes(h: Handle, req) -> int:
    """Device bytes a request holds while it runs (matrix, outputs, workspace)."""
    import ctypes
    from . import F32, KINDS, PREC_NATIVE, lib, _check
    m, n = req["m"], req["n"]
    nbytes = 4 * m * n
    ws = ctypes.c_size_t()
    if req["kind"] == "lsr":
        s = lsr_sketch_size(m, n)
        nbytes += 4 * m + 4 * s * (n + 1) + 8 * n
        _check(lib().rmm_sketch_workspace(h._h, F32, KINDS[LSR_SKETCH], m, n + 1, s, ctypes.byref(ws)),
               "rmm_sketch_workspace")
        w1 = ws.value
        _check(lib().rmm_lsr_solve_workspace(h._h, s, n, ctypes.byref(ws)), "rmm_lsr_solve_workspace")
        nbytes += max(w1, ws.value)
    else:
        k, p, _ = rsvd_params(n)
        nbytes += 4 * (m * k + k + n * k)
        _check(lib().rmm_rsvd_workspace(h._h, F32, PREC_NATIVE, m, n, k, p, ctypes.byref(ws)),
               "rmm_rsvd_workspace")
        nbytes += ws.value
    return nbytes


def _solve_one(h: Handle, req, A, b):
    """The library calls of one request (no grouping)."""
    m, n = req["m"], req["n"]
    if req["kind"] == "lsr":
        s = lsr_sketch_size(m, n)
        C = h.sketch(A, s, LSR_SKETCH, req["seed"], b=b)
        x, st = h.lsr_solve(C, n)
        return {"x": x, "resid": h.residual(A, b, x), "status": st}
    k, p, q = rsvd_params(n)
    U, sig, V, st = h.rsvd(A, k, p, q, req["seed"])
    return {"U": U, "sigma": sig, "V": V, "status": st}


def run_plain(requests, arrivals, make_input, device=None):
    """One request at a time, in arrival order, on one stream."""
    h = Handle(device)
    out, lat = {}, {}
    t0 = time.perf_counter()
    for rid in sorted(range(len(requests)), key=lambda i: arrivals[i]):
        while time.perf_counter() - t0 < arrivals[rid]:
            pass
        A, b = make_input(requests[rid])
        out[rid] = _solve_one(h, requests[rid], A, b)
        torch.cuda.synchronize()
        lat[rid] = time.perf_counter() - t0 - arrivals[rid]
    return out, lat, time.perf_counter() - t0


class Server:
    """The serving loop; see the module docstring."""

    def __init__(self, budget_bytes: int, streams: int = 4, device=None, max_batch: int = 64):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.handles = [Handle(self.device) for _ in range(streams)]
        self.sched = Scheduler(budget_bytes)
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.peak_bytes = 0
        self.rejected = []

    def _launch(self, slot, batch, requests, make_input):
        """Enqueue one admitted batch on stream `slot`; returns {rid: (event, outputs, inputs)}."""
        h, st = self.handles[slot], self.streams[slot]
        done = {}
        with torch.cuda.stream(st):
            inputs = {rid: make_input(requests[rid]) for rid in batch}
            lsr = [rid for rid in batch if requests[rid]["kind"] == "lsr"]
            if lsr:
                probs = []
                for rid in lsr:
                    r = requests[rid]
                    A, b = inputs[rid]
                    probs.append((A, b, lsr_sketch_size(r["m"], r["n"]), r["seed"]))
                Cs = h.sketch_batch(LSR_SKETCH, probs)
                for rid, C in zip(lsr, Cs):
                    A, b = inputs[rid]
                    x, stt = h.lsr_solve(C, requests[rid]["n"])
                    res = h.residual(A, b, x)
                    ev = torch.cuda.Event()
                    ev.record(st)
                    done[rid] = (ev, {"x": x, "resid": res, "status": stt}, inputs[rid])
            for rid in batch:
                if requests[rid]["kind"] != "rsvd":
                    continue
                A, _ = inputs[rid]
                out = _solve_one(h, requests[rid], A, None)
                ev = torch.cuda.Event()
                ev.record(st)
                done[rid] = (ev, out, inputs[rid])
        return done

    def run(self, requests, arrivals, make_input):
        """Serve `requests` arriving at `arrivals` (seconds from start).

        Returns (outputs by id, latency by id, wall seconds)."""
        order = sorted(range(len(requests)), key=lambda i: arrivals[i])
        nbytes = {rid: request_bytes(self.handles[0], requests[rid]) for rid in order}
        inflight, out, lat = {}, {}, {}
        nxt, slot = 0, 0
        t0 = time.perf_counter()
        while nxt < len(order) or inflight or self.sched.stats()["queued"]:
            now = time.perf_counter() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                try:
                    self.sched.submit(order[nxt], nbytes[order[nxt]])
                except RmmError:
                    self.rejected.append(order[nxt])  # larger than the whole budget
                nxt += 1
            admitted = self.sched.admit(self.max_batch)
            if admitted:
                inflight.update(self._launch(slot, admitted, requests, make_input))
                slot = (slot + 1) % len(self.streams)
                self.peak_bytes = max(self.peak_bytes, self.sched.stats()["in_use"])
            for rid in [r for r, v in inflight.items() if v[0].query()]:
                _, o, _ = inflight.pop(rid)
                out[rid] = o
                lat[rid] = time.perf_counter() - t0 - arrivals[rid]
                self.sched.complete(rid)
            if not admitted and nxt < len(order) and not inflight:
                # idle until the next arrival
                while time.perf_counter() - t0 < arrivals[order[nxt]]:
                    pass
        torch.cuda.synchronize()
        return out, lat, time.perf_counter() - t0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
