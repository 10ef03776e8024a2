"""Serving loop for randomized SVD and sketched least-squares requests.

Requests of different sizes arrive over time.  The loop

* admits them in arrival order under a device-memory budget (the native
  first-come-first-served scheduler, ``rmm_sched_*``).  Each stream's library
  handle gets one workspace, sized at start for the largest request shape the
  server accepts and charged against the budget once; a request holds the
  bytes of its own tensors (matrix, right-hand side, sketch and outputs)
  while it runs;
* places every admitted request on the stream with the least outstanding
  work (estimated from its size), so small requests are not queued behind
  large ones; LSR requests admitted together are split over the streams and
  each stream's share runs its CountSketch sketches as one grouped launch
  per stage (``rmm_sketch_batch``), then solves each sketched system
  (``rmm_lsr_solve``) and forms its residual; rsvd requests run
  ``rmm_rsvd``;
* generates each request's matrix on the device from its seed, on the
  request's stream right before its solve (the stand-in for its data
  arriving; the same generation is inside the plain comparator's latency);
* completes a request when the event recorded after its last launch has
  fired, records its latency from arrival and hands its outputs to the
  caller.

``run_plain`` is the comparator: the same library calls, one request at a
time, in arrival order, on one stream, without grouping.
"""

from __future__ import annotations

import math
import time

import torch

from . import Handle, RmmError, Scheduler

LSR_SKETCH = "countsketch"
MAX_SHAPE = (262144, 512)  # largest (m, n) the server sizes its workspaces for


def lsr_sketch_size(m: int, n: int) -> int:
    return min(m, 4 * n)


def rsvd_params(n: int):
    """(k, p, q) of an rsvd request on an n-column matrix."""
    return max(1, n // 8), 10, 2


def workspace_bytes(h: Handle, kind: str, m: int, n: int) -> int:
    """Library workspace of one request (held by its stream's handle)."""
    import ctypes
    from . import F32, KINDS, PREC_NATIVE, lib, _check
    ws = ctypes.c_size_t()
    if kind == "lsr":
        s = lsr_sketch_size(m, n)
        _check(lib().rmm_sketch_workspace(h._h, F32, KINDS[LSR_SKETCH], m, n + 1, s, ctypes.byref(ws)),
               "rmm_sketch_workspace")
        w1 = ws.value
        _check(lib().rmm_lsr_solve_workspace(h._h, s, n, ctypes.byref(ws)), "rmm_lsr_solve_workspace")
        w2 = ws.value
        _check(lib().rmm_residual_workspace(h._h, m, ctypes.byref(ws)), "rmm_residual_workspace")
        return max(w1, w2, ws.value)
    k, p, _ = rsvd_params(n)
    _check(lib().rmm_rsvd_workspace(h._h, F32, PREC_NATIVE, m, n, k, p, ctypes.byref(ws)),
           "rmm_rsvd_workspace")
    return ws.value


def _alloc(nbytes: int) -> int:
    """Bytes the caching allocator may charge for one tensor: 512-byte
    granules, and whole 2 MiB units from 1 MiB on (a large block can keep
    the unsplit tail of its segment)."""
    r = -(-max(nbytes, 1) // 512) * 512
    return -(-r // (2 << 20)) * (2 << 20) if r >= (1 << 20) else r


def request_bytes(req) -> int:
    """Device bytes of a request's own tensors, each at the allocator's
    granularity: its matrix with the temporaries of generating it (the spike
    factors; for LSR x*, the noise and b), the LSR sketch and the outputs."""
    m, n = req["m"], req["n"]
    k = max(1, n // 8)
    t = [4 * m * n, 4 * m * k, 4 * n * k]
    if req["kind"] == "lsr":
        s = lsr_sketch_size(m, n)
        t += [4 * n, 4 * m, 4 * m, 4 * m, 4 * m, 4 * s * (n + 1), 8 * n, 8, 4]
    else:
        kk, p, _ = rsvd_params(n)
        t += [4 * m * kk, 4 * kk, 4 * n * kk, 4]
    return sum(_alloc(x) for x in t)


def _cost(req) -> float:
    """Estimated device seconds of a request: a fixed chain of small launches
    plus its passes over A (2 for LSR, 2 q + 2 for rsvd) at 3 TB/s."""
    a = 4.0 * req["m"] * req["n"]
    if req["kind"] == "lsr":
        return 0.5e-3 + 2 * a / 3e12
    return 1.2e-3 + (2 * rsvd_params(req["n"])[2] + 2) * a / 3e12


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


def run_plain(requests, arrivals, make_input, device=None, on_done=None):
    """One request at a time, in arrival order, on one stream.  Returns
    (outputs by id (empty when on_done takes them), latency by id, wall seconds)."""
    h = Handle(device)
    out, lat = {}, {}
    t0 = time.perf_counter()
    for rid in sorted(range(len(requests)), key=lambda i: arrivals[i]):
        while time.perf_counter() - t0 < arrivals[rid]:
            pass
        A, b = make_input(requests[rid])
        o = _solve_one(h, requests[rid], A, b)
        torch.cuda.synchronize()
        lat[rid] = time.perf_counter() - t0 - arrivals[rid]
        if on_done:
            on_done(rid, o)
        else:
            out[rid] = o
    return out, lat, time.perf_counter() - t0


class Server:
    """The serving loop; see the module docstring."""

    def __init__(self, budget_bytes: int, streams: int = 4, device=None, max_batch: int = 64,
                 max_shape=MAX_SHAPE):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.handles = [Handle(self.device) for _ in range(streams)]
        m, n = max_shape
        self.ws_bytes = max(workspace_bytes(self.handles[0], kind, m, n) for kind in ("lsr", "rsvd"))
        self.reserved = streams * _alloc(self.ws_bytes)
        if self.reserved >= budget_bytes:
            raise ValueError("budget smaller than the streams' workspaces")
        for hd, st in zip(self.handles, self.streams):
            with torch.cuda.stream(st):
                hd.reserve(self.ws_bytes)
        self.max_shape = max_shape
        self.sched = Scheduler(budget_bytes - self.reserved)
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.peak_bytes = 0     # admitted request bytes plus the reserved workspaces
        self.rejected = []
        self.load = [0.0] * streams

    def _emit(self, slot, rid, outputs, inputs, done):
        ev = torch.cuda.Event()
        ev.record(self.streams[slot])
        done[rid] = (ev, outputs, inputs, slot)

    def _launch_lsr(self, slot, rids, requests, make_input, done):
        h, st = self.handles[slot], self.streams[slot]
        with torch.cuda.stream(st):
            inputs = {rid: make_input(requests[rid]) for rid in rids}
            probs = [(inputs[rid][0], inputs[rid][1],
                      lsr_sketch_size(requests[rid]["m"], requests[rid]["n"]), requests[rid]["seed"])
                     for rid in rids]
            Cs = h.sketch_batch(LSR_SKETCH, probs) if len(rids) > 1 else \
                [h.sketch(probs[0][0], probs[0][2], LSR_SKETCH, probs[0][3], b=probs[0][1])]
            for rid, C in zip(rids, Cs):
                A, b = inputs[rid]
                x, stt = h.lsr_solve(C, requests[rid]["n"])
                self._emit(slot, rid, {"x": x, "resid": h.residual(A, b, x), "status": stt}, inputs[rid],
                           done)

    def _launch_rsvd(self, slot, rid, requests, make_input, done):
        with torch.cuda.stream(self.streams[slot]):
            A, b = make_input(requests[rid])
            self._emit(slot, rid, _solve_one(self.handles[slot], requests[rid], A, None), (A, b), done)

    def _fit_groups(self, rids, requests):
        """Split LSR requests into runs whose grouped sketch fits the
        stream's reserved workspace (a grouped launch needs the partial
        slots of all its problems at once)."""
        h = self.handles[0]
        groups, cur = [], []
        for rid in rids:
            q = requests[rid]
            trial = cur + [rid]
            shapes = [(requests[r]["m"], requests[r]["n"], True,
                       lsr_sketch_size(requests[r]["m"], requests[r]["n"])) for r in trial]
            if cur and h.sketch_batch_workspace(LSR_SKETCH, shapes) > self.ws_bytes:
                groups.append(cur)
                cur = [rid]
            else:
                cur = trial
        if cur:
            groups.append(cur)
        return groups

    def _least_loaded(self):
        return min(range(len(self.streams)), key=lambda i: self.load[i])

    def _place(self, admitted, requests, make_input):
        """Enqueue the admitted requests; returns {rid: (event, outputs, inputs, slot)}."""
        done = {}
        lsr = [rid for rid in admitted if requests[rid]["kind"] == "lsr"]
        rsvd = [rid for rid in admitted if requests[rid]["kind"] != "lsr"]
        ns = len(self.streams)
        for g in range(min(ns, len(lsr))):
            for group in self._fit_groups(lsr[g::ns], requests):
                slot = self._least_loaded()
                self.load[slot] += sum(_cost(requests[r]) for r in group)
                self._launch_lsr(slot, group, requests, make_input, done)
        for rid in rsvd:
            slot = self._least_loaded()
            self.load[slot] += _cost(requests[rid])
            self._launch_rsvd(slot, rid, requests, make_input, done)
        return done

    def run(self, requests, arrivals, make_input, on_done=None):
        """Serve `requests` arriving at `arrivals` (seconds from start).

        Returns (outputs by id -- empty when on_done(rid, outputs) takes
        them --, latency by id, wall seconds)."""
        order = sorted(range(len(requests)), key=lambda i: arrivals[i])
        mm, nm = self.max_shape
        inflight, out, lat = {}, {}, {}
        nxt = 0
        t0 = time.perf_counter()
        while nxt < len(order) or inflight or self.sched.stats()["queued"]:
            now = time.perf_counter() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                rid = order[nxt]
                q = requests[rid]
                try:
                    if q["m"] > mm or q["n"] > nm:
                        raise RmmError(-1, "request larger than the server's workspaces")
                    self.sched.submit(rid, request_bytes(q))
                except RmmError:
                    self.rejected.append(rid)  # larger than the budget or the workspaces
                nxt += 1
            admitted = self.sched.admit(self.max_batch)
            if admitted:
                inflight.update(self._place(admitted, requests, make_input))
                self.peak_bytes = max(self.peak_bytes, self.sched.stats()["in_use"] + self.reserved)
            for rid in [r for r, v in inflight.items() if v[0].query()]:
                _, o, _, slot = inflight.pop(rid)
                lat[rid] = time.perf_counter() - t0 - arrivals[rid]
                self.load[slot] = max(0.0, self.load[slot] - _cost(requests[rid]))
                self.sched.complete(rid)
                if on_done:
                    on_done(rid, o)
                else:
                    out[rid] = o
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
