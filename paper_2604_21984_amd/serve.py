"""Serving loop for encoded images (random-access decode, Sec. 6.6: rendering from
cached top-K lists is the fast path).

* Resident sets: encoded site sets (derived records + list field) kept on the device.
* Requests: point queries (M points of one set), full renders (one set) and renders at a
  new resolution (Ho x Wo points over one set's image: the set's lists belong to its own
  pixel grid, so the request rebuilds lists on the new grid with a full refresh -- JFA
  prepass and 16 passes, Sec. 6.6 -- and renders from them).
* Admission by memory: a request is admitted when the device bytes it needs (its
  inputs and outputs) fit in what the budget has left; bytes return when it completes.
  A request that could never fit is rejected.
* Continuous batching: every scheduler turn launches whatever has been admitted since
  the last turn -- point queries of many requests across many sets as one
  ``sad_query_batch`` launch (a lone query: ``sad_query_points``, with no job table to
  upload), renders as their own launches -- on a pool of streams,
  without waiting for earlier launches; completions are found by polling events.
  Requests that arrive while others run are admitted as memory frees up and their work
  overlaps on the device with the work already there.
* A failing launch fails only the requests in it.
* Latency is arrival -> completion; p50 / p99 and throughput are reported.

The scheduler talks to a backend (``GpuBackend`` here; tests also drive it with a fake
backend with a simulated clock, memory and errors).
"""
import collections
import math
import threading
import time
from dataclasses import dataclass

QUERY, RENDER, RESCALE = "query", "render", "rescale"
RESCALE_PASSES = 16


@dataclass
class Request:
    rid: int
    set_id: int
    kind: str
    xy: object = None            # [M, 2] float32 device tensor (queries)
    M: int = 0
    t_arrival: float = 0.0
    t_admit: float = None
    t_launch: float = None
    t_done: float = None
    result: object = None
    error: str = None
    nbytes: int = 0
    ready: object = None         # backend marker: the request's inputs are written
    stream: object = None        # backend marker: the stream they are written on
    Ho: int = 0                  # output grid of a RESCALE request
    Wo: int = 0

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class ResidentSet:
    """One encoded image kept on the device."""

    def __init__(self, set_id, H, W, K, n_slots, rec, topk, score_scale=0.0):
        self.set_id, self.H, self.W, self.K, self.n_slots = set_id, H, W, K, n_slots
        self.rec, self.topk, self.score_scale = rec, topk, score_scale

    @classmethod
    def from_encoder(cls, set_id, enc):
        return cls(set_id, enc.H, enc.W, enc.cfg.K, enc.img.n_slots, enc.rec.clone(),
                   enc.topk.clone(), enc.cfg.score_scale)

    @classmethod
    def from_batch(cls, set_id, benc, b):
        H, W = benc.shapes[b]
        return cls(set_id, H, W, benc.K, benc.n_sites[b], benc.view_rec(b).clone(),
                   benc.view_list(benc.cur, b).clone(), benc.cfg.score_scale)

    def nbytes(self):
        return self.rec.numel() * 4 + self.topk.numel() * 4


def request_bytes(req, rset):
    """Device bytes a request holds while admitted: inputs, outputs and, for a render at a
    new resolution, the two list fields and the seed scratch of its refresh."""
    if req.kind == QUERY:
        return req.M * (8 + 12)
    if req.kind == RESCALE:
        return req.Ho * req.Wo * (12 + 2 * 4 * rset.K + 8)
    return 12 * rset.H * rset.W


class _OnStream:
    """Make `stream` the current stream of its device for a block (what
    torch.cuda.stream() does, without its per-call device lookups)."""
    __slots__ = ("C", "st", "prev")

    def __init__(self, C, st):
        self.C, self.st = C, st

    def __enter__(self):
        st = self.st
        # the current device's current stream: restoring it also restores the device
        self.prev = self.C._cuda_getCurrentStream(self.C._cuda_getDevice())
        if self.prev[0] == st.stream_id and self.prev[1] == st.device_index:
            self.prev = None           # already current
            return
        self.C._cuda_setStream(stream_id=st.stream_id, device_index=st.device_index,
                               device_type=st.device_type)

    def __exit__(self, *exc):
        if self.prev is not None:
            sid, di, dt = self.prev
            self.C._cuda_setStream(stream_id=sid, device_index=di, device_type=dt)


class GpuBackend:
    """Launches on a pool of default-priority HIP streams; completion via events.

    A request's inputs (the query points) may still be being written on the stream that
    was current when it was submitted: submit() records an event there, and every launch
    makes its stream wait for the events of its requests before reading their inputs.
    Events are pooled: a request's readiness event and a launch's completion event go
    back to the pool once the launch has been seen to finish (a readiness event is
    kept until then, so that a launch retried request by request waits again).  A
    direct launch (one request while nothing else is in flight, the scheduler's choice)
    runs on the stream the request's inputs were written on, which needs no wait: with
    no other launch to overlap, a pool stream would only add the wait's cost."""

    direct_launch = True   # the launch methods take direct=

    def __init__(self, device=None, n_streams=4):
        import torch

        from . import _lib as S
        self.torch, self.S = torch, S
        self.device = torch.device(device or "cuda")
        self.dev = (self.device.index if self.device.index is not None
                    else torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_streams)]
        self._next = 0
        self._images = {}  # (set id, shape, K, slots, scale) -> sad_image descriptor
        self._events = []  # free events
        self._callers = {}  # stream id -> Stream object of a submitting stream
        # torch's stream-id calls (no per-call device lookups); the public API otherwise
        self._fast = all(hasattr(torch._C, f) for f in ("_cuda_getCurrentStream",
                                                        "_cuda_setStream", "_cuda_getDevice"))

    def now(self):
        return time.perf_counter()

    def _event(self):
        return self._events.pop() if self._events else self.torch.cuda.Event()

    def _on(self, st):
        if self._fast:
            return _OnStream(self.torch._C, st)
        return self.torch.cuda.stream(st)

    def on_submit(self, req):
        if self._fast:
            sid, di, dt = self.torch._C._cuda_getCurrentStream(self.dev)
            caller = self._callers.get(sid)
            if caller is None:
                caller = self.torch.cuda.Stream(stream_id=sid, device_index=di, device_type=dt)
                self._callers[sid] = caller
        else:
            caller = self.torch.cuda.current_stream(self.device)
        ev = self._event()
        ev.record(caller)
        req.ready = ev
        req.stream = caller

    def _lane(self, reqs, direct):
        """The stream a launch runs on, its requests' inputs ordered before it: with
        direct, the one request's own submitting stream (stream order suffices); else
        the next pool stream, made to wait for every request's readiness event."""
        if direct and len(reqs) == 1 and reqs[0].stream is not None:
            return reqs[0].stream
        st = self._stream()
        self._wait_inputs(st, reqs)
        return st

    def _wait_inputs(self, st, reqs):
        for r in reqs:
            if r.ready is not None:   # kept until the launch is done: a retry waits again
                st.wait_event(r.ready)
            if r.xy is not None:
                r.xy.record_stream(st)   # the allocator keeps xy until st is done with it

    def free_bytes(self):
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return free

    def _stream(self):
        s = self.streams[self._next % len(self.streams)]
        self._next += 1
        return s

    def _image(self, rs):
        key = (rs.set_id, rs.H, rs.W, rs.K, rs.n_slots, rs.score_scale)
        img = self._images.get(key)
        if img is None:
            img = self.S.image(rs.H, rs.W, rs.K, rs.n_slots, rs.n_slots, rs.score_scale)
            self._images[key] = img
        return img

    def launch_queries(self, reqs, sets, direct=False):
        torch, S = self.torch, self.S
        K = sets[reqs[0].set_id].K
        n = len(reqs)
        if n == 1:  # one request: sad_query_points, with no job table to upload
            r, rs = reqs[0], sets[reqs[0].set_id]
            st = self._lane(reqs, direct)
            with self._on(st):
                out = torch.empty((r.M, 3), dtype=torch.float32, device=self.device)
                S.query_points(self._image(rs), rs.rec, rs.topk, r.xy, out)
                ev = self._event()
                ev.record(st)
            return {"event": ev, "reqs": reqs, "outs": [out], "keep": ()}
        arr = (S.SadQueryJob * n)()
        outs = []
        q0 = 0
        for j, r in enumerate(reqs):
            rs = sets[r.set_id]
            out = torch.empty((r.M, 3), dtype=torch.float32, device=self.device)
            outs.append(out)
            arr[j] = S.SadQueryJob(rs.rec.data_ptr(), rs.topk.data_ptr(), r.xy.data_ptr(),
                                   out.data_ptr(), r.M, q0, rs.H, rs.W, rs.n_slots, 0)
            q0 += r.M
        st = self._stream()
        self._wait_inputs(st, reqs)
        with self._on(st):
            host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).pin_memory()
            jobs = host.to(self.device, non_blocking=True)
            S.query_batch(jobs, n, q0, K)
            ev = self._event()
            ev.record(st)
        return {"event": ev, "reqs": reqs, "outs": outs, "keep": (host, jobs)}

    def launch_render(self, req, rset, direct=False):
        torch, S = self.torch, self.S
        st = self._lane([req], direct)
        with self._on(st):
            out = torch.empty((3, rset.H, rset.W), dtype=torch.float32, device=self.device)
            S.render_fwd(self._image(rset), rset.rec, rset.topk, out)
            ev = self._event()
            ev.record(st)
        return {"event": ev, "reqs": [req], "outs": [out], "keep": ()}

    def launch_rescale(self, req, rset, seed=0, direct=False):
        """A render of rset at req.Ho x req.Wo: refresh on that grid (JFA prepass and
        RESCALE_PASSES passes, J = 4), then render from the refreshed lists."""
        torch, S = self.torch, self.S
        st = self._lane([req], direct)
        Ho, Wo, K = req.Ho, req.Wo, rset.K
        with self._on(st):
            img = self._image(rset)
            a = torch.empty((K // 4, Ho, Wo, 4), dtype=torch.int32, device=self.device)
            b = torch.empty_like(a)
            scratch = torch.empty(Ho * Wo, dtype=torch.int64, device=self.device)
            S.refresh(img, Ho, Wo, rset.rec, a, b, scratch, RESCALE_PASSES, 4, seed, jfa=True)
            out = torch.empty((3, Ho, Wo), dtype=torch.float32, device=self.device)
            S.render_grid(img, Ho, Wo, rset.rec, a, Ho, Wo, out)
            ev = self._event()
            ev.record(st)
        return {"event": ev, "reqs": [req], "outs": [out], "keep": (a, b, scratch)}

    def done(self, h):
        return h["event"].query()

    def results(self, h):
        """The (request, output) pairs of a finished launch; its events go back to the
        pool (call once, after done(h))."""
        self._events.append(h.pop("event"))
        for r in h["reqs"]:
            if r.ready is not None:
                self._events.append(r.ready)
                r.ready = None
        return list(zip(h["reqs"], h["outs"]))


class Server:
    def __init__(self, backend, sets, mem_budget=None, max_batch_points=1 << 22, max_inflight=8,
                 reserve_frac=0.5, on_result=None):
        """on_result(request, output): called for every completed request; the default
        keeps the output on request.result.  A caller that keeps its requests but not
        their outputs (a load generator) passes one that drops it, so completed outputs
        do not pile up in device memory."""
        self.backend = backend
        self.on_result = on_result
        self.sets = {s.set_id: s for s in sets}
        if mem_budget is None:
            mem_budget = int(backend.free_bytes() * reserve_frac)
        self.budget = int(mem_budget)
        self.reserved = 0
        self.max_batch_points = int(max_batch_points)
        self.max_inflight = int(max_inflight)
        self._lock = threading.Lock()
        self._arrivals = collections.deque()
        self.pending = collections.deque()
        self.admitted = collections.deque()
        self.inflight = []
        self.completed = []
        self.launches = []       # (time, number of requests, number of sets) per launch
        self.peak_reserved = 0

    # ---- intake -------------------------------------------------------------------
    def submit(self, req):
        """Queue a request.  Its inputs may still be in flight on the submitting stream:
        the backend (on_submit) marks that point, and launches wait for it."""
        if req.t_arrival == 0.0:
            req.t_arrival = self.backend.now()
        hook = getattr(self.backend, "on_submit", None)
        if hook is not None:
            hook(req)
        with self._lock:
            self._arrivals.append(req)

    # ---- one scheduler turn -----------------------------------------------------------
    def step(self):
        with self._lock:
            while self._arrivals:
                self.pending.append(self._arrivals.popleft())
        self._poll()
        self._admit()
        self._launch()
        return bool(self.pending or self.admitted or self.inflight)

    def _admit(self):
        while self.pending:
            r = self.pending[0]
            rs = self.sets.get(r.set_id)
            if rs is None:
                self.pending.popleft()
                self._fail(r, f"unknown set {r.set_id}")
                continue
            need = request_bytes(r, rs)
            if need > self.budget:
                self.pending.popleft()
                self._fail(r, f"needs {need} bytes, budget {self.budget}")
                continue
            if self.reserved + need > self.budget:
                break  # FIFO: wait until memory frees up
            self.pending.popleft()
            r.nbytes = need
            r.t_admit = self.backend.now()
            self.reserved += need
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            self.admitted.append(r)

    def _direct(self):
        """Keyword arguments of a launch: a backend that can launch a lone request on
        its submitting stream is told to when nothing else is in flight."""
        if getattr(self.backend, "direct_launch", False):
            return {"direct": not self.inflight}
        return {}

    def _launch(self):
        while self.admitted and len(self.inflight) < self.max_inflight:
            head = self.admitted[0]
            if head.kind == RENDER:
                self.admitted.popleft()
                self._start([head], lambda rs=self.sets[head.set_id], r=head, kw=self._direct():
                             self.backend.launch_render(r, rs, **kw))
                continue
            if head.kind == RESCALE:
                self.admitted.popleft()
                self._start([head], lambda rs=self.sets[head.set_id], r=head, kw=self._direct():
                             self.backend.launch_rescale(r, rs, **kw))
                continue
            # gather admitted point queries with the head's K, up to the point budget
            K = self.sets[head.set_id].K
            batch, keep, total = [], collections.deque(), 0
            while self.admitted:
                r = self.admitted.popleft()
                if (r.kind == QUERY and self.sets[r.set_id].K == K and
                        (not batch or total + r.M <= self.max_batch_points)):
                    batch.append(r)
                    total += r.M
                else:
                    keep.append(r)
            self.admitted = keep
            self._start(batch, lambda b=batch, kw=self._direct():
                        self.backend.launch_queries(b, self.sets, **kw))

    def _start(self, reqs, fn):
        t = self.backend.now()
        for r in reqs:
            r.t_launch = t
        try:
            h = fn()
        except Exception as e:
            if len(reqs) > 1:  # find the failing request(s): launch each alone
                for r in reqs:
                    self._start([r], lambda r=r: self.backend.launch_queries([r], self.sets))
                return
            for r in reqs:
                self._release(r)
                self._fail(r, f"launch failed: {e}")
            return
        self.inflight.append(h)
        self.launches.append((t, len(reqs), len({r.set_id for r in reqs})))

    def _poll(self):
        still = []
        for h in self.inflight:
            if self.backend.done(h):
                t = self.backend.now()
                for r, out in self.backend.results(h):
                    if self.on_result is None:
                        r.result = out
                    else:
                        self.on_result(r, out)
                    r.t_done = t
                    self._release(r)
                    self.completed.append(r)
            else:
                still.append(h)
        self.inflight = still

    def _release(self, r):
        self.reserved -= r.nbytes
        r.nbytes = 0

    def _fail(self, r, msg):
        r.error = msg
        r.t_done = self.backend.now()
        self.completed.append(r)

    # ---- driving ----------------------------------------------------------------------
    def drain(self, timeout=60.0, idle_sleep=0.0):
        t_end = time.perf_counter() + timeout
        while self.step():
            if time.perf_counter() > t_end:
                raise TimeoutError("server did not drain")
            if idle_sleep:
                time.sleep(idle_sleep)

    def stats(self):
        ok = [r for r in self.completed if r.error is None]
        lat = sorted(r.latency for r in ok)
        if not ok:
            return {"completed": 0, "failed": len(self.completed)}
        t0 = min(r.t_arrival for r in ok)
        t1 = max(r.t_done for r in ok)
        pts = sum(r.M for r in ok if r.kind == QUERY)
        px = sum(self.sets[r.set_id].H * self.sets[r.set_id].W for r in ok if r.kind == RENDER)
        px += sum(r.Ho * r.Wo for r in ok if r.kind == RESCALE)

        def pct(q):
            return lat[min(len(lat) - 1, max(0, math.ceil(q * len(lat)) - 1))]

        span = max(t1 - t0, 1e-9)
        multi = [n for _, n, _ in self.launches]
        return {"completed": len(ok), "failed": len(self.completed) - len(ok),
                "p50_ms": 1e3 * pct(0.50), "p99_ms": 1e3 * pct(0.99),
                "mean_ms": 1e3 * sum(lat) / len(lat), "throughput_rps": len(ok) / span,
                "points_per_s": pts / span, "render_px_per_s": px / span,
                "launches": len(self.launches),
                "mean_requests_per_launch": sum(multi) / max(len(multi), 1),
                "peak_reserved_bytes": self.peak_reserved, "budget_bytes": self.budget}


def poisson_arrivals(rate, duration, rng):
    """Arrival times of a Poisson process of the given rate on [0, duration)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


def wait_until(t, spin=5e-4):
    """Sleep until perf_counter() reaches t: a coarse sleep, then a spin for the last
    `spin` seconds (a plain sleep overshoots by tens of microseconds)."""
    dt = t - time.perf_counter()
    if dt > spin:
        time.sleep(dt - spin)
    while time.perf_counter() < t:
        pass


def run_open_loop(server, requests, times, timeout=120.0):
    """Open-loop driver: request i arrives `times[i]` seconds after the start.  The
    scheduler's own thread submits every request whose arrival time has passed, with
    that arrival time as its t_arrival (so the wait until the scheduler notices it is
    part of its latency), runs scheduler turns while work is in flight, and sleeps until
    the next arrival when idle.  One thread: no feeder thread contends with the
    scheduler for the interpreter lock.  Returns when every request has completed
    (TimeoutError after `timeout` seconds)."""
    order = sorted(range(len(requests)), key=lambda i: times[i])
    n = len(requests)
    t_start = time.perf_counter()
    nxt = 0
    while nxt < n or len(server.completed) < n:
        now = time.perf_counter()
        while nxt < n and t_start + times[order[nxt]] <= now:
            r = requests[order[nxt]]
            r.t_arrival = t_start + times[order[nxt]]
            server.submit(r)
            nxt += 1
        busy = server.step()
        if now - t_start > timeout:
            raise TimeoutError(f"open loop: {len(server.completed)} of {n} requests done")
        if not busy and nxt < n:
            wait_until(t_start + times[order[nxt]])
