"""Continuous-batching server for independent hydro runs on one GPU.

Each request is a whole hydro run: a cubic box, its initial state (supplied
with the request, or built from an initial-condition family and seed), and
a number of steps.  The server admits arriving requests while
the HBM ledger (state ping-pong buffers plus the request's share of the
batch workspace) stays within the budget and a slot is free, keeps every
admitted state resident on the device, and advances all active requests
together: one batched ghost-fill (or timestep) launch and one batched advance
per iteration for each set of method parameters (advance_boxes, each box
with its own timestep, so a request's result does not depend on what it is
batched with).  Requests that arrive while others run join at the next
iteration; finished ones leave immediately and their memory returns to the
ledger.  Joining and leaving rewrite the work list of a plan made once with
a capacity (hydro_plan_update) and the batch's pointer arrays by
asynchronous copies from pinned memory, and a request's initial state is
uploaded the same way: the loop never waits for the device except to bound
how far it runs ahead.

The paper's codes keep all simulation data on the GPU and copy to the host
only for checkpoints (Sec. III), reuse device memory through a caching pool
allocator (Sec. III), and find that small boxes need many-at-once execution
to fill a GPU (Sec. IV-A); this loop applies the three to a stream of runs.

The scheduler is written against a small executor interface so the
admission and retirement logic can be exercised without a GPU; the only
product executor is GpuExecutor, which calls the HIP library.
"""
import collections
import math
import time


class Request:
    __slots__ = ("id", "arrival", "n", "steps", "family", "seed", "remaining", "need",
                 "t_admit", "t_done", "done_token", "handle", "result", "cells", "payload")

    def __init__(self, spec):
        self.id = spec["id"]
        self.arrival = float(spec["arrival"])
        self.n = int(spec["n"])
        self.steps = int(spec["steps"])
        self.family = spec["family"]
        self.seed = spec["seed"]
        self.remaining = self.steps
        self.cells = self.n ** 3
        self.need = 0
        self.t_admit = None
        self.t_done = None
        self.done_token = None
        self.handle = None
        self.result = None
        # the client's initial state (host state array, box, params), if it
        # came with the request
        self.payload = spec.get("state")


def _params_key(prm):
    return (float(prm["gamma"]), float(prm["cfl"]), tuple(float(g) for g in prm["grav"]),
            int(prm.get("flatten", 0)))


class _Group:
    """The active requests that share one set of method parameters: advanced
    by one batched call per stage with one capacity plan, one workspace that
    only grows, per-slot timesteps and pointer arrays, all on one stream.
    Membership changes rewrite the plan's work list and the pointer arrays by
    asynchronous copies from pinned host memory; nothing synchronises the
    host with the device."""

    RING = 8  # pinned staging slots for the pointer arrays

    def __init__(self, ex, prm):
        torch, hydro = ex.torch, ex.hydro
        self.ex = ex
        self.prm = prm
        cap = ex.max_active
        self.plan = hydro.Plan.with_capacity(cap)
        self.ws = torch.empty(256, dtype=torch.uint8, device=ex.device)
        self.dt = torch.zeros(cap, dtype=torch.float64, device=ex.device)
        self.dt_next = torch.zeros(cap, dtype=torch.float64, device=ex.device)
        self.ptr = torch.zeros((2, cap), dtype=torch.int64, device=ex.device)
        self.pa, self.pb = self.ptr[0], self.ptr[1]
        self.host = [torch.zeros((2, cap), dtype=torch.int64).pin_memory()
                     for _ in range(self.RING)]
        self.host_ev = [None] * self.RING
        self.slot = 0
        self.members = []
        self.have_dt = False

    def set_members(self, reqs):
        torch = self.ex.torch
        self.members = list(reqs)
        if not reqs:
            return
        n = len(reqs)
        self.plan.update([r.handle["box"] for r in reqs])
        if self.plan.ws_bytes > self.ws.numel():
            # grown geometrically; the caching allocator reuses the old block
            # in stream order
            self.ws = torch.empty(max(self.plan.ws_bytes, int(1.25 * self.ws.numel())),
                                  dtype=torch.uint8, device=self.ex.device)
        k = self.slot
        self.slot = (k + 1) % self.RING
        if self.host_ev[k] is not None:
            self.host_ev[k].synchronize()  # the copy that last used this slot
        h = self.host[k]
        h[0, :n] = torch.tensor([r.handle["U"].data_ptr() for r in reqs], dtype=torch.int64)
        h[1, :n] = torch.tensor([r.handle["Un"].data_ptr() for r in reqs], dtype=torch.int64)
        # (stream-ordered: launches queued before this copy still read the old
        # pointers, later ones the new)
        self.ptr[:, :n].copy_(h[:, :n], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self.host_ev[k] = ev
        self.pa, self.pb = self.ptr[0], self.ptr[1]
        self.have_dt = False  # the membership changed: timesteps from estimate_dt_boxes

    def step(self):
        if not self.members:
            return
        h = self.ex.hydro
        if self.have_dt:  # timesteps of the states the previous iteration produced
            h.fill_ghosts_boxes(self.plan, self.pa)
            self.dt, self.dt_next = self.dt_next, self.dt
        else:
            h.estimate_dt_boxes(self.plan, self.pa, self.prm, self.dt, None)
        h.advance_boxes(self.plan, self.pa, self.pb, self.prm, self.dt, self.ws, self.ex.err,
                        dt_stride=1, dt_next=self.dt_next)
        self.have_dt = True
        for r in self.members:
            r.handle["U"], r.handle["Un"] = r.handle["Un"], r.handle["U"]
        self.pa, self.pb = self.pb, self.pa

    def close(self):
        self.plan.close()


class GpuExecutor:
    """Device side of the server: states in device memory, one group per set
    of method parameters (each with a capacity plan updated in place as
    requests join and leave), every launch on the current stream."""

    def __init__(self, device="cuda", keep_results=False, max_active=64):
        import torch
        from . import hydro, inputs
        self.torch = torch
        self.hydro = hydro
        self.inputs = inputs
        self.device = device
        self.keep_results = keep_results
        self.max_active = int(max_active)
        hydro.lib()
        self.groups = {}
        self.err = torch.zeros(1, dtype=torch.int32, device=device)

    # -- memory ledger: state ping-pong buffers plus the box's workspace share
    def bytes_needed(self, req):
        # (the sizes depend only on the box's cell counts and ghost depth: a
        # request without a state gets the families' cubic box)
        box = req.payload[1] if req.payload is not None else self.inputs.box_desc((req.n,) * 3)
        return 2 * 8 * self.hydro.state_elems(box) + self.hydro.workspace_bytes(box)

    # -- membership
    def admit(self, req):
        torch = self.torch
        if req.payload is not None:
            U, box, prm = req.payload
            req.payload = None  # uploaded: the host copy is no longer held
        else:
            U, box, prm = self.inputs.request_state({"family": req.family, "n": req.n,
                                                     "seed": req.seed})
        key = _params_key(prm)
        if key not in self.groups:
            self.groups[key] = _Group(self, dict(prm))
        # pinned staging and an asynchronous upload: the host does not wait for
        # the device work already queued
        Ud = torch.as_tensor(U, dtype=torch.float64).pin_memory().to(self.device,
                                                                    non_blocking=True)
        req.handle = {"U": Ud, "Un": torch.empty_like(Ud), "box": box, "group": key}

    def release(self, req):
        if self.keep_results:
            req.result = req.handle["U"].cpu().numpy()
        req.handle = None

    def set_batch(self, reqs):
        if len(reqs) > self.max_active:
            raise ValueError("more active requests than the executor's capacity")
        by = {k: [] for k in self.groups}
        for r in reqs:
            by[r.handle["group"]].append(r)
        for k, g in self.groups.items():
            if [id(r) for r in by[k]] != [id(r) for r in g.members]:
                g.set_members(by[k])

    # -- one iteration: every active request advances one step with its own dt
    def step(self):
        for g in self.groups.values():
            g.step()

    def mark(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        return ev

    def wait(self, token):
        token.synchronize()

    def elapsed(self, t0_token, token):
        return t0_token.elapsed_time(token) * 1e-3

    def error_bits(self):
        return int(self.err.item())

    def close(self):
        for g in self.groups.values():
            g.close()
        self.groups = {}


class Server:
    """Admission, batching and retirement.  ``clock`` returns seconds; the
    executor supplies device timing tokens (events), so latency is measured
    on the device timeline: completion = end of the request's last step."""

    def __init__(self, executor, budget_bytes=200e9, max_active=64, max_ahead=2,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = float(budget_bytes)
        self.max_active = int(max_active)
        self.max_ahead = int(max_ahead)
        self.clock = clock
        self.sleep = sleep
        self.ledger = 0.0
        self.peak_ledger = 0.0
        self.iterations = 0
        self.peak_active = 0

    def run(self, specs):
        reqs = [Request(s) for s in specs]
        for r in reqs:
            r.need = self.ex.bytes_needed(r)
            if r.need > self.budget:
                raise ValueError("request %d needs %.3g B, more than the %.3g B budget"
                                 % (r.id, r.need, self.budget))
        pending = collections.deque(sorted(reqs, key=lambda r: (r.arrival, r.id)))
        active = []
        inflight = collections.deque()
        done = []
        t0 = self.clock()
        t0_tok = self.ex.mark()
        changed = False
        cap = getattr(self.ex, "max_active", None)
        if cap is not None and cap < self.max_active:
            raise ValueError("the executor holds %d requests, fewer than max_active" % cap)
        while pending or active:
            now = self.clock() - t0
            # admission: FIFO, while a slot and the budget allow
            while (pending and pending[0].arrival <= now and len(active) < self.max_active
                   and self.ledger + pending[0].need <= self.budget):
                r = pending.popleft()
                self.ex.admit(r)
                r.t_admit = now
                self.ledger += r.need
                active.append(r)
                changed = True
            self.peak_ledger = max(self.peak_ledger, self.ledger)
            if not active:
                # idle until the next arrival (the device drains meanwhile)
                while inflight:
                    self.ex.wait(inflight.popleft())
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
                continue
            if changed:
                self.ex.set_batch(active)
                changed = False
            self.peak_active = max(self.peak_active, len(active))
            self.ex.step()
            self.iterations += 1
            for r in active:
                r.remaining -= 1
            fin = [r for r in active if r.remaining == 0]
            tok = self.ex.mark()
            inflight.append(tok)
            if fin:
                for r in fin:
                    r.done_token = tok
                    self.ex.release(r)
                    self.ledger -= r.need
                    done.append(r)
                active = [r for r in active if r.remaining > 0]
                changed = True
            # bound how far the host runs ahead of the device
            while len(inflight) > self.max_ahead:
                self.ex.wait(inflight.popleft())
        while inflight:
            self.ex.wait(inflight.popleft())
        for r in done:
            r.t_done = self.ex.elapsed(t0_tok, r.done_token)
        self.requests = sorted(done, key=lambda r: r.id)
        return self.requests

    def metrics(self, skip=0):
        """Latency percentiles and throughput over the requests after the first
        ``skip`` (by id, the warm-up)."""
        rs = [r for r in self.requests if r.id >= skip]
        lat = sorted(r.t_done - r.arrival for r in rs)
        cu = sum(r.cells * r.steps for r in rs)
        t_first = min(r.arrival for r in rs)
        t_last = max(r.t_done for r in rs)
        span = max(t_last - t_first, 1e-12)

        def pct(q):
            if not lat:
                return None
            k = min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))
            return lat[k]

        return {"requests": len(rs), "p50_s": pct(0.50), "p99_s": pct(0.99),
                "mean_s": sum(lat) / len(lat) if lat else None,
                "cell_updates": cu, "span_s": span, "cu_per_s": cu / span,
                "iterations": self.iterations, "peak_active": self.peak_active,
                "peak_ledger_bytes": self.peak_ledger}
