"""Continuous-batching request loop over many independent solves.

Requests arrive as a Poisson stream; each asks for ``nsteps`` RK steps of its
own periodic box (size, polynomial order, equation mask and viscosity of its
own).  The loop

* admits requests in arrival order while their device footprint fits the
  memory budget and a batch slot is free,
* sets up each admitted solve (mesh, metrics, initial state) on a worker
  thread while the GPU keeps stepping the others,
* adds it to the running batch at the next RK step boundary, where every
  member advances with its own dt in the same launches (``hdg_batch_*``),
* removes members as they finish, freeing their slot and memory for the
  next admission,

and records per-request latency (arrival to completion) split into queueing,
set-up and stepping.  The scheduler is written against a small backend
interface so its admission and refill logic is testable without a GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the stream
    n: int                      # periodic box of n^3 elements
    P: int                      # polynomial order
    frac: float                 # fraction of viscous (NS-LES) elements
    nu: float                   # kinematic viscosity
    seed: int
    nsteps: int = 50
    # filled in by the loop
    t_admit: float = math.nan
    t_join: float = math.nan
    t_done: float = math.nan
    steps_done: int = 0
    nodes: int = 0
    est_bytes: int = 0
    result: object = None
    refused: str = ""           # why the request was not served ("" if it was)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def make_requests(count: int = 256, rate: float = 20.0, seed: int = 0, n_range=(4, 24), p_range=(2, 6),
                  frac_range=(0.2, 0.8), nu_range=(1e-4, 1e-2), nsteps: int = 50) -> list[Request]:
    """Seeded request stream: exponential inter-arrival times at `rate` per
    second, n and P uniform over the inclusive ranges, mask fraction and nu
    uniform over theirs."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        out.append(Request(rid=i, arrival=float(t[i]), n=int(rng.integers(n_range[0], n_range[1] + 1)),
                           P=int(rng.integers(p_range[0], p_range[1] + 1)),
                           frac=float(rng.uniform(*frac_range)), nu=float(rng.uniform(*nu_range)),
                           seed=1_000_003 * seed + i, nsteps=nsteps))
    return out


def footprint_bytes(n: int, P: int) -> int:
    """Device bytes of one solve: state and RK register (caller), the library's
    ping-pong state, metric terms in FP64 and FP32, mass, viscous part, and
    per-face geometry (FP64 + FP32) and viscous traces, with a small margin."""
    ne = n ** 3
    N = P + 1
    nodes = ne * N ** 3
    faces = 3 * ne
    per_node = 32 + 32 + 32 + 80 + 40 + 8 + 24
    per_face_node = 32 + 16 + 48
    return int(1.05 * (nodes * per_node + faces * N * N * per_face_node + ne * 128)) + (1 << 16)


class Backend:
    """What the scheduler needs from the device side."""

    def setup(self, req: Request):                      # worker thread: returns a handle
        raise NotImplementedError

    def join(self, handle) -> int:                      # main thread: add to the batch, returns slot
        raise NotImplementedError

    def step(self, nsteps: int):                        # advance every member, wait for completion
        raise NotImplementedError

    def leave(self, slot: int, handle):                 # remove from the batch, release device memory
        raise NotImplementedError


@dataclass
class ServeStats:
    requests: list              # served to completion
    wall_s: float
    steps_launched: int
    max_members: int
    peak_bytes: int
    dof_evals: float
    member_counts: list = field(default_factory=list)
    refused: list = field(default_factory=list)   # refused on their own (``Request.refused`` says why)

    def summary(self) -> dict:
        if not self.requests:
            return {"requests": 0, "refused": len(self.refused), "wall_s": self.wall_s}
        lat = np.array([r.latency for r in self.requests])
        queue = np.array([r.t_admit - r.arrival for r in self.requests])
        setup = np.array([r.t_join - r.t_admit for r in self.requests])
        stepping = np.array([r.t_done - r.t_join for r in self.requests])

        def pct(a, p):
            return float(np.percentile(a, p))
        return {
            "requests": len(self.requests), "refused": len(self.refused),
            "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99), "mean_latency_s": float(lat.mean()),
            "p50_queue_s": pct(queue, 50), "p99_queue_s": pct(queue, 99),
            "p50_setup_s": pct(setup, 50), "p99_setup_s": pct(setup, 99),
            "p50_stepping_s": pct(stepping, 50), "p99_stepping_s": pct(stepping, 99),
            "wall_s": self.wall_s, "batch_calls": self.steps_launched,
            "max_concurrent_members": self.max_members, "peak_admitted_bytes": self.peak_bytes,
            "dof_residual_evals_per_s": self.dof_evals / self.wall_s,
            "mean_members_per_call": float(np.mean(self.member_counts)) if self.member_counts else 0.0,
        }


def serve(requests: list[Request], backend: Backend, mem_budget: int, max_members: int,
          max_steps_per_call: int = 10, setup_workers: int = 4, clock=time.perf_counter,
          sleep=time.sleep, realtime: bool = True) -> ServeStats:
    """Run the request stream to completion.  With `realtime`, a request is
    only visible once the clock has passed its arrival time; otherwise all
    arrive at once (a backlog).

    A request that can never be served is refused on its own and the stream
    goes on: one whose footprint exceeds the whole memory budget (refused on
    arrival, before it could hold up the queue behind it) and one whose
    set-up raises (its memory is released).  Refused requests are listed in
    ``ServeStats.refused`` with the reason in ``Request.refused``."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    for r in reqs:
        r.est_bytes = footprint_bytes(r.n, r.P)
    refused = []
    pending = collections.deque()
    setups = {}                       # future -> request
    ready = collections.deque()       # (request, handle) set up, waiting to join
    active = {}                       # slot -> (request, handle)
    used = 0
    peak = 0
    max_seen = 0
    calls = 0
    dof = 0.0
    counts = []
    done = []
    t0 = clock()
    nxt = 0
    with cf.ThreadPoolExecutor(max_workers=setup_workers) as pool:
        while len(done) + len(refused) < len(reqs):
            now = clock() - t0
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                r = reqs[nxt]
                nxt += 1
                if r.est_bytes > mem_budget:
                    r.refused = f"needs {r.est_bytes} bytes, more than the budget {mem_budget}"
                    r.t_done = clock() - t0
                    refused.append(r)
                else:
                    pending.append(r)
            # admission: arrival order, memory budget, slots (set-up ones count)
            while pending and used + pending[0].est_bytes <= mem_budget and \
                    len(active) + len(setups) + len(ready) < max_members:
                r = pending.popleft()
                used += r.est_bytes
                peak = max(peak, used)
                r.t_admit = clock() - t0
                setups[pool.submit(backend.setup, r)] = r
            for fut in [f for f in setups if f.done()]:
                r = setups.pop(fut)
                try:
                    ready.append((r, fut.result()))
                except Exception as ex:            # this request only: release it and go on
                    r.refused = f"set-up failed: {ex}"
                    r.t_done = clock() - t0
                    used -= r.est_bytes
                    refused.append(r)
            # join at the step boundary
            while ready:
                r, h = ready.popleft()
                slot = backend.join(h)
                r.t_join = clock() - t0
                active[slot] = (r, h)
            if active:
                k = min(max_steps_per_call, min(r.nsteps - r.steps_done for r, _ in active.values()))
                backend.step(k)
                calls += 1
                counts.append(len(active))
                max_seen = max(max_seen, len(active))
                t_now = clock() - t0
                for slot in list(active):
                    r, h = active[slot]
                    r.steps_done += k
                    dof += 3.0 * k * 4 * r.nodes
                    if r.steps_done >= r.nsteps:
                        r.result = backend.leave(slot, h)
                        r.t_done = t_now
                        del active[slot]
                        used -= r.est_bytes
                        done.append(r)
            else:
                # idle: wait for a set-up to finish or the next arrival
                waits = [f for f in setups]
                timeout = 0.002
                if not waits and nxt < len(reqs) and realtime:
                    timeout = max(0.0, reqs[nxt].arrival - (clock() - t0))
                if waits:
                    cf.wait(waits, timeout=0.05, return_when=cf.FIRST_COMPLETED)
                elif timeout > 0:
                    sleep(min(timeout, 0.05))
    wall = clock() - t0
    return ServeStats(done, wall, calls, max_seen, peak, dof, counts, refused)


def taylor_green_device(torch, X, amp: float, seed: int):
    """Taylor-Green vortex (the benchmark workloads' formula) evaluated on the
    device from node coordinates X (n_elem, 3, N^3), plus seeded i.i.d.
    U[-amp, amp] velocity noise from a device generator: a request's initial
    state costs no host arithmetic."""
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    q = torch.empty((X.shape[0], 4, X.shape[2]), dtype=torch.float64, device=X.device)
    q[:, 0] = (torch.cos(2 * x) + torch.cos(2 * y)) * (torch.cos(2 * z) + 2.0) / 16.0
    q[:, 1] = torch.sin(x) * torch.cos(y) * torch.cos(z)
    q[:, 2] = -torch.cos(x) * torch.sin(y) * torch.cos(z)
    q[:, 3] = 0.0
    if amp > 0:
        g = torch.Generator(device=X.device)
        g.manual_seed(int(seed))
        noise = torch.rand(q[:, 1:4].shape, generator=g, dtype=torch.float64, device=X.device)
        q[:, 1:4] += (2.0 * noise - 1.0) * amp
    return q


class HdgBackend(Backend):
    """Device backend: one hdg batch on a non-blocking stream.  Set-up on a
    worker thread builds the mesh (host geometry and uploads, under the
    library's device lock); joining, on the stepping thread between batch
    calls, uploads the node coordinates, evaluates the initial state and the
    time step on the device and adds the member."""

    C0SQ = 25.0

    def __init__(self, ctx, max_members: int, prec: int, torch, stream=None, keep_results: bool = False):
        """keep_results: a finished request's result is a dict of its final and
        initial states (host arrays), time step and mesh, else whether its
        final state is finite."""
        from . import hdg, workloads as W
        self.hdg, self.W, self.torch = hdg, W, torch
        self.ctx = ctx
        self.prec = prec
        self.batch = hdg.hdg_batch_create(ctx, max_members)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.keep = keep_results
        self._boxes = {}
        self._lock = threading.Lock()

    def _box(self, n):
        with self._lock:
            if n not in self._boxes:
                mesh = self.W.periodic_box(n, Pg=1)
                self._boxes[n] = (mesh, self.W.min_edge_length(mesh))
            return self._boxes[n]

    def setup(self, r: Request):
        hdg, W = self.hdg, self.W
        mesh, hmin = self._box(r.n)
        flag = W.bernoulli_mask(mesh.n_elem, r.frac, r.seed)
        m = hdg.hdg_mesh_create(self.ctx, mesh, r.P, flag,
                                hdg.make_params(c0sq=self.C0SQ, nu=r.nu, les_model=1, C_les=0.1))
        r.nodes = m.n_elem * m.N3
        return {"mesh": m, "X": hdg.hdg_mesh_node_coords(m), "hmin": hmin, "req": r}

    def _initial(self, h):
        """Initial state and dt on the device: half the convective limit
        0.5 h_min / ((P + 1)^2 max(|u| + sqrt(|u|^2 + c0^2)))."""
        torch = self.torch
        r = h["req"]
        q = taylor_green_device(torch, torch.from_numpy(h["X"]).cuda(), 0.01, r.seed)
        lam = self.hdg.hdg_max_wave_speed(h["mesh"], q, stream=torch.cuda.current_stream())
        return q, 0.5 * 0.5 * h["hmin"] / ((r.P + 1) ** 2 * lam)

    def join(self, h) -> int:
        with self.torch.cuda.stream(self.stream):
            q, dt = self._initial(h)
            dq = self.torch.empty_like(q)
        self.stream.synchronize()
        h.update(q=q, dq=dq, dt=dt)
        if self.keep:
            h["q0"] = q.cpu().numpy()
        h.pop("X")
        return self.hdg.hdg_batch_add(self.batch, h["mesh"], q, dq, dt)

    def step(self, nsteps: int):
        self.hdg.hdg_batch_rk3_steps(self.batch, nsteps, prec=self.prec, stream=self.stream)
        self.stream.synchronize()

    def leave(self, slot: int, h):
        q = h["q"]
        self.hdg.hdg_batch_remove(self.batch, slot)
        if self.keep:
            # final state, time step, initial state and the mesh (for checks)
            return {"q": q.cpu().numpy(), "dt": h["dt"], "q0": h["q0"], "mesh": h["mesh"]}
        return bool(self.torch.isfinite(q).all().item())

    def make_alone(self, r: Request):
        """The same solve, set up on its own: (mesh, q, dq, dt)."""
        h = self.setup(r)
        q, dt = self._initial(h)
        self.torch.cuda.synchronize()
        return h["mesh"], q, self.torch.empty_like(q), dt
