"""Continuous-batching server for VQE energy and gradient requests on one GPU.

Requests of mixed qubit counts arrive over time (the paper's bond-length
evaluations are independent, Eq. 7 of arXiv 2601.09951, which is what lets
any subset of them share a launch).  The scheduler

* admits an arrived request into a batch when a slot and device memory are
  free (memory per batch = the exact workspace the library reports, checked
  against a byte budget), otherwise it waits;
* forms batches per class (qubit count, ansatz, energy-only or with
  gradient), FIFO inside a class, up to ``max_batch`` requests, while the
  class's earlier batches may still be on the device;
* launches each batch on its class's HIP stream, so batches of different
  classes overlap on the GPU, and records a completion event;
* polls completion events, returns results and frees the batch's memory,
  then admits whatever has arrived meanwhile.

All computation runs in libvqe (vqe_energy / vqe_energy_grad with one
Hamiltonian per instance); this module only schedules.  ``run_plain`` is the
baseline: the same requests one at a time, in arrival order, one launch
sequence each, with a host synchronisation per request.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import vqe


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    want_grad: bool
    energy: float
    grad: Optional[np.ndarray]
    arrival: float
    done: float
    batch_size: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class LibvqeExecutor:
    """Executes batches with libvqe on one device.

    Batches run on a small fixed set of HIP streams (default priority), each
    on a hardware queue of its own (vqe_stream_create): the runtime otherwise
    maps streams onto a small pool of hardware queues, and the work of two
    streams on one queue runs in order.  The longest batches (20 qubits and
    more) get one stream and the short classes spread over the others, so a
    short request never waits behind a long batch.  Results are copied
    to pinned host memory on the batch's own stream, and the completion event
    follows that copy, so nothing runs on the null stream and collecting a
    finished batch does not wait for the device.
    """

    def __init__(self, ctx: vqe.Context, device: int = 0, n_streams: int = 4):
        self.ctx = ctx
        self.dev = torch.device(f"cuda:{device}")
        self._circuits: Dict[str, vqe.Circuit] = {}
        self._streams = [ctx.dedicated_stream(i) for i in range(max(2, n_streams))]

    def _circuit(self, spec) -> vqe.Circuit:
        key = spec.shape_key()
        if key not in self._circuits:
            self._circuits[key] = vqe.Circuit.from_spec(self.ctx, spec)
        return self._circuits[key]

    def stream_index(self, key) -> int:
        n = key[0]
        if n >= 20:
            return 0
        rest = len(self._streams) - 1
        return 1 + min(rest - 1, (n - 1) // 4)

    def hamiltonian(self, req):
        if req.integrals is not None:
            i = req.integrals
            return vqe.Hamiltonian.from_integrals(self.ctx, i.h1, i.h2, i.e_core)
        return vqe.Hamiltonian.from_sum(self.ctx, req.pauli)

    def release(self, ham):
        ham.close()  # stream-ordered in the library: no device synchronisation

    def request_bytes(self, key, req) -> int:
        """Upper estimate of one request's share of a batch workspace."""
        state = 16 << req.n
        return state * (2 if key[2] else 1) + 64 * req.circuit.n_gates + (1 << 20)

    def batch_bytes(self, key, reqs, hams) -> int:
        """Exact workspace of a batch, as the library reports it."""
        C = self._circuit(reqs[0].circuit)
        return vqe.workspace_bytes(self.ctx, C, hams, len(reqs), 1 if key[2] else 0)

    def launch(self, key, reqs, hams, nbytes):
        C = self._circuit(reqs[0].circuit)
        B = len(reqs)
        s = self._streams[self.stream_index(key)]
        theta_h = torch.from_numpy(np.stack([r.theta for r in reqs]).astype(np.float64)).pin_memory()
        with torch.cuda.stream(s):
            theta = theta_h.to(self.dev, non_blocking=True)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
            e = torch.empty(B, dtype=torch.float64, device=self.dev)
            e_h = torch.empty(B, dtype=torch.float64, pin_memory=True)
            if key[2]:
                g = torch.empty(B, C.n_params, dtype=torch.float64, device=self.dev)
                vqe.energy_grad(self.ctx, C, hams, theta, ws=ws, out_e=e, out_g=g)
                g_h = torch.empty(B, C.n_params, dtype=torch.float64, pin_memory=True)
                g_h.copy_(g, non_blocking=True)
            else:
                g = g_h = None
                vqe.energy(self.ctx, C, hams, theta, ws=ws, out=e)
            e_h.copy_(e, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"theta": theta, "theta_h": theta_h, "ws": ws, "e": e, "g": g, "e_h": e_h, "g_h": g_h,
                "event": ev}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle):
        handle["event"].synchronize()
        e = handle["e_h"].numpy().copy()
        g = handle["g_h"].numpy().copy() if handle["g_h"] is not None else None
        return e, g

    def drain(self):
        for s in self._streams:
            s.synchronize()

    def close(self):
        self.drain()
        for c in self._circuits.values():
            c.close()
        self._circuits.clear()


@dataclasses.dataclass
class _Batch:
    key: tuple
    reqs: list
    hams: list
    handle: object
    nbytes: int


class Server:
    """Continuous batching: admission by slots and memory, per-class FIFO batches."""

    def __init__(self, executor, mem_budget: int = 32 << 30, max_batch: int = 128,
                 max_inflight_per_class: int = 2):
        self.ex = executor
        self.mem_budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight_per_class)
        self.stats = collections.Counter()

    @staticmethod
    def _class(req) -> tuple:
        return (req.n, req.circuit.shape_key(), bool(req.want_grad))

    def _finish(self, b: _Batch, now: float) -> List[Result]:
        e, g = self.ex.collect(b.handle)
        out = [Result(r.rid, r.n, r.want_grad, float(e[i]), None if g is None else np.array(g[i]), r.arrival,
                      now, len(b.reqs)) for i, r in enumerate(b.reqs)]
        for h in b.hams:
            self.ex.release(h)
        return out

    def run(self, requests, realtime: bool = True, clock=None) -> List[Result]:
        """Serve a request stream; arrival times are honoured when realtime."""
        clock = clock or time.perf_counter
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: Dict[tuple, collections.deque] = collections.defaultdict(collections.deque)
        inflight: List[_Batch] = []
        results: List[Result] = []
        used = 0
        total = len(pending)
        t0 = clock()
        while len(results) < total:
            now = clock() - t0
            progressed = False
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.popleft()
                waiting[self._class(r)].append(r)
                progressed = True
            # completions free slots and memory
            still = []
            for b in inflight:
                if self.ex.done(b.handle):
                    results.extend(self._finish(b, clock() - t0))
                    used -= b.nbytes
                    progressed = True
                else:
                    still.append(b)
            inflight = still
            # admission: oldest class first; FIFO inside a class; as many as fit
            for key in sorted((k for k in waiting if waiting[k]), key=lambda k: waiting[k][0].arrival):
                q = waiting[key]
                if sum(1 for b in inflight if b.key == key) >= self.max_inflight:
                    continue
                take, hams = [], []
                est = 0
                while q and len(take) < self.max_batch:
                    need = self.ex.request_bytes(key, q[0])
                    if used + est + need > self.mem_budget:
                        break
                    take.append(q.popleft())
                    hams.append(self.ex.hamiltonian(take[-1]))
                    est += need
                nbytes = self.ex.batch_bytes(key, take, hams) if take else 0
                while take and used + nbytes > self.mem_budget:  # the estimate was short: give back the newest
                    q.appendleft(take.pop())
                    self.ex.release(hams.pop())
                    nbytes = self.ex.batch_bytes(key, take, hams) if take else 0
                if not take:
                    if not inflight:
                        raise MemoryError(f"request {q[0].rid} (n={q[0].n}) exceeds the memory budget alone")
                    self.stats["memory_waits"] += 1
                    continue
                inflight.append(_Batch(key, take, hams, self.ex.launch(key, take, hams, nbytes), nbytes))
                used += nbytes
                self.stats["batches"] += 1
                self.stats["max_batch_seen"] = max(self.stats["max_batch_seen"], len(take))
                self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
                self.stats["peak_inflight"] = max(self.stats["peak_inflight"], len(inflight))
                progressed = True
            if not progressed:
                time.sleep(20e-6)
        self.ex.drain()
        return sorted(results, key=lambda r: r.rid)


def run_plain(ctx: vqe.Context, requests, realtime: bool = True, device: int = 0) -> List[Result]:
    """Baseline: arrival order, one request per launch sequence, host sync each."""
    dev = torch.device(f"cuda:{device}")
    circuits: Dict[str, vqe.Circuit] = {}
    results = []
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda q: q.arrival):
        if realtime:
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(20e-6)
        key = r.circuit.shape_key()
        if key not in circuits:
            circuits[key] = vqe.Circuit.from_spec(ctx, r.circuit)
        C = circuits[key]
        if r.integrals is not None:
            H = vqe.Hamiltonian.from_integrals(ctx, r.integrals.h1, r.integrals.h2, r.integrals.e_core)
        else:
            H = vqe.Hamiltonian.from_sum(ctx, r.pauli)
        th = torch.from_numpy(r.theta[None, :].astype(np.float64)).to(dev)
        if r.want_grad:
            e, g = vqe.energy_grad(ctx, C, H, th)
            g = g.cpu().numpy()[0]
        else:
            e = vqe.energy(ctx, C, H, th)
            g = None
        ev = float(e.cpu().numpy()[0])  # host synchronisation per request
        results.append(Result(r.rid, r.n, r.want_grad, ev, g, r.arrival, time.perf_counter() - t0, 1))
        H.close()
    for c in circuits.values():
        c.close()
    return sorted(results, key=lambda q: q.rid)


def latency_summary(results: List[Result], wall: float = None) -> dict:
    lat = np.array([r.latency for r in results])
    if wall is None:
        wall = max(r.done for r in results) - min(r.arrival for r in results)
    per_n = {}
    for n in sorted({r.n for r in results}):
        ln = np.array([r.latency for r in results if r.n == n])
        per_n[f"{n}q"] = {"count": int(ln.size), "p50_ms": round(float(np.percentile(ln, 50)) * 1e3, 3),
                          "p99_ms": round(float(np.percentile(ln, 99)) * 1e3, 3)}
    return {"requests": len(results), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "evals_per_s": round(len(results) / wall, 1), "wall_s": round(wall, 3), "per_n": per_n}
