"""Continuous-batching request loop for key-switching requests.

Requests are Rotate (Algorithm 3) or Mult with relinearization and Rescale
(Algorithm 2) at a ring degree N and a level chosen per request, from many
clients each holding its own rotation and relinearization keys.  The loop
  - admits an arrived request when an output slot of its N is free (the
    device memory of ciphertexts is a fixed pool of slots);
  - keeps per-client keys resident in HBM up to a byte budget, evicting the
    least recently used key that no in-flight step reads, and uploading
    misses from pinned host copies on the step's stream (full keys, or
    seeded keys whose rows b_j alone are stored and moved);
  - forms a step from the queue: the oldest request's (N, op) group, up to
    max_batch requests of it in arrival order whatever their levels, issued
    as one batched call over uneven limb counts (hks_batch_rotate_mixed /
    hks_batch_mult_relin_mixed, with full or seeded keys);
  - keeps up to `lanes` steps in flight, each lane with its own stream and
    contexts (workspaces), so steps of different groups overlap on the GPU;
  - records arrival, start and completion times; completion is when the
    step's event is seen complete.
The executor is separate from the scheduling so that the scheduling can be
checked with a simulated executor and clock.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    client: int
    op: str        # "rotate" or "mult"
    log_n: int
    level: int
    arrival: float  # seconds from the start of the run
    k: int = 1      # rotation index (rotate)
    start: float = -1.0
    done: float = -1.0
    slot: int = -1

    @property
    def group(self):
        # requests of one N and op share a step at any levels (one launch
        # sequence serves uneven limb counts)
        return (self.log_n, self.op)


def poisson_requests(n_req: int, rate: float, n_clients: int, log_ns=(15, 16), levels=(3, 35),
                     p_rotate: float = 0.5, seed: int = 0) -> list:
    """n_req requests with exponential inter-arrival times (rate per second):
    client uniform; N = 2^15 for even clients, 2^16 for odd; op rotate with
    probability p_rotate else mult; level uniform in [levels[0], levels[1]];
    rotation index 1 + client mod 8."""
    g = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(g.exponential(1.0 / rate, n_req))
    clients = g.integers(0, n_clients, n_req)
    ops = g.random(n_req) < p_rotate
    lv = g.integers(levels[0], levels[1] + 1, n_req)
    out = []
    for i in range(n_req):
        c = int(clients[i])
        out.append(Request(rid=i, client=c, op="rotate" if ops[i] else "mult", log_n=log_ns[c % len(log_ns)],
                           level=int(lv[i]), arrival=float(t[i]), k=1 + c % 8))
    return out


class Engine:
    """The scheduling loop.  `executor` provides
        submit(lane, requests) -> handle   (enqueue one step; requests share a group)
        done(handle) -> bool
        slots(log_n) -> number of output slots of that N
    `clock()` returns seconds since the run started, `idle(dt)` waits (or
    advances a simulated clock) when nothing can progress."""

    def __init__(self, executor, lanes: int, max_batch: int, clock=None, idle=None):
        self.ex = executor
        self.lanes = lanes
        self.max_batch = max_batch
        self._t0 = None
        self.clock = clock or self._wall
        self.idle = idle or (lambda dt: time.sleep(min(dt, 1e-4)))

    def _wall(self):
        return time.perf_counter() - self._t0

    def run(self, requests: list, one_at_a_time: bool = False) -> dict:
        """Serve `requests` (sorted by arrival).  one_at_a_time: steps of one
        request on one lane, the next issued only after the previous
        completes (the plain baseline)."""
        self._t0 = time.perf_counter()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        # free output slots per N, handed out least recently freed first
        free = {n: collections.deque(range(self.ex.slots(n))) for n in {r.log_n for r in requests}}
        queue = []          # admitted, not started: heap of (arrival, rid, request)
        inflight = {}       # lane -> (handle, [requests])
        lanes = 1 if one_at_a_time else self.lanes
        max_batch = 1 if one_at_a_time else self.max_batch
        n_done = 0
        while n_done < len(requests):
            now = self.clock()
            progressed = False
            # completions
            for lane, (h, batch) in list(inflight.items()):
                if self.ex.done(h):
                    t = self.clock()
                    for r in batch:
                        r.done = t
                        free[r.log_n].append(r.slot)
                    n_done += len(batch)
                    del inflight[lane]
                    progressed = True
            # admission: arrived requests with a free output slot of their N
            while pending and pending[0].arrival <= now and free[pending[0].log_n]:
                r = pending.popleft()
                r.slot = free[r.log_n].popleft()
                heapq.heappush(queue, (r.arrival, r.rid, r))
                progressed = True
            # issue steps on free lanes
            for lane in range(lanes):
                if lane in inflight or not queue:
                    continue
                _, _, head = queue[0]
                grp = head.group
                take, keep = [], []
                while queue and len(take) < max_batch:
                    item = heapq.heappop(queue)
                    (take if item[2].group == grp else keep).append(item)
                for item in keep:
                    heapq.heappush(queue, item)
                batch = [item[2] for item in take]
                t = self.clock()
                for r in batch:
                    r.start = t
                inflight[lane] = (self.ex.submit(lane, batch), batch)
                progressed = True
            if not progressed:
                nxt = pending[0].arrival - now if pending and not inflight else 5e-5
                self.idle(max(nxt, 1e-6))
        return summarize(requests)


def summarize(requests: list) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "throughput_per_s": len(requests) / span if span > 0 else float("inf"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


class HksExecutor:
    """Runs steps through the library: per lane a HIP stream and one context
    per N (contexts own workspaces, so lanes never share one); per N a pool of
    output slots [2][L][N] and of input ciphertexts per level; keys through
    a KeyStore."""

    def __init__(self, params: dict, lanes: int, max_batch: int, slots_per_n: int, keystore, inputs, seeds=None):
        """seeds: key id -> seed when the key store holds seeded keys (only
        their rows b_j; the rows a_j are regenerated in the key-switch kernel,
        Sec. 5.3), else None (full keys)."""
        import torch
        from . import hks
        self.hks, self.torch = hks, torch
        self.params = params      # log_n -> (q list, p list, dnum)
        self.ctx = [{n: hks.Context(n, q, p, d, max_batch=max_batch) for n, (q, p, d) in params.items()}
                    for _ in range(lanes)]
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.L = {n: len(q) for n, (q, p, d) in params.items()}
        self.out = {n: [hks.empty((2 * self.L[n] << n,)) for _ in range(slots_per_n)] for n in params}
        self.keys = keystore
        self.seeds = seeds
        self.inputs = inputs      # (log_n, level) -> list of device ciphertexts [2][level][N]

    def slots(self, log_n):
        return len(self.out[log_n])

    def out_level(self, r):
        return r.level if r.op == "rotate" else r.level - 1

    def out_view(self, r):
        lv = self.out_level(r)
        return self.out[r.log_n][r.slot][: 2 * lv << r.log_n].view(2, lv, 1 << r.log_n)

    def in_ct(self, r, which=0):
        pool = self.inputs[(r.log_n, r.level)]
        return pool[(r.rid + which) % len(pool)]

    def submit(self, lane, batch):
        hks, torch = self.hks, self.torch
        s = self.streams[lane]
        r0 = batch[0]
        ctx = self.ctx[lane][r0.log_n]
        kind = "rot" if r0.op == "rotate" else "rlk"
        kids = [(r.client, kind, r.log_n) for r in batch]
        keys = [self.keys.acquire(k, s) for k in kids]
        with torch.cuda.stream(s):
            outs = [self.out_view(r) for r in batch]
            a, b = [self.in_ct(r) for r in batch], [self.in_ct(r, 1) for r in batch]
            levels = [r.level for r in batch]
            seeds = None if self.seeds is None else [self.seeds[k] for k in kids]
            if r0.op == "rotate":
                gals = [hks.hks_galois_for_rotation(r.k, r.log_n) for r in batch]
                hks.hks_batch_rotate_mixed(ctx, a, levels, gals, keys, outs, seeds=seeds, stream=s)
            else:
                hks.hks_batch_mult_relin_mixed(ctx, a, b, levels, keys, True, outs, seeds=seeds, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.keys.hold(kids, ev)
        return ev

    def done(self, ev):
        if ev.query():
            self.keys.release(ev)
            return True
        return False

    def close(self):
        self.torch.cuda.synchronize()
        for lane in self.ctx:
            for c in lane.values():
                c.close()


class KeyStore:
    """Switching keys resident on the device up to `budget` bytes, in
    fixed-size device slots; a miss uploads the key's pinned host copy on the
    requesting stream.  Least recently used keys not read by an in-flight
    step are evicted first."""

    def __init__(self, host_keys: dict, budget: int):
        """host_keys: key id -> pinned host tensor; budget in bytes (at least
        lanes * max_batch keys, the most that steps in flight can hold)."""
        import torch
        self.torch = torch
        self.host = host_keys  # key id -> pinned host tensor
        self.slot_words = max(t.numel() for t in host_keys.values())
        self.n_slots = max(1, budget // (8 * self.slot_words))
        self.slots = [None] * self.n_slots   # device buffers, allocated on first use
        self.where = collections.OrderedDict()  # key id -> slot (LRU order)
        self.refs = collections.Counter()
        self.held = {}
        self.ready = {}  # key id -> event recorded after its upload
        self.uploads = 0

    def acquire(self, kid, stream):
        torch = self.torch
        if kid in self.where:
            self.where.move_to_end(kid)
            s = self.where[kid]
        else:
            if len(self.where) < self.n_slots:
                s = len(self.where)
            else:
                victim = next((k for k in self.where if self.refs[k] == 0), None)
                if victim is None:
                    raise RuntimeError("key budget smaller than the keys of the steps in flight")
                s = self.where.pop(victim)
            if self.slots[s] is None:
                self.slots[s] = torch.empty(self.slot_words, dtype=torch.int64, device="cuda").view(torch.uint64)
            src = self.host[kid]
            with torch.cuda.stream(stream):
                self.slots[s][: src.numel()].copy_(src.reshape(-1), non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(stream)
            self.ready[kid] = ev
            self.where[kid] = s
            self.uploads += 1
        # a key uploaded on another lane's stream is read after its copy
        stream.wait_event(self.ready[kid])
        self.refs[kid] += 1
        src = self.host[kid]
        return self.slots[s][: src.numel()].view(src.shape)

    def preload(self, stream):
        """Uploads every key (in key order) until the budget is full: with a
        budget above the key set, every key is resident afterwards."""
        for kid in list(self.host)[: self.n_slots]:
            self.acquire(kid, stream)
            self.refs[kid] -= 1
        stream.synchronize()

    def hold(self, kids, handle):
        self.held[id(handle)] = kids

    def release(self, handle):
        for k in self.held.pop(id(handle), []):
            self.refs[k] -= 1
