"""A request loop for the encrypted-histogram path with continuous batching.

Parties send three kinds of requests to the GPU that holds the keys and the
resident encrypted gradients of the current round:

* ``encrypt``   -- the active party encrypts a batch of gradient values;
* ``aggregate`` -- a passive party asks for the encrypted histogram of one
  tree node over its own feature bins (Sec. III-B), read from the resident
  ciphertexts;
* ``decrypt``   -- the active party decrypts a returned histogram.

The loop runs on one host thread against wall-clock time.  Requests that have
arrived wait in a FIFO queue; a request is admitted when its estimated device
memory footprint fits in the free part of the HBM budget (the configured
budget, capped by the device memory that is free when the server starts) and
an in-flight slot is free.  Before the clock starts, the backend runs the
largest launch of each kind the trace can form on every stream, so the
library's per-stream workspaces never grow (and never wait) mid-trace.  Every loop turn groups what was admitted into launches -- all
admitted aggregate jobs of one key become one batched persistent launch, all
admitted decryptions of one key one launch over their concatenated
ciphertexts, each encryption its own launch -- and puts each launch on the
next of several streams, so launches admitted while others run overlap on the
device.  Completion is observed by polling one event per launch; memory and
slots are released then.  With ``policy="fifo"`` the same loop degenerates to
the plain baseline: one request per launch, one stream, arrival order.

The device work goes through a ``Backend``; ``GpuBackend`` calls the HIP
library, and the scheduling logic is independent of it (tests drive it with a
simulated backend on the CPU).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional, Sequence, Tuple


@dataclass
class Request:
    rid: int
    kind: str                    # "encrypt" | "aggregate" | "decrypt"
    key_id: str
    arrival: float               # seconds from the start of the trace
    party: int = 0
    payload: Dict[str, Any] = field(default_factory=dict)
    # filled by the server
    bytes: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Any = None
    status: str = "new"          # new | queued | running | done | rejected | cancelled

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


@dataclass
class Launch:
    requests: List[Request]
    handle: Any
    bytes: int
    stream_slot: int


class Backend:
    """Device operations the server needs."""

    n_streams: int = 1

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def launch(self, kind: str, key_id: str, reqs: Sequence[Request], slot: int) -> Any:
        """Enqueue one launch for these requests (same kind and key)."""
        raise NotImplementedError

    def done(self, handle: Any) -> bool:
        raise NotImplementedError

    def finish(self, handle: Any, reqs: Sequence[Request]) -> None:
        """Store each request's result (called once the launch is done)."""
        raise NotImplementedError


class Server:
    def __init__(self, backend: Backend, hbm_budget: int, max_inflight: int = 8,
                 policy: str = "continuous", clock=time.perf_counter, sleep=time.sleep,
                 idle_sleep: float = 2e-4):
        if policy not in ("continuous", "fifo"):
            raise ValueError(policy)
        self.backend = backend
        # the budget never exceeds what the device can still give (a backend
        # that knows its device reports that)
        dev = backend.device_budget() if hasattr(backend, "device_budget") else None
        self.budget = int(hbm_budget) if dev is None else min(int(hbm_budget), int(dev))
        self.max_inflight = 1 if policy == "fifo" else max_inflight
        self.policy = policy
        self.clock = clock
        self.sleep = sleep
        self.idle_sleep = idle_sleep
        self.queue: deque = deque()
        self.inflight: List[Launch] = []
        self.used = 0
        self.peak_used = 0
        self.launches = 0
        self._slot = 0
        self._cancelled: set = set()

    # ----------------------------------------------------------- admission
    def cancel(self, rid: int) -> None:
        """Cancels a request that has not been admitted yet."""
        self._cancelled.add(rid)

    def _admit(self, now: float) -> List[Request]:
        admitted: List[Request] = []
        slots = self.max_inflight - len(self.inflight)
        while self.queue and slots > 0:
            r = self.queue[0]
            if r.rid in self._cancelled:
                self.queue.popleft()
                r.status = "cancelled"
                continue
            if r.bytes > self.budget:
                self.queue.popleft()
                r.status = "rejected"
                continue
            if self.used + r.bytes > self.budget:
                break  # head of line waits for memory; FIFO order is kept
            self.queue.popleft()
            self.used += r.bytes
            self.peak_used = max(self.peak_used, self.used)
            r.t_admit = now
            r.status = "running"
            admitted.append(r)
            if self.policy == "fifo":
                break
            # requests of one kind and key admitted together share one launch,
            # so only a new group costs a slot
            if not any(a.kind == r.kind and a.key_id == r.key_id and a.kind != "encrypt"
                       for a in admitted[:-1]):
                slots -= 1
        return admitted

    def _dispatch(self, admitted: List[Request]) -> None:
        groups: Dict[Tuple[str, str], List[Request]] = {}
        order: List[Tuple[str, str]] = []
        for r in admitted:
            if r.kind == "encrypt" or self.policy == "fifo":
                k = (r.kind, r.key_id, r.rid)
            else:
                k = (r.kind, r.key_id)
            if k not in groups:
                groups[k] = []
                order.append(k)
            groups[k].append(r)
        for k in order:
            reqs = groups[k]
            slot = self._slot % max(1, self.backend.n_streams if self.policy == "continuous" else 1)
            self._slot += 1
            h = self.backend.launch(reqs[0].kind, reqs[0].key_id, reqs, slot)
            self.launches += 1
            self.inflight.append(Launch(reqs, h, sum(r.bytes for r in reqs), slot))

    def _reap(self, now: float) -> int:
        done = 0
        keep = []
        for L in self.inflight:
            if self.backend.done(L.handle):
                self.backend.finish(L.handle, L.requests)
                for r in L.requests:
                    r.t_done = now
                    r.status = "done"
                self.used -= L.bytes
                done += len(L.requests)
            else:
                keep.append(L)
        self.inflight = keep
        return done

    # ----------------------------------------------------------------- loop
    def run(self, trace: Sequence[Request], time_limit: float = 600.0) -> Dict[str, Any]:
        reqs = sorted(trace, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            r.bytes = int(self.backend.footprint(r))
            r.status = "new"
        if hasattr(self.backend, "prepare"):
            # before the clock starts: size whatever per-stream state the
            # largest launches of this trace need, so none grows mid-trace
            self.backend.prepare(reqs, self.max_inflight)
        t0 = self.clock()
        nxt = 0
        remaining = len(reqs)
        while remaining:
            now = self.clock() - t0
            if now > time_limit:
                raise TimeoutError(f"serving loop exceeded {time_limit} s with {remaining} requests left")
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                reqs[nxt].status = "queued"
                self.queue.append(reqs[nxt])
                nxt += 1
            finished = self._reap(now)
            remaining -= finished
            before = len(self.queue)
            admitted = self._admit(now)
            dropped = before - len(self.queue) - len(admitted)
            remaining -= dropped
            if admitted:
                self._dispatch(admitted)
            if not finished and not admitted and not dropped:
                self.sleep(self.idle_sleep)
        makespan = self.clock() - t0
        return summarize(reqs, makespan, self)


def percentile(xs: Sequence[float], q: float) -> Optional[float]:
    if not xs:
        return None
    xs = sorted(xs)
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def summarize(reqs: Sequence[Request], makespan: float, server: Optional[Server] = None) -> Dict[str, Any]:
    done = [r for r in reqs if r.status == "done"]
    lat = [r.latency for r in done]
    out: Dict[str, Any] = {
        "requests": len(reqs),
        "completed": len(done),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "cancelled": sum(r.status == "cancelled" for r in reqs),
        "makespan_s": round(makespan, 4),
        "throughput_req_s": round(len(done) / makespan, 3) if makespan > 0 else None,
        "p50_ms": None if not lat else round(percentile(lat, 0.5) * 1e3, 3),
        "p99_ms": None if not lat else round(percentile(lat, 0.99) * 1e3, 3),
        "by_kind": {},
    }
    for kind in ("encrypt", "aggregate", "decrypt"):
        lk = [r.latency for r in done if r.kind == kind]
        if lk:
            out["by_kind"][kind] = {"n": len(lk), "p50_ms": round(percentile(lk, 0.5) * 1e3, 3),
                                    "p99_ms": round(percentile(lk, 0.99) * 1e3, 3)}
    if server is not None:
        out["launches"] = server.launches
        out["peak_hbm_bytes"] = server.peak_used
        out["policy"] = server.policy
    return out


# ============================================================== GPU backend
class GpuBackend(Backend):
    """Runs requests with the HIP library on the current device.

    keys: {key_id: he.Key}; pools: {key_id: pipeline.Resident} (the resident
    encrypted gradients that aggregate requests read); bins: {(key_id,
    party): (uint8 [F_max, rows] device tensor, n_bins)} (each passive
    party's feature bins)."""

    def __init__(self, keys, pools, bins, n_streams: int = 4, chunk: int = 0, enc_slice: int = 0):
        import torch
        from . import he
        self.he = he
        self.torch = torch
        self.keys = keys
        self.pools = pools
        self.bins = bins
        self.n_streams = n_streams
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.chunk = chunk
        # encryptions longer than enc_slice values go out as several launches
        # (consecutive stretches of the same seeded r stream), so launches of
        # other streams can run between them; 0 = one launch
        self.enc_slice = enc_slice

    def device_budget(self, reserve: int = 2 << 30) -> int:
        """Free device memory now, less a reserve for the allocator."""
        free, _ = self.torch.cuda.mem_get_info()
        return max(0, int(free) - reserve)

    def prepare(self, reqs: Sequence[Request], max_group: int) -> None:
        """Runs, on every stream, the largest launch of each kind and key the
        trace can form (the largest encryption slice; the `max_group` largest
        decryptions, resp. aggregations, of one key merged into one launch),
        so the library's per-stream workspaces reach their final size before
        serving starts and never grow (a growth waits for the stream)."""
        torch, he = self.torch, self.he
        plans = []
        for kid in sorted({r.key_id for r in reqs}):
            mine = [r for r in reqs if r.key_id == kid]
            enc = [r for r in mine if r.kind == "encrypt"]
            if enc:
                n = max(r.payload["m"].numel() for r in enc)
                plans.append(("encrypt", kid, min(n, self.enc_slice or n)))
            dec = sorted((r.payload["ct"].numel() // (2 * self.keys[kid].limbs) for r in mine
                          if r.kind == "decrypt"), reverse=True)[:max_group]
            if dec:
                plans.append(("decrypt", kid, sum(dec)))
            agg = sorted((r for r in mine if r.kind == "aggregate"), key=lambda r: r.bytes,
                         reverse=True)[:max_group]
            if agg:
                plans.append(("aggregate", kid, agg))
        for st in self.streams:
            with torch.cuda.stream(st):
                for kind, kid, arg in plans:
                    key = self.keys[kid]
                    if kind == "encrypt":
                        m = torch.zeros(arg, dtype=torch.int64, device="cuda")
                        he.encrypt(key, m, seed=1, stream=st)
                    elif kind == "decrypt":
                        pool = self.pools[kid]
                        flat = pool.ct.view(-1, 2 * key.limbs)
                        reps = -(-arg // flat.shape[0])
                        ct = flat if reps == 1 else flat.repeat(reps, 1)
                        he.decrypt(key, ct[:arg].contiguous(), stream=st)
                    else:
                        jobs = []
                        for r in arg:
                            table, B = self.bins[(kid, r.party)]
                            jobs += [he.Job(idx, table[:F], B) for (idx, F) in r.payload["jobs"]]
                        he.hist_aggregate(key, self.pools[kid].ctm, jobs, form=he.HE_FORM_MONT,
                                          chunk=self.chunk, stream=st)
        torch.cuda.synchronize()

    # Footprint estimates mirror the buffers each launch allocates (outputs
    # plus library workspace).
    def footprint(self, req: Request) -> int:
        L = self.keys[req.key_id].limbs
        p = req.payload
        if req.kind == "encrypt":
            n = p["m"].numel()
            return n * (8 + 2 * L * 4 + 2 * L * 4) + (64 << 20)
        if req.kind == "decrypt":
            n = p["ct"].numel() // (2 * L)
            return n * (8 + L * 4) + (64 << 20)
        S = 2 * L
        tot = 0
        B = self.bins[(req.key_id, req.party)][1]
        for (idx, F) in p["jobs"]:
            n = idx.numel()
            items = F * ((n + 63) // 64 + min(B, n))
            tot += F * B * 2 * S * 4 + F * n * 4 + items * (16 + 2 * S * 4) + F * B * 20
        return tot + (16 << 20)

    def launch(self, kind: str, key_id: str, reqs: Sequence[Request], slot: int):
        torch, he = self.torch, self.he
        key = self.keys[key_id]
        st = self.streams[slot % self.n_streams]
        with torch.cuda.stream(st):
            if kind == "encrypt":
                (r,) = reqs
                m = r.payload["m"]
                n = m.numel()
                out = torch.empty((n, 2 * key.limbs), dtype=torch.int32, device=m.device)
                step = self.enc_slice or n
                off0 = r.payload.get("offset", 0)
                for a in range(0, n, step):
                    b = min(n, a + step)
                    he.encrypt(key, m[a:b], seed=r.payload["seed"], offset=off0 + a, out=out[a:b], stream=st)
                r.result = out
                outs = None
            elif kind == "aggregate":
                pool = self.pools[key_id]
                jobs, owners = [], []
                for r in reqs:
                    table, B = self.bins[(key_id, r.party)]
                    for (idx, F) in r.payload["jobs"]:
                        jobs.append(he.Job(idx, table[:F], B))
                        owners.append(r)
                he.hist_aggregate(key, pool.ctm, jobs, form=he.HE_FORM_MONT, chunk=self.chunk, stream=st)
                outs = (jobs, owners)
            else:
                cts = [r.payload["ct"].reshape(-1, 2 * key.limbs) for r in reqs]
                allct = cts[0] if len(cts) == 1 else torch.cat(cts, 0)
                m, _, _ = he.decrypt(key, allct, stream=st)
                outs = (m, [c.shape[0] for c in cts])
            ev = torch.cuda.Event()
            ev.record(st)
        return (kind, reqs, outs, ev)

    def done(self, handle) -> bool:
        return handle[3].query()

    def finish(self, handle, reqs) -> None:
        kind, reqs, outs, _ = handle
        if kind == "aggregate":
            jobs, owners = outs
            for r in reqs:
                r.result = [j.hist for j, o in zip(jobs, owners) if o is r]
        elif kind == "decrypt":
            m, sizes = outs
            off = 0
            for r, n in zip(reqs, sizes):
                r.result = m[off:off + n]
                off += n


def build_trace(rng, n_requests: int, rate: float, setups: Dict[str, Dict[str, Any]],
                key_share: Dict[str, float], mix=(0.10, 0.45, 0.45), enc_range=(1_000, 100_000),
                max_decrypt: int = 64 * 256 * 2, feature_range=(8, 128)) -> List[Request]:
    """Poisson arrivals (mean `rate` per second) of encrypt / aggregate /
    decrypt requests.  setups[key_id] holds the device-resident state of one
    key: "m" (int64 [rows*2] encoded gradients), "ct" (int32 [rows, 2, 2L]),
    "nodes" (list of int32 device tensors: the tree's node sample lists),
    "parties" (number of passive parties with bins for this key), "f_max".
    Request payloads are views of that state (nothing is copied); encrypt
    and decrypt payloads also name the flat index of their first value
    ("first") in the setup's gradient / ciphertext arrays."""
    import numpy as np
    from synth.workloads import poisson_arrivals
    times = poisson_arrivals(n_requests, rate, rng)
    ids = list(key_share)
    probs = np.array([key_share[k] for k in ids], dtype=np.float64)
    probs /= probs.sum()
    out = []
    for i, t in enumerate(times):
        kid = ids[int(rng.choice(len(ids), p=probs))]
        st = setups[kid]
        u = rng.random()
        rows = st["ct"].shape[0]
        if u < mix[0]:
            lo, hi = enc_range
            n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            n = min(n, rows)
            off = int(rng.integers(0, rows - n + 1))
            req = Request(i, "encrypt", kid, float(t), payload={
                "m": st["m"][2 * off:2 * (off + n)], "seed": int(rng.integers(1, 2 ** 62)), "offset": 0,
                "first": 2 * off})
        elif u < mix[0] + mix[1]:
            node = st["nodes"][int(rng.integers(len(st["nodes"])))]
            F = int(rng.integers(feature_range[0], min(feature_range[1], st["f_max"]) + 1))
            req = Request(i, "aggregate", kid, float(t), party=int(rng.integers(st["parties"])),
                          payload={"jobs": [(node, F)]})
        else:
            n = int(rng.integers(1, min(max_decrypt, 2 * rows) + 1))
            flat = st["ct"].view(-1, st["ct"].shape[-1])
            off = int(rng.integers(0, flat.shape[0] - n + 1))
            req = Request(i, "decrypt", kid, float(t), payload={"ct": flat[off:off + n], "first": off})
        out.append(req)
    return out


def clone_request(r: Request) -> Request:
    return Request(r.rid, r.kind, r.key_id, r.arrival, r.party, dict(r.payload))


def run_alone(backend: Backend, req: Request) -> Any:
    """Runs one request by itself (one launch on slot 0) and waits for it."""
    h = backend.launch(req.kind, req.key_id, [req], 0)
    while not backend.done(h):
        time.sleep(1e-4)
    backend.finish(h, [req])
    return req.result


def make_setup(key, rows: int, depth: int, n_parties: int, f_max: int, rng, r_seed: int,
               bin_choices=(16, 64, 256)):
    """Device-resident state of one key for serving: the round's encrypted
    gradients (canonical and Montgomery form), the node sample lists of a
    depth-`depth` tree over them, and each passive party's feature bins
    (Zipf(1.1) over a bin count drawn from `bin_choices`)."""
    import torch
    from synth import workloads as W
    from . import pipeline
    grads_h = W.gradients(rows, rng)
    grads = torch.from_numpy(grads_h).cuda()
    res = pipeline.encrypt_gradients(key, grads, r_seed)
    m = pipeline.he.encode(grads.reshape(-1).contiguous())
    levels = W.tree_levels(rows, depth, rng)
    nodes = [torch.from_numpy(n.view("int32")).cuda() for lvl in levels for n in lvl]
    bins, bins_h = {}, {}
    for p in range(n_parties):
        B = int(rng.choice(list(bin_choices)))
        bins_h[p] = W.bins_zipf(f_max, rows, B, rng)
        bins[p] = (torch.from_numpy(bins_h[p]).cuda(), B)
    torch.cuda.synchronize()
    return {"key": key, "pool": res, "m": m, "ct": res.ct, "nodes": nodes, "bins": bins,
            "parties": n_parties, "f_max": f_max,
            # host copies of the inputs, for checking results
            "grads_h": grads_h, "bins_h": bins_h, "r_seed": r_seed,
            "nodes_h": [n for lvl in levels for n in lvl]}


def backend_for(setups: Dict[str, Dict[str, Any]], n_streams: int = 4, chunk: int = 0,
                enc_slice: int = 0) -> "GpuBackend":
    keys = {k: s["key"] for k, s in setups.items()}
    pools = {k: s["pool"] for k, s in setups.items()}
    bins = {(k, p): v for k, s in setups.items() for p, v in s["bins"].items()}
    return GpuBackend(keys, pools, bins, n_streams=n_streams, chunk=chunk, enc_slice=enc_slice)
