"""Continuous-batching server for droplet / wetting cases.

Requests arrive over time (each carries its arrival time).  A request is
admitted, first come first served, as soon as its HBM footprint fits the free
budget and a slot is free; admitted cases join the running group of their
lattice and storage at the next chunk boundary and advance together with the
cases already resident.  Each group has its own stream (default priority):
a chunk is launched on every group before any of them is polled, so groups of
different lattices (2D and 3D) run on the device at the same time.  A chunk is
at most `chunk_steps` steps and never takes a case past its step cap.  After
every chunk the groups are polled: cases that are steady (max |phi(t) -
phi(t - chunk)| <= steady_tol), non-finite, or at their step cap (the
request's "max_steps", else the server's) leave, their memory is freed and
waiting requests are admitted.

The executor is an interface (`Executor`): `GpuExecutor` drives the HIP
library; tests drive the same scheduler with a fake executor and clock.
Time-to-steady is measured from a request's arrival to the poll that found it
steady; time-to-result from arrival to the poll at which the case left
(steady, non-finite or capped).
"""
import collections
import time


class Executor:
    """What the scheduler needs from a backend."""

    def now(self):
        raise NotImplementedError

    def wait_until(self, t):
        raise NotImplementedError

    def footprint(self, req):
        raise NotImplementedError

    def admit(self, req):
        """Create the case on the device and add it to its group; returns a key."""
        raise NotImplementedError

    def step(self, nsteps):
        """Advance every admitted case nsteps (asynchronous on the device is
        fine: poll() waits)."""
        raise NotImplementedError

    def poll(self):
        """{key: dict(steady=bool, nonfinite=bool, steps=int, theta_deg=..., mass=...)}"""
        raise NotImplementedError

    def release(self, key):
        """Remove the case, free its memory; returns its final record (dict)."""
        raise NotImplementedError


class GpuExecutor(Executor):
    """Cases on the GPU, one group per (lattice, storage), each group on a
    stream of its own (default priority) so that the groups overlap."""

    def __init__(self, keep_fields=False, variant_2d=-1, variant_3d=-1):
        from . import pflbm as P
        self.P = P
        self.groups = {}
        self.streams = {}
        self.cases = {}
        self.keep_fields = keep_fields
        self.variants = {P.D2Q9: variant_2d, P.D3Q19: variant_3d, P.D3Q19_D3Q7: variant_3d}
        self._next = 0

    def now(self):
        return time.perf_counter()

    def wait_until(self, t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def params(self, req):
        return self.P.params_from_case(req, req.get("storage", "f32"),
                                       steady_tol=req.get("steady_tol", 1e-5))

    def footprint(self, req):
        return self.P.footprint(self.params(req))

    def admit(self, req):
        import torch
        prm = self.params(req)
        gk = (prm.lattice, prm.storage)
        if gk not in self.groups:
            self.streams[gk] = torch.cuda.Stream()          # default priority
            g = self.P.Group(stream=self.streams[gk])
            g.set_tile(self.variants[prm.lattice], 0)
            self.groups[gk] = g
        case = self.P.Case(prm, req["mask"], req["phi0"], stream=self.streams[gk])
        self.groups[gk].add(case)
        key = self._next
        self._next += 1
        self.cases[key] = (case, gk)
        return key

    def step(self, nsteps):
        # every group's chunk is enqueued on its own stream before poll() waits
        for g in self.groups.values():
            if len(g.members):
                g.step(nsteps)

    def poll(self):
        out = {}
        by_case = {id(c): k for k, (c, _) in self.cases.items()}
        for g in self.groups.values():
            if not len(g.members):
                continue
            diags, flags = g.poll()
            for m, d, f in zip(g.members, diags, flags):
                out[by_case[id(m)]] = dict(steady=bool(f & 1), nonfinite=bool(f & 2),
                                           steps=d["step"], theta_deg=d["theta_deg"],
                                           mass=d["mass"], residual=d["steady_residual"])
        return out

    def close(self):
        """Destroy the remaining cases and the groups."""
        for key in list(self.cases):
            case, gk = self.cases.pop(key)
            self.groups[gk].remove(case)
            case.close()
        for g in self.groups.values():
            g.close()
        self.groups = {}

    def release(self, key):
        case, gk = self.cases.pop(key)
        d = case.diagnostics()
        rec = dict(steps=d["step"], theta_deg=d["theta_deg"], mass=d["mass"],
                   nonfinite=d["nonfinite"])
        if self.keep_fields:
            rec["fields"] = case.fields()
        self.groups[gk].remove(case)
        case.close()
        return rec


class Server:
    def __init__(self, executor, budget_bytes, max_slots=64, chunk_steps=1000,
                 max_steps=200000):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk_steps)
        self.max_steps = int(max_steps)

    def run(self, requests):
        """Serve `requests` (dicts with 'arrival_s'); returns (records, summary)."""
        ex = self.ex
        pending = collections.deque(sorted(range(len(requests)),
                                           key=lambda i: requests[i]["arrival_s"]))
        waiting = collections.deque()
        active = {}             # key -> request index
        steps_done = {}         # key -> steps at the last poll
        used = 0
        fps = {}
        rec = [dict(index=i, arrival_s=requests[i]["arrival_s"],
                lattice=requests[i].get("lattice", "D2Q9")) for i in range(len(requests))]
        t0 = ex.now()
        busy = 0.0

        def clock():
            return ex.now() - t0

        while pending or waiting or active:
            now = clock()
            while pending and requests[pending[0]]["arrival_s"] <= now:
                waiting.append(pending.popleft())
            # admission: first come first served, by footprint and slots
            while waiting and len(active) < self.max_slots:
                i = waiting[0]
                fp = ex.footprint(requests[i])
                if fp > self.budget:
                    waiting.popleft()
                    rec[i].update(refused="footprint exceeds the budget", footprint=fp)
                    continue
                if used + fp > self.budget:
                    break
                waiting.popleft()
                key = ex.admit(requests[i])
                active[key] = i
                fps[key] = fp
                used += fp
                rec[i].update(admit_s=clock(), footprint=fp)
            if not active:
                if pending:
                    ex.wait_until(t0 + requests[pending[0]]["arrival_s"])
                    continue
                break
            tb = clock()
            # a chunk never takes a case past its step cap
            left = min(int(requests[i].get("max_steps", self.max_steps)) - steps_done.get(k, 0)
                       for k, i in active.items())
            ex.step(max(1, min(self.chunk, left)))
            status = ex.poll()
            busy += clock() - tb
            done_t = clock()
            for key, st in status.items():
                i = active.get(key)
                if i is None:
                    continue
                steps_done[key] = int(st["steps"])
                if st.get("residual") is not None:
                    rec[i].setdefault("residuals", []).append((int(st["steps"]), st["residual"]))
                cap = int(requests[i].get("max_steps", self.max_steps))
                finished = st["steady"] or st["nonfinite"] or st["steps"] >= cap
                if not finished:
                    continue
                r = ex.release(key)
                del active[key]
                used -= fps.pop(key)
                rec[i].update(r)
                rec[i]["done_s"] = done_t
                rec[i]["time_to_result_s"] = done_t - rec[i]["arrival_s"]
                rec[i]["steady"] = bool(st["steady"])
                rec[i]["status"] = ("steady" if st["steady"] else
                                    "nonfinite" if st["nonfinite"] else "step cap")
                if st["steady"]:
                    rec[i]["time_to_steady_s"] = done_t - rec[i]["arrival_s"]
        wall = clock()
        return rec, summarize(rec, wall, busy, requests)


def percentile(xs, q):
    if not xs:
        return None
    s = sorted(xs)
    k = (len(s) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def _nodes(req):
    if "nodes" in req:
        return int(req["nodes"])
    n = 1
    for v in req["shape"]:
        n *= int(v)
    return n


def summarize(rec, wall, busy, requests):
    tts = [r["time_to_steady_s"] for r in rec if "time_to_steady_s" in r]
    ttr = [r["time_to_result_s"] for r in rec if "time_to_result_s" in r]
    served = [r for r in rec if "done_s" in r]
    node_steps = sum(int(r.get("steps", 0)) * _nodes(requests[r["index"]]) for r in served)
    span = max(max(q["arrival_s"] for q in requests), 1e-9) if requests else 0.0
    by_lattice = {}
    for r in rec:
        b = by_lattice.setdefault(r["lattice"], dict(requests=0, steady=0, capped=0, nonfinite=0))
        b["requests"] += 1
        st = r.get("status")
        if st == "steady":
            b["steady"] += 1
        elif st == "step cap":
            b["capped"] += 1
        elif st == "nonfinite":
            b["nonfinite"] += 1
    return dict(requests=len(rec), served=len(served), steady=len(tts),
                refused=sum(1 for r in rec if "refused" in r),
                wall_s=wall, gpu_busy_s=busy, utilisation=busy / wall if wall > 0 else None,
                cases_per_s=len(served) / wall if wall > 0 else None,
                aggregate_MLUPS=node_steps / wall / 1e6 if wall > 0 else None,
                p50_time_to_steady_s=percentile(tts, 50),
                p99_time_to_steady_s=percentile(tts, 99),
                p50_time_to_result_s=percentile(ttr, 50),
                p99_time_to_result_s=percentile(ttr, 99),
                offered_rate_per_s=(len(requests) / span) if span else None,
                by_lattice=by_lattice)
