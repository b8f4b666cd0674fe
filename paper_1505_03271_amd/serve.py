"""Continuous-batching service of Rayleigh-Benard FV-LB runs on one GPU.

Requests (grid side n, Ra, Pr, steps) arrive over time.  A request is
admitted, first come first served, as soon as a group slot is free and its
device memory fits the HBM budget (one that needs more than the whole budget
is rejected at once and listed in the result); it then keeps its state resident in HBM
until it has done exactly its steps, when its Nusselt numbers are read
(FP64 device reductions) and its memory is released.  A request whose
populations became non-finite (the kernels raise its flag, and the group
skips it from then on) is listed as failed, with no result, and is left out
of the latency and throughput figures.  Admission, scheduling
and completion happen only between group launches (graph boundaries).

Which admitted requests run in the next launch is the policy:

* "all": every admitted request (processor sharing: each advances one step
  per group step, whatever its size);
* "srpt": shortest remaining work first, preemptive, with aging.  Admitted
  requests are ranked by cells x remaining steps, divided by 1 + (time
  since admission) / age_s so that a long request that has waited is not
  starved, and the first run, as many as it takes to hold `min_cells`
  cells (enough work to fill the device; fewer cells per launch lower the
  throughput); the others wait resident in HBM and resume later exactly
  where they stopped (leaving and re-joining a group does not change a
  member's result).

    from paper_1505_03271_amd.serve import Server
    stats = Server(storage="bf16", hbm_budget=16e9).run(trace)

The physical set-up of a request follows the paper's recipe for its
Rayleigh-Benard runs (sec. 5): tau = tau_g = 1/2 for the smaller relaxation
time, free-fall velocity about 0.1, tanh wall refinement, periodic sides;
see workloads.rb_params.
"""
import time
from collections import deque

import numpy as np

from . import Group, LBError, Sim, current_stream, cell_bytes

LB_EUNSTABLE = 5

POLICIES = ("all", "srpt")


def request_bytes(n, storage, thermal=True):
    """Device memory of one request: two population buffers plus metric."""
    return 2 * n * n * cell_bytes(storage, thermal) + 64 * n + 4096


class Server:
    def __init__(self, storage="bf16", hbm_budget=16e9, max_sims=128, graph_steps=100, stream=None,
                 stretch=2.0, policy="srpt", min_cells=8e6, age_s=5.0, max_resident=None):
        """max_sims: group slots (requests running in one launch);
        max_resident: admitted requests held in HBM (default max_sims; with
        "all" every resident request runs, so it is at most max_sims)."""
        if policy not in POLICIES:
            raise ValueError(f"policy must be one of {POLICIES}")
        if not age_s > 0:
            raise ValueError("age_s must be > 0")
        self.storage = storage
        self.hbm_budget = float(hbm_budget)
        self.graph_steps = int(graph_steps)
        self.stretch = stretch
        self.policy = policy
        self.min_cells = float(min_cells)
        self.age_s = float(age_s)
        self.stream = stream if stream is not None else current_stream()
        self.group = Group(max_sims, self.stream)
        self.max_sims = max_sims
        self.max_resident = max_sims if max_resident is None or policy == "all" else int(max_resident)

    def _make(self, req):
        import workloads
        n = req["n"]
        # cfl (optional, default 1): dt in units of the smallest cell
        P = workloads.rb_params(req["Ra"], req["Pr"], n, n, aspect=1.0, stretch=self.stretch,
                                cfl=req.get("cfl", 1.0))
        rho, ux, uy, T = workloads.rb_fields(n, P["yf"], P["dT"], P["T0"], P["beta_g"],
                                            seed_index=1000 + req["id"])
        sim = Sim(n, n, scheme="heun", storage=self.storage, thermal=True, wall_y=True, dt=P["dt"], tau=P["tau"],
                  tau_g=P["tau_g"], beta_g=P["beta_g"], T0=P["T0"], T_bottom=P["T_bottom"], T_top=P["T_top"],
                  stream=self.stream)
        sim.set_grid(P["xf"], P["yf"])
        sim.init(rho, ux, uy, T)
        return sim

    def _choose(self, resident, now):
        """Request ids to run in the next launch (now: the server clock)."""
        ids = sorted(resident, key=lambda k: resident[k]["admitted"])
        if self.policy == "all":
            return ids[:self.max_sims]

        def rank(k):
            r = resident[k]
            work = r["req"]["n"] ** 2 * r["left"]
            return (work / (1.0 + max(now - r["admitted"], 0.0) / self.age_s), r["admitted"])

        ids.sort(key=rank)
        run, cells = [], 0
        for k in ids[:self.max_sims]:
            run.append(k)
            cells += resident[k]["req"]["n"] ** 2
            if cells >= self.min_cells:
                break
        return run

    def run(self, trace, time_scale=1.0, log=None):
        """Serve `trace` (list of dicts with id, arrival [s], n, Ra, Pr, steps).
        Arrival times are replayed on the wall clock (scaled by time_scale).
        Returns per-request records and summary statistics."""
        pending = deque(sorted(trace, key=lambda r: r["arrival"]))
        queue = deque()
        resident = {}  # request id -> dict(req, sim, need, admitted, left, slot)
        done, rejected, failed = [], [], []
        used = 0.0
        cell_steps = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        launches = preemptions = 0
        phase = dict(prep_s=0.0, launch_s=0.0, wait_s=0.0, completion_s=0.0, idle_s=0.0)
        while pending or queue or resident:
            now = clock()
            while pending and pending[0]["arrival"] * time_scale <= now:
                queue.append(pending.popleft())
            # admission to HBM at the graph boundary, first come first served
            t = clock()
            while queue and len(resident) < self.max_resident:
                req = queue[0]
                need = request_bytes(req["n"], self.storage)
                if need > self.hbm_budget:   # can never fit: reject, serve the rest
                    queue.popleft()
                    rejected.append(dict(id=req["id"], n=req["n"], need_bytes=need))
                    if log:
                        log(f"req {req['id']:4d} n={req['n']:5d} rejected: needs {need:.3e} B, "
                            f"more than the whole budget")
                    continue
                if used + need > self.hbm_budget:
                    break
                queue.popleft()
                resident[req["id"]] = dict(req=req, sim=self._make(req), need=need, admitted=clock(),
                                           left=req["steps"], slot=None)
                used += need
            if not resident:
                if pending:  # idle until the next arrival
                    time.sleep(max(0.0, pending[0]["arrival"] * time_scale - clock()))
                    phase["idle_s"] += clock() - t
                continue
            # the members of the next launch
            run = set(self._choose(resident, clock()))
            for k, r in resident.items():
                if r["slot"] is not None and k not in run:
                    self.group.remove(r["slot"])
                    r["slot"] = None
                    preemptions += 1
            for k in sorted(run, key=lambda k: resident[k]["admitted"]):
                r = resident[k]
                if r["slot"] is None:
                    r["slot"] = self.group.add(r["sim"], r["left"])
            t1 = clock()
            phase["prep_s"] += t1 - t
            self.group.step(self.graph_steps)
            launches += 1
            t2 = clock()
            left = self.group.remaining()   # synchronises
            t3 = clock()
            phase["launch_s"] += t2 - t1
            phase["wait_s"] += t3 - t2
            for k in list(resident):
                r = resident[k]
                if r["slot"] is None:
                    continue
                r["left"] = left[r["slot"]]
                if r["left"] > 0:
                    continue
                req = r["req"]
                try:
                    nu = r["sim"].nusselt()   # raises LB_EUNSTABLE if the run blew up
                except LBError as e:
                    if e.code != LB_EUNSTABLE:
                        raise
                    nu = None
                t_done = clock()
                self.group.remove(r["slot"])
                r["sim"].close()
                del resident[k]
                used -= r["need"]
                if nu is None:   # not a result: listed apart, out of the latency and throughput figures
                    failed.append(dict(id=req["id"], n=req["n"], steps=req["steps"], Ra=req["Ra"], Pr=req["Pr"],
                                       finished=t_done, reason="non-finite populations"))
                    if log:
                        log(f"req {req['id']:4d} n={req['n']:5d} failed: non-finite populations")
                    continue
                cell_steps += req["n"] ** 2 * req["steps"]
                done.append(dict(id=req["id"], n=req["n"], steps=req["steps"], arrival=req["arrival"] * time_scale,
                                 admitted=r["admitted"], finished=t_done, latency=t_done - req["arrival"] * time_scale,
                                 queue_wait=r["admitted"] - req["arrival"] * time_scale, nu=nu))
                if log:
                    log(f"req {req['id']:4d} n={req['n']:5d} steps={req['steps']:6d} "
                        f"latency {done[-1]['latency']:.2f}s nu_vol={nu[2]:.3f}")
            phase["completion_s"] += clock() - t3
        makespan = clock()
        lat = np.array([d["latency"] for d in done])
        return dict(requests=done, n_requests=len(done), rejected=rejected, failed=failed, makespan_s=makespan,
                    p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                    p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                    aggregate_mlups=cell_steps / makespan / 1e6 if makespan > 0 else None,
                    graph_launches=launches, graph_steps=self.graph_steps, policy=self.policy,
                    min_cells=self.min_cells if self.policy == "srpt" else None,
                    age_s=self.age_s if self.policy == "srpt" else None, preemptions=preemptions,
                    phases_s={k: round(v, 3) for k, v in phase.items()})

    def close(self):
        self.group.close()
