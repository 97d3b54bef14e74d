"""Serving shear-protocol jobs on one GPU.

A request is a whole simulation: a seeded synthetic suspension, a shear protocol and a
number of lattice steps; its result is the time-averaged stress (and G', G'' for
oscillatory shear).  Two ways of serving the same requests are measured:

* the plain loop: one job at a time in arrival order, every kernel launched one by one
  (``Simulation`` on the null stream);
* the batched server: jobs are admitted first come first served while the sum of their
  device footprints stays within a budget; an admitted job has all its steps queued at once
  on its own stream (``susp_batch_launch``: recorded step graphs, autotuned brick shape),
  so that jobs run side by side and none waits for another; a finished job leaves at once,
  freeing room for the next (continuous batching).

Latency of a job = time its result is available - its arrival time.  Arrivals are a
Poisson process.  The scheduling logic (``Server``) only talks to an executor object, so
that it can be tested on the CPU with a stand-in.
"""
from __future__ import annotations

import math
import multiprocessing
import time
from collections import deque
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import synth

# ---------------------------------------------------------------------------------------
# the request mix


@dataclass
class JobSpec:
    """One request: what to simulate and for how many steps."""
    jid: int
    kind: str                 # "2d" (monolayer, oscillatory) or "3d" (bulk, simple shear)
    L: int
    phi: float
    seed: int
    steps: int
    gamma_dot: float = 0.0    # 3d
    g0: float = 0.0           # 2d: strain amplitude
    theta: float = 0.0        # 2d: phase
    period: int = 1000        # 2d: steps per period
    arrival: float = 0.0      # seconds after the start


def mixed_jobs(n=64, seed=1904, steps=3000, period=1000, u_max=0.05):
    """Half quasi-2D monolayers (L in 128..384 step 32, L x L x 10, area fraction 0.70-0.80,
    oscillatory shear, steps/period periods split 2 initial + 1 observed), half 3D bulk
    suspensions (L in 64..128 step 16, phi 0.50-0.56, simple shear with log-uniform rate).
    Rates and amplitudes are drawn so that the Lees-Edwards velocity stays below u_max
    lattice units per step (the low-Mach range of the lattice-Boltzmann fluid)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        if i % 2 == 0:
            L = int(rng.choice(np.arange(128, 385, 32)))
            om = 2.0 * math.pi / period
            g0 = float(rng.uniform(0.2, 1.0)) * u_max / (L * om)
            jobs.append(JobSpec(i, "2d", L, float(rng.uniform(0.70, 0.80)), int(rng.integers(1 << 30)),
                                steps, g0=g0, theta=float(rng.uniform(0.0, math.pi)), period=period))
        else:
            L = int(rng.choice(np.arange(64, 129, 16)))
            hi = min(1e-3, u_max / L)
            gd = float(math.exp(rng.uniform(math.log(1e-5), math.log(hi))))
            jobs.append(JobSpec(i, "3d", L, float(rng.uniform(0.50, 0.56)), int(rng.integers(1 << 30)),
                                steps, gamma_dot=gd))
    return jobs


def workload(spec: JobSpec) -> synth.Workload:
    if spec.kind == "2d":
        ncyc_I = max(1, (2 * spec.steps) // (3 * spec.period))
        ncyc_F = max(1, spec.steps // spec.period - ncyc_I)
        return synth.monolayer(spec.L, 10, spec.phi, spec.seed, g0_I=spec.g0, g0_F=spec.g0,
                               theta=spec.theta, period=spec.period, ncyc_I=ncyc_I, ncyc_F=ncyc_F)
    return synth.bulk3d(spec.L, spec.phi, spec.gamma_dot, spec.seed)


def build_workloads(specs, workers=8):
    """Packings of all jobs (CPU, in worker processes).  The workers are spawned, not forked:
    the caller may already hold the GPU, and a forked copy of such a process is unsafe."""
    if workers <= 1:
        return [workload(s) for s in specs]
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(workload, specs))


def poisson_arrivals(n, rate, seed=1905):
    """Arrival times of n requests at the given mean rate (per second), first at 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def percentile(values, q):
    v = np.sort(np.asarray(values, dtype=float))
    if not v.size:
        return float("nan")
    return float(np.percentile(v, q))


def fifo_schedule(arrivals, service):
    """One server, first come first served: finish times given arrival and service times."""
    finish = np.zeros(len(arrivals))
    t = 0.0
    for i in np.argsort(arrivals, kind="stable"):
        t = max(t, arrivals[i]) + service[i]
        finish[i] = t
    return finish


# ---------------------------------------------------------------------------------------
# scheduling


@dataclass
class Done:
    jid: int
    arrival: float
    admitted: float
    finished: float
    result: object = None
    status: int = 0


@dataclass
class Server:
    """Continuous batching with first-come-first-served admission by footprint.

    Every admitted job runs on its own stream with a run of ``chunk`` steps queued; as soon
    as a job's run has completed the next one is queued (a whole job at once would overflow
    the hardware queue and block the host), so jobs run side by side and none waits for
    another.  The loop admits arrivals while they fit, tops up the jobs, collects finished
    ones (result, then memory) and otherwise sleeps a poll interval.  A job whose run reports
    a failure (an unstable state) is evicted at once, without a result, and its memory goes
    to the next; the other jobs go on.

    executor: footprint(job) -> bytes, add(job) -> slot or None (does not fit now),
              launch(slot, steps), poll(slot) -> (done, status), result(slot) -> object,
              remove(slot).
    clock:    function returning seconds (wall clock on the GPU)."""
    executor: object
    budget: int
    chunk: int = 100
    poll_s: float = 0.001
    clock: object = time.perf_counter
    sleep: object = time.sleep
    log: list = field(default_factory=list)
    host_s: float = 0.0   # time spent admitting jobs and queueing their steps
    progress: object = None  # progress(finished, total), called as jobs finish

    def run(self, jobs):
        ex = self.executor
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        queue = deque()
        active = {}   # slot -> [job, admitted time, steps not yet queued, worst status]
        done = []
        for j in jobs:
            if ex.footprint(j) > self.budget:
                raise ValueError("job %d can never fit in the budget" % j.jid)

        def top_up(slot):
            v = active[slot]
            n = min(self.chunk, v[2])
            h0 = self.clock()
            ex.launch(slot, n)
            self.host_s += self.clock() - h0
            v[2] -= n

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            while queue:  # first come first served: the head waits until it fits
                h0 = self.clock()
                slot = ex.add(queue[0])
                self.host_s += self.clock() - h0
                if slot is None:
                    break
                j = queue.popleft()
                active[slot] = [j, now(), j.steps, 0]
                top_up(slot)
            progressed = False
            for slot in list(active):
                ok, status = ex.poll(slot)
                if not ok:
                    continue
                progressed = True
                v = active[slot]
                v[3] = v[3] or status
                if v[2] > 0 and not status:
                    top_up(slot)
                    continue
                del active[slot]
                res = ex.result(slot) if not status else None  # a failed job is evicted
                ex.remove(slot)
                done.append(Done(v[0].jid, v[0].arrival, v[1], now(), res, v[3]))
                if self.progress is not None:
                    self.progress(len(done), len(jobs))
            self.log.append((now(), len(active)))
            if not progressed:
                wait = self.poll_s
                if not active and not queue and pending:
                    wait = max(wait, pending[0].arrival - now())
                self.sleep(wait)
        return sorted(done, key=lambda d: d.jid)


@dataclass
class LockstepServer:
    """Continuous batching in lockstep runs: every admitted job takes the same run of steps,
    and each kernel of a step is one launch over all of them (``susp_batch_launch_all``).

    When a run has completed, the jobs that finished (or failed: evicted without a result)
    leave at once, the arrivals waiting are admitted first come first served while their
    footprints fit, and the next run starts with everyone admitted.  Admission waits for the
    run boundary because creating a job makes synchronous calls on the job's stream, and a
    stream can share a hardware queue with a lockstep stream: during a run they would wait
    for the queued run.  A run is ``chunk`` steps, or fewer if a job needs fewer to finish.

    executor: footprint(job) -> bytes, add(job) -> slot or None, launch_all(steps),
              poll(slot) -> (done, status), result(slot) -> object, remove(slot)."""
    executor: object
    budget: int
    chunk: int = 100
    poll_s: float = 0.0005
    clock: object = time.perf_counter
    sleep: object = time.sleep
    log: list = field(default_factory=list)
    host_s: float = 0.0
    progress: object = None
    runs: list = field(default_factory=list)  # per run: [launched, queued, completed, jobs, steps]

    def run(self, jobs):
        ex = self.executor
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        queue = deque()
        active = {}   # slot -> [job, admitted time, steps not yet run, worst status]
        running = []  # slots of the run on the GPU
        done = []
        for j in jobs:
            if ex.footprint(j) > self.budget:
                raise ValueError("job %d can never fit in the budget" % j.jid)
        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            progressed = False
            if running:
                states = [ex.poll(s) for s in running]
                if all(d for d, _ in states):
                    progressed = True
                    self.runs[-1][2] = now()
                    for s, (_, status) in zip(running, states):
                        v = active[s]
                        v[3] = v[3] or status
                        if v[2] > 0 and not status:
                            continue
                        del active[s]
                        res = ex.result(s) if not status else None
                        ex.remove(s)
                        done.append(Done(v[0].jid, v[0].arrival, v[1], now(), res, v[3]))
                        if self.progress is not None:
                            self.progress(len(done), len(jobs))
                    running = []
            if not running:
                while queue:
                    h0 = self.clock()
                    slot = ex.add(queue[0])
                    self.host_s += self.clock() - h0
                    if slot is None:
                        break
                    j = queue.popleft()
                    active[slot] = [j, now(), j.steps, 0]
            if not running and active:
                n = min(self.chunk, min(v[2] for v in active.values()))
                h0 = self.clock()
                ex.launch_all(n)
                self.host_s += self.clock() - h0
                self.runs.append([h0 - t0, now(), None, len(active), n])
                running = list(active)
                for s in running:
                    active[s][2] -= n
                progressed = True
            self.log.append((now(), len(active)))
            if not progressed:
                wait = self.poll_s
                if not active and not queue and pending:
                    wait = max(wait, pending[0].arrival - now())
                self.sleep(wait)
        return sorted(done, key=lambda d: d.jid)


# ---------------------------------------------------------------------------------------
# GPU executors (library calls only)


def job_params(spec, w, precision=1, brick=None):
    from . import susp
    kw = dict(w.params)
    if brick is not None:
        kw["brick_y"], kw["brick_z"] = brick
    return susp.make_params(w.box, radius=w.radius, pos=w.pos, vel=w.vel, omega=w.omega,
                            precision=precision, **kw)


class BatchExecutor:
    """Jobs in a susp_batch: autotuned brick shapes, one stream per job (``Server``), or
    the default brick in lockstep runs (``LockstepServer``, autotune off)."""

    def __init__(self, workloads, budget, max_jobs=64, precision=1, autotune=True):
        from . import susp
        self.susp = susp
        self.w = workloads
        self.precision = precision
        self.autotune = autotune
        self.batch = susp.Batch(max_jobs, budget, autotune=autotune)
        self._slot_job = {}
        self._fp = {}
        self.bricks = {}

    def footprint(self, spec):
        if spec.jid not in self._fp:
            self._fp[spec.jid] = self.susp.footprint_bytes(job_params(spec, self.w[spec.jid], self.precision))
        return self._fp[spec.jid]

    def tune(self, specs):
        """Autotune every lattice kind up front (the choice is cached by the batch)."""
        for s in specs:
            self.bricks[s.jid] = self.batch.tune(job_params(s, self.w[s.jid], self.precision))

    def add(self, spec):
        p = job_params(spec, self.w[spec.jid], self.precision)
        self.bricks[spec.jid] = self.batch.tune(p) if self.autotune else None
        slot = self.batch.add(p)
        if slot is not None:
            self._slot_job[slot] = spec.jid
        return slot

    def launch(self, slot, n):
        self.batch.launch(slot, n)

    def launch_all(self, n):
        self.batch.launch_all(n)

    def poll(self, slot):
        return self.batch.poll(slot)

    def result(self, slot):
        sig, gg = self.batch.stress(slot)
        R = self.batch.job(slot).get_particles()[0]
        return sig, gg, R

    def remove(self, slot):
        self.batch.remove(slot)
        self._slot_job.pop(slot, None)

    def close(self):
        self.batch.close()


def run_alone(spec, w, precision=1, brick=None, stream=None, graphs=0):
    """One job from start to result: the plain path, kernels one by one on the null stream
    unless a stream is given; graphs > 0 replays recorded step graphs of 2 x graphs steps
    instead.  Returns (seconds, (stress, G'/G'', positions))."""
    from . import susp
    import torch
    t0 = time.perf_counter()
    sim = susp.Simulation(job_params(spec, w, precision, brick), stream=stream)
    if graphs:
        sim.use_graphs(graphs)
    sim.step(spec.steps, check=False)
    sig, gg = sim.stress()
    R = sim.get_particles()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.close()
    return dt, (sig, gg, R)


def lockstep_probe(n_jobs=24, steps=100, seed=1904, budget=32 << 30, workers=8, log=print):
    """Per-step time of the request mix: every job alone (recorded step graphs on a stream,
    after 20 warm-up steps), summed, against one lockstep step of all of them together."""
    import torch
    from . import susp
    specs = mixed_jobs(n_jobs, seed, 1000)
    ws = build_workloads(specs, workers)
    st = torch.cuda.Stream()
    alone = []
    for s in specs:
        sim = susp.Simulation(job_params(s, ws[s.jid]), stream=st)
        sim.use_graphs(5)
        sim.step(20, check=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(steps, check=False)
        torch.cuda.synchronize()
        alone.append((time.perf_counter() - t) / steps * 1e3)
        sim.close()
    ex = BatchExecutor(ws, budget, max_jobs=n_jobs, autotune=False)
    slots = [ex.add(s) for s in specs]
    if None in slots:
        raise RuntimeError("the mix does not fit in the budget")

    def run(n):
        ex.launch_all(n)
        for k in slots:
            while not ex.poll(k)[0]:
                time.sleep(0.0002)
    run(20)  # issued directly (the jobs are new)
    run(20)  # records the pair of steps as a graph
    t = time.perf_counter()
    run(steps)
    lock = (time.perf_counter() - t) / steps * 1e3
    ex.close()
    nodes = sum(int(np.prod(ws[s.jid].box)) for s in specs)
    log("mix probe: %d jobs, %d nodes; alone %.3f ms per step summed, lockstep %.3f ms" % (n_jobs, nodes, sum(alone), lock))
    return {"jobs": n_jobs, "nodes": nodes, "steps": steps, "alone_ms_per_step_sum": round(sum(alone), 4),
            "alone_ms_per_step": [round(a, 4) for a in alone], "lockstep_ms_per_step": round(lock, 4),
            "ratio": round(sum(alone) / lock, 3)}


def serve_benchmark(n_jobs=64, steps=3000, budget=32 << 30, seed=1904, workers=8, recheck=None,
                    log=print, mode="lockstep"):
    """The plain loop and the batched server on the same requests; returns a summary.

    mode "lockstep": ``LockstepServer`` (one launch per kernel over all jobs, default brick);
    "streams": ``Server`` (one stream per job, autotuned bricks).

    The plain loop is timed twice, with every kernel launched one by one and with recorded
    step graphs replayed on a stream; the speedups are taken against the faster of the two.
    Every job (recheck=None), or the first `recheck`, is run alone again with the brick shape
    the server used, and its result compared bit for bit with the batched one."""
    import torch
    specs = mixed_jobs(n_jobs, seed, steps)
    t = time.perf_counter()
    ws = build_workloads(specs, workers)
    log("serving: %d jobs packed in %.1f s" % (n_jobs, time.perf_counter() - t))
    # plain loop: service time of every job alone, launches one by one, then graph replay
    service_l = np.zeros(n_jobs)
    for k, s in enumerate(specs):
        service_l[s.jid], _ = run_alone(s, ws[s.jid])
        if (k + 1) % 8 == 0:
            log("serving: plain loop %d/%d jobs, %.1f s" % (k + 1, n_jobs, float(service_l.sum())))
    gstream = torch.cuda.Stream()
    service_g = np.zeros(n_jobs)
    for s in specs:
        service_g[s.jid], _ = run_alone(s, ws[s.jid], stream=gstream, graphs=5)
    t_l, t_g = float(service_l.sum()), float(service_g.sum())
    log("serving: plain loop %.1f s (launches) / %.1f s (graphs) for %d jobs" % (t_l, t_g, n_jobs))
    service = service_g if t_g < t_l else service_l
    t_plain = float(service.sum())
    rate = n_jobs / (0.25 * t_plain)
    arr = poisson_arrivals(n_jobs, rate, seed + 1)
    for s, a in zip(specs, arr):
        s.arrival = float(a)
    fin_plain = fifo_schedule(arr, service)
    lat_plain = fin_plain - arr
    # batched server
    every = lambda k, n: k % 8 == 0 and log("serving: batched %d/%d jobs done" % (k, n))
    if mode == "lockstep":
        ex = BatchExecutor(ws, budget, max_jobs=n_jobs, autotune=False)
        t_tune = 0.0
        make = lambda: LockstepServer(ex, budget, progress=every)
    elif mode == "streams":
        ex = BatchExecutor(ws, budget, max_jobs=n_jobs)
        t = time.perf_counter()
        ex.tune(specs)
        t_tune = time.perf_counter() - t
        log("serving: autotuned %d lattice kinds in %.1f s" % (len(set((s.kind, s.L) for s in specs)), t_tune))
        make = lambda: Server(ex, budget, progress=every)
    else:
        raise ValueError("mode must be lockstep or streams")
    srv = make()
    done = srv.run(specs)
    torch.cuda.synchronize()
    # capacity: the same requests all present at the start (the server never idles)
    sat = [JobSpec(**{**s.__dict__, "arrival": 0.0}) for s in specs]
    t = time.perf_counter()
    srv_sat = make()
    srv_sat.run(sat)
    torch.cuda.synchronize()
    t_sat = time.perf_counter() - t
    ex.close()
    lat_b = np.array([d.finished - d.arrival for d in done])
    make_b = max(d.finished for d in done)
    make_p = float(fin_plain.max())
    # the same jobs alone must give the same results bit for bit
    same = 0
    checked = done if recheck is None else done[:recheck]
    for d in checked:
        s = specs[d.jid]
        _, res = run_alone(s, ws[s.jid], brick=ex.bricks[s.jid])
        ok = d.result is not None and all(np.array_equal(a, b) for a, b in zip(res, d.result))
        same += int(ok)
    peak = max((a for _, a in srv.log), default=0)
    peak_sat = max((a for _, a in srv_sat.log), default=0)
    return {
        "server": mode,
        "jobs": n_jobs,
        "steps_per_job": steps,
        "budget_bytes": int(budget),
        "arrival_rate_per_s": round(rate, 4),
        "plain_loop_s_launches": round(t_l, 3),
        "plain_loop_s_graphs": round(t_g, 3),
        "plain_baseline": "graphs" if t_g < t_l else "launches",
        "plain_jobs_per_hour": round(3600.0 * n_jobs / make_p, 1),
        "batched_jobs_per_hour": round(3600.0 * n_jobs / make_b, 1),
        "speedup": round(make_p / make_b, 3),
        "plain_capacity_jobs_per_hour": round(3600.0 * n_jobs / t_plain, 1),
        "batched_capacity_jobs_per_hour": round(3600.0 * n_jobs / t_sat, 1),
        "capacity_speedup": round(t_plain / t_sat, 3),
        "plain_p50_latency_s": round(percentile(lat_plain, 50), 3),
        "plain_p99_latency_s": round(percentile(lat_plain, 99), 3),
        "batched_p50_latency_s": round(percentile(lat_b, 50), 3),
        "batched_p99_latency_s": round(percentile(lat_b, 99), 3),
        "max_jobs_in_flight": int(peak),
        "max_jobs_in_flight_capacity": int(peak_sat),
        "autotune_s": round(t_tune, 2),
        "admission_host_s": round(srv.host_s, 2),
        "identical_alone": "%d/%d" % (same, len(checked)),
        "unstable_jobs": int(sum(1 for d in done if d.status != 0)),
    }
