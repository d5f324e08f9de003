"""Served form: a request loop with continuous batching.

Jet runs arrive over (wall-clock) time, each with its payload (the grid's
metric set and the initial state, built by the client in host memory), and
are served first come, first served.  A run is admitted when it has arrived,
a slot is free, its device footprint fits the HBM budget, and the runs
already resident do not yet give the stage kernels ``tiles_per_cu`` tiles per
compute unit (8: enough that the tail of each stage launch, where the last
tiles finish while other workgroups find no more, stays short; fewer tiles
cost throughput, more cost latency); its payload is then uploaded
and the run joins the resident set, where its state, metrics, clock and time
step stay in HBM for its whole life.  The resident set advances in chunks of
steps no longer than the shortest remaining run, so runs that arrive while
others are on the GPU join at the next chunk and finished runs leave,
freeing their slot and memory.  Two ways of advancing the resident set:

* ``mode="batch"`` (default): one batch over all resident runs -- one
  persistent launch per RK stage whose workgroups claim the tiles of every
  member, the step replayed from a hipGraph captured once; runs join and
  leave with ``Batch.add`` / ``Batch.remove`` (no new capture).  Members
  march chunks of ``batch_kchunk`` planes: the batch fills the device with
  many members, so no run needs short chunks to fill it by itself;
* ``mode="streams"``: every run owns a HIP stream and its steps are issued
  on it, so the device runs the stage kernels of small runs side by side.

The host never waits for a chunk, only for a run that completes (and, in
batch mode, for the queued steps when the member set changes).  All GPU
arithmetic happens in the HIP library through the C ABI; this module only
schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import binding as B
from . import inputs as I


@dataclass
class Run:
    rid: int
    arrival: float
    dims: tuple
    mach: float
    re_d: float
    steps: int
    seed: int
    admitted: float = -1.0
    finished: float = -1.0
    remaining: int = 0
    footprint: int = 0
    solver: Optional[B.Solver] = None
    tiles: int = 0
    stream: object = None
    result: Optional[np.ndarray] = None
    ok: bool = True
    payload: Optional[tuple] = None   # (metrics 10 x N, state 5 x N), host arrays

    @property
    def points(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_runs(stream: List[dict]) -> List[Run]:
    return [Run(r, s["arrival"], tuple(s["dims"]), s["mach"], s["re_d"], s["steps"], s["seed"])
            for r, s in enumerate(stream)]


def _params(run: Run, precision: int, tile, kchunk: int = 0):
    """Solver parameters of a run; tile None (kchunk 0) leaves the tiling
    (the chunk length) to the library."""
    return B.params_default(precision=precision, mach_j=run.mach, re_d=run.re_d,
                            tile_i=tile[0] if tile else 0, tile_j=tile[1] if tile else 0, kchunk=kchunk)


def make_payload(run: Run) -> tuple:
    """The request's payload as a client builds it: the uniform jet box's
    metric set and initial state in host memory."""
    g, q = I.jet_box_case(run.dims, mach=run.mach, seed=run.seed)
    return g.metrics, q


def attach_payloads(runs: List[Run]) -> None:
    for r in runs:
        if r.payload is None:
            r.payload = make_payload(r)


def start_run(run: Run, precision: int, tile, kchunk: int = 0, stream=None) -> B.Solver:
    """Allocate the run's workspace and upload its payload (on ``stream``,
    the run's own stream, when given)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    m, q = run.payload if run.payload is not None else make_payload(run)
    s = B.Solver(run.dims, _params(run, precision, tile, kchunk), stream=st)
    s.set_grid_metrics(m)
    s.set_state(q)
    return s


def footprint(run: Run, precision: int, tile, kchunk: int = 0) -> int:
    return B.workspace_bytes(run.dims, _params(run, precision, tile, kchunk))


def stage_tiles(solver: B.Solver) -> int:
    """workgroups of one stage launch of a (periodic) run"""
    ti, tj, kc = solver.tiling()
    ni, nj, nk = solver.dims
    return -(-ni // ti) * -(-nj // tj) * -(-nk // kc)


@dataclass
class ServeStats:
    runs: int
    wall_s: float
    latencies: List[float]
    point_stages: float
    max_resident: int
    max_resident_bytes: int
    chunks: int
    failed: int = 0
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = np.asarray(self.latencies)
        return {
            "runs": self.runs, "wall_s": self.wall_s,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "runs_per_hour": self.runs / self.wall_s * 3600.0 if self.wall_s > 0 else None,
            "point_stage_updates_per_s": self.point_stages / self.wall_s if self.wall_s > 0 else None,
            "max_resident_runs": self.max_resident, "max_resident_bytes": self.max_resident_bytes,
            "chunks": self.chunks, "failed": self.failed, **self.extra,
        }


class JetServer:
    """Continuous-batching server for jet runs on one GPU."""

    def __init__(self, precision: int = B.JZ_FP64, budget_bytes: int = 200 << 30, max_resident: int = 64,
                 chunk_steps: int = 20, tile=None, keep_results: bool = False, fill_tiles: Optional[int] = None,
                 mode: str = "batch", tiles_per_cu: float = 8.0, batch_kchunk: int = 32):
        if mode not in ("streams", "batch"):
            raise ValueError("mode is 'streams' or 'batch'")
        self.mode = mode
        self.precision = precision
        self.budget = int(budget_bytes)
        self.max_resident = int(max_resident)
        self.chunk = int(chunk_steps)
        self.tile = tuple(tile) if tile else None
        self.keep_results = keep_results
        # resident tiles at which admission stops (None: tiles_per_cu times
        # the compute units, read from the first admitted run)
        self.fill_tiles = fill_tiles
        self.tiles_per_cu = float(tiles_per_cu)
        self.kchunk = int(batch_kchunk) if mode == "batch" else 0

    def serve(self, runs: List[Run], time_scale: float = 1.0) -> ServeStats:
        """Play the arrival stream (arrival times scaled by time_scale) and
        return latency and throughput figures."""
        import torch
        pending = deque(sorted(runs, key=lambda r: r.arrival))
        resident: List[Run] = []
        finishing: List[Run] = []     # done on the device (or queued to be), results not read yet
        batch: Optional[B.Batch] = None
        used, used_tiles = 0, 0
        max_res, max_bytes, chunks, failed = 0, 0, 0, 0
        point_stages = 0.0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        upload_s, collect_s = 0.0, 0.0   # host time in admissions (uploads) and in reading results

        def collect(rs):
            nonlocal used, failed, collect_s
            tc = time.perf_counter()
            for r in rs:
                try:
                    # on the run's own stream, which follows its last step
                    out = r.solver.get_state() if self.keep_results else None
                    r.solver.residual_norms()
                except B.JzError:
                    r.ok = False
                    failed += 1
                    out = None
                r.result = out
                r.finished = now()
                r.solver.close()
                r.solver = None
                used -= r.footprint
            collect_s += time.perf_counter() - tc

        try:
            while pending or resident or finishing:
                # admission: arrived, a free slot, the footprint fits the budget,
                # and the resident runs do not fill the device yet; the payload
                # upload overlaps the steps already queued
                while pending and pending[0].arrival * time_scale <= now() and len(resident) < self.max_resident:
                    if resident and self.fill_tiles is not None and used_tiles >= self.fill_tiles:
                        break
                    r = pending[0]
                    fp = footprint(r, self.precision, self.tile, self.kchunk)
                    if fp > self.budget:
                        pending.popleft()          # can never fit: reject
                        r.ok, r.finished = False, now()
                        failed += 1
                        continue
                    if used + fp > self.budget:
                        break
                    pending.popleft()
                    tu = time.perf_counter()
                    r.footprint = fp
                    # every run uploads, and is read back, on a stream of its
                    # own: after a removal the run's stream waits for the
                    # batch's queued steps, and a stream shared with the next
                    # admissions would hold their uploads behind those steps
                    r.stream = torch.cuda.Stream()
                    r.solver = start_run(r, self.precision, self.tile, self.kchunk, stream=r.stream)
                    r.tiles = stage_tiles(r.solver)
                    if self.fill_tiles is None:
                        _, cus = r.solver.occupancy()
                        self.fill_tiles = int(self.tiles_per_cu * cus)
                    if self.mode == "batch":
                        if batch is None:
                            batch = B.Batch([r.solver])
                            batch.set_timing(True)
                        else:
                            batch.add(r.solver)
                    upload_s += time.perf_counter() - tu
                    r.admitted = now()
                    r.remaining = r.steps
                    used += fp
                    used_tiles += r.tiles
                    resident.append(r)
                max_res = max(max_res, len(resident))
                max_bytes = max(max_bytes, used)
                earlier, finishing = finishing, []
                if resident:
                    # Enqueue the next chunk without waiting for the device: the
                    # host knows every run's progress, and the streams order the work.
                    n = min(self.chunk, min(r.remaining for r in resident))
                    if self.mode == "batch":
                        batch.advance(n)
                    else:
                        for r in resident:
                            r.solver.advance(n)
                    chunks += 1
                    point_stages += sum(r.points for r in resident) * 5.0 * n
                    for r in list(resident):
                        r.remaining -= n
                        if r.remaining == 0:
                            if batch is not None:
                                batch.remove(r.solver)   # no wait: its stream follows this chunk
                            resident.remove(r)
                            used_tiles -= r.tiles
                            finishing.append(r)
                # read the runs that finished in the previous chunk while the
                # device works on this one (all of them if nothing is queued)
                collect(earlier)
                if not resident:
                    collect(finishing)
                    finishing = []
                    if pending and not resident:
                        wait = pending[0].arrival * time_scale - now()
                        if wait > 0:
                            time.sleep(min(wait, 0.05))
        except BaseException:
            # release what is on the device before the error propagates
            if batch is not None:
                batch.close()
            for r in resident + finishing:
                if r.solver is not None:
                    r.solver.close()
                    r.solver = None
            raise
        gpu_step_s = None
        if batch is not None:
            batch.synchronize()
            gpu_step_s = batch.timing()[0] / 1e3
            batch.close()
        torch.cuda.synchronize()
        wall = now()
        ok = [r for r in runs if r.ok]
        extra = {"host_upload_s": upload_s, "host_collect_s": collect_s}
        if gpu_step_s is not None:
            extra["gpu_step_s"] = gpu_step_s   # the batch's steps, timed by events on its stream
        return ServeStats(len(ok), wall, [r.latency for r in ok], point_stages, max_res, max_bytes, chunks,
                          failed, extra)


def run_alone(run: Run, precision: int, tile, keep_result: bool = False):
    """The run by itself on an otherwise idle GPU, with the library's launch
    shape for its size (chunks short enough to fill the device): (seconds
    from the upload of its payload to its result, final state)."""
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    s = start_run(run, precision, tile)
    s.advance(run.steps)
    out = s.get_state() if keep_result else None
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    s.close()
    return el, out


def sequential_baseline(runs: List[Run], precision: int, tile) -> dict:
    """Each run alone, in arrival order, one at a time (first come first
    served, no overlap): latencies from the measured solo durations."""
    durations = [run_alone(r, precision, tile)[0] for r in sorted(runs, key=lambda r: r.arrival)]
    t_free, lat = 0.0, []
    for r, d in zip(sorted(runs, key=lambda r: r.arrival), durations):
        start = max(t_free, r.arrival)
        t_free = start + d
        lat.append(t_free - r.arrival)
    wall = t_free - min(r.arrival for r in runs)
    pts = sum(r.points * 5.0 * r.steps for r in runs)
    lat = np.asarray(lat)
    return {"runs": len(runs), "wall_s": wall, "busy_s": float(sum(durations)),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "runs_per_hour": len(runs) / wall * 3600.0, "point_stage_updates_per_s": pts / sum(durations)}
