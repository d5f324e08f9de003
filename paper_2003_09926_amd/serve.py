"""Served form: a request loop with continuous batching.

Jet runs arrive over (wall-clock) time and are served first come, first
served.  A run is admitted when it has arrived, a slot is free, its device
footprint fits the HBM budget, and the runs already resident do not yet give
the stage kernel enough workgroups to fill the device (``fill_tiles``, one
round of workgroups); its grid and initial state are then built directly in
device memory and it joins the resident set.  Small runs thus share the GPU
until together they fill it, while a run that fills it by itself runs alone
and keeps first-come latency.  The resident set advances in chunks of steps no
longer than the shortest remaining run, so runs that arrive while others are
on the GPU join at the next chunk and finished runs leave, freeing their slot
and memory.  Each run keeps its own state, metrics, clock and time step in
HBM for its whole life.  Two ways of advancing the resident set:

* ``mode="streams"`` (default): every run owns a HIP stream and the chunk of
  each resident run is issued on it, so the device runs the stage kernels of
  small runs side by side; joining and leaving cost nothing;
* ``mode="batch"``: one batch over all resident runs (one persistent launch
  per RK stage, step replayed from a hipGraph), rebuilt when the resident set
  changes.

The host never waits for a chunk, only for a run that completes.
All GPU arithmetic happens in the HIP library through the C ABI; this module
only schedules.
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

    @property
    def points(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_runs(stream: List[dict]) -> List[Run]:
    return [Run(r, s["arrival"], tuple(s["dims"]), s["mach"], s["re_d"], s["steps"], s["seed"])
            for r, s in enumerate(stream)]


def _params(run: Run, precision: int, tile):
    """Solver parameters of a run; tile None leaves the tiling to the library."""
    return B.params_default(precision=precision, mach_j=run.mach, re_d=run.re_d,
                            tile_i=tile[0] if tile else 0, tile_j=tile[1] if tile else 0)


def start_run(run: Run, precision: int, tile, device="cuda", stream=None) -> B.Solver:
    """Allocate the run's workspace, build its uniform jet box in device
    memory (on ``stream``, the run's own stream, when given) and hand grid and
    state to the library."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(st):
        s = B.Solver(run.dims, _params(run, precision, tile), stream=st)
        m, q = I.jet_box_device(run.dims, run.mach, run.seed, device)
        s.set_grid_metrics(m)
        s.set_state(q.reshape(-1))
    return s


def footprint(run: Run, precision: int, tile) -> int:
    return B.workspace_bytes(run.dims, _params(run, precision, tile))


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
                 mode: str = "streams"):
        if mode not in ("streams", "batch"):
            raise ValueError("mode is 'streams' or 'batch'")
        self.mode = mode
        self.precision = precision
        self.budget = int(budget_bytes)
        self.max_resident = int(max_resident)
        self.chunk = int(chunk_steps)
        self.tile = tuple(tile) if tile else None
        self.keep_results = keep_results
        # workgroups that fill the device for one round of the stage kernel
        # (None: taken from the first admitted run's occupancy)
        self.fill_tiles = fill_tiles

    def serve(self, runs: List[Run], time_scale: float = 1.0) -> ServeStats:
        """Play the arrival stream (arrival times scaled by time_scale) and
        return latency and throughput figures."""
        import torch
        pending = deque(sorted(runs, key=lambda r: r.arrival))
        resident: List[Run] = []
        batch: Optional[B.Batch] = None
        used, used_tiles = 0, 0
        max_res, max_bytes, chunks, failed = 0, 0, 0, 0
        point_stages = 0.0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or resident:
            changed = False
            # admission: arrived, a free slot, and the footprint fits the budget
            while pending and pending[0].arrival * time_scale <= now() and len(resident) < self.max_resident:
                if resident and self.fill_tiles is not None and used_tiles >= self.fill_tiles:
                    break                      # the resident runs already fill the device
                r = pending[0]
                fp = footprint(r, self.precision, self.tile)
                if fp > self.budget:
                    pending.popleft()          # can never fit: reject
                    r.ok, r.finished = False, now()
                    failed += 1
                    continue
                if used + fp > self.budget:
                    break
                pending.popleft()
                r.footprint = fp
                r.stream = torch.cuda.Stream() if self.mode == "streams" else None
                r.solver = start_run(r, self.precision, self.tile, stream=r.stream)
                r.tiles = stage_tiles(r.solver)
                if self.fill_tiles is None:
                    per_cu, cus = r.solver.occupancy()
                    self.fill_tiles = max(1, per_cu) * cus
                r.admitted = now()
                r.remaining = r.steps
                used += fp
                used_tiles += r.tiles
                resident.append(r)
                changed = True
            max_res = max(max_res, len(resident))
            max_bytes = max(max_bytes, used)
            if not resident:
                if pending:
                    wait = pending[0].arrival * time_scale - now()
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            # Enqueue the next chunk without waiting for the device: the host
            # knows every run's progress, and the stream orders the work (a
            # batch waits for earlier work on the stream and the stream for
            # the batch).  The host waits only when a run completes.
            n = min(self.chunk, min(r.remaining for r in resident))
            if self.mode == "streams" or len(resident) == 1:
                # each run's own launches, on its own stream
                if batch is not None:
                    batch.close()
                    batch = None
                for r in resident:
                    r.solver.advance(n)
            else:
                if changed or batch is None:
                    if batch is not None:
                        batch.close()
                    batch = B.Batch([r.solver for r in resident])
                batch.advance(n)
            chunks += 1
            point_stages += sum(r.points for r in resident) * 5.0 * n
            done = []
            for r in resident:
                r.remaining -= n
                if r.remaining == 0:
                    done.append(r)
            if done:
                if batch is not None:
                    batch.close()
                    batch = None
                for r in done:
                    if r.stream is not None:
                        r.stream.synchronize()
                    else:
                        torch.cuda.synchronize()
                t_done = now()
                for r in done:
                    try:
                        out = r.solver.get_state() if self.keep_results else None
                        r.solver.residual_norms()
                    except B.JzError:
                        r.ok = False
                        failed += 1
                        out = None
                    r.result = out
                    r.finished = t_done
                    r.solver.close()
                    r.solver = None
                    used -= r.footprint
                    used_tiles -= r.tiles
                    resident.remove(r)
        if batch is not None:
            batch.close()
        torch.cuda.synchronize()
        wall = now()
        ok = [r for r in runs if r.ok]
        return ServeStats(len(ok), wall, [r.latency for r in ok], point_stages, max_res, max_bytes, chunks,
                          failed)


def run_alone(run: Run, precision: int, tile, keep_result: bool = False):
    """The run by itself on an otherwise idle GPU: (seconds, final state)."""
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
