"""Benchmark of the jet-LES hot path on one MI355X.

Default workload: one GPU's share of a production jet mesh -- the 512 x 256 x
256 separable tanh-stretched periodic grid (33.5M nodes) with analytic FP64
metrics, Mach 1.4 round jet at Re_D = 1e6 with 1 % seeded velocity noise,
advanced by the FP64 fused residual + five-stage RK path.  One "step" is one
full RK step (five fused stage kernels, the norm and dt reductions).

Prints one JSON line: point-stage updates per second (N x 5 x steps / time)
with the inputs resident in HBM, the roofline record of the stage kernel
(algorithmic bytes per launch / mean launch time from HIP events), and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (512, 256, 256)
PROFILES = os.path.join(ROOT, "profiles")


def _kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("jz_stage_kernel.h", "jz_stage.hip", "jz_stage32.hip", "jz_internal.h"):
        with open(os.path.join(ROOT, "paper_2003_09926_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str):
    """HBM bytes per launch measured with rocprofv3 counters, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec or rec.get("kernel_hash") != _kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(min_seconds: float = 10.0):
    """The oracle, as it stands (plain FP64 C++, -O3, OpenMP over outer
    loops), on the host cores: the stride-4 subsample of the workload (128 x
    64 x 64 nodes, same grid family and jet) stepped for at least
    ``min_seconds`` on all cores (the reported value), then for a few steps on
    one thread; and the 64 x 48 x 48 jet box (4 steps) on all cores."""
    import oracle
    from paper_2003_09926_amd import inputs as I

    def timed(dims, P, m, q, min_s, min_steps):
        steps, t0 = 0, time.perf_counter()
        while True:
            q, _, _, _ = oracle.step(dims, P, m, q)
            steps += 1
            el = time.perf_counter() - t0
            if el >= min_s and steps >= min_steps:
                return steps, el

    all_cores = oracle.threads(0)
    g, q = I.stretched_jet_case(DIMS, seed=2, stride=4)
    P = oracle.default_params(re_d=1.0e6)
    oracle.step(g.dims, P, g.metrics, q)          # warm (page-in, thread pool)
    steps, el = timed(g.dims, P, g.metrics, q, min_seconds, 2)
    oracle.threads(1)
    steps1, el1 = timed(g.dims, P, g.metrics, q, 0.0, 2)
    oracle.threads(all_cores)
    gb, qb = I.jet_box_case((64, 48, 48), seed=1)
    Pb = oracle.default_params()
    oracle.step(gb.dims, Pb, gb.metrics, qb)
    steps_b, el_b = timed(gb.dims, Pb, gb.metrics, qb, 0.0, 4)
    return {"value": g.n * 5 * steps / el, "unit": "point-stage updates/s", "cores": all_cores,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{steps} steps of the 128x64x64 stride-4 subsample of the 512x256x256 "
                      f"stretched jet grid (FP64 C++ oracle, -O3, OpenMP, {all_cores} threads), {el:.1f} s",
            "one_thread": {"value": g.n * 5 * steps1 / el1, "cores": 1,
                           "sample": f"{steps1} steps of the same subsample, {el1:.1f} s"},
            "jet_box_64x48x48": {"value": gb.n * 5 * steps_b / el_b, "cores": all_cores,
                                 "sample": f"{steps_b} steps of the 64x48x48 periodic jet box, {el_b:.2f} s"}}


def fp32_error_vs_oracle():
    """Config-3 error: the FP32-flux form against the FP64 oracle on the
    128 x 64 x 64 stride-4 subsample after 1 and 100 steps (relative L2 per
    conserved variable)."""
    import numpy as np
    import oracle
    from paper_2003_09926_amd import binding as B
    from paper_2003_09926_amd import inputs as I
    g, q = I.stretched_jet_case(DIMS, seed=2, stride=4)
    P = oracle.default_params(re_d=1.0e6)
    rel = lambda a, b: [float(np.linalg.norm(a[v] - b[v]) / np.linalg.norm(b[v])) for v in range(5)]
    with B.Solver(g.dims, B.params_default(re_d=1.0e6, precision=B.JZ_FP32_FLUX)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(1)
        g1 = s.get_state()
        s.advance(99)
        g100 = s.get_state()
    o1, _, _, _ = oracle.step(g.dims, P, g.metrics, q)
    o100, _, _, _ = oracle.advance(g.dims, P, g.metrics, q, 100)
    names = ["rho", "rho_u", "rho_v", "rho_w", "e"]
    return {"grid": "128x64x64 stride-4 subsample", "after_1_step": dict(zip(names, rel(g1, o1))),
            "after_100_steps": dict(zip(names, rel(g100, o100)))}


def _time_solver(s, n_adv: int, steps: int, warmup: int):
    """Advance warmup steps, then time `steps` steps: wall clock around the
    launches with the inputs resident, and hipEvents around each stage-kernel
    launch.  Returns (value, ms_per_step, avg_launch_ms, bytes_per_launch)."""
    import torch
    s.advance(warmup)
    torch.cuda.synchronize()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stage_ms, launches, stage_bytes = s.timing()
    s.set_timing(False)
    s.residual_norms()     # raises if the run went non-finite
    return (n_adv * 5 * steps / el, el * 1e3 / steps, stage_ms / max(launches, 1),
            stage_bytes / max(launches, 1))


def _rate_gbs(fn, nbytes_moved: int, reps: int = 10) -> float:
    """GB/s of `nbytes_moved` per call of fn, timed with events over reps
    calls after three untimed ones."""
    import torch
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return nbytes_moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def _stream_rate_gbs(nbytes: int = 2 << 30) -> float:
    """HBM rate a plain elementwise stream reaches on this GPU: b = 1.0 * a
    over 2 GiB of float32 (bytes read plus bytes written per second, GB/s),
    the achievable counterpart of the published peak."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    r = _rate_gbs(lambda: torch.mul(a, 1.0, out=b), 2 * nbytes)
    del a, b
    return r


def hbm_rates(nbytes: int = 2 << 30) -> dict:
    """Plain streaming rates of the GPU's HBM (GB/s, bytes read plus bytes
    written): the runtime's device-to-device copy, an elementwise stream,
    a read-only sum and a write-only fill, over nbytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {"bytes": nbytes,
           "device_copy": _rate_gbs(lambda: b.copy_(a), 2 * nbytes),
           "elementwise_stream": _rate_gbs(lambda: torch.mul(a, 1.0, out=b), 2 * nbytes),
           "read_sum": _rate_gbs(lambda: a.view(torch.float64).sum(), nbytes),
           "write_fill": _rate_gbs(lambda: b.fill_(1.0), nbytes)}
    del a, b
    return out


def run_block(form: str, steps: int, warmup: int, with_cpu: bool, with_error: bool, stats_interval: int = 0,
              with_secondary: bool = False):
    """fp64 / fp32: the periodic stretched jet block.  domain-fp64 /
    domain-fp32: the jet in a bounded 512 x 256 x 256 domain (uniform grid
    over x in [0, 4], y, z in [-1.5, 1.5]) with supersonic inflow at the jet
    exit and Riemann-invariant far field on the other five faces.
    cylinder-fp64 / cylinder-fp32: the jet on a 512 (axial) x 256 (radial) x
    256 (azimuthal) cylindrical mesh, radius 1.5, with the jet exit, far field
    at the outflow and lateral surface, the centreline and the periodic
    azimuth.  In both, the boundary kernels run after every stage inside the
    timed region, and the rate counts the advanced nodes."""
    import torch
    from paper_2003_09926_amd import binding as B
    from paper_2003_09926_amd import inputs as I

    torch.cuda.set_device(0)
    prec_name = form.split("-")[-1]
    prec = B.JZ_FP64 if prec_name == "fp64" else B.JZ_FP32_FLUX
    domain = form.startswith("domain")
    cylinder = form.startswith("cylinder")
    if domain:
        g, q, bc = I.jet_domain_case(DIMS, mach=1.4, seed=2)
        P = B.params_default(re_d=1.0e6, precision=prec, bc=bc)
        n_adv = (DIMS[0] - 4) * (DIMS[1] - 4) * (DIMS[2] - 4)
    elif cylinder:
        g, q, bc = I.jet_cylinder_case(DIMS, mach=1.4, seed=2)
        P = B.params_default(re_d=1.0e6, precision=prec, bc=bc, stats_interval=stats_interval)
        n_adv = (DIMS[0] - 4) * (DIMS[1] - 4) * DIMS[2]
    else:
        g, q = I.stretched_jet_case(DIMS, seed=2)
        P = B.params_default(re_d=1.0e6, precision=prec)
        n_adv = g.n
    s = B.Solver(g.dims, P)
    if cylinder:
        s.set_grid_coords(g.x, g.y, g.z, g.period)   # Thomas-Lombard metrics on the GPU
    else:
        s.set_grid_metrics(g.metrics)
    s.set_state(q)
    value, ms_step, avg_ms, bytes_per_launch = _time_solver(s, n_adv, steps, warmup)
    secondary = None
    if with_secondary and form == "fp64":
        # the FP32-flux form on the same resident workload, timed the same way
        s32 = B.Solver(g.dims, B.params_default(re_d=1.0e6, precision=B.JZ_FP32_FLUX))
        s32.set_grid_metrics(g.metrics)
        s32.set_state(q)
        v32, ms32, avg32, bytes32 = _time_solver(s32, n_adv, steps, warmup)
        s32.close()
        ach32 = bytes32 / (avg32 * 1e-3) / 1e9
        secondary = {"form": "fp32", "value": v32, "unit": "point-stage updates/s", "ms_per_step": ms32,
                     "speedup_vs_fp64": v32 / value,
                     "dtype": "f32 (fluxes) + f64 (accumulation, J, norms)",
                     "roofline": {"bound": "hbm", "achieved": ach32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": ach32 / HBM_PEAK_GBS, "traffic": _traffic("stage_fp32flux"),
                                  "kernel": "stage_fp32flux", "avg_launch_ms": avg32,
                                  "algorithmic_bytes_per_launch": bytes32}}
    del q
    stats_info = None
    if cylinder and stats_interval > 0:
        # the statistics of the run, and the potential core on the axis
        # (ring j = 0; the jet exit velocity is the Mach number)
        from paper_2003_09926_amd import stats as ST
        st = s.stats()
        ni, nj, nk = DIMS
        axis_u = st["mean_u"].reshape(nk, nj, ni)[0, 0, :]
        stats_info = {"interval": stats_interval, "samples": st["samples"],
                      "potential_core_length": ST.potential_core_length(g.axes[0], axis_u, 1.4),
                      "max_rms_u": float(st["rms_u"].max())}
    s.close()
    stream_gbs = _stream_rate_gbs()
    if secondary is not None:
        r32 = secondary["roofline"]
        r32["achievable_gbs"] = stream_gbs
        r32["frac_of_achievable"] = r32["achieved"] / stream_gbs
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernel = "stage_fp64" if prec_name == "fp64" else "stage_fp32flux"
    traffic = None if (domain or cylinder) else _traffic(kernel)
    out = {
        "metric": "point-stage updates/s", "value": value, "unit": "point-stage updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32 (fluxes) + f64 (accumulation, J, norms)",
        "data": "synthetic",
        "config": {"workload": (f"jet_domain_512x256x256_inflow_farfield_{prec_name}" if domain else
                                f"jet_cylinder_512x256x256_centreline_{prec_name}" if cylinder else
                                f"jet_512x256x256_stretched_{prec_name}"),
                   "dims": list(DIMS), "mach": 1.4, "re_d": 1.0e6, "seed": 2, "stages_per_step": 5,
                   "form": form, "advanced_nodes": n_adv},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "achievable_gbs": stream_gbs, "frac_of_achievable": achieved / stream_gbs},
    }
    if stats_info is not None:
        out["stats"] = stats_info
    if secondary is not None:
        out["secondary"] = secondary
    if with_error and form == "fp32":
        out["error_vs_oracle"] = fp32_error_vs_oracle()
    if with_cpu and not (domain or cylinder):
        out["cpu_baseline"] = cpu_baseline()
    return out


def run_batch(prec_name: str, steps: int, warmup: int):
    """Config 4: 64 periodic jet boxes [0,4) x [-1.5,1.5)^2 whose ni, nj, nk are
    uniform in [32, 160] (seed 4), Mach U[1.2, 2.0], Re_D log-uniform in
    [1e5, 1e6], each with its own CFL time step, advanced together; compared
    with the same blocks advanced one after another."""
    import tempfile
    import torch
    from paper_2003_09926_amd import binding as B
    from paper_2003_09926_amd import inputs as I

    torch.cuda.set_device(0)
    prec = B.JZ_FP64 if prec_name == "fp64" else B.JZ_FP32_FLUX
    tile = (28, 12) if prec == B.JZ_FP64 else (28, 20)
    mix = I.batch_mix(seed=4)
    members = []
    for blk in mix:
        g = I.uniform_box(*blk["dims"])
        q = I.jet_state(g, blk["mach"], blk["seed"])
        s = B.Solver(g.dims, B.params_default(precision=prec, mach_j=blk["mach"], re_d=blk["re_d"],
                                              tile_i=tile[0], tile_j=tile[1]))
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        members.append(s)
    npts = sum(m.n for m in members)
    b = B.Batch(members)
    cache = os.path.join(tempfile.gettempdir(), "jetles_batch_tune.txt")
    choice, _ = b.autotune(trial_steps=2, cache_path=cache)
    b.advance(warmup)
    b.synchronize()
    torch.cuda.synchronize()
    b.set_timing(True)
    t0 = time.perf_counter()
    b.advance(steps)
    b.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev_ms, ev_steps, _ = b.timing()
    b.close()
    for m in members:
        m.residual_norms()   # raises if a member went non-finite
    # the same blocks one after another, same tile shape, each with the chunk
    # length the library picks for its size (short enough to fill the device)
    for m in members:
        m.set_tiling(choice[0], choice[1], 0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for m in members:
        m.advance(steps)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1
    for m in members:
        m.close()
    value = npts * 5 * steps / el
    return {
        "metric": "point-stage updates/s", "value": value, "unit": "point-stage updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == B.JZ_FP64 else "f32 (fluxes) + f64 (accumulation, J, norms)",
        "data": "synthetic",
        "config": {"workload": f"batch_64_jet_boxes_{prec_name}", "blocks": len(mix), "points": npts,
                   "dims_range": [32, 160], "seed": 4, "form": f"batch-{prec_name}",
                   "autotuned_tile": list(choice), "graph": True},
        "sequential": {"value": npts * 5 * steps / el_seq, "ms_per_step": el_seq * 1e3 / steps,
                       "speedup_of_batch": el_seq / el},
        "event_ms_per_step": ev_ms / max(ev_steps, 1),
    }


def run_serve(prec_name: str, nruns: int, with_sequential: bool, mode: str = "batch"):
    """Config 5: Poisson arrivals (mean 20 runs/s, seed 5) of cubic jet runs
    n^3, n uniform in [48, 192], Mach U[1.2, 2.0], Re_D log-uniform
    [1e5, 1e6], 200 steps each at CFL 0.5, admitted under a 200 GB budget,
    served by continuous batching; compared with each run alone, one at a
    time in arrival order."""
    import torch
    from paper_2003_09926_amd import binding as B
    from paper_2003_09926_amd import inputs as I
    from paper_2003_09926_amd import serve as S

    torch.cuda.set_device(0)
    prec = B.JZ_FP64 if prec_name == "fp64" else B.JZ_FP32_FLUX
    tile = None  # the library's default tiling for the precision
    stream = I.arrival_stream(seed=5, nruns=nruns, rate=20.0)
    runs = S.make_runs(stream)
    S.attach_payloads(runs)   # the clients' requests: payloads in host memory before the clock starts
    srv = S.JetServer(precision=prec, budget_bytes=200 << 30, max_resident=32, chunk_steps=20, tile=tile,
                      mode=mode)
    st = srv.serve(runs)
    summ = st.summary()
    out = {
        "metric": "point-stage updates/s", "value": summ["point_stage_updates_per_s"],
        "unit": "point-stage updates/s", "n_gpus": 1, "steps": 200, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == B.JZ_FP64 else "f32 (fluxes) + f64 (accumulation, J, norms)",
        "data": "synthetic",
        "config": {"workload": f"served_jet_runs_{prec_name}", "runs": nruns, "arrival_rate_per_s": 20.0,
                   "n_range": [48, 192], "steps_per_run": 200, "budget_gb": 200, "max_resident": 32,
                   "chunk_steps": 20, "seed": 5, "form": f"serve-{prec_name}", "mode": mode,
                   "admit_until_tiles_per_cu": srv.tiles_per_cu, "member_kchunk": srv.kchunk,
                   "payload": "host arrays built before the clock starts, uploaded at admission"},
        "serve": summ,
    }
    if with_sequential:
        out["alone_sequential"] = S.sequential_baseline(runs, prec, tile)
    return out


def run_split(prec_name: str, parts, steps: int, warmup: int):
    """The one-device domain split: the 512 x 256 x 256 stretched jet in
    parts[0] x parts[1] sub-blocks along xi and zeta with two ghost layers,
    halo copies after every stage; compared with the unsplit block (same
    steps, same box).  The rate counts the block's own nodes."""
    import torch
    from paper_2003_09926_amd import binding as B
    from paper_2003_09926_amd import inputs as I

    torch.cuda.set_device(0)
    prec = B.JZ_FP64 if prec_name == "fp64" else B.JZ_FP32_FLUX
    g, q = I.stretched_jet_case(DIMS, seed=2)
    P = B.params_default(re_d=1.0e6, precision=prec)
    d = B.Domain(g.dims, P, parts=parts)
    d.set_grid_metrics(g.metrics)
    d.set_state(q)
    d.advance(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.advance(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d.close()
    s = B.Solver(g.dims, P)
    s.set_grid_metrics(g.metrics)
    s.set_state(q)
    s.advance(warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.advance(steps)
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t1
    s.close()
    value = g.n * 5 * steps / el
    return {
        "metric": "point-stage updates/s", "value": value, "unit": "point-stage updates/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": el * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == B.JZ_FP64 else "f32 (fluxes) + f64 (accumulation, J, norms)",
        "data": "synthetic",
        "config": {"workload": f"jet_512x256x256_stretched_split_{parts[0]}x{parts[1]}_{prec_name}",
                   "parts_xi_zeta": list(parts), "ghost_layers": 2, "form": f"split-{prec_name}"},
        "unsplit": {"value": g.n * 5 * steps / el1, "ms_per_step": el1 * 1e3 / steps},
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="fp64",
                    choices=["fp64", "fp32", "domain-fp64", "domain-fp32", "cylinder-fp64", "cylinder-fp32",
                             "batch-fp64", "batch-fp32", "serve-fp64", "serve-fp32", "split-fp64", "split-fp32"],
                    help="fp64: FP64 path (default); fp32: FP32-flux form on the same workload; "
                         "domain-*: bounded jet domain with inflow and far-field faces; "
                         "cylinder-*: cylindrical jet mesh with the centreline; "
                         "batch-*: 64 uneven blocks in one persistent launch per stage; "
                         "serve-*: the served arrival stream; split-*: the block split into sub-blocks")
    ap.add_argument("--no-error", action="store_true", help="fp32 form: skip the error-vs-oracle run")
    ap.add_argument("--runs", type=int, default=100, help="serve forms: length of the arrival stream")
    ap.add_argument("--no-sequential", action="store_true", help="serve forms: skip the alone baseline")
    ap.add_argument("--serve-mode", default="batch", choices=["streams", "batch"],
                    help="serve forms: one batch over the resident runs, or each run on its own stream")
    ap.add_argument("--parts", default="2,2", help="split forms: parts along xi and zeta")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-secondary", action="store_true",
                    help="fp64 form: skip the FP32-flux form timed on the same workload")
    ap.add_argument("--stats-interval", type=int, default=0,
                    help="cylinder forms: accumulate time-averaged statistics every this many steps")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="instead of the workload, run 5 plain device copies of MIB MiB "
                         "(reference kernel for the HBM byte counters)")
    ap.add_argument("--hbm-rates", action="store_true",
                    help="instead of the workload, print the HBM rates of plain streaming kernels")
    a = ap.parse_args(argv)
    if a.hbm_rates:
        print(json.dumps({"hbm_rates_gbs": [hbm_rates(g << 30) for g in (1, 2, 4, 8)]}), flush=True)
        return
    if a.copy_calibrate:
        import torch
        n = a.copy_calibrate * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibrate_bytes_each_way": n * 8, "copies": 5}), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs one GPU per process and measures one GPU; "
                                   "--gpus above 1 is not supported"}), flush=True)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if a.form.startswith("batch"):
        out = run_batch(a.form.split("-")[1], a.steps, a.warmup)
    elif a.form.startswith("serve"):
        out = run_serve(a.form.split("-")[1], a.runs, not a.no_sequential, a.serve_mode)
    elif a.form.startswith("split"):
        out = run_split(a.form.split("-")[1], tuple(int(x) for x in a.parts.split(",")), a.steps, a.warmup)
    else:
        out = run_block(a.form, a.steps, a.warmup, with_cpu=(rank == 0 and not a.no_cpu),
                        with_error=not a.no_error, stats_interval=a.stats_interval,
                        with_secondary=not a.no_secondary)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
