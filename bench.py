#!/usr/bin/env python3
"""Throughput of the MI355X isoAdvector step (FP64 cell-steps/s) with a roofline line.

Default workload: the 3D graded 256x128x128 hexahedral box (4.19M cells) with a water column
plus a 3D wave, advected by a uniform stream plus a Taylor-Green vortex at Courant 0.5,
100 steps (synthetic inputs from wavegen, generated on the host, uploaded before timing).

Prints ONE JSON line.  Fields beyond the basic contract:
  roofline      dominant kernel: algorithmic bytes (or flops) per launch / mean launch time,
                measured with HIP events recorded around each kernel on the step's stream
                over a second pass of the same K steps (the throughput pass has no event
                between kernels: each event adds a dispatch gap); traffic from committed
                rocprofv3 counters when they belong to the current kernel source, else null
  cpu_baseline  the CPU oracle on a bounded sample of the same workload, on every host CPU the
                process may use (OpenMP over cells; the value) and on one thread, with the CPU model
  step_roofline the whole step's algorithmic bytes per cell-step x cell-steps/s / 8 TB/s
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 isoAdvector cell-steps/s + % HBM roofline; batched vs plain; adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
# sources of the kernels that the profiled commands launch (their meshes are hexahedra only, so the
# polyhedron kernel of big.hip is not among them)
KERNEL_SRCS = [os.path.join(ROOT, "paper_1804_01130_amd", "csrc", n) for n in ("kernels.hip", "device_common.h",
                                                                                "internal.h", "gfm.hip", "relax.hip")]
PROFILES = os.path.join(ROOT, "profiles")
# FP64 operations credited per interface cell for vertex interpolation, the isovalue search, the
# isoface and the swept-face integrals (a fixed per-unit figure, independent of the iteration
# counts of this implementation)
FLOP_PER_SURFACE_CELL = 11000.0
COPY_N = 1 << 27  # doubles moved by the calibration copy (1 GiB read, 1 GiB written)
KERNEL_KEYS = {"k_find_surface": "find_surface", "k_surface": "surface", "k_update": "update",
               "k_bound_sweep": "bound_sweep", "k_bound_end": "bound_end",
               "k_gfm_faces": "gfm_faces", "k_relax_blend": "relax_blend", "k_stats": "stats"}
# the commands whose rocprofv3 output --summarize-profiles reads: a window of 20 steps after 5
# warm-up steps, with only the step's own kernels (the summaries record the window's interface-cell
# count, so a line timed over another window compares at its own count)
_PROF_ARGS = ("--steps 20 --warmup 5 --no-cpu-baseline --no-ensemble --no-adjoint --no-variants --no-gfm "
              "--no-relax --no-poly")
# the traffic passes also take the ghost-fluid face data and the relaxation blend (after the steps)
_PROF_ARGS_TRAFFIC = "--steps 20 --warmup 5 --no-cpu-baseline --no-ensemble --no-adjoint --no-variants --no-poly"
PROFILE_COMMANDS = {
    "stats": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -T -f csv "
             "-d /root/repo/gpurun_out/prof_stats -o run -- python3 /root/repo/bench.py --workload {w} " + _PROF_ARGS +
             " > /root/repo/gpurun_out/prof_stats/bench.json",
    "fetch": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE -T -f csv "
             "-d /root/repo/gpurun_out/prof_fetch -o run -- python3 /root/repo/bench.py --workload {w} " + _PROF_ARGS_TRAFFIC +
             " --copy-calibration > /root/repo/gpurun_out/prof_fetch/bench.json",
    "write": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE -T -f csv "
             "-d /root/repo/gpurun_out/prof_write -o run -- python3 /root/repo/bench.py --workload {w} " + _PROF_ARGS_TRAFFIC +
             " --copy-calibration > /root/repo/gpurun_out/prof_write/bench.json",
    "sq": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS "
          "SQ_INSTS_VMEM_RD SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU -T -f csv -d /root/repo/gpurun_out/prof_sq "
          "-o run -- python3 /root/repo/bench.py --workload {w} " + _PROF_ARGS + " > /root/repo/gpurun_out/prof_sq/bench.json",
    # the batched ensemble alone (no plain comparison), whose timed run ends the process
    "ensemble": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -T -f csv "
                "-d /root/repo/gpurun_out/prof_ens -o run -- python3 /root/repo/bench.py --ensemble-only --steps 20 "
                "--warmup 3 > /root/repo/gpurun_out/prof_ens/bench.json",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name):
    import wavegen as W
    if name == "violent_3d":
        return W.violent_3d()
    if name == "airy_2d":
        return W.airy_1024x256()
    if name == "cosine_2d":
        return W.cosine_uniform()
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_path(workload):
    return os.path.join(PROFILES, f"hbm_traffic_{workload}.txt")


def read_kv(path):
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        out[k.strip()] = v.strip()
    return out


def committed_traffic(kernel, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary, if the counters
    were taken on the current kernel source (else None)."""
    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    d = read_kv(path)
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    v = d.get(f"{kernel}.bytes_per_launch")
    return float(v) if v is not None else None


def algorithmic(kernel, mesh_info, n_surface, n_flux, n_cells):
    """(quantity per launch, unit, bound) of each kernel's compulsory work: bytes that must cross
    HBM for the memory-bound kernels, FP64 operations of the method for the interface kernel."""
    if kernel == "update":
        # alpha, V read + alpha_new written (8 B each) per cell; per flux face phi (8 B) and the
        # owner/neighbour pair (2 x 4 B); dV of interface-upwind faces (8 B, <= 6 per interface cell)
        return (24.0 * n_cells + 16.0 * n_flux + 8.0 * 3 * n_surface), "GB/s", "hbm"
    if kernel == "find_surface":
        return (8.0 * n_cells + 4.0 * n_surface), "GB/s", "hbm"
    if kernel == "surface":
        return FLOP_PER_SURFACE_CELL * n_surface, "TFLOP/s", "alu"
    return None, None, "hbm"


def step_bytes_per_cell(n_cells, n_flux, n_surface):
    """Algorithmic bytes of one whole step per cell: alpha in/out, V, phi and connectivity per flux
    face, and ~1.1 KB per interface cell (vertex stencils, coordinates, velocity, face writes)."""
    return (24.0 * n_cells + 16.0 * n_flux + 1100.0 * n_surface) / n_cells


def host_cpu():
    """The host's logical CPU count, the CPUs this process may run on, and the CPU model."""
    model = "unknown"
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "usable": usable, "model": model}


def _oracle_rate(O, om, w, threads, budget_s):
    """Cell-steps/s of the oracle on `threads` threads over the first steps of the workload that fit
    in about budget_s seconds."""
    O.set_threads(threads)
    phi, U = w.phi_U(0)
    a = np.array(w.alpha0, copy=True)
    t0 = time.perf_counter()
    steps = 0
    while True:
        if not w.steady:
            phi, U = w.phi_U(steps)
        a, _ = om.step(a, phi, U, w.dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= w.n_steps or el / steps * (steps + 1) > 1.5 * budget_s:
            break
    return w.mesh.n_cells * steps / el, steps, el


def cpu_baseline(w, budget_s=20.0):
    """The oracle as it stands on bounded samples of the same workload: on every CPU this process
    may use (OpenMP over cells; the value reported) and on one thread."""
    from oracle import oracle as O
    O.build()
    om = O.OracleMesh(w.mesh)
    host = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", host["usable"]) or host["usable"])
    v1, s1, e1 = _oracle_rate(O, om, w, 1, 0.35 * budget_s)
    vn, sn, en = _oracle_rate(O, om, w, threads, 0.65 * budget_s)
    return {"value": vn, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sn} of {w.n_steps} steps of the same workload on {threads} threads, {en:.1f} s",
            "single_thread": {"value": v1, "unit": "cell-steps/s", "cores": 1,
                              "sample": f"first {s1} of {w.n_steps} steps, {e1:.1f} s"},
            "host": host}


def copy_calibration(dev):
    """A plain streaming copy kernel (elementwise multiply by one) of COPY_N doubles, three times."""
    import torch
    src = torch.ones(COPY_N, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {COPY_N * 8} bytes read and written per launch, 3 launches")


def _find(dirname, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(ROOT, dirname, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {dirname}")
    return hits[-1]


def _kernel_key(name):
    for k, v in KERNEL_KEYS.items():
        if k in name:
            return v
    if "elementwise" in name or "Mul" in name or "mul" in name:
        return "copy"
    return None


def _pmc_per_dispatch(path, counter):
    import csv
    vals = {}
    for row in csv.DictReader(open(path)):
        if row.get("Counter_Name") != counter:
            continue
        key = _kernel_key(row.get("Kernel_Name", ""))
        if key is None:
            continue
        vals.setdefault(key, []).append(float(row["Counter_Value"]))
    return vals


def summarize_ensemble_profile():
    """profiles/kernel_stats_airy_ensemble_64.txt from the rocprofv3 kernel trace of the ensemble
    command: the step kernels of the timed batched run (the last K steps of the process)."""
    import csv
    run = json.loads(open(os.path.join(ROOT, "gpurun_out/prof_ens/bench.json")).read())
    steps, ens = int(run["steps"]), run["ensemble"]
    trace = sorted(csv.DictReader(open(_find("gpurun_out/prof_ens", "kernel_trace.csv"))),
                   key=lambda r: int(r["Start_Timestamp"]))
    keys = [("surface_big" if "k_surface_big" in r["Kernel_Name"] else _kernel_key(r["Kernel_Name"]), r)
            for r in trace]
    finds = [int(r["Start_Timestamp"]) for k, r in keys if k == "find_surface"]
    if len(finds) < steps:
        raise SystemExit("fewer find_surface dispatches than timed steps in the ensemble trace")
    t0 = finds[-steps]
    by = {}
    for k, r in keys:
        if k in ("find_surface", "surface", "surface_big", "update", "bound_sweep", "bound_end") and \
                int(r["Start_Timestamp"]) >= t0:
            by.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    lines = [f"# rocprofv3 kernel trace, workload {ens['workload']}: the timed batched run",
             f"# command (repository root): {PROFILE_COMMANDS['ensemble']}",
             f"# kernel_source_sha: {run['kernel_source_sha']}",
             f"# window: the last {steps} steps (the graph replay the benchmark times, after {run['warmup']} warm-up "
             f"steps and the capture run); {ens['interface_cells']} interface cells at its start; launch shapes "
             f"{ens['tuned_config']}",
             "# kernel | dispatches | per step | mean us | min us | max us"]
    tot = 0.0
    for k in ("find_surface", "surface", "surface_big", "update", "bound_sweep", "bound_end"):
        if k not in by:
            continue
        d = by[k]
        tot += sum(d) / steps
        lines.append(f"k_{k} | {len(d)} | {len(d) / steps:g} | {np.mean(d):.2f} | {min(d):.2f} | {max(d):.2f}")
    lines.append(f"# kernels per step {tot:.1f} us; the run's events gave {ens['batched_ms_per_step'] * 1e3:.1f} us/step "
                 f"({ens['batched_cell_steps_per_s']:.3e} cell-steps/s, {ens['hbm_frac']:.4f} of the HBM roofline at "
                 f"{ens['bytes_per_cell_step']:.1f} B/cell-step)")
    lines.append("# whole process (rocprofv3 --stats): name | calls | total ms | average us | min us | max us | share %")
    for r in csv.DictReader(open(_find("gpurun_out/prof_ens", "kernel_stats.csv"))):
        lines.append(f"{r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}")
    open(os.path.join(PROFILES, "kernel_stats_airy_ensemble_64.txt"), "w").write("\n".join(lines) + "\n")


def summarize_profiles(workload):
    """profiles/kernel_stats_<workload>.txt and profiles/hbm_traffic_<workload>.txt from the
    rocprofv3 output of PROFILE_COMMANDS (kernel trace; FETCH_SIZE and WRITE_SIZE counter passes,
    each scaled by what the counter reads for the calibration copy of known size)."""
    import csv
    os.makedirs(PROFILES, exist_ok=True)
    cmds = {k: v.format(w=workload) for k, v in PROFILE_COMMANDS.items()}
    run = json.loads(open(os.path.join(ROOT, "gpurun_out/prof_stats/bench.json")).read())
    steps, warmup = int(run["steps"]), int(run["warmup"])
    n_s = float(run["config"]["interface_cells"])
    # every kernel of the step in launch order: warm-up steps, one step with statistics, the timed
    # steps, the pass with an event around each kernel group (whose means the benchmark reports),
    # and a pass with statistics
    passes = warmup + 1 + 3 * steps
    trace = list(csv.DictReader(open(_find("gpurun_out/prof_stats", "kernel_trace.csv"))))
    by = {}
    for r in sorted(trace, key=lambda r: int(r["Start_Timestamp"])):
        k = _kernel_key(r["Kernel_Name"])
        if k in ("find_surface", "surface", "update", "bound_sweep", "bound_end"):
            by.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    lines = [f"# rocprofv3 kernel trace, workload {workload}: the window the benchmark line times",
             f"# command (repository root): {cmds['stats']}",
             f"# kernel_source_sha: {run['kernel_source_sha']}",
             f"# window: the {steps} steps after {warmup} warm-up steps, in the pass with an event around each "
             f"kernel group; interface cells per step {n_s:.0f} on average "
             f"({run['config']['interface_cells_range'][0]}-{run['config']['interface_cells_range'][1]})",
             "# kernel | dispatches in the window | mean us | min us | max us"]
    means = {}
    for k, d in by.items():
        per = len(d) // passes
        if per * passes != len(d):
            raise SystemExit(f"{k}: {len(d)} dispatches do not split into {passes} steps")
        win = d[(warmup + 1 + steps) * per:(warmup + 1 + 2 * steps) * per]
        means[k] = float(np.mean(win))
        lines.append(f"k_{k} | {len(win)} | {means[k]:.2f} | {min(win):.2f} | {max(win):.2f}")
    if "surface" in means:
        tf = FLOP_PER_SURFACE_CELL * n_s / (means["surface"] * 1e-6) / 1e12
        lines.append(f"# k_surface: {FLOP_PER_SURFACE_CELL:.0f} flop x {n_s:.0f} interface cells / {means['surface']:.2f} us"
                     f" = {tf:.3f} TFLOP/s = {tf / FP64_VECTOR_TFLOPS:.4f} of the {FP64_VECTOR_TFLOPS} TFLOP/s FP64 peak"
                     f" (the line reported {run['roofline']['frac']:.4f} from its own events)")
    lines.append("# whole run (rocprofv3 --stats): name | calls | total ms | average us | min us | max us | share %")
    for r in csv.DictReader(open(_find("gpurun_out/prof_stats", "kernel_stats.csv"))):
        lines.append(f"{r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}")
    open(os.path.join(PROFILES, f"kernel_stats_{workload}.txt"), "w").write("\n".join(lines) + "\n")

    fetch = _pmc_per_dispatch(_find("gpurun_out/prof_fetch", "counter_collection.csv"), "FETCH_SIZE")
    write = _pmc_per_dispatch(_find("gpurun_out/prof_write", "counter_collection.csv"), "WRITE_SIZE")
    shas = set()
    for d in ("gpurun_out/prof_fetch", "gpurun_out/prof_write"):
        out = json.loads(open(os.path.join(ROOT, d, "bench.json")).read())
        shas.add(out["kernel_source_sha"])
    if len(shas) != 1:
        raise SystemExit(f"counter passes ran on different kernel sources: {shas}")
    copy_bytes = COPY_N * 8.0
    # the copy dispatches are the largest elementwise launches of the run
    cf = max(fetch.get("copy", [0.0])) * 1024.0
    cw = max(write.get("copy", [0.0])) * 1024.0
    if cf <= 0 or cw <= 0:
        raise SystemExit("calibration copy not found in the counter output")
    sf, sw = copy_bytes / cf, copy_bytes / cw
    lines = [f"# HBM traffic per launch from rocprofv3 counters, workload {workload}",
             f"# FETCH_SIZE pass: {cmds['fetch']}",
             f"# WRITE_SIZE pass: {cmds['write']}",
             f"# calibration: elementwise copy of {COPY_N} doubles ({copy_bytes:.0f} B read, {copy_bytes:.0f} B "
             f"written); counters read {cf:.0f} B fetched and {cw:.0f} B written.  The scales are these ratios, "
             f"measured in the same run: FETCH_SIZE reports half of what the copy reads (consistent with the "
             f"derived counter taking each read request as 64 B where this GPU moves 128 B per request; "
             f"the ratio, not that reading, is what scales the kernels' counts)",
             "# <kernel>.fetch_kib / .write_kib: mean counter value per dispatch (KiB);"
             " bytes_per_launch = fetch x scale_fetch + write x scale_write",
             f"kernel_source_sha: {shas.pop()}",
             f"scale_fetch: {sf:.6f}",
             f"scale_write: {sw:.6f}"]
    for k in ("find_surface", "surface", "update", "bound_sweep", "bound_end", "gfm_faces", "relax_blend"):
        if k not in fetch or k not in write:
            continue
        fk = float(np.mean(fetch[k]))
        wk = float(np.mean(write[k]))
        lines += [f"{k}.dispatches: {len(fetch[k])}", f"{k}.fetch_kib: {fk:.1f}", f"{k}.write_kib: {wk:.1f}",
                  f"{k}.bytes_per_launch: {fk * 1024.0 * sf + wk * 1024.0 * sw:.0f}"]
    open(traffic_path(workload), "w").write("\n".join(lines) + "\n")

    # instruction mix per wave from the SQ counter pass (when it was taken)
    sq_dir = os.path.join(ROOT, "gpurun_out/prof_sq")
    if os.path.isdir(sq_dir):
        sq_sha = json.loads(open(os.path.join(sq_dir, "bench.json")).read())["kernel_source_sha"]
        per = {}
        for r in csv.DictReader(open(_find("gpurun_out/prof_sq", "counter_collection.csv"))):
            k = _kernel_key(r["Kernel_Name"])
            if k is not None:
                did = r.get("Dispatch_Id", r.get("Correlation_Id"))
                d = per.setdefault(k, {}).setdefault(r["Counter_Name"], {})
                d[did] = d.get(did, 0.0) + float(r["Counter_Value"])
        lines = [f"# SQ instruction counters per dispatch (mean over dispatches), workload {workload}",
                 f"# command (repository root): {cmds['sq']}",
                 f"# kernel_source_sha: {sq_sha}",
                 "# per-wave figures divide by SQ_WAVES; SQ_BUSY_CYCLES is summed over the shader engines",
                 "# kernel | dispatches | waves | VALU/wave | SALU/wave | VMEM_RD/wave | LDS/wave | WAVE_CYCLES/wave | "
                 "VALU instructions"]
        for k in ("surface", "update", "find_surface", "bound_sweep", "bound_end", "gfm_faces", "relax_blend"):
            if k not in per:
                continue
            mean = {n: sum(v.values()) / max(len(v), 1) for n, v in per[k].items()}
            nd = len(per[k]["SQ_WAVES"])
            wv = mean["SQ_WAVES"]
            lines.append(f"k_{k} | {nd} | {wv:.0f} | {mean['SQ_INSTS_VALU'] / wv:.0f} | {mean['SQ_INSTS_SALU'] / wv:.0f} | "
                         f"{mean['SQ_INSTS_VMEM_RD'] / wv:.1f} | {mean['SQ_INSTS_LDS'] / wv:.1f} | "
                         f"{mean['SQ_WAVE_CYCLES'] / wv:.0f} | {mean['SQ_INSTS_VALU']:.4g}")
        open(os.path.join(PROFILES, f"sq_counters_{workload}.txt"), "w").write("\n".join(lines) + "\n")
    log(f"[bench] wrote profiles for {workload}")


def ensemble_bench(steps, warmup, tune_cache=None, plain=True):
    """64 Airy domains of uneven sizes: the batched path (one launch per kernel over all members,
    autotuned launch shapes, a captured graph of the whole run) against the plain path (each
    member's own plan, step by step), on the same per-step fields resident in HBM."""
    import torch
    import wavegen as W
    from wavegen.device import EnsembleAiryFields
    from paper_1804_01130_amd import Batch, Mesh, Plan, default_options
    dev = torch.device("cuda:0")
    t0 = time.time()
    ws = W.airy_ensemble(64, seed=1, steps=steps)
    meshes = [Mesh.from_arrays(w.mesh) for w in ws]
    batch = Batch(meshes, default_options())
    N, F = batch.n_cells, batch.n_faces
    co, fo = batch.layout()
    S = warmup + steps
    ef = EnsembleAiryFields(ws, dev)
    phi_all = torch.empty((S, F), dtype=torch.float64, device=dev)
    U_all = torch.empty((S, 3 * N), dtype=torch.float64, device=dev)
    for n in range(S):
        ef.fields(n, phi_all[n], U_all[n])
    dts = np.array([w.dt for w in ws])
    alpha0 = torch.tensor(batch.concat_cells([w.alpha0 for w in ws]), device=dev)
    log(f"[bench] ensemble: {len(ws)} members, {N} cells, {F} faces, fields for {S} steps, set up in "
        f"{time.time() - t0:.1f} s")
    cfg, tune_ms = batch.tune(alpha0, phi_all[0], U_all[0], dts, n_trial=3, cache_path=tune_cache)
    # warm-up steps, then the timed run from the state they reach
    a = alpha0.clone()
    batch.advect(a, phi_all, U_all, dts, warmup, F, 3 * N)
    start = a.clone()
    phi_t, U_t = phi_all[warmup:], U_all[warmup:]
    batch.advect(a, phi_t, U_t, dts, steps, F, 3 * N)  # captures the run's graph
    a.copy_(start)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.advect(a, phi_t, U_t, dts, steps, F, 3 * N)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    n_s = int(((start > 1e-8) & (start < 1.0 - 1e-8)).sum().item())
    batched = a.cpu().numpy()
    nflux = sum(m.info()["n_flux_faces"] for m in meshes)
    b_alg = (24.0 * N + 16.0 * nflux + 1100.0 * n_s) / N
    vb = N * steps / (ms_b * 1e-3)
    if not plain:  # the batched run alone (its kernels are then the last ones of the process)
        out = {"workload": f"airy_ensemble_64 ({len(ws)} members, {N} cells)", "steps": steps, "cells": N,
               "interface_cells": n_s, "batched_cell_steps_per_s": vb, "batched_ms_per_step": ms_b / steps,
               "tuned_config": cfg, "hbm_frac": b_alg * vb / (HBM_PEAK_GBS * 1e9), "bytes_per_cell_step": b_alg}
        log(f"[bench] ensemble: batched {ms_b / steps * 1e3:.1f} us/step, config {cfg}")
        batch.close()
        return out
    # plain: every member through its own plan, step by step
    plans = [Plan(m, default_options()) for m in meshes]
    st = [start[co[d]:co[d + 1]].clone() for d in range(len(ws))]
    tmp = [torch.empty_like(x) for x in st]
    Um = []
    for d in range(len(ws)):
        nd = int(co[d + 1] - co[d])
        u = torch.empty((steps, 3 * nd), dtype=torch.float64, device=dev)
        for k in range(3):
            u[:, k * nd:(k + 1) * nd] = U_t[:, k * N + co[d]:k * N + co[d + 1]]
        Um.append(u)
    phis = [[phi_t[n, fo[d]:fo[d + 1]] for d in range(len(ws))] for n in range(steps)]
    for d, p in enumerate(plans):  # one untimed step each
        p.step(st[d], phis[0][d], Um[d][0], dts[d], out=tmp[d])
    for d in range(len(ws)):
        st[d].copy_(start[co[d]:co[d + 1]])
    torch.cuda.synchronize()
    e0.record()
    for n in range(steps):
        for d, p in enumerate(plans):
            p.step(st[d], phis[n][d], Um[d][n], dts[d], out=tmp[d])
            st[d], tmp[d] = tmp[d], st[d]
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    plain = torch.cat(st).cpu().numpy()
    out = {"workload": f"airy_ensemble_64 ({len(ws)} members, {N} cells)", "steps": steps, "cells": N,
           "interface_cells": n_s, "batched_cell_steps_per_s": vb,
           "plain_cell_steps_per_s": N * steps / (ms_p * 1e-3), "speedup": ms_p / ms_b,
           "batched_ms_per_step": ms_b / steps, "plain_ms_per_step": ms_p / steps,
           "bitwise_equal": bool(np.array_equal(batched, plain)), "tuned_config": cfg,
           "hbm_frac": b_alg * vb / (HBM_PEAK_GBS * 1e9), "bytes_per_cell_step": b_alg}
    log(f"[bench] ensemble: batched {ms_b / steps * 1e3:.1f} us/step, plain {ms_p / steps * 1e3:.1f} us/step, "
        f"speed-up {ms_p / ms_b:.1f}, bitwise equal {out['bitwise_equal']}, config {cfg}")
    for p in plans:
        p.close()
    batch.close()
    del phi_all, U_all, Um, phis, phi_t, U_t
    torch.cuda.empty_cache()
    return out


def variants_bench(gm, w, phis, Us, sel, a_start, args):
    """The same K steps from the same state with the step's variants: the isoface velocity by
    cell-point interpolation (us_mode 1), and the averaged fields of an outer iteration (the
    fields of the step and of the next one, averaged as the kernels read them)."""
    import torch
    from paper_1804_01130_amd import Plan, default_options
    out = {}
    for name, us_mode, avg in (("us_mode_1", 1, False), ("averaged_fields", 0, True)):
        plan = Plan(gm, default_options(us_mode=us_mode))
        a = a_start.clone()
        b = torch.empty_like(a)
        nxt = (lambda n: 0) if w.steady else (lambda n: min(n + 1, len(phis) - 1))
        kw = lambda n: dict(phi1=phis[nxt(n)], U1=Us[nxt(n)]) if avg else {}
        for n in range(args.warmup):  # warm-up from the same state, then restart
            plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b, **kw(n))
            a, b = b, a
        a.copy_(a_start)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for n in range(args.warmup, args.warmup + args.steps):
            plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b, **kw(n))
            a, b = b, a
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out[name] = {"ms_per_step": ms, "cell_steps_per_s": w.mesh.n_cells / (ms * 1e-3)}
        log(f"[bench] variant {name}: {ms * 1e3:.1f} us/step")
        plan.close()
        del a, b
    return out


# vertical axis and still-water level of each workload (inputs of the ghost-fluid face data)
GRAVITY = {"violent_3d": ((0.0, 0.0, -9.81), (0.0, 0.0, 0.5)), "airy_2d": ((0.0, -9.81, 0.0), (0.0, 0.5, 0.0)),
           "cosine_2d": ((0.0, -9.81, 0.0), (0.0, 0.5, 0.0))}
RHO_HEAVY, RHO_LIGHT = 1000.0, 1.2


def gfm_bench(gm, plan, workload, a, reps=20):
    """Ghost-fluid face data (iso_gfm_faces, Eqs. 12-20) from the state the timed steps reached, with
    a synthetic dynamic pressure: time per call and its HBM roofline.  Algorithmic bytes per call:
    per face the owner/neighbour pair (8 B) and the five outputs (40 B); per cell alpha and p_d read
    once (16 B); per interface face the two cell centroids (48 B)."""
    import torch
    import wavegen as W
    g, level = GRAVITY[workload]
    xc = gm.geometry()[1]
    a_host = a.cpu().numpy()
    p = torch.tensor(W.dynamic_pressure(xc, a_host, RHO_HEAVY, RHO_LIGHT, g, level, seed=7), device=a.device)
    out = plan.gfm_faces(a, p, RHO_HEAVY, RHO_LIGHT, g)
    for _ in range(3):
        plan.gfm_faces(a, p, RHO_HEAVY, RHO_LIGHT, g, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.gfm_faces(a, p, RHO_HEAVY, RHO_LIGHT, g, out=out)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    n_if = int((out["lambda"] >= 0).sum().item())
    nf, nc = gm.n_faces, gm.n_cells
    q = 48.0 * nf + 16.0 * nc + 48.0 * n_if
    achieved = q / (us * 1e-6) / 1e9
    log(f"[bench] ghost-fluid face data: {us:.1f} us per call, {n_if} interface faces, {achieved:.0f} GB/s")
    return {"us_per_call": us, "faces": nf, "interface_faces": n_if, "algorithmic_bytes_per_launch": q,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic("gfm_faces", workload), "rho": [RHO_HEAVY, RHO_LIGHT], "g": list(g)}


# relaxation zones at both ends of each workload's periodic direction (inner edge, outward direction,
# length), about 15 % of the domain each
RELAX_ZONES = {
    "violent_3d": [((0.3003, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.3), ((1.6997, 0.0, 0.0), (1.0, 0.0, 0.0), 0.3)],
    "airy_2d": [((0.6003, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.6), ((3.3997, 0.0, 0.0), (1.0, 0.0, 0.0), 0.6)],
    "cosine_2d": [((0.3003, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.3), ((1.6997, 0.0, 0.0), (1.0, 0.0, 0.0), 0.3)],
}


def relax_bench(plan, workload, a, target, reps=50):
    """Relaxation-zone blending (iso_relax_blend) of the state the timed steps reached towards the
    initial field: time per call and its HBM roofline.  Algorithmic bytes per call: 36 B per zone
    cell (index 4, weight 8, alpha read and written 16, target 8)."""
    import torch
    n = plan.set_relaxation(RELAX_ZONES[workload])
    x = a.clone()
    for _ in range(3):
        plan.relax_blend(x, target)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.relax_blend(x, target)
    e1.record()
    torch.cuda.synchronize()
    plan.set_relaxation([])
    us = e0.elapsed_time(e1) / reps * 1e3
    q = 36.0 * n
    achieved = q / (us * 1e-6) / 1e9
    log(f"[bench] relaxation blend: {us:.1f} us per call, {n} zone cells, {achieved:.0f} GB/s")
    return {"us_per_call": us, "zone_cells": n, "algorithmic_bytes_per_launch": q, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic("relax_blend", workload)}


def poly_bench(steps, warmup):
    """The step on cells other than hexahedra: the violent 3D case's ingredients on 48x24x24
    hexahedra each cut into six tetrahedra (165,888 cells, steady flow), on 64x32x32 cut into
    prisms, and on 64x32x32 hexahedra mostly merged into polyhedra of 10 and 16 faces (26,112
    cells, the polyhedron kernel), also with the faces two polyhedra share joined into polygons of 6
    and 8 points (the kernel's general face loops); K steps from the sampled initial field, timed
    like the main line."""
    import torch
    import wavegen as W
    from paper_1804_01130_amd import Mesh, Plan, default_options
    out = {}
    for kind, n in (("tet", (48, 24, 24)), ("prism", (64, 32, 32)), ("merged", (64, 32, 32)),
                    ("merged_joined", (64, 32, 32))):
        t0 = time.time()
        w = W.poly_violent(kind, nx=n[0], ny=n[1], nz=n[2], steps=steps)
        gm = Mesh.from_arrays(w.mesh)
        plan = Plan(gm, default_options())
        phi, U = (torch.tensor(v, device="cuda:0") for v in w.phi_U(0))
        a = torch.tensor(w.alpha0, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(warmup):
            plan.step(a, phi, U, w.dt, out=b)
            a, b = b, a
        _, st = plan.step(a, phi, U, w.dt, out=b, stats=True)
        a, b = b, a
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.step(a, phi, U, w.dt, out=b)
            a, b = b, a
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[kind] = {"workload": w.name, "cells": w.mesh.n_cells, "interface_cells": st["n_surface"],
                     "ms_per_step": ms, "cell_steps_per_s": w.mesh.n_cells / (ms * 1e-3),
                     "interface_cells_per_s": st["n_surface"] / (ms * 1e-3)}
        log(f"[bench] {w.name}: {w.mesh.n_cells} cells, {st['n_surface']} interface cells, {ms * 1e3:.1f} us/step "
            f"(set up in {time.time() - t0:.1f} s)")
        plan.close()
        gm.close()
    return out


def adjoint_bench(every=10):
    """The adjoint workload: 256x128 Airy, 50 steps, loss sum (alpha_T - alpha_target)^2; time of the
    forward pass (plain steps) and of the backward pass (recomputing each segment from its checkpoint
    with traced steps, then the adjoint steps), both through the same torch autograd Function."""
    import torch
    import wavegen as W
    from paper_1804_01130_amd import Mesh, Plan, default_options
    from paper_1804_01130_amd.autograd import advect
    dev = torch.device("cuda:0")
    base, target = W.adjoint_case()
    S = base.n_steps
    T = lambda x: torch.tensor(x, device=dev)
    phis = torch.stack([T(base.phi_U(n)[0]) for n in range(S)]).contiguous()
    Us = torch.stack([T(base.phi_U(n)[1]) for n in range(S)]).contiguous()
    plan = Plan(Mesh.from_arrays(base.mesh), default_options())
    tplan = Plan(Mesh.from_arrays(target.mesh), default_options())
    at = T(target.alpha0)
    tb = torch.empty_like(at)
    for n in range(S):
        tplan.step(at, T(target.phi_U(n)[0]), T(target.phi_U(n)[1]), target.dt, out=tb)
        at, tb = tb, at
    a0 = T(base.alpha0)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    best = None
    for rep in range(4):  # the first repetition warms up (adjoint workspace, allocator)
        x0 = a0.clone().requires_grad_(True)
        ph = phis.clone().requires_grad_(True)
        torch.cuda.synchronize()
        e0.record()
        aT = advect(x0, ph, plan, Us, base.dt, checkpoint_every=every)
        L = ((aT - at) ** 2).sum()
        e1.record()
        L.backward()
        e2.record()
        torch.cuda.synchronize()
        f, b = e0.elapsed_time(e1), e1.elapsed_time(e2)
        if rep > 0 and (best is None or f + b < best[0] + best[1]):
            best = (f, b, L.item())
    f, b, Lv = best
    out = {"workload": "airy_2d_256x128 (32768 cells), 50 steps, loss sum (alpha_T - alpha_target)^2",
           "checkpoint_every": every, "forward_ms": f, "backward_ms": b, "adjoint_fwd_ratio": b / f,
           "loss": Lv, "note": "backward = recomputation of each segment from its checkpoint + adjoint steps"}
    log(f"[bench] adjoint: forward {f:.2f} ms, backward {b:.2f} ms, ratio {b / f:.2f}")
    out["violent_3d"] = adjoint_bench_3d(every)
    return out


def adjoint_bench_3d(every=10, steps=20):
    """The adjoint on a bounding-heavy 3D state: the graded violent box at 128x64x64 (524k cells), 20
    steps from its initial field, loss sum alpha_T^2; forward and backward as above, and the cells
    the redistribution lists per step."""
    import torch
    import wavegen as W
    from paper_1804_01130_amd import Mesh, Plan, default_options
    from paper_1804_01130_amd.autograd import advect
    dev = torch.device("cuda:0")
    w = W.violent_3d(nx=128, ny=64, nz=64, steps=steps)
    plan = Plan(Mesh.from_arrays(w.mesh), default_options())
    phi, U = w.phi_U(0)
    phis = torch.tensor(phi, device=dev)[None, :].expand(steps, -1).contiguous()
    Us = torch.tensor(U, device=dev)[None, :].expand(steps, -1).contiguous()
    a0 = torch.tensor(w.alpha0, device=dev)
    a, b = a0.clone(), torch.empty_like(a0)
    active = []
    for n in range(steps):
        _, st = plan.step(a, phis[n], Us[n], w.dt, out=b, stats=True)
        active.append(st["n_bound_active"])
        a, b = b, a
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    best = None
    for rep in range(3):
        x0 = a0.clone().requires_grad_(True)
        ph = phis.clone().requires_grad_(True)
        torch.cuda.synchronize()
        e0.record()
        aT = advect(x0, ph, plan, Us, w.dt, checkpoint_every=every)
        L = (aT ** 2).sum()
        e1.record()
        L.backward()
        e2.record()
        torch.cuda.synchronize()
        f, bk = e0.elapsed_time(e1), e1.elapsed_time(e2)
        if rep > 0 and (best is None or f + bk < best[0] + best[1]):
            best = (f, bk)
    f, bk = best
    log(f"[bench] adjoint 3D: forward {f:.2f} ms, backward {bk:.2f} ms, ratio {bk / f:.2f}, "
        f"cells listed for redistribution per step {np.mean(active):.0f}")
    plan.close()
    return {"workload": f"{w.name} ({w.mesh.n_cells} cells), {steps} steps, loss sum alpha_T^2",
            "checkpoint_every": every, "forward_ms": f, "backward_ms": bk, "adjoint_fwd_ratio": bk / f,
            "bound_active_per_step": float(np.mean(active))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="violent_3d", choices=["violent_3d", "airy_2d", "cosine_2d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--surface-waves", type=int, default=0, help="register budget of the interface kernel (1-4)")
    ap.add_argument("--surface-blocks", type=int, default=0, help="work-groups of the interface kernel (0: default)")
    ap.add_argument("--bound-blocks", type=int, default=0, help="work-groups of the bounding sweeps (0: default)")
    ap.add_argument("--block-cells", type=int, default=0, help="threads per block of the per-cell kernels (0: default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a plain copy kernel of known size (scale of the HBM counters)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-vs-plain ensemble measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the interpolated isoface velocity and averaged-field step timings")
    ap.add_argument("--no-gfm", action="store_true", help="skip the ghost-fluid face data timing")
    ap.add_argument("--no-relax", action="store_true", help="skip the relaxation-zone blending timing")
    ap.add_argument("--no-poly", action="store_true", help="skip the tetrahedral and prismatic meshes")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="time only the batched ensemble run (no plain comparison), for its kernel profile")
    ap.add_argument("--summarize-profiles", action="store_true",
                    help="write the profiles/ summaries from the rocprofv3 output of PROFILE_COMMANDS")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.workload)
        if os.path.isdir(os.path.join(ROOT, "gpurun_out/prof_ens")):
            summarize_ensemble_profile()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the step has no multi-GPU path in this "
              f"build", file=sys.stderr)
        sys.exit(2)
    if args.ensemble_only:
        ens = ensemble_bench(args.steps, args.warmup, plain=False)
        print(json.dumps({"ensemble": ens, "steps": args.steps, "warmup": args.warmup,
                          "kernel_source_sha": kernel_source_sha()}), flush=True)
        return

    import torch
    from paper_1804_01130_amd import Mesh, Plan

    t0 = time.time()
    w = build_workload(args.workload)
    log(f"[bench] workload {w.name}: {w.mesh.n_cells} cells, generated in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    gm = Mesh.from_arrays(w.mesh)
    info = gm.info()
    from paper_1804_01130_amd import default_options
    plan = Plan(gm, default_options(surface_waves=args.surface_waves, surface_blocks=args.surface_blocks,
                                    bound_blocks=args.bound_blocks, block_cells=args.block_cells))
    n_steps_total = args.warmup + args.steps
    if w.steady:
        phi, U = w.phi_U(0)
        phis = [torch.tensor(phi, device=dev)]
        Us = [torch.tensor(U, device=dev)]
    else:
        phis, Us = [], []
        for n in range(n_steps_total):
            phi, U = w.phi_U(n)
            phis.append(torch.tensor(phi, device=dev))
            Us.append(torch.tensor(U, device=dev))
    a = torch.tensor(w.alpha0, device=dev)
    b = torch.empty_like(a)
    sel = (lambda n: 0) if w.steady else (lambda n: n)
    for n in range(args.warmup):
        plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b)
        a, b = b, a
    _, st = plan.step(a, phis[sel(args.warmup)], Us[sel(args.warmup)], w.dt, out=b, stats=True)
    n_surface = st["n_surface"]
    a_start = a.clone()
    torch.cuda.synchronize()
    # throughput: the K steps back to back, with no event between the kernels of a step
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for n in range(args.warmup, n_steps_total):
        plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b)
        a, b = b, a
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # per-kernel durations: the same K steps again from the same state, with HIP events on the
    # plan's stream around each kernel group (each event adds a dispatch gap, hence the second pass)
    a.copy_(a_start)
    plan.set_timing(args.steps)
    for n in range(args.warmup, n_steps_total):
        plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    kms, nrec = plan.timing()
    # the interface cells of each step of the window: a third pass with statistics (untimed)
    a.copy_(a_start)
    ns = []
    for n in range(args.warmup, n_steps_total):
        _, stw = plan.step(a, phis[sel(n)], Us[sel(n)], w.dt, out=b, stats=True)
        ns.append(stw["n_surface"])
        a, b = b, a
    n_surface = float(np.mean(ns))  # interface cells per step over the timed window
    variants = None if args.no_variants else variants_bench(gm, w, phis, Us, sel, a_start, args)
    gfm = None if args.no_gfm else gfm_bench(gm, plan, args.workload, a)
    relax = None if args.no_relax else relax_bench(plan, args.workload, a, torch.tensor(w.alpha0, device=dev))
    del a_start
    ms_per_step = ms / args.steps
    cells = w.mesh.n_cells
    value = cells * args.steps / (ms * 1e-3)
    log(f"[bench] {args.steps} steps in {ms:.3f} ms ({ms_per_step * 1e3:.1f} us/step); kernels (ms total): "
        + ", ".join(f"{k} {v:.3f}" for k, v in kms.items()))

    # dominant kernel and its roofline
    dom = max(kms, key=kms.get)
    mean_s = kms[dom] / max(nrec, 1) * 1e-3
    n_flux = info["n_flux_faces"]
    q, unit, bound = algorithmic(dom, info, n_surface, n_flux, cells)
    if bound == "hbm" and q is not None:
        achieved = q / mean_s / 1e9
        peak = HBM_PEAK_GBS
        traffic = committed_traffic(dom, args.workload)
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s",
                "frac": achieved / peak, "traffic": traffic, "mean_launch_us": mean_s * 1e6,
                "algorithmic_bytes_per_launch": q}
    elif bound == "alu" and q is not None:
        achieved = q / mean_s / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_TFLOPS, "traffic": committed_traffic(dom, args.workload),
                "mean_launch_us": mean_s * 1e6, "algorithmic_flop_per_launch": q}
    else:
        roof = {"kernel": dom, "bound": bound, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "mean_launch_us": mean_s * 1e6}
    b_alg = step_bytes_per_cell(cells, n_flux, n_surface)
    step_frac = b_alg * value / (HBM_PEAK_GBS * 1e9)

    if args.copy_calibration:
        copy_calibration(dev)

    ens = None
    if not args.no_ensemble:
        del phis, Us, a, b, plan, gm
        torch.cuda.empty_cache()
        ens = ensemble_bench(args.steps, args.warmup)
    adj = None if args.no_adjoint else adjoint_bench()
    poly = None if args.no_poly else poly_bench(min(args.steps, 50), args.warmup)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample of the same workload")
        cpu = cpu_baseline(w, args.cpu_budget)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "cells": cells, "flux_faces": n_flux, "interface_cells": n_surface,
                   "interface_cells_range": [int(min(ns)), int(max(ns))],
                   "courant": 0.5 if args.workload != "cosine_2d" else 0.25, "dt": w.dt},
        "roofline": roof,
        "step_roofline": {"bytes_per_cell_step": b_alg, "achieved_GBs": b_alg * value / 1e9,
                          "frac": step_frac},
        "kernel_ms_per_step": {k: v / max(nrec, 1) for k, v in kms.items()},
        "kernel_source_sha": kernel_source_sha(),
        "cpu_baseline": cpu,
        "variants": variants,
        "gfm_faces": gfm,
        "relax_blend": relax,
        "ensemble": ens,
        "adjoint": adj,
        "cells_other_than_hexahedra": poly,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
