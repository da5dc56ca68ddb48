#!/usr/bin/env python
"""Throughput benchmark of the GW+C core-level path on one MI355X.

One step = one core-state solve of the benzene-sized workload (N_basis = 300,
N_occ = 21 with 6 C1s levels, N_aux = 1200, 32 imaginary and 400 real
frequencies per core, eta = 0.1 eV): gwc_sigma_core in FULL mode for one core
state (Pi builds, LUs, quadrature, residues, E_QP) followed by
gwc_spectral_cumulant (n_t = 2^18, 0.01 eV); consecutive steps take the cores
in rotation.  Inputs are resident in HBM before the timed region.  The metric
is core-state solves per second.

Printed: one JSON line with the throughput, the Pi-build roofline (algorithmic
FP64 flops / HIP-event kernel time against the 78.6 TFLOP/s FP64 MFMA peak),
the CPU oracle timed on a bounded sample of the same workload (child process),
and optional legs (precision forms, DECOUPLED mode, whole c3 / c4 core states,
CD-WAC, the fully analytic route, evGW0, peak probes), each started only while
its estimated duration fits the wall-clock limit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "core-state Σc(ω) solves/sec + Π-build MFMA util; p50/p99 latency, mixed vs FP64"
FP64_MFMA_PEAK_TFLOPS = 78.6
# FP64 vector (FMA) peak: 256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 78.6
# dense MFMA peaks of the mixed forms (TFLOP/s): 16-bit 2.5 P, fp8 5.0 P
MIXED_MFMA_PEAK_TFLOPS = {"bf16x3": 2500.0, "fp16x3": 2500.0, "fp8": 5000.0}
# timer of the bordered factorisation: LDL^T without pivoting unless
# GWC_FACTORIZATION=lu selects the partial-pivoting LU
FACT_TIMER = "lu_bordered" if os.environ.get("GWC_FACTORIZATION") == "lu" else "ldlt_bordered"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pi_build_f64_c2_traffic.json")
PI_SOURCE = os.path.join(ROOT, "paper_2412_17132_amd", "csrc", "kernels_pi.hip")


def emit(record: dict, jsonl=None) -> None:
    """Prints the result line and, with --jsonl, appends it (with a UTC time stamp
    and the git revision when available) as one line of a JSON-lines log."""
    print(json.dumps(record), flush=True)
    if jsonl:
        import datetime
        import subprocess
        rec = dict(record)
        rec["logged_utc"] = datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds")
        try:
            rec["git_rev"] = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short", "HEAD"],
                                            capture_output=True, text=True, timeout=10).stdout.strip() or None
        except (OSError, subprocess.SubprocessError):
            rec["git_rev"] = None
        with open(jsonl, "a") as f:
            f.write(json.dumps(rec) + "\n")


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _traffic_per_task():
    """HBM bytes per Pi-build frequency (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed rocprofv3 PMC summary, or None when absent or taken on
    a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != _sha(PI_SOURCE):
        return None
    return t.get("bytes_per_task")


def _blas_threads():
    """Threads of the BLAS behind NumPy/SciPy (what the oracle's GEMMs and
    factorisations use)."""
    try:
        from threadpoolctl import threadpool_info
        for info in threadpool_info():
            if info.get("internal_api") in ("openblas", "mkl", "blis"):
                return int(info.get("num_threads"))
    except Exception:
        pass
    return os.cpu_count()


def cpu_baseline_child(args):
    """The oracle timed on a bounded sample of one core-state solve (FULL mode,
    core 0 of the workload), in a process of its own (no torch, no GPU).

    Timed: the imaginary axis of the core in full (one Cholesky per node, all
    N_basis border vectors), an evenly strided sample of its residue tasks
    (one pivoted LU each) until --cpu-seconds is spent, the quadrature at every
    point, and one full-size cumulant.  The solve time is extrapolated to all of
    the core state's residue tasks by the mean task time.  Prints one JSON line."""
    import numpy as np

    from oracle import cumulant as OC
    from oracle import sigma as OS
    from workloads import CONFIGS, EV_PER_HA, system_from_config

    s = system_from_config(CONFIGS[args.config])
    c, n = 0, int(s.core_idx[0])
    L = OS.ov_matrix(s.M_ov)
    d = OS.transition_energies(s.eps, s.n_occ)
    t0 = time.perf_counter()
    W = OS.w_imag_axis(L, d, s.M_oo, s.M_ov, [n], s.omega_imag)[0]
    t_imag = time.perf_counter() - t0

    grid = [float(x) for x in s.omega_real[c]] + [float(s.eps[n])]
    tasks = []
    for j, w in enumerate(grid):
        m_subset = None if args.mode == "full" or j == len(grid) - 1 else [n]
        tasks += [(m, z) for m, _, z in OS.residue_terms(s.eps, s.occ, w, s.eta, m_subset)]
    stride = max(1, len(tasks) // 997)
    order = [k for r in range(stride) for k in range(r, len(tasks), stride)]
    done = 0
    t0 = time.perf_counter()
    for k in order:
        m, z = tasks[k]
        OS.screened_element(L, d, OS.pair_vector(s.M_oo, s.M_ov, n, m), z)
        done += 1
        if time.perf_counter() - t0 > args.cpu_seconds:
            break
    t_task = (time.perf_counter() - t0) / done

    # the same residue tasks on one thread (the first few of the sample)
    t_task1, done1 = None, 0
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for k in order[:3]:
                m, z = tasks[k]
                OS.screened_element(L, d, OS.pair_vector(s.M_oo, s.M_ov, n, m), z)
                done1 += 1
            t_task1 = (time.perf_counter() - t0) / done1
    except ImportError:
        pass

    t0 = time.perf_counter()
    for w in grid:
        OS.imag_integral(W, s.eps, s.omega_imag, s.w_imag, w)
    t_quad = time.perf_counter() - t0

    im = np.zeros(len(grid) - 1)
    im[: im.size // 2] = -1e-3  # the cumulant's cost does not depend on the values
    e_qp = float(s.eps[n]) - 0.8
    t0 = time.perf_counter()
    OC.spectral_cumulant(s.omega_real[c], im, float(s.eps[n]), e_qp, s.eta, 2 ** 18,
                         0.01 / EV_PER_HA, 3500, e_qp - 30 / EV_PER_HA)
    t_cum = time.perf_counter() - t0

    t_solve = t_imag + len(tasks) * t_task + t_quad + t_cum
    print(json.dumps({
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": _blas_threads(),
        "kind": "oracle",
        "sample": (f"one {args.mode.upper()} core-state solve of {args.config} (core 0): imaginary axis "
                   f"in full ({t_imag:.1f} s), {done} of its {len(tasks)} residue tasks evenly "
                   f"strided ({t_task * 1e3:.1f} ms each), quadrature at all {len(grid)} points "
                   f"({t_quad:.2f} s), one 2^18-point cumulant ({t_cum:.1f} s); extrapolated by "
                   f"task count to {t_solve:.0f} s per solve"),
        "sampled_s": t_imag + done * t_task + t_quad + t_cum,
        "cpu_model": _cpu_model(),
        # one thread: the residue tasks timed on one thread, the imaginary axis
        # scaled by the same ratio (both are dense FP64 factorisations)
        "single_thread": None if t_task1 is None else {
            "value": 1.0 / ((t_imag + len(tasks) * t_task) * t_task1 / t_task + t_quad + t_cum),
            "unit": "solves/s", "task_ms": t_task1 * 1e3, "tasks_timed": done1,
            "note": "residue part and imaginary axis scaled by the one-thread task time"},
    }), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args, timeout_s=150):
    """Runs cpu_baseline_child in a child process with a time limit and returns
    its record (or the reason it has none)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--config", args.config,
           "--mode", args.mode, "--cpu-seconds", str(args.cpu_seconds)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        return {"value": None, "unit": "solves/s", "kind": "oracle", "error": f"timed out after {timeout_s} s"}
    for line in reversed(r.stdout.strip().splitlines()):
        try:
            return json.loads(line)
        except ValueError:
            continue
    return {"value": None, "unit": "solves/s", "kind": "oracle",
            "error": f"exit {r.returncode}: {r.stderr.strip()[-300:]}"}

def residue_task_count(eps, occ, core_idx, omega_real, mode="full"):
    """Residue terms (n, w, m) with a nonzero prefactor (Eq. cd_prefactors:
    occupied m at or above w, virtual m at or below w) on each core's grid plus
    w = eps_n; DECOUPLED keeps only m = n on the grid.  Bookkeeping for the
    reported task counts."""
    import numpy as np
    eps = np.asarray(eps)
    occupied = np.asarray(occ) > 0
    omega_real = np.asarray(omega_real).reshape(len(core_idx), -1)
    def live(w):
        return (occupied & (eps >= w)) | (~occupied & (eps <= w))

    total = 0
    for c, n in enumerate(core_idx):
        n = int(n)
        for w in omega_real[c]:
            total += int(live(w).sum()) if mode == "full" else int(live(w)[n])
        total += int(live(float(eps[n])).sum())
    return total


def measure_peaks(gwc):
    """Device peaks re-measured by the library's probes (register-operand MFMA
    loops, a 4 GiB device copy), beside the datasheet figures."""
    return {
        "fp64_mfma_tflops": gwc.probe_peak("fp64_mfma"),
        "bf16_mfma_tflops": gwc.probe_peak("bf16_mfma"),
        "fp16_mfma_tflops": gwc.probe_peak("fp16_mfma"),
        "fp8_k32_mfma_tflops": gwc.probe_peak("fp8_mfma_k32"),
        "fp8_k128_mfma_tflops": gwc.probe_peak("fp8_mfma_k128"),
        "hbm_copy_gbs": gwc.probe_peak("hbm_copy"),
        "datasheet": {"fp64_mfma_tflops": 78.6, "bf16_mfma_tflops": 2500.0,
                      "fp16_mfma_tflops": 2500.0, "fp8_mfma_tflops": 5000.0, "hbm_gbs": 8000.0},
    }


def sampled_main(args):
    """Large workloads (c3, c4) whose FULL solve takes minutes to hours: time
    one core state at two real-grid sizes (1 and --sample-points points, spread
    over its grid) on a device-resident system, take the per-task cost from the
    difference, and extrapolate to the full grid.  Labelled as sampled."""
    import numpy as np
    import torch

    import paper_2412_17132_amd as gwc
    from paper_2412_17132_amd.serve import ResidentSystem
    from workloads import CONFIGS, EV_PER_HA, system_from_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = CONFIGS[args.config]
    s = system_from_config(cfg)
    n_core = s.n_core
    n_tasks_full = residue_task_count(s.eps, s.occ, s.core_idx, s.omega_real, args.mode)
    rs = ResidentSystem.from_system(s)
    core = s.core_idx[:1]
    n_real = s.omega_real.shape[1]

    def run(k):
        idx = np.unique(np.linspace(0, n_real - 1, k).round().astype(int))
        w = np.ascontiguousarray(s.omega_real[:1, idx])
        tasks = residue_task_count(s.eps, s.occ, core, w, args.mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = rs.sigma_core(core, s.omega_imag, s.w_imag, w, s.eta, mode=args.mode,
                            precision=args.precision)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, tasks, out

    print(f"sampled {cfg.name}: warm-up", file=sys.stderr, flush=True)
    run(1)
    gwc.timing_enable(True)
    t_a, n_a, _ = run(1)
    print(f"sampled {cfg.name}: 1 point, {n_a} tasks, {t_a:.2f} s", file=sys.stderr, flush=True)
    t_b, n_b, out = run(args.sample_points)
    print(f"sampled {cfg.name}: {args.sample_points} points, {n_b} tasks, {t_b:.2f} s",
          file=sys.stderr, flush=True)
    pi = gwc.timing_get("pi_build_f64" if args.precision == "fp64" else "pi_build_mixed")
    lu = gwc.timing_get(FACT_TIMER)
    gwc.timing_enable(False)
    t_task = (t_b - t_a) / (n_b - n_a)
    t_fixed = max(t_a - n_a * t_task, 0.0)
    d_omega = 0.01 / EV_PER_HA
    e_qp = float(out["e_qp"][0])
    wg = torch.as_tensor(np.ascontiguousarray(s.omega_real[0]), device="cuda:0")
    im_full = torch.zeros_like(wg)  # cumulant cost does not depend on the values
    gwc.gwc_spectral_cumulant(wg, im_full, float(s.eps[core[0]]), e_qp, s.eta, 2 ** 18, d_omega,
                              3500, e_qp - 30 / EV_PER_HA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gwc.gwc_spectral_cumulant(wg, im_full, float(s.eps[core[0]]), e_qp, s.eta, 2 ** 18, d_omega,
                              3500, e_qp - 30 / EV_PER_HA)
    torch.cuda.synchronize()
    t_cum = time.perf_counter() - t0
    t_solve = t_fixed + (n_tasks_full / n_core) * t_task + t_cum
    pi_tf = pi["flops"] / (pi["total_ms"] / 1e3) / 1e12 if pi["total_ms"] > 0 else 0.0
    lu_tf = lu["flops"] / (lu["total_ms"] / 1e3) / 1e12 if lu["total_ms"] > 0 else 0.0
    peak = FP64_MFMA_PEAK_TFLOPS if args.precision == "fp64" else MIXED_MFMA_PEAK_TFLOPS[args.precision]
    mfma = pi_tf if args.precision == "fp64" else 3.0 * pi_tf
    rs.close()
    line = {
        "metric": METRIC,
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 2,
        "warmup": 1,
        "ms_per_step": t_solve * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description} -- SAMPLED: one core state at 1 and "
                               f"{args.sample_points} real points ({n_a} and {n_b} residue tasks), "
                               f"extrapolated to {n_tasks_full / n_core:.0f} tasks per core state",
                   "n_basis": cfg.n_basis, "n_occ": cfg.n_occ, "n_core": n_core, "n_aux": cfg.n_aux,
                   "n_imag": cfg.n_imag, "n_real": n_real, "mode": args.mode,
                   "precision": args.precision, "parallelism": "single-gpu"},
        "sampled": {"t_fixed_s": t_fixed, "t_task_ms": t_task * 1e3, "t_cumulant_s": t_cum,
                    "tasks_per_core_state": n_tasks_full / n_core},
        "roofline": {"bound": "mfma", "achieved": mfma, "peak": peak, "unit": "TFLOP/s",
                     "frac": mfma / peak, "traffic": None,
                     "kernel": "pi_build_f64" if args.precision == "fp64" else "pi_build_mixed",
                     "avg_launch_ms": pi["total_ms"] / max(pi["launches"], 1)},
        "kernels": {"pi_build": {"ms": pi["total_ms"], "launches": pi["launches"], "tflops": pi_tf},
                    FACT_TIMER: {"ms": lu["total_ms"], "launches": lu["launches"], "tflops": lu_tf}},
    }
    emit(line, args.jsonl)


def _satellites(w, A, e_qp, Z, eta, min_sep_ev=0.5, rel_height=0.05):
    """Satellite peaks: local maxima of A - Z L_eta(w - E_QP) more than 0.5 eV
    below E_QP with height >= 5 % of that remainder's maximum there, refined by
    a parabola (the paper's criterion is in its SI, which is not available)."""
    import numpy as np
    from workloads import EV_PER_HA
    A = A - Z * (eta / np.pi) / ((w - e_qp) ** 2 + eta * eta)
    region = w < e_qp - min_sep_ev / EV_PER_HA
    if not np.any(region):
        return []
    top = np.max(A[region])
    idx = np.where((A[1:-1] > A[:-2]) & (A[1:-1] >= A[2:]))[0] + 1
    out = []
    for i in idx:
        if not region[i] or A[i] < rel_height * top:
            continue
        y0, y1, y2 = A[i - 1], A[i], A[i + 1]
        den = y0 - 2 * y1 + y2
        dx = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append(w[i] + dx * (w[i + 1] - w[i]))
    return out


def serve_main(args):
    """Poisson arrivals of single-core-state requests (DECOUPLED + A(w)) from a
    pool of device-resident molecules with N_basis ~ U{40..max}, N_aux = 4 N_basis,
    N_occ = N_basis / 15; prints one JSON line with p50/p99 latency and solves/s."""
    import threading

    import numpy as np
    import torch

    from paper_2412_17132_amd.serve import ResidentSystem, Server
    from workloads import EV_PER_HA, serving_request_config, system_from_config

    if args.gpus != 1:
        print("bench.py --serve runs on one GPU only", file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    rng = np.random.default_rng(5)
    sizes = sorted(int(x) for x in rng.integers(40, args.serve_max_nbasis + 1, args.serve_pool))
    mols = [system_from_config(serving_request_config(nb, 1000 + i)) for i, nb in enumerate(sizes)]
    res = [ResidentSystem.from_system(s) for s in mols]
    nbasis = [s.n_basis for s in mols]
    for s in mols:  # host copies are no longer needed
        s.M_oo = s.M_ov = None
    precision = args.precision
    srv = Server(n_slots=args.serve_slots, hbm_budget_bytes=args.serve_budget_gb * 2 ** 30)

    def submit(i, c):
        s = mols[i]
        return srv.submit(res[i], c, s.omega_imag, s.w_imag, s.omega_real[c], s.eta, mode="decoupled",
                          precision=precision, n_t=2 ** 18, d_omega=0.01 / EV_PER_HA, n_out=3500,
                          omega_out_min_rel=-30 / EV_PER_HA)

    # warm-up: one request per molecule (also builds the split operands)
    for i, s in enumerate(mols):
        srv.wait(submit(i, 0))
    gaps = rng.exponential(1.0 / args.serve_rate, args.serve_requests)
    picks = [(int(rng.integers(len(mols))), None) for _ in range(args.serve_requests)]
    picks = [(i, int(rng.integers(len(mols[i].core_idx)))) for i, _ in picks]
    tickets = [None] * args.serve_requests

    def feeder():
        t0 = time.perf_counter()
        at = 0.0
        for k, (i, c) in enumerate(picks):
            at += gaps[k]
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[k] = submit(i, c)

    th = threading.Thread(target=feeder)
    t_start = time.perf_counter()
    th.start()
    # results are collected in arrival order while the feeder still submits
    out = []
    for k in range(len(tickets)):
        while tickets[k] is None:
            time.sleep(0.005)
        out.append(srv.wait(tickets[k]))
        if (k + 1) % 20 == 0:
            print(f"serve: {k + 1}/{len(tickets)} requests done "
                  f"({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)
    th.join()
    wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    lat = np.array([r["t_end"] - r["t_submit"] for r in out])
    first = min(r["t_submit"] for r in out)
    last = max(r["t_end"] for r in out)
    nbs = [nbasis[i] for i, _ in picks]
    line = {
        "metric": METRIC,
        "value": len(out) / (last - first),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(out),
        "warmup": len(mols),
        "ms_per_step": 1e3 * (last - first) / len(out),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else precision,
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson stream, lambda={args.serve_rate}/s, {len(out)} "
                               f"single-core-state requests (DECOUPLED + A(w)), {len(mols)} resident "
                               f"molecules N_basis {sizes}, N_aux = 4 N_basis",
                   "precision": precision, "slots": args.serve_slots,
                   "hbm_budget_gb": args.serve_budget_gb, "parallelism": "single-gpu"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "per": "request (arrival to result)"},
        "serving": {"offered_rate": args.serve_rate,
                    "achieved_rate": len(out) / (last - first),
                    "wall_s": wall, "peak_concurrent_requests": st["peak_active"],
                    "peak_in_use_gb": st["peak_in_use_bytes"] / 2 ** 30,
                    "kept_split_operands_gb": st["kept_bytes"] / 2 ** 30,
                    "refused_requests": st["refused"],
                    "mean_nbasis": float(np.mean(nbs))},
    }
    emit(line, args.jsonl)


class Guard:
    """Wall-clock guard of the optional legs: a leg starts only when its
    estimated duration still fits before the limit (seconds since the process
    started); a leg that does not start is recorded as skipped."""

    def __init__(self, limit_s):
        self.limit = float(limit_s)

    def elapsed(self):
        return time.perf_counter() - T_START

    def run(self, res, name, estimate_s, fn):
        if self.elapsed() + estimate_s > self.limit:
            res[name] = {"skipped": "budget", "estimate_s": round(estimate_s, 1),
                         "elapsed_s": round(self.elapsed(), 1), "limit_s": self.limit}
            print(f"bench: leg {name} skipped (estimate {estimate_s:.0f} s, elapsed "
                  f"{self.elapsed():.0f} s of {self.limit:.0f} s)", file=sys.stderr, flush=True)
            return
        print(f"bench: leg {name} (estimate {estimate_s:.0f} s, elapsed {self.elapsed():.0f} s)",
              file=sys.stderr, flush=True)
        t = time.perf_counter()
        res[name] = fn()
        res[name]["leg_wall_s"] = round(time.perf_counter() - t, 2)


def _rate(t):
    return t["flops"] / (t["total_ms"] / 1e3) / 1e12 if t["total_ms"] > 0 else 0.0


def _sigma_rel(ref_out, out):
    """max and median over points of |dSigma^c| / max|Sigma^c_ref| (one core)."""
    import numpy as np
    a = ref_out["sigma_c"][0].cpu().numpy()
    b = out["sigma_c"][0].cpu().numpy()
    ca = a[..., 0] + 1j * a[..., 1]
    cb = b[..., 0] + 1j * b[..., 1]
    rel = np.abs(cb - ca) / np.max(np.abs(ca))
    return rel


def _compare_solves(ref, res, eta, n_out, d_omega):
    """E_QP, satellite-position and Sigma^c deviations of one set of core-state
    solves from another (both {core: (out, A, z)})."""
    import numpy as np
    from workloads import EV_PER_HA
    deq, worst, lowest, rels, by_core = [], 0.0, 0.0, [], []
    for c, (out, A, z) in res.items():
        if c not in ref:
            continue
        r_out, r_A, r_z = ref[c]
        eq_r, eq_m = float(r_out["e_qp"][0]), float(out["e_qp"][0])
        deq.append(abs(eq_m - eq_r))
        wr = eq_r - 30 / EV_PER_HA + np.arange(n_out) * d_omega
        wm = eq_m - 30 / EV_PER_HA + np.arange(n_out) * d_omega
        pr = _satellites(wr, r_A.cpu().numpy(), eq_r, float(r_z[0]), eta)
        pm = _satellites(wm, A.cpu().numpy(), eq_m, float(z[0]), eta)
        for p in pr:
            if pm:
                worst = max(worst, float(np.min(np.abs(np.asarray(pm) - p))))
        if pr and pm:  # the lowest-lying satellite (closest to the QP peak)
            d = float(np.min(np.abs(np.asarray(pm) - max(pr))))
            lowest = max(lowest, d)
            by_core.append(round(d * EV_PER_HA * 1e3, 3))
        if out.get("sigma_c") is not None and r_out.get("sigma_c") is not None:
            rels.append(_sigma_rel(r_out, out))
    rec = {"cores_compared": len(deq),
           "e_qp_max_dev_mev": float(max(deq) * EV_PER_HA * 1e3) if deq else None,
           "satellite_max_shift_mev": worst * EV_PER_HA * 1e3,
           "lowest_satellite_shift_mev": lowest * EV_PER_HA * 1e3,
           "lowest_satellite_shift_mev_by_core": by_core}
    if rels:
        allr = np.concatenate(rels)
        rec["sigma_c_rel_dev"] = {"max": float(allr.max()), "median": float(np.median(allr))}
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6, help="timed core-state solves")
    ap.add_argument("--warmup", type=int, default=2, help="untimed core-state solves before them")
    ap.add_argument("--config", default="c2", help="workload (default: the benzene-sized c2)")
    ap.add_argument("--mode", default="full", choices=["full", "decoupled"])
    ap.add_argument("--n-real", type=int, default=None,
                    help="override the real grid size (a reduced run, not the named workload)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "bf16x3", "fp16x3", "fp8"],
                    help="precision of the timed path (default FP64)")
    ap.add_argument("--compare", default="bf16x3,fp8",
                    help="comma-separated mixed-precision forms also timed (one solve per core "
                         "state) with their E_QP / satellite / Sigma^c deviations from FP64, or none")
    ap.add_argument("--legs", default="cpu,mixed,decoupled,c3,c4,wac,analytic,evgw0,peaks",
                    help="optional legs after the timed region, in order (comma-separated)")
    ap.add_argument("--time-limit", type=float, default=450.0,
                    help="start no optional leg that would end later than this many seconds "
                         "after the process started")
    ap.add_argument("--sample-points", type=int, default=0,
                    help="sampled run for large workloads (c3, c4): one core state at 1 and this "
                         "many real points, extrapolated to the full grid")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="residue-task time budget of the CPU oracle sample")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: a Poisson stream of single-core-state "
                         "requests through the continuous-batching server")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="arrivals per second")
    ap.add_argument("--serve-pool", type=int, default=6, help="distinct molecules (device-resident)")
    ap.add_argument("--serve-max-nbasis", type=int, default=1100)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=96.0)
    ap.add_argument("--jsonl", default=None,
                    help="also append the result line (plus time stamp and git revision) to this "
                         "JSON-lines file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.cpu_baseline_child:
        return cpu_baseline_child(args)
    if args.calibrate_copy:
        import torch
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 2 ** 30, "bytes_written": 2 ** 30,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout "
              "is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve_main(args)
    if args.sample_points:
        return sampled_main(args)

    import numpy as np
    import torch

    import paper_2412_17132_amd as gwc
    from workloads import CONFIGS, EV_PER_HA, system_from_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")
    dev = torch.device("cuda:0")
    guard = Guard(args.time_limit)
    cfg = CONFIGS[args.config]
    over = {} if args.n_real is None else {"n_real": args.n_real}
    s = system_from_config(cfg, **over)
    d = gwc.to_device(s, dev)
    n_core = s.n_core
    n_t, d_omega, n_out = 2 ** 18, 0.01 / EV_PER_HA, 3500

    def solve(c, precision=args.precision, mode=args.mode, wac=None, sh=s, sd=d):
        """One core-state solve: Sigma^c_n on its grid (FULL) or Sigma^c_n(eps_n)
        plus Im Sigma^dec (DECOUPLED), E_QP, and A_n(w) from the cumulant."""
        out = gwc.gwc_sigma_core(sd["eps"], sd["occ"], sd["M_oo"], sd["M_ov"], sd["core_idx"][c:c + 1],
                                 sd["omega_imag"], sd["w_imag"], sd["omega_real"][c:c + 1], sd["eta"],
                                 mode=mode, precision=precision, wac=wac)
        e_qp = float(out["e_qp"][0])
        n = int(sh.core_idx[c])
        A, z = gwc.gwc_spectral_cumulant(sd["omega_real"][c], out["im_sigma_dec"][0], float(sh.eps[n]),
                                         e_qp, sh.eta, n_t, d_omega, n_out, e_qp - 30 / EV_PER_HA)
        return out, A, z

    tasks_of = [residue_task_count(s.eps, s.occ, s.core_idx[c:c + 1], s.omega_real[c:c + 1], args.mode)
                for c in range(n_core)]
    print(f"bench: {cfg.name} {args.mode} {args.precision}, {args.warmup} warm-up + {args.steps} timed "
          f"core-state solves", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        solve(k % n_core)
    torch.cuda.synchronize()
    gwc.timing_enable(True)
    lat, last = [], {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        last[k % n_core] = solve(k % n_core)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pi_name = "pi_build_f64" if args.precision == "fp64" else "pi_build_mixed"
    pi = gwc.timing_get(pi_name)
    lu = gwc.timing_get(FACT_TIMER)
    gwc.timing_enable(False)
    t_step = elapsed / args.steps
    print(f"bench: timed region {elapsed:.2f} s ({t_step:.3f} s per core-state solve)",
          file=sys.stderr, flush=True)

    n_tasks = sum(tasks_of[k % n_core] for k in range(args.steps))
    launches = max(pi["launches"], 1)
    achieved = _rate(pi)
    tpt = _traffic_per_task()
    pi_tasks = args.steps * len(s.omega_imag) + n_tasks
    tpl = None if tpt is None else tpt * pi_tasks / launches
    peak = FP64_MFMA_PEAK_TFLOPS
    if args.precision != "fp64":
        # three 16-bit (or 8-bit) MFMA products per algorithmic multiply-add
        achieved, peak, tpl = 3.0 * achieved, MIXED_MFMA_PEAK_TFLOPS[args.precision], None
    res = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg.name}: {cfg.description}; one step = one core-state solve "
                         f"({args.mode.upper()} Sigma^c on {s.omega_real.shape[1]} points + E_QP + "
                         f"A(w)), cores in rotation" + ("" if args.n_real is None else
                                                        f" (n_real={args.n_real})")),
            "n_basis": cfg.n_basis, "n_occ": cfg.n_occ, "n_core": n_core, "n_aux": cfg.n_aux,
            "n_imag": cfg.n_imag, "n_real": s.omega_real.shape[1], "eta_ev": cfg.eta_ev,
            "mode": args.mode, "precision": args.precision,
            "residue_tasks_timed": n_tasks, "cumulant_n_t": n_t, "parallelism": "single-gpu",
        },
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "per": "core-state solve"},
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": tpl,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": pi_name,
            "launches": pi["launches"],
            "avg_launch_ms": pi["total_ms"] / launches,
            "flops_per_launch": pi["flops"] / launches,
        },
        "kernels": {
            pi_name: {"ms": pi["total_ms"], "launches": pi["launches"], "tflops": _rate(pi)},
            FACT_TIMER: {"ms": lu["total_ms"], "launches": lu["launches"], "tflops": _rate(lu)},
        },
    }

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    compare = [] if args.compare == "none" else [x.strip() for x in args.compare.split(",") if x.strip()]

    def leg_cpu():
        return cpu_baseline(args)

    def leg_mixed(prec):
        def run():
            solve(0, prec)  # warm-up (also builds the split operands)
            torch.cuda.synchronize()
            gwc.timing_enable(True)
            got = {}
            tm = time.perf_counter()
            for c in range(n_core):
                got[c] = solve(c, prec)
            torch.cuda.synchronize()
            el = time.perf_counter() - tm
            pim = gwc.timing_get("pi_build_mixed")
            lum = gwc.timing_get(FACT_TIMER)
            gwc.timing_enable(False)
            alg = _rate(pim)
            rec = {"precision": prec, "value": n_core / el, "unit": "solves/s",
                   "ms_per_step": el / n_core * 1e3, "speedup_vs_fp64": t_step / (el / n_core),
                   "pi_build_ms": pim["total_ms"], "pi_build_algorithmic_tflops": alg,
                   "pi_build_mfma_tflops": 3.0 * alg,
                   "pi_build_mfma_peak_tflops": MIXED_MFMA_PEAK_TFLOPS[prec],
                   "pi_build_mfma_frac": 3.0 * alg / MIXED_MFMA_PEAK_TFLOPS[prec],
                   "factorization_ms": lum["total_ms"]}
            rec["vs_fp64"] = _compare_solves(last, got, s.eta, n_out, d_omega)
            return rec
        return run

    def leg_decoupled():
        solve(0, mode="decoupled")
        torch.cuda.synchronize()
        td = time.perf_counter()
        for c in range(n_core):
            solve(c, mode="decoupled")
        torch.cuda.synchronize()
        el = time.perf_counter() - td
        return {"value": n_core / el, "unit": "solves/s", "ms_per_step": el / n_core * 1e3,
                "residue_tasks": residue_task_count(s.eps, s.occ, s.core_idx, s.omega_real, "decoupled"),
                "precision": args.precision}

    def leg_wac():
        wp = gwc.wac_paper_settings()
        solve(0, wac=wp)
        torch.cuda.synchronize()
        got = {}
        tw = time.perf_counter()
        for c in range(n_core):
            got[c] = solve(c, wac=wp)
        torch.cuda.synchronize()
        el = time.perf_counter() - tw
        rec = {"value": n_core / el, "unit": "solves/s", "ms_per_step": el / n_core * 1e3,
               "speedup_vs_cd": t_step / (el / n_core),
               "settings": {k: (v * EV_PER_HA if k in ("core_min", "core_max") else v) for k, v in wp.items()},
               "settings_units": "core window in eV",
               "reference_factorisations_per_solve": wp["n_core_pts"] + wp["n_val_pts"]}
        rec["dev_from_cd"] = _compare_solves(last, got, s.eta, n_out, d_omega)
        # the paper's production setting: DECOUPLED spectra, here also on
        # core-localised inputs (core/other RI coefficients scaled by 1e-3)
        dec = {}
        for label, sh in (("decoupled", s), ("decoupled_core_localised", None)):
            if sh is None:
                sh = system_from_config(cfg, structured=True, **over)
            sd = d if sh is s else gwc.to_device(sh, dev)
            cd_dec = {c: solve(c, mode="decoupled", sh=sh, sd=sd) for c in range(n_core)}
            torch.cuda.synchronize()
            tw = time.perf_counter()
            wac_dec = {c: solve(c, mode="decoupled", wac=wp, sh=sh, sd=sd) for c in range(n_core)}
            torch.cuda.synchronize()
            el_d = time.perf_counter() - tw
            dec[label] = {"solves_per_s": n_core / el_d,
                          "dev_from_cd": _compare_solves(cd_dec, wac_dec, sh.eta, n_out, d_omega)}
        rec.update(dec)
        return rec

    def leg_analytic():
        def astep():
            return gwc.gwc_sigma_analytic(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                                          d["omega_real"], d["eta"])
        astep()
        torch.cuda.synchronize()
        gwc.timing_enable(True)
        ta = time.perf_counter()
        aout = astep()
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        ja, jp = gwc.timing_get("jacobi_apply"), gwc.timing_get("jacobi_pairs")
        gwc.timing_enable(False)
        ja_tf = _rate(ja)
        deq = [abs(float(aout["e_qp"][c]) - float(last[c][0]["e_qp"][0])) for c in last]
        return {"value": n_core / el, "unit": "solves/s (all core states in one call)",
                "ms_per_call": el * 1e3, "n_ov": int(s.M_ov.shape[1] * s.M_ov.shape[2]),
                "jacobi_sweeps": int(aout["sweeps"][0]),
                "jacobi_apply": {"ms": ja["total_ms"], "launches": ja["launches"],
                                 "avg_launch_ms": ja["total_ms"] / max(ja["launches"], 1),
                                 "bound": "mfma", "achieved": ja_tf, "peak": FP64_MFMA_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": ja_tf / FP64_MFMA_PEAK_TFLOPS},
                "jacobi_pairs_ms": jp["total_ms"],
                "e_qp_dev_from_cd_mev": float(max(deq) * EV_PER_HA * 1e3) if deq else None}

    def leg_evgw0():
        from workloads import vv_block
        dvv = torch.as_tensor(vv_block(s), device=dev)

        def evstep():
            return gwc.gwc_evgw0(d["eps"], d["occ"], d["M_oo"], d["M_ov"], dvv, d["core_idx"],
                                 d["omega_real"], d["eta"])
        evstep()
        torch.cuda.synchronize()
        te = time.perf_counter()
        eout = evstep()
        torch.cuda.synchronize()
        el = time.perf_counter() - te
        eq = eout["e_qp"].cpu().numpy()
        e1 = eout["e_first"].cpu().numpy()
        core = s.core_idx
        return {"value": n_core / el, "unit": "solves/s (core states; every state iterated)",
                "ms_per_call": el * 1e3, "states_iterated": int(s.n_basis),
                "outer_iterations": int(eout["outer"][0]), "max_newton_steps": int(eout["newton"].max()),
                "core_shift_g0w0_ev": [float(x) for x in (e1[core] - s.eps[core]) * EV_PER_HA],
                "core_shift_evgw0_ev": [float(x) for x in (eq[core] - s.eps[core]) * EV_PER_HA]}

    def leg_whole(name, mode, mixed=()):
        """One whole core state (core 0) of a larger workload, unsampled, in FP64
        and then in each precision form of `mixed` on the same resident system
        (speed-up and deviation from the FP64 solve)."""
        def run():
            cf = CONFIGS[name]
            tg = time.perf_counter()
            sh = system_from_config(cf)
            sd = gwc.to_device(sh, dev)
            t_gen = time.perf_counter() - tg
            tasks = residue_task_count(sh.eps, sh.occ, sh.core_idx[:1], sh.omega_real[:1], mode)
            torch.cuda.synchronize()
            gwc.timing_enable(True)
            tw = time.perf_counter()
            out, A, z = solve(0, "fp64", mode, None, sh, sd)
            torch.cuda.synchronize()
            el = time.perf_counter() - tw
            p, u = gwc.timing_get("pi_build_f64"), gwc.timing_get(FACT_TIMER)
            gwc.timing_enable(False)
            e_qp = float(out["e_qp"][0])
            rec = {"workload": f"{cf.name}: {cf.description}; core 0, {mode.upper()}, FP64, whole and "
                               f"unsampled (no warm-up: first call on this system)",
                   "value": 1.0 / el, "unit": "solves/s", "s_per_solve": el,
                   "residue_tasks": tasks, "n_imag": cf.n_imag, "n_real": cf.n_real,
                   "pi_build": {"ms": p["total_ms"], "launches": p["launches"], "tflops": _rate(p),
                                "frac": _rate(p) / FP64_MFMA_PEAK_TFLOPS},
                   FACT_TIMER: {"ms": u["total_ms"], "launches": u["launches"], "tflops": _rate(u)},
                   "e_qp_shift_ev": (e_qp - float(sh.eps[0])) * EV_PER_HA,
                   "setup_s": t_gen}
            ref = {0: (out, A, z)}
            for prec in mixed:
                gwc.timing_enable(True)
                tw = time.perf_counter()
                got = solve(0, prec, mode, None, sh, sd)
                torch.cuda.synchronize()
                el_m = time.perf_counter() - tw
                pm, um = gwc.timing_get("pi_build_mixed"), gwc.timing_get(FACT_TIMER)
                gwc.timing_enable(False)
                issued = 3 * _rate(pm)
                rec.setdefault("mixed", {})[prec] = {
                    "s_per_solve": el_m, "speedup_vs_fp64": el / el_m,
                    "pi_build_ms": pm["total_ms"], "pi_build_algorithmic_tflops": _rate(pm),
                    "pi_build_mfma_frac": issued / MIXED_MFMA_PEAK_TFLOPS[prec],
                    "factorization_ms": um["total_ms"],
                    "vs_fp64": _compare_solves(ref, {0: got}, sh.eta, n_out, d_omega),
                    "note": "first call in this precision on the system (includes building its split operands)"}
                del got
            del sd, out, A, z, ref
            torch.cuda.empty_cache()
            return rec
        return run

    def leg_peaks():
        return measure_peaks(gwc)

    # per-task time of the timed path, scaled by the Pi-build work of a task
    # (N_aux^2 N_ov), estimates the larger workloads for the wall-clock guard
    t_task = elapsed / max(n_tasks + args.steps * len(s.omega_imag), 1)

    def scaled(name, mode):
        cf = CONFIGS[name]
        probe = system_from_config(cf, n_aux=1)  # energies and grids do not depend on N_aux
        k = residue_task_count(probe.eps, probe.occ, probe.core_idx[:1], probe.omega_real[:1], mode)
        w = (cf.n_aux / cfg.n_aux) ** 2 * (cf.n_ov / cfg.n_ov)
        return 1.25 * (k + cf.n_imag) * t_task * w + 20.0

    for leg in legs:
        if leg == "cpu":
            print("bench: cpu baseline (child process)", file=sys.stderr, flush=True)
            res["cpu_baseline"] = leg_cpu()
        elif leg == "mixed" and args.precision == "fp64":
            for prec in compare:
                guard.run(res.setdefault("mixed", {}), prec, 1.0 * (n_core + 1) * t_step + 5,
                          leg_mixed(prec))
        elif leg == "decoupled" and args.mode == "full":
            guard.run(res, "decoupled", 0.3 * (n_core + 1) * t_step + 5, leg_decoupled)
        elif leg == "c3" and args.config == "c2":
            guard.run(res, "c3_full_fp64", 1.6 * scaled("c3", "full"),
                      leg_whole("c3", "full", ("bf16x3", "fp16x3")))
        elif leg == "c4" and args.config == "c2":
            guard.run(res, "c4_decoupled_fp64", 1.6 * scaled("c4", "decoupled"),
                      leg_whole("c4", "decoupled", ("bf16x3", "fp8")))
        elif leg == "wac":
            guard.run(res, "wac", 0.6 * (n_core + 1) * t_step + 10, leg_wac)
        elif leg == "analytic" and args.mode == "full":
            guard.run(res, "analytic", 10.0, leg_analytic)
        elif leg == "evgw0" and args.mode == "full":
            guard.run(res, "evgw0", 15.0, leg_evgw0)
        elif leg == "peaks":
            guard.run(res, "peaks_measured", 15.0, leg_peaks)
            pk = res["peaks_measured"]
            if "fp64_mfma_tflops" in pk and args.precision == "fp64":
                res["roofline"]["peak_measured"] = pk["fp64_mfma_tflops"]
                res["roofline"]["frac_of_measured"] = achieved / pk["fp64_mfma_tflops"]
    res["wall_s"] = round(guard.elapsed(), 1)
    emit(res, args.jsonl)

if __name__ == "__main__":
    main()
