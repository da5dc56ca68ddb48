#!/usr/bin/env python
"""Throughput benchmark of the GW+C core-level path on one MI355X.

One step = one pass of the whole path over the benzene-sized workload
(N_basis = 300, N_occ = 21 with 6 C1s levels, N_aux = 1200, 32 imaginary and
400 real frequencies per core, eta = 0.1 eV): gwc_sigma_core in FULL mode for
all 6 core states (Pi builds, LUs, quadrature, residues, E_QP) followed by
gwc_spectral_cumulant for each core (n_t = 2^18, 0.01 eV).  Inputs are
resident in HBM before the timed region.  The metric is core-state solves per
second (one solve = Sigma^c_n on its grid + E_QP + A_n(w)).

Printed: one JSON line with the throughput, the Pi-build roofline (algorithmic
FP64 flops / HIP-event kernel time against the 78.6 TFLOP/s FP64 MFMA peak)
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "core-state Σc(ω) solves/sec + Π-build MFMA util; p50/p99 latency, mixed vs FP64"
FP64_MFMA_PEAK_TFLOPS = 78.6
# FP64 vector (FMA) peak: 256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 78.6
# dense MFMA peaks of the mixed forms (TFLOP/s): 16-bit 2.5 P, fp8 5.0 P
MIXED_MFMA_PEAK_TFLOPS = {"bf16x3": 2500.0, "fp16x3": 2500.0, "fp8": 5000.0}
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


def cpu_baseline(system, mode, n_tasks_per_core, budget_tasks=24):
    """Times the oracle on a bounded sample and extrapolates to solves/s:
    the imaginary axis of all cores, `budget_tasks` residue tasks, and one
    cumulant at full size."""
    import numpy as np

    from oracle import cumulant as OC
    from oracle import sigma as OS
    from workloads import EV_PER_HA

    threads = None
    try:
        from threadpoolctl import threadpool_info
        for info in threadpool_info():
            if info.get("internal_api") in ("openblas", "mkl", "blis"):
                threads = int(info.get("num_threads"))
                break
    except Exception:
        pass
    if threads is None:
        threads = os.cpu_count()

    s = system
    cores = [int(n) for n in s.core_idx]
    L = OS.ov_matrix(s.M_ov)
    d = OS.transition_energies(s.eps, s.n_occ)
    t0 = time.perf_counter()
    W = OS.w_imag_axis(L, d, s.M_oo, s.M_ov, cores, s.omega_imag)
    t_imag = time.perf_counter() - t0

    rng = np.random.default_rng(0)
    done = 0
    t0 = time.perf_counter()
    while done < budget_tasks:
        c = int(rng.integers(len(cores)))
        j = int(rng.integers(s.omega_real.shape[1]))
        n = cores[c]
        for m, f, z in OS.residue_terms(s.eps, s.occ, float(s.omega_real[c, j]), s.eta):
            OS.screened_element(L, d, OS.pair_vector(s.M_oo, s.M_ov, n, m), z)
            done += 1
            if done >= budget_tasks:
                break
    t_task = (time.perf_counter() - t0) / done

    c = 0
    n = cores[c]
    im = np.zeros(s.omega_real.shape[1])
    t0 = time.perf_counter()
    I = OS.imag_integral(W[c], s.eps, s.omega_imag, s.w_imag, float(s.omega_real[c, 0]))
    t_quad = (time.perf_counter() - t0) * (s.omega_real.shape[1] + 1)
    im[: im.size // 2] = -1e-3
    e_qp = float(s.eps[n]) - 0.8
    t0 = time.perf_counter()
    OC.spectral_cumulant(s.omega_real[c], im, float(s.eps[n]), e_qp, 0.1 / EV_PER_HA, 2 ** 18,
                         0.01 / EV_PER_HA, 3500, e_qp - 30 / EV_PER_HA)
    t_cum = time.perf_counter() - t0
    del I

    t_solve = t_imag / len(cores) + n_tasks_per_core * t_task + t_quad + t_cum
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"imaginary axis of all {len(cores)} cores ({t_imag:.1f} s), {done} residue "
                   f"tasks ({t_task * 1e3:.0f} ms each), one 2^18-point cumulant ({t_cum:.1f} s); "
                   f"extrapolated to {n_tasks_per_core:.0f} residue tasks per core-state solve"),
    }


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
        "hbm_copy_gbs": gwc.probe_peak("hbm_copy"),
        "datasheet": {"fp64_mfma_tflops": 78.6, "bf16_mfma_tflops": 2500.0,
                      "fp16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0},
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
    lu = gwc.timing_get("lu_bordered")
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
                    "lu_bordered": {"ms": lu["total_ms"], "launches": lu["launches"], "tflops": lu_tf}},
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
    th.join()
    out = []
    for k, t in enumerate(tickets):
        out.append(srv.wait(t))
        if (k + 1) % 20 == 0:
            print(f"serve: {k + 1}/{len(tickets)} requests done", file=sys.stderr, flush=True)
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
                    "mean_nbasis": float(np.mean(nbs))},
    }
    emit(line, args.jsonl)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", help="workload (default: the benzene-sized c2)")
    ap.add_argument("--mode", default="full", choices=["full", "decoupled"])
    ap.add_argument("--n-real", type=int, default=None,
                    help="override the real grid size (a reduced run, not the named workload)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "bf16x3", "fp16x3", "fp8"],
                    help="precision of the timed path (default FP64)")
    ap.add_argument("--compare", default="bf16x3", choices=["none", "bf16x3", "fp16x3", "fp8"],
                    help="also time this mixed-precision form and report its speed-up and its "
                         "E_QP / satellite-position errors against the FP64 path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the peak-rate probes")
    ap.add_argument("--no-wac", action="store_true",
                    help="skip the CD-WAC leg (the paper's settings) reported beside the CD value")
    ap.add_argument("--no-decoupled", action="store_true",
                    help="skip the DECOUPLED-mode leg reported beside the FULL value")
    ap.add_argument("--no-analytic", action="store_true",
                    help="skip the fully analytic G0W0 leg (Casida eigensolve + pole sums)")
    ap.add_argument("--no-evgw", action="store_true",
                    help="skip the evGW0 leg (all states' energies iterated; M_vv of the workload)")
    ap.add_argument("--sample-points", type=int, default=0,
                    help="sampled run for large workloads (c3, c4): one core state at 1 and this "
                         "many real points, extrapolated to the full grid")
    ap.add_argument("--cpu-tasks", type=int, default=24)
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
    dev = torch.device("cuda:0")
    cfg = CONFIGS[args.config]
    over = {} if args.n_real is None else {"n_real": args.n_real}
    s = system_from_config(cfg, **over)
    d = gwc.to_device(s, dev)
    n_core = s.n_core
    n_t, d_omega = 2 ** 18, 0.01 / EV_PER_HA
    n_out = 3500

    def step(precision=args.precision, wac=None):
        out = gwc.gwc_sigma_core(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                                 d["omega_imag"], d["w_imag"], d["omega_real"], d["eta"],
                                 mode=args.mode, precision=precision, wac=wac)
        e_qp = out["e_qp"].cpu().numpy()
        spectra = []
        for c in range(n_core):
            n = int(s.core_idx[c])
            A, z = gwc.gwc_spectral_cumulant(d["omega_real"][c], out["im_sigma_dec"][c],
                                             float(s.eps[n]), float(e_qp[c]), s.eta, n_t, d_omega,
                                             n_out, float(e_qp[c]) - 30 / EV_PER_HA)
            spectra.append((A, z))
        return out, spectra

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gwc.timing_enable(True)
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        last = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pi = gwc.timing_get("pi_build_f64" if args.precision == "fp64" else "pi_build_mixed")
    lu = gwc.timing_get("lu_bordered")
    gwc.timing_enable(False)

    solves = args.steps * n_core
    value = solves / elapsed
    n_tasks = residue_task_count(s.eps, s.occ, s.core_idx, s.omega_real, args.mode)
    launches = max(pi["launches"], 1)
    achieved = pi["flops"] / (pi["total_ms"] / 1e3) / 1e12 if pi["total_ms"] > 0 else 0.0
    tpt = _traffic_per_task()
    pi_tasks = args.steps * (len(s.omega_imag) * n_core + n_tasks)
    tpl = None if tpt is None else tpt * pi_tasks / launches
    peak = FP64_MFMA_PEAK_TFLOPS
    if args.precision != "fp64":
        # three 16-bit MFMA products per algorithmic multiply-add; dense 16-bit peak
        achieved, peak, tpl = 3.0 * achieved, MIXED_MFMA_PEAK_TFLOPS[args.precision], None
    roofline = {
        "bound": "mfma",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": tpl,
        "kernel": "pi_build_f64",
        "avg_launch_ms": pi["total_ms"] / launches,
        "flops_per_launch": pi["flops"] / launches,
    }
    lu_achieved = lu["flops"] / (lu["total_ms"] / 1e3) / 1e12 if lu["total_ms"] > 0 else 0.0
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {cfg.description}" + ("" if args.n_real is None else f" (n_real={args.n_real})"),
            "n_basis": cfg.n_basis, "n_occ": cfg.n_occ, "n_core": n_core, "n_aux": cfg.n_aux,
            "n_imag": cfg.n_imag, "n_real": s.omega_real.shape[1], "eta_ev": cfg.eta_ev,
            "mode": args.mode, "precision": args.precision, "residue_tasks_per_step": n_tasks,
            "cumulant_n_t": n_t, "parallelism": "single-gpu",
        },
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "per": "step (all core states)"},
        "roofline": roofline,
        "kernels": {
            "pi_build_f64": {"ms": pi["total_ms"], "launches": pi["launches"], "tflops": achieved},
            "lu_bordered": {"ms": lu["total_ms"], "launches": lu["launches"], "tflops": lu_achieved},
        },
    }
    if args.compare != "none" and args.precision == "fp64":
        step(args.compare)  # warm-up of the mixed form
        torch.cuda.synchronize()
        gwc.timing_enable(True)
        tm = time.perf_counter()
        for _ in range(args.steps):
            mixed = step(args.compare)
        torch.cuda.synchronize()
        el_m = time.perf_counter() - tm
        pim = gwc.timing_get("pi_build_mixed")
        gwc.timing_enable(False)
        ref_out, ref_spec = last
        mx_out, mx_spec = mixed
        deq = np.abs(mx_out["e_qp"].cpu().numpy() - ref_out["e_qp"].cpu().numpy())
        w_axis = None
        worst = 0.0
        for c in range(n_core):
            eq_r = float(ref_out["e_qp"][c]); eq_m = float(mx_out["e_qp"][c])
            wr = eq_r - 30 / EV_PER_HA + np.arange(n_out) * d_omega
            wm = eq_m - 30 / EV_PER_HA + np.arange(n_out) * d_omega
            pr = _satellites(wr, ref_spec[c][0].cpu().numpy(), eq_r, float(ref_spec[c][1][0]), s.eta)
            pm = _satellites(wm, mx_spec[c][0].cpu().numpy(), eq_m, float(mx_spec[c][1][0]), s.eta)
            for p in pr:
                if pm:
                    worst = max(worst, float(np.min(np.abs(np.asarray(pm) - p))))
        sc_err = None
        if args.mode == "full":
            a = ref_out["sigma_c"].cpu().numpy(); b = mx_out["sigma_c"].cpu().numpy()
            rel = np.abs((b - a)[..., 0] + 1j * (b - a)[..., 1]) / np.max(np.abs(a[..., 0] + 1j * a[..., 1]))
            sc_err = {"max": float(rel.max()), "median": float(np.median(rel))}
        pim_tf = pim["flops"] / (pim["total_ms"] / 1e3) / 1e12 if pim["total_ms"] > 0 else 0.0
        res["mixed"] = {
            "precision": args.compare,
            "value": solves / el_m,
            "ms_per_step": el_m / args.steps * 1e3,
            "speedup_vs_fp64": elapsed / el_m,
            "pi_build_ms": pim["total_ms"],
            "pi_build_algorithmic_tflops": pim_tf,
            "pi_build_mfma_tflops": 3.0 * pim_tf,
            "pi_build_mfma_peak_tflops": MIXED_MFMA_PEAK_TFLOPS[args.compare],
            "pi_build_mfma_frac": 3.0 * pim_tf / MIXED_MFMA_PEAK_TFLOPS[args.compare],
            "e_qp_max_err_mev": float(deq.max() * EV_PER_HA * 1e3),
            "satellite_max_shift_mev": worst * EV_PER_HA * 1e3,
            "sigma_c_rel_err": sc_err,
        }
    if not args.no_wac:
        wp = gwc.wac_paper_settings()
        step(args.precision, wp)  # warm-up
        torch.cuda.synchronize()
        tw = time.perf_counter()
        for _ in range(args.steps):
            wres = step(args.precision, wp)
        torch.cuda.synchronize()
        el_w = time.perf_counter() - tw
        ref_out, ref_spec = last
        w_out, w_spec = wres
        deq = np.abs(w_out["e_qp"].cpu().numpy() - ref_out["e_qp"].cpu().numpy())
        worst = 0.0
        for c in range(n_core):
            eq_r = float(ref_out["e_qp"][c]); eq_w = float(w_out["e_qp"][c])
            wr = eq_r - 30 / EV_PER_HA + np.arange(n_out) * d_omega
            ww = eq_w - 30 / EV_PER_HA + np.arange(n_out) * d_omega
            pr = _satellites(wr, ref_spec[c][0].cpu().numpy(), eq_r, float(ref_spec[c][1][0]), s.eta)
            pw = _satellites(ww, w_spec[c][0].cpu().numpy(), eq_w, float(w_spec[c][1][0]), s.eta)
            for q in pr:
                if pw:
                    worst = max(worst, float(np.min(np.abs(np.asarray(pw) - q))))
        sc_err = None
        if args.mode == "full":
            a = ref_out["sigma_c"].cpu().numpy(); b = w_out["sigma_c"].cpu().numpy()
            rel = np.abs((b - a)[..., 0] + 1j * (b - a)[..., 1]) / np.max(np.abs(a[..., 0] + 1j * a[..., 1]))
            sc_err = {"max": float(rel.max()), "median": float(np.median(rel))}
        res["wac"] = {
            "value": solves / el_w, "unit": "solves/s", "ms_per_step": el_w / args.steps * 1e3,
            "speedup_vs_cd": elapsed / el_w,
            "settings": {k: (v * EV_PER_HA if k in ("core_min", "core_max") else v) for k, v in wp.items()},
            "settings_units": "core window in eV",
            "reference_factorisations_per_step": n_core * (wp["n_core_pts"] + wp["n_val_pts"]),
            "e_qp_max_dev_from_cd_mev": float(deq.max() * EV_PER_HA * 1e3),
            "satellite_max_shift_from_cd_mev": worst * EV_PER_HA * 1e3,
            "sigma_c_rel_dev_from_cd": sc_err,
        }
    if args.mode == "full" and not args.no_decoupled:
        mode_full = args.mode
        args.mode = "decoupled"
        step()  # warm-up
        torch.cuda.synchronize()
        td = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el_d = time.perf_counter() - td
        args.mode = mode_full
        res["decoupled"] = {
            "value": solves / el_d, "unit": "solves/s", "ms_per_step": el_d / args.steps * 1e3,
            "residue_tasks_per_step": residue_task_count(s.eps, s.occ, s.core_idx, s.omega_real,
                                                             "decoupled"),
            "precision": args.precision,
        }
    if args.mode == "full" and not args.no_analytic:
        def astep():
            return gwc.gwc_sigma_analytic(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                                          d["omega_real"], d["eta"])
        astep()  # warm-up
        torch.cuda.synchronize()
        gwc.timing_enable(True)
        ta = time.perf_counter()
        for _ in range(args.steps):
            aout = astep()
        torch.cuda.synchronize()
        el_a = time.perf_counter() - ta
        ja, jp = gwc.timing_get("jacobi_apply"), gwc.timing_get("jacobi_pairs")
        gwc.timing_enable(False)
        ja_tf = ja["flops"] / (ja["total_ms"] / 1e3) / 1e12 if ja["total_ms"] > 0 else 0.0
        ref_out = last[0]
        deq = np.abs(aout["e_qp"].cpu().numpy() - ref_out["e_qp"].cpu().numpy())
        res["analytic"] = {
            "value": solves / el_a, "unit": "solves/s", "ms_per_step": el_a / args.steps * 1e3,
            "speedup_vs_cd": elapsed / el_a,
            "n_ov": int(s.M_ov.shape[1] * s.M_ov.shape[2]),
            "jacobi_sweeps": int(aout["sweeps"][0]),
            "jacobi_apply": {"ms_per_step": ja["total_ms"] / args.steps,
                             "launches_per_step": ja["launches"] / args.steps,
                             "avg_launch_ms": ja["total_ms"] / max(ja["launches"], 1),
                             "bound": "alu", "achieved": ja_tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": ja_tf / FP64_VECTOR_PEAK_TFLOPS},
            "jacobi_pairs_ms_per_step": jp["total_ms"] / args.steps,
            "e_qp_dev_from_cd_mev": float(deq.max() * EV_PER_HA * 1e3),
        }
    if args.mode == "full" and not args.no_evgw:
        from workloads import vv_block
        dvv = torch.as_tensor(vv_block(s), device=dev)

        def evstep():
            return gwc.gwc_evgw0(d["eps"], d["occ"], d["M_oo"], d["M_ov"], dvv, d["core_idx"],
                                 d["omega_real"], d["eta"])
        evstep()  # warm-up
        torch.cuda.synchronize()
        te = time.perf_counter()
        for _ in range(args.steps):
            eout = evstep()
        torch.cuda.synchronize()
        el_e = time.perf_counter() - te
        eq = eout["e_qp"].cpu().numpy()
        e1 = eout["e_first"].cpu().numpy()
        core = s.core_idx
        res["evgw0"] = {
            "value": solves / el_e, "unit": "solves/s (core states, every state iterated)",
            "ms_per_step": el_e / args.steps * 1e3,
            "states_iterated": int(s.n_basis), "outer_iterations": int(eout["outer"][0]),
            "max_newton_steps": int(eout["newton"].max()),
            "core_shift_g0w0_ev": [float(x) for x in (e1[core] - s.eps[core]) * EV_PER_HA],
            "core_shift_evgw0_ev": [float(x) for x in (eq[core] - s.eps[core]) * EV_PER_HA],
        }
    if not args.no_peaks:
        pk = measure_peaks(gwc)
        res["peaks_measured"] = pk
        if args.precision == "fp64":
            res["roofline"]["peak_measured"] = pk["fp64_mfma_tflops"]
            res["roofline"]["frac_of_measured"] = achieved / pk["fp64_mfma_tflops"]
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(s, args.mode, n_tasks / n_core, args.cpu_tasks)
    emit(res, args.jsonl)


if __name__ == "__main__":
    main()
