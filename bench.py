"""Throughput of the Gamma-only LTMP2 hot path on one MI355X.

One step = one full energy E = E_d + E_x of one cell over all Laplace points
(every kernel of the path: Green's-function tiles + chi transforms + Coulomb
trace, and the transformed-state GEMM + synthesis + Fock-like pair
transforms), inputs resident in HBM.  Setup (orbital synthesis, overlap
densities, quadrature fit) is outside the timed region.

Prints one JSON line (rank 0).  Extra objects:
  roofline      dominant kernel stage: algorithmic work per launch divided
                by its mean event-timed duration, against the MI355X peak
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same cell,
                scaled to energies / s
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # FP64 vector and matrix, FLOP/s
PEAK_FP32 = 157.3e12     # FP32 vector and matrix, FLOP/s
PEAK_BF16 = 2.5e15       # BF16 dense matrix, FLOP/s
PEAK_HBM = 8.0e12        # bytes/s

# Sources of the pair-transform kernel; HBM traffic figures taken with
# rocprofv3 counters are only reported while these are unchanged.
PAIR_SOURCES = ("fft.hpp", "transforms.hpp", "kernels_fft.hpp", "grid_kernels.hip", "ltmp2.hip")
COPY_PROBE_BYTES = 1 << 30


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_06797_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(config, prec, kernel):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size),
    or None when no summary matches the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_{prec}_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json:"):
                d = json.loads(line.split(":", 1)[1])
                if d.get("kernel_hash") == kernel_hash():
                    return d
    return None


def copy_probe():
    """One plain copy of COPY_PROBE_BYTES (read + write) for counter scaling."""
    import torch
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    log(f"copy probe: {COPY_PROBE_BYTES} bytes read + written (kernel: elementwise mul)")
    del x, y


def workload(name):
    from synthetic import C1, C2, C3
    return {"c1": C1, "c2": C2, "c3": C3}[name]


def stage_work(info, n, stage, prec="fp64"):
    """Algorithmic (flops, bytes) of one energy for a timing stage (N_r: the
    internal transform grid)."""
    nr, ng, nh, no, nv, npw, nt = (info.n_r, info.n_g, info.n_h, info.n_occ, info.n_vir,
                                   info.n_pw, info.n_tau)
    es = 8 if prec == "fp64" else 4
    lg = math.log2(nr)
    if stage == "chi_tiles":      # symmetric real GEMMs, upper triangle only
        return nt * nr * nr * (no + nv) * 1.0, None
    if stage == "w_gemm":         # complex C x real basis, G' in H
        return nt * 4.0 * nh * no * nv * npw, None
    if stage == "pair":           # N_o^2 complex 3-D FFTs per outer G' (H and -H)
        return nt * ng * no * no * 5.0 * nr * lg / 2.0 * 1.0, None
    if stage == "chi_rows":       # read the real chi rows once
        return None, nt * es * nr * nr
    if stage == "chi_cols":       # read chi(r, G') once
        return None, nt * 2 * es * nh * nr
    if stage == "w_synth":
        return nt * nh * no * 5.0 * nr * lg, None
    return None, None


def stage_roofline(stage, ms_tot, launches, steps, prec, work):
    """Achieved rate of one stage against its MI355X peak.  GEMM stages are
    matrix-core bound: in the BF16x3 form each algorithmic flop costs three
    BF16 MFMA flops, so mfma_frac = 3 x achieved / 2.5 PFLOP/s."""
    flops, byts = work
    per_launch_s = ms_tot / 1000.0 / max(launches, 1)
    if per_launch_s <= 0:
        return None
    if flops is not None:
        ach = flops * steps / max(launches, 1) / per_launch_s
        if stage in ("pair", "w_synth"):
            peak, bound = (PEAK_FP64 if prec == "fp64" else PEAK_FP32), "alu"
            roof = {"bound": bound, "achieved": ach / 1e12, "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": ach / peak}
        else:
            peak = {"fp64": PEAK_FP64, "fp32": PEAK_FP32, "bf16x3": PEAK_BF16}[prec]
            mult = 3.0 if prec == "bf16x3" else 1.0
            roof = {"bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": ach / peak, "mfma_frac": mult * ach / peak}
    else:
        ach = byts * steps / max(launches, 1) / per_launch_s
        roof = {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": ach / PEAK_HBM}
    roof["launches_per_step"] = launches / steps
    roof["mean_launch_ms"] = 1000.0 * per_launch_s
    return roof


def cpu_baseline(spec, m, e, c, budget_s=25.0):
    """FP64 oracle on one occupied orbital of the same cell, scaled up.

    Sample: Laplace MP2 restricted to the occupied subset {HOMO}: overlap
    densities of that orbital with every virtual (both orderings) and the
    one (i, j) pair's integrals and Laplace sums.  The full energy needs
    N_occ times the density work and N_occ^2 times the pair work.
    """
    import numpy as np
    from oracle.mp2 import Problem
    from oracle.quadrature import minimax_laplace
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    P = Problem(spec.L, spec.n, spec.eaux, m, e, c, spec.n_occ, occ=[spec.n_occ - 1])
    tau, w, _ = minimax_laplace(*P.x_range(), spec.n_tau)
    t0 = time.perf_counter()
    _ = P.psi_o, P.psi_v
    t1 = time.perf_counter()
    _ = P.n_ov, P.n_vo
    t2 = time.perf_counter()
    P.energies(tau, w)
    t3 = time.perf_counter()
    no = spec.n_occ
    full = (t1 - t0) * (spec.n_occ + 0) / 1.0 + (t2 - t1) * no + (t3 - t2) * no * no
    return {"value": 1.0 / full, "unit": "energies/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle LT-MP2 for occupied subset {{HOMO}} of the {spec.n}^3 cell "
                      f"(orbitals {t1 - t0:.1f}s, pair densities {t2 - t1:.1f}s, "
                      f"one pair {t3 - t2:.1f}s); full energy = orbitals + "
                      f"{no} x densities + {no}^2 x pair = {full:.0f}s"}


def roofline(timing, work_of, steps, prec):
    """Roofline entry of the dominant stage: work_of(stage) -> (flops, bytes) per step."""
    dom = max(timing, key=lambda k: timing[k][0])
    ms_tot, launches = timing[dom]
    roof = stage_roofline(dom, ms_tot, launches, steps, prec, work_of(dom))
    roof = {"bound": roof.pop("bound"), "achieved": roof.pop("achieved"), "peak": roof.pop("peak"),
            "unit": roof.pop("unit"), "frac": roof.pop("frac"), "traffic": None, **roof}
    roof["kernel"] = dom
    return roof


def all_stage_rooflines(timing, work_of, steps, prec):
    out = {}
    for st, (ms_tot, launches) in timing.items():
        w = work_of(st)
        if launches and (w[0] is not None or w[1] is not None):
            out[st] = stage_roofline(st, ms_tot, launches, steps, prec, w)
    return out


def bench_batch(args):
    """64 independent cells of uneven size per step (graph replay), cells/s."""
    import numpy as np
    import torch
    from synthetic import batch_specs, make_cell
    from paper_1611_06797_amd import Batch

    specs = batch_specs()
    t = time.time()
    data = [make_cell(s) for s in specs]
    log(f"{len(specs)} cells ready ({time.time() - t:.1f}s)")
    torch.cuda.set_device(0)
    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[args.prec]
    weights = os.path.join(ROOT, "paper_1611_06797_amd", "data", "laplace_mlp.bin")
    cells = [dict(L=s.L, n_fft=s.n, ecut=s.ecut, eaux=s.eaux, miller=m, eps=e, coeff=c,
                  n_occ=s.n_occ, n_tau=s.n_tau) for s, (m, e, c) in zip(specs, data)]
    t = time.time()
    b = Batch(cells, prec=prec, mlp_weights=weights if args.quad == "learned" else None,
              stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    t_setup = time.time() - t
    st = b.stats()
    log(f"setup {t_setup:.1f}s: {st.n_groups} groups, device {st.device_bytes / 2**30:.1f} GiB")
    # first call tunes and runs eagerly, the second captures the graph
    warm = max(args.warmup, 2)
    for k in range(warm):
        t = time.time()
        b.energy()
        log(f"warmup {k}: {time.time() - t:.2f}s graph_ready={b.stats().graph_ready}")
    groups = [b.group(g) for g in range(st.n_groups)]
    log("groups:", groups)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ed, ex = b.energy()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{args.steps} steps: {dt:.3f}s; sum E = {float(np.sum(ed + ex)):.10f}")
    # one more (eager, event-timed) evaluation for the per-stage roofline
    b.set_timing(True)
    ed_t, ex_t = b.energy()
    timing = b.get_timing()
    b.set_timing(False)
    log("stage ms (eager timed pass):", {k: round(v[0], 2) for k, v in timing.items()})
    infos = [b.cell_info(k) for k in range(len(specs))]
    b.close()

    def work_of(stage):
        fl, by = 0.0, 0.0
        for inf, s in zip(infos, specs):
            f1, b1 = stage_work(inf, s.n, stage, args.prec)
            fl = fl + f1 if f1 is not None else None
            by = by + b1 if b1 is not None else None
        return (fl if fl else None), (by if by else None)

    roof = roofline(timing, work_of, 1, args.prec)
    stage_roofs = all_stage_rooflines(timing, work_of, 1, args.prec)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)...")
        cpu = cpu_baseline_batch(specs, data, infos)
    out = {"metric": "LTMP2 energies/sec", "value": len(specs) * args.steps / dt,
           "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": warm,
           "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32"}[args.prec],
           "data": "synthetic",
           "config": {"workload": f"{len(specs)} independent gamma-only LTMP2 cells, "
                                  "L~U[6,14] bohr, grids 15-30, E_cut=7.5 Ha, E_aux=5 Ha, "
                                  "N_occ=round(8+5(L-6)), N_tau~U{6..12}, batch seed 0",
                      "precision": args.prec,
                      "quadrature": "learned+3 Remez" if args.quad == "learned" else "plain",
                      "groups": groups},
           "energy": {"sum_e_direct": float(np.sum(ed)), "sum_e_exchange": float(np.sum(ex)),
                      "timed_pass_max_diff": float(max(np.abs(ed_t - ed).max(),
                                                       np.abs(ex_t - ex).max()))},
           "stage_ms_eager_pass": {k: v[0] for k, v in timing.items()},
           "setup_s": t_setup, "roofline": roof, "stage_roofline": stage_roofs,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(specs, data, infos):
    """Oracle time per cell on three sampled cells, spread over the batch by
    the pair-transform operation count (which dominates the oracle too)."""
    order = sorted(range(len(specs)), key=lambda k: specs[k].L)
    picks = [order[0], order[len(order) // 2], order[-1]]
    ratios, notes = [], []
    for k in picks:
        r = cpu_baseline(specs[k], *data[k])
        t_full = 1.0 / r["value"]
        w = stage_work(infos[k], specs[k].n, "pair")[0]
        ratios.append(t_full / w)
        notes.append(f"cell {k} (n={specs[k].n}, N_occ={specs[k].n_occ}): {t_full:.0f}s")
    c = sum(ratios) / len(ratios)
    total = c * sum(stage_work(inf, s.n, "pair")[0] for inf, s in zip(infos, specs))
    return {"value": len(specs) / total, "unit": "cells/s", "cores": r["cores"], "kind": "oracle",
            "sample": "oracle full-energy estimates (occupied subset {HOMO}, scaled) of cells "
                      + ", ".join(notes) + f"; batch total {total:.0f}s by pair operation count"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4"],
                    help="c1/c2/c3 single cells; c4 the 64-cell batch (cells/s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--quad", default="learned", choices=["plain", "learned"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB copy kernel first (scale for HBM counter runs)")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip timing the plain FP64 form beside the headline form")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the LTMP2 path runs on one GPU (no sharded form is built); --gpus must be 1"}))
        sys.exit(2)

    if args.config == "c4":
        return bench_batch(args)

    import numpy as np
    import torch
    from synthetic import make_cell
    from paper_1611_06797_amd import Context

    spec = workload(args.config)
    log("workload", spec)
    t = time.time()
    m, e, c = make_cell(spec)
    log(f"cell ready ({time.time() - t:.1f}s): n_pw={m.shape[0]}")
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
    stream = torch.cuda.current_stream()
    t = time.time()
    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[args.prec]
    weights = os.path.join(ROOT, "paper_1611_06797_amd", "data", "laplace_mlp.bin")
    t = time.time()
    ctx = Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c, spec.n_occ, spec.n_tau,
                  stream=stream.cuda_stream, prec=prec,
                  mlp_weights=weights if args.quad == "learned" else None)
    torch.cuda.synchronize()
    t_setup = time.time() - t
    info = ctx.info
    log(f"setup {t_setup:.1f}s: n_g={info.n_g} n_vir={info.n_vir} "
        f"device {info.device_bytes / 2**30:.1f} GiB quad_delta={info.quad_delta:.3e} "
        f"quad_flags={info.quad_flags}")
    for k in range(args.warmup):
        t = time.time()
        ctx.energy()
        log(f"warmup {k}: {time.time() - t:.2f}s")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ed, ex, pt, qe = ctx.energy()
        log(f"step {k}: E_d={ed:.10f} E_x={ex:.10f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = ctx.get_timing()
    ms_step = 1000.0 * dt / args.steps
    log("stage ms per step:", {k: round(v[0] / args.steps, 2) for k, v in timing.items()})
    tau_used, w_used, _ = ctx.get_quadrature()
    ctx.close()

    # plain FP64 form on the same cell and the same quadrature (equal accuracy reference)
    ref = None
    if not args.no_fp64_reference and args.prec != "fp64":
        ctx64 = Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c, spec.n_occ, spec.n_tau,
                        stream=stream.cuda_stream, prec=0, tau=tau_used, w=w_used)
        ctx64.energy()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            ed64, ex64, _, _ = ctx64.energy()
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t1
        ctx64.close()
        ref = {"fp64_energies_per_s": args.steps / dt64, "speedup": dt64 / dt,
               "dE_direct": ed - ed64, "dE_exchange": ex - ex64,
               "tolerance": spec.n_occ * 1e-6}
        log(f"plain fp64: {args.steps / dt64:.4f} energies/s; speedup {dt64 / dt:.2f}x; "
            f"dE_d {ed - ed64:.2e} dE_x {ex - ex64:.2e}")

    # dominant kernel stage and its roofline
    work_of = lambda st: stage_work(info, spec.n, st, args.prec)  # noqa: E731
    roof = roofline(timing, work_of, args.steps, args.prec)
    stage_roofs = all_stage_rooflines(timing, work_of, args.steps, args.prec)
    tr = load_traffic(args.config, args.prec, roof["kernel"])
    if tr is not None:
        roof["traffic"] = tr["bytes_per_launch"]
        roof["traffic_source"] = tr["source"]

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)...")
        cpu = cpu_baseline(spec, m, e, c)
    out = {"metric": "LTMP2 energies/sec", "value": args.steps / dt, "unit": "energies/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32"}[args.prec],
           "data": "synthetic",
           "config": {"workload": f"gamma-only LTMP2 cell L={spec.L} bohr, {spec.n}^3 grid, "
                                  f"E_cut={spec.ecut} Ha (n_pw={info.n_pw}), "
                                  f"E_aux={spec.eaux} Ha (n_g={info.n_g}), "
                                  f"n_occ={spec.n_occ}, n_tau={spec.n_tau}, seed={spec.seed}",
                      "precision": args.prec,
                      "quadrature": "learned+3 Remez (certified)" if info.quad_flags & 1
                      else "plain minimax"},
           "energy": {"e_direct": ed, "e_exchange": ex, "quad_delta": qe},
           "stage_ms_per_step": {k: v[0] / args.steps for k, v in timing.items()},
           "setup_s": t_setup, "fp64_reference": ref,
           "roofline": roof, "stage_roofline": stage_roofs, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
