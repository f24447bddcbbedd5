"""Throughput of the Gamma-only LTMP2 hot path on one MI355X.

Single cells (default: the 40^3 mixed-precision cell, 160 occupied, 10
Laplace points): one step = one Laplace point tau_n of the whole path
(Green's-function tiles + chi transforms + Coulomb trace for E_d(tau_n), the
transformed-state GEMM + synthesis + Fock-like pair transforms for
E_x(tau_n)); step k evaluates tau_{k mod N_tau}, so N_tau consecutive steps
are one energy E = sum_n w_n (E_d(tau_n) + E_x(tau_n)), and the reported
value is energies/s = steps / (N_tau * seconds).  With --step-unit energy a
step is one full energy instead.  The 64-cell batch: one step = one batch
energy (cells/s).  Inputs are resident in HBM; setup (orbital synthesis,
overlap densities, quadrature fit) is outside the timed region.

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

# Sources of the pair-transform kernel (device code and its launch shapes);
# HBM traffic figures taken with rocprofv3 counters are only reported while
# these are unchanged.
PAIR_SOURCES = ("fft.hpp", "transforms.hpp", "kernels_fft.hpp", "grid_kernels.hip")
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


def cpu_baseline(spec, m, e, c, ctx_tau=None):
    """FP64 oracle on the occupied subset {HOMO} of the same cell, scaled up.

    The oracle's energy is three measured parts: orbitals on the grid (one
    inverse FFT per state), overlap densities (two forward FFTs per
    occupied-virtual pair) and, per occupied pair (i, j), the integrals
    <ij|ab>, <ab|ji> (two GEMMs over the auxiliary set) and their Laplace
    sums.  The sample times each part for i = j = HOMO with every virtual
    state; the full energy needs (N_occ + N_vir) / (1 + N_vir) times the
    orbital work, N_occ times the density work and N_occ^2 times the pair
    work.
    """
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
    no, nv = spec.n_occ, len(e) - spec.n_occ
    f_orb = (no + nv) / (1.0 + nv)
    full = (t1 - t0) * f_orb + (t2 - t1) * no + (t3 - t2) * no * no
    del P
    return {"value": 1.0 / full, "unit": "energies/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Laplace MP2 of the {spec.n}^3 cell restricted to the occupied "
                      f"subset {{HOMO}} with all {nv} virtuals, measured in three parts: "
                      f"orbitals {t1 - t0:.1f}s, overlap densities {t2 - t1:.1f}s, one occupied "
                      f"pair {t3 - t2:.1f}s; full energy = {f_orb:.4f} x orbitals + {no} x "
                      f"densities + {no}^2 x pair = {full:.0f}s",
            "sample_seconds": t3 - t0}


def cpu_whole_small():
    """The oracle's whole energy (canonical + Laplace) of the 12^3 cell, timed."""
    from synthetic import C1, make_cell
    from oracle.mp2 import Problem
    from oracle.quadrature import minimax_laplace
    m, e, c = make_cell(C1)
    t0 = time.perf_counter()
    P = Problem(C1.L, C1.n, C1.eaux, m, e, c, C1.n_occ)
    tau, w, _ = minimax_laplace(*P.x_range(), C1.n_tau)
    P.energies(tau, w)
    return {"cell": "L=8 bohr, 12^3 grid, N_occ=4, N_tau=8", "seconds": time.perf_counter() - t0}


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


def cached_cell(spec, cache_dir):
    """make_cell(spec), stored in / read back from cache_dir when given."""
    import numpy as np
    from synthetic import make_cell
    if not cache_dir:
        return make_cell(spec)
    tag = f"cell_L{spec.L}_n{spec.n}_e{spec.ecut}_s{spec.seed}_a{spec.amp}"
    path = os.path.join(cache_dir, tag + ".npz")
    if os.path.exists(path):
        with np.load(path) as z:
            return z["miller"], z["eps"], z["coeff"]
    m, e, c = make_cell(spec)
    os.makedirs(cache_dir, exist_ok=True)
    np.savez(path, miller=m, eps=e, coeff=c)
    return m, e, c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4"],
                    help="c1/c2/c3 single cells; c4 the 64-cell batch (cells/s)")
    ap.add_argument("--step-unit", default="tau", choices=["tau", "energy"],
                    help="single cells: one Laplace point per step (default) or one energy")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--quad", default="learned", choices=["plain", "learned"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB copy kernel first (scale for HBM counter runs)")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip timing the plain FP64 form beside the headline form")
    ap.add_argument("--cell-cache", default=None,
                    help="directory for the generated cell arrays (reused when present)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs the LTMP2 path on one GPU (there is no "
                                   "sharded form); run with --gpus 1"}))
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
    m, e, c = cached_cell(spec, args.cell_cache)
    log(f"cell ready ({time.time() - t:.1f}s): n_pw={m.shape[0]}")
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
    stream = torch.cuda.current_stream()
    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[args.prec]
    weights = os.path.join(ROOT, "paper_1611_06797_amd", "data", "laplace_mlp.bin")
    t = time.time()
    ctx = Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c, spec.n_occ, spec.n_tau,
                  stream=stream.cuda_stream, prec=prec,
                  mlp_weights=weights if args.quad == "learned" else None)
    torch.cuda.synchronize()
    t_setup = time.time() - t
    info = ctx.info
    nt = info.n_tau
    log(f"setup {t_setup:.1f}s: n_g={info.n_g} n_vir={info.n_vir} n_grid={info.n_grid} "
        f"device {info.device_bytes / 2**30:.1f} GiB quad_delta={info.quad_delta:.3e} "
        f"quad_flags={info.quad_flags}")
    tau_used, w_used, _ = ctx.get_quadrature()
    per_tau = np.full((nt, 2), np.nan)

    def step(k):
        if args.step_unit == "energy":
            ed, ex, pt, _ = ctx.energy()
            per_tau[:] = pt
            return
        it = k % nt
        per_tau[it, 0] = ctx.chi(it)
        per_tau[it, 1] = ctx.exchange(it)

    for k in range(args.warmup):
        t = time.time()
        step(k)
        log(f"warmup {k}: {time.time() - t:.2f}s")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
        if args.step_unit == "energy" or (k + 1) % nt == 0:
            log(f"step {k}: E_d={w_used @ per_tau[:, 0]:.10f} E_x={w_used @ per_tau[:, 1]:.10f}")
        else:
            log(f"step {k}: tau_{k % nt} E_d(tau)={per_tau[k % nt, 0]:.10f} "
                f"E_x(tau)={per_tau[k % nt, 1]:.10f}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = ctx.get_timing()
    ctx.set_timing(False)
    per_energy = nt if args.step_unit == "tau" else 1
    energies = args.steps / per_energy
    ms_step = 1000.0 * dt / args.steps
    log("stage ms per energy:", {k: round(v[0] / energies, 2) for k, v in timing.items()})
    # every tau point evaluated at least once: the energy of the headline form
    if np.isnan(per_tau).any():
        for it in range(nt):
            if np.isnan(per_tau[it, 0]):
                per_tau[it] = (ctx.chi(it), ctx.exchange(it))
    ed, ex = float(w_used @ per_tau[:, 0]), float(w_used @ per_tau[:, 1])
    qe = info.quad_delta
    ctx.close()

    # plain FP64 form on the same cell and the same quadrature, one full
    # energy timed (the equal-accuracy reference of the speed-up)
    ref = None
    if not args.no_fp64_reference and args.prec != "fp64":
        t = time.time()
        ctx64 = Context(spec.L, spec.n, spec.ecut, spec.eaux, m, e, c, spec.n_occ, spec.n_tau,
                        stream=stream.cuda_stream, prec=0, tau=tau_used, w=w_used)
        torch.cuda.synchronize()
        log(f"fp64 setup {time.time() - t:.1f}s")
        # one full energy, one Laplace point at a time (a progress line per point)
        pt64 = np.zeros((nt, 2))
        t1 = time.perf_counter()
        for it in range(nt):
            pt64[it] = (ctx64.chi(it), ctx64.exchange(it))
            log(f"fp64 point {it}: {time.perf_counter() - t1:.1f}s")
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t1
        ed64, ex64 = float(w_used @ pt64[:, 0]), float(w_used @ pt64[:, 1])
        ctx64.close()
        tol = spec.n_occ * 1e-6
        ref = {"fp64_energies_per_s": 1.0 / dt64, "fp64_seconds_per_energy": dt64,
               "speedup": (dt64 / (dt / energies)), "e_direct_fp64": ed64,
               "e_exchange_fp64": ex64, "dE_direct": ed - ed64, "dE_exchange": ex - ex64,
               "dE_direct_per_tau_max": float(np.abs(per_tau[:, 0] - pt64[:, 0]).max()),
               "dE_exchange_per_tau_max": float(np.abs(per_tau[:, 1] - pt64[:, 1]).max()),
               "tolerance": tol,
               "within_tolerance": bool(abs(ed - ed64) < tol and abs(ex - ex64) < tol)}
        log(f"plain fp64: {1.0 / dt64:.4f} energies/s; speedup {ref['speedup']:.2f}x; "
            f"dE_d {ed - ed64:.2e} dE_x {ex - ex64:.2e} (bar {tol:.1e})")

    # dominant kernel stage and its roofline
    work_of = lambda st: stage_work(info, spec.n, st, args.prec)  # noqa: E731
    roof = roofline(timing, work_of, energies, args.prec)
    stage_roofs = all_stage_rooflines(timing, work_of, energies, args.prec)
    tr = load_traffic(args.config, args.prec, roof["kernel"])
    if tr is not None:
        roof["traffic"] = tr["bytes_per_launch"]
        roof["traffic_source"] = tr["source"]

    cpu = whole = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)...")
        cpu = cpu_baseline(spec, m, e, c)
        whole = cpu_whole_small()
        cpu["whole_energy_small_cell"] = whole
        log(f"cpu baseline: {cpu['sample']}")
    unit_txt = (f"one step = one Laplace point (direct + exchange), {nt} steps = one energy"
                if args.step_unit == "tau" else "one step = one energy")
    out = {"metric": "LTMP2 energies/sec", "value": energies / dt, "unit": "energies/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32"}[args.prec],
           "data": "synthetic",
           "config": {"workload": f"gamma-only LTMP2 cell L={spec.L} bohr, {spec.n}^3 grid, "
                                  f"E_cut={spec.ecut} Ha (n_pw={info.n_pw}), "
                                  f"E_aux={spec.eaux} Ha (n_g={info.n_g}), "
                                  f"n_occ={spec.n_occ}, n_tau={spec.n_tau}, seed={spec.seed}; "
                                  + unit_txt,
                      "precision": args.prec,
                      "quadrature": "learned+3 Remez (certified)" if info.quad_flags & 1
                      else "plain minimax",
                      "transform_grid": info.n_grid},
           "energy": {"e_direct": ed, "e_exchange": ex, "quad_delta": qe,
                      "per_tau": per_tau.tolist()},
           "stage_ms_per_energy": {k: v[0] / energies for k, v in timing.items()},
           "setup_s": t_setup, "fp64_reference": ref,
           "roofline": roof, "stage_roofline": stage_roofs, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
