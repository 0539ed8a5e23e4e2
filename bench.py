"""Benchmark of the U(1)-symmetric MPS gate path on one MI355X.

Workload: the linear-optics boson-sampling circuit with L = 32 modes,
16 single photons in modes 0-15, local dimension d = 4, 32 brickwork layers
of seeded beam splitters (496 gates), chi_max = 512, discarded-weight cutoff
1e-12, complex128 arithmetic.  One step is the whole circuit from the Fock
product state (every gate is one two-site update: Theta formation, gate,
per-sector Jacobi SVD, cut, update); the gates of a layer go through the
device together.  The state for every step is created before the timed
region (inputs resident in HBM).

Printed: one JSON line (stdout) with gate applies/s, the roofline of the
dominant kernel (HIP events on the library's stream over the timed region)
and the CPU oracle timed on saturated gates of the same shape (the whole
circuit's oracle time estimated from them); under "forms", the precision form
against the plain one on a saturated chi=2048 state (sector products on the
matrix cores, gate applies/s, their difference), the batching form (several
circuits per launch: copies of this circuit with other seeds, and the 512
circuits of the mixed-size workload) and the serving form (Poisson arrivals,
continuous batching, p50/p99 latency from arrival to result, unfinished
requests censored); under "tebd", Hamiltonian time evolution with dense
Trotter gates (an XXZ chain and a Bose-Hubbard chain with the particle number
as the charge, a transverse-field Ising chain with Z_2 and a clock chain with
Z_3 charges; 64 sites each, quenched from product states).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 2.4 GHz x 128 FP64 flop/clk

# HBM bytes per launch of the dominant Jacobi step kernel on this workload
# (jacobi_block_step8: the circuit's updates take blocks of 8), from two
# rocprofv3 --pmc runs of `bench.py --steps 1 --warmup 0 --no-cpu-baseline
# --batch-copies 0 --mix-circuits 0 --chi2048-layers 0 --serve-seconds 0
# --samples 4096 --no-tebd`
# (FETCH_SIZE, WRITE_SIZE; mean over the 37824 launches) scaled by the same
# counters on a plain 256 MiB copy (`bench.py --copy-probe`: FETCH_SIZE reads
# 131085.2 KiB and WRITE_SIZE 262144 KiB per copy, so reads scale by 1.99980
# and writes by 1).  Valid only for the Jacobi source (csrc/jacobi.hip), the
# inner sweep count per visit (kMaxInnerSweeps in csrc/runtime.cpp) and the
# block size it was taken on.
MEASURED_TRAFFIC = {
    "kernels_sha256": "12dacabb38dad06b357254205d6132dbed451e54da57798eafcafd2e5fcb4414",
    "max_inner": 1,
    "jacobi_block": 8,
    "fetch_kib": 17616.5, "write_kib": 23400.7,
    "fetch_scale": 262144.0 / 131085.2, "write_scale": 1.0,
}


def measured_traffic(block: int):
    """Bytes per launch from the counters, or None once the kernel source, its
    inner sweep count or the Jacobi block size differs from the counted run."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2303_11409_amd", "csrc")
    try:
        with open(os.path.join(csrc, "jacobi.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        with open(os.path.join(csrc, "runtime.cpp")) as f:
            inner = re.search(r"kMaxInnerSweeps = (\d+);", f.read())
    except OSError:
        return None
    t = MEASURED_TRAFFIC
    if sha != t["kernels_sha256"] or inner is None or int(inner.group(1)) != t["max_inner"]:
        return None
    if block != t["jacobi_block"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0
METRIC = "gate applies/s + sector-GEMM TFLOP/s at χ=2048 vs plain; p50/p99 latency"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_info() -> dict:
    """Host CPU model, the cores this process may run on and the BLAS threads."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = affinity
    return {"cpu_model": model, "affinity_cores": affinity, "blas_threads": int(blas)}


def cpu_baseline(cfg, shapes, budget: float = 60.0):
    """The oracle (dense TEBD, NumPy/LAPACK, complex128) timed per gate on
    saturated states of the same shape as the benchmark circuit's bonds, and
    the whole circuit's oracle time estimated from them.

    A gate of the oracle costs one dense (chi_s d) x (d chi_{s+2}) SVD plus
    BLAS-3 products; its time is measured on a synthetic saturated state
    (L=32, N=16, d=4; circuits.synthetic_state at chi = 64, 128, 256, 512,
    imported by Eq. (E2)) at the central gate of the circuit's first layer.
    ``shapes`` lists the (chi_s, chi_{s+2}) of every gate of the circuit (from
    the GPU run); each gate is charged the measured time of the sample with
    the nearest m n min(m, n) (m, n the dense matrix's sides), scaled by that
    product.  A sample predicted to exceed ``budget`` seconds is skipped (the
    largest one measured then stands for the larger gates).  Also reported: the
    saturated rate at the largest sample alone, and one chi=128 gate on one
    thread beside the same gate on all BLAS threads."""
    import numpy as np
    from oracle import dense_mps
    from workloads import circuits
    info = cpu_info()
    L, N, d = cfg["L"], sum(cfg["occupation"]), cfg["d"]
    gate = {g.site: g for g in circuits.brickwork_layers(L, 1, 2)[0]}[L // 2 - 2]
    samples = []
    t_all = time.perf_counter()
    for chi in (64, 128, 256, 512):
        # a doubling of chi costs about 8x: stop before a sample would overrun the budget
        if samples and samples[-1]["seconds"] * 8.0 > budget:
            break
        ch, gam, lam = circuits.synthetic_state(L, N, d, chi, seed=31)
        m = dense_mps.DenseMPS.from_vidal(d, N, ch, gam, lam, chi_max=chi, cutoff=cfg["cutoff"])
        del gam
        s = gate.site
        dm, dn = m.t[s].shape[0] * d, d * m.t[s + 1].shape[2]
        t0 = time.perf_counter()
        m.apply_gate(s, gate.u)
        samples.append({"chi": chi, "m": dm, "n": dn, "seconds": time.perf_counter() - t0})
    single = None
    try:
        from threadpoolctl import threadpool_limits
        ch, gam, lam = circuits.synthetic_state(L, N, d, 128, seed=31)
        m = dense_mps.DenseMPS.from_vidal(d, N, ch, gam, lam, chi_max=128, cutoff=cfg["cutoff"])
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            m.apply_gate(gate.site, gate.u)
            t1 = time.perf_counter() - t0
        single = {"chi": 128, "seconds_one_thread": t1,
                  "seconds_all_threads": next(x["seconds"] for x in samples if x["chi"] == 128)}
    except Exception:
        pass
    sampled = time.perf_counter() - t_all

    def work(m_, n_):
        return float(m_) * n_ * min(m_, n_)

    logw = np.array([np.log(work(x["m"], x["n"])) for x in samples])
    est = 0.0
    for cl, cr in shapes:
        w = work(cl * d, d * cr)
        k = int(np.argmin(np.abs(logw - np.log(w))))
        est += samples[k]["seconds"] * w / work(samples[k]["m"], samples[k]["n"])
    sat = samples[-1]
    return {"value": len(shapes) / est, "unit": "gate applies/s", "cores": info["blas_threads"],
            "kind": "oracle",
            "sample": f"one gate (central site, layer 1, seed 2) on each saturated synthetic state of the "
                      f"benchmark's shape (L=32, N=16, d=4; chi = {', '.join(str(x['chi']) for x in samples)}): dense (chi d) x (d chi) "
                      f"complex128 SVD per gate, {sampled:.1f} s in total; the circuit's {len(shapes)} gates "
                      f"charged by their (chi_s d) x (d chi_s+2) shapes from the GPU run, nearest sample "
                      f"scaled by m n min(m, n): estimated {est:.0f} s for the whole circuit",
            "circuit_seconds_estimate": est,
            "saturated_gate_applies_per_s": {"chi": sat["chi"], "value": 1.0 / sat["seconds"]},
            "samples": samples, "single_thread": single, **info}


def sample_flops(m, pats):
    """Algorithmic flops of the sampler for the drawn patterns (see the JSON note)."""
    L, d = m.L, m.d
    blocks = [m.bond_sectors(b) for b in range(L + 1)]
    tot = 0
    for p in pats.tolist():
        c = 0
        for s in range(L - 1, -1, -1):
            nc = blocks[s + 1].get(c, 0)
            for i in range(d):
                nr = blocks[s].get(c + i, 0)
                if nr:
                    tot += 8 * nr * nc + 8 * nr * nr
            nr = blocks[s].get(c + p[s], 0)
            tot += 8 * nr * nc
            c += p[s]
    return float(tot)


def run_tebd(MPS, dev, cfg):
    """One Hamiltonian time evolution (dense Trotter gates, one layer per call)."""
    layers = [([g.site for g in lay], [g.g4 for g in lay]) for lay in cfg["layers"]]
    ng = sum(len(s) for s, _ in layers)
    m = MPS(cfg["occupation"], cfg["d"], chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], device=dev,
            modulus=cfg.get("modulus", 0))
    m.sync()
    t0 = time.perf_counter()
    disc = 0.0
    for sites, gs in layers:
        disc += float(sum(m.apply_layer_dense(sites, gs)))
    m.sync()
    el = time.perf_counter() - t0
    out = {"gates": ng, "layers": len(layers), "seconds": el, "value": ng / el, "unit": "gate applies/s",
           "norm_loss": 1.0 - m.norm2(), "discarded_total": disc, "max_bond_dim": max(m.bond_dims())}
    m.close()
    return out


def copy_probe(torch) -> int:
    """Three launches of a plain copy of a known size: FETCH_SIZE and WRITE_SIZE of
    these dispatches, divided by the bytes moved, scale the counters read on the
    Jacobi kernel to HBM bytes."""
    n = 1 << 25                                   # 2^25 float64 = 256 MiB
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ok = bool(torch.equal(dst, src))
    print(json.dumps({"copy_probe": {"bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                                     "launches": 3, "ok": ok}}), flush=True)
    return 0 if ok else 1


def run_batched(cfgs, MPS, apply_batch, dev, keep_first=False, sweep_graph=1, jacobi_block=0):
    """The batching form: layer k of every circuit in one mps_apply_batch call,
    each Jacobi sweep's step launches replayed from a captured HIP graph.
    States are created before the timed region.  Returns (gates, seconds, first
    state if keep_first, host planning seconds)."""
    import torch
    states = [MPS(c["occupation"], c["d"], chi_max=c["chi_max"], cutoff=c["cutoff"], device=dev,
                  sweep_graph=sweep_graph, jacobi_block=jacobi_block) for c in cfgs]
    lays = []
    depth = max(len(c["layers"]) for c in cfgs)
    for k in range(depth):
        row = []
        for c in cfgs:
            lay = c["layers"][k] if k < len(c["layers"]) else []
            row.append(([g.site for g in lay], [g.u for g in lay]))
        lays.append(row)
    gates = sum(len(s) for row in lays for s, _ in row)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for row in lays:
        apply_batch(states, row)
    for m in states:
        m.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan_s = sum(m.stats()["host_plan_ms"] for m in states) / 1e3
    first = states[0] if keep_first else None
    for m in states[1 if keep_first else 0:]:
        m.close()
    return gates, el, first, plan_s


def run_serving(args, rate, window, circuits):
    """One serving window: Poisson arrivals at `rate` of the serving mix, continuous
    batching, results read out at completion; no drain after the window (requests
    unfinished at its end are reported as censored)."""
    import numpy as np
    from paper_2303_11409_amd import serving
    n = int(rate * window * 1.2) + 8
    specs = circuits.serving_mix_specs(n, seed=5)
    reqs = serving.poisson_requests(specs, rate=rate, seed=5, build=circuits.config_from_spec, n_patterns=16)
    import torch
    from paper_2303_11409_amd import TorchDevice
    # two lanes: the large circuits (chi_max >= 1024) on one stream, the rest on another
    devs = [TorchDevice(stream=torch.cuda.Stream()) for _ in range(2)]
    srv = serving.Server(int(args.serve_budget_gib * 2**30), max_active=[args.serve_max_large, args.serve_max_active],
                         devices=devs,
                         lane_of=lambda sp: 0 if sp["chi_max"] >= 1024 else 1, state_opts={"sweep_graph": 1})
    rep = srv.run(reqs, until=window)
    lat = rep.latencies()
    cens = rep.censored_latencies()
    arrived = sum(1 for r in reqs if r.arrival < rep.seconds)
    done_gates = sum(len(r.cfg["gates"]) for r in rep.completed)

    def gates_of(sp):
        return sp["depth"] * (sp["L"] // 2) - (sp["depth"] // 2) * (1 - sp["L"] % 2)

    mean_gates = float(np.mean([gates_of(sp) for sp in specs]))
    executed = rep.gates / rep.seconds
    return {
        "arrival_rate": rate, "window_s": rep.seconds, "arrived": arrived, "completed": len(rep.completed),
        "completed_over_arrived": len(rep.completed) / max(arrived, 1),
        "pending": rep.pending, "refused": len(rep.refused), "iterations": rep.iterations,
        "peak_active": rep.peak_active, "peak_admitted_gib": rep.peak_bytes / 2**30,
        "gate_applies_per_s": executed,
        "completed_gate_applies_per_s": done_gates / rep.seconds,
        "requests_per_s": len(rep.completed) / rep.seconds,
        # every arrival: unfinished requests count as censored at the window's end
        # (arrival to end), so these percentiles are lower bounds over all arrivals
        "latency_all_arrivals_censored_s": {"p50": percentile(list(cens), 50), "p99": percentile(list(cens), 99),
                                            "censored": rep.pending},
        "latency_completed_s": {"p50": percentile(list(lat), 50), "p99": percentile(list(lat), 99),
                                "max": float(lat.max()) if lat.size else None},
        "offered_gate_applies_per_s": rate * mean_gates,
        # arrivals per second the measured gate rate could sustain for this mix
        "sustainable_arrival_rate": executed / mean_gates,
    }


BF16_DENSE_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix-core peak


def precision_chi2048(MPS, dev, circuits, layers: int):
    """The precision workload's saturated regime in both forms: a synthetic
    chi=2048 state (L=64, N=32, d=4; bond charges Gaussian around N(L-k)/L,
    normalised to 2048 and clipped by the Fock bound; complex Gaussian Gamma on
    the allowed blocks; lambda 1..1e-4; seed 30) through `layers` brickwork
    layers of the 64-mode circuit's angles (seed 3), chi_max = 2048, cutoff
    1e-12, once in the plain complex128 form and once with the split-BF16
    sector products.  Reports gate applies/s per form, the sector products
    (plain FP64 against split BF16 on the matrix cores), the Jacobi's rate
    against the FP64 peak, and the forms' difference on 1024 amplitudes drawn
    along the state's charge paths (seed 107)."""
    import numpy as np
    import torch
    from paper_2303_11409_amd.binding import FORM_PLAIN_C128, FORM_SPLIT_BF16X3
    ch, gam, lam = circuits.synthetic_state(64, 32, 4, 2048, seed=30)
    lays = circuits.brickwork_layers(64, layers, 3)
    pats = circuits.charge_path_patterns(ch, 4, 1024, 107)
    ngates = sum(len(l) for l in lays)
    res, amps = {}, {}
    for form in (FORM_PLAIN_C128, FORM_SPLIT_BF16X3):
        m = MPS.from_vidal(4, 32, ch, gam, lam, chi_max=2048, cutoff=1e-12, form=form, device=dev)
        m.set_timing(True)
        m.reset_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lay in lays:
            m.apply_layer([g.site for g in lay], [g.u for g in lay])
        m.sync()
        el = time.perf_counter() - t0
        res[form] = (m.stats(), el)
        amps[form] = m.amplitudes(pats)
        m.close()
    sp, tp = res[FORM_PLAIN_C128]
    ss, ts = res[FORM_SPLIT_BF16X3]
    flops = sp["theta_flops"]
    split_ms = ss["split_ms"] + ss["gemm_ms"] + ss["theta_ms"]
    a, r = amps[FORM_SPLIT_BF16X3], amps[FORM_PLAIN_C128]
    # every output tile shape of the products forced in turn on the first layer
    shapes = {}
    lay0 = lays[0]
    for v, name in enumerate(("64x64", "32x64", "64x32", "32x32")):
        m = MPS.from_vidal(4, 32, ch, gam, lam, chi_max=2048, cutoff=1e-12, form=FORM_SPLIT_BF16X3, device=dev,
                           tile_tuning=2 + v)
        m.set_timing(True)
        m.apply_layer([g.site for g in lay0], [g.u for g in lay0])
        m.sync()
        st = m.stats()
        shapes[name] = {"gemm_ms": st["gemm_ms"], "mfma_executed_flops": st["gemm_mfma_flops"],
                        "frac_of_bf16_peak": st["gemm_mfma_flops"] / st["gemm_ms"] / 1e9 / BF16_DENSE_PEAK_TFLOPS}
        m.close()
    jac = {}
    for key, (st, _) in (("plain", res[FORM_PLAIN_C128]), ("split_bf16x3", res[FORM_SPLIT_BF16X3])):
        jl = max(st["jacobi_launches"], 1)
        jac[key] = {"ms": st["jacobi_ms"], "aux_ms": st["jacobi_aux_ms"],
                    "tflops": st["jacobi_flops"] / max(st["jacobi_ms"], 1e-9) / 1e9,
                    "frac_of_fp64_peak": st["jacobi_flops"] / max(st["jacobi_ms"], 1e-9) / 1e9
                    / FP64_VECTOR_PEAK_TFLOPS,
                    "launches": jl, "sweeps_per_sector": st["sweeps"] / max(st["sectors"], 1)}
    return {
        "workload": f"{layers} brickwork layers ({ngates} gates; circuit seed 3) of the 64-mode precision circuit "
                    "applied to a synthetic saturated chi=2048 state: L=64, N=32, d=4, bond k charges Gaussian "
                    "(width 3) around N(L-k)/L normalised to 2048 and clipped by the Fock bound, complex Gaussian "
                    "Gamma on the allowed blocks, lambda 1..1e-4 (seed 30); chi_max=2048, cutoff 1e-12",
        "gates": ngates,
        "gate_applies_per_s": {"plain": ngates / tp, "split_bf16x3": ngates / ts},
        "seconds": {"plain": tp, "split_bf16x3": ts},
        "algorithmic_flops": flops,
        "plain": {"kernel": "theta_kernel (complex128 products and gate mix fused, FP64 FMA)",
                  "ms": sp["theta_ms"], "tflops": flops / sp["theta_ms"] / 1e9,
                  "frac_of_fp64_peak": flops / sp["theta_ms"] / 1e9 / FP64_VECTOR_PEAK_TFLOPS},
        "split_bf16x3": {
            "kernel": "split_planes_kernel (BF16 planes, 3 parts per value) + split_gemm_kernel "
                      "(v_mfma_f32_32x32x16_bf16, 8 part products per real product, FP32 accumulation per "
                      "32-wide k chunk, chunks summed in FP64) + theta_mix_kernel (FP64 gate mix)",
            "gemm_ms": ss["gemm_ms"], "mix_ms": ss["theta_ms"],
            "tflops_algorithmic": flops / ss["gemm_ms"] / 1e9,
            "mfma_executed_flops": ss["gemm_mfma_flops"],
            "mfma_executed_tflops": ss["gemm_mfma_flops"] / ss["gemm_ms"] / 1e9,
            "frac_of_bf16_peak": ss["gemm_mfma_flops"] / ss["gemm_ms"] / 1e9 / BF16_DENSE_PEAK_TFLOPS,
            # without tile padding: 8 BF16 products per real product of the algorithmic work
            "mfma_useful_tflops": 8.0 * flops / ss["gemm_ms"] / 1e9,
            "frac_of_bf16_peak_useful": 8.0 * flops / ss["gemm_ms"] / 1e9 / BF16_DENSE_PEAK_TFLOPS,
            "split_ms": ss["split_ms"],
            "theta_speedup_vs_plain": sp["theta_ms"] / split_ms,
            "tile_chosen": ("64x64", "32x64", "64x32", "32x32")[ss["gemm_variant"]],
            "tile_tunings": ss["tile_tunings"],
            "tile_shapes_first_layer": shapes},
        "jacobi": jac,
        "split_vs_plain_amplitude_rel_err": float(np.linalg.norm(a - r) / np.linalg.norm(r)),
        "split_vs_plain_amplitude_max_err": float(np.max(np.abs(a - r)) / np.max(np.abs(r))),
        "amplitudes": "1024 patterns along the state's charge paths (seed 107)",
    }


def precision_full(MPS, dev, circuits):
    """The whole precision circuit (L=64, 32 photons in even modes, d=4, 64
    layers = 2016 gates, seed 3, chi_max=2048, cutoff 1e-12) from the Fock
    state, in both forms; 1024 uniform patterns (seed 103)."""
    import numpy as np
    import torch
    from paper_2303_11409_amd.binding import FORM_PLAIN_C128, FORM_SPLIT_BF16X3
    cfg = circuits.config_precision(seed=3, chi_max=2048)
    pats = circuits.sample_patterns(64, 32, 4, 1024, 103)
    out, amps = {}, {}
    for key, form in (("plain", FORM_PLAIN_C128), ("split_bf16x3", FORM_SPLIT_BF16X3)):
        m = MPS(cfg["occupation"], 4, chi_max=2048, cutoff=1e-12, form=form, device=dev)
        m.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for li, lay in enumerate(cfg["layers"]):
            m.apply_layer([g.site for g in lay], [g.u for g in lay])
            if li % 16 == 15:
                log(f"  {key}: layer {li + 1}/{len(cfg['layers'])}, {time.perf_counter() - t0:.1f} s")
        m.sync()
        el = time.perf_counter() - t0
        st = m.stats()
        amps[key] = m.amplitudes(pats)
        out[key] = {"seconds": el, "gate_applies_per_s": len(cfg["gates"]) / el, "norm2": m.norm2(),
                    "max_bond_dim": max(m.bond_dims()), "jacobi_ms": st["jacobi_ms"],
                    "theta_ms": st["theta_ms"] + st["gemm_ms"] + st["split_ms"],
                    "min_cut_margin": st["min_margin"]}
        m.close()
        log(f"  {key}: {el:.1f} s")
    a, r = amps["split_bf16x3"], amps["plain"]
    out["split_vs_plain_amplitude_rel_err"] = float(np.linalg.norm(a - r) / np.linalg.norm(r))
    out["workload"] = ("L=64, 32 photons in even modes, d=4, 64 brickwork layers (2016 gates, seed 3), "
                       "chi_max=2048, cutoff 1e-12; 1024 uniform patterns (seed 103)")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-copies", type=int, default=8,
                    help="batching form: seeds of the same circuit run together (0 = skip)")
    ap.add_argument("--mix-circuits", type=int, default=512,
                    help="batching form: circuits of the mixed-size workload run together (0 = skip)")
    ap.add_argument("--chi2048-layers", type=int, default=4,
                    help="precision form: brickwork layers applied to the saturated chi=2048 state in both "
                         "forms (0 = skip)")
    ap.add_argument("--precision-full", action="store_true",
                    help="also run the whole 2016-gate chi_max=2048 precision circuit in both forms "
                         "(several minutes)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="serving form: length of the serving window at --serve-rate (0 = skip)")
    ap.add_argument("--serve-low-seconds", type=float, default=20.0,
                    help="serving form: length of the window at --serve-low-rate")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="serving form: arrivals per second")
    ap.add_argument("--serve-low-rate", type=float, default=0.5,
                    help="serving form: a second window at this rate, within the device's capacity (0 = skip)")
    ap.add_argument("--serve-max-active", type=int, default=64,
                    help="serving form: most requests active at once in the lane of the batching-mix circuits")
    ap.add_argument("--serve-max-large", type=int, default=16,
                    help="serving form: most requests active at once in the lane of the chi_max=1024 circuits")
    ap.add_argument("--serve-budget-gib", type=float, default=96.0)
    ap.add_argument("--samples", type=int, default=4096,
                    help="exact output samples drawn from the final state (0 = skip)")
    ap.add_argument("--no-tebd", action="store_true",
                    help="skip the Hamiltonian time-evolution workloads (XXZ, Bose-Hubbard)")
    ap.add_argument("--jacobi-block", type=int, default=0,
                    help="vectors per Jacobi block of the headline circuit (0: chosen per update by the library; 8 or 16)")
    ap.add_argument("--sweep-graph", type=int, default=0,
                    help="headline circuit: 1 replays each Jacobi sweep from a captured HIP graph")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (the "
                         "reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_probe:
        return copy_probe(torch)

    from paper_2303_11409_amd import MPS, TorchDevice, apply_batch
    from workloads import circuits

    torch.cuda.set_device(0)
    cfg = circuits.config_plain_gpu()
    layers = [([g.site for g in lay], [g.u for g in lay]) for lay in cfg["layers"]]
    ngates = sum(len(s) for s, _ in layers)
    dev = TorchDevice()

    def new_state():
        return MPS(cfg["occupation"], cfg["d"], chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], device=dev,
                   jacobi_block=args.jacobi_block, sweep_graph=args.sweep_graph)

    def run(m):
        for sites, us in layers:
            m.apply_layer(sites, us)
        m.sync()

    def run_shapes(m):
        """The circuit once, recording each gate's outer bond dimensions."""
        shapes = []
        for sites, us in layers:
            dims = m.bond_dims()
            shapes.extend((dims[s], dims[s + 2]) for s in sites)
            m.apply_layer(sites, us)
        m.sync()
        return shapes

    shapes = None
    for w in range(max(args.warmup, 1)):
        t = time.perf_counter()
        m = new_state()
        if shapes is None:
            shapes = run_shapes(m)
        else:
            run(m)
        m.close()
        log(f"untimed run {w + 1}: {time.perf_counter() - t:.2f} s")

    states = [new_state() for _ in range(args.steps)]
    for m in states:
        m.set_timing(True)
        m.reset_stats()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i, m in enumerate(states):
        ts = time.perf_counter()
        run(m)
        lat.append(time.perf_counter() - ts)
        log(f"step {i + 1}/{args.steps}: {lat[-1]:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    agg = None
    for m in states:
        st = m.stats()
        if agg is None:
            agg = st
        else:
            for k, v in st.items():
                if k == "min_margin":
                    agg[k] = min(agg[k], v)
                elif k == "max_discarded":
                    agg[k] = max(agg[k], v)
                elif k in ("jacobi_block", "gemm_variant"):
                    agg[k] = v
                else:
                    agg[k] += v
    sampling = None
    if args.samples > 0:
        log(f"sampling {args.samples} output patterns from the final state ...")
        us = np.random.default_rng(7).random((args.samples, cfg["L"]))
        # one untimed call of the same size sizes the pinned staging; then the
        # median of three timed calls
        states[0].sample(us)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            ts = time.perf_counter()
            spats, sprob = states[0].sample(us)
            times.append(time.perf_counter() - ts)
        sel = sorted(times)[1]
        sflops = sample_flops(states[0], spats)
        sampling = {"workload": f"{args.samples} exact samples (chain rule over the left environments, "
                                "uniforms seed 7) of the final state of one step, host-to-host, median of 3 "
                                "calls after one untimed call",
                    "samples": args.samples, "seconds": sel, "value": args.samples / sel, "unit": "samples/s",
                    "distinct_patterns": int(len({tuple(p) for p in spats.tolist()})),
                    "max_prob": float(sprob.max()),
                    "kernel_flops": sflops,
                    "kernel_flops_note": "the sampler's algorithmic work: per sample and mode, 8 n_r n_c "
                                         "(w = B v) + 8 n_r^2 (w^H E w) per admissible occupation, plus one more "
                                         "B v for the drawn one; n = charge-block sizes along the drawn path "
                                         "(the grouped rounds reuse the drawn w, so they do the first two "
                                         "terms only)"}
        log(f"  {args.samples / sel:.0f} samples/s")
    norm_loss = 1.0 - states[0].norm2()
    max_chi = max(states[0].bond_dims())
    probe = circuits.sample_patterns(32, 16, 4, 64, 102)
    plain_amps = states[0].amplitudes(probe)
    for m in states:
        m.close()

    forms = {}
    if args.batch_copies > 0:
        B = args.batch_copies
        log(f"batching form: {B} seeds of the same circuit ...")
        cfgs = [circuits.config_plain_gpu(seed=2 + i) for i in range(B)]
        # Jacobi blocks of 16 throughout: what the per-update rule picks for
        # batches this large, fixed so that the seed-2 state can be compared bit
        # for bit with the single circuit run with the same blocks
        g, el, first, plan_s = run_batched(cfgs, MPS, apply_batch, dev, keep_first=True, jacobi_block=16)
        batch_amps = first.amplitudes(probe)
        first.close()
        alone = MPS(cfg["occupation"], cfg["d"], chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], device=dev,
                    jacobi_block=16)
        run(alone)
        alone_amps = alone.amplitudes(probe)
        alone.close()
        forms["batching_same_circuit"] = {
            "workload": f"{B} circuits: the plain workload with circuit seeds 2..{B + 1}, "
                        "each layer of all circuits in one mps_apply_batch call, Jacobi blocks of 16",
            "circuits": B, "gates": g, "seconds": el, "value": g / el, "unit": "gate applies/s",
            "vs_plain": (g / el) / (args.steps * ngates / elapsed), "host_plan_s": plan_s,
            "seed2_bitwise_equal_to_plain_same_blocks": bool(np.array_equal(batch_amps, alone_amps)),
            "seed2_vs_plain_default_blocks_max_rel_diff":
                float(np.max(np.abs(batch_amps - plain_amps)) / np.max(np.abs(plain_amps)))}
        log(f"  {g / el:.1f} gate applies/s")
    if args.mix_circuits > 0:
        n = args.mix_circuits
        log(f"batching form: {n} circuits of the mixed workload ...")
        cfgs = circuits.config_batch_mix(512)[:n]
        g, el, _, plan_s = run_batched(cfgs, MPS, apply_batch, dev)
        forms["batching_mix"] = {
            "workload": f"{n} of the 512 mixed circuits (circuit i: L ~ U{{16..48}}, floor(L/2) photons "
                        "in the first modes, d=4, depth L, chi_max ~ U{64,128,256,512}, cutoff 1e-12, "
                        "seed 4000+i; mix seed 4), complex128, layer k of all circuits in one "
                        "mps_apply_batch call, Jacobi sweeps replayed from captured HIP graphs",
            "circuits": n, "gates": g, "seconds": el, "value": g / el, "unit": "gate applies/s",
            "vs_plain": (g / el) / (args.steps * ngates / elapsed), "host_plan_s": plan_s}
        log(f"  {g / el:.1f} gate applies/s")

    # dominant kernel: the blocked Jacobi step (one launch per round-robin step);
    # updates take blocks of 8 (jacobi_block_step8) or 16 (jacobi_block_step)
    j8 = {"ms": agg["jacobi8_ms"], "launches": agg["jacobi8_launches"], "flops": agg["jacobi8_flops"]}
    j16 = {"ms": agg["jacobi_ms"] - j8["ms"], "launches": agg["jacobi_launches"] - j8["launches"],
           "flops": agg["jacobi_flops"] - j8["flops"]}
    jblock = 8 if j8["ms"] >= j16["ms"] else 16
    dom, other = (j8, j16) if jblock == 8 else (j16, j8)
    launches = max(dom["launches"], 1)
    per_launch_flops = dom["flops"] / launches
    avg_ms = dom["ms"] / launches
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
    kname = {8: "jacobi_block_step8", 16: "jacobi_block_step"}
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(jblock),
                "kernel": kname[jblock], "jacobi_block": jblock,
                "avg_launch_ms": avg_ms,
                "flops_per_launch": per_launch_flops, "launches": launches,
                "other_block_size": {"kernel": kname[24 - jblock], "launches": other["launches"],
                                     "ms": other["ms"],
                                     "tflops": other["flops"] / max(other["ms"], 1e-9) / 1e9}}
    props = torch.cuda.get_device_properties(0)
    value = args.steps * ngates / elapsed
    if args.chi2048_layers > 0:
        log(f"precision form: {args.chi2048_layers} layers of a saturated chi=2048 state, plain and split ...")
        forms["precision_chi2048"] = precision_chi2048(MPS, dev, circuits, args.chi2048_layers)
        g = forms["precision_chi2048"]
        log(f"  products: plain {g['plain']['tflops']:.1f} TFLOP/s, split "
            f"{g['split_bf16x3']['tflops_algorithmic']:.1f} (MFMA {100 * g['split_bf16x3']['frac_of_bf16_peak']:.1f}% "
            f"of BF16 peak); {g['gate_applies_per_s']['plain']:.1f} / {g['gate_applies_per_s']['split_bf16x3']:.1f} "
            f"gate applies/s; split vs plain {g['split_vs_plain_amplitude_rel_err']:.2e}")
    if args.precision_full:
        log("precision form: the whole 2016-gate chi_max=2048 circuit, plain and split ...")
        forms["precision_full_circuit"] = precision_full(MPS, dev, circuits)
    tebd = {}
    if not args.no_tebd:
        from workloads import hamiltonians
        for key, make in (("xxz", hamiltonians.config_xxz_quench),
                          ("bose_hubbard", hamiltonians.config_bose_hubbard_quench),
                          ("ising_z2", hamiltonians.config_ising_quench),
                          ("clock_z3", hamiltonians.config_clock_quench)):
            c = make()
            log(f"Hamiltonian TEBD ({key}, L={c['L']}, d={c['d']}, chi_max={c['chi_max']}) ...")
            r = run_tebd(MPS, dev, c)
            r["workload"] = " ".join((make.__doc__ or "").split(":", 1)[-1].split())
            tebd[key] = r
            log(f"  {r['value']:.1f} gate applies/s, max bond dim {r['max_bond_dim']}")
    if args.serve_seconds > 0:
        log(f"serving form: {args.serve_seconds:.0f} s at {args.serve_rate:g} requests/s ...")
        forms["serving"] = run_serving(args, args.serve_rate, args.serve_seconds, circuits)
        forms["serving"]["workload"] = (
            "Poisson arrivals of the serving mix (95% batching-mix circuits, 5% L=64, 32 photons, "
            "chi_max=1024, depth 64; request j seed 5000+j, 16 sampled amplitudes each), admitted by "
            f"an HBM budget of {args.serve_budget_gib:g} GiB, two lanes (chi_max=1024 requests, at most "
            f"{args.serve_max_large} active; the rest, at most {args.serve_max_active} active) each on its own "
            "stream and host thread, one "
            "batch call per layer of all active requests of a lane; window without drain, unfinished "
            "requests reported as censored")
        log(f"  {forms['serving']['gate_applies_per_s']:.1f} gate applies/s, "
            f"{forms['serving']['completed']} completed")
        if args.serve_low_rate > 0 and args.serve_low_seconds > 0:
            log(f"serving form: {args.serve_low_seconds:.0f} s at {args.serve_low_rate:g} requests/s ...")
            low = run_serving(args, args.serve_low_rate, args.serve_low_seconds, circuits)
            low["note"] = "same mix at an arrival rate within the device's capacity"
            forms["serving_low_rate"] = low
            log(f"  {low['gate_applies_per_s']:.1f} gate applies/s, {low['completed']} completed")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gate applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "boson-sampling brickwork L=32, N=16 photons in modes 0-15, d=4, "
                               "32 layers (496 beam splitters, seed 2), chi_max=512, cutoff 1e-12, "
                               "complex128 (plain form)",
                   "L": 32, "photons": 16, "d": 4, "layers": 32, "gates_per_step": ngates,
                   "chi_max": 512, "cutoff": 1e-12, "form": "plain complex128, layer-batched"},
        "roofline": roofline,
        "latency_s": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "unit": "s per circuit"},
        "kernels": {
            "theta_tflops": agg["theta_flops"] / max(agg["theta_ms"], 1e-9) / 1e9,
            "jacobi_tflops": agg["jacobi_flops"] / max(agg["jacobi_ms"], 1e-9) / 1e9,
            "theta_ms": agg["theta_ms"] / args.steps, "jacobi_ms": agg["jacobi_ms"] / args.steps,
            "jacobi_aux_ms": agg["jacobi_aux_ms"] / args.steps,
            "select_ms": agg["select_ms"] / args.steps, "update_ms": agg["update_ms"] / args.steps,
            "jacobi_launches_per_step": agg["jacobi_launches"] / args.steps,
            "jacobi_sweeps_per_sector": agg["sweeps"] / max(agg["sectors"], 1),
        },
        "device": {"name": props.name, "cus": props.multi_processor_count,
                   "lds_per_block": getattr(props, "shared_memory_per_block", None),
                   "lds_per_cu": getattr(props, "shared_memory_per_multiprocessor", None)},
        "forms": forms,
        "tebd": tebd,
        "sampling": sampling,
        "result": {"norm_loss": norm_loss, "max_bond_dim": max_chi,
                   "max_discarded": agg["max_discarded"], "min_cut_margin": agg["min_margin"]},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on saturated gates of the benchmark's shape ...")
        out["cpu_baseline"] = cpu_baseline(cfg, shapes)
        log(f"  {out['cpu_baseline']['value']:.3f} gate applies/s (whole-circuit estimate)")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
