#!/usr/bin/env python3
"""Benchmark of the IRL optimisation step on one MI355X.

Workload (default, --config c3): 20 spatial orbitals, 10 alpha + 10 beta
electrons, the 2^20 determinants of the seeded CISD-like selection (excitation
rank <= 4 from the aufbau determinant, top 2^20 by the seeded |c| model);
random molecule-like integrals (seed 0); network V = 40, H = 256 (P = 10,536),
so D~ would be 1,048,576 x 10,537 FP64 (88.4 GB): the exact FP64 path keeps the
factored Jacobian d = 1 - tanh^2 (1,048,576 x 256) instead; Krylov dimension 20,
one kept vector, tolerance 1e-12; the Hamiltonian's rows inside the set are
stored once (setup) and streamed by every apply.  Secondary figures in the same
line: the FP32-operator path of the same workload (FP32 D~ copy, FP64 energy,
gradient and solver) against the FP64 steps, and the 853,776-determinant full
space (12 orbitals, 6 alpha + 6 beta, V = 24, H = 64).

A timed step is one optimisation step: network evaluation (D~, Z, E,
gradient), the implicitly restarted Lanczos solve (operator applies,
recurrence, restarts) and the parameter update.  W warm-up steps run from
theta_0; theta is then reset to theta_0 and K steps are timed, so the timed
region is the first K steps of the trajectory.  Inputs are resident in HBM
before timing starts.

Prints one JSON line (stdout); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "time per IRL step & operator HBM GB/s vs roofline; solves/s, p99 step latency"
HAM_KERNELS = ["hashed-pull", "rank-pull", "string-product", "beta-blocked-pull", "stored-rows"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FP64_PEAK_TFLOPS = 78.6          # vector FP64 FMA rate: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz


def kernel_bytes(kind, ns, ncols, s_build):
    """Algorithmic HBM bytes of one launch of a dense-D~ kernel (reads + writes the
    kernel must do).  The stream kernels read the FP64 copy of D~ (8 B per element)
    or, for the *_fp32 kinds, the FP32 copy; the build writes every copy (s_build B)."""
    sD = 4 if kind.endswith("_fp32") else 8
    if kind.startswith("gemv_t"):   # read D~, read the two row vectors
        return ns * ncols * sD + 2 * ns * 8
    if kind.startswith("gemv"):     # read D~, read v, write w
        return ns * ncols * sD + ncols * 8 + ns * 8
    if kind == "dtilde_build":      # write D~ (and psi)
        return ns * ncols * s_build + ns * 8
    return None


CSRC = os.path.join(ROOT, "paper_2601_01437_amd", "csrc")


FULL_MIN_ROWS = 32768     # full spaces from this size take the string-split factored kernels


def fac_full_kernel(kind, info, rows, H):
    """Whether the factored product of this kind runs as the full-space (string-split)
    kernel: every row of a full space of at least FULL_MIN_ROWS rows, n <= 16, at most
    512 tiles of 16 beta strings, and H <= 64 for the forward pass and D~ v."""
    if not info.full_space or rows != info.n_dets or rows < FULL_MIN_ROWS or info.n_orb > 16:
        return False
    if (info.n_beta_strings + 15) // 16 > 512:
        return False
    return kind == "gemv_t" or H <= 64


def stored_alg_bytes(info, ns):
    """Algorithmic HBM bytes of one stored-row apply: every off-diagonal element's
    value and target once, plus w, the diagonal and u.  The systems timed here take
    the default layout: LDS-sliced (16-bit targets) up to 256 slices of 2^14 rows,
    L2-blocked (32-bit targets) beyond."""
    per_elem = 10 if ns <= 256 * (1 << 14) else 12
    return info.stored_elements * per_elem + 3 * 8 * ns


def kernel_roofline(kind, ns, ncols, H, factored, s_build, info, stored_bytes):
    """(name, bound, algorithmic work per launch, unit, peak, source files) of one
    timed kernel kind, or None.

    - Dense D~ streams and the dense build: HBM bytes (kernel_bytes).
    - Factored Jacobian (d = 1 - t^2 stored, N_s x H): the forward pass writes d and
      psi; D~ v reads d and psi and writes w; the apply's backward pass D~^T [w, u]
      reads d, psi, w and u.  The matrix-core forms also read the keys (8 B per
      row); the full-space forms read per-string tables instead (kilobytes).  HBM
      bytes: the matrix-core work, 2 N_s V H flops per product, is below the byte
      time at 8 TB/s for these shapes, and the full-space forms have none.
    - Hamiltonian apply: stored rows stream each off-diagonal element once (an FP64
      value and its target, 2 bytes in the LDS-sliced layout, 4 in the L2-blocked
      one) and read w and the diagonal and write u once (HBM); padding slots, row
      offsets and per-slice partial sums are the layout's overhead, not counted.
      The enumerating kernels do one FP64 multiply-add per candidate excitation
      (2 flops against the vector FP64 peak)."""
    P1 = ncols
    if kind in ("gemv", "gemv_t", "dtilde_build") and factored:
        name = {"gemv": "fac_jvp", "gemv_t": "fac_vjp", "dtilde_build": "fac_forward"}[kind]
        keys = 0 if fac_full_kernel(kind, info, ns, H) else 8
        nbytes = {"gemv": ns * (8 * H + 16 + keys) + 8 * P1, "gemv_t": ns * (8 * H + 24 + keys) + 16 * P1,
                  "dtilde_build": ns * (8 * H + 8 + keys)}[kind]
        return name, "hbm", nbytes, "GB/s", HBM_PEAK_GBPS, ("fac.hip", "internal.h")
    if kind in ("gemv", "gemv_t", "gemv_fp32", "gemv_t_fp32", "dtilde_build"):
        src = ("dtilde.hip", "internal.h") if kind != "dtilde_build" else ("nqs.hip", "internal.h")
        return kind, "hbm", kernel_bytes(kind, ns, ncols, s_build), "GB/s", HBM_PEAK_GBPS, src
    if kind == "ham_apply":
        if info.ham_kernel == 4:
            return ("ham_apply", "hbm", stored_alg_bytes(info, ns), "GB/s", HBM_PEAK_GBPS,
                    ("hamiltonian.hip", "internal.h"))
        return ("ham_apply", "alu", 2.0 * ns * info.max_connections, "TFLOP/s", FP64_PEAK_TFLOPS,
                ("hamiltonian.hip", "internal.h"))
    return None


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload, src_hash):
    """HBM traffic per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != src_hash:
        return None
    return float(m_val.group(1))


def cpu_baseline(wl, keys_fn, applies_per_step, sample_rows=1_000_000, chunk=None, budget_s=20.0):
    """The oracle's matrix-free apply (oracle.nqs rows, oracle C Slater-Condon
    rows, numpy products) timed on a row sample and scaled to one step.  The
    sample is a seeded random row subset, processed in chunks until about
    budget_s seconds of host time are spent (or sample_rows rows are done)."""
    import numpy as np

    from oracle import capply, nqs
    keys = keys_fn()
    ns = keys.size
    h, g = wl.integrals()
    theta = wl.theta()
    rng = np.random.default_rng(0)
    order = rng.permutation(ns)[:min(sample_rows, ns)]
    if chunk is None:
        chunk = max(256, min(20_000, (1 << 28) // (8 * (wl.P + 1))))   # D~ chunks of <= 256 MiB
    v = rng.normal(size=wl.P + 1)
    wfull = rng.normal(size=ns)       # Slater-Condon cost does not depend on w's values
    t_build = t_dv = t_h = t_dt = 0.0
    done = 0
    t_start = time.perf_counter()
    for c0 in range(0, order.size, chunk):
        if done and time.perf_counter() - t_start > budget_s:
            break
        rs = np.sort(order[c0:c0 + chunk])
        done += rs.size
        t = time.perf_counter()
        D = nqs.dtilde(keys[rs], wl.n, wl.V, wl.H, theta)
        t_build += time.perf_counter() - t
        t = time.perf_counter()
        w = D @ v
        t_dv += time.perf_counter() - t
        t = time.perf_counter()
        u = capply.apply(wl.n, h, g, keys, wfull, rows=rs)
        t_h += time.perf_counter() - t
        t = time.perf_counter()
        _ = D.T @ np.stack([w, u], axis=1)
        t_dt += time.perf_counter() - t
        del D
    rows = np.sort(order[:done])
    scale = ns / rows.size
    per_apply = (t_dv + t_h + t_dt) * scale
    per_eval = (t_build + t_h + t_dt) * scale          # D~, H psi, gradient pass
    per_step = applies_per_step * per_apply + per_eval
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same apply on one thread (OpenMP and BLAS limited), on a smaller sample
    one = None
    try:
        from threadpoolctl import threadpool_limits
        rs = rows[: max(1, min(rows.size, chunk, max(64, rows.size // 16)))]
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            D = nqs.dtilde(keys[rs], wl.n, wl.V, wl.H, theta)
            t_b1 = time.perf_counter() - t
            t = time.perf_counter()
            w = D @ v
            u = capply.apply(wl.n, h, g, keys, wfull, rows=rs)
            _ = D.T @ np.stack([w, u], axis=1)
            t_a1 = time.perf_counter() - t
        one = {"ms_per_apply": t_a1 * ns / rs.size * 1e3, "ms_dtilde_build": t_b1 * ns / rs.size * 1e3,
               "sample_rows": int(rs.size)}
    except ImportError:
        pass
    cpu_model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 1.0 / per_step,
        "unit": "IRL steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{rows.size} of {ns} rows: oracle network rows, oracle C Slater-Condon rows "
                   f"and numpy D~ products timed ({t_build + t_dv + t_h + t_dt:.1f} s) and scaled "
                   f"by {scale:.2f} to {applies_per_step:.1f} operator applies + 1 evaluation "
                   f"per step (apply count from the GPU run)"),
        "ms_per_apply": per_apply * 1e3,
        "ms_per_step": per_step * 1e3,
        "one_thread": one,
        "host": {"cpu_model": cpu_model, "logical_cpus": os.cpu_count()},
    }


def measured_hbm_peak(torch, gib=4, reps=5):
    """The achieved HBM rate of plain streaming on this GPU, next to the 8 TB/s
    datasheet peak the rooflines use: a read-only reduction (torch sum of a
    gib GiB FP64 tensor, bytes read / time) and a device-to-device copy
    (gib / 2 GiB each way, bytes read + written / time); best of reps, timed with
    HIP events on the current stream, outside the timed region of the bench."""
    n = (gib << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    half = x[: n // 2]
    y = torch.empty_like(half)
    x.sum()
    y.copy_(half)
    read, copy = [], []
    for _ in range(reps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        x.sum()
        e1.record()
        y.copy_(half)
        e2.record()
        e2.synchronize()
        read.append(n * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        copy.append(2 * (n // 2) * 8 / (e1.elapsed_time(e2) * 1e-3) / 1e9)
    del x, y, half
    torch.cuda.empty_cache()
    return {"read_GBps": max(read), "copy_GBps": max(copy), "bytes": n * 8,
            "method": f"torch sum of {gib} GiB FP64 (read) and a {gib / 2:g} GiB device copy, best of {reps}"}


def run_batch_bench(args):
    """64 independent solves (n ~ U{8..16}, half filled, full space capped at
    2^18 determinants, H ~ U{16..128}, FP64, m = 20, k = 1): one optimisation
    step each, (a) one after another with the solo path, (b) as batches of
    grouped kernels admitted in waves by workspace footprint.  --jacobian picks
    the factored Jacobian (default) or dense D~ copies for both."""
    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd import Batch, System

    wls = synth.batch_workloads(args.solves)
    log(f"building {len(wls)} systems")
    systems, thetas0 = [], []
    for w in wls:
        h, g = w.integrals()
        systems.append(System(w.n, w.na, w.nb, h, g, dets=w.dets(),
                              flags=B.IRL_SYS_STORE_BLOCKS if args.store_blocks else 0))
        thetas0.append(torch.tensor(w.theta(), dtype=torch.float64, device="cuda"))
    fl = B.IRL_WS_FACTORED if args.jacobian == "factored" else B.IRL_WS_FP64
    sizes = [B.irl_workspace_query(s.handle, w.P + 1, fl) for s, w in zip(systems, wls)]
    for s, w in zip(systems, wls):
        s.workspace(w.P + 1, fl)
    torch.cuda.synchronize()
    log(f"workspaces: {sum(sizes) / 1e9:.1f} GB")
    # selected (capped) sets: store H's rows while they fit beside the workspaces
    n_stored, stored_bytes, t = 0, 0, time.perf_counter()
    if not args.matrix_free:
        for s in systems:
            if s.info.full_space:
                continue
            free = torch.cuda.mem_get_info()[0]
            ok, need = s.store_hamiltonian(max(0, free - (8 << 30)))
            n_stored += ok
            stored_bytes += need if ok else 0
    log(f"stored rows for {n_stored} selected sets: {stored_bytes / 1e9:.1f} GB, "
        f"{(time.perf_counter() - t) * 1e3:.0f} ms")
    kernels = [s.info.ham_kernel for s in systems]
    opts = dict(m=20, k_keep=1, tol=1e-12)
    tune_report = None
    if args.autotune:
        # launch shapes per member from the autotuner (bit-neutral; outside the
        # timed passes, like the stored-row build); the untuned sequential pass
        # is timed first for comparison
        from paper_2601_01437_amd import autotune
        for s, w, th0 in zip(systems, wls, thetas0):
            s.step(th0.clone(), w.V, w.H, ws_flags=fl, want_dtheta=False, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, w, th0 in zip(systems, wls, thetas0):
            s.step(th0.clone(), w.V, w.H, ws_flags=fl, want_dtheta=False, **opts)
        torch.cuda.synchronize()
        t_untuned = time.perf_counter() - t0
        cache = autotune.TuneCache(args.tune_cache)
        t0 = time.perf_counter()
        choices = []
        for s, w, th0 in zip(systems, wls, thetas0):
            s.evaluate(w.V, w.H, th0.clone(), ws_flags=fl, want_grad=False)
            choices.append(autotune.tune_system(s, w.H, cache=cache))
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        tuned = {}
        for c in choices:
            for name, e in c.items():
                d = tuned.setdefault(name, {"members": 0, "changed": 0, "cached": 0})
                d["members"] += 1
                d["changed"] += e["value"] != 0
                d["cached"] += e["cached"]
        tune_report = {"sequential_untuned_ms": t_untuned * 1e3, "tuning_s": t_tune,
                       "knobs": tuned, "cache": args.tune_cache,
                       "values": [{k: e["value"] for k, e in c.items()} for c in choices]}
        log(f"autotune: {t_tune:.1f} s, {tuned}; untuned sequential {t_untuned * 1e3:.1f} ms")

    def solo_pass():
        out = []
        t0 = time.perf_counter()
        for s, w, th0 in zip(systems, wls, thetas0):
            th = th0.clone()
            rc, r, _, _ = s.step(th, w.V, w.H, ws_flags=fl, want_dtheta=False, **opts)
            out.append((rc, r.lambda_min, r.E_after, r.n_apply))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    # admission waves by footprint (first fit, input order)
    budget = args.hbm_budget_gb * 1e9
    waves, cur, used = [], [], 0.0
    for i, sz in enumerate(sizes):
        if cur and used + sz > budget:
            waves.append(cur)
            cur, used = [], 0.0
        cur.append(i)
        used += sz
    if cur:
        waves.append(cur)

    def batch_pass():
        out = [None] * len(wls)
        t0 = time.perf_counter()
        for wave in waves:
            ths = [thetas0[i].clone() for i in wave]
            bt = Batch([systems[i] for i in wave], ths, [wls[i].V for i in wave],
                       [wls[i].H for i in wave], ws_flags=fl)
            res, status, _ = bt.step(**opts)
            for j, i in enumerate(wave):
                out[i] = (status[j], res[j].lambda_min, res[j].E_after, res[j].n_apply)
            bt.close()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    def kernel_totals(handles):
        tot = {k: [0.0, 0] for k in B.STAT_KINDS}
        for hnd in handles:
            for k, (ms, cnt) in B.irl_stats_get(hnd).items():
                tot[k][0] += ms
                tot[k][1] += cnt
            B.irl_stats_enable(hnd, False)
        return {k: {"ms_total": v[0], "launches": v[1]} for k, v in tot.items() if v[1]}

    solo_pass()                          # warm-up (module load, allocator)
    batch_pass()
    t_solo, r_solo = solo_pass()
    log(f"sequential: {t_solo * 1e3:.1f} ms")
    t_batch, r_batch = batch_pass()
    log(f"batched: {t_batch * 1e3:.1f} ms in {len(waves)} wave(s)")
    # kernel-time breakdown of each pass (separate, untimed runs: events add host work)
    for s in systems:
        B.irl_stats_enable(s.handle, True)
    solo_pass()
    k_solo = kernel_totals([s.handle for s in systems])
    B.irl_stats_enable(systems[0].handle, True)
    batch_pass()
    k_batch = kernel_totals([systems[0].handle])
    log("kernel ms sequential: " + ", ".join(f"{k} {v['ms_total']:.0f}" for k, v in k_solo.items()))
    log("kernel ms batched:    " + ", ".join(f"{k} {v['ms_total']:.0f}" for k, v in k_batch.items()))
    dlam = max(abs(a[1] - b_[1]) / max(1.0, abs(a[1])) for a, b_ in zip(r_solo, r_batch))
    dE = max(abs(a[2] - b_[2]) for a, b_ in zip(r_solo, r_batch))
    out = {
        "metric": METRIC,
        "value": len(wls) / t_batch,
        "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"c4: {len(wls)} independent solves, n ~ U{{8..16}} half filled, "
                                f"full space capped at 2^18 determinants, H ~ U{{16..128}}, "
                                f"seeds 0..{len(wls) - 1}, one IRL step each (m=20, k=1, tol=1e-12), FP64, "
                                + ("factored Jacobian" if args.jacobian == "factored" else "dense D~ copies")),
                   "waves": len(waves), "workspace_GB": sum(sizes) / 1e9,
                   "ham_kernels": {HAM_KERNELS[k]: kernels.count(k) for k in sorted(set(kernels))},
                   "stored_rows_GB": stored_bytes / 1e9},
        "sequential_solves_per_s": len(wls) / t_solo,
        "speedup_vs_sequential": t_solo / t_batch,
        "max_rel_dlambda_batched_vs_sequential": dlam,
        "max_abs_dE_after_batched_vs_sequential": dE,
        "kernels_sequential": k_solo,
        "kernels_batched": k_batch,
        "applies": [r[3] for r in r_batch],
        "converged": sum(1 for r in r_batch if r[0] in (0, 2)),
        "autotune": tune_report,
    }
    print(json.dumps(out), flush=True)


def run_serving_bench(args):
    """Serving: requests (one optimisation step of a fresh network on the c1, c2
    or c3 system) arrive as a Poisson process (20/s, seed 0) over about
    args.serve_seconds; the mix is chosen so the offered load is 0.7 of the
    measured one-at-a-time capacity.  Served with resident slots per class and
    one lane per class (FP32 operator with the FP64 solver, or FP64 through the
    factored Jacobian), then against the plain sequential FP64 schedule (dense
    D~ copies) of the same arrivals."""
    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd.serving import (ClassPool, ClassSpec, Request, Server,
                                              latency_summary, run_sequential)

    rate = 20.0
    names = ("c1", "c2", "c3")
    wl = {c: synth.WORKLOADS[c] for c in names}
    ints = {c: wl[c].integrals() for c in names}
    dets = {c: wl[c].dets() for c in names}
    slots = {"c1": 16, "c2": 8, "c3": 1}

    factored = args.serve_operator == "fp64-factored"

    def make_pools(precision, nslots, fac=False):
        pools = {}
        for c in names:
            w = wl[c]
            h, g = ints[c]
            pools[c] = ClassPool(ClassSpec(c, w.n, w.na, w.nb, w.V, w.H, h, g, dets=dets[c], m=w.m,
                                           k_keep=w.k, precision=precision, slots=nslots[c],
                                           store_rows_bytes=32 << 30, factored=fac))
        torch.cuda.synchronize()
        return pools

    def service_ms(pools, reps):
        out = {}
        for c in names:
            r = Request(-1, c, 0.0, synth.nqs_theta(wl[c].V, wl[c].H, 999))
            pools[c].step([r])                       # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps[c]):
                pools[c].step([r])
            torch.cuda.synchronize()
            out[c] = (time.perf_counter() - t) / reps[c] * 1e3
        return out

    t_setup = time.perf_counter()
    pools = make_pools(B.IRL_FP64 if factored else B.IRL_FP32, slots, factored)
    log(f"resident pools ready in {time.perf_counter() - t_setup:.1f} s: "
        + ", ".join(f"{c} {len(p.systems)} slots {p.device_bytes() / 1e9:.1f} GB" for c, p in pools.items()))
    svc = service_ms(pools, {"c1": 5, "c2": 3, "c3": 1})
    log(f"one-at-a-time {args.serve_operator} service ms: " + ", ".join(f"{c} {v:.1f}" for c, v in svc.items()))
    # mix c1 : c2 : c3 = (1 - 6x) : 5x : x with offered load rate * E[service] = 0.7
    t1, t2, t3 = (svc[c] / 1e3 for c in names)
    x = (0.7 / rate - t1) / (5 * t2 + t3 - 6 * t1)
    x = float(min(max(x, 0.0), 1.0 / 6.0))
    mix = {"c1": 1 - 6 * x, "c2": 5 * x, "c3": x}
    offered = rate * sum(mix[c] * svc[c] / 1e3 for c in names)
    n_req = int(rate * args.serve_seconds)
    arr, picks = synth.serving_arrivals(n_req, rate, mix, seed=0)
    log(f"mix {', '.join(f'{c} {mix[c]:.3f}' for c in names)}; offered load {offered:.2f}; "
        f"{n_req} requests over {arr[-1]:.1f} s")

    def requests():
        return [Request(i, picks[i], float(arr[i]), synth.nqs_theta(wl[picks[i]].V, wl[picks[i]].H, 1000 + i))
                for i in range(n_req)]

    served = requests()
    makespan = Server(pools).run(served)
    lat = {"all": latency_summary(served)}
    for c in names:
        lat[c] = latency_summary([r for r in served if r.cls == c])
    log(f"served {n_req} in {makespan:.1f} s: p50 {lat['all']['p50_ms']:.1f} ms, "
        f"p99 {lat['all']['p99_ms']:.1f} ms")
    # a result in the mix equals the result alone (solo path, slot 0)
    checked = equal = 0
    c3_left = 2
    for r in served:
        if r.cls == "c3":
            if c3_left == 0:
                continue
            c3_left -= 1
        alone = Request(r.rid, r.cls, 0.0, r.theta)
        pools[r.cls].step([alone])
        checked += 1
        equal += (alone.lambda_min == r.lambda_min and alone.E_after == r.E_after
                  and alone.n_apply == r.n_apply and alone.status == r.status)
    torch.cuda.synchronize()
    log(f"mix vs alone: {equal}/{checked} bitwise equal")
    batch_sizes = [r.batch_size for r in served]
    for p in pools.values():
        p.close()
    pools = None
    torch.cuda.empty_cache()

    pools64 = make_pools(B.IRL_FP64, {c: 1 for c in names})
    svc64 = service_ms(pools64, {"c1": 5, "c2": 3, "c3": 1})
    log("sequential FP64 service ms: " + ", ".join(f"{c} {v:.1f}" for c, v in svc64.items()))
    seq = requests()
    makespan64 = run_sequential(pools64, seq)
    lat64 = {"all": latency_summary(seq)}
    for c in names:
        lat64[c] = latency_summary([r for r in seq if r.cls == c])
    log(f"sequential FP64: {n_req} in {makespan64:.1f} s: p50 {lat64['all']['p50_ms']:.1f} ms, "
        f"p99 {lat64['all']['p99_ms']:.1f} ms")
    dE = [abs(a.E_after - b_.E_after) for a, b_ in zip(served, seq) if np.isfinite(a.E_after)]
    for p in pools64.values():
        p.close()
    foot = footprint_leg(args)
    out = {
        "metric": METRIC,
        "value": n_req / makespan,
        "unit": "solves/s",
        "n_gpus": 1, "steps": n_req, "warmup": 1,
        "ms_per_step": lat["all"]["p50_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (factored Jacobian)" if factored else "f32 operator, f64 solver", "data": "synthetic",
        "config": {"workload": (f"c5: Poisson arrivals {rate:g}/s seed 0, {n_req} requests, each one IRL "
                                f"step of a fresh network (theta seed 1000 + request) on the c1 (4,900 "
                                f"full), c2 (853,776 full) or c3 (2^20 selected, stored rows) system; "
                                f"continuous admission into resident slots, one lane per class, "
                                f"{'FP64 factored-Jacobian' if factored else 'FP32'} operator"),
                   "mix": mix, "offered_load": offered, "slots": slots,
                   "service_ms_served": svc, "service_ms_fp64_dense": svc64},
        "latency_ms": lat,
        "mean_batch_size": float(np.mean(batch_sizes)),
        "makespan_s": makespan,
        "sequential_fp64": {"solves_per_s": n_req / makespan64, "makespan_s": makespan64,
                            "latency_ms": lat64},
        "mix_equals_alone": {"checked": checked, "bitwise_equal": equal},
        "max_abs_dE_after_served_vs_fp64_dense": float(max(dE)) if dE else None,
        "footprint_admission": foot,
    }
    print(json.dumps(out), flush=True)


def footprint_leg(args):
    """Admission by footprint: requests of classes that no pool holds in advance
    (random full spaces of 6 to 12 orbitals and selected sets of 2^12 to 2^17
    determinants of 16 to 20 orbitals, hidden widths 16 to 128; FP64 through the
    factored Jacobian, stored rows for the selected sets), Poisson arrivals 40/s for
    args.serve_seconds / 2, admitted whenever their slot's bytes fit a 3 GiB budget (about two
    of the largest classes, so slots are evicted and requests wait)."""
    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd.serving import ClassSpec, FootprintServer, Request, latency_summary

    rng = np.random.default_rng(7)
    specs = []
    for i in range(10):
        if i % 2 == 0:
            n = int(rng.integers(6, 13))
            na = nb = n // 2
            dets = None
        else:
            n = int(rng.integers(16, 21))
            na = nb = n // 2
            dets = synth.cisd_like_selected_set(n, na, nb, int(2 ** rng.integers(12, 18)), seed=100 + i)
        H = int(2 ** rng.integers(4, 8))
        h, g = synth.integrals(n, 100 + i)
        specs.append(ClassSpec(f"f{i}", n, na, nb, 2 * n, H, h, g, dets=dets, m=20, k_keep=1,
                               precision=B.IRL_FP64, slots=1, store_rows_bytes=(8 << 30) if dets is not None else 0,
                               factored=True))
    rate, secs = 40.0, max(args.serve_seconds / 2, 2.0)
    n_req = int(rate * secs)
    arr = np.cumsum(rng.exponential(1 / rate, size=n_req))
    picks = rng.integers(0, len(specs), size=n_req)
    reqs = [Request(i, specs[p].name, float(arr[i]), synth.nqs_theta(specs[p].V, specs[p].H, 2000 + i, scale=0.1),
                    spec=specs[p]) for i, p in enumerate(picks)]
    budget = 3 << 30
    srv = FootprintServer(budget, lanes=4, max_batch=8)
    try:
        makespan = srv.run(reqs)
        adm = srv.adm
        stats = {"created": adm.created, "evicted": adm.evicted, "reused": adm.reused,
                 "peak_bytes": adm.peak, "budget_bytes": budget}
    finally:
        srv.close()
    torch.cuda.empty_cache()
    lat = latency_summary(reqs)
    log(f"footprint admission: {n_req} requests of {len(specs)} classes in {makespan:.1f} s, "
        f"p50 {lat['p50_ms']:.1f} ms, p99 {lat['p99_ms']:.1f} ms, {stats}")
    return {"requests": n_req, "classes": len(specs), "rate_per_s": rate, "makespan_s": makespan,
            "solves_per_s": n_req / makespan, "latency_ms": lat, **stats,
            "ok": sum(1 for r in reqs if r.status in (0, 2))}


def run_ablation_bench(args):
    """Optimiser comparison (the shape of the paper's Fig. 2c): from the same theta_0
    on one workload, implicitly restarted Lanczos (IRL, m = 20, k = 1 by default), IRL
    in the connected tangent basis (mode C), IRL on the sampled (VMC) estimators,
    standard Lanczos (SL: one m = 20 Lanczos process per step, no restart, Algorithm
    2) and Adam (two step sizes).  E* is the energy where IRL's lowest eigenvalue reaches
    |lambda| <= 1e-12 (a stationary point of this network); each method reports the
    steps and seconds to E - E* <= 1e-3, 1e-6, 1e-9 and 1e-12 Ha, within its step
    and time caps (if IRL does not reach |lambda| <= 1e-12 within its cap, E* is the
    lowest energy any method reached).  FP64 factored Jacobian throughout."""
    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd import System

    wl = synth.WORKLOADS[args.ablation_workload]
    h, g = wl.integrals()
    sysm = System(wl.n, wl.na, wl.nb, h, g, dets=wl.dets())
    fl = B.IRL_WS_FACTORED
    theta0 = torch.tensor(wl.theta(), dtype=torch.float64, device="cuda")
    thresholds = (1e-3, 1e-6, 1e-9, 1e-12)

    def lanczos_run(m, k, restarts, flags, cap, tcap, info, mode=B.IRL_MODE_A):
        th = theta0.clone()
        Es, ts, lams = [], [], []
        applies = restarts_done = not_conv = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(cap):
            rc, r, _, _ = sysm.step(th, wl.V, wl.H, m=m, k_keep=k, tol=1e-12, max_restarts=restarts,
                                    flags=flags | (B.IRL_STEP_GRAPH if args.graph else 0), ws_flags=fl,
                                    want_dtheta=False, mode=mode)
            torch.cuda.synchronize()
            if not Es:
                Es.append(r.E_before)
                ts.append(0.0)
            Es.append(r.E_after)
            ts.append(time.perf_counter() - t0)
            lams.append(r.lambda_min)
            applies += r.n_apply
            restarts_done += r.n_restart
            not_conv += rc == B.IRL_ENOTCONV
            if rc == B.IRL_ESTEP or abs(r.lambda_min) <= 1e-12 or ts[-1] > tcap:
                break
        info.update(applies_per_step=applies / max(1, len(lams)), restarts_per_step=restarts_done / max(1, len(lams)),
                    steps_not_converged=not_conv, last_lambda=lams[-1] if lams else None)
        return np.array(Es), np.array(ts), lams

    def vmc_run(m, k, nsamp, cap, tcap, info):
        """IRL on the sampled estimators: each step draws nsamp configurations from
        |psi|^2 at the current theta (fresh seeded uniforms) and solves the sampled
        centred matrix; the recorded energies are the exact ones on the set."""
        th = theta0.clone()
        rng = np.random.default_rng(wl.seed + 1)
        Es, ts, lams = [], [], []
        applies = not_conv = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flv = fl | B.IRL_WS_SAMPLED
        for it in range(cap):
            u = torch.tensor(rng.random(nsamp), dtype=torch.float64, device="cuda")
            sysm.evaluate(wl.V, wl.H, th, ws_flags=flv, want_grad=False)
            out, _, _ = sysm.vmc_sample(u)
            rc, r, _, _ = sysm.step(th, wl.V, wl.H, m=m, k_keep=k, tol=1e-12, max_restarts=300,
                                    flags=B.IRL_STEP_WS_CURRENT | (B.IRL_STEP_GRAPH if args.graph else 0),
                                    ws_flags=flv, want_dtheta=False)
            torch.cuda.synchronize()
            if not Es:
                Es.append(out.E_exact)
                ts.append(0.0)
            Es.append(r.E_after if np.isfinite(r.E_after) else Es[-1])
            ts.append(time.perf_counter() - t0)
            lams.append(r.lambda_min)
            applies += r.n_apply
            not_conv += rc == B.IRL_ENOTCONV
            if rc == B.IRL_ESTEP or ts[-1] > tcap:
                break
        info.update(applies_per_step=applies / max(1, len(lams)), steps_not_converged=not_conv,
                    last_lambda=lams[-1] if lams else None, samples_per_step=nsamp)
        return np.array(Es), np.array(ts), lams

    def adam_run(lr, cap, tcap):
        th = theta0.clone()
        m = torch.zeros(wl.P, dtype=torch.float64, device="cuda")
        v = torch.zeros_like(m)
        Es, ts = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, cap + 1):
            _, E = sysm.adam_step(wl.V, wl.H, th, m, v, t, ws_flags=fl, lr=lr)
            Es.append(E)
            ts.append(time.perf_counter() - t0)
            if ts[-1] > tcap:
                break
        return np.array(Es), np.array(ts)

    log(f"ablation on {wl.name}: IRL reference")
    lanczos_run(20, 1, 0, 0, 1, 1e9, {})                  # warm-up
    mk = args.ablation_irl
    irl_name = f"IRL (m={mk[0]}, k={mk[1]})"
    info = {irl_name: {}, "SL (m=20, no restart)": {}}
    E_irl, t_irl, lam_irl = lanczos_run(mk[0], mk[1], 300, 0, args.irl_steps, args.irl_seconds, info[irl_name])
    irl_converged = abs(lam_irl[-1]) <= 1e-12
    log(f"IRL: {len(E_irl) - 1} steps, E {E_irl[-1]:.12f}, lambda {lam_irl[-1]:.2e}, {info[irl_name]}")
    E_sl, t_sl, lam_sl = lanczos_run(20, 1, 0, B.IRL_STEP_FULL_CYCLES, args.sl_steps, args.irl_seconds,
                                     info["SL (m=20, no restart)"])
    runs = {irl_name: (E_irl, t_irl), "SL (m=20, no restart)": (E_sl, t_sl)}
    conn_name = f"IRL connected basis (mode C, m={mk[0]}, k={mk[1]})"
    info[conn_name] = {}
    E_c, t_c, lam_c = lanczos_run(mk[0], mk[1], 300, 0, args.irl_steps, args.irl_seconds, info[conn_name],
                                  mode=B.IRL_MODE_C)
    log(f"IRL mode C: {len(E_c) - 1} steps, E {E_c[-1]:.12f}, lambda {lam_c[-1]:.2e}, {info[conn_name]}")
    runs[conn_name] = (E_c, t_c)
    if args.ablation_vmc_samples > 0:
        vmc_name = f"IRL sampled estimators (VMC, {args.ablation_vmc_samples} draws, m={mk[0]}, k={mk[1]})"
        info[vmc_name] = {}
        E_v, t_v, lam_v = vmc_run(mk[0], mk[1], args.ablation_vmc_samples, args.irl_steps, args.irl_seconds,
                                  info[vmc_name])
        log(f"IRL VMC: {len(E_v) - 1} steps, E {E_v[-1]:.12f}, lambda {lam_v[-1]:.2e}, {info[vmc_name]}")
        runs[vmc_name] = (E_v, t_v)
    for lr in args.adam_lr:
        E_a, t_a = adam_run(lr, args.adam_steps, args.adam_seconds)
        runs[f"Adam (lr={lr:g})"] = (E_a, t_a)
    # E*: IRL's stationary point, else the lowest energy any method reached
    E_star = float(E_irl[-1]) if irl_converged else float(min(E.min() for E, _ in runs.values()))
    log(f"E* = {E_star:.12f} ({'IRL stationary point' if irl_converged else 'lowest energy reached'})")
    out_methods = {}
    for name, (E, t) in runs.items():
        err = E - E_star
        reach = {}
        for thr in thresholds:
            idx = np.nonzero(err <= thr)[0]
            reach[f"{thr:g}"] = None if idx.size == 0 else {"steps": int(idx[0]), "seconds": float(t[idx[0]])}
        out_methods[name] = {"steps_run": int(len(E) - (1 if name.startswith(("IRL", "SL")) else 0)),
                             "seconds": float(t[-1]), "ms_per_step": float(t[-1] / max(1, len(E) - 1) * 1e3),
                             "final_error": float(err[-1]), "best_error": float(err.min()), "reach": reach,
                             **info.get(name, {})}
        log(f"{name}: {out_methods[name]['steps_run']} steps, {t[-1]:.3f} s, final E - E* = {err[-1]:.3e}")
    irl_t = out_methods[irl_name]["reach"]["1e-12"]
    out = {
        "metric": "steps and time to E - E* <= 1e-12 Ha (IRL, IRL connected basis, standard Lanczos, Adam)",
        "value": irl_t["seconds"] if irl_t else None,
        "unit": "s (IRL to 1e-12 Ha)",
        "n_gpus": 1, "steps": int(len(E_irl) - 1), "warmup": 1,
        "ms_per_step": out_methods[irl_name]["ms_per_step"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"optimiser comparison on {wl.name}: {wl.n} orbitals {wl.na}a+{wl.nb}b, "
                                f"V={wl.V} H={wl.H} (P={wl.P}), same theta_0 (seed {wl.seed}); IRL m={mk[0]} k={mk[1]} "
                                f"tol=1e-12; SL m=20 without restart; Adam beta=(0.9, 0.999) eps=1e-8, "
                                f"at most {args.adam_steps} steps or {args.adam_seconds:g} s"),
                   "E_star": E_star, "E_star_is_irl_stationary_point": bool(irl_converged)},
        "methods": out_methods,
        "trajectories": {name: [float(x) for x in (E[:60] if len(E) <= 60 else
                                                     E[np.unique(np.geomspace(1, len(E) - 1, 60).astype(int))])]
                         for name, (E, t) in runs.items()},
    }
    print(json.dumps(out), flush=True)


def vmc_cpu_baseline(wl, nsamp, applies_per_step, sample_draws=40, sample_rows=16384):
    """The oracle's sampled step on the host, timed on bounded parts and scaled:
    orbital-by-orbital draws (sample_draws of them), network rows, local energies
    (oracle C Slater-Condon rows) and the sample-mean product of Eq.
    matrix_vec_prod on sample_rows rows, scaled to nsamp draws and one product per
    operator apply."""
    import numpy as np

    from oracle import capply, nqs, space, vmc
    keys = wl.dets()
    if keys is None:
        keys = space.full_space(wl.n, wl.na, wl.nb)
    h, g = wl.integrals()
    theta = wl.theta()
    rng = np.random.default_rng(0)
    ns = keys.size
    psi_all = rng.normal(size=ns)            # draw cost does not depend on the values
    t = time.perf_counter()
    vmc.sample_autoregressive(keys, wl.n, wl.na, wl.nb, psi_all, rng.random(sample_draws))
    t_draw = (time.perf_counter() - t) / sample_draws
    rows = np.sort(rng.choice(ns, size=min(sample_rows, ns), replace=False))
    t = time.perf_counter()
    D = nqs.dtilde(keys[rows], wl.n, wl.V, wl.H, theta)
    t_rows = time.perf_counter() - t
    t = time.perf_counter()
    hpsi = capply.apply(wl.n, h, g, keys, psi_all, rows=rows)
    t_eloc = time.perf_counter() - t
    O = vmc.log_derivatives(D)
    Eloc = hpsi / D[:, 0]
    v = rng.normal(size=wl.P + 1)
    r = np.arange(rows.size)
    t = time.perf_counter()
    vmc.sampled_mvp(r, O, Eloc, v)
    t_mvp = time.perf_counter() - t
    scale = nsamp / rows.size
    per_step = nsamp * t_draw + (t_rows + t_eloc) * scale + applies_per_step * t_mvp * scale
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": 1.0 / per_step, "unit": "sampled IRL steps/s", "cores": cores, "kind": "oracle",
        "sample": (f"{sample_draws} orbital-by-orbital draws over {ns} determinants "
                   f"({t_draw * 1e3:.1f} ms each) and {rows.size} rows of network values, local "
                   f"energies and the Eq. matrix_vec_prod product, scaled to {nsamp} draws and "
                   f"{applies_per_step:.1f} products per step (apply count from the GPU run)"),
        "ms_per_step": per_step * 1e3, "ms_per_draw": t_draw * 1e3,
    }


def select_live_kinds(args, B, warm, has_roofline):
    """Kernel classes bracketed by events inside the timed region: the one with a
    roofline and the largest total time over the warm-up steps (each event pair
    costs a few microseconds of queue time per launch); every class with
    --all-events or without warm-up figures; none with --graph or --no-events."""
    if args.graph or args.no_events:
        return []
    ranked = sorted((k for k, v in warm.items() if v[1] and has_roofline(k)), key=lambda k: -warm[k][0])
    if args.all_events or not ranked:
        return list(B.STAT_KINDS)
    return ranked[:1]


def run_vmc_bench(args):
    """Sampled VMC step (Eq. matrix_vec_prod estimator) on one workload: each step
    evaluates psi, d and H psi at theta on the set, draws N configurations from
    |psi|^2 (irl_vmc_sample; uniforms from a seeded host generator, in HBM before
    the timed region), and runs one IRL solve on the sampled centred matrix with
    the update.  Reports sampled steps/s, draws/s and per-kernel rooflines."""
    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd import System

    wl = synth.WORKLOADS[args.vmc_workload]
    h, g = wl.integrals()
    sysm = System(wl.n, wl.na, wl.nb, h, g, dets=wl.dets())
    ns = sysm.ns
    gathered = not args.vmc_all_rows
    ws_flags = B.IRL_WS_FACTORED | (B.IRL_WS_SAMPLED if gathered else 0)
    theta0 = torch.tensor(wl.theta(), dtype=torch.float64, device="cuda")
    theta = theta0.clone()
    N = args.vmc_samples
    rng = np.random.default_rng(wl.seed)
    U = torch.tensor(rng.random((args.warmup + args.steps, N)), dtype=torch.float64, device="cuda")
    log(f"vmc on {wl.name}: {ns} determinants, P={wl.P}, {N} draws per step, m={wl.m} k={wl.k}")

    def one_step(i):
        sysm.evaluate(wl.V, wl.H, theta, ws_flags=ws_flags, want_grad=False)
        out, _, _ = sysm.vmc_sample(U[i])
        rc, r, _, _ = sysm.step(theta, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, ws_flags=ws_flags,
                                flags=B.IRL_STEP_WS_CURRENT | B.IRL_STEP_NO_EVAL_AFTER, want_dtheta=False)
        return out, rc, r

    B.irl_stats_select(sysm.handle, None)
    B.irl_stats_enable(sysm.handle, args.warmup > 0 and not args.graph)
    for i in range(args.warmup):
        out, rc, r = one_step(i)
        log(f"warmup {i}: E_sampled={out.E_sampled:.10f} E={out.E_exact:.10f} unique={out.n_unique} "
            f"lambda={r.lambda_min:.3e} applies={r.n_apply}")
    warm = B.irl_stats_get(sysm.handle)
    B.irl_stats_enable(sysm.handle, False)
    theta.copy_(theta0)
    torch.cuda.synchronize()
    # events in the timed region around the dominant kernel class only (as in the
    # main bench); every class's times from an untimed rerun below
    live = select_live_kinds(args, B, warm, lambda k: kernel_roofline(k, ns, wl.P + 1, wl.H, True, 0,
                                                                       sysm.info, 0) is not None)
    B.irl_stats_select(sysm.handle, live or None)
    B.irl_stats_enable(sysm.handle, bool(live))
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out, rc, r = one_step(args.warmup + i)
        steps.append({"E_sampled": out.E_sampled, "E": out.E_exact, "E_loc_var": out.E_loc_var,
                      "unique": out.n_unique, "lambda_min": r.lambda_min, "applies": r.n_apply,
                      "converged": r.converged})
        log(f"step {i}: E_sampled={out.E_sampled:.10f} E={out.E_exact:.10f} unique={out.n_unique} "
            f"lambda={r.lambda_min:.3e} applies={r.n_apply}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = B.irl_stats_get(sysm.handle)
    B.irl_stats_enable(sysm.handle, False)
    if len(live) < len(B.STAT_KINDS):
        theta_end = theta.clone()
        theta.copy_(theta0)
        B.irl_stats_select(sysm.handle, None)
        B.irl_stats_enable(sysm.handle, True)
        for i in range(args.steps):
            one_step(args.warmup + i)
        rerun = B.irl_stats_get(sysm.handle)
        B.irl_stats_enable(sysm.handle, False)
        theta.copy_(theta_end)
        stats = {k: (stats[k] if k in live else rerun[k]) for k in rerun}
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kern = {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / v[1] if v[1] else None,
                "timed_live": k in live}
            for k, v in stats.items() if v[1]}
    rooflines = {}
    mean_unique = sum(st["unique"] for st in steps) / len(steps)
    for k, v in kern.items():
        # the operator's products run over the drawn rows only when they are gathered
        rows = mean_unique if gathered and k in ("gemv", "gemv_t") else ns
        spec = kernel_roofline(k, rows, wl.P + 1, wl.H, True, 0, sysm.info, 0)
        if spec is None:
            continue
        name, bound, work, unit, peak, src = spec
        scale = 1e9 if unit == "GB/s" else 1e12
        achieved = work / (v["ms_avg"] * 1e-3) / scale
        src_hash = source_hash([os.path.join(CSRC, f) for f in src])
        rooflines[name] = {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                           "frac": achieved / peak, "traffic": None,
                           ("bytes_per_launch" if unit == "GB/s" else "flops_per_launch"): work,
                           "ms_avg": v["ms_avg"], "ms_total": v["ms_total"], "launches": v["launches"],
                           "source_hash": src_hash}
    roof = max(rooflines.values(), key=lambda r: r["ms_total"]) if rooflines else None
    if len(live) == 1 and live[0] in kern:
        spec = kernel_roofline(live[0], ns, wl.P + 1, wl.H, True, 0, sysm.info, 0)
        roof = rooflines.get(spec[0], roof) if spec else roof
    applies = sum(st["applies"] for st in steps) / len(steps)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sampled step, bounded sample)")
        cpu = vmc_cpu_baseline(wl, N, applies)
    out = {
        "metric": "sampled VMC IRL steps/s", "value": args.steps / (t1 - t0), "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"sampled VMC step on {wl.name}: {wl.n} orbitals {wl.na}a+{wl.nb}b, "
                                f"{ns} determinants, V={wl.V} H={wl.H} (P={wl.P}), {N} draws per step, "
                                f"IRL m={wl.m} k={wl.k} tol=1e-12 on the sampled centred matrix, "
                                f"factored Jacobian, exact evaluation of psi and H psi on the set, "
                                f"operator products over "
                                f"{'the gathered drawn rows' if gathered else 'every row'}"),
                   "mean_unique_rows": mean_unique,
                   "kernel_events_in_timed_region": live if len(live) < len(B.STAT_KINDS) else "all"},
        "draws_per_s": N * args.steps / (t1 - t0),
        "roofline": {k: v for k, v in roof.items()} if roof else None,
        "rooflines": rooflines,
        "kernels": kern,
        "steps_detail": steps,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def fp32_operator_comparison(args, B, sysm, wl, theta0, first64, torch):
    """The FP32-operator path of the same workload beside the FP64 steps: an FP32
    copy of D~ (FP32 products, FP32 accumulation inside a row block), FP64 energy,
    gradient, Lanczos and QR; without and with the FP64 polish of the Ritz pair
    (the polish restarts the FP64 factored solve from the FP32 Ritz vector, so the
    step then meets the FP64 tolerances); and the plain FP64 form, which streams an
    FP64 copy of D~ (twice the FP32 copy's bytes).  Each variant runs K steps from
    theta_0; the first step's eigenvalue and energy after the update are compared
    with the factored FP64 path's."""
    out = {}
    for name, fl, prec, flags in (("fp32", B.IRL_WS_FP32, B.IRL_FP32, B.IRL_STEP_NO_POLISH),
                                  ("fp32_polished", B.IRL_WS_FP32 | B.IRL_WS_FACTORED, B.IRL_FP32, 0),
                                  ("fp64_dense", B.IRL_WS_FP64, B.IRL_FP64, 0)):
        sysm.ws = None
        torch.cuda.empty_cache()
        th = theta0.clone()
        rs, ms = [], []
        for i in range(args.warmup + args.steps):
            if i == args.warmup:
                th.copy_(theta0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, r, _, _ = sysm.step(th, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, precision=prec,
                                    flags=flags, ws_flags=fl, want_dtheta=False)
            torch.cuda.synchronize()
            if i >= args.warmup:
                ms.append((time.perf_counter() - t) * 1e3)
                rs.append(r)
        r0 = rs[0]
        out[name] = {"ms_per_step": sum(ms) / len(ms), "applies_fp32": r0.n_apply_lo,
                     "applies_fp64": r0.n_apply - r0.n_apply_lo, "lambda": r0.lambda_min,
                     "E_after": r0.E_after, "converged": r0.converged}
        if first64 is not None:
            out[name]["dlambda_vs_fp64"] = r0.lambda_min - first64["lambda_min"]
        log(f"{name}: {out[name]['ms_per_step']:.1f} ms per step, lambda {r0.lambda_min:.6e}")
    sysm.ws = None
    torch.cuda.empty_cache()
    # the FP64 first step's energy after the update (the timed steps skip it)
    th = theta0.clone()
    rc, r64, _, _ = sysm.step(th, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, precision=B.IRL_FP64,
                              ws_flags=B.IRL_WS_FACTORED, want_dtheta=False)
    for name in out:
        out[name]["dE_after_vs_fp64"] = out[name]["E_after"] - r64.E_after
    out["fp64_first_step"] = {"lambda": r64.lambda_min, "E_after": r64.E_after, "norm_T": r64.norm_T}
    sysm.ws = None
    torch.cuda.empty_cache()
    return out


def full_space_secondary(args, B, synth, System, torch):
    """K steps of the exact FP64 path (factored Jacobian) on the 853,776-determinant
    full space (12 orbitals, 6 alpha + 6 beta, V = 24, H = 64, m = 40, k = 10), with
    per-kernel averages from events around every launch of an untimed rerun."""
    wl = synth.WORKLOADS["c2"]
    h, g = wl.integrals()
    s = System(wl.n, wl.na, wl.nb, h, g)
    theta0 = torch.tensor(wl.theta(), dtype=torch.float64, device="cuda")
    th = theta0.clone()

    def step():
        return s.step(th, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, ws_flags=B.IRL_WS_FACTORED,
                      flags=B.IRL_STEP_NO_EVAL_AFTER, want_dtheta=False)
    for _ in range(args.warmup):
        step()
    th.copy_(theta0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    applies = 0
    for _ in range(args.steps):
        rc, r, _, _ = step()
        applies += r.n_apply
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    th.copy_(theta0)
    B.irl_stats_select(s.handle, None)
    B.irl_stats_enable(s.handle, True)
    for _ in range(args.steps):
        step()
    st = B.irl_stats_get(s.handle)
    B.irl_stats_enable(s.handle, False)
    s.close()
    kern = {k: v[0] / v[1] for k, v in st.items() if v[1]}
    log(f"full space: {ms:.2f} ms per step, ham {kern.get('ham_apply', 0):.3f} ms per apply")
    return {"workload": "12 orbitals 6a+6b full space (853,776 determinants), V=24 H=64 (P=1624), "
                        "factored FP64, m=40 k_keep=10",
            "steps": args.steps, "ms_per_step": ms, "steps_per_s": 1000.0 / ms,
            "applies_per_step": applies / args.steps, "kernel_ms_avg": kern}


def warm_start_leg(args, B, sysm, wl, theta, theta0, precision, step_flags, ws_flags, cold, torch):
    """The timed steps again from theta0 with each Lanczos process after the first
    started at the previous step's Ritz vector (IRL_STEP_WARM_START, an option:
    Algorithm 1 and the headline steps start from a random unit vector).  Reports
    the rate, the applies and the largest energy and eigenvalue differences from
    the cold-started trajectory; theta is left as the timed steps left it."""
    if args.block > 1 or not cold:
        return None
    theta_end = theta.clone()
    theta.copy_(theta0)
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        flags = step_flags | (B.IRL_STEP_WARM_START if i else 0)
        rc, r, _, _ = sysm.step(theta, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, precision=precision,
                                flags=flags, ws_flags=ws_flags, want_dtheta=False)
        rows.append((r.E_before, r.lambda_min, r.n_apply, r.converged))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    theta.copy_(theta_end)
    log(f"warm start: {ms:.1f} ms per step, applies {[a for _, _, a, _ in rows]}")
    return {"value": 1000.0 / ms, "unit": "IRL steps/s", "ms_per_step": ms,
            "applies_per_step": sum(a for _, _, a, _ in rows) / len(rows),
            "all_converged": all(c == 1 for _, _, _, c in rows),
            "max_abs_dE_vs_cold": max(abs(e - c["E"]) for (e, _, _, _), c in zip(rows, cold)),
            "max_abs_dlambda_vs_cold": max(abs(l - c["lambda_min"]) for (_, l, _, _), c in zip(rows, cold))}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c3s", "c4", "c5", "ablation", "vmc"])
    ap.add_argument("--no-secondary", dest="secondary", action="store_false",
                    help="c3: skip the FP32-operator comparison and the full-space (12-orbital) steps")
    ap.add_argument("--vmc-workload", default="c2", choices=["c1", "c2", "c3s"],
                    help="vmc: workload of the sampled step")
    ap.add_argument("--vmc-samples", type=int, default=1 << 17, help="vmc: draws per step")
    ap.add_argument("--vmc-all-rows", action="store_true",
                    help="vmc: run the sampled operator's products over every row (zero weights "
                         "outside the draws) instead of the gathered drawn rows")
    ap.add_argument("--ablation-workload", default="c1", choices=["c1", "c2", "c3s"],
                    help="ablation: workload of the optimiser comparison")
    ap.add_argument("--adam-lr", type=float, nargs="+", default=[1e-3, 1e-2], help="ablation: Adam step sizes")
    ap.add_argument("--adam-steps", type=int, default=20000, help="ablation: Adam step cap")
    ap.add_argument("--adam-seconds", type=float, default=20.0, help="ablation: Adam time cap per step size")
    ap.add_argument("--sl-steps", type=int, default=400, help="ablation: standard Lanczos step cap")
    ap.add_argument("--irl-steps", type=int, default=400, help="ablation: IRL step cap")
    ap.add_argument("--irl-seconds", type=float, default=60.0, help="ablation: IRL and SL time cap")
    ap.add_argument("--ablation-vmc-samples", type=int, default=4096,
                    help="ablation: draws per step of the sampled-estimator IRL run (0: skip it)")
    ap.add_argument("--ablation-irl", type=int, nargs=2, default=[20, 1], metavar=("M", "K"),
                    help="ablation: IRL Krylov dimension and vectors kept per restart")
    ap.add_argument("--serve-operator", default="fp32", choices=["fp32", "fp64-factored"],
                    help="c5: operator of the served classes (FP32 D~ copy with the FP64 solver, "
                         "or FP64 through the factored Jacobian)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="c5: length of the arrival window in seconds")
    ap.add_argument("--solves", type=int, default=64, help="c4: number of independent solves")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="c4: keep the built-in launch shapes (default: per-member autotuned shapes)")
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="c4: autotuner cache file (read if present, written after tuning)")
    ap.add_argument("--hbm-budget-gb", type=float, default=240.0,
                    help="c4: device memory admitted per wave of batched solves")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="operator precision (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--store-blocks", action="store_true",
                    help="c4: store the selected sets' rows in the L2-blocked layout")
    ap.add_argument("--jacobian", default="factored", choices=["dense", "factored"],
                    help="FP64 operator: products with the factored Jacobian of the network "
                         "(default) or streams of the dense D~")
    ap.add_argument("--block", type=int, default=0,
                    help="vectors per operator pass: 0/1 implicitly restarted Lanczos, 2..8 block Lanczos")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured Lanczos cycles (HIP graphs) where a solve tests only at the "
                         "end of each cycle (operators under 256 MB per apply); the timed region "
                         "then runs without per-kernel events")
    ap.add_argument("--all-events", action="store_true",
                    help="bracket every kernel launch with events in the timed region (default: only "
                         "the dominant kernel class, named by the warm-up steps)")
    ap.add_argument("--no-events", action="store_true",
                    help="time the steps without per-kernel events (kernel times then come from an "
                         "untimed rerun of the same steps)")
    ap.add_argument("--polish", action="store_true",
                    help="FP32 operator: keep an FP64 copy of D~ and refine the Ritz pair in FP64")
    ap.add_argument("--no-fp64-reference", dest="fp64_reference", action="store_false",
                    help="FP32 operator: skip the FP64 step used to report the precision gap")
    ap.add_argument("--force-hash", action="store_true", help="general hashed Hamiltonian kernel")
    ap.add_argument("--matrix-free", action="store_true",
                    help="selected sets: enumerate excitations on every apply instead of "
                         "streaming stored rows")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2601_01437_amd import binding as B
    from paper_2601_01437_amd import System

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}), flush=True)
        return
    if args.config == "c4":
        run_batch_bench(args)
        return
    if args.config == "c5":
        run_serving_bench(args)
        return
    if args.config == "ablation":
        run_ablation_bench(args)
        return
    if args.config == "vmc":
        run_vmc_bench(args)
        return
    wl = synth.WORKLOADS[args.config]
    h, g = wl.integrals()
    log(f"workload {wl.name}: n={wl.n} {wl.na}a+{wl.nb}b V={wl.V} H={wl.H} P={wl.P} m={wl.m} k={wl.k}")
    t = time.perf_counter()
    dets = wl.dets()
    sysm = System(wl.n, wl.na, wl.nb, h, g, dets=dets,
                  flags=B.IRL_SYS_FORCE_HASH if args.force_hash else 0)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t) * 1e3
    ns = sysm.ns
    log(f"system ready: {ns} determinants, ham kernel {sysm.info.ham_kernel}, {setup_ms:.1f} ms")
    theta0 = torch.tensor(wl.theta(), dtype=torch.float64, device="cuda")
    theta = theta0.clone()
    prec_name = args.precision or "fp64"
    precision = B.IRL_FP64 if prec_name == "fp64" else B.IRL_FP32
    # FP32 operator: FP32 copy of D~ only, unless the FP64 polish of the Ritz pair is asked for
    if precision == B.IRL_FP64:
        ws_flags = B.IRL_WS_FACTORED if args.jacobian == "factored" else B.IRL_WS_FP64
    else:
        ws_flags = B.IRL_WS_FP32 | (B.IRL_WS_FP64 if args.polish else 0)
    step_flags = (B.IRL_STEP_NO_EVAL_AFTER | (0 if args.polish else B.IRL_STEP_NO_POLISH)
                  | (B.IRL_STEP_GRAPH if args.graph else 0))
    if args.block > 1:
        ws_flags |= B.IRL_WS_BLOCK
    sysm.workspace(wl.P + 1, ws_flags)
    log(f"workspace {sysm.ws.numel() / 2**30:.2f} GiB")
    store = None
    if not sysm.info.full_space and not args.matrix_free:
        free = torch.cuda.mem_get_info()[0]
        t = time.perf_counter()
        stored, need = sysm.store_hamiltonian(max(0, free - (4 << 30)))
        store = {"stored": stored, "bytes": need, "ms": (time.perf_counter() - t) * 1e3}
        log(f"stored rows: {stored}, {need / 2**30:.2f} GiB, {store['ms']:.1f} ms")

    def one_step():
        rc, r, _, _ = sysm.step(theta, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12,
                                precision=precision, flags=step_flags,
                                ws_flags=ws_flags, want_dtheta=False, block=args.block)
        return rc, r

    ncols = wl.P + 1
    factored = bool(ws_flags & B.IRL_WS_FACTORED) and precision == B.IRL_FP64
    s_build = (8 if ws_flags & B.IRL_WS_FP64 else 0) + (4 if ws_flags & B.IRL_WS_FP32 else 0)
    stored_bytes = store["bytes"] if store and store["stored"] else 0

    # events over the warm-up steps name the dominant kernel class
    B.irl_stats_select(sysm.handle, None)
    B.irl_stats_enable(sysm.handle, args.warmup > 0 and not args.graph)
    for i in range(args.warmup):
        rc, r = one_step()
        log(f"warmup {i}: E={r.E_before:.12f} lambda={r.lambda_min:.3e} applies={r.n_apply} "
            f"restarts={r.n_restart} conv={r.converged} {r.ms_eval + r.ms_solve + r.ms_after:.1f} ms")
    warm = B.irl_stats_get(sysm.handle)
    B.irl_stats_enable(sysm.handle, False)
    theta.copy_(theta0)
    torch.cuda.synchronize()
    # Per-kernel events in the timed region: by default only around the dominant
    # class (each event pair costs a few microseconds of queue time per launch);
    # --all-events brackets every launch; none with graph replay (events would turn
    # the replay off) or --no-events.  Every class's times then come from an untimed
    # rerun of the same steps.
    live = select_live_kinds(args, B, warm, lambda k: kernel_roofline(k, ns, ncols, wl.H, factored, s_build,
                                                                       sysm.info, stored_bytes) is not None)
    events = bool(live)
    B.irl_stats_select(sysm.handle, live or None)
    B.irl_stats_enable(sysm.handle, events)
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        rc, r = one_step()
        step_ms = (time.perf_counter() - ts) * 1e3
        steps.append({"E": r.E_before, "lambda_min": r.lambda_min, "applies": r.n_apply,
                      "applies_fp32": r.n_apply_lo,
                      "restarts": r.n_restart, "converged": r.converged,
                      "residual_est": r.residual_est, "residual_explicit": r.residual_explicit,
                      "status": rc, "ms": step_ms})
        log(f"step {i}: E={r.E_before:.12f} lambda={r.lambda_min:.3e} applies={r.n_apply} "
            f"restarts={r.n_restart} conv={r.converged} {step_ms:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = B.irl_stats_get(sysm.handle)
    B.irl_stats_enable(sysm.handle, False)
    rerun = None
    if len(live) < len(B.STAT_KINDS):
        theta_end = theta.clone()
        theta.copy_(theta0)
        B.irl_stats_select(sysm.handle, None)
        B.irl_stats_enable(sysm.handle, True)
        for i in range(args.steps):
            one_step()
        rerun = B.irl_stats_get(sysm.handle)
        B.irl_stats_enable(sysm.handle, False)
        theta.copy_(theta_end)
        # live classes keep their timed-region figures
        stats = {k: (stats[k] if k in live else rerun[k]) for k in rerun}
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    applies = sum(s["applies"] for s in steps)
    # final energy after the last update
    Zf, Ef, _ = sysm.evaluate(wl.V, wl.H, theta, ws_flags=ws_flags, want_grad=False)
    warm_leg = warm_start_leg(args, B, sysm, wl, theta, theta0, precision, step_flags, ws_flags, steps, torch)

    # dominant kernel and its roofline (every kernel kind's beside it)
    kern = {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / v[1] if v[1] else None,
                "timed_live": k in live}
            for k, v in stats.items() if v[1]}
    if rerun is not None:
        for k in live:
            if k in kern and rerun[k][1]:
                kern[k]["ms_avg_untimed_rerun"] = rerun[k][0] / rerun[k][1]
    rooflines = {}
    for k, v in kern.items():
        spec = kernel_roofline(k, ns, ncols, wl.H, factored, s_build, sysm.info, stored_bytes)
        if spec is None:
            continue
        name, bound, work, unit, peak, src = spec
        scale = 1e9 if unit == "GB/s" else 1e12
        achieved = work / (v["ms_avg"] * 1e-3) / scale
        src_hash = source_hash([os.path.join(CSRC, f) for f in src])
        rooflines[name] = {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak,
                           "unit": unit, "frac": achieved / peak,
                           "traffic": read_traffic(name, wl.name, src_hash) if bound == "hbm" or
                           name == "ham_apply" else None,
                           ("bytes_per_launch" if unit == "GB/s" else "flops_per_launch"): work,
                           "ms_avg": v["ms_avg"], "ms_total": v["ms_total"], "launches": v["launches"],
                           "source_hash": src_hash}
    roof = max(rooflines.values(), key=lambda r: r["ms_total"]) if rooflines else None
    if len(live) == 1 and live[0] in kern:
        # the kernel whose launches were bracketed live in the timed region
        spec = kernel_roofline(live[0], ns, ncols, wl.H, factored, s_build, sysm.info, stored_bytes)
        roof = rooflines.get(spec[0], roof) if spec else roof
    # whole operator apply: K6 + K4 + K7 + reduction averages, against the HBM bytes the
    # kernels of one apply must move (the D~ copy streamed twice, or for the factored
    # Jacobian d and psi twice with w and u; the Hamiltonian's stored rows or, when it
    # enumerates, its input and output vectors)
    operator = {}
    ham_avg = kern["ham_apply"]["ms_avg"]
    red_avg = kern.get("reduce", {}).get("ms_avg") or 0.0
    ham_bytes = stored_alg_bytes(sysm.info, ns) if stored_bytes else 2 * 8 * ns
    for tag, g6, g7, sDo in (("fp64", "gemv", "gemv_t", 8), ("fp32", "gemv_fp32", "gemv_t_fp32", 4)):
        if g6 not in kern or g7 not in kern:
            continue
        apply_ms = kern[g6]["ms_avg"] + ham_avg + kern[g7]["ms_avg"] + red_avg
        if tag == "fp64" and factored:
            b6 = kernel_roofline(g6, ns, ncols, wl.H, True, s_build, sysm.info, stored_bytes)[2]
            b7 = kernel_roofline(g7, ns, ncols, wl.H, True, s_build, sysm.info, stored_bytes)[2]
            moved = b6 + b7 + ham_bytes
            operator["fp64_factored"] = {
                "applies": kern[g6]["launches"], "ms_per_apply": apply_ms,
                "bytes_per_apply": moved, "GBps": moved / (apply_ms * 1e-3) / 1e9,
                "frac_hbm": moved / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                "network_products_frac_hbm": (b6 + b7) / ((kern[g6]["ms_avg"] + kern[g7]["ms_avg"]) * 1e-3)
                / 1e9 / HBM_PEAK_GBPS,
                "dense_method_bytes_per_apply": 2 * ns * ncols * 8 + 6 * 8 * ns}
            continue
        moved = 2 * ns * ncols * sDo + 2 * 8 * ns + ham_bytes
        operator[tag] = {"applies": kern[g6]["launches"], "ms_per_apply": apply_ms,
                         "bytes_per_apply": moved, "GBps": moved / (apply_ms * 1e-3) / 1e9,
                         "frac_hbm": moved / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                         "stream_frac_hbm": (2 * ns * ncols * sDo) / ((kern[g6]["ms_avg"] + kern[g7]["ms_avg"]) * 1e-3)
                         / 1e9 / HBM_PEAK_GBPS}
    operator["ham_ms_per_apply"] = ham_avg
    operator["ham_candidates_per_s"] = ns * sysm.info.max_connections / (ham_avg * 1e-3)

    fp64_ref = None
    if precision == B.IRL_FP32 and args.fp64_reference:
        # the same first step from theta0 on the FP32 path and on the FP64 path
        def first_step(prec, fl, flags):
            th = theta0.clone()
            rc, r, _, _ = sysm.step(th, wl.V, wl.H, m=wl.m, k_keep=wl.k, tol=1e-12, precision=prec,
                                    flags=flags, ws_flags=fl, want_dtheta=False, block=args.block)
            return r
        r32 = first_step(precision, ws_flags, step_flags & ~B.IRL_STEP_NO_EVAL_AFTER)
        sysm.ws = None
        torch.cuda.empty_cache()
        t = time.perf_counter()
        r64 = first_step(B.IRL_FP64, B.IRL_WS_FP64 | (ws_flags & B.IRL_WS_BLOCK), 0)
        ms64 = (time.perf_counter() - t) * 1e3
        fp64_ref = {"ms_fp64_step": ms64, "applies_fp64": r64.n_apply,
                    "lambda_fp64": r64.lambda_min, "E_after_fp64": r64.E_after,
                    "dlambda": r32.lambda_min - r64.lambda_min, "dE_after": r32.E_after - r64.E_after}
        log(f"fp64 reference step: {ms64:.1f} ms, dlambda {fp64_ref['dlambda']:.3e}, "
            f"dE_after {fp64_ref['dE_after']:.3e}")

    fp32_op = None
    if precision == B.IRL_FP64 and args.config == "c3" and args.secondary:
        fp32_op = fp32_operator_comparison(args, B, sysm, wl, theta0, steps[0] if steps else None, torch)
    full_space = None
    if args.config == "c3" and args.secondary:
        sysm.ws = None
        torch.cuda.empty_cache()
        full_space = full_space_secondary(args, B, synth, System, torch)

    hbm_ref = measured_hbm_peak(torch)
    log(f"measured HBM reference: read {hbm_ref['read_GBps']:.0f} GB/s, copy {hbm_ref['copy_GBps']:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a row sample)")
        from oracle import space
        keys_fn = (lambda: space.full_space(wl.n, wl.na, wl.nb)) if dets is None else (lambda: dets)
        cpu = cpu_baseline(wl, keys_fn, applies_per_step=applies / args.steps)
        log(f"cpu baseline: {cpu['ms_per_step']:.0f} ms per step")

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "IRL steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if precision == B.IRL_FP64 else
                  "f32 operator / f64 solver" + (" + f64 polish" if args.polish else "")),
        "data": "synthetic",
        "config": {"workload": (f"{wl.name}: {wl.n} orbitals {wl.na}a+{wl.nb}b "
                                f"{'full space' if dets is None else 'selected set'} "
                                f"({ns} determinants), random molecule-like integrals seed {wl.seed}, "
                                f"one-hidden-layer tanh network V={wl.V} H={wl.H} (P={wl.P}), "
                                + (f"factored Jacobian (d {ns}x{wl.H} FP64, D~ {ns}x{ncols} never formed), "
                                   if factored else f"D~ {ns}x{ncols} {prec_name.upper()}, ")
                                + f"IRL m={wl.m} k_keep={wl.k} "
                                f"tol=1e-12" + (f", block Lanczos with {args.block} vectors per pass"
                                                if args.block > 1 else "")),
                   "n_dets": ns, "P": wl.P, "m": wl.m, "k_keep": wl.k, "block": args.block,
                   "graph_replay": bool(args.graph),
                   "kernel_events_in_timed_region": live if len(live) < len(B.STAT_KINDS) else "all",
                   "ham_kernel": HAM_KERNELS[sysm.info.ham_kernel]},
        "roofline": roof,
        "rooflines": rooflines,
        "cpu_baseline": cpu,
        "operator": operator,
        "kernels": kern,
        "applies_per_step": applies / args.steps,
        "setup_ms": setup_ms,
        "stored_rows": store,
        "hbm_reference": hbm_ref,
        "fp64_reference": fp64_ref,
        "fp32_operator": fp32_op,
        "full_space_12_orbitals": full_space,
        "trajectory": steps,
        "E_final": Ef,
        "warm_start": warm_leg,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
