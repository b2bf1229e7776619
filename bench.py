#!/usr/bin/env python3
"""Throughput of the LLG hot path on one MI355X.

A timed step is one classical RK4 step forward plus its reverse (adjoint)
through the checkpointed rollout (checkpoint every 10 steps: the forward
sweep, then per segment a taped re-run and the reverse sweep), in float32,
on the 512x512x32 demag-dominated workload (2.5 nm cells, Ms 8e5, A 1.3e-11,
alpha 0.5, seeded smoothed random start; the loss seed is the gradient of
the masked mean of m_z).  Inputs are resident in HBM before the timed
region.  Prints one JSON line.

Also reported, outside the timed region:
* the live roofline of the dominant kernel (HIP events on its stream) and
  the whole step's fraction under the algorithmic bytes model;
* per workload (film 128x32x1, dmi 256x256x16, demag 512x512x32, adjoint
  256x256x8, large 1024x1024x64): H_eff Mcells/s and RK4 steps/s in float32
  and float64 with their fractions of the HBM roofline under the bytes model,
  the errors of H_eff and of one step against the FP64 oracle (stored values
  at seeded cells, written by tests/golden/make_workload_golden.py), float32
  against float64 after the workload's N steps, the adjoint workload's
  gradient against the oracle's, the large workload's forward+adjoint rate,
  and the FP64 oracle's own rates on a sample of each workload;
* the Standard Problem 4 integrator comparison and the batched film;
* the FP64 CPU oracle timed on a bounded sample of the headline workload.
"""
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

METRIC = "H_eff Mcells/s + RK4 steps/s, FP32 vs FP64 at stated err, 512×512×32; fwd+bwd"
PEAK_HBM_GBS = 8000.0
DOMINANT = "zconv"          # largest share of GPU time in the timed step (rocprofv3 summary)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "zconv_demag512_traffic.txt")


def kernel_bytes(kind, n, es):
    """Algorithmic HBM bytes of one launch of a kernel family (compulsory
    reads and writes of its inputs/outputs; zero padding never touched)."""
    nx, ny, nz = n
    Px = max(2, 1 << (2 * nx - 1).bit_length())
    Py = max(2, 1 << (2 * ny - 1).bit_length())
    Pz = max(2, 1 << (2 * nz - 1).bit_length())
    Hx, Hy, Hz = Px // 2 + 1, Py // 2 + 1, Pz // 2 + 1
    N = nx * ny * nz
    cx = 2 * es
    x1 = 3 * nz * ny * Hx * cx          # half spectrum after the x pass
    x2 = 3 * nz * Py * Hx * cx          # after the y pass
    tensor = 6 * Hz * Hy * Hx * es      # octant of the real spectrum
    if kind == "zconv":
        return 2 * x2 + tensor
    if kind in ("yfwd", "yinv"):
        return x1 + x2
    if kind == "xfwd":
        return 3 * N * es + x1
    raise ValueError(kind)


def stage_bytes(s, taped=False):
    """Algorithmic bytes per cell of one RK4 stage kernel (float32): inverse x
    pass input 24, stage input 12 (+ m_n and the accumulator 12 each from
    s = 2), outputs accumulator 12 (s < 4), next input 12, forward x pass 24;
    a taped stage also writes H 12 and |x| 4, stage 1 a copy of y 12, stage 4
    a copy of the new state 12."""
    b = 24 + 12 + (24 if s > 1 else 0) + (12 if s < 4 else 0) + 12 + 24
    if taped:
        b += 16 + (12 if s in (1, 4) else 0)
    return b


def bstage_bytes(s):
    """Reverse stage (float32): reads Y1 24, mu (stencil) 12, y_s 12, H_s 12,
    kappa 12, lambda 12 (+ |x_s| 4, xi_5 12, y_{s-1} 12 from s = 2); writes
    lambda 12 (+ kappa 12, mu_{s-1} 12, forward x pass 24 from s = 2)."""
    return 84 + 12 + ((4 + 12 + 12) + (12 + 12 + 24) if s > 1 else 0)


BSTART_BYTES = 12 + 12 + 12 + 4 + 12 + 12 + 12 + 12 + 24   # reads gm, y4, y5, |x5|; writes xi5, gm, kappa, mu, X1
CONV_BYTES = 72 + 120 + 72                                  # y forward, z pass with the product, y inverse


def model_bytes_per_cell(kind):
    """Algorithmic HBM bytes per cell (float32; float64 doubles them):
    heff: x forward 36 + convolution 264 + inverse x pass with the local
    field 48 = 348; rk4: one step of four stages and four convolutions;
    fwdbwd: one checkpointed forward+adjoint step (forward step, taped
    re-run, reverse start and four reverse stages with a convolution each)."""
    if kind == "heff":
        return 36 + CONV_BYTES + 48
    fwd = 4 * CONV_BYTES + sum(stage_bytes(s) for s in (1, 2, 3, 4))
    if kind == "rk4":
        return fwd
    taped = 4 * CONV_BYTES + sum(stage_bytes(s, True) for s in (1, 2, 3, 4))
    rev = BSTART_BYTES + 4 * CONV_BYTES + sum(bstage_bytes(s) for s in (1, 2, 3, 4))
    return fwd + taped + rev


def source_hash():
    h = hashlib.sha256()
    for f in ("conv.hip", "magx_common.hpp"):
        with open(os.path.join(ROOT, "paper_2602_12242_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, or None if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_launch")


def err_norm(a, b):
    import torch
    a = a.double()
    b = b.double()
    num = torch.sqrt(((a - b) ** 2).sum(0)).max()
    den = torch.sqrt((b ** 2).sum(0)).max()
    return float(num / den)


def cpu_baseline(w, budget_cells=(128, 128, 32)):
    """FP64 oracle, one forward+adjoint RK4 step on a sub-box of the workload
    (same cells and material), scaled to the full box by cell count."""
    import numpy as np

    from oracle import adjoint as oadj
    from oracle import llg as ollg
    from oracle import newell as onewell
    from oracle.params import Grid, Params
    from workloads import random_unit_field

    n = budget_cells
    g = Grid(*n, *w.d)
    mat = w.material()
    p = Params(**{k: mat[k] for k in ("Ms", "A", "D", "Ku", "eK", "Hbias", "alpha", "terms", "renorm")})
    spec = onewell.spectrum(g)
    m = random_unit_field(n, w.seed, w.smooth).astype(np.float32).astype(np.float64)
    lam = np.zeros_like(m)
    lam[2] = 1.0 / m[2].size
    # steps of the sample: repeat until about 10 s of CPU work (at most 20)
    steps = 0
    t0 = time.perf_counter()
    while True:
        m1 = ollg.rk4_step(g, p, m, w.dt, spec)           # forward sweep
        oadj.rk4_step_vjp(g, p, m, w.dt, lam, spec)       # taped re-run + reverse
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= 10.0 or steps >= 20:
            break
        m = m1
    sub = n[0] * n[1] * n[2]
    rate = (steps / dt) * sub / w.ncell
    return {"value": rate, "unit": "steps/s", "cores": onewell._workers(), "kind": "oracle",
            "sample": f"{steps} fwd+bwd RK4 steps on a {n[0]}x{n[1]}x{n[2]} sub-box of the workload "
                      f"({dt:.1f} s), scaled by cell count {sub}/{w.ncell}"}


GOLDEN = os.path.join(ROOT, "tests", "golden")
SAMPLED = {"film": "film_sampled.npz", "dmi": "dmi256_sampled.npz", "demag": "demag512_sampled.npz",
           "adjoint": "adjoint256_sampled.npz"}
NSTEP_DRIFT = {"dmi": 1000, "demag": 200, "large": 50}


def _sampled_errors(gold, H, m1):
    """Normwise H_eff error (denominator max |H| over every cell, stored) and
    absolute one-step error at the stored oracle cells."""
    import numpy as np
    x, y, z = (_cuda_index(v) for v in gold["cells"].T)
    Hs = H[:, z, y, x].T.double().cpu().numpy()
    ms = m1[:, z, y, x].T.double().cpu().numpy()
    eh = float(np.sqrt(((Hs - gold["H"]) ** 2).sum(1)).max() / float(gold["hmax"]))
    em = float(np.abs(ms - gold["m1"]).max())
    return eh, em


def _cuda_index(v):
    import torch
    return torch.from_numpy(v.astype("int64")).cuda()


def oracle_rates(w, max_cells=(128, 128)):
    """FP64 oracle H_eff and one RK4 step timed on a sub-box of the workload
    (at most 128 x 128 cells per layer, all layers), scaled by cell count."""
    import numpy as np

    from oracle import field as ofield
    from oracle import llg as ollg
    from oracle import newell as onewell
    from oracle.params import Grid, Params
    from workloads import random_unit_field

    n = (min(w.n[0], max_cells[0]), min(w.n[1], max_cells[1]), w.n[2])
    g = Grid(*n, *w.d)
    mat = w.material()
    p = Params(**{k: mat[k] for k in ("Ms", "A", "D", "Ku", "eK", "Hbias", "alpha", "terms", "renorm")})
    spec = onewell.spectrum(g)
    m = random_unit_field(n, w.seed, w.smooth).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    ofield.heff(g, p, m, spec)
    t1 = time.perf_counter()
    ollg.rk4_step(g, p, m, w.dt, spec)
    t2 = time.perf_counter()
    sub = n[0] * n[1] * n[2]
    return {"heff_mcells_per_s": round(sub / (t1 - t0) / 1e6, 3),
            "rk4_steps_per_s": round(sub / w.ncell / (t2 - t1), 5),
            "cores": onewell._workers(),
            "sample": f"one H_eff and one RK4 step on {n[0]}x{n[1]}x{n[2]} cells, scaled by cell count"}


CONFIG_NAMES = ("film", "dmi", "demag", "adjoint", "large")


def _reps_for(fn, seconds, lo=3, hi=5000):
    """Repetitions of fn that take about `seconds` (one call timed after a warm-up)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - a, 1e-7)
    return int(max(lo, min(hi, seconds / one)))


def config_measurements(magx, torch, timeit, names=CONFIG_NAMES, oracle=True):
    """Every workload in float32 and float64: rates, roofline fractions under
    the bytes model, errors against the oracle and between precisions."""
    import numpy as np

    from workloads import WORKLOADS, bernoulli_mask, initial_state, tangent_direction
    out = {}
    hb = model_bytes_per_cell("heff")
    rb = model_bytes_per_cell("rk4")
    for name in names:
        w = WORKLOADS[name]
        N = w.ncell
        p = magx.make_params(**w.material())
        m0 = torch.from_numpy(initial_state(w, np.float32)).cuda()
        gold = np.load(os.path.join(GOLDEN, SAMPLED[name])) if name in SAMPLED else None
        rec = {"cells": N, "grid": "x".join(str(v) for v in w.n), "dt_s": w.dt}
        res = {}
        for dt_name, dt_code in (("f64", magx.F64), ("f32", magx.F32)):
            es = 8 if dt_code == magx.F64 else 4
            ctx = magx.Context(w.n, w.d, dt_code)
            m = m0.to(ctx.tdtype)
            H = ctx.field()
            # repetitions for about 50 ms of calls (at least 3): a film's call
            # lasts tens of microseconds, so a few calls would time the host;
            # the best of three such runs, since a film's host-bound calls slow
            # down while other work (the oracle timing before) still holds cores
            rh = _reps_for(lambda: ctx.heff(m, p, out=H), 0.05)
            t_h = min(timeit(lambda: ctx.heff(m, p, out=H), rh) for _ in range(3))
            y = m.clone()
            nst = 2 if name == "large" else 5
            rs = _reps_for(lambda: ctx.step(y, p, w.dt, nst), 0.05)
            t_s = min(timeit(lambda: ctx.step(y, p, w.dt, nst), rs) for _ in range(3)) / nst
            m1 = m.clone()
            ctx.step(m1, p, w.dt, 1)
            H = ctx.heff(m, p)
            r = {"heff_mcells_per_s": round(N / t_h / 1e6, 1), "rk4_steps_per_s": round(1.0 / t_s, 2),
                 "heff_model_frac": round(hb * (es // 4) * N / t_h / 1e9 / PEAK_HBM_GBS, 4),
                 "rk4_model_frac": round(rb * (es // 4) * N / t_s / 1e9 / PEAK_HBM_GBS, 4)}
            if gold is not None:
                eh, em = _sampled_errors(gold, H, m1)
                r["err_heff_vs_oracle"] = eh
                r["err_m_1step_vs_oracle"] = em
            res[dt_name] = (r, H.double().cpu(), m1.double().cpu())
            if name in NSTEP_DRIFT:
                mN = m.clone()
                ctx.step(mN, p, w.dt, NSTEP_DRIFT[name])
                res[dt_name] = res[dt_name] + (mN.double().cpu(),)
            del ctx, H, y, m1, m
            torch.cuda.empty_cache()
        r64, H64, m64 = res["f64"][:3]
        r32, H32, m32 = res["f32"][:3]
        rec["f32"], rec["f64"] = r32, r64
        rec["err_heff_f32_vs_f64"] = err_norm(H32, H64)
        rec["err_m_1step_f32_vs_f64"] = float((m32 - m64).abs().max())
        if name in NSTEP_DRIFT:
            rec[f"err_m_{NSTEP_DRIFT[name]}steps_f32_vs_f64"] = float((res["f32"][3] - res["f64"][3]).abs().max())
        if name == "adjoint":
            g = np.load(os.path.join(GOLDEN, "adjoint256_grad.npz"))
            ctx = magx.Context(w.n, w.d, magx.F32)
            mask = torch.from_numpy(bernoulli_mask(w.n, w.extra["mask_seed"])).cuda().float()
            store = ctx.checkpoint_store(w.steps, w.ckpt)
            tape = ctx.tape(w.ckpt)
            mwork = ctx.field()
            mm = m0.clone()
            gm = ctx.field()

            def fb():
                mm.copy_(m0)
                ctx.rollout_forward(mm, p, w.dt, w.steps, w.ckpt, store)
                gm.zero_()
                gm[2] = mask / mask.sum()
                return ctx.rollout_backward(store, p, w.dt, w.steps, w.ckpt, gm, tape=tape, mwork=mwork)[1]

            t_fb = timeit(fb, 2)
            gh = fb()
            torch.cuda.synchronize()
            m0d = m0.double().cpu().numpy()
            proj = np.array([float((gm.double().cpu().numpy() * tangent_direction(m0d, int(sd))).sum())
                             for sd in g["seeds"]])
            rec["fwdbwd_f32"] = {"steps": w.steps, "checkpoint": w.ckpt,
                                 "steps_per_s": round(w.steps / t_fb, 2),
                                 "model_frac": round(model_bytes_per_cell("fwdbwd") * N * w.steps / t_fb / 1e9
                                                     / PEAK_HBM_GBS, 4),
                                 "err_grad_vs_oracle": float(np.linalg.norm(proj - g["proj"]) / np.linalg.norm(g["proj"])),
                                 "err_dHbias_vs_oracle": float(np.linalg.norm(gh.double().cpu().numpy() - g["gHbias"])
                                                               / np.linalg.norm(g["gHbias"])),
                                 "directions": int(len(g["seeds"]))}
            del ctx, store, tape, mwork, gm
            torch.cuda.empty_cache()
        if name == "large":
            ctx = magx.Context(w.n, w.d, magx.F32)
            store = ctx.checkpoint_store(w.steps, w.ckpt)
            tape = ctx.tape(w.ckpt)
            mwork = ctx.field()
            mm = m0.clone()
            gm = ctx.field()
            mask = torch.from_numpy(bernoulli_mask(w.n, w.extra["mask_seed"])).cuda().float()

            def fb():
                mm.copy_(m0)
                ctx.rollout_forward(mm, p, w.dt, w.steps, w.ckpt, store)
                gm.zero_()
                gm[2] = mask / mask.sum()
                ctx.rollout_backward(store, p, w.dt, w.steps, w.ckpt, gm, tape=tape, mwork=mwork)

            t_fb = timeit(fb, 1)
            gb = model_bytes_per_cell("fwdbwd") * N * w.steps / t_fb / 1e9
            rec["fwdbwd_f32"] = {"steps": w.steps, "checkpoint": w.ckpt, "seconds": round(t_fb, 3),
                                 "steps_per_s": round(w.steps / t_fb, 2), "model_GBps": round(gb, 1),
                                 "model_frac": round(gb / PEAK_HBM_GBS, 4)}
            del ctx, store, tape, mwork, gm, mm
            torch.cuda.empty_cache()
        if oracle:
            rec["oracle"] = oracle_rates(w)
        out[name] = rec
    return out


def integrator_comparison(magx, torch, timeit):
    """Standard Problem 4 film at 0.78125 nm (640x160x4, FP32): time to cover
    one 1.25e-13 s interval with RK4 (5 steps of 2.5e-14 s, 20 field
    evaluations) and with the multirate method (1 step, 3 field evaluations
    and 36 exchange-only stages), and each one's deviation from a fine RK4
    reference (100 steps of 1.25e-15 s)."""
    import numpy as np

    from workloads import WORKLOADS, initial_state
    w = WORKLOADS["sp4_fine"]
    ctx = magx.Context(w.n, w.d, magx.F32)
    p = magx.make_params(**w.material())
    m0 = torch.from_numpy(initial_state(w, np.float32)).cuda()
    a, b, ref = ctx.field(), ctx.field(), ctx.field()
    T = w.extra["interval"]
    t_rk4 = timeit(lambda: (a.copy_(m0), ctx.step(a, p, w.dt, w.steps)), 10)
    t_mri = timeit(lambda: (b.copy_(m0), ctx.step_mri(b, p, w.extra["dt_mri"], 1, w.extra["dt_fast"])), 10)
    ref.copy_(m0)
    ctx.step(ref, p, T / 100, 100)
    torch.cuda.synchronize()
    return {"cells": w.ncell, "interval_s": T,
            "rk4_ms": round(1e3 * t_rk4, 4), "mri_ms": round(1e3 * t_mri, 4),
            "rk4_field_evals": 4 * w.steps, "mri_field_evals": 3, "mri_exchange_stages": 36,
            "err_rk4_vs_fine": float((a - ref).abs().max()), "err_mri_vs_fine": float((b - ref).abs().max()),
            "paper_gv100_time_to_solution_s": {"rk4": 0.133, "mri": 0.069}}


def batched_throughput(magx, torch, timeit, B=16, steps=10):
    """B independent film systems (128x32x1) advanced as one batch versus one
    after another through a single-system context: member-steps per second."""
    import numpy as np

    from workloads import WORKLOADS, random_unit_field
    w = WORKLOADS["film"]
    p = magx.make_params(**w.material())
    single = magx.Context(w.n, w.d, magx.F32)
    batch = magx.Context(w.n, w.d, magx.F32, nbatch=B)
    ms = torch.from_numpy(np.stack([random_unit_field(w.n, 5000 + b, 3) for b in range(B)])).to(
        "cuda", torch.float32).contiguous()
    mb = ms.clone()
    one = ms[0].clone()
    t_batch = timeit(lambda: batch.step(mb, p, w.dt, steps), 5)
    t_single = timeit(lambda: single.step(one, p, w.dt, steps), 5)
    return {"members": B, "cells_per_member": w.ncell, "steps": steps,
            "batched_member_steps_per_s": round(B * steps / t_batch, 1),
            "sequential_member_steps_per_s": round(steps / t_single, 1)}


def _pmc_rows(path, counter):
    """(kernel name, value) per dispatch from a rocprofv3 result: a rocpd
    SQLite database (*_results.db) or a counter_collection.csv."""
    rows = []
    if path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(path)
        for name, cn, cv in con.execute("select name, counter_name, counter_value from pmc_events"):
            if cn == counter:
                rows.append((name, float(cv)))
        return rows
    import csv
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == counter:
                rows.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return rows


def trace_summary(db, out_path, title, command):
    """Writes a kernel-time summary (rocprofv3 --kernel-trace --stats result)."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                            "order by total_duration desc"))
    lines = ["# rocprofv3 kernel trace: " + title, "",
             "command: `" + command + "`", "",
             "| kernel | calls | total ms | mean us | share % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| {short} | {calls} | {tot / 1e3:.3f} | {avg:.1f} | {pct:.1f} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def pmc_summarize(fetch_csv, write_csv, command):
    """HBM bytes per launch of the dominant kernel from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    library's plain copy kernel moving a known 12N bytes each way."""
    from workloads import WORKLOADS
    N = WORKLOADS["demag"].ncell
    known = 12.0 * N
    out = {"kernel": DOMINANT, "workload": "demag 512x512x32 FP32", "source_hash": source_hash(),
           "command": command}
    total = 0.0
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _pmc_rows(path, counter)
        copy = [v * 1024.0 for k, v in rows if "magx::copy_kernel" in k]
        dom = [v * 1024.0 for k, v in rows if re.search(r"magx::" + DOMINANT + r"\w*_kernel", k)]
        if not copy or not dom:
            raise SystemExit(f"{path}: no {counter} rows for copy_kernel / {DOMINANT}_kernel")
        factor = known / (sum(copy) / len(copy))
        per = factor * sum(dom) / len(dom)
        out[f"{label}_raw_bytes_per_launch"] = sum(dom) / len(dom)
        out[f"{label}_calibration_factor"] = factor
        out[f"{label}_bytes_per_launch"] = per
        total += per
    out["bytes_per_launch"] = total
    out["algorithmic_bytes_per_launch"] = kernel_bytes(DOMINANT, WORKLOADS["demag"].n, 4)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc-summarize":
        pmc_summarize(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--trace-summarize":
        trace_summary(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64/H_eff side measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", choices=CONFIG_NAMES, default=None,
                    help="measure this workload alone (no headline step; for profiling runs)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: magx runs on one GPU; the decomposition over several GPUs (z slabs with two "
              "all-to-all exchanges per H_eff) is designed but not implemented, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2602_12242_amd import magx
    from workloads import WORKLOADS, bernoulli_mask, initial_state

    def timeit(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps

    if args.config:
        torch.cuda.set_device(0)
        print(json.dumps({"configs": config_measurements(magx, torch, timeit, (args.config,), oracle=False)}),
              flush=True)
        return

    w = WORKLOADS["demag"]
    n, d = w.n, w.d
    N = w.ncell
    ckpt = w.ckpt
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m0_host = initial_state(w, np.float32)
    mask = bernoulli_mask(n, 2004)
    seed_host = np.zeros((3,) + mask.shape, dtype=np.float64)
    seed_host[2] = mask / mask.sum()

    ctx = magx.Context(n, d, magx.F32)
    p = magx.make_params(**w.material())
    m0 = torch.from_numpy(m0_host).to(dev)
    gseed = torch.from_numpy(seed_host).to(dev, torch.float32)
    store = ctx.checkpoint_store(args.steps, ckpt)
    tape = ctx.tape(min(ckpt, args.steps))
    mwork = ctx.field()
    m = ctx.field()
    gm = ctx.field()

    def fwd_bwd(k):
        m.copy_(m0)
        ctx.rollout_forward(m, p, w.dt, k, ckpt, store)
        gm.copy_(gseed)
        _, gh = ctx.rollout_backward(store, p, w.dt, k, ckpt, gm, tape=tape, mwork=mwork)
        return gh

    for _ in range(max(0, args.warmup)):
        fwd_bwd(1)
    torch.cuda.synchronize()

    ctx.profile_start(DOMINANT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd_bwd(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kern_ms = ctx.profile_stop()
    T = t1 - t0
    value = args.steps / T
    step_bytes = model_bytes_per_cell("fwdbwd") * N * args.steps

    avg_ms = kern_ms / max(launches, 1)
    algo = kernel_bytes(DOMINANT, n, 4)
    achieved = algo / (avg_ms * 1e-3) / 1e9
    traffic = traffic_per_launch()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": DOMINANT,
                "algorithmic_bytes_per_launch": algo, "avg_launch_ms": round(avg_ms, 5), "launches": launches}

    extras = {}
    if not args.no_extras:
        # practical bandwidth of the passes' access patterns on this device:
        # plain copy, and in-place read + write with the z and y tilings
        probe = {}
        for kind, label in ((0, "copy"), (1, "z_tiling"), (2, "y_tiling")):
            nbytes = ctx.memory_probe(kind)
            t = timeit(lambda: ctx.memory_probe(kind), 10)
            probe[label + "_GBps"] = round(nbytes / t / 1e9, 1)
        roofline["pattern_ceilings"] = probe
        del store, tape, mwork
        torch.cuda.empty_cache()
        extras["configs"] = config_measurements(magx, torch, timeit)
        extras["sp4_fine_interval"] = integrator_comparison(magx, torch, timeit)
        extras["batched_film"] = batched_throughput(magx, torch, timeit)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * T / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "demag 512x512x32 cells of 2.5 nm, FP32, checkpointed (every 10) "
                               "forward+adjoint RK4 step, dt 1e-13 s",
                   "cells": N, "checkpoint": ckpt, "dt_s": w.dt},
        "roofline": roofline,
        "step_model": {"bytes_per_cell": model_bytes_per_cell("fwdbwd"),
                       "GBps": round(step_bytes / T / 1e9, 1),
                       "frac": round(step_bytes / T / 1e9 / PEAK_HBM_GBS, 4)},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
