"""Throughput of the fused Reg-FLBM D3Q27 step on one MI355X.

Workload (fixed): 512^3 periodic box, rho0 = 1, tau = 0.6 (all hydrodynamic
modes), ghosts at tau = 1, kT = 1e-5, Philox4x32-7 noise, Taylor-Green initial
velocity of amplitude 0.01, FP32 population storage.  One step = one fused
stream + collide kernel over the whole box.  The populations are resident in
HBM before the timed region starts.

Prints one JSON line: MLUPS (million lattice updates per second), the HBM
roofline of the step kernel, the CPU oracle baseline on a bounded sample, and
extra figures (FP16/BF16 storage, deterministic Reg-LBM, copy-kernel ceiling).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS at 512^3 D3Q27 + % HBM roofline; FP16-store vs FP32 at ≤1% "
          "⟨u²⟩ error")
PEAK_HBM_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 216, "f16": 108, "bf16": 108}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_f32_512_traffic.txt")
KERNEL_SOURCES = ["paper_2507_08820_amd/csrc/step.hip", "paper_2507_08820_amd/csrc/node_body.inc",
                  "paper_2507_08820_amd/csrc/d3q27.hpp", "paper_2507_08820_amd/csrc/philox.hpp",
                  "paper_2507_08820_amd/csrc/storage.hpp", "paper_2507_08820_amd/csrc/kernels.hpp",
                  "paper_2507_08820_amd/csrc/fastdiv.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(dims, storage, kT, steps, warmup, tau=0.6, stats_every=0, followups=()):
    """Times `steps` steps of one lattice after `warmup` steps.  Each follow-up
    (label, kT, stats_every, steps) is then timed on the same lattice (the same
    placement in HBM, so the comparison with the main figure is fair)."""
    import torch

    import paper_2507_08820_amd as rf
    import workloads as wl

    kw = dict(storage=storage, kT=kT, tau=tau, tau_bulk=tau, tau_ghost=1.0, seed=3)
    lat = rf.Lattice(dims, **kw)
    rho, u = wl.taylor_green_device(dims, amp=0.01, device=lat.device)
    lat.init_equilibrium(rho, u)
    del rho, u
    lat.stats_config(stats_every)
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = lat.time_steps(steps)  # HIP events on the lattice's stream around the K launches
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.sync()
    n = dims[0] * dims[1] * dims[2]
    r = dict(ms=ms, wall_s=wall, mlups=n * steps / (ms * 1e-3) / 1e6, ms_per_step=ms / steps, followups={})
    log(f"{dims} {storage} kT={kT}{f' stats every {stats_every}' if stats_every else ''}: {steps} steps, "
        f"{r['ms_per_step']:.4f} ms/step, {r['mlups']:.0f} MLUPS")
    for label, f_kT, f_stats, f_steps in followups:
        f_kw = dict(kw, kT=f_kT)
        if storage != "f32" and f_kT == 0.0:
            # keep the storage unit the noisy run derived from k_BT, sqrt(rho0 kT / cs2)
            f_kw["storage_scale"] = (3.0 * kT) ** 0.5
        lat.set_params(**f_kw)
        lat.stats_config(f_stats)
        lat.step(2)
        f_ms = lat.time_steps(f_steps)
        lat.sync()
        r["followups"][label] = dict(ms_per_step=f_ms / f_steps, mlups=n * f_steps / (f_ms * 1e-3) / 1e6)
        log(f"  same lattice, {label}: {f_ms / f_steps:.4f} ms/step, {r['followups'][label]['mlups']:.0f} MLUPS")
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return r


def precision_study(dims=(128, 128, 128), kts=(1e-4, 1e-5, 1e-6), steps=400, every=2):
    """<u^2> / (kT / rho0) for FP32, FP16 and BF16 storage with the same seed
    (the same noise), thermalised start, tau = 0.6: the FP16/BF16 deviation from
    FP32 isolates the storage precision."""
    import numpy as np
    import torch

    import paper_2507_08820_amd as rf

    out = {}
    for kT in kts:
        row = {}
        for storage in ("f32", "f16", "bf16"):
            lat = rf.Lattice(dims, storage=storage, kT=kT, tau=0.6, seed=21)
            lat.init_thermal()
            lat.stats_config(every)
            lat.step(steps)
            st = lat.stats()
            lat.close()
            n = st["samples"] * st["nodes"]
            row[storage] = float(np.sum(st["sum_u2"]) / n / (3 * kT))
        row["f16_minus_f32"] = row["f16"] - row["f32"]
        row["bf16_minus_f32"] = row["bf16"] - row["f32"]
        out[f"kT={kT:g}"] = {k: round(v, 6) for k, v in row.items()}
        log(f"precision kT={kT:g}: {out[f'kT={kT:g}']}")
    torch.cuda.empty_cache()
    return out


def precision_full(dims=(512, 512, 512), kts=(1e-4, 1e-5, 1e-6), steps=1000, every=10, sk_every=100):
    """The storage-precision form on the benchmark workload: thermal
    fluctuations on the Taylor-Green flow (A = 0.01), tau = 0.6, ghosts at 1,
    the same seed (the same noise) for FP32, FP16 and BF16 storage.  Per kT:
    <u^2> (flow plus fluctuations) and the momentum S(|n|) / (3 rho0 kT) on
    shells 4..64 (away from the Taylor-Green modes), and the 16-bit storages'
    differences from FP32."""
    import numpy as np
    import torch

    import paper_2507_08820_amd as rf
    import workloads as wl

    out = {}
    for kT in kts:
        res = {}
        for storage in ("f32", "f16", "bf16"):
            lat = rf.Lattice(dims, storage=storage, kT=kT, tau=0.6, tau_bulk=0.6, tau_ghost=1.0, seed=3)
            rho, u = wl.taylor_green_device(dims, amp=0.01, device=lat.device)
            lat.init_thermal(rho, u)
            del rho, u
            lat.stats_config(every)
            for _ in range(steps // sk_every):
                lat.sk_sample()
                lat.step(sk_every)
            st = lat.stats()
            n = st["samples"] * st["nodes"]
            js = sum(lat.sk(f)[0] for f in ("jx", "jy", "jz"))
            _, counts, ns = lat.sk("jx")
            lat.sync()
            lat.close()
            del lat
            torch.cuda.empty_cache()
            res[storage] = dict(u2=float(np.sum(st["sum_u2"]) / n),
                                sk=js[4:65] / counts[4:65] / ns / (3 * kT))
        row = {"u2_f32": res["f32"]["u2"], "sk_mean_f32": float(np.mean(res["f32"]["sk"]))}
        for s16 in ("f16", "bf16"):
            row[f"u2_rel_diff_{s16}"] = (res[s16]["u2"] - res["f32"]["u2"]) / res["f32"]["u2"]
            row[f"sk_max_abs_diff_{s16}"] = float(np.max(np.abs(res[s16]["sk"] - res["f32"]["sk"])))
        out[f"kT={kT:g}"] = {k: float(f"{v:.6g}") for k, v in row.items()}
        log(f"precision 512^3 kT={kT:g}: {out[f'kT={kT:g}']}")
    return {"box": list(dims), "steps": steps, "stats_every": every, "sk_every": sk_every,
            "start": "thermal fluctuations on Taylor-Green A=0.01", "rows": out}


def run_batch(storage, steps=2000, sep_steps=200, graph_steps=20, stats_steps=2000, stats_every=10):
    """The 64-replica workload: boxes 32^3..96^3, tau in [0.55, 1.2], kT in
    [1e-6, 1e-4], Taylor-Green A = 0.01 per box; aggregate MLUPS of the
    persistent hipGraph-replayed launch over `steps` steps and of one launch
    per replica over `sep_steps`.  Then equipartition of the batched form:
    every replica restarted from thermal fluctuations at rest and run
    `stats_steps` batched steps with statistics every `stats_every` steps;
    ER(u^2) = <u^2> / (3 kT / rho0) and ER(rho) = <d rho^2> / (rho0 kT / cs2)
    per replica."""
    import numpy as np
    import torch

    import paper_2507_08820_amd as rf
    import workloads as wl

    table = wl.replica_table(64, seed=5)
    reps = [dict(dims=t["dims"], kT=t["kT"], tau=t["tau"], seed=t["seed"], stream_id=t["stream_id"])
            for t in table]
    b = rf.Batch(reps, storage=storage)
    for r, t in enumerate(table):
        rho, u = wl.taylor_green_device(t["dims"], amp=0.01, device=b.device)
        b[r].init_equilibrium(rho, u)
    b.set_launch(256, 8, graph_steps)
    tile, bpc, _ = b.autotune(trial_steps=10)
    b.set_launch(tile, bpc, graph_steps)
    b.step(graph_steps)
    b.sync()
    ms = b.time_steps(steps)
    b.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step_separate(sep_steps)
    e1.record()
    torch.cuda.synchronize()
    ms_sep = e0.elapsed_time(e1)
    b.sync()
    n = b.nodes
    out = {"replicas": len(reps), "nodes": n, "tile": tile, "blocks_per_cu": bpc,
           "graph_steps": graph_steps, "steps": steps,
           "mlups_persistent_graph": round(n * steps / (ms * 1e-3) / 1e6, 1),
           "mlups_one_launch_per_replica": round(n * sep_steps / (ms_sep * 1e-3) / 1e6, 1)}
    out["gain"] = round(out["mlups_persistent_graph"] / out["mlups_one_launch_per_replica"], 3)
    # equipartition of every replica in the batched form
    for r in range(len(reps)):
        b[r].init_thermal()
    b.stats_config(stats_every)
    b.step(stats_steps)
    b.sync()
    er_u2, er_rho = [], []
    for r, t in enumerate(table):
        st = b[r].stats()
        m = st["samples"] * st["nodes"]
        er_u2.append(float(np.sum(st["sum_u2"]) / m / (3 * t["kT"])))
        var_rho = st["sum_drho2"] / m - (st["sum_drho"] / m) ** 2
        er_rho.append(float(var_rho / (3 * t["kT"])))
    er_u2, er_rho = np.array(er_u2), np.array(er_rho)
    out["equipartition"] = {
        "steps": stats_steps, "stats_every": stats_every, "start": "thermal fluctuations at rest",
        "er_u2_mean": round(float(er_u2.mean()), 5), "er_u2_min": round(float(er_u2.min()), 5),
        "er_u2_max": round(float(er_u2.max()), 5),
        "er_rho_mean": round(float(er_rho.mean()), 5), "er_rho_min": round(float(er_rho.min()), 5),
        "er_rho_max": round(float(er_rho.max()), 5),
        "max_abs_error": round(float(max(np.abs(er_u2 - 1).max(), np.abs(er_rho - 1).max())), 5)}
    log(f"batch {storage}: {out}")
    b.close()
    torch.cuda.empty_cache()
    return out


TABLE3_TAUS = (0.5001, 0.5005, 0.501, 0.505, 0.51, 0.55, 0.7, 1.0, 1.5, 2.0, 5.0, 10.0, 50.0, 100.0)
TABLE3_FILE = os.path.join(ROOT, "tests", "golden", "table3_er.txt")


def paper_table3():
    """Table III as printed: {(model, tau): [ER(rho), ER(sum rho u), ER(sum Pi_aa),
    ER(sum Pi_ab)]}, models "reg" and "bgk" (BGK only where the paper prints it)."""
    out = {}
    with open(TABLE3_FILE) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [float(t) for t in line.split()]
            out[("reg", v[0])] = v[1:5]
            if all(x == x for x in v[5:9]):  # not nan
                out[("bgk", v[0])] = v[5:9]
    return out


def table3_run(dims=(256, 256, 256), taus=TABLE3_TAUS, bgk_taus=(0.5005,) + TABLE3_TAUS[3:],
               kT=1.0 / 3000.0, burn=2000, steps=20000, every=50, sk_every=500):
    """Equilibration ratios of Sec. III (Table III, every tau of the table) and
    the |k|-resolved ratio of the total momentum (Fig. 2: min and max over
    4 <= |k| <= 64) on a periodic box at rest, rho0 = 1, kT = 1/3000,
    thermalised start, ghosts at tau = 1.  BGK is also run at tau = 0.5005,
    below the range where the paper reports it stable."""
    import numpy as np
    import torch

    import paper_2507_08820_amd as rf

    cs2 = 1.0 / 3.0
    mu = kT / cs2
    paper = paper_table3()
    rows = []
    for model, tlist in (("reg", taus), ("bgk", bgk_taus)):
        for tau in tlist:
            lat = rf.Lattice(dims, kT=kT, tau=tau, tau_bulk=tau, tau_ghost=1.0, model=model, seed=7)
            lat.init_thermal()
            lat.step(burn)
            lat.stats_config(every)
            lat.reset_stats()
            for snap in range(steps // sk_every):
                lat.step(sk_every)
                lat.sk_sample()
                if (snap + 1) % 10 == 0:
                    log(f"table3 {model} tau={tau}: {(snap + 1) * sk_every} of {steps} steps")
            try:
                lat.sync()
                stable = True
            except rf.RFLBMError:
                stable = False
            s = lat.stats()
            n = s["samples"] * s["nodes"]
            var = lambda a, b: b / n - (a / n) ** 2
            row = {"model": model, "tau": tau, "stable": stable, "samples": s["samples"],
                   "ER_rho": var(s["sum_drho"], s["sum_drho2"]) / mu,
                   "ER_sum_rho_u": float(np.sum(var(s["sum_j"], s["sum_j2"]))) / (3 * kT),
                   "ER_sum_Pi_aa": float(np.sum(var(s["sum_pi"][:3], s["sum_pi2"][:3]))) / (3 * mu * 2 / 9),
                   "ER_sum_Pi_ab": float(np.sum(var(s["sum_pi"][3:], s["sum_pi2"][3:]))) / (3 * mu / 9)}
            sums = sum(lat.sk(f)[0] for f in ("jx", "jy", "jz"))
            _, counts, ns = lat.sk("jx")
            k = np.arange(len(sums))
            sel = (k >= 4) & (k <= 64) & (counts > 0)
            erk = sums[sel] / counts[sel] / ns / (3 * kT)
            row["ER_sum_rho_u_k4_64_min"] = float(erk.min())
            row["ER_sum_rho_u_k4_64_max"] = float(erk.max())
            row = {k2: (None if not stable and k2.startswith("ER") else
                        round(v, 5) if isinstance(v, float) else v) for k2, v in row.items()}
            row["paper_ER_rho_rho_u_Pi_aa_Pi_ab"] = paper.get((model, tau)) if abs(kT - 1.0 / 3000.0) < 1e-12 else None
            log(f"table3 {row}")
            rows.append(row)
            lat.close()
            del lat
            torch.cuda.empty_cache()
    return {"box": list(dims), "kT": kT, "burn_in": burn, "steps": steps, "stats_every": every,
            "sk_every": sk_every, "rows": rows}


# Field groups of Table III and their FDT variances per component (rho0 = 1,
# mu = kT / cs2): rho, the three rho u_a, the three Pi_aa, the three Pi_ab.
ER_GROUPS = (("rho", ("rho",), 1.0), ("sum_rho_u", ("jx", "jy", "jz"), None),
             ("sum_Pi_aa", ("pi_xx", "pi_yy", "pi_zz"), 2.0 / 9.0),
             ("sum_Pi_ab", ("pi_xy", "pi_xz", "pi_yz"), 1.0 / 9.0))


def er_from_stats(s, kT):
    """ER of each Table III group from the FP64 step statistics (every sampled
    step, variance about the mean over all samples)."""
    import numpy as np
    mu = kT / (1.0 / 3.0)
    n = s["samples"] * s["nodes"]
    var = lambda a, b: b / n - (a / n) ** 2
    return {"rho": var(s["sum_drho"], s["sum_drho2"]) / mu,
            "sum_rho_u": float(np.sum(var(s["sum_j"], s["sum_j2"]))) / (3 * kT),
            "sum_Pi_aa": float(np.sum(var(s["sum_pi"][:3], s["sum_pi2"][:3]))) / (3 * mu * 2 / 9),
            "sum_Pi_ab": float(np.sum(var(s["sum_pi"][3:], s["sum_pi2"][3:]))) / (3 * mu / 9)}


def group_theory(kT, weight):
    mu = kT / (1.0 / 3.0)
    return kT if weight is None else mu * weight


def table3_protocol(dims=(256, 256, 256), reg_taus=(0.5001, 0.505, 0.51, 1.0, 10.0, 50.0, 100.0),
                    bgk_taus=(0.505, 0.51, 10.0, 50.0, 100.0), kT=1.0 / 3000.0, burn=2000, steps=500000,
                    blocks=10, every=50, snap_every=5000, out_path=None, storage="f32"):
    """Table III and Figs. 1-2 of Sec. III at the paper's protocol: periodic box
    at rest, rho0 = 1, kT = 1/3000, ghosts at tau = 1, `steps` measured steps
    with a snapshot of rho, rho u and Pi every `snap_every` steps.  Thermalised
    start and `burn` unmeasured steps first.  Two estimators of each ER:
      - "snapshots": the paper's, the spatial variance of each snapshot about
        its own mean (from the structure-factor shell sums: by Parseval the sum
        over all n != 0 of |dm^(n)|^2 is N times that variance), averaged over
        the snapshots;
      - "dense": the step statistics sampled every `every` steps.
    The run is cut into `blocks` equal blocks; each ER is the mean over blocks
    and its standard error the blocks' standard deviation over sqrt(blocks).
    The |k|-resolved ratio of each group (Fig. 1) is the snapshot shell sums
    over the whole run; Fig. 2 is its minimum and maximum over 4 <= |k| <= 64.
    Each finished tau is appended as one JSON line to out_path."""
    import numpy as np
    import torch

    import paper_2507_08820_amd as rf

    paper = paper_table3()
    names = [g[0] for g in ER_GROUPS]
    n_nodes = dims[0] * dims[1] * dims[2]
    per_block = steps // blocks
    assert per_block % snap_every == 0 and per_block % every == 0
    rows = []
    for model, tlist in (("reg", reg_taus), ("bgk", bgk_taus)):
        for tau in tlist:
            t0 = time.time()
            lat = rf.Lattice(dims, kT=kT, tau=tau, tau_bulk=tau, tau_ghost=1.0, model=model, seed=7,
                             storage=storage)
            lat.init_thermal()
            lat.step(burn)
            lat.stats_config(every)
            dense = {k: [] for k in names}
            snaps = {k: [] for k in names}
            shell = None
            stable = True
            for b in range(blocks):
                lat.reset_stats()
                lat.reset_sk()
                for _ in range(per_block // snap_every):
                    lat.step(snap_every)
                    lat.sk_sample()
                try:
                    lat.sync()
                except rf.RFLBMError:
                    stable = False
                    break
                for k, v in er_from_stats(lat.stats(), kT).items():
                    dense[k].append(v)
                fields = {f: lat.sk(f) for f in rf.FIELDS}
                counts, ns = fields["rho"][1], fields["rho"][2]
                if shell is None:
                    shell = {f: np.zeros_like(fields[f][0]) for f in rf.FIELDS}
                    shell_counts, shell_samples = counts.copy(), 0
                shell_samples += ns
                for f in rf.FIELDS:
                    shell[f] += fields[f][0]
                for name, comps, weight in ER_GROUPS:
                    tot = sum(fields[f][0].sum() for f in comps)
                    snaps[name].append(tot / (n_nodes * ns) / (len(comps) * group_theory(kT, weight)))
                log(f"table3 {model} tau={tau}: block {b + 1}/{blocks} ({(b + 1) * per_block} steps, "
                    f"{time.time() - t0:.0f} s) snapshots ER {[round(snaps[k][-1], 4) for k in names]}")
            row = {"model": model, "tau": tau, "stable": stable}
            if stable:
                for est, vals in (("dense", dense), ("snapshots", snaps)):
                    row[est] = {k: [round(float(np.mean(v)), 5), round(float(np.std(v, ddof=1) / np.sqrt(len(v))), 5)]
                                for k, v in vals.items()}
                k = np.arange(len(shell_counts))
                sel = shell_counts > 0
                spectra = {}
                for name, comps, weight in ER_GROUPS:
                    er_k = np.full(len(k), np.nan)
                    er_k[sel] = (sum(shell[f][sel] for f in comps) / shell_counts[sel] / shell_samples
                                 / (len(comps) * group_theory(kT, weight)))
                    spectra[name] = [None if not np.isfinite(v) else round(float(v), 4) for v in er_k]
                    band = er_k[(k >= 4) & (k <= 64) & sel]
                    row.setdefault("fig2_min_max_k4_64", {})[name] = [round(float(band.min()), 4),
                                                                      round(float(band.max()), 4)]
                row["fig1_er_by_shell"] = spectra
                row["shell_counts"] = [int(c) for c in shell_counts]
            row["paper"] = (dict(zip(names, paper[(model, tau)])) if (model, tau) in paper
                            and abs(kT - 1.0 / 3000.0) < 1e-12 else None)
            row["seconds"] = round(time.time() - t0, 1)
            log(f"table3 {model} tau={tau}: {json.dumps({k: row.get(k) for k in ('stable', 'snapshots', 'paper')})}")
            if out_path:
                with open(out_path, "a") as fh:
                    fh.write(json.dumps(row) + "\n")
            rows.append(row)
            lat.close()
            del lat
            torch.cuda.empty_cache()
    return {"box": list(dims), "kT": kT, "burn_in": burn, "steps": steps, "blocks": blocks,
            "stats_every": every, "snapshot_every": snap_every, "storage": storage, "rows": rows}


VALU_CMD = ("rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU -d <out>/prof_valu_{s} -o valu --output-format csv "
             "-- python3 bench.py --profile --profile-storage {s}")
# Issue rate of plain FP32 vector instructions measured on the MI355X (a probe of
# eight independent FMA chains per lane): 97.5 lanes per cycle per CU at the
# 2.4 GHz peak clock, i.e. one wave64 instruction per 2.63 cycles per SIMD
# (4 SIMDs per CU).  Transcendental instructions and 32 x 32 -> 64-bit
# multiply-adds issued 3.2 and about 2.6-4.5 times slower in the same probe.
FMA_CYCLES_PER_WAVE_INSTR = 4 * 64 / 97.5
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9


def summarize_valu(out_dir, storage, dims=(512, 512, 512)):
    """profiles/step_<storage>_512_valu.txt: per step kernel, the mean over its
    dispatches of the VALU and SALU instructions per node (SQ_INSTS_* count
    wave instructions, one node per lane), and the time those VALU
    instructions take at the measured plain-FP32 issue rate on every SIMD: a
    lower bound of the kernel time (slower instructions take longer)."""
    import csv
    import glob

    files = glob.glob(os.path.join(out_dir, f"prof_valu_{storage}", "*counter_collection.csv"))
    if not files:
        raise FileNotFoundError(f"prof_valu_{storage}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    n = dims[0] * dims[1] * dims[2]
    acc = {}
    for r in rows:
        m = re.search(r"(step_\w*kernel<[^>]*>)", r["Kernel_Name"])
        if not m:
            continue
        short = m.group(1)
        acc.setdefault(short, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    path = os.path.join(ROOT, "profiles", f"step_{storage}_512_valu.txt")
    mean = lambda v: sum(v) / len(v) if v else 0.0
    trace_ms = trace_kernel_ms(storage)
    with open(path, "w") as fh:
        fh.write(f"# VALU and SALU instructions of the step kernels, 512^3 {storage.upper()} bench workload "
                 "(4 timed + 2 warm-up steps)\n")
        fh.write(f"# command: {VALU_CMD.format(s=storage)}\n")
        fh.write(f"# kernel_source_hash = {kernel_hash()}\n")
        fh.write(f"# issue ms: VALU wave instructions x {FMA_CYCLES_PER_WAVE_INSTR:.2f} cycles / "
                 f"({SIMDS} SIMDs x {CLOCK_HZ / 1e9:.1f} GHz)\n")
        fh.write(f"# VALU issue %: issue ms / the kernel's mean duration in "
                 f"profiles/step_{storage}_512_kernel_trace.txt (same kernel source), the share of the\n"
                 "# kernel's time the SIMDs need to issue its VALU instructions at the plain FP32 rate\n")
        fh.write("kernel | dispatches | VALU instructions per node | SALU instructions per node | issue ms | "
                 "kernel ms | VALU issue %\n")
        for k, c in sorted(acc.items()):
            valu, salu = c.get("SQ_INSTS_VALU", []), c.get("SQ_INSTS_SALU", [])
            issue_ms = mean(valu) * FMA_CYCLES_PER_WAVE_INSTR / (SIMDS * CLOCK_HZ) * 1e3
            kms = trace_ms.get(k)
            share = f"{kms:.3f} | {100.0 * issue_ms / kms:.1f}" if kms else "- | -"
            fh.write(f"{k} | {len(valu)} | {mean(valu) * 64 / n:.0f} | {mean(salu) * 64 / n:.0f} | "
                     f"{issue_ms:.3f} | {share}\n")
    return path


def trace_kernel_ms(storage):
    """{short kernel name: mean duration in ms} from the committed kernel trace
    summary of a storage type, or {} when it is missing or was taken on
    another kernel source."""
    path = os.path.join(ROOT, "profiles", f"step_{storage}_512_kernel_trace.txt")
    if not os.path.exists(path):
        return {}
    out, same_source = {}, False
    with open(path) as fh:
        for line in fh:
            if line.startswith("# kernel_source_hash"):
                same_source = line.split("=")[1].strip() == kernel_hash()
            m = re.search(r"(step_\w*kernel<[^>]*>)\S* \| \d+ \| (\d+)", line)
            if m and not line.startswith("#"):
                out[m.group(1)] = float(m.group(2)) * 1e-6
    return out if same_source else {}


PROFILE_CMDS = {
    "trace": "rocprofv3 --kernel-trace --stats -d <out>/prof_trace -o trace --output-format csv "
             "-- python3 bench.py --steps 60 --warmup 10 --no-extra --no-cpu-baseline",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -d <out>/prof_fetch -o fetch --output-format csv "
             "-- python3 bench.py --profile",
    "write": "rocprofv3 --pmc WRITE_SIZE -d <out>/prof_write -o write --output-format csv "
             "-- python3 bench.py --profile",
}


TRACE16_CMD = ("rocprofv3 --kernel-trace --stats -d <out>/prof_trace_{s} -o trace --output-format csv "
               "-- python3 bench.py --profile --profile-storage {s} --profile-steps 40")


def summarize_trace(out_dir, storage, dims=(512, 512, 512)):
    """profiles/step_<storage>_512_kernel_trace.txt for a 16-bit storage: the
    rocprofv3 kernel statistics of a profiling run of 10 warm-up + 40 timed
    steps and the mean of the even and odd step kernels (warm-up included)."""
    import csv
    import glob

    files = glob.glob(os.path.join(out_dir, f"prof_trace_{storage}", "*kernel_stats.csv"))
    if not files:
        raise FileNotFoundError(f"prof_trace_{storage}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    n = dims[0] * dims[1] * dims[2]
    steps = [r for r in rows if re.search(r"step_\w*kernel<", r["Name"])]
    path = os.path.join(ROOT, "profiles", f"step_{storage}_512_kernel_trace.txt")
    with open(path, "w") as fh:
        fh.write(f"# rocprofv3 kernel statistics, 512^3 {storage.upper()} bench workload (k_BT = 1e-5,\n")
        fh.write("# 10 warm-up + 40 timed steps, averages include the warm-up; one launch per step)\n")
        fh.write(f"# command: {TRACE16_CMD.format(s=storage)}\n")
        fh.write(f"# kernel_source_hash = {kernel_hash()}\n")
        fh.write("Name | Calls | AverageNs | MinNs | MaxNs\n")
        for r in steps:
            fh.write(f"{r['Name']} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']}\n")
        total = sum(float(r["AverageNs"]) * int(r["Calls"]) for r in steps)
        calls = sum(int(r["Calls"]) for r in steps)
        if calls:
            mean = total / calls
            fh.write(f"# mean step kernel: {mean:.0f} ns -> "
                     f"{BYTES_PER_UPDATE[storage] * n / (mean * 1e-9) / 1e9:.1f} GB/s algorithmic, "
                     f"{n / (mean * 1e-9) / 1e6:.0f} MLUPS\n")
    return path


def summarize_profiles(out_dir, dims=(512, 512, 512)):
    """Writes the profiles/ summaries from the CSVs of the three rocprofv3 runs
    of `bench.py --profile` (kernel trace, FETCH_SIZE, WRITE_SIZE)."""
    import csv
    import glob

    def rows(pattern):
        files = glob.glob(os.path.join(out_dir, pattern))
        if not files:
            raise FileNotFoundError(pattern)
        with open(files[0]) as fh:
            return list(csv.DictReader(fh))

    stats = rows("prof_trace/*kernel_stats.csv")
    fetch = rows("prof_fetch/*counter_collection.csv")
    write = rows("prof_write/*counter_collection.csv")
    n = dims[0] * dims[1] * dims[2]
    algo = BYTES_PER_UPDATE["f32"] * n  # bytes per launch
    copy_bytes = 1 << 30

    def kind(name):
        # FP32, Philox-7, no statistics: the even step is the one-wave kernel,
        # the odd step the whole-row kernel (the tiled ones when rows are off);
        # template arguments <storage, rounds, omega_g = 1, statistics, odd> of
        # the whole-row kernel, <storage, odd, rounds, statistics, omega_g = 1>
        # of the tiled one
        if "copy_kernel" in name:
            return "copy"
        if re.search(r"step_row_kernel<0, 7, \w+, false, true>|step_kernel<0, true, 7, false\b", name):
            return "odd"
        if re.search(r"step_wave_kernel<0, 7\b|step_kernel<0, false, 7, false\b", name):
            return "even"
        return None

    def per_kernel(rs):
        out = {}
        for r in rs:
            key = kind(r["Kernel_Name"])
            if key:
                out.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)  # KiB -> B
        return {k: sum(v) / len(v) for k, v in out.items()}

    fb, wb = per_kernel(fetch), per_kernel(write)
    f_scale, w_scale = copy_bytes / fb["copy"], copy_bytes / wb["copy"]
    traffic = {k: fb[k] * f_scale + wb[k] * w_scale for k in ("even", "odd")}
    mean_traffic = (traffic["even"] + traffic["odd"]) / 2
    dur = {}
    for r in stats:
        key = kind(r["Name"])
        if key in ("even", "odd"):
            dur[key] = float(r["AverageNs"])
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("# HBM traffic of the fused step kernel, 512^3 FP32 bench workload\n")
        fh.write(f"# commands: {PROFILE_CMDS['fetch']}\n#           {PROFILE_CMDS['write']}\n")
        fh.write("# counters are KiB per dispatch, scaled by what they read for copy_kernel moving 1 GiB\n")
        fh.write(f"fetch_scale = {f_scale:.5f}\nwrite_scale = {w_scale:.5f}\n")
        for k in ("even", "odd"):
            fh.write(f"{k}_fetch_bytes = {fb[k] * f_scale:.0f}\n{k}_write_bytes = {wb[k] * w_scale:.0f}\n")
            fh.write(f"{k}_traffic_over_algorithmic = {traffic[k] / algo:.4f}\n")
        fh.write(f"algorithmic_bytes_per_launch = {algo}\n")
        fh.write(f"hbm_bytes_per_launch = {mean_traffic:.0f}\n")
        fh.write(f"kernel_source_hash = {kernel_hash()}\n")
    with open(os.path.join(ROOT, "profiles", "step_f32_512_kernel_trace.txt"), "w") as fh:
        fh.write("# rocprofv3 kernel statistics of the benchmark command itself (512^3 FP32\n")
        fh.write("# workload, 10 warm-up + 60 timed steps; averages include the warm-up steps)\n")
        fh.write(f"# command: {PROFILE_CMDS['trace']}\n")
        fh.write(f"# kernel_source_hash = {kernel_hash()}\n")
        fh.write("Name | Calls | AverageNs | MinNs | MaxNs\n")
        for r in stats:
            if any(t in r["Name"] for t in ("step_kernel", "step_row_kernel", "step_wave_kernel", "copy_kernel",
                                            "init_eq_kernel")):
                fh.write(f"{r['Name']} | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                         f"{r['MinNs']} | {r['MaxNs']}\n")
        if dur:
            mean = (dur["even"] + dur["odd"]) / 2
            fh.write(f"# mean even/odd step kernel: {mean:.0f} ns -> "
                     f"{algo / (mean * 1e-9) / 1e9:.1f} GB/s algorithmic, "
                     f"{n / (mean * 1e-9) / 1e6:.0f} MLUPS\n")
    return traffic, dur


def profile_run(dims, storage="f32", steps=4):
    import torch

    import paper_2507_08820_amd as rf

    run_gpu(dims, storage, 1e-5, steps, 2 if steps <= 4 else 10)
    nbytes = 1 << 30
    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rf.copy(dst, src, nbytes)
    torch.cuda.synchronize()
    log(f"copied {nbytes} bytes")


def profile_batch_run(storage, steps=40, graph_steps=20):
    """The 64-replica workload in the launch shape the benchmark's autotuner
    picks (256-node tiles, one block per tile), replayed from a captured graph
    of graph_steps steps, for rocprofv3."""
    import paper_2507_08820_amd as rf
    import workloads as wl

    table = wl.replica_table(64, seed=5)
    reps = [dict(dims=t["dims"], kT=t["kT"], tau=t["tau"], seed=t["seed"], stream_id=t["stream_id"])
            for t in table]
    b = rf.Batch(reps, storage=storage)
    for r, t in enumerate(table):
        rho, u = wl.taylor_green_device(t["dims"], amp=0.01, device=b.device)
        b[r].init_equilibrium(rho, u)
    b.set_launch(256, 0, graph_steps)
    b.step(graph_steps)
    b.step(steps)
    b.sync()
    log(f"batch {storage}: {b.nodes} nodes, {graph_steps + steps} steps")
    b.close()


BATCH_TRACE_CMD = ("rocprofv3 --kernel-trace --stats -d <out>/prof_batch_{s} -o trace --output-format csv "
                   "-- python3 bench.py --profile-batch {s}")


def summarize_batch_trace(out_dir, storage, nodes=None):
    """profiles/batch64_<storage>_kernel_trace.txt: rocprofv3 kernel statistics
    of the 64-replica workload (one batch_kernel launch per step for all
    replicas) and the aggregate rate of the mean launch."""
    import csv
    import glob

    import workloads as wl

    files = glob.glob(os.path.join(out_dir, f"prof_batch_{storage}", "*kernel_stats.csv"))
    if not files:
        raise FileNotFoundError(f"prof_batch_{storage}")
    with open(files[0]) as fh:
        rows = [r for r in csv.DictReader(fh) if "batch_kernel<" in r["Name"]]
    if nodes is None:
        nodes = sum(int(t["dims"][0]) * int(t["dims"][1]) * int(t["dims"][2]) for t in wl.replica_table(64, seed=5))
    path = os.path.join(ROOT, "profiles", f"batch64_{storage}_kernel_trace.txt")
    with open(path, "w") as fh:
        fh.write(f"# rocprofv3 kernel statistics, 64-replica batch workload ({nodes} nodes, {storage.upper()},\n")
        fh.write("# 256-node tiles, one block per tile, graphs of 20 steps; 60 steps)\n")
        fh.write(f"# command: {BATCH_TRACE_CMD.format(s=storage)}\n")
        fh.write(f"# kernel_source_hash = {kernel_hash()}\n")
        fh.write("Name | Calls | AverageNs | MinNs | MaxNs\n")
        for r in rows:
            fh.write(f"{r['Name']} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']}\n")
        total = sum(float(r["AverageNs"]) * int(r["Calls"]) for r in rows)
        calls = sum(int(r["Calls"]) for r in rows)
        if calls:
            mean = total / calls
            fh.write(f"# mean batch step kernel: {mean:.0f} ns -> {nodes / (mean * 1e-9) / 1e6:.0f} MLUPS "
                     f"aggregate, {BYTES_PER_UPDATE[storage] * nodes / (mean * 1e-9) / 1e9:.1f} GB/s algorithmic\n")
    return path


def copy_ceiling(nbytes=4 << 30, reps=20):
    import torch

    import paper_2507_08820_amd as rf

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rf.copy(dst, src, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rf.copy(dst, src, nbytes)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(size, min_seconds=10.0, max_steps=200):
    """The FP64 oracle as it stands on a size^3 sample of the benchmark workload
    (Taylor-Green, tau 0.6, kT 1e-5, the same noise): whole steps until at least
    min_seconds have passed.  Returns (MLUPS, threads, steps, seconds)."""
    import oracle
    import workloads as wl

    dims = (size, size, size)
    rho, u = wl.taylor_green(dims, amp=0.01)
    f = oracle.init_equilibrium(dims, rho, u)
    p = oracle.make_params(kT=1e-5, tau_shear=0.6, tau_bulk=0.6, seed=3)
    n = dims[0] * dims[1] * dims[2]
    steps, t0 = 0, time.perf_counter()
    while steps < max_steps and (time.perf_counter() - t0) < min_seconds:
        f = oracle.step(p, dims, f, steps)
        steps += 1
    dt = time.perf_counter() - t0
    return n * steps / dt / 1e6, oracle.threads(), steps, dt


def cpu_baseline(min_seconds=10.0):
    """The oracle on all host threads (128^3 sample) and on one thread (64^3
    sample, in a child process with OMP_NUM_THREADS=1), with the CPU model."""
    import subprocess

    mlups, threads, steps, dt = oracle_rate(128, min_seconds)
    out = {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"128^3 Taylor-Green box (same tau, kT, noise), {steps} steps, FP64, {dt:.1f} s, "
                     f"{threads} OpenMP threads",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", "64",
                        "--cpu-baseline-seconds", str(min_seconds)], env=env, capture_output=True, text=True,
                       timeout=300)
    if r.returncode == 0:
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["value_1_thread"] = one["mlups"]
        out["sample_1_thread"] = (f"64^3 sample of the same workload, {one['steps']} steps, FP64, "
                                  f"{one['seconds']:.1f} s, {one['threads']} thread")
    else:
        out["value_1_thread"] = None
        out["sample_1_thread"] = "one-thread run failed: " + r.stderr[-300:]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--table3", action="store_true",
                    help="equilibration ratios of Table III at 256^3, kT = 1/3000 (a physics "
                         "check against the paper, not a throughput figure)")
    ap.add_argument("--table3-taus", metavar="T1,T2,...",
                    help="with --table3: Reg-FLBM taus to run (default: every tau of Table III)")
    ap.add_argument("--table3-bgk-taus", metavar="T1,T2,...",
                    help="with --table3: BGK-FLBM taus to run ('' for none)")
    ap.add_argument("--table3-kT", type=float, default=1.0 / 3000.0,
                    help="with --table3: temperature (the paper's 1/3000 by default)")
    ap.add_argument("--table3-steps", type=int, default=None,
                    help="measured steps; --table3: 20 000 (400 statistics samples, 40 S(k) snapshots), "
                         "--table3-protocol: 500 000 (statistics every 50 steps, 100 snapshots)")
    ap.add_argument("--cpu-baseline-worker", type=int, metavar="SIZE", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=10.0, help=argparse.SUPPRESS)
    ap.add_argument("--table3-protocol", action="store_true",
                    help="Table III / Figs. 1-2 at the paper's protocol (256^3, 500 000 steps, 100 snapshots)")
    ap.add_argument("--table3-size", type=int, default=256)
    ap.add_argument("--table3-blocks", type=int, default=10)
    ap.add_argument("--table3-out", metavar="PATH", help="append one JSON line per finished tau")
    ap.add_argument("--profile-storage", default="f32", choices=["f32", "f16", "bf16"],
                    help="with --profile: storage of the profiled workload")
    ap.add_argument("--profile-batch", choices=["f32", "f16"],
                    help="run the 64-replica workload (60 graph-replayed steps) for rocprofv3")
    ap.add_argument("--summarize-batch-trace", metavar="DIR",
                    help="write profiles/batch64_{f32,f16}_kernel_trace.txt from the kernel-trace CSVs under DIR")
    ap.add_argument("--profile-steps", type=int, default=4,
                    help="with --profile: timed steps (2 warm-up steps up to 4, else 10)")
    ap.add_argument("--summarize-valu", metavar="DIR",
                    help="write profiles/step_<storage>_512_valu.txt from the VALU counter CSVs under DIR")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write profiles/step_{f16,bf16}_512_kernel_trace.txt from the kernel-trace CSVs under DIR")
    ap.add_argument("--precision512", action="store_true",
                    help="storage precision on the 512^3 workload: FP16 and BF16 against FP32 with "
                         "the same noise, kT in {1e-4, 1e-5, 1e-6}, 1000 steps")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write profiles/ summaries from the rocprofv3 CSVs under DIR")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: 2 warm-up and 4 timed steps of the bench "
                         "workload, then one copy of 1 GiB (the counter calibration kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Reg-FLBM path here is single-GPU "
              "(no multi-GPU sharding is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    dims = (args.size,) * 3
    if args.cpu_baseline_worker:
        mlups, threads, steps, dt = oracle_rate(args.cpu_baseline_worker, args.cpu_baseline_seconds)
        print(json.dumps({"mlups": mlups, "threads": threads, "steps": steps, "seconds": dt}))
        return
    if args.summarize:
        print(summarize_profiles(args.summarize))
        return
    if args.profile:
        profile_run(dims, args.profile_storage, args.profile_steps)
        return
    if args.profile_batch:
        profile_batch_run(args.profile_batch)
        return
    if args.summarize_batch_trace:
        for storage in ("f32", "f16"):
            print(summarize_batch_trace(args.summarize_batch_trace, storage))
        return
    if args.summarize_valu:
        for storage in ("f32", "f16"):
            print(summarize_valu(args.summarize_valu, storage))
        return
    if args.summarize_trace:
        for storage in ("f16", "bf16"):
            print(summarize_trace(args.summarize_trace, storage))
        return
    if args.precision512:
        print(json.dumps(precision_full()))
        return
    if args.table3_protocol:
        kw = {}
        if args.table3_taus is not None:
            kw["reg_taus"] = tuple(float(t) for t in args.table3_taus.split(",") if t)
        if args.table3_bgk_taus is not None:
            kw["bgk_taus"] = tuple(float(t) for t in args.table3_bgk_taus.split(",") if t)
        steps = args.table3_steps or 500000
        n = args.table3_size
        print(json.dumps(table3_protocol(dims=(n, n, n), kT=args.table3_kT, steps=steps,
                                         blocks=args.table3_blocks, every=50,
                                         snap_every=steps // (10 * args.table3_blocks),
                                         out_path=args.table3_out, **kw)))
        return
    if args.table3:
        kw = {}
        if args.table3_taus is not None:
            kw["taus"] = tuple(float(t) for t in args.table3_taus.split(",") if t)
        if args.table3_bgk_taus is not None:
            kw["bgk_taus"] = tuple(float(t) for t in args.table3_bgk_taus.split(",") if t)
        steps = args.table3_steps or 20000
        print(json.dumps(table3_run(kT=args.table3_kT, steps=steps, every=steps // 400, sk_every=steps // 40,
                                    **kw)))
        return
    short = max(20, args.steps // 4)
    followups = () if args.no_extra else (("stats_every_step", 1e-5, 1, short), ("kT0_reg_lbm", 0.0, 0, short))
    main_run = run_gpu(dims, "f32", 1e-5, args.steps, args.warmup, followups=followups)
    n = dims[0] * dims[1] * dims[2]
    achieved = BYTES_PER_UPDATE["f32"] * n / (main_run["ms_per_step"] * 1e-3) / 1e9
    traffic = measured_traffic() if dims == (512, 512, 512) else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}

    extra = {}
    if not args.no_extra:
        for name, storage in (("f16_store", "f16"), ("bf16_store", "bf16")):
            r = run_gpu(dims, storage, 1e-5, short, 5, followups=(("kT0_reg_lbm", 0.0, 0, short),))
            extra[name] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                           "hbm_gbs": round(BYTES_PER_UPDATE[storage] * n / (r["ms_per_step"] * 1e-3) / 1e9, 1)}
            # the deterministic step on the same lattice (bandwidth bound: row-aligned kernels)
            f = r["followups"]["kT0_reg_lbm"]
            extra[name + "_kT0"] = {"mlups": round(f["mlups"], 1), "ms_per_step": round(f["ms_per_step"], 4)}
        # same lattice as the main figure
        for name, label in (("f32_stats_every_step", "stats_every_step"), ("reg_lbm_kT0_f32", "kT0_reg_lbm")):
            f = main_run["followups"][label]
            extra[name] = {"mlups": round(f["mlups"], 1), "ms_per_step": round(f["ms_per_step"], 4)}
        extra["f16_gain_over_f32"] = round(extra["f16_store"]["mlups"] / main_run["mlups"], 3)
        extra["noise_cost_factor"] = round(extra["reg_lbm_kT0_f32"]["mlups"] / main_run["mlups"], 3)
        extra["stats_cost_factor"] = round(extra["f32_stats_every_step"]["mlups"] / main_run["mlups"], 3)
        extra["u2_over_kT_by_storage_128cube"] = precision_study()
        # the headline 512^3 Taylor-Green workload, same noise for every storage
        extra["precision_512_taylor_green"] = precision_full(kts=(1e-5,), steps=200, every=10, sk_every=50)
        extra["batch64_f32"] = run_batch("f32")
        extra["batch64_f16"] = run_batch("f16")
        cc = copy_ceiling()
        log(f"copy kernel: {cc:.0f} GB/s")
        extra["copy_kernel_GBps"] = round(cc, 1)
        extra["frac_of_copy_ceiling"] = round(achieved / cc, 4)

    cpu = None if args.no_cpu_baseline else cpu_baseline()
    if cpu:
        log(f"cpu oracle: {cpu['value']:.3f} MLUPS on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Reg-FLBM D3Q27 {dims[0]}^3 periodic box, Taylor-Green A=0.01, "
                               "rho0=1, tau=0.6, ghost tau=1, kT=1e-5, Philox4x32-7, FP32 storage",
                   "box": list(dims), "tau": 0.6, "kT": 1e-5, "storage": "f32"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
