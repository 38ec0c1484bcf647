"""Benchmark: subdomain bounds per second of the 20-iteration alpha/beta
optimisation (and of plain evaluation) on one MI355X.

A step is one cv_bound_optimize call: 20 x (back-substitution of every layer
with relaxation and concretisation, adjoint forward sweep with gradients,
projected Adam) plus the final evaluation, over one batch of B subdomains x m
specification rows resident in HBM.  Inputs are synthetic (seeded generator
shaped like the paper's verifiers); the network's intermediate bounds come
from the library's own per-layer CROWN pass.

Prints one JSON line.  `--gpus N` with N > 1 exits: the bound path runs on one GPU.
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

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

WORKLOAD_TEXT = {
    "mlp_small": "ReLU MLP 784-100-100-10, 16 subdomains x 9 spec rows, split depth 4",
    "mlp_deep": "ReLU MLP 784-200x6-10, 1024 subdomains x 9 spec rows, split depth 1-8",
    "cnn_base": "CNN conv3-8k4s2p1, conv8-16k4s2p1, FC1024-100-10; 2048 subdomains x 9, depth 1-12",
    "cnn_wide": "CNN conv3-16k4s2p1, conv16-32k4s2p1, FC2048-100-10; 8 props x 512 subdomains x 9, depth 1-16",
    "cnn_deep": "CNN conv3-8k4s2p1, 2x conv8-8k3s1p1, conv8-8k4s2p1, FC512-100-10; 64 props, 8192 subdomains x 9, "
                "depth 1-16",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 (16 hex digits) of the device-code sources: every file under
    csrc/ except the host-side ABI layer api.hip, whose changes do not alter
    what a kernel reads or writes."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2103_06624_amd", "csrc"))):
        if f == "api.hip":
            continue
        with open(os.path.join(ROOT, "paper_2103_06624_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload, conv_plan):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources under the same conv plan; else
    None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    if rec.get("_about", {}).get(f"conv_plan_{workload}") != conv_plan:
        return None
    return ent.get("bytes_per_launch")


# ---- rocprofv3 counter runs -> per-kernel figures (host only) --------------
# The counter runs profile `bench.py --profile-only`, whose last work is the
# per-kernel timing pass: every launch of one gradient pass and one plain
# evaluation issued 8 times back to back.  Its dispatches are therefore the
# last 8 x (launches per pass) x reps of the run, in pass order, and are named
# here from the pass's own kernel list (first appearances in pass order).


def counter_dispatches(d):
    """Dispatches of a rocprofv3 --pmc CSV run under directory d, in dispatch
    order: {kernel, grid, counters {name: value}}."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    disp = {}
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = (int(r.get("Process_Id") or 0), int(r["Dispatch_Id"]))
                e = disp.setdefault(k, {"kernel": r["Kernel_Name"], "grid": int(r["Grid_Size"]), "c": {}})
                e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


def last_json_line(path):
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])


def name_profile_pass(disp, prof):
    """{kernel name of the timing pass: [its dispatches]} from a counter run of
    `bench.py --profile-only` whose printed line is prof."""
    kern = prof["kernels"]
    reps = prof["profile_reps"]
    n = 8 * reps * sum(k["launches_per_pass"] for k in kern)
    tail = disp[-n:]
    if len(tail) != n:
        raise SystemExit("counter run holds fewer dispatches than the timing pass")
    # a group of 8 takes the name its (symbol, grid) had before while that
    # name has launches left in the current pass, else the next name not yet
    # seen (two names may share a symbol and grid)
    order = [k["name"] for k in kern]
    per_pass = {k["name"]: k["launches_per_pass"] for k in kern}
    groups_per_rep = sum(per_pass.values())
    key_names, out, seen, left = {}, {}, [], {}
    for gi, i in enumerate(range(0, n, 8)):
        if gi % groups_per_rep == 0:
            left = dict(per_pass)
        grp = tail[i:i + 8]
        key = (grp[0]["kernel"], grp[0]["grid"])
        if any((g["kernel"], g["grid"]) != key for g in grp):
            raise SystemExit(f"dispatch group at {i} is not 8 launches of one kernel")
        name = next((nm for nm in key_names.get(key, []) if left[nm] > 0), None)
        if name is None:
            fresh = [nm for nm in order if nm not in seen]
            if not fresh:
                raise SystemExit(f"dispatch group at {i}: no kernel name left for {key}")
            name = fresh[0]
            seen.append(name)
            key_names.setdefault(key, []).append(name)
        left[name] -= 1
        out.setdefault(name, []).extend(grp)
    for k in kern:
        got = len(out.get(k["name"], ()))
        if got != 8 * reps * k["launches_per_pass"]:
            raise SystemExit(f"{k['name']}: {got} dispatches, expected {8 * reps * k['launches_per_pass']}")
    return out


def copy_factor(d, counter, mib):
    """Known bytes of one mib-MiB device copy / what `counter` (KiB) reads for
    it: the mean over the calibration run's last 3 dispatches (the copies)."""
    disp = counter_dispatches(d)[-3:]
    if len({x["kernel"] for x in disp}) != 1:
        raise SystemExit("calibration run does not end with 3 copies of one kernel")
    kib = sum(x["c"][counter] for x in disp) / 3
    return (mib << 20) / (kib * 1024.0)


def ingest_traffic(args):
    """Write the workload's entry of profiles/traffic.txt from a FETCH_SIZE
    and a WRITE_SIZE counter run of --profile-only and the two counters'
    readings of a plain copy (--calib-only)."""
    fetch_dir, write_dir, cal_f, cal_w, prof_path = args.ingest_traffic
    prof = last_json_line(prof_path)
    ff = copy_factor(cal_f, "FETCH_SIZE", args.calib_copy_mib)
    fw = copy_factor(cal_w, "WRITE_SIZE", args.calib_copy_mib)
    fetch = name_profile_pass(counter_dispatches(fetch_dir), prof)
    write = name_profile_pass(counter_dispatches(write_dir), prof)
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
    h = kernel_source_hash()
    ent = {}
    for name in fetch:
        fb = sum(x["c"]["FETCH_SIZE"] for x in fetch[name]) / len(fetch[name]) * 1024 * ff
        wb = sum(x["c"]["WRITE_SIZE"] for x in write[name]) / len(write[name]) * 1024 * fw
        ent[name] = {"bytes_per_launch": int(fb + wb), "fetch_bytes": int(fb), "write_bytes": int(wb),
                     "dispatches": len(fetch[name]), "source_hash": h}
    rec["_about"] = {k: v for k, v in rec.get("_about", {}).items() if not k.startswith(("what", "commands"))}
    rec["_about"]["what"] = (
        "HBM bytes per launch per kernel = mean FETCH_SIZE x fetch factor + mean WRITE_SIZE x write factor "
        "(KiB per dispatch, over the kernel's dispatches in bench.py --profile-only's per-kernel timing pass, "
        "every launch issued 8 times back to back); factors = known bytes of a plain device copy "
        "(bench.py --calib-only, 256 MiB) / what the same counter reads for it.  Valid for the kernel sources "
        "of source_hash (sha256 of paper_2103_06624_amd/csrc/* except the host-side api.hip, first 16 hex "
        "digits) and the conv plan conv_plan_<workload> the counter runs' autotuner chose.")
    rec["_about"]["commands"] = [
        "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv "
        "-d $REPO/gpurun_out/pmc_fetch -o run -- python3 $REPO/bench.py --workload <W> --profile-only "
        "--profile-reps 1 > $REPO/gpurun_out/pmc_fetch.out",
        "(the same with --pmc WRITE_SIZE into pmc_write)",
        "timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $REPO/gpurun_out/cal_fetch -o run "
        "-- python3 $REPO/bench.py --calib-only --calib-copy-mib 256 (and WRITE_SIZE into cal_write)",
        "python3 bench.py --ingest-traffic gpurun_out/pmc_fetch gpurun_out/pmc_write gpurun_out/cal_fetch "
        "gpurun_out/cal_write gpurun_out/pmc_fetch.out"]
    rec["_about"][f"factors_{prof['workload']}"] = {"fetch": round(ff, 4), "write": round(fw, 4)}
    rec["_about"][f"conv_plan_{prof['workload']}"] = prof["conv_plan"]
    rec[prof["workload"]] = ent
    # entries taken on other kernel sources are stale: drop them
    for w in [w for w in rec if not w.startswith("_")]:
        rec[w] = {k: v for k, v in rec[w].items() if v.get("source_hash") == h}
        if not rec[w]:
            del rec[w]
    for k in [k for k in rec["_about"] if k.startswith(("factors_", "conv_plan_"))]:
        if k.split("_", 1)[1].replace("plan_", "", 1) not in rec:
            del rec["_about"][k]
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    algo = {k["name"]: k["bytes_per_launch"] for k in prof["kernels"]}
    for name, e in sorted(ent.items(), key=lambda kv: -kv[1]["bytes_per_launch"]):
        print(f"{name:32s} HBM {e['bytes_per_launch'] / 1e6:10.1f} MB/launch  algorithmic "
              f"{algo.get(name, 0) / 1e6:10.1f} MB  ratio {e['bytes_per_launch'] / max(algo.get(name, 1), 1):6.2f}")


def counters_summary(args):
    """Per-kernel counter figures of the timing pass (markdown table) from
    counter runs of --profile-only: MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES /
    (GRBM_GUI_ACTIVE / 8 XCDs x 1024 SIMDs), instructions per dispatch.
    Arguments: a run's printed output, then its counter directories; or
    (output, directory) pairs, one per run, where the runs' autotuners may
    have chosen different plans (a kernel is then summarised from the runs
    that hold it)."""
    a = args.counters_summary
    paired = len(a) % 2 == 0 and all(os.path.isfile(x) for x in a[0::2]) and all(os.path.isdir(x) for x in a[1::2])
    runs = [(a[i], a[i + 1]) for i in range(0, len(a), 2)] if paired else [(a[0], d) for d in a[1:]]
    merged, us, tf = {}, {}, {}
    for out, d in runs:
        prof = last_json_line(out)
        for k in prof["kernels"]:
            us.setdefault(k["name"], k["avg_us"])
            tf.setdefault(k["name"], k["tflops"])
        for name, lst in name_profile_pass(counter_dispatches(d), prof).items():
            m = merged.setdefault(name, {})
            for c in {c for x in lst for c in x["c"]}:
                m[c] = sum(x["c"].get(c, 0.0) for x in lst) / len(lst)
    print("| kernel | avg us (HIP events) | TFLOP/s | MFMA busy | VALU insts/disp (M) | MFMA insts/disp (M) | "
          "LDS insts/disp (M) | LDS bank conflict / LDS active |")
    print("|---|---|---|---|---|---|---|---|")
    for name, m in merged.items():
        gr = m.get("GRBM_GUI_ACTIVE", 0.0) / 8
        busy = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (gr * 1024) if gr and "SQ_VALU_MFMA_BUSY_CYCLES" in m else None
        bank = (m["SQ_LDS_BANK_CONFLICT"] / m["SQ_LDS_IDX_ACTIVE"]
                if m.get("SQ_LDS_IDX_ACTIVE") and "SQ_LDS_BANK_CONFLICT" in m else None)
        f = lambda c: f"{m[c] / 1e6:.2f}" if c in m else "-"
        print(f"| {name} | {us.get(name, 0):.1f} | {tf.get(name, 0):.1f} | "
              f"{'-' if busy is None else f'{busy:.3f}'} | {f('SQ_INSTS_VALU')} | {f('SQ_INSTS_MFMA')} | "
              f"{f('SQ_INSTS_LDS')} | {'-' if bank is None else f'{bank:.3f}'} |")


def trace_summary(args):
    """Per-kernel durations of the timing pass from a rocprofv3
    --kernel-trace database of --profile-only (the `kernels` view), beside the
    pass's own HIP-event averages (markdown)."""
    import sqlite3
    prof = last_json_line(args.trace_summary[0])
    con = sqlite3.connect(args.trace_summary[1])
    disp = [{"kernel": n, "grid": gx * gy * gz, "us": d / 1e3}
            for n, gx, gy, gz, d in con.execute(
                "select name, grid_x, grid_y, grid_z, duration from kernels order by dispatch_id")]
    named = name_profile_pass(disp, prof)
    ev = {k["name"]: k for k in prof["kernels"]}
    print("| kernel | symbol | dispatches | rocprofv3 avg us | HIP-event avg us | rocprof / events |")
    print("|---|---|---|---|---|---|")
    for name, lst in named.items():
        a = sum(x["us"] for x in lst) / len(lst)
        sym = lst[0]["kernel"].replace("void ", "").replace("cvb::(anonymous namespace)::", "").split("(")[0]
        print(f"| {name} | `{sym}` | {len(lst)} | {a:.1f} | {ev[name]['avg_us']:.1f} | "
              f"{a / ev[name]['avg_us']:.3f} |")


def library_gemm_context(wl, rows):
    """torch.mm (the ROCm BLAS library) on [rows, d_i] x [d_i, d_(i-1)] for
    each distinct dense back-substitution shape: what a plain library GEMM of
    the same size reaches on this GPU, without the relaxation epilogue."""
    import torch

    from paper_2103_06624_amd import synth
    torch.backends.cuda.matmul.allow_tf32 = False
    shapes = []
    for ly in wl.net.layers[:-1]:  # the last layer is folded into the spec
        if ly.kind == synth.DENSE:
            d_out, d_in = ly.weight.shape
            if (d_in, d_out) not in shapes and len(shapes) < 4:
                shapes.append((d_in, d_out))
    out = []
    for n, k in shapes:
        a = torch.randn(rows, k, device="cuda")
        b = torch.randn(k, n, device="cuda")
        for _ in range(5):
            c = a @ b
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(50):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 50 * 1e3
        out.append({"m": rows, "n": n, "k": k, "us": round(us, 2), "tflops": round(2.0 * rows * n * k / us / 1e6, 2)})
        del a, b, c
    return out


def bab_context(wl, lo, up, args):
    """Throughput of the library's branch and bound on one property of the
    workload (context for the paper's branches/s figures)."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2103_06624_amd import bab as gb
    from paper_2103_06624_amd import synth
    from paper_2103_06624_amd.api import BoundProblem

    layers = list(wl.net.layers)
    p = 0
    one = BoundProblem(layers, wl.x_lo[p:p + 1], wl.x_hi[p:p + 1], wl.C[p:p + 1], lo[p:p + 1], up[p:p + 1],
                       np.zeros(1, np.int32), np.zeros(2, np.int64), [], [], [])
    lb0, ub0, _ = one.upper(one.alpha_init(), one.zeros_beta())
    t = ((lb0 + ub0) / 2).cpu().numpy().reshape(-1)
    one.close()
    last = layers[-1]
    W = np.vstack([last.weight, np.zeros((1, last.weight.shape[1]), np.float32)])
    b = np.concatenate([last.bias, np.ones(1, np.float32)])
    layers[-1] = dataclasses.replace(last, weight=W, bias=b, out_shape=(W.shape[0], 1, 1))
    C = np.hstack([wl.C[p], -t[:, None]]).astype(np.float32)
    torch.cuda.synchronize()
    r = gb.bab(layers, wl.x_lo[p], wl.x_hi[p], C, lo[p], up[p], batch=args.bab_batch, max_rounds=args.bab_rounds,
               iters=args.iters, lr_alpha=args.lr_alpha, lr_beta=args.lr_beta, decay=args.decay, warm=args.bab_warm)
    # rounds that split a full batch (after the pool has grown to it), and the
    # optimiser's own rate over the same rounds (the rest of a round: the
    # handle's re-targeting, the upper bound, the pool on the host)
    full = [(n, s, o) for n, s, o in r["per_round"] if n >= 2 * args.bab_batch]
    fb = sum(n for n, _, _ in full)
    return {"domains_per_s": round(r["domains"] / r["seconds"], 1), "domains": r["domains"], "rounds": r["rounds"],
            "batch": args.bab_batch, "seconds": round(r["seconds"], 3), "verdict": r["verdict"],
            "lb": r["lb"], "ub": r["ub"], "warm_start": bool(args.bab_warm),
            "full_batch_rounds": len(full),
            "full_batch_domains_per_s": round(fb / sum(s for _, s, _ in full), 1) if full else None,
            "full_batch_optimizer_domains_per_s": round(fb / sum(o for _, _, o in full), 1) if full else None}


def joint_context(wl, lo, up, args):
    """Joint optimisation of intermediate bounds (Eq. opt_non_convex) at the
    root of every property (one unsplit subdomain each): seconds and bounds
    of 20 joint iterations beside the plain optimiser's on the same
    subdomains, and how much the intermediate bounds narrowed."""
    import numpy as np
    import torch

    from paper_2103_06624_amd.api import BoundProblem

    P = wl.n_props
    pb = BoundProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo, up, np.arange(P, dtype=np.int32),
                      np.zeros(P + 1, np.int64), [], [], [])
    opt = dict(iters=args.iters, lr_alpha=args.lr_alpha, lr_beta=args.lr_beta, decay=args.decay)
    a, b = pb.alpha_init(), pb.zeros_beta()
    pb.optimize_joint(a.clone(), b.clone(), **opt)  # builds the passes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best_j, _, lo_j, up_j = pb.optimize_joint(a.clone(), b.clone(), bounds=True, **opt)
    torch.cuda.synchronize()
    t_j = time.perf_counter() - t0
    pb.optimize(a.clone(), b.clone(), **opt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best_p, _ = pb.optimize(a.clone(), b.clone(), **opt)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    gain = (best_j - best_p).cpu().numpy()
    d1 = wl.net.layers[0].d_out
    w_root = (up - lo)[:, d1:]
    w_j = (up_j - lo_j).cpu().numpy()[:, d1:]
    pb.close()
    return {"subdomains": P, "spec_rows": int(wl.C.shape[1]), "seconds": round(t_j, 4),
            "plain_seconds": round(t_p, 4), "mean_bound_joint": float(best_j.mean().item()),
            "mean_bound_plain": float(best_p.mean().item()), "mean_gain": float(gain.mean()),
            "rows_improved": int((gain > 0).sum()), "rows": int(gain.size),
            "intermediate_width_ratio": float(np.mean(w_j / np.maximum(w_root, 1e-12)))}


def cpu_baseline(name, wl, lo, up, sp, gpu, seconds, seconds_1t, iters, lr_a, lr_b, decay, n_sound=64):
    """The FP64 oracle on this host, fed the very inputs the GPU path saw (the
    workload, the GPU's own float32 root bounds and split sets):

      * timing: the per-subdomain 20-iteration optimisation (the unit of the
        GPU metric) on random subdomains, with the BLAS threads at all cores
        for about `seconds`, then at one thread for about `seconds_1t`;
      * rel_err: the GPU's optimised bounds against the oracle's on the timed
        subdomains (the same algorithm in float32 and float64);
      * soundness: at the GPU's own final iterate (alpha, beta) of the
        optimisation, the count of rows whose float32 bound exceeds the
        float64 bound at those variables, and the largest excess, in plain
        float32 mode and in sound mode (each with its own root bounds)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import batch as ob
    from oracle import beta_crown as bc

    t0 = time.perf_counter()
    net64 = bc.dense_net(wl.net.layers)
    t_net = time.perf_counter() - t0

    def problem(lo_, up_, sp_):
        return ob.OracleProblem(wl.net.layers, wl.x_lo, wl.x_hi, wl.C, lo_, up_, sp_.dom_prop, sp_.split_ptr,
                                sp_.layer, sp_.neuron, sp_.side, net64=net64)

    orc = problem(lo, up, sp)
    cfg = bc.AdamConfig(iters=iters, lr_alpha=lr_a, lr_beta=lr_b, decay=decay)
    a0 = orc.default_alpha_flat()
    z = np.zeros(orc.nnz * orc.m)
    order = np.random.default_rng(123).permutation(orc.B)

    def timed(budget):
        # subdomains in one fixed random order, as many as fit the budget
        done, errs = 0, []
        t1 = time.perf_counter()
        while done < orc.B and time.perf_counter() - t1 < budget:
            d = int(order[done])
            best, *_ = orc.optimize(d, a0, z, cfg)
            errs.append(float(np.max(np.abs(gpu["best"][d] - best) / np.maximum(np.abs(best), 1.0))))
            done += 1
        return done, time.perf_counter() - t1, errs

    done_all, el_all, errs = timed(seconds)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        done_1, el_1, errs1 = timed(seconds_1t)
    if len(errs1) > len(errs):
        errs = errs1

    def soundness(o, g):
        """rows where the float32 bound lies above the float64 bound at the same variables"""
        ds = order[:min(n_sound, o.B)]
        ex = []
        for d in ds:
            d = int(d)
            ref = o.eval(d, g["alpha"], g["beta"])
            ex.append(np.asarray(g["last"][d], np.float64) - ref)
            ex[-1] = np.stack([ex[-1], np.abs(ref)])
        ex = np.concatenate(ex, axis=1)
        exc = ex[0]
        return {"rows": int(exc.size), "subdomains": int(len(ds)), "violations": int(np.sum(exc > 0)),
                "max_excess": float(max(exc.max(), 0.0)),
                "max_rel_excess": float(max((exc / np.maximum(ex[1], 1.0)).max(), 0.0)),
                "max_rel_below": float(max((-exc / np.maximum(ex[1], 1.0)).max(), 0.0))}

    snd = {"plain": soundness(orc, gpu)}
    rel_sound = None
    if gpu.get("sound") is not None:
        gs = gpu["sound"]
        orc_s = problem(gs["lo"], gs["up"], gs["splits"])
        snd["sound_mode"] = soundness(orc_s, gs)
        ers = []
        a0s = orc_s.default_alpha_flat()
        zs = np.zeros(orc_s.nnz * orc_s.m)
        for d in order[:8]:
            best, *_ = orc_s.optimize(int(d), a0s, zs, cfg)
            ers.append(float(np.max(np.abs(gs["best"][int(d)] - best) / np.maximum(np.abs(best), 1.0))))
        rel_sound = {"max": max(ers), "subdomains": len(ers)}
    cb = {
        "value": done_all / el_all,
        "unit": "subdomain bounds/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{done_all} random subdomains of {orc.B} ({orc.m} spec rows each), {iters}-iteration Adam, "
                  f"float64 NumPy on the GPU path's own root bounds and splits; {el_all:.1f} s with {threads} BLAS "
                  f"threads; conv layers as dense matrices (built in {t_net:.1f} s, not timed); "
                  f"host has {os.cpu_count()} CPUs",
        "one_core": {"value": done_1 / el_1 if done_1 else None, "cores": 1,
                     "sample": f"the first {done_1} of the same random subdomains, {el_1:.1f} s, BLAS limited to 1 thread"},
    }
    rel = {"max": max(errs), "subdomains": len(errs)} if errs else None
    return cb, rel, snd, rel_sound


def kernel_table(pb, a0, b0, reps):
    """Per-kernel durations with HIP events on the launch stream (each launch
    of one gradient pass and one plain evaluation issued 8 times back to back
    between two events), algorithmic flops and bytes per launch."""
    stats = pb.profile(a0, b0, reps=reps)
    kern = []
    for s in stats:
        avg_ms = s["total_ms"] / (s["reps"] * s["launches"])
        fl = s["flops"] / s["launches"]
        by = s["bytes"] / s["launches"]
        kern.append(dict(name=s["name"], launches_per_pass=s["launches"], avg_us=avg_ms * 1e3,
                         tflops=(fl / (avg_ms * 1e-3) / 1e12) if fl else 0.0,
                         gbs=by / (avg_ms * 1e-3) / 1e9, share=s["total_ms"], flops_per_launch=fl,
                         bytes_per_launch=by))
    tot = sum(k["share"] for k in kern)
    for k in kern:
        k["share"] = round(k["share"] / tot, 4)
    return stats, kern


def roofline(stats, kern, name, conv_plan):
    dom = max(kern, key=lambda k: k["share"])
    if dom["flops_per_launch"] > 0:
        # the dense GEMMs and the conv layers' implicit GEMMs run on the matrix cores
        bound = "mfma" if dom["name"].startswith(("gemm", "chain", "conv")) else "alu"
        roof = {"bound": bound, "achieved": round(dom["tflops"], 3), "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(dom["tflops"] / PEAK_FP32_MFMA_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / PEAK_HBM_GBS, 4)}
    roof["traffic"] = traffic_for(dom["name"], name, conv_plan)
    roof["kernel"] = dom["name"]
    roof["avg_us"] = round(dom["avg_us"], 3)
    roof["algorithmic_bytes_per_launch"] = dom["bytes_per_launch"]
    roof["algorithmic_flops_per_launch"] = dom["flops_per_launch"]
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cnn_deep", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--lr-alpha", type=float, default=0.01)
    ap.add_argument("--lr-beta", type=float, default=0.05)
    ap.add_argument("--decay", type=float, default=0.98)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle timing budget at all host cores")
    ap.add_argument("--cpu-seconds-1t", type=float, default=10.0, help="oracle timing budget at one thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the context legs (upper bound, sound mode, l2 balls, optimised root bounds, "
                         "branch and bound, library GEMM)")
    ap.add_argument("--profile-only", action="store_true",
                    help="build the batch, autotune, then run only the per-kernel timing pass (for rocprofv3)")
    ap.add_argument("--profile-reps", type=int, default=5)
    ap.add_argument("--bab-rounds", type=int, default=16, help="branch-and-bound rounds timed as context")
    ap.add_argument("--bab-batch", type=int, default=1024, help="subdomains split per branch-and-bound round")
    ap.add_argument("--bab-warm", action="store_true", help="warm-start branch-and-bound children from their parents")
    ap.add_argument("--plan", default=None, help="dense-chain plan bwd,fwd (1,1 fused chains, 0,0 per-layer kernels); overrides the autotuner")
    ap.add_argument("--parts", type=int, default=0,
                    help="concurrent sub-batches of the optimiser (0: the library's default)")
    ap.add_argument("--conv-variant", type=int, default=None,
                    help="force one conv kernel variant on every conv layer (0-3; overrides the autotuner)")
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="size of the plain device copy of --calib-only (counter calibration)")
    ap.add_argument("--calib-only", action="store_true",
                    help="only the plain device copy of --calib-copy-mib MiB (a counter run's calibration)")
    ap.add_argument("--ingest-traffic", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR",
                                                          "CAL_WRITE_DIR", "PROFILE_OUT"),
                    help="host only: write profiles/traffic.txt's entry from counter runs of --profile-only")
    ap.add_argument("--counters-summary", nargs="+", metavar="PATH",
                    help="host only: PROFILE_OUT then counter-run directories of --profile-only; "
                         "prints a markdown table per kernel")
    ap.add_argument("--trace-summary", nargs=2, metavar=("PROFILE_OUT", "RESULTS_DB"),
                    help="host only: the timing pass's kernel durations from a rocprofv3 --kernel-trace database")
    args = ap.parse_args()
    if args.trace_summary:
        return trace_summary(args)
    if args.ingest_traffic:
        return ingest_traffic(args)
    if args.counters_summary:
        return counters_summary(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 (subdomains are "
                                   "independent, so a batch would shard across GPUs by subdomain ranges, "
                                   "one process each; that is not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_06624_amd import api, synth

    torch.cuda.set_device(0)
    if args.calib_only:
        n = args.calib_copy_mib * (1 << 20) // 4
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_mib": args.calib_copy_mib}))
        return
    name = args.workload
    log(f"[bench] workload {name}: building inputs")
    wl = synth.make(name)
    t0 = time.perf_counter()
    lo, up = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi)
    t_root = time.perf_counter() - t0
    sp = synth.attach_splits(wl, lo, up)
    pb = api.BoundProblem.from_workload(wl, lo, up)
    B, m = pb.B, pb.m
    if args.parts:
        pb.set_parts(args.parts)
    if not args.no_autotune:
        log("[bench] autotune")
        pb.autotune()
    if args.plan:
        cb, cf = (int(x) for x in args.plan.split(","))
        pb.set_plan(cb, cf)
    if args.conv_variant is not None:
        pb.set_conv_variant(args.conv_variant)
    variant_names = ["row-major/LDS weights", "row-major/global weights", "subdomain-major/LDS weights",
                     "subdomain-major/global weights"]
    conv_plan = {f"layer{i + 1}": {"back_substitution": variant_names[pb.conv_variant(i + 1, 0)],
                                   "adjoint": variant_names[pb.conv_variant(i + 1, 1)]}
                 for i, ly in enumerate(wl.net.layers) if ly.kind == synth.CONV}
    a0 = pb.alpha_init()
    b0 = pb.zeros_beta()

    if args.profile_only:
        log(f"[bench] profile pass only ({args.profile_reps} reps)")
        stats, kern = kernel_table(pb, a0, b0, args.profile_reps)
        torch.cuda.synchronize()
        print(json.dumps({"workload": name, "profile_reps": args.profile_reps, "conv_plan": conv_plan,
                          "roofline": roofline(stats, kern, name, conv_plan),
                          "kernels": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in kk.items()}
                                      for kk in kern]}), flush=True)
        return

    alpha, beta = a0.clone(), b0.clone()
    best = torch.empty(pb.n_rows, device="cuda")
    last = torch.empty(pb.n_rows, device="cuda")
    opt = dict(iters=args.iters, lr_alpha=args.lr_alpha, lr_beta=args.lr_beta, decay=args.decay, lb_best=best,
               lb_last=last)
    log(f"[bench] B={B} m={m} n_alpha={pb.n_alpha} n_beta={pb.n_beta}; warmup {args.warmup}")
    for _ in range(args.warmup):
        pb.optimize(alpha, beta, **opt)
    torch.cuda.synchronize()

    # ---- timed region: K optimisation steps
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pb.optimize(alpha, beta, **opt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el / args.steps * 1e3
    value = B / (ms_step / 1e3)
    log(f"[bench] {ms_step:.3f} ms per step, {value:.1f} subdomain bounds/s")

    # ---- plain evaluation of the same batch
    lb = torch.empty(pb.n_rows, device="cuda")
    for _ in range(3):
        pb.eval(a0, b0, out=lb)
    torch.cuda.synchronize()
    n_eval = max(20, args.steps * 5)
    t0 = time.perf_counter()
    for _ in range(n_eval):
        pb.eval(a0, b0, out=lb)
    torch.cuda.synchronize()
    ms_eval = (time.perf_counter() - t0) / n_eval * 1e3

    # ---- a clean 20-iteration run from the default start: the bounds and the
    # final iterate the oracle leg checks
    alpha.copy_(a0)
    beta.copy_(b0)
    pb.optimize(alpha, beta, **opt)
    gpu = {"best": best.view(B, m).cpu().numpy().astype(np.float64),
           "last": last.view(B, m).cpu().numpy().astype(np.float64),
           "alpha": alpha.cpu().numpy(), "beta": beta.cpu().numpy(), "sound": None}

    ctx = {}
    n_sound = max(3, args.steps // 4)
    if not args.no_context:
        # ---- the primal side on the same batch: bound, x*, the network at x*
        # and the split check (cv_bound_upper), at the default start
        log("[bench] upper bound")
        for _ in range(3):
            _, ub, sat = pb.upper(a0, b0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_eval):
            _, ub, sat = pb.upper(a0, b0)
        torch.cuda.synchronize()
        ms_upper = (time.perf_counter() - t0) / n_eval * 1e3
        ctx["upper_bound"] = {"value": round(B / (ms_upper / 1e3), 1),
                              "unit": "subdomain (lower, upper) bound pairs/s", "ms_per_call": round(ms_upper, 4),
                              "rows_meeting_splits": int(sat.sum().item()),
                              "rows_below_zero": int((ub < 0).sum().item())}

        # ---- sound mode end to end: the sound root bounds (every bound moved
        # outward by its rigorous float32 margin), subdomains drawn against
        # them, and the margin on every reported bound; optimiser throughput,
        # the margin against the plain float32 bound of the same problem, and
        # the final iterate for the oracle's soundness count
        log("[bench] sound mode")
        lo_s, up_s = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi, sound=True)
        wl_s = synth.make(name)
        sp_s = synth.attach_splits(wl_s, lo_s, up_s)
        pb_s = api.BoundProblem.from_workload(wl_s, lo_s, up_s, sp_s)
        if args.parts:
            pb_s.set_parts(args.parts)
        pb_s.set_sound(1)
        a_s0, b_s0 = pb_s.alpha_init(), pb_s.zeros_beta()
        a_s, b_s = a_s0.clone(), b_s0.clone()
        best_s = torch.empty(pb_s.n_rows, device="cuda")
        last_s = torch.empty(pb_s.n_rows, device="cuda")
        opt_s = dict(opt, lb_best=best_s, lb_last=last_s)
        for _ in range(2):
            pb_s.optimize(a_s, b_s, **opt_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_sound):
            pb_s.optimize(a_s, b_s, **opt_s)
        torch.cuda.synchronize()
        ms_sound = (time.perf_counter() - t0) / n_sound * 1e3
        a_s.copy_(a_s0)
        b_s.copy_(b_s0)
        pb_s.optimize(a_s, b_s, **opt_s)
        gpu["sound"] = {"best": best_s.view(B, m).cpu().numpy().astype(np.float64),
                        "last": last_s.view(B, m).cpu().numpy().astype(np.float64),
                        "alpha": a_s.cpu().numpy(), "beta": b_s.cpu().numpy(), "lo": lo_s, "up": up_s,
                        "splits": sp_s}
        lb_s = pb_s.eval(a_s0, b_s0)
        pb_s.set_sound(0)
        lb_p = pb_s.eval(a_s0, b_s0)
        rel_margin = ((lb_p - lb_s) / lb_p.abs().clamp(min=1.0)).max().item()
        ctx["sound_mode"] = {"value": round(pb_s.B / (ms_sound / 1e3), 1), "unit": "subdomain bounds/s",
                             "ms_per_step": round(ms_sound, 4), "root_bounds": "sound (float64 with its rounding margin, rounded outward)",
                             "max_rel_margin": rel_margin, "min_margin": (lb_p - lb_s).min().item()}
        pb_s.close()

        # ---- l2-ball input sets: the same properties over the balls of radius
        # eps around x0 (inscribed in the unclipped box, whose root bounds hold
        # over them), same subdomain count; optimiser throughput
        log("[bench] l2 balls")
        x0 = np.asarray(wl.x0, np.float32)
        eps_l2 = np.full(wl.n_props, wl.eps, np.float32)
        lo_b, up_b = api.root_bounds(wl.net.layers, np.nextafter(x0 - eps_l2[:, None], np.float32(-np.inf)),
                                     np.nextafter(x0 + eps_l2[:, None], np.float32(np.inf)))
        wl_b = synth.make(name)
        sp_b = synth.attach_splits(wl_b, lo_b, up_b)
        pb_b = api.BoundProblem.from_workload(wl_b, lo_b, up_b, sp_b)
        if args.parts:
            pb_b.set_parts(args.parts)
        pb_b.set_input_l2(x0, eps_l2)
        a_b, b_b = pb_b.alpha_init(), pb_b.zeros_beta()
        opt_b = dict(iters=args.iters, lr_alpha=args.lr_alpha, lr_beta=args.lr_beta, decay=args.decay)
        for _ in range(2):
            pb_b.optimize(a_b.clone(), b_b.clone(), **opt_b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_sound):
            best_b, _ = pb_b.optimize(a_b.clone(), b_b.clone(), **opt_b)
        torch.cuda.synchronize()
        ms_l2 = (time.perf_counter() - t0) / n_sound * 1e3
        ctx["l2_ball"] = {"value": round(pb_b.B / (ms_l2 / 1e3), 1), "unit": "subdomain bounds/s",
                          "ms_per_step": round(ms_l2, 4), "radius": float(wl.eps),
                          "mean_bound": float(best_b.mean().item())}
        pb_b.close()

        # ---- optimised intermediate bounds (each bound over its own alpha',
        # 20 Adam steps): time, how much they narrow the intervals, and what
        # they do to the bound of the batch at the default start
        log("[bench] optimised root bounds")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo_o, up_o = api.root_bounds(wl.net.layers, wl.x_lo, wl.x_hi, opt_iters=args.iters, lr_alpha=0.1,
                                     decay=args.decay)
        t_ropt = time.perf_counter() - t0
        w_c, w_o = (up - lo), (up_o - lo_o)
        # the same generator keys: only subdomains that split a neuron the
        # tighter bounds made stable change
        wl_o = synth.make(name)
        sp_o = synth.attach_splits(wl_o, lo_o, up_o)
        pb_o = api.BoundProblem.from_workload(wl_o, lo_o, up_o, sp_o)
        lb_o = pb_o.eval(pb_o.alpha_init(), pb_o.zeros_beta())
        lb_c = pb.eval(a0, b0)
        ctx["optimised_root_bounds"] = {"seconds": round(t_ropt, 3),
                                        "mean_width_ratio": float(np.mean(w_o / np.maximum(w_c, 1e-12))),
                                        "rows_improved": int((lb_o > lb_c).sum().item()),
                                        "mean_bound_gain": float((lb_o - lb_c).mean().item())}
        pb_o.close()

        # ---- joint optimisation of intermediate bounds at every property's root
        log("[bench] joint optimisation of intermediate bounds")
        ctx["joint_intermediate_bounds"] = joint_context(wl, lo, up, args)

        # ---- branch and bound (Alg. 1) on property 0 of the workload, each
        # row's objective offset to the middle of its root [lower, upper]
        # bound (an extra constant output carries the offsets), so that the
        # search has to branch; a fixed number of rounds of `batch` splits each
        log("[bench] branch and bound")
        ctx["branch_and_bound"] = bab_context(wl, lo, up, args)

        # ---- context: the vendor library's plain FP32 GEMM (no epilogue) at
        # the back-substitution shapes of the dense layers, same rows
        ctx["library_fp32_gemm"] = library_gemm_context(wl, pb.n_rows)

    # ---- per-kernel durations with HIP events on the launch stream
    log("[bench] per-kernel event timing")
    stats, kern = kernel_table(pb, a0, b0, args.profile_reps)
    roof = roofline(stats, kern, name, conv_plan)
    on_mfma = [s for s in stats if s["name"].startswith(("gemm", "chain", "conv"))]
    gemm_fl = sum(s["flops"] for s in on_mfma)
    gemm_ms = sum(s["total_ms"] / s["reps"] for s in on_mfma)
    all_ms = sum(s["total_ms"] / s["reps"] for s in stats)

    line = {
        "metric": "subdomain bounds/sec (20-iter alpha/beta opt) vs plain eval; rel err vs FP64",
        "value": round(value, 1),
        "unit": "subdomain bounds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: {WORKLOAD_TEXT[name]}", "subdomains": B, "spec_rows": m,
                   "adam_iters": args.iters, "lr_alpha": args.lr_alpha, "lr_beta": args.lr_beta,
                   "lr_decay": args.decay, "root_bounds": "per-layer CROWN on the GPU"},
        "plain_eval": {"value": round(B / (ms_eval / 1e3), 1), "unit": "subdomain bounds/s",
                       "ms_per_eval": round(ms_eval, 4)},
        "roofline": roof,
        "conv_plan": conv_plan,
        "mfma_kernels_tflops": round(gemm_fl / (gemm_ms * 1e-3) / 1e12, 3) if gemm_ms else None,
        "mfma_kernels_time_share": round(gemm_ms / all_ms, 4) if all_ms else None,
    }
    line.update(ctx)
    line["kernels"] = [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in kk.items()} for kk in kern]
    line["root_bounds_s"] = round(t_root, 3)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cb, rel, snd, rel_sound = cpu_baseline(name, wl, lo, up, sp, gpu, args.cpu_seconds, args.cpu_seconds_1t,
                                               args.iters, args.lr_alpha, args.lr_beta, args.decay)
        line["cpu_baseline"] = cb
        line["rel_err_vs_fp64"] = rel
        line["soundness"] = snd
        if rel_sound is not None:
            line["rel_err_vs_fp64_sound_mode"] = rel_sound
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
