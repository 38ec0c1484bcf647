"""Host-side tools of bench.py that turn rocprofv3 output into the committed
profiles (no GPU): the naming of a counter run's timing-pass dispatches, the
per-kernel counter table over one or several runs, and the source hash that
keys the traffic record."""
import csv
import json
import os
import types

import pytest

import bench


def _prof(kernels, reps=1):
    return {"profile_reps": reps,
            "kernels": [{"name": n, "launches_per_pass": k, "avg_us": 10.0 * (i + 1), "tflops": 1.0 + i}
                        for i, (n, k) in enumerate(kernels)]}


def _write_run(tmp, tag, prof, launches, counters, lead=()):
    """A counter run: its printed line, and a CSV with the dispatches of
    `lead` (autotuner launches) followed by the timing pass, every launch
    issued 8 times; launches = [(symbol, grid)] in pass order per rep."""
    out = tmp / f"{tag}.out"
    out.write_text("[bench] some log line\n" + json.dumps(prof) + "\n")
    d = tmp / tag / "run"
    d.mkdir(parents=True)
    rows, did = [], 0
    seq = [(s, g, 1) for s, g in lead] + [(s, g, 8) for _ in range(prof["profile_reps"]) for s, g in launches]
    for sym, grid, times in seq:
        for _ in range(times):
            did += 1
            for c, v in counters.items():
                rows.append({"Process_Id": 7, "Dispatch_Id": did, "Kernel_Name": sym, "Grid_Size": grid,
                             "Counter_Name": c, "Counter_Value": v})
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    return str(out), str(tmp / tag)


def test_profile_pass_names_follow_pass_order_and_shared_symbols(tmp_path):
    # two names share a symbol and grid (a first-layer step and a later layer's)
    prof = _prof([("bwd", 2), ("fwd_x", 1), ("fwd", 2)], reps=2)
    launches = [("k_bwd", 64), ("k_bwd", 64), ("k_fwd", 32), ("k_fwd", 32), ("k_fwd", 32)]
    out, d = _write_run(tmp_path, "a", prof, launches, {"SQ_INSTS_VALU": 5.0}, lead=[("k_tune", 8)] * 3)
    named = bench.name_profile_pass(bench.counter_dispatches(d), prof)
    assert {k: len(v) for k, v in named.items()} == {"bwd": 32, "fwd_x": 16, "fwd": 32}
    assert all(x["kernel"] == "k_fwd" for x in named["fwd_x"] + named["fwd"])


def test_profile_pass_rejects_a_misaligned_run(tmp_path):
    prof = _prof([("bwd", 1), ("fwd", 1)])
    out, d = _write_run(tmp_path, "a", prof, [("k_bwd", 64), ("k_fwd", 32)], {"SQ_INSTS_VALU": 1.0})
    disp = bench.counter_dispatches(d)
    with pytest.raises(SystemExit):
        bench.name_profile_pass(disp[:-1], prof)  # one dispatch short: groups straddle two kernels


def test_counters_summary_merges_runs_with_different_plans(tmp_path, capsys):
    # the two counter runs chose different dense kernels; the conv kernel is common
    pa = _prof([("conv", 1), ("dense_a", 1)])
    pb = _prof([("chain", 1), ("conv", 1)])
    ca = {"GRBM_GUI_ACTIVE": 8.0, "SQ_VALU_MFMA_BUSY_CYCLES": 512.0, "SQ_INSTS_LDS": 3e6}
    cb = {"GRBM_GUI_ACTIVE": 8.0, "SQ_INSTS_VALU": 2e6, "SQ_INSTS_MFMA": 1e6}
    oa, da = _write_run(tmp_path, "A", pa, [("k_conv", 64), ("k_dense", 16)], ca)
    ob, db = _write_run(tmp_path, "B", pb, [("k_chain", 16), ("k_conv", 64)], cb)
    bench.counters_summary(types.SimpleNamespace(counters_summary=[oa, da, ob, db]))
    rows = {ln.split("|")[1].strip(): [c.strip() for c in ln.split("|")[2:-1]]
            for ln in capsys.readouterr().out.splitlines()[2:]}
    assert set(rows) == {"conv", "dense_a", "chain"}
    # conv: MFMA busy from run A (512 / (8 / 8 x 1024)), instruction counts from run B
    assert rows["conv"][2] == "0.500" and rows["conv"][3] == "2.00" and rows["conv"][4] == "1.00"
    assert rows["conv"][5] == "3.00"
    assert rows["dense_a"][3] == "-" and rows["chain"][2] == "-"


def test_counters_summary_single_output_form(tmp_path, capsys):
    p = _prof([("conv", 1)])
    o, da = _write_run(tmp_path, "A", p, [("k_conv", 64)], {"SQ_INSTS_VALU": 4e6})
    _, db = _write_run(tmp_path, "B", p, [("k_conv", 64)], {"SQ_INSTS_MFMA": 1e6})
    bench.counters_summary(types.SimpleNamespace(counters_summary=[o, da, db]))
    line = capsys.readouterr().out.splitlines()[2]
    cells = [c.strip() for c in line.split("|")[1:-1]]
    assert cells[0] == "conv" and cells[4] == "4.00" and cells[5] == "1.00"


def test_kernel_source_hash_covers_device_sources_only(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0 and bench.kernel_source_hash() == h
    # a copy of the sources: editing the host ABI layer keeps the hash, a kernel source changes it
    src = os.path.join(bench.ROOT, "paper_2103_06624_amd", "csrc")
    dst = tmp_path / "paper_2103_06624_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in os.listdir(src):
        (dst / f).write_bytes(open(os.path.join(src, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h
    (dst / "api.hip").write_text((dst / "api.hip").read_text() + "\n// host-only edit\n")
    assert bench.kernel_source_hash() == h
    (dst / "conv.hip").write_text((dst / "conv.hip").read_text() + "\n// kernel edit\n")
    assert bench.kernel_source_hash() != h
