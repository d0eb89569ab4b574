"""Summaries of rocprofv3 output for the query path (a developer utility).

    python -m paper_1807_08692_amd.profsum trace TRACE_CSV > summary.md
    python -m paper_1807_08692_amd.profsum traffic FETCH_CSV WRITE_CSV OUT_JSON [--merge] > table.md
    python -m paper_1807_08692_amd.profsum mfma COUNTER_CSV > mfma.md
    python -m paper_1807_08692_amd.profsum counters COUNTER_CSV > counters.md

`trace` reads a --kernel-trace CSV (one row per dispatch) and prints, per
kernel, the dispatch count and mean duration over all dispatches and over the
working dispatches only: the solver queues iterations ahead of its stopping
test, and an iteration queued after every column stopped returns at once
(a few microseconds), which would otherwise pull the mean down.

`traffic` reads the FETCH_SIZE and WRITE_SIZE counter CSVs of two --pmc runs
that include a 1 GiB device copy (the library's own probe copy kernel,
hd::k_probe_copy of hd_probe_memory mode 1, or grid 131072 of
__amd_rocclr_copyBuffer), scales each counter by what it reads for that copy
(1 GiB read and written),
and writes per-kernel HBM-side bytes per dispatch to OUT_JSON together with a
SHA-256 of each kernel's source file, so that a later run can tell whether the
kernel has changed since the counters were taken.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# kernel name prefix -> (kind used by bench.py, source file)
KINDS = {
    "hd::k_spmm": ("spmm", "k_spmm.hip"),
    "hd::k_ut_p_tn": ("ut_p", "k_ugemm_bf16.hip"),
    "hd::k_ut_p": ("ut_p", "k_ugemm.hip"),
    "hd::k_u_c_tn": ("u_c", "k_ugemm_bf16.hip"),
    "hd::k_uc_update_r_tn": ("u_c", "k_ugemm_bf16.hip"),
    "hd::k_u_c": ("u_c", "k_ugemm.hip"),
    "hd::k_update_xp_pt": ("update_xp", "k_cg.hip"),
    "hd::k_update_xp": ("update_xp", "k_cg.hip"),
    "hd::k_update_r": ("update_r", "k_cg.hip"),
    "hd::k_combine_tn": ("combine", "k_ugemm_bf16.hip"),
    "hd::k_combine": ("combine", "k_ugemm.hip"),
    "hd::k_xt": ("combine", "k_ugemm.hip"),
    "hd::k_sim_bf16": ("sim", "k_ugemm_bf16.hip"),
    "hd::k_sim": ("sim", "k_sim.hip"),
    "hd::k_cg_persist": ("cg_persist", "k_persist.hip"),
    "hd::k_combine_narrow": ("combine", "k_persist.hip"),
    "hd::k_probe_read": ("probe", "k_probe.hip"),
    "hd::k_probe_copy": ("probe", "k_probe.hip"),
    "hd::k_probe_gather": ("probe", "k_probe.hip"),
    "hd::k_probe_graph": ("probe", "k_probe.hip"),
    "hd::k_gram_tn": ("eig", "k_eig_gemm.hip"),
    "hd::k_rotate_nn": ("eig", "k_eig_gemm.hip"),
}


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def kind_of(name: str):
    n = short(name)
    for pre in sorted(KINDS, key=len, reverse=True):
        if n == pre or n.startswith(pre + "<"):
            return KINDS[pre]
    return None


def sha(fname: str) -> str:
    with open(os.path.join(CSRC, fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def trace(path: str, work_frac: float = 0.05) -> str:
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in per.values())
    out = ["| kernel | dispatches | mean us (all) | working dispatches | mean us (working) | % of GPU time |",
           "|---|---|---|---|---|---|"]
    for k in sorted(per, key=lambda k: -sum(per[k])):
        v = per[k]
        if not k.startswith("hd::") or sum(v) < 1e-4 * total:
            continue
        mx = max(v)
        work = [t for t in v if t >= work_frac * mx]
        out.append(f"| {k} | {len(v)} | {sum(v) / len(v):.1f} | {len(work)} | {sum(work) / len(work):.1f} "
                   f"| {100 * sum(v) / total:.2f} |")
    return "\n".join(out)


def traffic(fetch_csv: str, write_csv: str, out_json: str, merge: bool = False) -> str:
    def agg(fn):
        a = collections.defaultdict(list)
        copy = []
        for r in csv.DictReader(open(fn)):
            v = float(r["Counter_Value"])
            if ("copyBuffer" in r["Kernel_Name"] and r["Grid_Size"] == "131072") or \
                    short(r["Kernel_Name"]) == "hd::k_probe_copy":
                copy.append(v)
            a[short(r["Kernel_Name"])].append(v)
        return a, copy
    fs, cf = agg(fetch_csv)
    ws, cw = agg(write_csv)
    if not cf or not cw:
        raise SystemExit("no 1 GiB copy dispatch in the counter runs (bench.py --probes 1 or --copy-calibration)")
    kf = 1048576.0 / (sum(cf) / len(cf))
    kw = 1048576.0 / (sum(cw) / len(cw))
    rows = ["| kernel | dispatches | FETCH_SIZE KiB (mean) | fetched GB | WRITE_SIZE KiB (mean) | written GB |",
            "|---|---|---|---|---|---|"]
    res = {"scale_fetch": kf, "scale_write": kw, "kernels": {}}
    for k in sorted(fs, key=lambda k: -sum(fs[k])):
        kd = kind_of(k)
        if not k.startswith("hd::"):
            continue
        # working dispatches only (a skipped iteration fetches a few bytes)
        mx = max(fs[k])
        f = [v for v in fs[k] if v >= 0.05 * mx]
        wv = [v for v in ws.get(k, []) if v >= 0.05 * max(ws.get(k, [0.0]) or [0.0])] or [0.0]
        fb, wb = sum(f) / len(f) * kf * 1024, sum(wv) / len(wv) * kw * 1024
        rows.append(f"| {k} | {len(f)} | {sum(f) / len(f):.0f} | {fb / 1e9:.3f} | {sum(wv) / len(wv):.0f} | {wb / 1e9:.3f} |")
        if kd:
            res["kernels"][k] = {"kind": kd[0], "fetch_bytes": fb, "write_bytes": wb,
                                 "source": kd[1], "sha256": sha(kd[1])}
    if merge and os.path.exists(out_json):
        # add this run's kernels (for instance another launch variant) to an
        # existing summary; entries of kernels measured again are replaced
        old = json.load(open(out_json))
        old["kernels"].update(res["kernels"])
        res["kernels"] = old["kernels"]
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    head = (f"Counter scaling from the 1 GiB copy: FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f}.\n\n")
    return head + "\n".join(rows)


def mfma(path: str) -> str:
    """Matrix-core use per kernel from a --pmc pass with SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_BUSY_CU_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_LDS_BANK_CONFLICT and
    GRBM_GUI_ACTIVE: per dispatch, each counter summed over its instances;
    means over the working dispatches (CU-busy cycles >= 5% of the kernel's
    largest). MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x
    SQ_BUSY_CU_CYCLES); LDS conflict = SQ_LDS_BANK_CONFLICT / SQ_BUSY_CU_CYCLES."""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])][r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
    out = ["| kernel | dispatches | MFMA busy | bf16 MFMA ops (x512 flop) per dispatch | LDS bank-conflict cycles / CU-busy cycles |",
           "|---|---|---|---|---|"]
    rows = []
    for k, disp in per.items():
        if not k.startswith("hd::"):
            continue
        busy = [d.get("SQ_BUSY_CU_CYCLES", 0.0) for d in disp.values()]
        mx = max(busy) if busy else 0.0
        work = [d for d in disp.values() if mx > 0 and d.get("SQ_BUSY_CU_CYCLES", 0.0) >= 0.05 * mx]
        if not work:
            continue
        mean = {c: sum(d.get(c, 0.0) for d in work) / len(work) for c in work[0]}
        if mean.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) <= 0.0:
            continue
        cu = mean.get("SQ_BUSY_CU_CYCLES", 0.0)
        rows.append((mean["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * len(work),
                     f"| {k} | {len(work)} | {mean.get('SQ_VALU_MFMA_BUSY_CYCLES', 0.0) / (4 * cu):.3f} "
                     f"| {mean['SQ_INSTS_VALU_MFMA_MOPS_BF16']:.4g} | {mean.get('SQ_LDS_BANK_CONFLICT', 0.0) / cu:.3f} |"))
    out += [r for _, r in sorted(rows, reverse=True)]
    return "\n".join(out)


def counters(path: str) -> str:
    """Per kernel, the mean of each counter per working dispatch (each counter
    summed over its instances; working = its first counter >= 5% of the
    kernel's largest), from one --pmc pass (e.g. TCC_HIT_sum TCC_MISS_sum, or
    TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_DRAM_sum)."""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    names = []
    for r in csv.DictReader(open(path)):
        per[short(r["Kernel_Name"])][r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
        if r["Counter_Name"] not in names:
            names.append(r["Counter_Name"])
    out = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    rows = []
    for k, disp in per.items():
        if not k.startswith("hd::"):
            continue
        first = [d.get(names[0], 0.0) for d in disp.values()]
        mx = max(first) if first else 0.0
        work = [d for d in disp.values() if mx > 0 and d.get(names[0], 0.0) >= 0.05 * mx]
        if not work:
            continue
        mean = [sum(d.get(c, 0.0) for d in work) / len(work) for c in names]
        rows.append((mean[0] * len(work), f"| {k} | {len(work)} | " + " | ".join(f"{v:.4g}" for v in mean) + " |"))
    out += [r for _, r in sorted(rows, reverse=True)]
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        print(trace(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], merge="--merge" in sys.argv[5:]))
    elif sys.argv[1] == "mfma":
        print(mfma(sys.argv[2]))
    elif sys.argv[1] == "counters":
        print(counters(sys.argv[2]))
    else:
        raise SystemExit(__doc__)
