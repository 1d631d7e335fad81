"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2208_12187_amd.profile_summary trace <kernel_stats.csv>
    python -m paper_2208_12187_amd.profile_summary bytes <fetch counter_collection.csv> \
        <write counter_collection.csv> <copy GiB> [<counters json to write>]

    python -m paper_2208_12187_amd.profile_summary mfma <counter_collection.csv>
    python -m paper_2208_12187_amd.profile_summary sq <counter_collection.csv>

``trace`` prints the per-kernel table of a ``--kernel-trace --stats`` run.
``mfma`` reads a run with the derived counters MfmaUtil (MFMA-busy cycles
over GPU-active cycles times the SIMD count, in percent) and MfmaFlopsF32 /
MfmaFlopsF64 / MfmaFlopsBF16 (512 times the MFMA operation counts) and prints
their per-dispatch means for every kernel.
``sq`` reads a run with wave-state counters (SQ_WAVE_CYCLES, SQ_WAIT_ANY,
SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS,
SQ_ACTIVE_INST_VMEM, SQ_WAIT_INST_LDS, SQ_LDS_BANK_CONFLICT) and prints, per
kernel, each as a share of the wave-cycles (bank conflicts as a share of
the LDS-active cycles).
``bytes`` reads one FETCH_SIZE pass and one WRITE_SIZE pass of the same
command, calibrates each counter against the plain device-to-device copy of
``copy GiB`` that the bench makes before timing (``--copy-gib``; the copy
reads and writes exactly that many bytes), and prints per-kernel HBM bytes.
With a json path it also records the FP32 d = 64 adjoint's per-launch
counters, the calibration factors and a hash of the kernel sources, which
the bench uses for the ``traffic`` field while the sources are unchanged.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "__amd_rocclr_copyBuffer"
# The FP32 d = 64 adjoint stage: its instances (the slices with and without the
# sampled last step) are summed per launch of the stage.
ADJOINT = "qoc::k_adjoint<float, 64, qoc::StdOps<float, 64>, false"


def short(name: str) -> str:
    name = name.replace("void ", "", 1)
    return name.split("(qoc::Work")[0].split("(int,")[0]


def csrc_sha256() -> str:
    csrc = os.path.join(HERE, "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read() for n in sorted(os.listdir(csrc)))
    return hashlib.sha256(src).hexdigest()


def trace_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg ms | min ms | max ms | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def per_kernel(path: str, counter: str):
    """kernel -> list of per-dispatch counter values (KiB)."""
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def calibration(vals, copy_gib: float) -> float:
    copies = vals.get(COPY_KERNEL, [])
    if not copies:
        raise SystemExit(f"no {COPY_KERNEL} dispatch: run the bench with --copy-gib")
    return copy_gib * (1 << 20) / max(copies)


def bytes_table(fetch_csv: str, write_csv: str, copy_gib: float, json_out: str | None = None) -> str:
    fv = per_kernel(fetch_csv, "FETCH_SIZE")
    wv = per_kernel(write_csv, "WRITE_SIZE")
    fs, ws = calibration(fv, copy_gib), calibration(wv, copy_gib)
    lines = [f"Calibration: the {copy_gib:g} GiB copy reads and writes {copy_gib * (1 << 20):.1f} KiB; "
             f"FETCH_SIZE reported {max(fv[COPY_KERNEL]):.1f} KiB and WRITE_SIZE {max(wv[COPY_KERNEL]):.1f} KiB, "
             f"so FETCH_SIZE is scaled by {fs:.4f} and WRITE_SIZE by {ws:.4f}.", "",
             "| kernel | dispatches | FETCH_SIZE KiB (raw, mean) | WRITE_SIZE KiB (raw, mean) | "
             "HBM read MB (scaled) | HBM write MB (scaled) |", "|---|---|---|---|---|---|"]
    for k in fv:
        if not k.startswith("qoc::") or k not in wv:
            continue
        f = sum(fv[k]) / len(fv[k])
        w = sum(wv[k]) / len(wv[k])
        lines.append(f"| `{k}` | {len(fv[k])} | {f:.1f} | {w:.1f} | {f * fs * 1.024e-3:.1f} | {w * ws * 1.024e-3:.1f} |")
    if json_out:
        inst = [k for k in fv if k.startswith(ADJOINT)]
        if not inst:
            raise SystemExit(f"no {ADJOINT}...> dispatch in {fetch_csv}")
        f = sum(sum(fv[k]) / len(fv[k]) for k in inst)
        w = sum(sum(wv[k]) / len(wv[k]) for k in inst)
        with open(json_out, "w") as fh:
            json.dump({"kernel": "k_adjoint<float, 64>", "fetch_kib": f, "write_kib": w, "fetch_scale": fs,
                       "write_scale": ws, "csrc_sha256": csrc_sha256(),
                       "workload": "fp32 d=64 m=12 N=2000 batch 32"}, fh, indent=1)
    return "\n".join(lines)


def mfma_table(path: str) -> str:
    names = ("MfmaUtil", "MfmaFlopsF32", "MfmaFlopsF64", "MfmaFlopsBF16")
    vals = {n: per_kernel(path, n) for n in names}
    kernels = [k for k in vals["MfmaUtil"] if k.startswith("qoc::")]
    out = ["| kernel | dispatches | MFMA busy % | MFMA GFLOP per dispatch (F32 / F64 / BF16) |", "|---|---|---|---|"]
    for k in kernels:
        u = vals["MfmaUtil"][k]
        fl = [sum(vals[n].get(k, [0.0])) / max(len(vals[n].get(k, [])), 1) / 1e9 for n in names[1:]]
        out.append(f"| `{k}` | {len(u)} | {sum(u) / len(u):.1f} | {fl[0]:.2f} / {fl[1]:.2f} / {fl[2]:.2f} |")
    return "\n".join(out)


SQ_SHARES = ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
             "SQ_ACTIVE_INST_VMEM", "SQ_WAIT_INST_LDS")


def sq_table(path: str) -> str:
    vals = {n: per_kernel(path, n) for n in ("SQ_WAVE_CYCLES", "SQ_LDS_BANK_CONFLICT") + SQ_SHARES}
    mean = lambda n, k: sum(vals[n].get(k, [0.0])) / max(len(vals[n].get(k, [])), 1)
    head = " | ".join(n.replace("SQ_", "") for n in SQ_SHARES)
    out = [f"| kernel | dispatches | {head} (share of wave-cycles) | LDS bank-conflict share of LDS-active |",
           "|---|---|" + "---|" * (len(SQ_SHARES) + 1)]
    for k in vals["SQ_WAVE_CYCLES"]:
        if not k.startswith("qoc::"):
            continue
        wc = mean("SQ_WAVE_CYCLES", k)
        if wc <= 0:
            continue
        shares = " | ".join(f"{mean(n, k) / wc:.3f}" for n in SQ_SHARES)
        lds = mean("SQ_ACTIVE_INST_LDS", k)
        bc = mean("SQ_LDS_BANK_CONFLICT", k) / lds if lds > 0 else 0.0
        out.append(f"| `{k}` | {len(vals['SQ_WAVE_CYCLES'][k])} | {shares} | {bc:.3f} |")
    return "\n".join(out)


def main(argv=None):
    a = sys.argv[1:] if argv is None else argv
    if a and a[0] == "trace" and len(a) == 2:
        print(trace_table(a[1]))
    elif a and a[0] == "mfma" and len(a) == 2:
        print(mfma_table(a[1]))
    elif a and a[0] == "sq" and len(a) == 2:
        print(sq_table(a[1]))
    elif a and a[0] == "bytes" and len(a) in (4, 5):
        print(bytes_table(a[1], a[2], float(a[3]), a[4] if len(a) == 5 else None))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main()
