"""Summaries of rocprofv3 results for the committed profiles (text only).

    python -m paper_2201_06174_amd.profiling stats DB TITLE COMMAND [TOP] > profiles/NAME.md
    python -m paper_2201_06174_amd.profiling traffic FETCH_DB WRITE_DB KERNEL COPY_BYTES COMMAND > profiles/NAME.txt
    python -m paper_2201_06174_amd.profiling mfma DB SOURCES KERNEL [KERNEL ...] -- COMMAND > profiles/NAME.txt

``stats`` renders the kernel-trace statistics table of one ``--kernel-trace --stats``
run.  ``traffic`` combines one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of
``bench.py --traffic-pass``: that pass first launches a plain device copy of
COPY_BYTES bytes (it reads and writes exactly that many bytes), then the timed
feature kernel.  Each counter of the feature kernel is scaled by COPY_BYTES over what
the same counter reads for the copy, and the result is stored together with a
digest of the kernel's source files, so a later change of the kernel makes the
stored figure stale (bench.py then reports the traffic as null).  ``mfma`` reads one run with
the MFMA_COUNTERS and stores, per named kernel, the matrix-core flops the hardware counted for
one launch (SQ_INSTS_VALU_MFMA_MOPS_* count multiply and add operations in units of 512), with
the digest of the source set SOURCES (fp32, lowp or adjoint).
"""
from __future__ import annotations

import hashlib
import os
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# the sources of the FP32 feature kernel's code, launch shape and memory accesses (the
# host-built constant tables change values, not traffic)
FP32_KERNEL_SOURCES = ("sal_project.hip", "sal_stage.h", "sal_grid.h", "sal_passb.h", "sal_aux.h", "sal_internal.h")


LOWP_KERNEL_SOURCES = ("sal_lowp.hip", "sal_stage.h", "sal_grid.h", "sal_aux.h", "sal_internal.h")
ADJOINT_SOURCES = FP32_KERNEL_SOURCES + ("sal_backward.hip", "sal_device.h")
SOURCE_SETS = {"fp32": FP32_KERNEL_SOURCES, "lowp": LOWP_KERNEL_SOURCES, "adjoint": ADJOINT_SOURCES}

# one rocprofv3 --pmc pass: 5 SQ counters and 1 GRBM counter
MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F16",
                 "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def source_digest(files=FP32_KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read() + b"\0")
    return h.hexdigest()[:16]


def stats_rows(db):
    con = sqlite3.connect(db)
    try:
        return list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    finally:
        con.close()


def launches_by_grid(db):
    """[(kernel, grid work-items, workgroup size, calls, average us)] from the dispatch records,
    largest total first: one kernel runs at several sizes in a run (the timed volume, the
    batch members), and only the launches of one size compare with a timed figure."""
    con = sqlite3.connect(db)
    try:
        rows = list(con.execute("select name, grid_x, workgroup_x, duration from kernels"))
    finally:
        con.close()
    acc = defaultdict(list)
    for name, gx, wx, dur in rows:
        acc[(name, gx, wx)].append(dur)
    out = [(k[0], k[1], k[2], len(v), sum(v) / len(v) / 1e3) for k, v in acc.items()]
    return sorted(out, key=lambda r: -r[3] * r[4])


def stats_markdown(db, title, command, top=30) -> str:
    """Every kernel of the run, then its `top` launch-size groups with the largest total time."""
    out = ["# %s" % title, "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
           "rocprofv3 kernel-trace statistics (durations in microseconds):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in stats_rows(db):
        out.append("| `%s` | %d | %.1f | %.2f | %.2f |" % (name, calls, total, avg, pct))
    out += ["", "The same dispatches by launch size (grid in work-items; the %d with the largest total time):" % top,
            "", "| kernel | grid | workgroup | calls | average us |", "|---|---|---|---|---|"]
    for name, gx, wx, calls, avg in launches_by_grid(db)[:top]:
        out.append("| `%s` | %d | %d | %d | %.2f |" % (name, gx, wx, calls, avg))
    return "\n".join(out) + "\n"


def counter_per_dispatch(db, counter):
    """{kernel name: [value of `counter` summed over its instances, per dispatch]}."""
    con = sqlite3.connect(db)
    try:
        rows = list(con.execute("select kernel_name, dispatch_id, value from counters_collection where counter_name = ?",
                                (counter,)))
    finally:
        con.close()
    per = defaultdict(float)
    names = {}
    for name, disp, val in rows:
        per[disp] += float(val)
        names[disp] = name
    out = defaultdict(list)
    for disp in sorted(per):
        out[names[disp]].append(per[disp])
    return out


def _pick(per, substrs, at_least=0.0):
    """(name, values) of the kernel matching one of `substrs` with the largest mean, keeping
    only its dispatches whose value is at least `at_least`."""
    hits = []
    for k, v in per.items():
        if any(sub in k for sub in substrs):
            v = [x for x in v if x >= at_least]
            if v:
                hits.append((k, v))
    if not hits:
        raise KeyError("no dispatch of a kernel matching %r" % (substrs,))
    return max(hits, key=lambda kv: sum(kv[1]) / len(kv[1]))


def traffic_text(fetch_db, write_db, kernel, copy_bytes, command) -> str:
    lines = ["# HBM traffic of one launch of %s" % kernel, "command: %s" % command]
    vals = {}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        per = counter_per_dispatch(db, counter)
        # the device-to-device copy runs as the runtime's blit kernel; smaller copies of the
        # run (tables, parameters) are left out by size
        copy_name, copy_kib = _pick(per, ("copyBuffer",), at_least=copy_bytes / 1024.0 / 16)
        kern_name, kern_kib = _pick(per, (kernel,))
        copy_mean = sum(copy_kib) / len(copy_kib)
        kern_mean = sum(kern_kib) / len(kern_kib)
        factor = copy_bytes / (copy_mean * 1024.0)
        vals[counter] = kern_mean * 1024.0 * factor
        lines += ["%s_copy_kib_per_dispatch: %.1f" % (counter.lower(), copy_mean),
                  "%s_copy_factor: %.4f" % (counter.lower(), factor),
                  "%s_kernel_kib_per_dispatch: %.1f" % (counter.lower(), kern_mean),
                  "%s_kernel_dispatches: %d" % (counter.lower(), len(kern_kib)),
                  "%s_bytes_per_launch: %.0f" % (counter.lower(), vals[counter])]
    lines += ["kernel_name: %s" % kern_name, "copy_kernel: %s" % copy_name, "copy_bytes: %d" % copy_bytes,
              "traffic_bytes_per_launch: %.0f" % (vals["FETCH_SIZE"] + vals["WRITE_SIZE"]),
              "source_digest: %s" % source_digest()]
    return "\n".join(lines) + "\n"


def mfma_text(db, sources, kernels, command) -> str:
    """Matrix-core flops per launch of each kernel (mean over its dispatches in the run)."""
    per = {c: counter_per_dispatch(db, c) for c in MFMA_COUNTERS}
    lines = ["# Matrix-core work per launch, counted by the hardware", "command: %s" % command]
    for k in kernels:
        name, mops = None, 0.0
        for c in ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F16"):
            hits = {n: v for n, v in per[c].items() if k in n}
            if hits:
                n, v = max(hits.items(), key=lambda kv: sum(kv[1]) / len(kv[1]))
                name = n
                mops += sum(v) / len(v)
        if name is None:
            raise KeyError("no dispatch of a kernel matching %r" % k)
        busy = per["SQ_VALU_MFMA_BUSY_CYCLES"].get(name, [0.0])
        key = k.replace(" ", "")
        lines += ["%s.kernel_name: %s" % (key, name),
                  "%s.dispatches: %d" % (key, len(busy)),
                  "%s.mfma_flops_per_launch: %.0f" % (key, 512.0 * mops),
                  "%s.mfma_busy_cycles_per_launch: %.0f" % (key, sum(busy) / len(busy))]
    lines.append("source_digest: %s" % source_digest(SOURCE_SETS[sources]))
    return "\n".join(lines) + "\n"


def read_mfma(path, kernel, sources):
    """Stored matrix-core flops per launch of `kernel`, or None when missing or stale."""
    t = read_traffic(path)
    if not t or t.get("source_digest") != source_digest(SOURCE_SETS[sources]):
        return None
    v = t.get("%s.mfma_flops_per_launch" % kernel.replace(" ", ""))
    return float(v) if v is not None else None


def read_traffic(path):
    """Parsed key/value lines of a stored traffic summary, or None."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        sys.stdout.write(stats_markdown(argv[1], argv[2], argv[3], *(int(a) for a in argv[4:5])))
        return 0
    if len(argv) >= 5 and argv[0] == "mfma" and "--" in argv:
        cut = argv.index("--")
        sys.stdout.write(mfma_text(argv[1], argv[2], argv[3:cut], " ".join(argv[cut + 1:])))
        return 0
    if len(argv) >= 6 and argv[0] == "traffic":
        sys.stdout.write(traffic_text(argv[1], argv[2], argv[3], int(argv[4]), argv[5]))
        return 0
    sys.stderr.write(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
