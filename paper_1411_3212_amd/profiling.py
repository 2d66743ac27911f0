"""Summaries of rocprofv3 output for the kernels of libsj.

``stats``   kernel-trace statistics (``*_kernel_stats.csv``) -> a text table of
            the kernels by total time, with calls and average duration.
``traffic`` two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch)
            -> HBM bytes per dispatch of one kernel, each counter scaled by
            what it reads for the plain device copy of known size that
            ``bench.py --copy-probe`` runs (256 MiB read + 256 MiB written).

A traffic summary records a hash of the kernel sources; ``load_traffic``
returns nothing once the sources differ from the ones profiled.

    python -m paper_1411_3212_amd.profiling stats KERNEL_STATS_CSV OUT_TXT "COMMAND"
    python -m paper_1411_3212_amd.profiling traffic FETCH_CSV WRITE_CSV KERNEL OUT_TXT "COMMANDS"
"""
from __future__ import annotations

import csv
import hashlib
import re
import sys
from collections import defaultdict
from pathlib import Path

PKG = Path(__file__).resolve().parent
KERNEL_SOURCES = ["csrc/sj_kernels.hip", "csrc/sj_device.h", "csrc/sj_prims.hip"]
PROBE_BYTES = 256 << 20  # bytes read (and written) by one copy-probe dispatch


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update((PKG / rel).read_bytes())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    m = re.match(r"(?:void )?(sj::[A-Za-z0-9_]+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name.split("(")[0][:48]


def stats(csv_path: str, out_txt: str, command: str, top: int = 24) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}",
             f"# kernel sources: {source_hash()}",
             f"{'kernel':44s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'share':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        t = float(r["TotalDurationNs"])
        lines.append(f"{_short(r['Name']):44s} {int(r['Calls']):6d} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {t / 1e6:9.3f} {100 * t / tot:5.1f}%")
    lines.append(f"# all kernels: {tot / 1e6:.3f} ms")
    text = "\n".join(lines) + "\n"
    Path(out_txt).write_text(text)
    return text


def _per_kernel(csv_path):
    rows = list(csv.DictReader(open(csv_path)))
    agg = defaultdict(list)
    for r in rows:
        agg[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    probe = sorted((float(r["Counter_Value"]) for r in rows
                    if "copyBuffer" in r["Kernel_Name"]), reverse=True)
    return agg, probe


def traffic(fetch_csv: str, write_csv: str, kernel: str, out_txt: str, commands: str) -> str:
    fk, fprobe = _per_kernel(fetch_csv)
    wk, wprobe = _per_kernel(write_csv)
    # the three largest copy dispatches are the probe (256 MiB each)
    fcal = (PROBE_BYTES / 1024) / (sum(fprobe[:3]) / 3)
    wcal = (PROBE_BYTES / 1024) / (sum(wprobe[:3]) / 3)
    f = sum(fk[kernel]) / len(fk[kernel])
    w = sum(wk[kernel]) / len(wk[kernel])
    total = (f * fcal + w * wcal) * 1024
    text = "\n".join([
        f"# HBM traffic per dispatch of {kernel}",
        f"# commands: {commands}",
        f"# kernel sources: {source_hash()}",
        f"kernel {kernel}",
        f"dispatches {len(fk[kernel])}",
        f"fetch_kib {f:.1f}",
        f"write_kib {w:.1f}",
        f"probe_fetch_kib {sum(fprobe[:3]) / 3:.1f} (expected {PROBE_BYTES / 1024:.0f}; scale {fcal:.4f})",
        f"probe_write_kib {sum(wprobe[:3]) / 3:.1f} (expected {PROBE_BYTES / 1024:.0f}; scale {wcal:.4f})",
        f"traffic_bytes {total:.0f}",
    ]) + "\n"
    Path(out_txt).write_text(text)
    return text


def load_traffic(path) -> dict | None:
    """Parsed traffic summary, or None if missing or taken on other sources."""
    p = Path(path)
    if not p.exists():
        return None
    text = p.read_text()
    m = re.search(r"# kernel sources: ([0-9a-f]+)", text)
    if not m or m.group(1) != source_hash():
        return None
    out = {}
    for line in text.splitlines():
        if line.startswith("#"):
            continue
        k, _, v = line.partition(" ")
        out[k] = v
    return {"kernel": out.get("kernel"), "bytes": float(out["traffic_bytes"]),
            "fetch_kib": float(out["fetch_kib"]), "write_kib": float(out["write_kib"])}


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif cmd == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6]))
    else:
        raise SystemExit(__doc__)
