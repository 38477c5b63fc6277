"""Per-launch HBM bytes of the propagator kernels from two rocprofv3 counter
runs (FETCH_SIZE, then WRITE_SIZE) of ``bench.py --copy-probe-mib 512``.

Both counters read KiB leaving L2 per dispatch.  Each is scaled by what it
reads for the library's plain copy kernel (``k_copy_probe``) moving a known
512 MiB, then the mean over the dispatches of each kernel is written, with
the hash of that kernel's sources, to ``profiles/lam128_hbm_traffic.txt``,
the file ``bench.py`` reads for ``roofline.traffic``.

Usage: python -m paper_1204_5434_amd.traffic_summary COUNTER_RUN_DIR
(the directory holding the two runs' ``pmc_FETCH_SIZE/`` and ``pmc_WRITE_SIZE/``
output).  Prints the table rows of every kernel as well.
"""
import collections
import csv
import os
import statistics
import sys

from . import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_KIB = 512 * 1024


def _load(path):
    rows = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return rows


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def _kind(short: str):
    if "k_zpass<" in short:
        return "zpass"
    if "k_yzpass<" in short:
        return "yzpass"
    if "k_spass<" in short:
        # template arguments <T, N1, N2, Y, ...>: Y = 1 is the y pass
        return "ypass" if short.rstrip(">").split(",")[3].strip() == "1" else "xpass"
    if "k_density<" in short:
        return "density"
    return None


def summarize(base: str):
    F = _load(os.path.join(base, "pmc_FETCH_SIZE", "lam128_counter_collection.csv"))
    W = _load(os.path.join(base, "pmc_WRITE_SIZE", "lam128_counter_collection.csv"))
    probe = [k for k in F if "k_copy_probe" in k][0]
    fs = COPY_KIB / statistics.median(F[probe])
    ws = COPY_KIB / statistics.median(W[probe])
    txt = ["# HBM bytes per launch (FETCH_SIZE x %.4f + WRITE_SIZE x %.4f, KiB -> bytes), lam128" % (fs, ws),
           "# kind:precision bytes kernel source-hash-of-that-kernel"]
    rows, seen = [], set()
    for k in sorted(F, key=lambda k: -len(F[k])):  # most-dispatched first: tuner probes come later
        s = _short(k)
        kind = _kind(s) if s.startswith("pft::k_") else None
        if kind is None:
            continue
        f = statistics.mean(F[k]) * fs * 1024
        w = statistics.mean(W.get(k, [0.0])) * ws * 1024
        prec = "f64" if "double" in s else "f32"
        rows.append((s, len(F[k]), f / 2 ** 20, w / 2 ** 20))
        if (kind, prec) in seen:
            continue
        seen.add((kind, prec))
        txt.append(f"{kind}:{prec} {f + w:.0f} {s.replace(' ', '')} {build.kernel_hash(kind)}")
    return txt, rows


def main(argv):
    if len(argv) != 2:
        raise SystemExit("usage: python -m paper_1204_5434_amd.traffic_summary COUNTER_RUN_DIR")
    txt, rows = summarize(argv[1])
    with open(os.path.join(ROOT, "profiles", "lam128_hbm_traffic.txt"), "w") as fh:
        fh.write("\n".join(txt) + "\n")
    print("\n".join(txt))
    print("| Kernel | Dispatches | Read (MiB) | Write (MiB) |")
    for s, n, r, w in rows:
        print(f"| `{s}` | {n} | {r:.1f} | {w:.1f} |")


if __name__ == "__main__":
    main(sys.argv)
