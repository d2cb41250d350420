"""Helpers for profiling the solver with rocprofv3.

    python -m paper_1805_06688_amd.profiling copy [MiB]
        a plain device-to-device copy of a known size (HBM-counter calibration)
    python -m paper_1805_06688_amd.profiling stats KERNEL_STATS_CSV
        markdown table of a rocprofv3 --stats kernel summary
    python -m paper_1805_06688_amd.profiling counters COUNTER_CSV REGEX
        mean value per dispatch of every counter for kernels matching REGEX
    python -m paper_1805_06688_amd.profiling source-hash
        hash of the HIP kernel sources (counters are tied to one version)
    python -m paper_1805_06688_amd.profiling traffic FETCH_CSV WRITE_CSV CLASS REGEX [REGEX2 ...] [--ff FF --wf WF]
            [--launches-of REGEX]
        HBM bytes per launch of one kernel class of the library's instrumentation (a launch of the FFT operator
        is one dispatch of each of its two passes, REGEX and REGEX2) from a FETCH_SIZE and a WRITE_SIZE run,
        each counter scaled by its copy-kernel factor (FF, WF; default 2, 1); with --launches-of the launches
        are counted by that regex's dispatches (the preconditioner runs one product kernel twice)
"""
import json
import csv
import hashlib
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_hash():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def copy(mib=512, reps=8):
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}: {mib * 1024} KiB read and {mib * 1024} KiB written per dispatch")


def _demangle_template(name):
    """Name and template arguments of a mangled kernel (bool, int, float and double arguments only)."""
    m = re.match(r"_ZN12_GLOBAL__N_1(\d+)", name)
    if not m:
        return name
    n = int(m.group(1))
    rest = name[m.end():]
    ident, rest = rest[:n], rest[n:]
    if not rest.startswith("I"):
        return ident
    args, i = [], 1
    while i < len(rest) and rest[i] != "E":
        a = re.match(r"L([bi])(n?\d+)E", rest[i:])
        if a:
            v = a.group(2).replace("n", "-")
            args.append(("true" if v == "1" else "false") if a.group(1) == "b" else v)
            i += a.end()
        elif rest[i] in "fd":
            args.append("float" if rest[i] == "f" else "double")
            i += 1
        else:
            return ident
    return ident + "<" + ", ".join(args) + ">"


def short_name(name):
    if name.startswith("_Z"):
        name = _demangle_template(name)
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def stats(path):
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        if t < 1e-3 * total:
            continue
        print(f"| `{short_name(r['Name'])}` | {r['Calls']} | {t / 1e6:.1f} | {float(r['AverageNs']) / 1e3:.1f} "
              f"| {100 * t / total:.1f} |")


def counters(path, regex):
    pat = re.compile(regex)
    acc = {}
    for r in csv.DictReader(open(path)):
        if not pat.search(r.get("Kernel_Name", "")):
            continue
        key = (short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"), r["Counter_Name"])
        v = acc.setdefault(key, [0, 0.0])
        v[0] += 1
        v[1] += float(r["Counter_Value"])
    for (k, g, c), (n, tot) in sorted(acc.items()):
        print(f"{k} grid={g} {c}: dispatches={n} mean={tot / n:.1f}")


def _kib(path, regex, counter):
    pat = re.compile(regex)
    tot, n = 0.0, 0
    for r in csv.DictReader(open(path)):
        if pat.search(r.get("Kernel_Name", "")) and r["Counter_Name"] == counter:
            tot += float(r["Counter_Value"])
            n += 1
    return tot, n


def traffic(fetch_csv, write_csv, cls, regexes, ff=2.0, wf=1.0, launches_of=None):
    """Bytes per launch of a kernel class.  A launch is one dispatch of each REGEX, or with launches_of
    (for a class whose launch runs one kernel more than once) the number of launches is the dispatch count
    of that regex and the REGEXes' dispatches are summed."""
    fetch, write, counts = [], [], []
    for rx in regexes:
        f, n = _kib(fetch_csv, rx, "FETCH_SIZE")
        w, m = _kib(write_csv, rx, "WRITE_SIZE")
        fetch.append(f)
        write.append(w)
        counts += [n, m]
    if launches_of:
        _, n = _kib(fetch_csv, launches_of, "FETCH_SIZE")
        _, m = _kib(write_csv, launches_of, "WRITE_SIZE")
        counts = [n, m]
    if not counts[0] or len(set(counts)) != 1:
        raise SystemExit(f"dispatch counts differ or are zero: {counts}")
    n = counts[0]
    per = (ff * sum(fetch) + wf * sum(write)) * 1024.0 / n
    out = {"class": int(cls), "kernels": list(regexes), "source_hash": source_hash(),
           "counter_factors": {"FETCH_SIZE": ff, "WRITE_SIZE": wf}, "launches": n,
           "fetch_kib_per_launch": [f / n for f in fetch], "write_kib_per_launch": [w / n for w in write],
           "bytes_per_launch": per}
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else ""
    if cmd == "copy":
        copy(int(sys.argv[2]) if len(sys.argv) > 2 else 512)
    elif cmd == "stats":
        stats(sys.argv[2])
    elif cmd == "counters":
        counters(sys.argv[2], sys.argv[3])
    elif cmd == "source-hash":
        print(source_hash())
    elif cmd == "traffic":
        import argparse
        ap = argparse.ArgumentParser()
        ap.add_argument("fetch_csv")
        ap.add_argument("write_csv")
        ap.add_argument("cls", type=int)
        ap.add_argument("regex", nargs="+")
        ap.add_argument("--ff", type=float, default=2.0)
        ap.add_argument("--wf", type=float, default=1.0)
        ap.add_argument("--launches-of", default=None)
        a = ap.parse_args(sys.argv[2:])
        traffic(a.fetch_csv, a.write_csv, a.cls, a.regex, a.ff, a.wf, a.launches_of)
    else:
        print(__doc__)
        sys.exit(2)
