"""Text summary of rocprofv3 runs for one kernel: average duration from a
``--kernel-trace --stats`` run, and HBM bytes per dispatch from two ``--pmc``
runs (FETCH_SIZE, WRITE_SIZE; kilobytes per dispatch).  Each counter is
scaled by what it reads for the library's streaming copy kernel
(``k_copy_probe``, which reads and writes a known number of bytes per
dispatch) in the same run, so the reported bytes are in the units of a copy
whose traffic is known.

    python -m paper_2003_11069_amd.profile_summary --kernel k_main \\
        --trace T_results.db --fetch F_results.db --write W_results.db \\
        --copy-bytes 1073741824 --command "<command that made the runs>" \\
        --alg-bytes <algorithmic bytes per launch> --out profiles/<name>.txt

The summary records ``kernel_source_sha256`` of the lattice Boltzmann
sources; ``bench.py`` uses ``hbm_bytes_per_launch`` only while that hash
matches the sources it runs.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import statistics

_PKG = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """Hash of the lattice Boltzmann kernel code (csrc/lb_kernels.hpp) and of
    the launch-shape definitions (the #define lines of csrc/lb_internal.hpp)."""
    h = hashlib.sha256()
    csrc = os.path.join(_PKG, "csrc")
    with open(os.path.join(csrc, "lb_kernels.hpp"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "lb_internal.hpp"), "rb") as fh:
        for line in fh:
            if line.lstrip().startswith(b"#define LBNCI_") or line.lstrip().startswith(b"#define LB_"):
                h.update(line)
    return h.hexdigest()[:16]


def trace_stats(db: str):
    """[(name, calls, total_us, avg_us, percent)] from a kernel-trace run."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    c.close()
    return [(n, int(k), float(t), float(a), float(p)) for n, k, t, a, p in rows]  # microseconds


def counter_per_dispatch(db: str, counter: str):
    """{kernel name: [value per dispatch in dispatch order]} for one counter."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id order by dispatch_id", (counter,)).fetchall()
    c.close()
    out = {}
    for name, _, v in rows:
        out.setdefault(name, []).append(float(v))
    return out


def counters_table(dbs, pattern: str, copy_bytes=None):
    """Rows (kernel, grid in workgroups, dispatches, {counter: mean per
    dispatch}) of every kernel whose name contains ``pattern``, from any
    number of --pmc runs; FETCH_SIZE / WRITE_SIZE become bytes when a copy
    kernel of ``copy_bytes`` read + written per dispatch ran in the same run."""
    rows, scale = {}, {}
    for db in dbs:
        c = sqlite3.connect(db)
        q = ("select kernel_name, dispatch_id, counter_name, sum(value), grid_size_x / workgroup_size_x, "
             "grid_size_y, grid_size_z from counters_collection group by dispatch_id, counter_name")
        per = {}
        for name, did, cn, v, gx, gy, gz in c.execute(q).fetchall():
            per.setdefault((name, gx, gy, gz, cn), []).append(float(v))
        c.close()
        for (name, gx, gy, gz, cn), vals in per.items():
            if "k_copy_probe" in name and copy_bytes and cn in ("FETCH_SIZE", "WRITE_SIZE") and len(vals) > 1:
                scale[cn] = copy_bytes / (statistics.median(vals[1:]) * 1024.0)
            if pattern not in name:
                continue
            rows.setdefault((name, gx, gy, gz), {})[cn] = vals
    out = []
    for (name, gx, gy, gz), d in rows.items():
        m = {}
        for cn, vals in d.items():
            v = statistics.mean(vals)
            if cn in scale:
                v = v * 1024.0 * scale[cn]
            m[cn] = v
        n = max(len(v) for v in d.values())
        out.append((name, (gx, gy, gz), n, m))
    return out, scale


def _match(d: dict, key: str):
    names = [n for n in d if key in n]
    if not names:
        raise SystemExit(f"no kernel matching {key!r}")
    return max(names, key=lambda n: len(d[n]) if isinstance(d[n], list) else 0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", default=None)
    ap.add_argument("--write", default=None)
    ap.add_argument("--copy-bytes", type=int, default=None, help="bytes read (and written) per copy dispatch")
    ap.add_argument("--top", type=int, default=12, help="kernels listed from the trace")
    ap.add_argument("--no-hash", action="store_true", help="omit the LB source hash (other kernels)")
    ap.add_argument("--alg-bytes", type=float, default=None, help="algorithmic bytes per launch")
    ap.add_argument("--command", required=True, help="the command that produced the runs")
    ap.add_argument("--workload", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--table", nargs="*", default=None,
                    help="--pmc runs: per-kernel counter table of the kernels matching --kernel")
    a = ap.parse_args(argv)

    stats = trace_stats(a.trace)
    lines = [f"# rocprofv3 summary: {a.kernel} {a.workload}".rstrip(),
             f"command: {a.command}"]
    if not a.no_hash:
        lines.append(f"kernel_source_sha256: {kernel_source_hash()}")
    lines += ["",
              "## kernel trace (--kernel-trace --stats)",
              f"{'kernel':<70} {'calls':>6} {'avg_us':>10} {'total_us':>12} {'pct':>6}"]
    for n, k, t, av, p in stats[:a.top]:
        lines.append(f"{n[:70]:<70} {k:>6} {av:>10.3f} {t:>12.1f} {p:>6.2f}")
    if a.fetch and a.write and a.copy_bytes:
        fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE")
        write = counter_per_dispatch(a.write, "WRITE_SIZE")
        kf, kw = _match(fetch, a.kernel), _match(write, a.kernel)
        cf, cw = _match(fetch, "k_copy_probe"), _match(write, "k_copy_probe")
        # the first copy dispatch only initialises its source (write only)
        copy_fetch_kib = statistics.median(fetch[cf][1:])
        copy_write_kib = statistics.median(write[cw][1:])
        s_f = a.copy_bytes / (copy_fetch_kib * 1024.0)
        s_w = a.copy_bytes / (copy_write_kib * 1024.0)
        f_kib = statistics.mean(fetch[kf])
        w_kib = statistics.mean(write[kw])
        hbm = f_kib * 1024.0 * s_f + w_kib * 1024.0 * s_w
        lines += ["",
                  "## HBM counters (--pmc FETCH_SIZE, --pmc WRITE_SIZE; KiB per dispatch)",
                  f"copy kernel ({a.copy_bytes} B read + written per dispatch): "
                  f"FETCH_SIZE {copy_fetch_kib:.1f} KiB, WRITE_SIZE {copy_write_kib:.1f} KiB",
                  f"scale factors: fetch {s_f:.4f}, write {s_w:.4f}",
                  f"{a.kernel}: FETCH_SIZE {f_kib:.1f} KiB x {s_f:.4f} = {f_kib * 1024 * s_f:.0f} B, "
                  f"WRITE_SIZE {w_kib:.1f} KiB x {s_w:.4f} = {w_kib * 1024 * s_w:.0f} B "
                  f"({len(fetch[kf])} / {len(write[kw])} dispatches)",
                  f"hbm_bytes_per_launch: {hbm:.0f}"]
        if a.alg_bytes:
            lines.append(f"algorithmic_bytes_per_launch: {a.alg_bytes:.0f} (measured / algorithmic = "
                         f"{hbm / a.alg_bytes:.3f})")
    if a.table:
        rows, scale = counters_table(a.table, a.kernel, a.copy_bytes)
        cns = sorted({cn for _, _, _, m in rows for cn in m})
        lines += ["", f"## counters per dispatch (--pmc runs; mean over dispatches of one grid)"]
        if scale:
            lines.append("FETCH_SIZE / WRITE_SIZE in bytes, scaled by the copy kernel: " +
                         ", ".join(f"{k} x {v:.4f}" for k, v in sorted(scale.items())))
        lines.append(f"{'kernel':<44} {'grid':>14} " + " ".join(f"{cn[:22]:>22}" for cn in cns))
        for name, g, n, m in sorted(rows, key=lambda r: (r[0], r[1])):
            short = name.replace("void ", "").split("(")[0][:44]
            lines.append(f"{short:<44} {str(g):>14} " +
                         " ".join(f"{m[cn]:>22.4g}" if cn in m else f"{'-':>22}" for cn in cns))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
