"""Memory-traffic summary from two rocprofv3 --pmc runs (FETCH_SIZE, then
WRITE_SIZE) of `bench.py --kernels-only`.

The counters are read per dispatch in KiB.  They are converted to bytes with
factors taken from the plain copy kernel of the same run, whose true traffic is
known (8 bytes read and 8 written per element): bytes = counter * factor.
"""
from __future__ import annotations

import re
import sqlite3
from collections import defaultdict

import numpy as np

# the SMO-1 kernel of the fine levels (z-marching) whose traffic and duration
# the bench's roofline figure uses
SMO_KERNEL = "k_smo1_z<double>"


def _last_run(seq, key):
    """Indices of the trailing run of consecutive entries of `seq` (dispatch
    order; entries (kernel, grid, ...)) whose kernel is `key` and whose grid is
    that of the last one: the timing hook's back-to-back launches, which can
    follow the build-time schedule trials of the same kernel on other levels
    directly (other grids)."""
    idx = [i for i, (k, *_rest) in enumerate(seq) if k == key]
    if not idx:
        return []
    run = [idx[-1]]
    grid = seq[idx[-1]][1]
    while run[-1] - 1 >= 0 and seq[run[-1] - 1][0] == key and seq[run[-1] - 1][1] == grid:
        run.append(run[-1] - 1)
    return run[::-1]


def _load(path: str, counter: str):
    con = sqlite3.connect(path)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                       "from counters_collection order by dispatch_id").fetchall()
    out = []
    for did, name, grid, cname, val in rows:
        if cname != counter:
            continue
        m = re.search(r"(k_\w+)(<[^(]*>)?\(", name)
        key = (m.group(1) + (m.group(2) or "")) if m else name[:40]
        out.append((did, key, int(grid), float(val)))
    return out


def traffic_summary(fetch_db: str, write_db: str, n: int, src_hash: str) -> str:
    fe = _load(fetch_db, "FETCH_SIZE")
    wr = _load(write_db, "WRITE_SIZE")
    n3 = n ** 3

    def by_kernel(rows, key):
        """mean counter of the timing hook's launches of `key` (the last run)"""
        seq = [(k, grid, v) for _, k, grid, v in rows]
        run = _last_run(seq, key)
        if not run:
            raise ValueError(f"no dispatch of {key}")
        return float(np.mean([seq[i][2] for i in run])), len(run), seq[run[-1]][1]

    cf, ncf, _ = by_kernel(fe, "k_copy")
    cw, ncw, _ = by_kernel(wr, "k_copy")
    # SMO-1: the timing hook's launches (the tuned level-0 schedule)
    f_fac = 8.0 * n3 / (cf * 1024.0)
    w_fac = 8.0 * n3 / (cw * 1024.0)
    sf, nsf, sgrid = by_kernel(fe, SMO_KERNEL)
    sw, nsw, _ = by_kernel(wr, SMO_KERNEL)
    smo_bytes = sf * 1024.0 * f_fac + sw * 1024.0 * w_fac
    alg = 25.0 * n3
    # LU-correction sweeps: all k_lu_* dispatches, per correction (6 in the run)
    lu_f = sum(v for _, k, _, v in fe if k.startswith("k_lu_"))
    lu_w = sum(v for _, k, _, v in wr if k.startswith("k_lu_"))
    n_lu = sum(1 for _, k, _, _ in fe if k.startswith("k_lu_forward"))
    lines = [
        f"# HBM traffic of {SMO_KERNEL} (SMO-1, FP64, level 0) and the level-0 LU-correction sweeps",
        "",
        f"- grid: `{n}^3` (8-ellipsoid workload, seed 1)",
        f"- kernels.hip sha256[:16]: `{src_hash}`",
        f"- copy kernel (k_copy, {n3} doubles): FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB per dispatch "
        f"({ncf}/{ncw} dispatches); true traffic {8 * n3 / 1024:.1f} KiB each way",
        f"- calibration factors: fetch x{f_fac:.4f}, write x{w_fac:.4f}",
        f"- {SMO_KERNEL}: FETCH_SIZE {sf:.1f} KiB, WRITE_SIZE {sw:.1f} KiB per dispatch ({nsf} dispatches, "
        f"grid {sgrid} work-items)",
        f"- SMO-1 bytes per launch (calibrated): `{smo_bytes:.6e}`",
        f"- SMO-1 algorithmic bytes per launch (25 B/cell): {alg:.6e}; measured/algorithmic = {smo_bytes / alg:.3f}",
        f"- LU sweeps: {n_lu} forward launches in the run (the build-time schedule trials included); FETCH "
        f"{lu_f:.1f} KiB, WRITE {lu_w:.1f} KiB over all k_lu_* dispatches (calibrated "
        f"{(lu_f * f_fac + lu_w * w_fac) * 1024:.6e} bytes)",
    ]
    return "\n".join(lines)


def kernel_stats_summary(db: str, n: int, top: int = 14) -> str:
    """Per-kernel totals from a rocprofv3 --kernel-trace database, plus the
    average duration of the level-0 SMO-1 launches of the bench's timing hook
    (the last run of back-to-back dispatches of the kernel, after the
    build-time schedule trials), which the bench's event timing of the same
    launches should match."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, grid_x, grid_y, grid_z from kernels order by start").fetchall()
    tot = defaultdict(lambda: [0, 0.0])
    seq = []
    for name, st, en, gx, gy, gz in rows:
        m = re.search(r"(k_\w+)(<[^(]*>)?\(", name)
        key = (m.group(1) + (m.group(2) or "")) if m else name.split("(")[0][:40]
        d = (en - st) / 1000.0
        tot[key][0] += 1
        tot[key][1] += d
        seq.append((key, (gx, gy, gz), d))
    allt = sum(v[1] for v in tot.values())
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| {k} | {c} | {t / 1000:.2f} | {t / c:.1f} | {100 * t / allt:.1f} |")
    run = _last_run(seq, SMO_KERNEL)
    if run:
        v = [seq[i][2] for i in run]
        g = seq[run[-1]][1]
        out.append("")
        out.append(f"{SMO_KERNEL} level-0 dispatches of the timing hook (grid {g[0]}x{g[1]}x{g[2]} work-items, "
                   f"{n}^3 cells): {len(v)} dispatches, average {np.mean(v):.1f} us, median {np.median(v):.1f} us")
    # the level-0 LU-correction of the timing hook: the last run of consecutive
    # k_lu_* dispatches holds whole corrections of equal length; per launch
    # position (forward heights up, then backward heights down) the mean duration
    lu = [i for i, s in enumerate(seq) if s[0].startswith("k_lu_")]
    if lu:
        tail = [lu[-1]]
        while tail[-1] - 1 >= 0 and seq[tail[-1] - 1][0].startswith("k_lu_"):
            tail.append(tail[-1] - 1)
        tail = tail[::-1]
        # launches per correction: the pattern repeats; find the period
        names = [seq[i][0] for i in tail]
        per = next((p for p in range(2, len(names) // 2 + 1)
                    if len(names) % p == 0 and names == names[:p] * (len(names) // p)), len(names))
        reps = len(names) // per
        d = np.array([seq[i][2] for i in tail]).reshape(reps, per)
        # the first correction warms up
        m = d[1:].mean(axis=0) if reps > 1 else d[0]
        out.append("")
        out.append(f"Level-0 LU-correction of the timing hook ({reps} corrections of {per} launches, the first "
                   f"left out of the means): {m.sum():.1f} us per correction; launches in order (us): "
                   + ", ".join(f"{x:.1f}" for x in m))
    return "\n".join(out)


def _lu_corrections(names):
    """(indices, launches per correction, corrections) of the trailing run of
    consecutive k_lu_* entries of `names` (dispatch order), which holds whole
    corrections of the same launch pattern (the timing hook's)."""
    lu = [i for i, k in enumerate(names) if k.startswith("k_lu_")]
    if not lu:
        return [], 0, 0
    tail = [lu[-1]]
    while tail[-1] - 1 >= 0 and names[tail[-1] - 1].startswith("k_lu_"):
        tail.append(tail[-1] - 1)
    tail = tail[::-1]
    seq = [names[i] for i in tail]
    per = next((q for q in range(2, len(seq) // 2 + 1)
                if len(seq) % q == 0 and seq == seq[:q] * (len(seq) // q)), len(seq))
    return tail, per, len(seq) // per


def lu_launch_summary(fetch_db: str, write_db: str, trace_db: str, n: int) -> str:
    """Per launch of the level-0 LU-correction of the timing hook (forward
    heights up, then backward heights down): mean duration from a
    --kernel-trace database and mean HBM bytes from the FETCH_SIZE and
    WRITE_SIZE databases of the same command, calibrated by the copy kernel
    (the first correction, which warms up, left out of the means)."""
    n3 = n ** 3
    fe = _load(fetch_db, "FETCH_SIZE")
    wr = _load(write_db, "WRITE_SIZE")

    def hook_mean(rows, key):
        seq = [(k, grid, v) for _, k, grid, v in rows]
        run = _last_run(seq, key)
        if not run:
            raise ValueError(f"no dispatch of {key}")
        return float(np.mean([seq[i][2] for i in run]))

    f_fac = 8.0 * n3 / (hook_mean(fe, "k_copy") * 1024.0)
    w_fac = 8.0 * n3 / (hook_mean(wr, "k_copy") * 1024.0)

    def per_launch(names, vals):
        idx, per, reps = _lu_corrections(names)
        if not idx:
            raise ValueError("no LU-correction dispatches")
        a = np.array([vals[i] for i in idx]).reshape(reps, per)
        return (a[1:].mean(axis=0) if reps > 1 else a[0]), [names[i] for i in idx[:per]], reps

    fb, kn, reps = per_launch([k for _, k, _, _ in fe], [v * 1024.0 * f_fac for *_, v in fe])
    wb, _, _ = per_launch([k for _, k, _, _ in wr], [v * 1024.0 * w_fac for *_, v in wr])
    con = sqlite3.connect(trace_db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    tn, td = [], []
    for name, st, en in rows:
        m = re.search(r"(k_\w+)(<[^(]*>)?\(", name)
        tn.append((m.group(1) + (m.group(2) or "")) if m else name.split("(")[0][:40])
        td.append((en - st) / 1000.0)
    dur, tkn, treps = per_launch(tn, td)
    if len(dur) != len(fb) or tkn != kn:
        raise ValueError(f"the trace and the counter runs hold different LU-correction launches: "
                         f"{len(tkn)} ({tkn[:3]} ...) against {len(kn)} ({kn[:3]} ...)")
    by = fb + wb
    out = [f"| launch | kernel | us | MB | GB/s |", "|---|---|---|---|---|"]
    for i, k in enumerate(kn):
        out.append(f"| {i} | {k} | {dur[i]:.1f} | {by[i] / 1e6:.1f} | {by[i] / (dur[i] * 1e-6) / 1e9:.0f} |")
    out.append(f"| all | {len(kn)} launches ({reps} corrections in the counter runs, {treps} in the trace) | "
               f"{dur.sum():.1f} | {by.sum() / 1e6:.1f} | {by.sum() / (dur.sum() * 1e-6) / 1e9:.0f} |")
    return "\n".join(out)


def counters_summary(db: str, kernels=(SMO_KERNEL, "k_copy")) -> str:
    """Per-dispatch averages of every counter of a rocprofv3 --pmc database for
    the named kernels (the timing hook's launches: the last run of
    back-to-back dispatches of each)."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, grid_size, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    disp = {}
    for did, name, grid, cname, val in rows:
        m = re.search(r"(k_\w+)(<[^(]*>)?\(", name)
        key = (m.group(1) + (m.group(2) or "")) if m else name[:40]
        d = disp.setdefault(did, (key, int(grid), defaultdict(list)))
        d[2][cname].append(float(val))
    seq = [disp[k] for k in sorted(disp)]
    out = []
    for k in kernels:
        run = _last_run(seq, k)
        if not run:
            continue
        acc = defaultdict(list)
        for i in run:
            for c, v in seq[i][2].items():
                acc[c] += v
        out.append(f"- {k} (grid {seq[run[-1]][1]} work-items, {len(run)} dispatches): "
                   + ", ".join(f"{c} {np.mean(v):.4g}" for c, v in sorted(acc.items())))
    return "\n".join(out)
