"""Benchmark of the cut-cell multigrid solve on one MI355X.

Workload: the unit box minus 8 seeded ellipsoids (Dirichlet walls, Neumann
obstacles), 256^3 cells, manufactured phi = exp(x + y/2) cos(3z).  One step is
one whole solve (outer residual, V-cycles with SMO-1, SMO-2 LU-corrections,
transfers and the bottom solve) from a zero guess to
max|r - L phi| / max|r| < 1e-10, with r resident in HBM.

Reported: the plain FP64 solve time (`value`), the mixed-precision solve (FP32
V-cycles inside FP64 defect correction) and a batched solve of many
right-hand sides on the same geometry (time per right-hand side), the SMO-1
smoother's achieved HBM bandwidth against the MI355X peak (`roofline`, timed
with HIP events on the library's stream), and the CPU oracle timed on a
bounded sample (`cpu_baseline`).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--batch 64]
                    [--no-mixed] [--no-batch] [--no-fmg] [--no-table4] [--no-multi] [--no-cpu-baseline] [--learned]
    python bench.py --large-mixed 0         # skip the FP64 and mixed solves of the same workload at 512^3
    python bench.py --kernels-only          # only the timing hooks (for counter runs)
    python bench.py --summarize-pmc FETCH_DB WRITE_DB   # traffic table from rocprofv3 --pmc output
    python bench.py --summarize-trace TRACE_DB          # kernel table from rocprofv3 --kernel-trace output
    python bench.py --summarize-counters PMC_DB         # per-kernel counter averages from rocprofv3 --pmc output
    python bench.py --summarize-lu FETCH_DB WRITE_DB TRACE_DB   # per-launch bytes and time of the LU-correction
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
T_START = time.perf_counter()
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
KERNEL_SRC = os.path.join(ROOT, "paper_2410_05865_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_smo1_z_ellipsoid256_traffic.md")


def _src_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(n: int, work_items: int = None):
    """HBM bytes per SMO-1 launch from the committed counter summary, or None if
    it is missing, for another size, taken from a different kernel source, or
    (work_items given) from launches of another schedule (grid size)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    h = re.search(r"kernels\.hip sha256\[:16\]: `([0-9a-f]+)`", text)
    v = re.search(r"SMO-1 bytes per launch \(calibrated\): `([0-9.eE+]+)`", text)
    m = re.search(r"grid: `(\d+)\^3`", text)
    g = re.search(r"dispatches, grid (\d+) work-items", text)
    if not (h and v and m) or h.group(1) != _src_hash() or int(m.group(1)) != n:
        return None
    if work_items is not None and not (g and int(g.group(1)) == work_items):
        return None
    return float(v.group(1))


def _cpu_baseline(n_sample: int, n_target: int, N_target: int, min_seconds: float = 10.0):
    """The oracle (plain numpy/scipy, FP64) on the same workload family at a
    size it can build within the bench (n_sample^3; its set-up, minutes of
    single-threaded Python at 128^3 and hours at 256^3, is not counted): its
    own complete solves to 1e-10 from the zero guess with its own V-cycle
    count, repeated to >= min_seconds.  `value` scales the time per solve by
    unknowns to the target grid (the V-cycle count does not grow with the grid:
    the V-cycle factor is h-independent); the sample itself and the GPU's
    time on the very same n_sample^3 problem are reported beside it."""
    import torch
    from oracle.fields import Field
    from oracle.multigrid import Hierarchy, MGParams
    from paper_2410_05865_amd import _lib, inputs

    dom, phi = inputs.ellipsoid_workload(n_sample)
    F = Field(phi)
    t0 = time.perf_counter()
    H = Hierarchy(dom)
    t_setup = time.perf_counter() - t0
    lv = H.fine
    r = lv.rhs(F.laplacian_desc(), F)
    reps, t_solve, cycles = 0, 0.0, 0
    while t_solve < min_seconds or reps == 0:      # a bounded ~10 s of CPU work
        t0 = time.perf_counter()
        x, hist = H.solve(r, MGParams(tol=1e-10))
        t_solve += time.perf_counter() - t0
        cycles = len(hist) - 1
        reps += 1
    per_solve = t_solve / reps
    # the GPU on the same problem (same right-hand side, same stopping rule)
    P = _lib.Problem(dom)
    rg = torch.zeros(n_sample ** 3, dtype=torch.float64, device="cuda")
    P.assemble_rhs(phi, phi, rg, f_mode=_lib.CC_LAPLACIAN)
    xg = torch.zeros_like(rg)

    def gsolve():
        xg.zero_()
        return P.solve(rg, xg)
    g_s, g_info = _timed(gsolve, 5, 1)
    P.close()
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    return {
        "value": per_solve * N_target / lv.N,
        "unit": "s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle multigrid solves to 1e-10 on the same 8-ellipsoid workload at {n_sample}^3 "
                   f"({lv.N} unknowns, {cycles} V-cycles of its own per solve; {reps} solves, {t_solve:.1f} s; "
                   f"set-up {t_setup:.0f} s not counted), scaled by unknowns to {n_target}^3; numpy stencil work "
                   f"is single-threaded, BLAS/SuperLU may use the listed cores"),
        "sample_s_per_solve": per_solve,
        "sample_v_cycles": cycles,
        "sample_unknowns": lv.N,
        "sample_setup_s": t_setup,
        "gpu_same_sample_s_per_solve": g_s,
        "gpu_same_sample_v_cycles": g_info["iterations"],
        "cpu_over_gpu_same_sample": per_solve / g_s,
    }


def _timed(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def _table4_leg(args, sec_plain_value=None):
    """The paper's Table 4 solving-time workloads at h = 1/n: the unit cube
    minus the sphere of radius 0.3 at the centre ('Multigrid solution' 146.46 s
    at h = 1/256 on one CPU thread) and minus the torus of Problem 2 (R = 0.2,
    r = 0.1; 380.84 s at h = 1/256); tolerance unstated.  Time to 1e-10 from
    the zero guess with the paper's omega = 0.5 and with omega = 0.8, and
    FMG(2) then V-cycles; the build time of each problem beside the paper's
    two setup rows."""
    import torch
    from paper_2410_05865_amd import _lib, inputs as inp
    dev = torch.device("cuda:0")
    n3 = args.n ** 3
    paper = {"sphere": {64: (8.25, 0.70, 5.72), 128: (8.10, 5.94, 24.76), 256: (7.96, 61.57, 146.46),
                        512: (7.90, 489.50, 1385.97)},
             "torus": {64: (10.71, 0.43, 7.32), 128: (10.73, 3.21, 51.60), 256: (10.52, 30.85, 380.84),
                       512: (10.25, 273.04, 3073.53)}}
    out = {"paper_conditions": "AMD Ryzen 9 7950X, one thread, omega 0.5, nu 3/3, tolerance not stated"}
    for name in ("sphere", "torus"):
        if name == "sphere":
            dom, phi = inp.sphere03_workload(args.n)
            desc = (f"unit cube minus the sphere r = 0.3 at the centre, {args.n}^3, Dirichlet walls and sphere, "
                    f"phi = exp(x + y/2) cos(3z)")
        else:
            dom, phi = inp.torus_problem(args.n)
            desc = (f"unit cube minus the torus R = 0.2, r = 0.1 about the z axis through the centre (Problem 2), "
                    f"{args.n}^3, Dirichlet walls, Neumann torus, u = cos(pi x) cos(pi y) sin(pi z)")
        pp = paper[name].get(args.n)
        res = {"workload": desc,
               "paper_s": None if pp is None else {"setup_bottom": pp[0], "setup_lu_correction": pp[1],
                                                   "multigrid_solution": pp[2]}}
        for omega in (0.5, 0.8):
            t0 = time.perf_counter()
            P = _lib.Problem(dom, omega=omega)
            t_build = time.perf_counter() - t0
            r = torch.zeros(n3, dtype=torch.float64, device=dev)
            P.assemble_rhs(phi, phi, r, f_mode=_lib.CC_LAPLACIAN)
            x = torch.zeros_like(r)

            def solve():
                x.zero_()
                return P.solve(r, x)
            s, info = _timed(solve, args.steps, args.warmup)
            li = [P.level_info(m) for m in range(P.num_levels)]
            leg = {"s_per_solve": s, "v_cycles": info["iterations"], "final_rel_residual": info["rel_residual"],
                   "build_s": t_build, "unknowns": li[0]["n_unknowns"],
                   # the paper's two setup rows: the bottom level's LU, the other levels' L22 LUs
                   "setup_bottom_s": li[-1]["lu_seconds"],
                   "setup_lu_correction_s": sum(x["lu_seconds"] for x in li[:-1]),
                   "setup_geometry_and_rows_s": sum(x["setup_seconds"] - x["lu_seconds"] for x in li)}
            if omega == 0.8:
                coarse = []
                for m in range(1, P.num_levels):
                    rm = torch.zeros(P.n(m) ** 3, dtype=torch.float64, device=dev)
                    P.assemble_rhs(phi, phi, rm, f_mode=_lib.CC_LAPLACIAN, level=m)
                    coarse.append(rm)

                def fmg_solve():
                    x.zero_()
                    P.fmg(r, x, 2, coarse_rhs=coarse)
                    return P.solve(r, x)
                sf, info_f = _timed(fmg_solve, args.steps, args.warmup)
                leg["fmg2_then_vcycles"] = {"s_per_solve": sf, "v_cycles_after_fmg": info_f["iterations"],
                                            "final_rel_residual": info_f["rel_residual"]}
                print(f"[bench {time.perf_counter() - T_START:6.1f} s] Table 4 {name}, omega 0.8, FMG(2) then V-cycles: "
                      f"{sf * 1e3:.1f} ms, {info_f['iterations']} V-cycles", file=sys.stderr, flush=True)
            if pp is not None:
                leg["speedup_vs_paper_multigrid_solution"] = pp[2] / s
            print(f"[bench {time.perf_counter() - T_START:6.1f} s] Table 4 {name}, omega {omega}: {s * 1e3:.1f} ms, "
                  f"{info['iterations']} V-cycles (build {t_build:.1f} s: bottom LU {leg['setup_bottom_s']:.2f} s, "
                  f"L22 LUs {leg['setup_lu_correction_s']:.2f} s)", file=sys.stderr, flush=True)
            res[f"omega_{omega}"] = leg
            P.close()
        out[name] = res
    return out


def _large_mixed_leg(args):
    """The ellipsoid workload at a larger grid (512^3: 131M unknowns): FP64 and
    mixed-precision solves to 1e-10 from the zero guess, and the max-norm
    difference of the two solutions."""
    import torch
    from paper_2410_05865_amd import _lib, inputs as inp
    n = args.large_mixed
    dom, phi = inp.ellipsoid_workload(n, seed=args.seed)
    t0 = time.perf_counter()
    P = _lib.Problem(dom)
    t_setup = time.perf_counter() - t0
    r = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    P.assemble_rhs(phi, phi, r, f_mode=_lib.CC_LAPLACIAN)
    x = torch.zeros_like(r)

    def solve():
        x.zero_()
        return P.solve(r, x)
    out = {"n": n, "unknowns": P.level_info(0)["n_unknowns"], "setup_s": t_setup}
    sols = {}
    for name, prec in (("fp64", _lib.CC_FP64), ("mixed", _lib.CC_MIXED)):
        P.set_precision(prec)
        sec, info = _timed(solve, args.steps, args.warmup)
        sols[name] = x.clone()
        out[name] = {"s_per_solve": sec, "v_cycles": info["iterations"], "final_rel_residual": info["rel_residual"]}
        print(f"[bench {time.perf_counter() - T_START:6.1f} s] {n}^3 {name}: {sec * 1e3:.1f} ms, {info['iterations']} V-cycles", file=sys.stderr, flush=True)
    diff = float((sols["mixed"] - sols["fp64"]).abs().max())
    out["mixed_speedup"] = out["fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
    out["max_abs_diff_mixed_vs_fp64"] = diff
    out["max_rel_diff_mixed_vs_fp64"] = diff / float(sols["fp64"].abs().max())
    P.close()
    del sols, r, x
    torch.cuda.empty_cache()
    return out


# uneven sizes whose coarsest level (the bottom LU, factored on the host at
# set-up) stays at or below 40^3, so the leg's eight builds take seconds each
MULTI_SIZES = (64, 72, 80, 128)
MULTI_COUNT = 8


def _multi_leg(args):
    """8 geometries of the ellipsoid family of uneven sizes (64^3, 72^3, 80^3,
    128^3 in turn, two of each; seeds 2000..2007), each with a Gaussian
    right-hand side, solved with GMRES(20) one after the other and all at once
    (cc_solve_multi: one stream and host thread per problem)."""
    import torch
    from paper_2410_05865_amd import _lib, inputs
    t0 = time.perf_counter()
    probs, rs, phis, dofs = [], [], [], 0
    for i in range(MULTI_COUNT):
        n = MULTI_SIZES[i % len(MULTI_SIZES)]
        dom = inputs.ellipsoid_domain(n=n, seed=2000 + i)
        P = _lib.Problem(dom, krylov=args.krylov)
        r = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        P.assemble_rhs(inputs.gaussian_rhs(dom, seed=3000 + i), None, r)
        probs.append(P)
        rs.append(r)
        phis.append(torch.zeros_like(r))
        dofs += P.level_info(0)["n_unknowns"]
    t_setup = time.perf_counter() - t0

    def seq():
        out = []
        for P, r, x in zip(probs, rs, phis):
            x.zero_()
            out.append(P.solve(r, x))
        return out


    def conc():
        for x in phis:
            x.zero_()
        torch.cuda.synchronize()
        return _lib.solve_multi(probs, rs, phis)

    s_seq, i_seq = _timed(seq, 1, 1)
    s_con, i_con = _timed(conc, 1, 1)
    # the plain multigrid iteration on the geometries where it converges (it
    # does not on every geometry of the family; GMRES above does): one after
    # the other, on host threads and streams, and in lockstep from one host
    # thread (each problem's captured step on its own stream per iteration)
    for P in probs:
        P.set_krylov(0)
    ok = [i for i, inf in enumerate(seq()) if inf["converged"]]
    sub = ([probs[i] for i in ok], [rs[i] for i in ok], [phis[i] for i in ok])

    def seq_ok():
        out = []
        for P, r, x in zip(*sub):
            x.zero_()
            out.append(P.solve(r, x))
        return out

    def conc_ok():
        for x in sub[2]:
            x.zero_()
        torch.cuda.synchronize()
        return _lib.solve_multi(*sub)

    def graph_ok():
        for x in sub[2]:
            x.zero_()
        torch.cuda.synchronize()
        return _lib.solve_multi_graph(*sub)
    p_seq, pi_seq = _timed(seq_ok, 1, 1)
    p_con, pi_con = _timed(conc_ok, 1, 1)
    p_gr, pi_gr = _timed(graph_ok, 1, 1)
    for P in probs:
        P.set_krylov(args.krylov)
        P.close()
    plain = {"geometries": [2000 + i for i in ok], "sequential_s": p_seq, "threads_streams_s": p_con,
             "lockstep_one_thread_s": p_gr, "all_converged": all(i["converged"] for i in pi_gr),
             "v_cycles": [i["iterations"] for i in pi_gr]}
    print(f"[bench {time.perf_counter() - T_START:6.1f} s] {len(ok)} geometries, plain iteration: sequential "
          f"{p_seq * 1e3:.0f} ms, threads {p_con * 1e3:.0f} ms, lockstep {p_gr * 1e3:.0f} ms", file=sys.stderr,
          flush=True)
    print(f"[bench {time.perf_counter() - T_START:6.1f} s] {MULTI_COUNT} geometries: sequential {s_seq * 1e3:.0f} ms, "
          f"concurrent {s_con * 1e3:.0f} ms (set-up {t_setup:.0f} s)", file=sys.stderr, flush=True)
    return {"problems": f"{MULTI_COUNT} ellipsoid geometries of sizes {', '.join(f'{m}^3' for m in MULTI_SIZES)} in turn "
                        f"(seeds 2000-{2000 + MULTI_COUNT - 1}), Gaussian right-hand sides, "
                        f"GMRES({args.krylov}) with the V-cycle",
            "unknowns": dofs, "setup_s": t_setup, "sequential_s": s_seq, "concurrent_s": s_con,
            "speedup": s_seq / s_con, "all_converged": all(i["converged"] for i in i_con),
            "v_cycles": [i["iterations"] for i in i_con], "plain_iteration": plain}


def _learned_leg(P, dom, phi, r_plain, coarse, args, stream):
    """The learned initial iterate: a depth-4, 32-channel U-Net (BF16 MFMA)
    trained on solver-generated pairs from 128^3 problems of the family (the
    network on their 64^3 level), then the benchmark problem solved for
    held-out Gaussian right-hand sides from the zero guess, from the full
    multigrid ascent that starts at the 64^3 level from the network's
    prediction there (cc_learned_fmg, 2 V-cycles per level), and after FMG(2)
    from the exact coarsest solve."""
    import torch
    from paper_2410_05865_amd import _lib, inputs, learned
    log = lambda s_: print(s_, file=sys.stderr, flush=True)
    net, info = learned.fit(n_fine=128, level=1, geometries=args.learned_geometries,
                            rhs_per_geometry=args.learned_rhs, steps=args.learned_steps, base_channels=32, depth=4,
                            seed=3, log=log, max_attempts=2 * args.learned_geometries + 4)
    level = next(m for m in range(P.num_levels) if P.n(m) == 64)
    n3 = args.n ** 3
    out = {"train": info, "rhs": "f = sum of 16 seeded Gaussians (seeds 9000 ..), g = 0", "held_out": []}
    with torch.cuda.stream(stream):
        fields = [inputs.gaussian_rhs(dom, seed=9000 + k) for k in range(args.learned_eval)]
        rb = torch.zeros(len(fields), n3, dtype=torch.float64, device="cuda")
        P.assemble_rhs_batched(fields, None, rb)
        cb = []
        for m in range(1, P.num_levels):
            bm = torch.zeros(len(fields), P.n(m) ** 3, dtype=torch.float64, device="cuda")
            P.assemble_rhs_batched(fields, None, bm, level=m)
            cb.append(bm)
        phi_ = torch.zeros(n3, dtype=torch.float64, device="cuda")
        for k in range(len(fields)):
            r = rb[k].contiguous()
            crs = [c[k].contiguous() for c in cb]

            def zero_guess():
                phi_.zero_()
                return P.solve(r, phi_)

            def learned_start():
                P.learned_fmg(net, level, learned.PHI_SCALE, r, phi_, cycles=2, coarse_rhs=crs)
                return P.solve(r, phi_)

            def fmg2():
                phi_.zero_()
                P.fmg(r, phi_, 2, coarse_rhs=crs)
                return P.solve(r, phi_)
            s0, i0 = _timed(zero_guess, 1, 1)
            s1, i1 = _timed(learned_start, 1, 1)
            s2, i2 = _timed(fmg2, 1, 1)
            out["held_out"].append({"zero_guess": {"s": s0, "v_cycles": i0["iterations"]},
                                    "learned_fmg_start": {"s_incl_inference": s1, "v_cycles": i1["iterations"],
                                                          "initial_rel_residual": i1["history"][0]},
                                    "fmg2": {"s": s2, "v_cycles_after_fmg": i2["iterations"]}})
    net.close()
    ho = out["held_out"]
    t0 = float(np.mean([h["zero_guess"]["s"] for h in ho]))
    t1 = float(np.mean([h["learned_fmg_start"]["s_incl_inference"] for h in ho]))
    t2 = float(np.mean([h["fmg2"]["s"] for h in ho]))
    out["mean_v_cycles"] = {"zero_guess": float(np.mean([h["zero_guess"]["v_cycles"] for h in ho])),
                            "learned_fmg_start": float(np.mean([h["learned_fmg_start"]["v_cycles"] for h in ho])),
                            "fmg2_then": float(np.mean([h["fmg2"]["v_cycles_after_fmg"] for h in ho]))}
    out["speedup_vs_zero_guess"] = t0 / t1
    out["speedup_vs_fmg2"] = t2 / t1
    log(f"[bench {time.perf_counter() - T_START:6.1f} s] learned FMG start: V-cycles {out['mean_v_cycles']}, "
        f"{t0 * 1e3:.1f} / {t1 * 1e3:.1f} / {t2 * 1e3:.1f} ms (zero / learned start / FMG(2))")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--learned", action="store_true",
                    help="also train the learned initial guess and compare it (several minutes; off by default)")
    ap.add_argument("--no-krylov", action="store_true")
    ap.add_argument("--no-fmg", action="store_true")
    ap.add_argument("--no-table4", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--large-mixed", type=int, default=512, metavar="N",
                    help="also solve the ellipsoid workload at N^3 in FP64 and mixed precision (0: skip)")
    ap.add_argument("--krylov", type=int, default=20)
    ap.add_argument("--learned-steps", type=int, default=2000)
    ap.add_argument("--learned-geometries", type=int, default=16,
                    help="128^3 geometries the training pairs come from (drawn until this many converge)")
    ap.add_argument("--learned-rhs", type=int, default=125, help="right-hand sides per training geometry")
    ap.add_argument("--learned-eval", type=int, default=10, help="held-out right-hand sides at the benchmark size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=64)
    ap.add_argument("--smoother-reps", type=int, default=50)
    ap.add_argument("--kernels-only", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DB")
    ap.add_argument("--summarize-counters", metavar="PMC_DB")
    ap.add_argument("--summarize-lu", nargs=3, metavar=("FETCH_DB", "WRITE_DB", "TRACE_DB"),
                    help="per-launch bytes and durations of the level-0 LU-correction of the timing hook")
    args = ap.parse_args()
    if args.summarize_lu:
        from paper_2410_05865_amd import profiling
        print(profiling.lu_launch_summary(*args.summarize_lu, n=args.n))
        return
    if args.summarize_counters:
        from paper_2410_05865_amd import profiling
        print(profiling.counters_summary(args.summarize_counters))
        return
    if args.summarize_pmc or args.summarize_trace:
        from paper_2410_05865_amd import profiling
        if args.summarize_pmc:
            print(profiling.traffic_summary(*args.summarize_pmc, n=args.n, src_hash=_src_hash()))
        if args.summarize_trace:
            print(profiling.kernel_stats_summary(args.summarize_trace, n=args.n))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)

    import torch
    from paper_2410_05865_amd import _lib, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    _lib.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    dom, phi = inputs.ellipsoid_workload(args.n, seed=args.seed)
    t0 = time.perf_counter()
    P = _lib.Problem(dom, stream=stream.cuda_stream)
    t_setup = time.perf_counter() - t0
    li0 = P.level_info(0)
    n3 = args.n ** 3

    with torch.cuda.stream(stream):
        if args.kernels_only:
            # the level-0 LU schedule the build usually keeps (8 entries per lane,
            # per-height launches, no cap), fixed so that separate profiler runs of
            # this mode launch the same LU kernels
            P.set_lu_schedule(0, 8, 0, 0)
            for which in (_lib.CC_TIME_SMO1, _lib.CC_TIME_COPY, _lib.CC_TIME_LU):
                P.time_kernel(which, 5)
            torch.cuda.synchronize()
            print(json.dumps({"kernels_only": True, "n": args.n}), flush=True)
            return
        r = torch.zeros(n3, dtype=torch.float64, device=dev)
        x = torch.zeros(n3, dtype=torch.float64, device=dev)
        P.assemble_rhs(phi, phi, r, f_mode=_lib.CC_LAPLACIAN)

        def solve_once():
            x.zero_()
            return P.solve(r, x)

        sec, info = _timed(solve_once, args.steps, args.warmup)
        print(f"[bench {time.perf_counter() - T_START:6.1f} s] plain FP64: {sec * 1e3:.1f} ms, {info['iterations']} V-cycles", file=sys.stderr, flush=True)
        x64 = x.clone()          # the FP64 solution every other leg of this workload is compared with

        def vs_fp64(y):
            d = float((y - x64).abs().max())
            return {"max_abs_diff_vs_fp64": d, "max_rel_diff_vs_fp64": d / float(x64.abs().max())}
        out_mixed = None
        if not args.no_mixed:
            P.set_precision(_lib.CC_MIXED)
            sec_m, info_m = _timed(solve_once, args.steps, args.warmup)
            P.set_precision(_lib.CC_FP64)
            print(f"[bench {time.perf_counter() - T_START:6.1f} s] mixed: {sec_m * 1e3:.1f} ms, {info_m['iterations']} V-cycles", file=sys.stderr, flush=True)
            out_mixed = {"s_per_solve": sec_m, "v_cycles": info_m["iterations"],
                         "final_rel_residual": info_m["rel_residual"], "speedup_vs_plain": sec / sec_m,
                         **vs_fp64(x)}
        out_krylov = None
        if not args.no_krylov:
            P.set_krylov(args.krylov)
            sec_k, info_k = _timed(solve_once, args.steps, args.warmup)
            P.set_krylov(0)
            print(f"[bench {time.perf_counter() - T_START:6.1f} s] GMRES({args.krylov}): {sec_k * 1e3:.1f} ms, {info_k['iterations']} V-cycles", file=sys.stderr,
                  flush=True)
            out_krylov = {"restart": args.krylov, "s_per_solve": sec_k, "v_cycles": info_k["iterations"],
                          "final_rel_residual": info_k["rel_residual"], "speedup_vs_plain": sec / sec_k}
            if not args.no_mixed:
                P.set_krylov(args.krylov)
                P.set_precision(_lib.CC_MIXED)
                sec_km, info_km = _timed(solve_once, args.steps, args.warmup)
                P.set_precision(_lib.CC_FP64)
                P.set_krylov(0)
                print(f"[bench {time.perf_counter() - T_START:6.1f} s] GMRES({args.krylov}) + FP32 V-cycle: {sec_km * 1e3:.1f} ms, "
                      f"{info_km['iterations']} V-cycles", file=sys.stderr, flush=True)
                out_krylov["mixed_preconditioner"] = {
                    "s_per_solve": sec_km, "v_cycles": info_km["iterations"],
                    "final_rel_residual": info_km["rel_residual"], "speedup_vs_plain": sec / sec_km,
                    **vs_fp64(x)}
        out_fmg = None
        if not args.no_fmg:
            # full multigrid first (FP64, c V-cycles per level), then the solve from its result
            # each coarser level's right-hand side: the same problem assembled there
            # (input data like r, not timed)
            coarse = []
            for m in range(1, P.num_levels):
                rm = torch.zeros(P.n(m) ** 3, dtype=torch.float64, device=dev)
                P.assemble_rhs(phi, phi, rm, f_mode=_lib.CC_LAPLACIAN, level=m)
                coarse.append(rm)
            legs = {}
            for cyc in (1, 2, 3):
                def fmg_solve(c=cyc):
                    x.zero_()
                    P.fmg(r, x, c, coarse_rhs=coarse)
                    return P.solve(r, x)
                sec_f, info_f = _timed(fmg_solve, args.steps, args.warmup)
                print(f"[bench {time.perf_counter() - T_START:6.1f} s] FMG({cyc}) + plain FP64: {sec_f * 1e3:.1f} ms, {info_f['iterations']} V-cycles after "
                      f"FMG", file=sys.stderr, flush=True)
                legs[str(cyc)] = {"s_per_solve": sec_f, "v_cycles_after_fmg": info_f["iterations"],
                                  "final_rel_residual": info_f["rel_residual"], "speedup_vs_plain": sec / sec_f}
            best = min(legs, key=lambda k: legs[k]["s_per_solve"])
            out_fmg = {"cycles_per_level": legs, "best_cycles": int(best)}
            if not args.no_krylov and not args.no_mixed:
                P.set_krylov(args.krylov)
                P.set_precision(_lib.CC_MIXED)

                def fmg_gmres():
                    x.zero_()
                    P.fmg(r, x, int(best), coarse_rhs=coarse)
                    return P.solve(r, x)
                sec_fg, info_fg = _timed(fmg_gmres, args.steps, args.warmup)
                P.set_precision(_lib.CC_FP64)
                P.set_krylov(0)
                print(f"[bench {time.perf_counter() - T_START:6.1f} s] FMG({best}) + GMRES({args.krylov}) with the FP32 V-cycle: {sec_fg * 1e3:.1f} ms, "
                      f"{info_fg['iterations']} V-cycles after FMG", file=sys.stderr, flush=True)
                out_fmg["then_gmres_fp32_vcycle"] = {"s_per_solve": sec_fg, "v_cycles_after_fmg": info_fg["iterations"],
                                                     "final_rel_residual": info_fg["rel_residual"],
                                                     "speedup_vs_plain": sec / sec_fg, **vs_fp64(x)}
        out_batch = None
        if not args.no_batch and args.batch > 0:
            B = args.batch
            # B independent right-hand sides, f_k = sum of 16 seeded Gaussians
            # (seeds 0 .. B-1), zero boundary data; assembled in one call per level
            # (input data like r, not timed)
            fields = [inputs.gaussian_rhs(dom, seed=k) for k in range(B)]
            t_as = time.perf_counter()
            rb = torch.zeros(B, n3, dtype=torch.float64, device=dev)
            P.assemble_rhs_batched(fields, None, rb)
            t_as = time.perf_counter() - t_as
            print(f"[bench {time.perf_counter() - T_START:6.1f} s] {B} right-hand sides assembled in {t_as:.1f} s", file=sys.stderr, flush=True)
            # each coarser level's right-hand sides of the same problems, for FMG
            coarse_b = []
            if not args.no_fmg:
                for m in range(1, P.num_levels):
                    bm = torch.zeros(B, P.n(m) ** 3, dtype=torch.float64, device=dev)
                    P.assemble_rhs_batched(fields, None, bm, level=m)
                    coarse_b.append(bm)
            xb = torch.zeros_like(rb)
            res = {}
            xb64 = None
            for prec, name in ((_lib.CC_FP64, "fp64"), (_lib.CC_MIXED, "mixed")):
                if name == "mixed" and args.no_mixed:
                    continue
                P.set_precision(prec)

                def solve_batch():
                    xb.zero_()
                    return P.solve_batched(rb, xb)

                sb, infos = _timed(solve_batch, 1, 1)
                res[name] = {"s_per_rhs": sb / B, "s_per_batch": sb,
                             "v_cycles": max(i["iterations"] for i in infos),
                             "max_final_rel_residual": max(i["rel_residual"] for i in infos),
                             "speedup_per_rhs_vs_plain": sec / (sb / B)}
                if name == "fp64":
                    xb64 = xb.clone()
                else:   # every member against its FP64 solution (max over members of the relative max-norm)
                    dm = (xb - xb64).abs().amax(dim=1) / xb64.abs().amax(dim=1)
                    res[name]["max_rel_diff_vs_fp64"] = float(dm.max())
                print(f"[bench {time.perf_counter() - T_START:6.1f} s] batched {name}: {sb * 1e3:.0f} ms for {B} rhs", file=sys.stderr, flush=True)
                if coarse_b:
                    def fmg_batch():
                        xb.zero_()
                        P.fmg_batched(rb, xb, 2, coarse_rhs=coarse_b)
                        return P.solve_batched(rb, xb)

                    sf, infos_f = _timed(fmg_batch, 1, 1)
                    res[name]["fmg2_then_batched"] = {
                        "s_per_rhs": sf / B, "s_per_batch": sf,
                        "v_cycles_after_fmg": max(i["iterations"] for i in infos_f),
                        "max_final_rel_residual": max(i["rel_residual"] for i in infos_f),
                        "speedup_per_rhs_vs_plain": sec / (sf / B)}
                    print(f"[bench {time.perf_counter() - T_START:6.1f} s] batched {name} after FMG(2): {sf * 1e3:.0f} ms for {B} rhs, "
                          f"{max(i['iterations'] for i in infos_f)} V-cycles", file=sys.stderr, flush=True)
            P.set_precision(_lib.CC_FP64)
            out_batch = {"rhs": B, "rhs_recipe": f"{B} independent right-hand sides, f_k = sum of 16 seeded "
                                                  f"Gaussians (seed k, sigma U[0.02, 0.1], centres outside the "
                                                  f"obstacles), g = 0", "assembly_s": t_as, **res}
            del rb, xb, xb64, coarse_b
            torch.cuda.empty_cache()
        # the timing hooks right after the legs of this problem (before the
        # other problems' legs), the state the kernel-trace run profiles
        ms_smo, by_smo = P.time_kernel(_lib.CC_TIME_SMO1, args.smoother_reps)
        # the hook's launch grid: n^3 / planes work-items for the z-marching
        # kernels, n^3 for one cell per thread
        march0, kz0 = P.stencil_schedule(0)
        smo_work_items = n3 // kz0 if march0 else n3
        ms_smo32, by_smo32 = P.time_kernel(_lib.CC_TIME_SMO1_F32, args.smoother_reps)
        ms_lu, by_lu = P.time_kernel(_lib.CC_TIME_LU, 10)
        ms_copy, by_copy = P.time_kernel(_lib.CC_TIME_COPY, args.smoother_reps)
        torch.cuda.synchronize()
        out_multi = None
        if not args.no_multi:
            out_multi = _multi_leg(args)
        out_t4 = None
        if not args.no_table4:
            out_t4 = _table4_leg(args)
        out_large = None
        if args.large_mixed:
            out_large = _large_mixed_leg(args)
        out_learned = None
        if args.learned:
            out_learned = _learned_leg(P, dom, phi, None, None, args, stream)

    N = li0["n_unknowns"]
    n_phi1 = N - li0["n_phi2"]
    # algorithmic bytes of one SMO-1 sweep: read e and r, write e' for every phi_1 cell
    # (24 B per phi_1 cell); the kernel also passes the other cells through and
    # reads the cell type: 25 B per cell of the n^3 grid (by_smo)
    alg_smo = 24.0 * n_phi1
    achieved = alg_smo / (ms_smo * 1e-3) / 1e9
    cycles = info["iterations"]
    out = {
        "metric": "time to 1e-10 rel. residual at 256^3 (plain vs mixed/learned) + smoother HBM GB/s",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"unit box minus 8 seeded ellipsoids (seed {args.seed}), Dirichlet walls, Neumann "
                        f"obstacles, manufactured phi = exp(x + y/2) cos(3z), {args.n}^3, plain FP64 V-cycles "
                        f"to 1e-10 max-norm relative residual",
            "n": args.n, "levels": P.num_levels, "unknowns": N, "phi2_rows": li0["n_phi2"],
            "lu_entries_level0": li0["lu_entries"],
            "omega": P.params.omega, "nu1": P.params.nu1, "nu2": P.params.nu2,
        },
        "v_cycles": cycles,
        "final_rel_residual": info["rel_residual"],
        "dof_per_s": N * cycles / sec,
        "setup_s": t_setup,
        "lu_schedule": [
            {"level": m, "n": li["n"], "entries_per_lane": li["lu_entries_per_lane"],
             "subtrees": li["lu_subtrees"], "subtree_cut": li["lu_subtree_cut"], "waves_cap": li["lu_waves_cap"],
             "trial_ms": [round(v, 4) for v in li["lu_tune_ms"]]}
            for m, li in ((m, P.level_info(m)) for m in range(P.num_levels))],
        "stencil_schedule": [
            {"level": m, "n": li["n"], "march": li["stencil_march"], "planes": li["stencil_planes"],
             "trial_us": [round(v, 1) for v in li["stencil_tune_us"]]}
            for m, li in ((m, P.level_info(m)) for m in range(P.num_levels))],
        "mixed": out_mixed,
        "krylov": out_krylov,
        "fmg": out_fmg,
        "batched": out_batch,
        "learned": out_learned,
        "multi_geometry": out_multi,
        "paper_table4": out_t4,
        "mixed_large": out_large,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_smo1_z<double> (SMO-1 weighted Jacobi, level 0)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic(args.n, smo_work_items),
            "ms_per_launch": ms_smo,
            "bytes_per_launch": alg_smo,
            "bytes_per_launch_basis": f"24 B per phi_1 cell x {n_phi1} phi_1 cells (read e, r; write e')",
            "kernel_bytes_all_cells": by_smo,
            "kernel_achieved_all_cells_GBs": by_smo / (ms_smo * 1e-3) / 1e9,
        },
        "roofline_other": {
            "k_smo1_z<float>": {"achieved_GBs": by_smo32 / (ms_smo32 * 1e-3) / 1e9, "ms_per_launch": ms_smo32,
                              "bytes_per_launch": by_smo32},
            "lu_correction_level0_fp64": {"achieved_GBs": by_lu / (ms_lu * 1e-3) / 1e9, "ms_per_correction": ms_lu,
                                          "bytes_per_correction": by_lu},
            "copy": {"achieved_GBs": by_copy / (ms_copy * 1e-3) / 1e9, "ms_per_launch": ms_copy,
                     "bytes_per_launch": by_copy},
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(args.cpu_sample_n, args.n, N)
    P.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
