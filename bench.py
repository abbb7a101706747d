#!/usr/bin/env python3
"""Benchmark: outer iterations/sec of the adaptively conditioned conic solver
on the 2M-variable sparse LP (m = 500k, n = 2M, 10M nonzeros, power-law row
degrees, row scales 10^U(-3,3)), FP32 iterate and SpMVs with FP64
reductions, on one MI355X.

A step is one outer iteration of Algorithm 2 (cone reflection, residual,
warm-started CG projection, fused update; conditioning at l in L, a KKT check
every `check_every` iterations).  Inputs are resident in HBM before timing.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the solver runs on
one GPU.
"""
import argparse
import hashlib
import threading
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6  # MI355X dense FP64 (vector and MFMA)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the LP (tests only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--workload", choices=["lp2m", "batch", "serve", "copy", "gather", "dense", "dense_solve",
                                           "ablation"],
                    default="lp2m",
                    help="lp2m: iterations/s on the 2M-variable LP (default); batch: 4096 small LPs in one "
                         "persistent launch; serve: Poisson request stream through the serving loop")
    ap.add_argument("--count", type=int, default=4096, help="batch: number of instances")
    ap.add_argument("--dense-n", type=int, default=30000, help="dense: n of the paper's random LP (m = 0.8 n)")
    ap.add_argument("--projection", choices=["cg", "factor"], default="cg",
                    help="dense: projection by warm-started CG or by the inverse of A_s A_s^T (formed at events)")
    ap.add_argument("--skip-cg-compare", action="store_true",
                    help="dense --projection factor: do not also time the CG projection over the same window")
    ap.add_argument("--requests", type=int, default=200, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrival rate (requests/s)")
    ap.add_argument("--workers", type=int, default=6, help="serve: worker streams of the server")
    ap.add_argument("--small-nnz", type=int, default=20_000, help="serve: largest request of the slot pool")
    ap.add_argument("--headline-only", action="store_true",
                    help="lp2m: only the timed window (no whole solves, SOCP, batch or serving sections)")
    ap.add_argument("--serve-requests", type=int, default=160,
                    help="lp2m: requests of the serving section (the first tenth is warm-up)")
    ap.add_argument("--state-file", default="", help=argparse.SUPPRESS)
    return ap.parse_args()


# ----------------------------------------------------------------------------
# CPU baseline: the oracle on the same instance, in a child process started
# before this process touches the GPU.
# ----------------------------------------------------------------------------
def cpu_child(args):
    from oracle.alg2 import Algorithm2, default_parameters
    from paper_2103_00736_amd import synth

    if args.workload == "batch":  # whole solves of a seeded subset, one at a time
        idx = np.random.default_rng(1).choice(args.count, size=6, replace=False)
        t0 = time.perf_counter()
        for i in idx:
            q = synth.config3(int(i))
            t, L = default_parameters(q.soc_sizes)
            Algorithm2(q.scipy_csr(), q.b, q.c, q.n_orth, q.soc_sizes, mu=1.0, t=t, schedule=L).run(
                20000, eps=1e-4, check_every=10, obj_stop=1.0)
        dt = time.perf_counter() - t0
        print(json.dumps({"iters": len(idx), "seconds": dt, "pcg_iters": 0, "what": "solves"}), flush=True)
        return
    if args.workload == "dense":  # the same recipe at n = 3000 (the full size takes minutes per iteration)
        q = synth.e3_lp(3000)
        t, L = default_parameters(q.soc_sizes)
        t0 = time.perf_counter()
        alg = Algorithm2(q.scipy_csr(), q.b, q.c, q.n_orth, q.soc_sizes, mu=1.0, t=t, schedule=L)
        for _ in range(10):
            alg.step()
        dt = time.perf_counter() - t0
        print(json.dumps({"iters": 10, "seconds": dt, "pcg_iters": 0, "what": "dense"}), flush=True)
        return
    # the 2M-variable LP: first whole solves of a seeded subset of the batch
    # recipe (while the GPU process warms up), then the timed iterations of
    # the oracle from the GPU's state after its warmup
    out = {}
    if not args.headline_only:
        q = synth.config0()
        t, L = default_parameters(q.soc_sizes)
        t0 = time.perf_counter()
        rec = Algorithm2(q.scipy_csr(), q.b, q.c, q.n_orth, q.soc_sizes, mu=1.0, t=t, schedule=L).run(
            20000, eps=1e-6, check_every=10, obj_stop=1.0)
        out["lp200"] = {"iters": int(rec["iters"]), "seconds": time.perf_counter() - t0, "kkt": rec["kkt"]}
        idx = np.random.default_rng(1).choice(4096, size=6, replace=False)
        t0 = time.perf_counter()
        for i in idx:
            q = synth.config3(int(i))
            t, L = default_parameters(q.soc_sizes)
            Algorithm2(q.scipy_csr(), q.b, q.c, q.n_orth, q.soc_sizes, mu=1.0, t=t, schedule=L).run(
                20000, eps=1e-4, check_every=10, obj_stop=1.0)
        out["batch"] = {"solves": len(idx), "seconds": time.perf_counter() - t0}
        # the serving trace: service times of its four smallest requests (the
        # oracle takes minutes on the larger ones)
        trace = synth.config4_trace(args.serve_requests, rate_per_s=200.0)
        small = sorted(trace, key=lambda r: r.m)[:4]
        times = []
        for r in small:
            q = r.problem()
            t, L = default_parameters(q.soc_sizes)
            t0 = time.perf_counter()
            Algorithm2(q.scipy_csr(), q.b, q.c, q.n_orth, q.soc_sizes, mu=1.0, t=t, schedule=L).run(
                20000, eps=1e-4, check_every=10, obj_stop=1.0)
            times.append({"m": r.m, "kind": r.kind, "seconds": time.perf_counter() - t0})
        out["serve"] = times
    from oracle.subspace import RangeProjector

    p = synth.config1(scale=args.scale)
    t, L = default_parameters(p.soc_sizes)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    deadline = time.time() + 900
    while not os.path.exists(args.state_file):
        if time.time() > deadline:
            raise RuntimeError("no state from the GPU process")
        time.sleep(0.2)
    with np.load(args.state_file) as z:
        l0, s0, O0 = int(z["l"]), z["s"].astype(np.float64), z["O"].astype(np.float64)
    # the state of iteration l0: the projector and d of steps 12-13 for its O
    t0 = time.perf_counter()
    alg.O = O0
    alg.proj = RangeProjector(alg.A, O0)
    Oc = O0 * alg.c
    alg.d = alg.proj.pinv_apply(alg.b) + 0.5 * alg.mu * (alg.proj.reflect(Oc) - Oc)
    alg.s = s0.copy()
    alg.l = l0
    setup_s = time.perf_counter() - t0
    pcg0 = alg.proj.cg_iters
    t0 = time.perf_counter()
    for _ in range(args.cpu_iters):
        alg.step()
    dt = time.perf_counter() - t0
    out["lp2m"] = {"iters": args.cpu_iters, "seconds": dt, "pcg_iters": alg.proj.cg_iters - pcg0, "from_l": l0,
                   "setup_s": setup_s}
    print(json.dumps(out), flush=True)


def start_cpu_baseline(args):
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--scale", str(args.scale),
           "--cpu-iters", str(args.cpu_iters), "--workload", args.workload, "--count", str(args.count),
           "--serve-requests", str(args.serve_requests)]
    if args.workload == "lp2m":
        cmd += ["--state-file", args.state_file] + (["--headline-only"] if args.headline_only else [])
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, cwd=ROOT)


def finish_cpu_baseline(proc, timeout_s=600):
    try:
        out, err = proc.communicate(timeout=timeout_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        return None
    if proc.returncode != 0:
        sys.stderr.write(err[-2000:])
        return None
    r = json.loads(out.strip().splitlines()[-1])
    if "lp2m" in r:
        q = r["lp2m"]
        base = {
            "value": q["iters"] / q["seconds"], "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": (f"outer iterations {q['from_l'] + 1}..{q['from_l'] + q['iters']} of the FP64 oracle "
                       f"(Algorithm 2 step by step: two reflections per iteration, each projection by SciPy PCG "
                       f"to 1e-12 relative residual from zero, {q['pcg_iters']} PCG steps in all) from the GPU's "
                       f"state after its warmup, on the same full-size instance; the first iterations of the "
                       f"GPU's timed window, whose CG instead stops at a 0.1 reduction warm-started from the "
                       f"last w; single-threaded scipy.sparse SpMV, {q['seconds']:.1f} s (plus "
                       f"{q['setup_s']:.1f} s for the projector and d of steps 12-13, not counted)"),
        }
        if "lp200" in r:
            base["lp200"] = r["lp200"]
        if "serve" in r:
            base["serve_oracle"] = r["serve"]
        if "batch" in r:
            base["batch_solves_per_s"] = r["batch"]["solves"] / r["batch"]["seconds"]
            base["batch_sample"] = (f"{r['batch']['solves']} seeded instances of the batch recipe solved one at a "
                                    f"time to 1e-4 KKT by the FP64 oracle, {r['batch']['seconds']:.1f} s")
        return base
    if r.get("what") == "dense":
        return {"value": r["iters"] / r["seconds"], "unit": "iters/s", "cores": 1, "kind": "oracle",
                "sample": f"first {r['iters']} iterations of the FP64 oracle on the same recipe at n = 3000, "
                          f"m = 2400 (dense Cholesky projections, l = 1 conditioning included), "
                          f"{r['seconds']:.1f} s; the oracle needs minutes per iteration at n = 30000"}
    if r.get("what") == "solves":
        return {"value": r["iters"] / r["seconds"], "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"{r['iters']} seeded instances of the batch recipe solved one at a time to 1e-4 KKT by "
                          f"the FP64 oracle (dense Cholesky projections), {r['seconds']:.1f} s"}
    return {
        "value": r["iters"] / r["seconds"], "unit": "iters/s", "cores": 1, "kind": "oracle",
        "sample": (f"first {r['iters']} outer iteration(s) of the FP64 oracle (Algorithm 2 step by step, "
                   f"l=1 conditioning with its two projections for d, SciPy PCG to 1e-12, "
                   f"{r['pcg_iters']} PCG steps) on the same full-size instance; single-threaded "
                   f"scipy.sparse SpMV, {r['seconds']:.1f} s"),
    }


# ----------------------------------------------------------------------------
# algorithmic bytes per launch of the two CG kernels (value type bytes vt)
# ----------------------------------------------------------------------------
def kernel_bytes(m, n, nnz, vt=4, slices=8):
    """Algorithmic bytes of one launch: what the product needs in CSR form, each
    array once (index + value per nonzero, row pointers, the gathered vector,
    the output), not what this layout adds (SELL padding, chunk row tables,
    slice partials)."""
    # k_cg_a_part: q = A_s t (its 8 column slices together)
    cg_a = (4 + vt) * nnz + 4 * (m + 1) + vt * n + vt * m
    # k_cg_t: t = A_s^T r + beta t_old
    cg_t = (4 + vt) * nnz + 4 * (n + 1) + vt * m + 2 * vt * n
    # k_cg_a_comb: 8 partials read, r and q read + written, w (FP64) read + written
    comb = slices * vt * m + 4 * vt * m + 16 * m
    return {"cg_a": cg_a, "cg_t": cg_t, "cg_comb": comb}


def traffic_record(kernel, workload="lp2m", source="acs_kernels.hip"):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2103_00736_amd", "csrc", source), "rb").read()
    if rec.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.cpu_child:
        cpu_child(args)
        return 0
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2
    profiled = sorted(k for k in os.environ if k.startswith("ROCPROF"))
    if profiled and not args.no_cpu_baseline:
        # under a profiler the oracle child would start from a process the
        # profiler's library has attached to the GPU: never start it there
        print(f"bench.py: profiler environment ({profiled[0]}, ...) present: CPU baseline skipped",
              file=sys.stderr, flush=True)
        args.no_cpu_baseline = True
    if args.workload == "lp2m" and not args.no_cpu_baseline:
        import tempfile

        fd, args.state_file = tempfile.mkstemp(prefix="acs_state_", suffix=".npz")
        os.close(fd)
        os.unlink(args.state_file)  # the child waits for the file to appear
    cpu_proc = (None if (args.no_cpu_baseline or args.workload in ("serve", "copy", "gather"))
                else start_cpu_baseline(args))
    try:
        if args.workload == "batch":
            return bench_batch(args, cpu_proc)
        if args.workload == "serve":
            return bench_serve(args)
        if args.workload == "copy":
            return bench_copy()
        if args.workload == "gather":
            return bench_gather()
        if args.workload == "dense_solve":
            return bench_dense_solve(args)
        if args.workload == "dense" and args.projection == "factor":
            return bench_dense_factor(args, cpu_proc)
        if args.workload == "dense":
            return bench_dense(args, cpu_proc)
        if args.workload == "ablation":
            return bench_ablation()
        return bench_lp2m(args, cpu_proc)
    finally:
        if cpu_proc and cpu_proc.poll() is None:
            cpu_proc.kill()
        if args.state_file and os.path.exists(args.state_file):
            os.unlink(args.state_file)


CLS_NAMES = ("update", "resid", "cg_t", "cg_a", "check", "cond", "fin", "cg_comb")


def timed_window(acs, prob, warmup, steps, state_file=""):
    """Outer iterations warmup+1 .. warmup+steps of a fresh state: every kernel
    class timed once in a replay (breakdown), then the timed region with HIP
    events on the dominant CG kernel only, then a replay without events."""
    cls = {k: getattr(acs, "KC_" + k.upper()) for k in CLS_NAMES}
    st = acs.State(prob, precision=acs.PREC_MIXED)
    st.step(warmup)
    snap = st.get(xyz=False)  # iterate after the warmup, replayed below
    if state_file:
        tmp = state_file + ".part.npz"
        np.savez(tmp, l=snap["l"], s=snap["s"], O=snap["O"])
        os.replace(tmp, state_file)

    def replay(classes):
        st.set(snap["l"], snap["s_prev"], snap["s"], snap["O"], snap["w"])
        cg0 = st.info().cg_steps
        st.profile(classes if classes else False)
        t0 = time.perf_counter()
        st.step(steps)
        t1 = time.perf_counter()
        st.profile(False)
        info = st.info()
        return t1 - t0, info.cg_steps - cg0, info, {k: st.timing(v) for k, v in cls.items()}

    _, _, _, prof_all = replay(list(cls.values()))
    dom = max(("cg_a", "cg_t"), key=lambda k: prof_all[k][1])
    _progress(f"timed region: {steps} iterations")
    elapsed, cg_timed, info, prof = replay([cls[dom]])
    no_ev_s, no_ev_cg, _, _ = replay(None)
    st.close()
    return {"elapsed": elapsed, "cg": cg_timed, "info": info, "dom": dom, "dom_timing": prof[dom],
            "prof_all": prof_all, "no_ev_s": no_ev_s, "no_ev_cg": no_ev_cg}


def roofline_of(win, m, n, nnz, workload):
    kb = kernel_bytes(m, n, nnz)
    dom = win["dom"]
    count, total_ms = win["dom_timing"]
    # CG launches issued after the device-side stop test has fired exit at once;
    # their (small) time is charged to the working launches: an upper bound
    avg_ms = total_ms / max(win["cg"], 1)
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": {"cg_a": "k_cg_a_part", "cg_t": "k_cg_t"}[dom], "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record(dom, workload), "avg_launch_ms": avg_ms, "launches": count,
            "working_launches": win["cg"], "algorithmic_bytes_per_launch": kb[dom]}


def whole_solve(acs, prob, p, eps=1e-4):
    """A whole solve from the initial state to eps KKT (acs_solve)."""
    x, y, z, info = acs.solve(prob, eps_kkt=eps, max_iter=20000)
    return {"status": {acs.SOLVED: "solved"}.get(info.status, f"status {info.status}"),
            "iterations": info.iterations, "cg_steps": info.cg_steps, "solve_s": info.solve_ms * 1e-3,
            "setup_s": info.setup_ms * 1e-3, "iters_per_s": info.iterations / max(info.solve_ms * 1e-3, 1e-9),
            "kkt": info.kkt, "eps_obj": info.eps_obj,
            "objective_rel_error": abs(info.pobj - p.p_star) / (1.0 + abs(p.p_star))}


def bench_lp2m(args, cpu_proc):
    from paper_2103_00736_amd import acs, synth

    t0 = time.perf_counter()
    p = synth.config1(scale=args.scale)
    gen_s = time.perf_counter() - t0
    rc = acs.lib().acs_init(0)
    if rc != 0:
        raise RuntimeError(acs.lib().acs_last_error().decode())
    prob = acs.Problem.from_synth(p)
    win = timed_window(acs, prob, args.warmup, args.steps, args.state_file)
    info1 = win["info"]
    roof = roofline_of(win, p.m, p.n, p.nnz, "lp2m")
    detail = {
        "cg_steps_per_iter": win["cg"] / args.steps,
        "kkt_after": info1.kkt, "eps_p": info1.eps_p, "eps_d": info1.eps_d, "eps_gap": info1.eps_gap,
        "pobj": info1.pobj, "p_star": p.p_star,
        "kernel_ms": {k: {"count": v[0], "total_ms": round(v[1], 3)} for k, v in win["prof_all"].items()},
        "kernel_ms_what": "every kernel class timed with events in a replay of the timed iterations",
        "timed_s": win["elapsed"], "gen_s": gen_s,
        "replay_without_events": {"iters_per_s": args.steps / win["no_ev_s"], "timed_s": win["no_ev_s"],
                                  "cg_steps": win["no_ev_cg"],
                                  "what": "the timed iterations replayed from the saved iterate without "
                                          "per-launch HIP events"},
    }
    if not args.headline_only:
        _progress("2M-variable LP: whole solve")
        detail["lp2m_whole_solve"] = whole_solve(acs, prob, p)
        del prob
        q0 = synth.config0()
        h0 = acs.Problem.from_synth(q0)
        # the first solve also loads the FP64 kernels' code (lazily, at their
        # first launch in the process): reported apart, the second is timed
        first = acs.solve(h0, precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=20000)[3]
        x0, y0, z0, i0 = acs.solve(h0, precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=20000)
        detail["lp200_fp64"] = {"workload": "LP 200x500, 2% density, FP64 end to end, to 1e-6 KKT",
                                "status": {acs.SOLVED: "solved"}.get(i0.status, f"status {i0.status}"),
                                "iterations": i0.iterations, "cg_steps": i0.cg_steps, "solve_s": i0.solve_ms * 1e-3,
                                "first_solve_s": first.solve_ms * 1e-3, "kkt": i0.kkt,
                                "objective_rel_error": abs(i0.pobj - q0.p_star) / (1 + abs(q0.p_star))}
        # the same with ACS_PROJ_AUTO, which takes the direct projection at this m
        acs.solve(h0, precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=20000, projection=acs.PROJ_AUTO)
        i1 = acs.solve(h0, precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=20000, projection=acs.PROJ_AUTO)[3]
        detail["lp200_fp64"]["projection_auto"] = {
            "status": {acs.SOLVED: "solved"}.get(i1.status, f"status {i1.status}"), "iterations": i1.iterations,
            "solve_s": i1.solve_ms * 1e-3, "kkt": i1.kkt,
            "objective_rel_error": abs(i1.pobj - q0.p_star) / (1 + abs(q0.p_star)),
            "what": "ACS_PROJ_AUTO: the direct projection (m <= 2048), second solve"}
        detail["socp1m"] = socp_section(acs, synth, args)
        detail["batch4096"] = batch_section(acs, synth, args.count)
        detail["serve"] = serve_section(acs, synth, args.serve_requests, 200.0, args.workers, args.small_nnz)
    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc else None
    if cpu and "lp200" in cpu:
        o = cpu.pop("lp200")
        if "lp200_fp64" in detail:
            detail["lp200_fp64"]["oracle"] = {"iterations": o["iters"], "solve_s": o["seconds"], "kkt": o["kkt"],
                                              "cores": 1, "what": "the FP64 oracle's whole solve, same rule"}
    if cpu and "serve_oracle" in cpu:
        o = cpu.pop("serve_oracle")
        if "serve" in detail:
            detail["serve"]["oracle_service_s"] = {
                "requests": o, "cores": 1,
                "what": "the FP64 oracle's whole solves of the trace's four smallest requests, one at a time"}
    if cpu and "batch_solves_per_s" in cpu and "batch4096" in detail:
        detail["batch4096"]["oracle_solves_per_s"] = cpu.pop("batch_solves_per_s")
        detail["batch4096"]["oracle_sample"] = cpu.pop("batch_sample") + " (1 core)"
    line = {
        "metric": "iters/sec + HBM GB/s (2M-var LP); batched solves/sec, p99 latency at 1e-4 KKT",
        "value": args.steps / win["elapsed"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * win["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sparse LP m={p.m} n={p.n} nnz={p.nnz}, power-law rows, row scales 1e+-3 "
                               f"(Algorithm 2, mu=1, t=9.2, L={{300,400,...}}, iterations {args.warmup + 1}.."
                               f"{args.warmup + args.steps})",
                   "precision": "FP32 matrix/iterate/CG vectors, FP64 CG solution, residual sweeps and reductions"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)
    return 0


def socp_section(acs, synth, args):
    """The 1M-variable SOCP: iterations/s over the same window as the LP, with
    the dominant kernel's roofline, and a whole solve."""
    t0 = time.perf_counter()
    q = synth.config2()
    gen_s = time.perf_counter() - t0
    _progress(f"SOCP {q.m}x{q.n}: window and whole solve")
    prob = acs.Problem.from_synth(q)
    win = timed_window(acs, prob, args.warmup, args.steps)
    return {"workload": f"SOCP m={q.m} n={q.n} nnz={q.nnz}, {len(q.soc_sizes)} Lorentz cones U{{3..50}} "
                        f"+ {q.n_orth} orthant, iterations {args.warmup + 1}..{args.warmup + args.steps}",
            "iters_per_s": args.steps / win["elapsed"], "cg_steps_per_iter": win["cg"] / args.steps,
            "iters_per_s_without_events": args.steps / win["no_ev_s"],
            "roofline": roofline_of(win, q.m, q.n, q.nnz, "socp1m"),
            "whole_solve": whole_solve(acs, prob, q), "gen_s": gen_s}


def bench_copy():
    """A plain device copy of exactly 1 GiB (torch), the calibration dispatch for HBM byte counters."""
    import torch

    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"metric": "copy GB/s (read+write)", "value": 2 * (1 << 30) / ms / 1e6, "unit": "GB/s",
                      "bytes_each_way": 1 << 30, "ms": ms}), flush=True)
    return 0


def bench_gather():
    """Gather ceiling of the CG's product kernels: the library's own SELL
    products (acs_state_spmv, FP32) on matrices with 5 random rows per column,
    so that every nonzero costs one random 4-byte read of the gathered vector,
    compared with the 2M-variable LP itself.  A^T x gathers from the m-vector
    (2 MB for m = 500k, 32 KB for m = 8192: resident in L1); A x gathers from
    the n-vector, 1 MB per XCD through the column slices."""
    import torch
    from paper_2103_00736_amd import acs, synth

    rc = acs.lib().acs_init(0)
    if rc != 0:
        raise RuntimeError(acs.lib().acs_last_error().decode())
    cases = [("uniform rows, m=500k (2 MB gathered by A^T x)", lambda: synth.lp_percol(500_000, 2_000_000, 5, 11)),
             ("uniform rows, m=131072 (512 KB gathered by A^T x)", lambda: synth.lp_percol(131072, 2_000_000, 5, 13)),
             ("uniform rows, m=32768 (128 KB gathered by A^T x)", lambda: synth.lp_percol(32768, 2_000_000, 5, 14)),
             ("uniform rows, m=8192 (32 KB gathered by A^T x)", lambda: synth.lp_percol(8192, 2_000_000, 5, 12)),
             ("uniform rows, m=64 (256 B gathered by A^T x: every gather hits L1)",
              lambda: synth.lp_percol(64, 2_000_000, 5, 15)),
             ("2M-variable LP, power-law rows", lambda: synth.config1())]
    out = {}
    dev = torch.device("cuda:0")
    for name, make in cases:
        _progress(f"gather case: {name}")
        p = make()
        st = acs.State(acs.Problem.from_synth(p))
        st.step(1)  # scaled values in place
        xn = torch.ones(p.n, dtype=torch.float32, device=dev)
        xm = torch.ones(p.m, dtype=torch.float32, device=dev)
        ym = torch.empty(p.m, dtype=torch.float32, device=dev)
        yn = torch.empty(p.n, dtype=torch.float32, device=dev)
        st.spmv(1, xm.data_ptr(), yn.data_ptr(), 5)
        st.spmv(0, xn.data_ptr(), ym.data_ptr(), 5)
        t_ms = st.spmv(1, xm.data_ptr(), yn.data_ptr(), 50)
        a_ms = st.spmv(0, xn.data_ptr(), ym.data_ptr(), 50)
        st.close()
        out[name] = {"m": p.m, "n": p.n, "nnz": int(p.nnz),
                     "At_x_us": t_ms * 1e3, "At_x_Ggather_per_s": p.nnz / (t_ms * 1e-3) / 1e9,
                     "A_x_us": a_ms * 1e3, "A_x_Ggather_per_s": p.nnz / (a_ms * 1e-3) / 1e9}
    first = next(iter(out.values()))
    print(json.dumps({"metric": "gather rate of the CG product kernels (A^T x, uniform rows, 2 MB vector)",
                      "value": first["At_x_Ggather_per_s"], "unit": "Ggather/s", "higher_is_better": True,
                      "data": "synthetic", "dtype": "f32",
                      "what": "acs_state_spmv with 50 back-to-back launches timed by HIP events; A x includes "
                              "the slice-combine kernel, A^T x the row-order permutation of its input",
                      "cases": out}), flush=True)
    return 0


def dense_kernel_bytes(m, n, vt=4):
    """Algorithmic bytes of the dense CG launches: A once (FP32) plus the vectors."""
    rows = 4 * m * n + vt * n + (3 * vt + 16) * m  # A_s t and the CG update of r, q, w
    cols = 4 * m * n + vt * m + 8 * m + 3 * vt * n  # A_s^T r (+ beta t_old, O t written)
    return {"cg_a": rows, "cg_t": cols}


def bench_dense(args, cpu_proc):
    """Iterations/s on the paper's random dense LP (Sec. V-B recipe) at n =
    30000, m = 24000: A is 2.9 GB of FP32 streamed twice per CG step."""
    from paper_2103_00736_amd import acs, synth

    t0 = time.perf_counter()
    p = synth.e3_lp(args.dense_n)
    gen_s = time.perf_counter() - t0
    rc = acs.lib().acs_init(0)
    if rc != 0:
        raise RuntimeError(acs.lib().acs_last_error().decode())
    prob = acs.Problem.from_synth(p)
    del p.A
    st = acs.State(prob, precision=acs.PREC_MIXED)
    warmup = min(args.warmup, 10)
    steps = min(args.steps, 20)
    _progress(f"dense LP {p.m}x{p.n}: warmup {warmup}")
    st.step(warmup)
    cls = {"update": acs.KC_UPDATE, "resid": acs.KC_RESID, "cg_t": acs.KC_CG_T, "cg_a": acs.KC_CG_A,
           "check": acs.KC_CHECK, "cond": acs.KC_COND, "fin": acs.KC_FIN}
    _progress(f"timed region: {steps} iterations")
    cg0 = st.info().cg_steps
    st.profile([acs.KC_CG_A])
    t1 = time.perf_counter()
    st.step(steps)
    t2 = time.perf_counter()
    st.profile(False)
    info = st.info()
    cg = info.cg_steps - cg0
    count, total_ms = st.timing(acs.KC_CG_A)
    kb = dense_kernel_bytes(p.m, p.n)
    avg_ms = total_ms / max(cg, 1)
    achieved = kb["cg_a"] / (avg_ms * 1e-3) / 1e9
    # breakdown of every class over a few more iterations
    st.profile(list(cls.values()))
    st.step(3)
    st.profile(False)
    prof = {k: st.timing(v) for k, v in cls.items()}
    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc else None
    elapsed = t2 - t1
    print(json.dumps({
        "metric": "iters/sec on the paper's dense random LP (Sec. V-B recipe)", "value": steps / elapsed,
        "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"dense LP m={p.m} n={p.n}, A~U[-1,1] (FP32, {4 * p.m * p.n / 1e9:.2f} GB), "
                               f"b=A|x|, c~N(0,1), t=9.2, L={{300,400,...}}",
                   "precision": "FP32 A and CG vectors, FP64 CG solution, residual sweeps and reductions"},
        "roofline": {"bound": "hbm", "kernel": "k_dense_rows (CG)", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_record("cg_a", "dense_lp"),
                     "avg_launch_ms": avg_ms,
                     "launches": count, "working_launches": cg, "algorithmic_bytes_per_launch": kb["cg_a"]},
        "cpu_baseline": cpu,
        "detail": {"cg_steps_per_iter": cg / steps, "gen_s": gen_s,
                   "kernel_ms": {k: {"count": v[0], "total_ms": round(v[1], 3)} for k, v in prof.items()},
                   "kernel_ms_what": "every kernel class timed in 3 further iterations",
                   "cg_t_bytes_per_launch": kb["cg_t"]},
    }), flush=True)
    return 0


def bench_dense_factor(args, cpu_proc):
    """Iterations/s on the dense LP at n = 30000 with the direct projection,
    over iterations 251-350: one conditioning event (l = 300), so the window
    carries one formation and inversion of A_s A_s^T (m = 24000) and 100
    applications of its inverse, the schedule's share of factorization work.
    The CG projection is timed over the same window for comparison."""
    from paper_2103_00736_amd import acs, synth

    t0 = time.perf_counter()
    p = synth.e3_lp(args.dense_n)
    gen_s = time.perf_counter() - t0
    rc = acs.lib().acs_init(0)
    if rc != 0:
        raise RuntimeError(acs.lib().acs_last_error().decode())
    prob = acs.Problem.from_synth(p)
    del p.A
    m, n = p.m, p.n
    warmup, steps = 250, 100
    fac_cls = {"syrk": acs.KC_FAC_SYRK, "update": acs.KC_FAC_UPDATE, "apply": acs.KC_FAC_APPLY,
               "panel": acs.KC_FAC_PANEL}
    rates = {"cg": None}
    for proj in (("factor",) if args.skip_cg_compare else ("factor", "cg")):
        st = acs.State(prob, precision=acs.PREC_MIXED,
                       projection=acs.PROJ_FACTOR if proj == "factor" else acs.PROJ_CG)
        _progress(f"dense LP {m}x{n}, {proj} projection: warmup {warmup}")
        st.step(warmup)
        _progress(f"timed region: {steps} iterations (event at l = 300 inside)")
        if proj == "factor":
            st.profile(list(fac_cls.values()))
        t1 = time.perf_counter()
        st.step(steps)
        t2 = time.perf_counter()
        rates[proj] = steps / (t2 - t1)
        if proj == "factor":
            st.profile(False)
            prof = {k: st.timing(v) for k, v in fac_cls.items()}
            elapsed = t2 - t1
            info = st.info()
        st.close()
    # Algorithmic work per launch:
    #   k_fac_syrk: the lower triangle of B B^T, m (m + 1) / 2 dot products of
    #     length n: m (m + 1) n flops;
    #   k_fac_update (one pass over S per group of up to 4 sweep steps
    #     K0 .. K0 + cnt - 1): every lower 64 x 64 tile of S outside block row
    #     and column K0 + cnt - 1 read and written once (16 bytes an entry)
    #     and the cnt 64-column panels W read once; 2 * 64 flops an entry for
    #     each step's term the tile takes (a tile on the row of group block
    #     K0 + h takes only the steps after it).  Per launch: the event's
    #     total over its launches;
    #   k_fac_apply: M^{-1} once (FP64) and three m-vectors.
    nb = (m + 63) // 64
    group = 4
    upd_bytes_sum = upd_flops_sum = 0
    upd_launches = 0
    low = np.tril(np.ones((nb, nb), dtype=bool))
    for k0 in range(0, nb, group):
        cnt = min(group, nb - k0)
        h = np.full(nb, -1)
        h[k0:k0 + cnt] = np.arange(cnt)
        terms = cnt - 1 - np.maximum(h[:, None], h[None, :])
        mask = low.copy()
        mask[k0 + cnt - 1, :] = False
        mask[:, k0 + cnt - 1] = False
        upd_flops_sum += 2 * 64 ** 3 * int(terms[mask].sum())
        upd_bytes_sum += 16 * 64 * 64 * int(mask.sum()) + cnt * 8 * 64 * 64 * nb
        upd_launches += 1
    upd_bytes = upd_bytes_sum // upd_launches
    upd_flops = upd_flops_sum // upd_launches
    syrk_flops = m * (m + 1) * n
    apply_bytes = 8 * m * m + 8 * 3 * m
    cnt_s, ms_s = prof["syrk"]
    cnt_u, ms_u = prof["update"]
    cnt_a, ms_a = prof["apply"]
    cnt_p, ms_p = prof["panel"]
    syrk_tf = syrk_flops * cnt_s / (ms_s * 1e-3) / 1e12 if ms_s > 0 else 0.0
    upd_gbs = upd_bytes * cnt_u / (ms_u * 1e-3) / 1e9 if ms_u > 0 else 0.0
    upd_tf = upd_flops * cnt_u / (ms_u * 1e-3) / 1e12 if ms_u > 0 else 0.0
    apply_gbs = apply_bytes * cnt_a / (ms_a * 1e-3) / 1e9 if ms_a > 0 else 0.0
    dom = max(("syrk", ms_s), ("update", ms_u), ("apply", ms_a), key=lambda kv: kv[1])[0]
    if dom == "apply":
        roof = {"bound": "hbm", "kernel": "k_fac_apply", "achieved": apply_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": apply_gbs / HBM_PEAK_GBS, "traffic": traffic_record("fac_apply", "dense_lp", "acs_factor.hip"),
                "avg_launch_ms": ms_a / max(cnt_a, 1), "launches": cnt_a, "algorithmic_bytes_per_launch": apply_bytes}
    elif dom == "syrk":
        roof = {"bound": "mfma", "kernel": "k_fac_syrk (FP64 MFMA)", "achieved": syrk_tf, "peak": FP64_PEAK_TFS,
                "unit": "TFLOP/s", "frac": syrk_tf / FP64_PEAK_TFS,
                "traffic": traffic_record("fac_syrk", "dense_lp", "acs_factor.hip"),
                "avg_launch_ms": ms_s / max(cnt_s, 1), "launches": cnt_s, "algorithmic_flops_per_launch": syrk_flops}
    elif upd_flops / (FP64_PEAK_TFS * 1e12) >= upd_bytes / (HBM_PEAK_GBS * 1e9):
        # four steps a pass over S: at the peaks its flops take longer than its bytes
        roof = {"bound": "mfma", "kernel": "k_fac_update (pass of four rank-64 sweep steps, FP64 MFMA)", "achieved": upd_tf,
                "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": upd_tf / FP64_PEAK_TFS,
                "traffic": traffic_record("fac_update", "dense_lp", "acs_factor.hip"),
                "avg_launch_ms": ms_u / max(cnt_u, 1), "launches": cnt_u, "algorithmic_flops_per_launch": upd_flops,
                "algorithmic_bytes_per_launch": upd_bytes, "hbm_gbs": upd_gbs}
    else:
        roof = {"bound": "hbm", "kernel": "k_fac_update (sweep steps)", "achieved": upd_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": upd_gbs / HBM_PEAK_GBS,
                "traffic": traffic_record("fac_update", "dense_lp", "acs_factor.hip"),
                "avg_launch_ms": ms_u / max(cnt_u, 1), "launches": cnt_u, "algorithmic_bytes_per_launch": upd_bytes,
                "fp64_tflops": upd_tf}
    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc else None
    print(json.dumps({
        "metric": "iters/sec on the paper's dense random LP (Sec. V-B recipe), direct projection",
        "value": steps / elapsed, "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dense LP m={m} n={n}, A~U[-1,1] (FP32 storage), b=A|x|, c~N(0,1), t=9.2, "
                               f"L={{300,400,...}}; iterations {warmup + 1}-{warmup + steps}",
                   "precision": "A_s A_s^T and its inverse in FP64 (MFMA), FP64 residual and apply; "
                                "FP32 iterate"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": {"gen_s": gen_s, "cg_iters_per_s_same_window": rates["cg"],
                   "speedup_vs_cg_same_window": rates["factor"] / rates["cg"] if rates["cg"] else None,
                   "syrk": {"count": cnt_s, "total_ms": ms_s, "tflops": syrk_tf},
                   "update": {"count": cnt_u, "total_ms": ms_u, "gbs": upd_gbs, "tflops": upd_tf},
                   "pivot_panel_mirror": {"count": cnt_p, "total_ms": ms_p},
                   "apply": {"count": cnt_a, "total_ms": ms_a, "gbs": apply_gbs},
                   "event_ms": ms_s + ms_u + ms_p,
                   "factor_info": {"iterations": info.iterations, "conditionings": info.conditionings}},
    }), flush=True)
    return 0


def bench_dense_solve(args):
    """Whole solves of the dense LP (n = 30000, m = 24000) to 1e-4 KKT in mixed
    precision, with the direct projection and with the CG projection: wall
    time of the iteration loop, iterations, conditioning events, KKT."""
    from paper_2103_00736_amd import acs, synth

    p = synth.e3_lp(args.dense_n)
    assert acs.lib().acs_init(0) == 0
    prob = acs.Problem.from_synth(p)
    del p.A
    out = {}
    for name, proj in (("factor", acs.PROJ_FACTOR), ("cg", acs.PROJ_CG)):
        _progress(f"dense LP {p.m}x{p.n}: full solve, {name} projection")
        st = acs.State(prob, precision=acs.PREC_MIXED, projection=proj, eps_kkt=1e-4, max_iter=20000)
        t0 = time.perf_counter()
        info = st.solve()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "status": info.status, "iterations": info.iterations,
                     "conditionings": info.conditionings, "kkt": info.kkt, "pobj": info.pobj,
                     "cg_steps": info.cg_steps}
        st.close()
    print(json.dumps({"metric": "time to 1e-4 KKT on the paper's dense random LP (Sec. V-B recipe)",
                      "value": out["factor"]["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
                      "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"dense LP m={p.m} n={p.n}, mixed precision, t=9.2, L={{300,400,...}}"},
                      "solves": out, "speedup_factor_vs_cg": out["cg"]["seconds"] / out["factor"]["seconds"]}),
          flush=True)
    return 0


def bench_ablation():
    """The paper's conditioning-schedule example (Sec. IV): iterations to 1e-6
    KKT of its 10 random 80 x 100 LPs under L = {}, {300}, {1..50} (t = 9.2), on
    the GPU (one batch launch per schedule) and with the FP64 oracle."""
    import scipy.sparse as sp
    from oracle.alg2 import Algorithm2, Schedule
    from paper_2103_00736_amd import acs, synth

    rc = acs.lib().acs_init(0)
    if rc != 0:
        raise RuntimeError(acs.lib().acs_last_error().decode())
    probs = [synth.e2_lp(i) for i in range(10)]
    handles = []
    for p in probs:
        A = sp.csr_matrix(p.A)
        handles.append(acs.Problem(p.m, p.n, A.indptr, A.indices, A.data, p.b, p.c, p.n_orth))
    sched = {"none": (0, 0, -1), "once_300": (300, 0, -1), "first_50": (1, 1, 50)}
    out = {}
    for name, (f, e, last) in sched.items():
        _progress(f"schedule {name}")
        b = acs.Batch(handles, eps_kkt=1e-6, max_iter=20000, auto_params=0, t=9.2, mu=1.0, check_every=10, obj_stop=0,
                      l_first=f, l_every=e, l_last=last)
        ms = b.run(20000)
        gpu = [b.result(i)[3].iterations for i in range(len(probs))]
        cpu = []
        for p in probs:
            alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=9.2,
                             schedule=Schedule(f, e, last))
            alg.run(20000, eps=1e-6, check_every=10)
            cpu.append(alg.l)
        out[name] = {"gpu_iterations": gpu, "oracle_iterations": cpu, "gpu_median": float(np.median(gpu)),
                     "oracle_median": float(np.median(cpu)), "batch_ms": ms}
    print(json.dumps({"metric": "iterations to 1e-6 KKT by conditioning schedule (paper Sec. IV example)",
                      "value": out["once_300"]["gpu_median"] / out["none"]["gpu_median"],
                      "unit": "median iterations with L={300} / with L={}", "higher_is_better": False,
                      "data": "synthetic", "dtype": "f32", "schedules": out}), flush=True)
    return 0


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _base_line(metric, value, unit, config, steps=1, ms=None):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": 0,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": config}


def batch_section(acs, synth, count):
    """`count` small LPs of the batch recipe in one persistent launch, against
    the plain one-instance GPU solver on a seeded subset."""
    t0 = time.perf_counter()
    probs = [synth.config3(i) for i in range(count)]
    handles = [acs.Problem.from_synth(p) for p in probs]
    gen_s = time.perf_counter() - t0
    _progress(f"generated {len(probs)} batch instances in {gen_s:.1f} s")
    b = acs.Batch(handles, eps_kkt=1e-4, max_iter=20000)
    t1 = time.perf_counter()
    b.autotune(sample=4, iters=20, cache_path=os.path.join("/tmp", "acs_lanes_gfx950.txt"))
    tune_s = time.perf_counter() - t1
    ms = b.run(20000)
    _progress(f"batch launch {ms:.1f} ms")
    infos = [b.result(i, xyz=False)[3] for i in range(len(probs))]
    solved = sum(1 for f in infos if f.status == acs.SOLVED)
    obj = [abs(f.pobj - p.p_star) / (1.0 + abs(p.p_star)) for p, f in zip(probs, infos)]
    # algorithmic bytes moved by the launch (mixed precision: FP32 CG sweeps, FP64 residual/update sweeps)
    byts = 0.0
    for p, f in zip(probs, infos):
        m, n, nnz = p.m, p.n, p.nnz
        cg = (4 * (n + 1) + 8 * nnz + 4 * m + 8 * n) + (4 * (m + 1) + 8 * nnz + 4 * n + 32 * m)
        it = (4 * (m + 1) + 12 * nnz + 4 * n + 12 * m) + (4 * (n + 1) + 12 * nnz + 8 * m + 20 * n)
        byts += f.cg_steps * cg + f.iterations * it
    achieved = byts / (ms * 1e-3) / 1e9
    b.close()
    # the plain one-instance GPU solver on a seeded subset, one at a time
    # the batch's uploads happen before its timed launch: time only the
    # iterations of each one-instance solve (info.solve_ms), not its set-up
    sub = np.random.default_rng(2).choice(len(probs), size=min(48, len(probs)), replace=False)
    per = 0.0
    for i in sub:
        per += acs.solve(handles[int(i)], eps_kkt=1e-4, max_iter=20000)[3].solve_ms * 1e-3
    per /= len(sub)
    value = len(probs) / (ms * 1e-3)
    return {"workload": f"{len(probs)} planted sparse LPs, m~U{{50..2000}}, n=2.5m, 1% density, "
                        f"sum nnz={sum(p.nnz for p in probs)}, one persistent graph-launched kernel",
            "solves_per_s": value, "launch_ms": ms, "solved": solved, "count": len(probs),
            "max_gpu_kkt": max(f.kkt for f in infos), "max_objective_rel_error": max(obj),
            "objective_rel_error_above_1e-4": [int(i) for i in np.nonzero(np.array(obj) > 1e-4)[0]],
            "mean_iterations": float(np.mean([f.iterations for f in infos])),
            "one_at_a_time_gpu_solves_per_s": 1.0 / per,
            "one_at_a_time_sample": f"{len(sub)} seeded instances solved sequentially by acs_solve, "
                                    f"iterations only (set-up excluded, as for the batch)",
            "speedup_vs_one_at_a_time": value * per,
            "roofline": {"bound": "hbm", "kernel": "k_batch", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic_record("batch", "batch4096", "acs_batch.hip"),
                         "avg_launch_ms": ms, "launches": 1, "algorithmic_bytes_per_launch": byts},
            "gen_s": gen_s, "autotune_s": tune_s}


def bench_batch(args, cpu_proc):
    """4096 small LPs (m ~ U{50..2000}, n = 2.5m, 1% density) in one persistent launch."""
    from paper_2103_00736_amd import acs, synth

    assert acs.lib().acs_init(0) == 0
    d = batch_section(acs, synth, args.count)
    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc else None
    line = _base_line("batched solves/sec at 1e-4 KKT", d["solves_per_s"], "solves/s",
                      {"workload": d["workload"],
                       "precision": "FP32 CG sweeps, FP64 residual/update sweeps and reductions"}, 1, d["launch_ms"])
    line["roofline"] = d.pop("roofline")
    line["cpu_baseline"] = cpu
    line["detail"] = d
    print(json.dumps(line), flush=True)
    return 0


def _serve_run(acs, srv_kw, trace, handles, arrivals, warm):
    """Submit every request at its arrival time (a client thread) and wait for all."""
    srv = acs.Server(**srv_kw)
    tickets = [None] * len(trace)
    lag = np.zeros(len(trace))  # arrival -> call of submit (the client was still in an earlier submit)
    start = time.perf_counter()

    def client():
        for i in range(len(trace)):
            delay = start + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            lag[i] = max(0.0, time.perf_counter() - (start + arrivals[i]))
            tickets[i] = srv.submit(handles[i], eps_kkt=1e-4, max_iter=20000)

    th = threading.Thread(target=client)
    th.start()
    th.join()
    res = []
    for i in range(len(trace)):
        x, y, z, info = srv.wait(tickets[i], -1)
        res.append(info)
    end = time.perf_counter()
    st = srv.stats()
    srv.close()
    srv_lat = np.array([f.latency_ms for f in res[warm:]])
    lat = srv_lat + 1e3 * lag[warm:]
    queue = np.array([f.queue_ms for f in res[warm:]])
    half = len(lat) // 2
    return {"requests": len(res), "warmup_excluded": warm,
            "offered_rate": (len(trace) - 1) / max(arrivals[-1], 1e-9), "solves_per_s": len(res) / (end - start),
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "latency_from": "the request's arrival time: the client's lag before submit (still inside an earlier "
                            "submit) plus the server's latency from the entry of submit to the result",
            "p50_p99_server_latency_ms": [float(np.percentile(srv_lat, 50)), float(np.percentile(srv_lat, 99))],
            "mean_client_lag_ms": float(1e3 * np.mean(lag[warm:])),
            "mean_queue_ms": float(np.mean(queue)),
            "queue_ms_first_half_vs_second_half": [float(np.mean(queue[:half])), float(np.mean(queue[half:]))],
            "solved": sum(1 for f in res if f.status == acs.SOLVED), "makespan_s": end - start,
            "peak_resident": st["peak_running"], "pool_ticks": st["ticks"]}


def serve_section(acs, synth, requests, rate, workers, small_nnz):
    """Poisson request stream (70% LP / 30% SOCP, m log-uniform in [1e3, 2e5])
    through the serving loop at the offered rate, then the same requests at
    a rate the server sustains (3/4 of the throughput it reached), against
    the same requests solved one at a time by acs_solve.  Every run starts
    from fresh problem handles, so each pays the per-problem layout build
    inside its timing, as a served request does."""
    trace = synth.config4_trace(requests, rate_per_s=rate)
    t0 = time.perf_counter()
    probs = []
    for k, r in enumerate(trace):
        probs.append(r.problem())
        if k % 40 == 0:
            _progress(f"generated {k + 1}/{len(trace)} requests")
    gen_s = time.perf_counter() - t0

    def fresh():
        return [acs.Problem.from_synth(q) for q in probs]

    srv_kw = dict(hbm_budget=160 << 30, max_slots=512, small_nnz=small_nnz, workers=workers, tick_iters=50)
    warm = max(1, len(trace) // 10)
    arrivals = np.array([r.arrival_s for r in trace])
    _progress(f"serving {len(trace)} requests at {rate:g}/s")
    offered = _serve_run(acs, srv_kw, trace, fresh(), arrivals, warm)
    sustained_rate = 0.75 * offered["solves_per_s"]
    _progress(f"serving them again at {sustained_rate:.2f}/s")
    sustained = _serve_run(acs, srv_kw, trace, fresh(), arrivals * (rate / sustained_rate), warm)
    _progress("the same requests one at a time")
    handles = fresh()
    lat = []
    t2 = time.perf_counter()
    for h in handles:
        t3 = time.perf_counter()
        acs.solve(h, eps_kkt=1e-4, max_iter=20000)
        lat.append(time.perf_counter() - t3)
    seq_s = time.perf_counter() - t2
    return {"workload": f"{len(trace)} requests of the Poisson trace, 70% LP / 30% SOCP, m log-uniform "
                        f"[1e3, 2e5], n=3m, 6 nnz/column, SOC sizes U{{3..30}}, sum nnz={sum(q.nnz for q in probs)}",
            "server": f"small_nnz={small_nnz} pool (persistent kernel ticks of 50 iterations) + {workers} worker "
                      f"streams",
            "at_offered_rate": offered, "at_sustainable_rate": sustained,
            "one_at_a_time_gpu_solves_per_s": len(handles) / seq_s,
            "one_at_a_time_p50_p99_solve_ms": [1e3 * float(np.percentile(lat, 50)), 1e3 * float(np.percentile(lat, 99))],
            "one_at_a_time_sample": f"all {len(handles)} requests solved sequentially by acs_solve",
            "served_vs_one_at_a_time": offered["solves_per_s"] * seq_s / len(handles),
            "gen_s": gen_s}


def bench_serve(args):
    """The serving section on its own (--requests, --rate, --workers, --small-nnz)."""
    from paper_2103_00736_amd import acs, synth

    assert acs.lib().acs_init(0) == 0
    d = serve_section(acs, synth, args.requests, args.rate, args.workers, args.small_nnz)
    o = d["at_offered_rate"]
    line = _base_line("served solves/sec and latency at 1e-4 KKT", o["solves_per_s"], "solves/s",
                      {"workload": d["workload"], "server": d["server"]}, o["requests"],
                      1e3 * o["makespan_s"] / o["requests"])
    line["roofline"] = None
    line["cpu_baseline"] = None
    line["detail"] = d
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
