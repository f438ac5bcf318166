"""Benchmark: edge-matrix AMG-PCG on one MI355X.

Workload: 3D linear elasticity on the unit cube, 64^3 vertices (786,432 dofs, 774,144 free),
P1 Kuhn tetrahedra, E = 1, nu = 0.3, clamped at x = 0, seeded uniform RHS (seed 1); FP64
hierarchy and V-cycle; two matching passes per level, coarsening stopped below 8192 dofs
(the coarsest level, 1051 vertices here, is inverted on the GPU at setup and applied as one dense
product), one symmetric multicolour block Gauss-Seidel sweep pre / post; PCG to
||r|| <= 1e-8 ||b||.  The same problem with coarsening stopped below 500 dofs (seven levels) is
reported beside it as "coarsest_500".

A step is one PCG solve to 1e-8 (V-cycle + CG kernels) on the hierarchy, with b resident in
HBM when the timed region starts.  Setup (host coarsening + device P_s / Galerkin / D^+ /
coarsest factor) is timed separately and reported in the same line.  The same solve with the
FP32 V-cycle inside the FP64 CG is timed after it and reported as "mixed_fp32_vcycle", and the
batched block-panel solve of 32 seeded load cases on the same hierarchy (FP64 and FP32 V-cycle)
as "batched", 16 independent cubes of uneven size solved together as "multi_mesh", and the
learned coarsening against the exact one on a heterogeneous cube as "learned_coarsening".

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


# Coarsening stops below this many dofs: on one GPU the dense inverse of a coarsest level of a
# few thousand dofs (one HBM-bound product per V-cycle) is cheaper than the launch-bound colour
# sweeps of the small levels it replaces.
COARSEST_DOFS = 8192


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="vertices per cube side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=17, help="cube side of the oracle sample")
    ap.add_argument("--batch", type=int, default=32,
                    help="right-hand sides of the batched block-panel solve (0: skip)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-coarsening section")
    ap.add_argument("--learned-n", type=int, default=40,
                    help="cube side of the learned-coarsening comparison (96: the full configuration)")
    ap.add_argument("--learned-inclusions", type=int, default=60,
                    help="stiff spherical inclusions of that cube (200 at 96^3)")
    ap.add_argument("--counter-pass", action="store_true",
                    help="run only the workload of the rocprofv3 counter passes (no JSON line)")
    ap.add_argument("--multi", type=int, default=16,
                    help="independent meshes of the multi-system solve (0: skip)")
    ap.add_argument("--coarsest", type=int, default=COARSEST_DOFS,
                    help="coarsening stops once a level has fewer dofs than this")
    ap.add_argument("--no-coarsest-500", action="store_true",
                    help="skip the comparison with coarsening stopped below 500 dofs")
    return ap.parse_args()


def cpu_baseline(n):
    """The CPU oracle (FP64 NumPy/SciPy, one process, BLAS limited to one thread) on a bounded
    sample: setup and PCG solve to 1e-8 on an n^3 cube of the same problem family; the solve
    is timed."""
    from threadpoolctl import threadpool_limits

    import oracle
    from gen import make_problem
    p = make_problem(n, seed=1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        h = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
        t_setup = time.perf_counter() - t0
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            x, it, rel, rel_true, conv = oracle.pcg(h, p.b, rtol=1e-8)
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": p.n_free_dofs / t, "unit": "dofs/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup ({t_setup:.1f} s) + PCG to 1e-8 ({it} its, median of 3: "
                      f"{t:.2f} s) on the {n}^3-vertex cube ({p.n_free_dofs} free dofs) of the "
                      f"same elasticity problem, one thread"}


def _timed_solves(E, torch, hier, b, x, stream, steps, warmup, precond):
    for _ in range(warmup):
        hier.solve(b, x, precond=precond)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    infos = []
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        _, info = hier.solve(b, x, precond=precond)
        infos.append(info)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    assert infos[-1]["status"] == E.EAMG_OK and infos[-1]["rel_res_true"] <= 1e-8, infos[-1]
    return ms, infos[-1]


def _profiled(E, hier, b, x, steps, precond):
    """Per-kernel durations with events on the solve stream, over the same number of steps."""
    E.eamg_profile_enable(hier.h, True)
    for _ in range(steps):
        hier.solve(b, x, precond=precond)
    kstats = E.eamg_profile_read(hier.h)
    E.eamg_profile_enable(hier.h, False)
    dom = kstats[0]
    achieved = dom["bytes"] / (dom["total_ms"] / 1e3) / 1e9
    roof = {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": 8000.0,
            "unit": "GB/s", "frac": achieved / 8000.0, "traffic": _traffic(dom["name"]),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "avg_launch_us": dom["total_ms"] / dom["launches"] * 1e3,
            "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"]}
    kern = [{"name": k["name"], "launches_per_step": k["launches"] / steps,
             "ms_per_step": k["total_ms"] / steps,
             "GBps": k["bytes"] / (k["total_ms"] / 1e3) / 1e9 if k["total_ms"] else None}
            for k in kstats[:12]]
    return roof, kern


def _coarsest_500(E, torch, p, stream, steps, warmup, ms_headline):
    """The headline problem with coarsening stopped below 500 dofs (the small-problem setting):
    setup, autotune and the FP64 solve timed the same way."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(coarsest_max_dofs=500), stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    E.eamg_autotune(h.h, 0, stream=stream)
    b = torch.tensor(p.b, device="cuda")
    x = torch.zeros_like(b)
    ms, info = _timed_solves(E, torch, h, b, x, stream, steps, warmup, E.EAMG_PRECOND_VCYCLE)
    st = h.stats()
    h.close()
    return {"value": p.n_free_dofs / (ms / 1e3), "unit": "dofs/s", "ms_per_step": ms,
            "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
            "levels": st["n_levels"], "level_vertices": st["n"], "setup_s": round(setup_s, 3),
            "headline_speedup": ms / ms_headline}


def _batch_rhs(p, m):
    """m seeded load cases (case c from default_rng([4, c])), uniform[-1, 1], Dirichlet dofs 0."""
    B = np.stack([np.random.default_rng([4, c]).uniform(-1.0, 1.0, p.n_dofs) for c in range(m)])
    B[:, np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    return B


def _batched(E, torch, hier, p, m, steps, warmup):
    """Batched block-panel solves of m right-hand sides, FP64 and FP32 V-cycle."""
    B = torch.tensor(_batch_rhs(p, m), device="cuda")
    X = torch.zeros_like(B)
    out = {"rhs": m}
    for prec, key in ((E.EAMG_PRECOND_VCYCLE, "fp64_vcycle"), (E.EAMG_PRECOND_VCYCLE_FP32, "fp32_vcycle")):
        for _ in range(warmup):
            hier.solve_batch(B, X, precond=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, infos = hier.solve_batch(B, X, precond=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        assert st == E.EAMG_OK and max(i["rel_res_true"] for i in infos) <= 1e-8, st
        E.eamg_profile_enable(hier.h, True)
        hier.solve_batch(B, X, precond=prec)
        ks = E.eamg_profile_read(hier.h)
        E.eamg_profile_enable(hier.h, False)
        dom = ks[0]
        ach = dom["bytes"] / (dom["total_ms"] / 1e3) / 1e9
        its = [i["iterations"] for i in infos]
        out[key] = {"ms_per_batch_solve": ms, "value": p.n_free_dofs * m / (ms / 1e3),
                    "unit": "dofs*rhs/s", "iterations_min_max": [min(its), max(its)],
                    "max_rel_res_true": max(i["rel_res_true"] for i in infos),
                    "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": ach,
                                 "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                                 "avg_launch_us": dom["total_ms"] / dom["launches"] * 1e3},
                    "kernels": [{"name": k["name"], "ms_per_solve": k["total_ms"],
                                 "GBps": k["bytes"] / (k["total_ms"] / 1e3) / 1e9}
                                for k in ks[:6]]}
    return out


def _multi_mesh(E, torch, steps, count=16, seed=4, coarsest=COARSEST_DOFS):
    """Independent meshes of uneven size solved together (eamg_solve_multi): count cubes with
    sides uniform in [8, 48] and Poisson ratios uniform in [0.2, 0.45], FP32 V-cycle in FP64 CG;
    against the same systems solved one after another."""
    from gen import make_problem
    rng = np.random.default_rng(seed)
    sides = rng.integers(8, 49, size=count)
    nus = rng.uniform(0.2, 0.45, size=count)
    t0 = time.perf_counter()
    sysm = []
    for c, (n, nu) in enumerate(zip(sides, nus)):
        p = make_problem(int(n), nu=float(nu), seed=100 + c)
        h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                        E.eamg_default_setup_params(vcycle_fp32=1, coarsest_max_dofs=coarsest))
        sysm.append((p, h))
    setup_s = time.perf_counter() - t0
    bs = [torch.tensor(p.b, device="cuda") for p, _ in sysm]
    xs = [torch.zeros_like(b) for b in bs]
    hs = [h.h for _, h in sysm]
    prec = E.EAMG_PRECOND_VCYCLE_FP32
    for (p, h), b, x in zip(sysm, bs, xs):
        h.solve(b, x, precond=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for (p, h), b, x in zip(sysm, bs, xs):
            h.solve(b, x, precond=prec)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 / steps
    E.eamg_solve_multi(hs, bs, xs, precond=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, infos = E.eamg_solve_multi(hs, bs, xs, precond=prec)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    assert st == E.EAMG_OK and max(i["rel_res_true"] for i in infos) <= 1e-8
    dofs = sum(p.n_free_dofs for p, _ in sysm)
    for _, h in sysm:
        h.close()
    return {"meshes": [int(n) for n in sides], "free_dofs": dofs, "setup_s": round(setup_s, 3),
            "coarsest_max_dofs": coarsest,
            "dtype": "f32 V-cycle in f64 CG", "ms_per_solve_all": ms,
            "value": dofs / (ms / 1e3), "unit": "dofs/s",
            "ms_one_after_another": seq_ms, "speedup_vs_one_after_another": seq_ms / ms,
            "iterations": [i["iterations"] for i in infos]}


def _learned(E, torch, n=40, inclusions=60):
    """Learned coarsening on a heterogeneous cube (stiff spherical inclusions, E = 1e4): the
    edge network is trained on the GPU on small meshes of the same kind (their exact
    criterion decisions), then the exact and the learned walk build hierarchies of the n^3
    mesh; criteria evaluations, setup time and PCG iterations are compared."""
    from gen import make_problem

    def hier(p, **kw):
        return E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                           E.eamg_default_setup_params(**kw))

    t0 = time.perf_counter()
    graphs = []
    for c, (m, inc, nu) in enumerate([(12, 8, 0.3), (14, 12, 0.4), (16, 16, 0.35), (13, 10, 0.45)]):
        p = make_problem(m, inclusions=inc, nu=nu, geometry_seed=10 + c, seed=c)
        h = hier(p, gnn_record=1)
        for k in range(E.eamg_coarsening_stats(h.h)["sample_passes"]):
            X, edges, nn, y, w = E.eamg_gnn_samples(h.h, k)
            if len(y) and w.sum() > 0:
                graphs.append((X, edges, nn, y, w))
        h.close()
    net = E.EdgeNet(seed=3)
    hist = net.train(graphs, epochs=200, lr=3e-3)
    train_s = time.perf_counter() - t0
    p = make_problem(n, inclusions=inclusions, nu=0.35, geometry_seed=96, seed=5)
    b = torch.tensor(p.b, device="cuda")
    out = {"workload": f"elasticity cube {n}^3, {inclusions} stiff spherical inclusions (E=1e4), "
                       f"nu=0.35; network trained on 4 meshes of 12^3..16^3",
           "train_s": round(train_s, 3), "train_loss": [float(hist[0]), float(hist[-1])]}
    for key, kw in (("exact", {}), ("learned", {"gnn": net.h.value, "gnn_skip": 0.2})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = hier(p, **kw)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        st = E.eamg_coarsening_stats(h.h)
        _, info = h.solve(b)
        out[key] = {"setup_s": round(setup_s, 3), "criteria_evaluations": st["evaluated"],
                    "mu_g_evaluations": st["evaluated_g"], "passed_over": st["skipped"],
                    "pcg_iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                    "oc": round(h.stats()["oc"], 4)}
        h.close()
    net.close()
    out["evaluations_saved"] = 1.0 - out["learned"]["criteria_evaluations"] / out["exact"]["criteria_evaluations"]
    return out


def _traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None if
    the summary is for another kernel or kernels.hip has changed since it was measured."""
    import hashlib
    import re
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        txt = open(os.path.join(root, "profiles", "traffic_k_gs_color_cube64.md")).read()
        src = open(os.path.join(root, "paper_2011_13325_amd", "csrc", "kernels.hip"), "rb").read()
    except OSError:
        return None
    k = re.search(r"^traffic_kernel: (.+)$", txt, re.M)
    v = re.search(r"^traffic_bytes_per_launch: (\d+)$", txt, re.M)
    h = re.search(r"^kernels_hip_sha256: ([0-9a-f]+)$", txt, re.M)
    if not (k and v and h) or k.group(1).strip() != kernel:
        return None
    if hashlib.sha256(src).hexdigest() != h.group(1):
        return None
    return float(v.group(1))


def _counter_pass():
    """Workload of the rocprofv3 counter passes (profiles/traffic_*.md): a calibration copy of
    64 MiB, then one FP64 solve of the bench problem with eager launches."""
    os.environ["EAMG_GRAPH"] = "0"
    import torch
    import paper_2011_13325_amd as E
    from gen import make_problem
    torch.cuda.set_device(0)
    n = 8 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    p = make_problem(64, seed=1)
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(coarsest_max_dofs=COARSEST_DOFS))
    E.eamg_autotune(h.h, 0)
    x, info = h.solve(torch.tensor(p.b, device="cuda"))
    torch.cuda.synchronize()
    print(f"counter pass: copy of {8 * n} bytes; solve {info['iterations']} iterations", flush=True)
    h.close()


def main():
    args = _args()
    if args.counter_pass:
        _counter_pass()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2011_13325_amd as E
    from gen import make_problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = make_problem(args.n, seed=1)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # FP32 copies of the V-cycle matrices are kept too, so that the same hierarchy serves the
    # FP64 solve (the headline) and the mixed-precision comparison
    prm = E.eamg_default_setup_params(vcycle_fp32=1, coarsest_max_dofs=args.coarsest)
    hier = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet, prm,
                       stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    # launch shapes measured on this hierarchy (single vector and 32-wide panels), once
    t0 = time.perf_counter()
    tune_before, tune_after = E.eamg_autotune(hier.h, panel_width=max(args.batch, 0), stream=stream)
    tune_s = time.perf_counter() - t0
    st = hier.stats()
    b = torch.tensor(p.b, device=dev)
    x = torch.zeros_like(b)
    ms, info = _timed_solves(E, torch, hier, b, x, stream, args.steps, args.warmup,
                             E.EAMG_PRECOND_VCYCLE)
    roof, kern = _profiled(E, hier, b, x, args.steps, E.EAMG_PRECOND_VCYCLE)
    ms32, info32 = _timed_solves(E, torch, hier, b, x, stream, args.steps, args.warmup,
                                 E.EAMG_PRECOND_VCYCLE_FP32)
    roof32, kern32 = _profiled(E, hier, b, x, args.steps, E.EAMG_PRECOND_VCYCLE_FP32)
    its = info["iterations"]
    vbytes, itbytes = E.eamg_traffic_model(hier.h, E.EAMG_PRECOND_VCYCLE)
    vbytes32, itbytes32 = E.eamg_traffic_model(hier.h, E.EAMG_PRECOND_VCYCLE_FP32)
    value = p.n_free_dofs / (ms / 1e3)
    out = {
        "metric": "AMG-PCG time to 1e-8 and dofs/s, FP64 vs mixed/batched; V-cycle HBM GB/s",
        "value": value, "unit": "dofs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"elasticity cube {args.n}^3 vertices (Kuhn P1, E=1, nu=0.3, "
                               f"clamped x=0, RHS seed 1), FP64 AMG-PCG to 1e-8, coarsening "
                               f"stopped below {args.coarsest} dofs",
                   "coarsest_max_dofs": args.coarsest,
                   "dofs": p.n_dofs, "free_dofs": p.n_free_dofs, "iterations": its,
                   "rel_res_true": info["rel_res_true"], "levels": st["n_levels"],
                   "level_vertices": st["n"], "vc": round(st["vc"], 4), "oc": round(st["oc"], 4),
                   "setup_s": round(setup_s, 3),
                   "autotune": {"s": round(tune_s, 3), "tuned_ms_before": tune_before,
                                "tuned_ms_after": tune_after},
                   "model_bytes_per_iteration": itbytes,
                   "model_GBps_whole_solve": itbytes * its / (ms / 1e3) / 1e9},
    }
    out["roofline"] = roof
    out["kernels"] = kern
    out["mixed_fp32_vcycle"] = {
        "value": p.n_free_dofs / (ms32 / 1e3), "unit": "dofs/s", "ms_per_step": ms32,
        "speedup_vs_fp64": ms / ms32, "iterations": info32["iterations"],
        "rel_res_true": info32["rel_res_true"], "dtype": "f32 V-cycle in f64 CG",
        "model_bytes_per_iteration": itbytes32,
        "model_GBps_whole_solve": itbytes32 * info32["iterations"] / (ms32 / 1e3) / 1e9,
        "roofline": roof32, "kernels": kern32[:8]}
    if args.batch > 0:
        out["batched"] = _batched(E, torch, hier, p, args.batch, args.steps, args.warmup)
        out["batched"]["speedup_per_rhs_vs_single_fp64"] = {
            k: out["batched"][k]["value"] / value for k in ("fp64_vcycle", "fp32_vcycle")}
    if not args.no_coarsest_500 and args.coarsest != 500:
        out["coarsest_500"] = _coarsest_500(E, torch, p, stream, args.steps, args.warmup, ms)
    if args.multi > 0:
        out["multi_mesh"] = _multi_mesh(E, torch, args.steps, count=args.multi,
                                        coarsest=args.coarsest)
    if not args.no_learned:
        out["learned_coarsening"] = _learned(E, torch, args.learned_n, args.learned_inclusions)
    levels = []
    for l in range(st["n_levels"]):
        li = E.eamg_level_info_get(hier.h, l)
        levels.append({"n": li["n"], "bs": li["bs"], "nnzb": li["nnzb_A"], "colors": li["n_colors"],
                       "nnzb_P": li["nnzb_P"]})
    out["config"]["level_info"] = levels
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
    hier.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
